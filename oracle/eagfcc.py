"""O2 for the advanced (electron-attached, EA) term of the GFCCSD Green's function.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What it computes (paper, Theory section): the second term of the GFCC Green's function,

    G^EA_pq(omega) = <Phi|(1 + Lambda) abar_p Y_q|Phi>,
    (omega - Hbar_N + i eta) Y_q |Phi> = abar_q^+ |Phi>,

with Y_q expanded in one-particle ``a_a^+`` and two-particle one-hole ``a_a^+ a_b^+ a_i``
operators (the Y_q expansion; GFCCSD truncation of T, Lambda and Y at two-body level).

Closed-shell spin-adapted basis (doublet), dimension v + o*v*v:

    y[0:v]                  = y_a     (coefficient of a^+_{a alpha})
    y[v + (j*v + a)*v + b]  = y_jab   (coefficient of a^+_{a alpha} a^+_{b beta} a_{j beta})

the same-spin component being y_jab - y_jba (checked by the brute force).

The working equations below were derived for this project from spin-orbital similarity-
transformed Hamiltonian elements by summing over the spin cases of this basis, and are
pinned term class by term class against the Fock-space brute force
(``oracle.fockspace.EABruteForce``); see ``tests/test_ea_oracle_pins.py``.

    s1[a]     = sum_c Fvv[a,c] y_c + sum_ld Fov[l,d] (2 y_lad - y_lda)
                + sum_lcd (2 Wvovv[a,l,c,d] - Wvovv[a,l,d,c]) y_lcd
    s2[j,a,b] = sum_c Wvvvo[a,b,c,j] y_c - sum_l Foo[l,j] y_lab + sum_c Fvv[a,c] y_jcb
                + sum_d Fvv[b,d] y_jad + sum_cd Wvvvv[a,b,c,d] y_jcd
                + sum_ld (2 Wovvo[l,b,d,j] - Wovov[l,b,j,d]) y_lad - sum_lc Wovov[l,a,j,c] y_lcb
                - sum_lc Wovvo[l,b,c,j] y_lca - sum_k Z_k t_kj^ab,
    Z_k       = sum_lcd (2(kc|ld) - (kd|lc)) y_lcd

with Foo, Fov, Fvv, Wovvo, Wovov the blocks of the IP part (``oracle.ipgfcc``) and

    Wvovv[a,l,c,d] = (ac|ld) - sum_k t_ka (kc|ld)
    Wvvvv[a,b,c,d] = (ac|bd) - sum_k t_kb (ac|kd) - sum_k t_ka (kc|bd) + sum_kl tau_kl^ab (kc|ld)
    Wvvvo[a,b,c,j] = (ac|bj) - sum_m Fov[m,c] t_mj^ab + sum_f t_jf Wvvvv[a,b,c,f]
                     + sum_mn (mc|nj) tau_mn^ab - sum_mf (mc|bf) t_mj^af
                     - sum_mf (mc|af) t_mj^fb + sum_mf (mf|ac) (2 t_mj^fb - t_mj^bf)
                     - sum_m t_ma [(mc|jb) - sum_nf (mc|nf)(t_nj^bf - 2 t_nj^fb) - sum_nf (mf|nc) t_nj^fb]
                     + sum_m t_mb [-(mj|ac) + sum_nf (mf|nc) t_nj^af]

Right-hand sides b_q = abar_q^+|Phi> (a virtual creator commutes with T; an occupied one
gives abar_i^+ = a_i^+ - sum_c t_i^c a_c^+ - 1/2 sum t_ik^cd a_c^+ a_d^+ a_k):
    virtual q = o + a:  b = e_a;     occupied q = i:  b_c = -t_ic,  b_jab = -t_ij^ab.
Left vectors c_p = <Phi|(1 + Lambda) abar_p restricted to the same space:
    occupied p = i:  c_b = -l_ib,  c_jab = -(2 l_ij^ab - l_ij^ba);
    virtual p = o + a:  c_b = d_ab - sum_i l_ib t_ia - sum_ijc (2 l_ij^bc - l_ij^cb) t_ij^ac,
                        c_jbc = 2 d_ab l_jc - d_ac l_jb - sum_i t_ia (2 l_ij^bc - l_ij^cb).
"""
from __future__ import annotations

import numpy as np

from . import ipgfcc as IP


def einsum(*a):
    return np.einsum(*a, optimize=True)


def integrals(sys):
    """Chemist integral blocks used by the EA part: (ov|vv), (vv|vv), (oo|ov), (oo|vv), (ov|ov)."""
    o = sys.n_occ
    L = sys.L
    Loo, Lov, Lvv = L[:, :o, :o], L[:, :o, o:], L[:, o:, o:]
    return {
        "ovov": einsum("Qpq,Qrs->pqrs", Lov, Lov),
        "ovvv": einsum("Qpq,Qrs->pqrs", Lov, Lvv),
        "vvvv": einsum("Qpq,Qrs->pqrs", Lvv, Lvv),
        "ooov": einsum("Qpq,Qrs->pqrs", Loo, Lov),
        "oovv": einsum("Qpq,Qrs->pqrs", Loo, Lvv),
    }


def intermediates(sys, im=None, g=None):
    """EA blocks of Hbar_N (alpha-beta components, connected form) plus the shared IP blocks."""
    if im is None:
        im = IP.intermediates(sys)
    if g is None:
        g = integrals(sys)
    ovov, ovvv, vvvv, ooov, oovv = g["ovov"], g["ovvv"], g["vvvv"], g["ooov"], g["oovv"]
    t1, t2 = sys.t1, sys.t2
    tau = t2 + einsum("ia,jb->ijab", t1, t1)
    Fov = im["Fov"]
    # (ac|ld) = ovvv[l,d,a,c]
    Wvovv = einsum("ldac->alcd", ovvv) - einsum("ka,kcld->alcd", t1, ovov)
    Wvvvv = (einsum("acbd->abcd", vvvv) - einsum("kb,kdac->abcd", t1, ovvv)
             - einsum("ka,kcbd->abcd", t1, ovvv) + einsum("klab,kcld->abcd", tau, ovov))
    # (ac|bj) = ovvv[j,b,a,c]; (mc|bf) = ovvv[m,c,b,f]; (mf|ac) = ovvv[m,f,a,c]
    # (mc|nj) = ooov[n,j,m,c]; (mj|ac) = oovv[m,j,a,c]; (mc|nf) = ovov[m,c,n,f]; (mc|jb) = ovov[m,c,j,b]
    Wvvvo = np.array(einsum("jbac->abcj", ovvv))
    Wvvvo -= einsum("mc,mjab->abcj", Fov, t2)
    Wvvvo += einsum("jf,abcf->abcj", t1, Wvvvv)
    Wvvvo += einsum("njmc,mnab->abcj", ooov, tau)
    Wvvvo -= einsum("mcbf,mjaf->abcj", ovvv, t2)
    Wvvvo -= einsum("mcaf,mjfb->abcj", ovvv, t2)
    Wvvvo += 2.0 * einsum("mfac,mjfb->abcj", ovvv, t2) - einsum("mfac,mjbf->abcj", ovvv, t2)
    Ymb = (einsum("mcjb->mbcj", ovov) - einsum("mcnf,njbf->mbcj", ovov, t2)
           + 2.0 * einsum("mcnf,njfb->mbcj", ovov, t2) - einsum("mfnc,njfb->mbcj", ovov, t2))
    Wvvvo -= einsum("ma,mbcj->abcj", t1, Ymb)
    Yma = -einsum("mjac->macj", oovv) + einsum("mfnc,njaf->macj", ovov, t2)
    Wvvvo += einsum("mb,macj->abcj", t1, Yma)
    return {"Foo": im["Foo"], "Fov": Fov, "Fvv": im["Fvv"], "Wovvo": im["Wovvo"], "Wovov": im["Wovov"],
            "Wvovv": Wvovv, "Wvvvv": Wvvvv, "Wvvvo": Wvvvo, "ovov": ovov, "t2": t2,
            "o": sys.n_occ, "v": sys.n_vir}


def split(y, o, v):
    return y[..., :v], y[..., v:].reshape(y.shape[:-1] + (o, v, v))


def sigma(eim, y):
    """Hbar_N applied to EA vectors y ([D] or [nb, D], real or complex)."""
    o, v = eim["o"], eim["v"]
    y = np.asarray(y)
    squeeze = y.ndim == 1
    if squeeze:
        y = y[None]
    y1, y2 = split(y, o, v)
    Foo, Fov, Fvv = eim["Foo"], eim["Fov"], eim["Fvv"]
    Wovvo, Wovov = eim["Wovvo"], eim["Wovov"]
    Wvovv, Wvvvv, Wvvvo = eim["Wvovv"], eim["Wvvvv"], eim["Wvvvo"]
    ovov, t2 = eim["ovov"], eim["t2"]
    s1 = einsum("ac,xc->xa", Fvv, y1)
    s1 += 2.0 * einsum("ld,xlad->xa", Fov, y2) - einsum("ld,xlda->xa", Fov, y2)
    s1 += 2.0 * einsum("alcd,xlcd->xa", Wvovv, y2) - einsum("aldc,xlcd->xa", Wvovv, y2)
    s2 = einsum("abcj,xc->xjab", Wvvvo, y1)
    s2 -= einsum("lj,xlab->xjab", Foo, y2)
    s2 += einsum("ac,xjcb->xjab", Fvv, y2) + einsum("bd,xjad->xjab", Fvv, y2)
    s2 += einsum("abcd,xjcd->xjab", Wvvvv, y2)
    s2 += 2.0 * einsum("lbdj,xlad->xjab", Wovvo, y2) - einsum("lbjd,xlad->xjab", Wovov, y2)
    s2 -= einsum("lajc,xlcb->xjab", Wovov, y2) + einsum("lbcj,xlca->xjab", Wovvo, y2)
    Z = 2.0 * einsum("kcld,xlcd->xk", ovov, y2) - einsum("kdlc,xlcd->xk", ovov, y2)
    s2 -= einsum("xk,kjab->xjab", Z, t2)
    out = np.concatenate([s1, s2.reshape(y.shape[0], -1)], axis=1)
    return out[0] if squeeze else out


def diagonal(eim):
    """Exact diagonal of Hbar_N in the EA basis."""
    o, v = eim["o"], eim["v"]
    Foo, Fvv, Wovvo, Wovov = eim["Foo"], eim["Fvv"], eim["Wovvo"], eim["Wovov"]
    Wvvvv, ovov, t2 = eim["Wvvvv"], eim["ovov"], eim["t2"]
    io, ia = np.arange(o), np.arange(v)
    d1 = np.diag(Fvv).copy()
    fo, fv = np.diag(Foo), np.diag(Fvv)
    d2 = (-fo[:, None, None] + fv[None, :, None] + fv[None, None, :]).copy()
    d2 += einsum("abab->ab", Wvvvv)[None]
    wvo = Wovvo[io[:, None], ia[None, :], ia[None, :], io[:, None]]  # [j,b] W_jbbj
    wov = Wovov[io[:, None], ia[None, :], io[:, None], ia[None, :]]  # [j,b] W_jbjb
    d2 += (2.0 * wvo - wov)[:, None, :]         # y_lad with l = j, d = b
    d2 -= wov[:, :, None]                        # y_lcb with l = j, c = a
    d2[:, ia, ia] -= wvo                         # y_lca with l = j, c = a = b
    # three-body: - sum_k (2 (ka|jb) - (kb|ja)) t_kj^ab
    d2 -= 2.0 * einsum("kajb,kjab->jab", ovov, t2) - einsum("kbja,kjab->jab", ovov, t2)
    return np.concatenate([d1, d2.reshape(-1)])


def explicit_matrix(eim):
    """Dense Hbar_N of the EA block, assembled element by element from the intermediates
    (Kronecker deltas rather than contractions), to check the contraction code."""
    o, v = eim["o"], eim["v"]
    D = v + o * v * v
    H = np.zeros((D, D))
    Foo, Fov, Fvv = eim["Foo"], eim["Fov"], eim["Fvv"]
    Wovvo, Wovov = eim["Wovvo"], eim["Wovov"]
    Wvovv, Wvvvv, Wvvvo = eim["Wvovv"], eim["Wvvvv"], eim["Wvvvo"]
    ovov, t2 = eim["ovov"], eim["t2"]

    def k2(j, a, b):
        return v + (j * v + a) * v + b

    for a in range(v):
        H[a, :v] = Fvv[a, :]
        C = np.zeros((o, v, v))
        C[:, a, :] += 2.0 * Fov
        C[:, :, a] -= Fov
        C += 2.0 * Wvovv[a] - Wvovv[a].transpose(0, 2, 1)
        H[a, v:] = C.reshape(-1)
    for j in range(o):
        for a in range(v):
            for b in range(v):
                row = k2(j, a, b)
                H[row, :v] = Wvvvo[a, b, :, j]
                C = np.zeros((o, v, v))  # coefficient of y[l, c, d]
                C[:, a, b] -= Foo[:, j]
                C[j, :, b] += Fvv[a, :]
                C[j, a, :] += Fvv[b, :]
                C[j] += Wvvvv[a, b]
                C[:, a, :] += 2.0 * Wovvo[:, b, :, j] - Wovov[:, b, j, :]
                C[:, :, b] -= Wovov[:, a, j, :]
                C[:, :, a] -= Wovvo[:, b, :, j]
                tk = t2[:, j, a, b]
                C -= 2.0 * einsum("k,kcld->lcd", tk, ovov) - einsum("k,kdlc->lcd", tk, ovov)
                H[row, v:] += C.reshape(-1)
    return H


def rhs(sys, q):
    """b_q = abar_q^+ |Phi> on the 1p + 2p1h space (q in [0, o + v))."""
    o, v = sys.n_occ, sys.n_vir
    b = np.zeros(v + o * v * v)
    if q >= o:
        b[q - o] = 1.0
    else:
        b[:v] = -sys.t1[q]
        b[v:] = -sys.t2[q].reshape(-1)
    return b


def left_vector(sys, p):
    """c_p = <Phi|(1 + Lambda) abar_p on the 1p + 2p1h space (p in [0, o + v))."""
    o, v = sys.n_occ, sys.n_vir
    t1, t2, l1, l2 = sys.t1, sys.t2, sys.l1, sys.l2
    ul = 2.0 * l2 - l2.transpose(0, 1, 3, 2)
    c = np.zeros(v + o * v * v)
    c2 = c[v:].reshape(o, v, v)
    if p < o:
        c[:v] = -l1[p]
        c2[...] = -ul[p]
    else:
        a = p - o
        c[:v] = -einsum("ib,i->b", l1, t1[:, a]) - einsum("ijbc,ijc->b", ul, t2[:, :, a, :])
        c[a] += 1.0
        c2[:, a, :] += 2.0 * l1
        c2[:, :, a] -= l1
        c2 -= einsum("i,ijbc->jbc", t1[:, a], ul)
    return c


def solve(sys, eim, q, omega, eta, tol=1e-12, restart=30, max_iter=5000, precond="jacobi"):
    """Y_q from (omega - Hbar_N + i eta) Y = b_q, solved as (-omega - i eta + Hbar_N) Y = -b_q
    by the same restarted GMRES as the IP part."""
    z = -omega - 1j * eta

    def apply_A(y):
        return z * y + sigma(eim, y)

    d = diagonal(eim)
    M = (lambda r: r / (z + d)) if precond == "jacobi" else None
    return IP.gmres(apply_A, -rhs(sys, q).astype(complex), tol=tol, restart=restart, max_iter=max_iter,
                    precond=M)


def greens(sys, eim, q, omegas, eta, ps=None, tol=1e-12, restart=30, precond="jacobi"):
    """G^EA_pq(omega) for p in ps (default [q]): array [n_omega][len(ps)]."""
    ps = [q] if ps is None else list(ps)
    C = np.stack([left_vector(sys, p) for p in ps])
    out = []
    for w in omegas:
        y, _, _ = solve(sys, eim, q, w, eta, tol=tol, restart=restart, precond=precond)
        out.append(C @ y)
    return np.array(out)
