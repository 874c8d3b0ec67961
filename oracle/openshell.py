"""The open-shell (spin-unrestricted) IP-GFCCSD: brute force and spin-orbital working equations.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's open-shell GFCCSD-IP treats alpha and beta electrons separately (Evaluation
section, Table 2).  Here the reference has n_occ_a alpha and n_occ_b beta electrons in n
spatial orbitals per spin with spin-dependent orbital energies and Cholesky vectors
(``synth.OpenShellSystem``); the retarded IP term of the Green's function (Theory section)

    G_qp(omega) = <Phi|(1 + Lambda) abar_q^+ X_p|Phi>,   (omega + Hbar_N - i eta) X_p = abar_p|Phi>,

is taken over spin orbitals p, q with X_p in the 1h + 2h1p space (all spin cases).

* ``OpenShellBruteForce`` -- needs no working equations: determinant matrices of H, T, Lambda
  in the N-electron sector and in both (N-1)-electron sectors (an alpha or a beta electron
  removed), Hbar = e^-T H e^T, and for every basis operator R_mu (a_i; a_a^+ a_j a_i, i < j)
  ``Hbar[mu', mu] = <mu'|[Hbar, R_mu]|Phi>``, ``b_p``, ``c_q`` from their definitions.
* The spin-orbital working equations (``so_arrays``, ``intermediates``, ``sigma``, ...) were
  written for this project from the spin-orbital similarity-transformed Hamiltonian and are
  pinned against the brute force (``tests/test_openshell_oracle_pins.py``).

Spin-orbital ordering used by the equations and the GPU library: occupied
[alpha 0..oa-1, beta 0..ob-1], virtual [alpha oa..n-1, beta ob..n-1]; orbital index
p in [0, o + v) runs over occupied then virtual (o = oa + ob, v = va + vb).

Vector layout (both orders of the hole pair stored): x[0:o] = r_i; x[o + (i*o + j)*v + a] = r_ij^a
with r_ji^a = -r_ij^a and r_ii^a = 0, where R = sum_i r_i a_i + 1/2 sum_ija r_ij^a a_a^+ a_j a_i.
A left vector carries 1/2 on its 2h1p block so that c . x counts every pair once.
"""
from __future__ import annotations

import numpy as np

from .fockspace import SpinOrbitalSystem, _expm_nilpotent, apply_string, op_matrix, sector
from . import ipgfcc as IP


def einsum(*a):
    return np.einsum(*a, optimize=True)


# ------------------------------------------------------------------ spin-orbital arrays

def orbitals(sys):
    """[(spin, spatial)] of occupied then virtual spin orbitals in the library's order."""
    n, oa, ob = sys.n, sys.n_occ_a, sys.n_occ_b
    occ = [(0, p) for p in range(oa)] + [(1, p) for p in range(ob)]
    vir = [(0, p) for p in range(oa, n)] + [(1, p) for p in range(ob, n)]
    return occ, vir


def so_arrays(sys):
    """Spin-orbital eps, Cholesky vectors L[Q][P][R] = d(sP,sR) L_s[Q,p,r], t1, t2, l1, l2."""
    occ, vir = orbitals(sys)
    orb = occ + vir
    o, v = len(occ), len(vir)
    n_so = o + v
    eps = np.array([(sys.eps_a, sys.eps_b)[s][p] for s, p in orb])
    Ls = (sys.La, sys.Lb)
    L = np.zeros((sys.n_chol, n_so, n_so))
    for k, (sk, pk) in enumerate(orb):
        for m, (sm, pm) in enumerate(orb):
            if sk == sm:
                L[:, k, m] = Ls[sk][:, pk, pm]
    oS = (sys.n_occ_a, sys.n_occ_b)

    def amps(a1, b1, aa, ab, bb):
        t1 = np.zeros((o, v))
        t2 = np.zeros((o, o, v, v))
        one = (a1, b1)
        two = {(0, 0): aa, (1, 1): bb}
        for i, (si, pi) in enumerate(occ):
            for a, (sa, pa) in enumerate(vir):
                if si == sa:
                    t1[i, a] = one[si][pi, pa - oS[si]]
        for i, (si, pi) in enumerate(occ):
            for j, (sj, pj) in enumerate(occ):
                for a, (sa, pa) in enumerate(vir):
                    for b, (sb, pb) in enumerate(vir):
                        ai, bj = pa - oS[sa], pb - oS[sb]
                        val = 0.0
                        if si == sj:
                            if sa == si and sb == si:
                                val = two[(si, si)][pi, pj, ai, bj]
                        elif si == 0:  # i alpha, j beta
                            if sa == 0 and sb == 1:
                                val = ab[pi, pj, ai, bj]
                            elif sa == 1 and sb == 0:
                                val = -ab[pi, pj, bj, ai]
                        else:  # i beta, j alpha
                            if sa == 0 and sb == 1:
                                val = -ab[pj, pi, ai, bj]
                            elif sa == 1 and sb == 0:
                                val = ab[pj, pi, bj, ai]
                        t2[i, j, a, b] = val
        return t1, t2

    t1, t2 = amps(sys.t1a, sys.t1b, sys.t2aa, sys.t2ab, sys.t2bb)
    l1, l2 = amps(sys.l1a, sys.l1b, sys.l2aa, sys.l2ab, sys.l2bb)
    return {"o": o, "v": v, "eps": eps, "L": L, "t1": t1, "t2": t2, "l1": l1, "l2": l2}


def antisym_integrals(so):
    """<pq||rs> over the spin-orbital list (occupied then virtual)."""
    L = so["L"]
    g = einsum("Qpr,Qqs->pqrs", L, L)  # <pq|rs> = (pr|qs)
    return g - g.transpose(0, 1, 3, 2)


# ------------------------------------------------------------------ brute force

def _op_into(ops, dets_in, idx_out):
    """Matrix of one operator string from a sector into another; determinants it sends
    elsewhere (or annihilates) give zero columns."""
    M = np.zeros((len(idx_out), len(dets_in)))
    for col, d in enumerate(dets_in):
        sg, d2 = apply_string(ops, d)
        if sg and d2 in idx_out:
            M[idx_out[d2], col] += sg
    return M


class OpenShellBruteForce:
    """Dense IP quantities of one tiny open-shell system over both ionised sectors.

    Basis (unique pairs): ``("1h", i)`` and ``("2h1p", i, j, a)`` with i < j, in the library's
    spin-orbital order; only operators that reach one of the two (N-1)-electron sectors are
    kept.  ``H`` is block diagonal over the sectors; ``b[p]``, ``c[q]`` for every spin orbital."""

    def __init__(self, sys):
        n, oa, ob = sys.n, sys.n_occ_a, sys.n_occ_b
        occ, vir = orbitals(sys)
        orb = occ + vir
        o = len(occ)
        self.o, self.v = o, len(vir)
        # determinant spin-orbital index of a library orbital: spin * n + spatial
        P = [s * n + p for s, p in orb]
        so = so_arrays(sys)
        A = antisym_integrals(so)
        # Hamiltonian over determinant spin orbitals
        N = 2 * n
        Adet = np.zeros((N, N, N, N))
        idx = np.array(P)
        Adet[np.ix_(idx, idx, idx, idx)] = A
        f = np.zeros((N, N))
        f[idx, idx] = so["eps"]
        occ_det = [P[k] for k in range(o)]
        h = f - sum(Adet[:, K, :, K] for K in occ_det)

        class _H:  # the Hamiltonian builder needs n, h and A only
            pass
        hb = _H()
        hb.n, hb.h, hb.A = n, h, Adet

        def terms(t1, t2, excite):
            out = []
            for i in range(o):
                for a in range(len(vir)):
                    c = t1[i, a]
                    if c != 0.0:
                        I, Av = P[i], P[o + a]
                        out.append((c, [(False, I), (True, Av)] if excite else [(False, Av), (True, I)]))
            for i in range(o):
                for j in range(i + 1, o):
                    for a in range(len(vir)):
                        for b in range(a + 1, len(vir)):
                            c = t2[i, j, a, b]
                            if c != 0.0:
                                I, J, Av, B = P[i], P[j], P[o + a], P[o + b]
                                out.append((c, [(False, I), (False, J), (True, B), (True, Av)] if excite
                                            else [(False, Av), (False, B), (True, J), (True, I)]))
            return out

        Tt = terms(so["t1"], so["t2"], True)
        Lt = terms(so["l1"], so["l2"], False)
        detsN, idxN = sector(n, oa, ob)
        phi_det = sum(1 << p for p in range(oa)) | sum(1 << (n + p) for p in range(ob))
        phi = np.zeros(len(detsN))
        phi[idxN[phi_det]] = 1.0
        HN = SpinOrbitalSystem.hamiltonian(hb, detsN, idxN)
        TN = op_matrix(Tt, detsN, idxN)
        eTN, emTN = _expm_nilpotent(TN), _expm_nilpotent(-TN)
        HbN = emTN @ HN @ eTN
        LamN = op_matrix(Lt, detsN, idxN)
        HbNphi = HbN @ phi
        braN = phi @ (np.eye(len(detsN)) + LamN) @ emTN

        basis = [("1h", i) for i in range(o)]
        basis += [("2h1p", i, j, a) for i in range(o) for j in range(i + 1, o) for a in range(len(vir))]
        sectors = {}
        for s in (0, 1):
            na, nb = (oa - 1, ob) if s == 0 else (oa, ob - 1)
            if na < 0 or nb < 0:
                continue
            dets, idm = sector(n, na, nb)
            H = SpinOrbitalSystem.hamiltonian(hb, dets, idm)
            T = op_matrix(Tt, dets, idm)
            eT, emT = _expm_nilpotent(T), _expm_nilpotent(-T)
            sectors[s] = (dets, idm, emT @ H @ eT, eT, emT)
        keep, Rs, sect_of = [], [], []
        for bb in basis:
            ops = [(False, P[bb[1]])] if bb[0] == "1h" else [(False, P[bb[1]]), (False, P[bb[2]]),
                                                              (True, P[o + bb[3]])]
            sg, d2 = apply_string(ops, phi_det)
            if not sg:
                continue
            for s, (dets, idm, _, _, _) in sectors.items():
                if d2 in idm:
                    keep.append(bb)
                    Rs.append(_op_into(ops, detsN, idm))
                    sect_of.append(s)
                    break
        self.basis = keep
        Dk = len(keep)
        evec = {s: np.zeros((len(sectors[s][0]), Dk)) for s in sectors}
        for mu, (R, s) in enumerate(zip(Rs, sect_of)):
            evec[s][:, mu] = R @ phi
        Hm = np.zeros((Dk, Dk))
        for mu, (R, s) in enumerate(zip(Rs, sect_of)):
            sig = sectors[s][2] @ evec[s][:, mu] - R @ HbNphi
            Hm[:, mu] = evec[s].T @ sig
        self.H = Hm
        norb = len(orb)
        self.b = np.zeros((norb, Dk))
        self.c = np.zeros((norb, Dk))
        for p in range(norb):
            s = P[p] // n
            if s not in sectors:
                continue
            dets, idm, _, eT, emT = sectors[s]
            Ap = op_matrix([(1.0, [(False, P[p])])], detsN, idm)
            self.b[p] = evec[s].T @ (emT @ Ap @ eTN @ phi)
            Aqd = op_matrix([(1.0, [(True, P[p])])], dets, idxN)
            self.c[p] = (braN @ Aqd @ eT) @ evec[s]
        # map between the unique basis and the library's full vectors
        v = len(vir)
        D = o + o * o * v
        self.D = D
        Emap = np.zeros((Dk, D))   # unique -> full (antisymmetric extension)
        for mu, bb in enumerate(keep):
            if bb[0] == "1h":
                Emap[mu, bb[1]] = 1.0
            else:
                _, i, j, a = bb
                Emap[mu, o + (i * o + j) * v + a] = 1.0
                Emap[mu, o + (j * o + i) * v + a] = -1.0
        self.Emap = Emap

    def full(self, u):
        """Unique-basis coefficients -> the library's full vector."""
        return u @ self.Emap

    def unique(self, x):
        """The library's full vector -> unique-basis coefficients (reads the i < j entries)."""
        sel = np.array([(bb[1] if bb[0] == "1h" else self.o + (bb[1] * self.o + bb[2]) * self.v + bb[3])
                        for bb in self.basis])
        return x[..., sel]

    def greens(self, omega, eta, p, q):
        """G_qp(omega) = c_q^T (omega - i eta + Hbar)^-1 b_p over the unique basis."""
        A = (omega - 1j * eta) * np.eye(self.H.shape[0]) + self.H
        return self.c[q] @ np.linalg.solve(A, self.b[p])


# ------------------------------------------------------------------ spin-orbital equations

def intermediates(sys, so=None):
    """Spin-orbital blocks of Hbar_N for the IP space (connected form)."""
    if so is None:
        so = so_arrays(sys)
    o, v = so["o"], so["v"]
    A = antisym_integrals(so)
    oo, vv = slice(0, o), slice(o, o + v)
    oooo, ooov, oovv = A[oo, oo, oo, oo], A[oo, oo, oo, vv], A[oo, oo, vv, vv]
    ovvo, ovvv, ovoo = A[oo, vv, vv, oo], A[oo, vv, vv, vv], A[oo, vv, oo, oo]
    vovv = A[vv, oo, vv, vv]
    eps = so["eps"]
    t1, t2 = so["t1"], so["t2"]
    tau = t2 + einsum("ie,jf->ijef", t1, t1) - einsum("if,je->ijef", t1, t1)

    Fov = einsum("nf,mnef->me", t1, oovv)
    Foo = (np.diag(eps[:o]) + einsum("ie,me->mi", t1, Fov) + einsum("ne,mnie->mi", t1, ooov)
           + 0.5 * einsum("inef,mnef->mi", t2, oovv))
    Fvv = (np.diag(eps[o:]) - einsum("ma,me->ae", t1, Fov) + einsum("mf,amef->ae", t1, vovv)
           - 0.5 * einsum("mnaf,mnef->ae", t2, oovv))
    Woooo = (oooo + einsum("je,mnie->mnij", t1, ooov) - einsum("ie,mnje->mnij", t1, ooov)
             + 0.5 * einsum("ijef,mnef->mnij", tau, oovv))
    Wooov = ooov + einsum("if,mnfe->mnie", t1, oovv)
    Wovvo = (ovvo + einsum("jf,mbef->mbej", t1, ovvv) - einsum("nb,mnej->mbej", t1, A[oo, oo, vv, oo])
             - einsum("jnfb,mnef->mbej", t2, oovv) - einsum("jf,nb,mnef->mbej", t1, t1, oovv))
    # bracket of the t1 terms of Wovoo: <mb||ej> - sum_nf t_nj^bf <mn||ef>
    Ybr = ovvo - einsum("njbf,mnef->mbej", t2, oovv)
    Wovoo = (ovoo - einsum("me,ijbe->mbij", Fov, t2) - einsum("nb,mnij->mbij", t1, Woooo)
             + 0.5 * einsum("mbef,ijef->mbij", ovvv, tau)
             + einsum("mnie,jnbe->mbij", ooov, t2) - einsum("mnje,inbe->mbij", ooov, t2)
             + einsum("ie,mbej->mbij", t1, Ybr) - einsum("je,mbei->mbij", t1, Ybr))
    return {"o": o, "v": v, "Fov": Fov, "Foo": Foo, "Fvv": Fvv, "Woooo": Woooo, "Wooov": Wooov,
            "Wovvo": Wovvo, "Wovoo": Wovoo, "oovv": oovv, "t2": t2, "so": so}


def split(x, o, v):
    return x[..., :o], x[..., o:].reshape(x.shape[:-1] + (o, o, v))


def sigma(im, x):
    """Hbar_N on full spin-orbital IP vectors x ([D] or [nb, D]); keeps r_ij^a antisymmetric."""
    o, v = im["o"], im["v"]
    x = np.asarray(x)
    squeeze = x.ndim == 1
    if squeeze:
        x = x[None]
    r1, r2 = split(x, o, v)
    Foo, Fov, Fvv = im["Foo"], im["Fov"], im["Fvv"]
    Woooo, Wooov, Wovvo, Wovoo = im["Woooo"], im["Wooov"], im["Wovvo"], im["Wovoo"]
    oovv, t2 = im["oovv"], im["t2"]
    s1 = -einsum("mi,xm->xi", Foo, r1) + einsum("me,xime->xi", Fov, r2)
    s1 -= 0.5 * einsum("mnie,xmne->xi", Wooov, r2)
    s2 = -einsum("maij,xm->xija", Wovoo, r1)
    s2 += einsum("ae,xije->xija", Fvv, r2)
    s2 -= einsum("mi,xmja->xija", Foo, r2) - einsum("mj,xmia->xija", Foo, r2)
    s2 += 0.5 * einsum("mnij,xmna->xija", Woooo, r2)
    s2 += einsum("maej,xime->xija", Wovvo, r2) - einsum("maei,xjme->xija", Wovvo, r2)
    Z = 0.5 * einsum("mnef,xmnf->xe", oovv, r2)
    s2 += einsum("xe,ijae->xija", Z, t2)
    out = np.concatenate([s1, s2.reshape(x.shape[0], -1)], axis=1)
    return out[0] if squeeze else out


def diagonal(im):
    """Exact diagonal of Hbar_N over the unique basis, laid out as a full vector (the (i, j) and
    (j, i) entries of a pair share the value; i = j entries follow the same formula)."""
    o, v = im["o"], im["v"]
    Foo, Fvv, Woooo, Wovvo = im["Foo"], im["Fvv"], im["Woooo"], im["Wovvo"]
    oovv, t2 = im["oovv"], im["t2"]
    fo, fv = np.diag(Foo), np.diag(Fvv)
    io, ia = np.arange(o), np.arange(v)
    d1 = -fo
    d2 = fv[None, None, :] - fo[:, None, None] - fo[None, :, None]
    d2 = d2 + einsum("ijij->ij", Woooo)[:, :, None]
    wvo = Wovvo[io[:, None], ia[None, :], ia[None, :], io[:, None]]  # [j, a] = W_jaaj
    d2 = d2 + wvo[None, :, :] + wvo[:, None, :]
    d2 = d2 + einsum("ijea,ijae->ija", oovv, t2)
    return np.concatenate([d1, d2.reshape(-1)])


def rhs(so, p):
    """b_p = abar_p|Phi> as a full vector: occupied p -> e_p; virtual p = o + a ->
    r_i = t_i^a, r_ij^b = t_ij^ab."""
    o, v = so["o"], so["v"]
    x = np.zeros(o + o * o * v)
    if p < o:
        x[p] = 1.0
    else:
        a = p - o
        x[:o] = so["t1"][:, a]
        x[o:] = so["t2"][:, :, a, :].reshape(-1)
    return x


def left_vector(so, q):
    """c_q = <Phi|(1 + Lambda) abar_q^+ as a full vector with 1/2 on its 2h1p block.

    occupied q:  c_i = d_qi - sum_e l_i^e t_q^e - 1/2 sum_jef l_ij^ef t_qj^ef,
                 c_ij^b = d_qi l_j^b - d_qj l_i^b - sum_e t_q^e l_ij^eb;
    virtual q = o + a:  c_i = l_i^a,  c_ij^b = l_ij^ab."""
    o, v = so["o"], so["v"]
    t1, t2, l1, l2 = so["t1"], so["t2"], so["l1"], so["l2"]
    if q < o:
        e = np.zeros(o)
        e[q] = 1.0
        c1 = e - einsum("ie,e->i", l1, t1[q]) - 0.5 * einsum("ijef,jef->i", l2, t2[q])
        c2 = einsum("i,jb->ijb", e, l1) - einsum("j,ib->ijb", e, l1) - einsum("e,ijeb->ijb", t1[q], l2)
    else:
        a = q - o
        c1 = l1[:, a].copy()
        c2 = l2[:, :, a, :].copy()
    return np.concatenate([c1, 0.5 * c2.reshape(-1)])


def solve(im, so, p, omega, eta, tol=1e-12, restart=30, max_iter=5000, precond="jacobi"):
    """X_p from (omega - i eta + Hbar_N) X = b_p by the restarted GMRES of the IP oracle."""
    z = omega - 1j * eta
    d = diagonal(im)
    M = (lambda r: r / (z + d)) if precond == "jacobi" else None
    return IP.gmres(lambda x: z * x + sigma(im, x), rhs(so, p).astype(complex), tol=tol, restart=restart,
                    max_iter=max_iter, precond=M)


def greens(im, so, p, omegas, eta, qs=None, tol=1e-12, restart=30):
    """G_qp(omega) for q in qs (default [p]): array [n_omega][len(qs)]."""
    qs = [p] if qs is None else list(qs)
    C = np.stack([left_vector(so, q) for q in qs])
    return np.array([C @ solve(im, so, p, w, eta, tol=tol, restart=restart)[0] for w in omegas])


def from_closed_shell(s):
    """The closed-shell system ``s`` (synth.System) as an open-shell one with identical spins:
    t_{i alpha j beta}^{a alpha b beta} = t2[i,j,a,b], same-spin t2[i,j,a,b] - t2[i,j,b,a]."""
    import synth
    aa = s.t2 - s.t2.transpose(0, 1, 3, 2)
    laa = s.l2 - s.l2.transpose(0, 1, 3, 2)
    return synth.OpenShellSystem(s.n, s.n_occ, s.n_occ, s.n_chol, s.eps.copy(), s.eps.copy(), s.L, s.L,
                                 s.t1, s.t1, aa, s.t2, aa, s.l1, s.l1, laa, s.l2, laa, s.seed)
