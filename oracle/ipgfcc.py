"""O2: matrix-free spin-adapted IP-GFCCSD oracle (closed shell), FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What it computes (paper, Theory section):

* the retarded IP term of the GFCC Green's function,
  ``G_qp(omega) = c_q^T X_p`` with ``(omega + Hbar_N - i eta) X_p = b_p``
  (the linear system for X_p, the compact form of G and its GFCCSD
  truncation at one- and two-body T, Lambda and X), using the bilinear
  (non-conjugated) product of the model-order-reduction equations;
* ``Hbar_N`` restricted to the 1h + 2h1p space of X_p;
* GMRES (GFCC Workflow and Bottlenecks: the minimal-residual Krylov solver chosen for these
  non-Hermitian systems, residual non-increasing, at most dim-many steps;
  the inverse diagonal of the Hamiltonian as the classic preconditioner).

The paper prints no working equations.  The closed-shell spin-adapted
formulas below were derived for this project from spin-orbital
similarity-transformed Hamiltonian elements by summing over the spin cases
of the doublet basis ``r_i = r_{i alpha}``,
``r_ija = r^{a beta}_{i alpha, j beta}`` (same-spin part ``r_ija - r_jia``).
Every term class is pinned against the Fock-space brute force
(``oracle.fockspace``) in the CPU tests.

Notation: chemist integrals ``(pq|rs) = sum_Q L[Q,p,q] L[Q,r,s]``; occupied
indices i j k l m n, virtual a b c d e f; ``t1[i,a]``, ``t2[i,j,a,b]``,
``l1[i,a]``, ``l2[i,j,a,b]``; Fock matrix ``diag(eps)``;
``tau[i,j,e,f] = t2[i,j,e,f] + t1[i,e] t1[j,f]``.
Vector layout: ``x[0:o] = r_i``, ``x[o + (i*o + j)*v + a] = r_ija``.
"""
from __future__ import annotations

import numpy as np


def einsum(*a):
    return np.einsum(*a, optimize=True)


# --------------------------------------------------------------------------
# integrals and intermediates (built once per system, paper, Implementation Details: constant
# intermediates of size <= O(o^2 v^2) precomputed before the GFCC loop)
# --------------------------------------------------------------------------

def integrals(sys):
    """Chemist integral blocks ``blk[p,q,r,s] = (pq|rs)`` for the index classes named."""
    o = sys.n_occ
    L = sys.L
    Loo, Lov, Lvv = L[:, :o, :o], L[:, :o, o:], L[:, o:, o:]
    return {
        "oooo": einsum("Qpq,Qrs->pqrs", Loo, Loo),
        "ooov": einsum("Qpq,Qrs->pqrs", Loo, Lov),
        "oovv": einsum("Qpq,Qrs->pqrs", Loo, Lvv),
        "ovov": einsum("Qpq,Qrs->pqrs", Lov, Lov),
        "ovvv": einsum("Qpq,Qrs->pqrs", Lov, Lvv),
    }


def intermediates(sys, g=None):
    """Spin-adapted Hbar blocks (alpha-beta-alpha-beta components), connected form."""
    o = sys.n_occ
    eps_o, eps_v = sys.eps[:o], sys.eps[o:]
    t1, t2 = sys.t1, sys.t2
    if g is None:
        g = integrals(sys)
    oooo, ooov, oovv, ovov, ovvv = g["oooo"], g["ooov"], g["oovv"], g["ovov"], g["ovvv"]
    tau = t2 + einsum("ie,jf->ijef", t1, t1)

    # F_me = sum_nf t_nf [2(me|nf) - (mf|ne)]
    Fov = 2.0 * einsum("nf,menf->me", t1, ovov) - einsum("nf,mfne->me", t1, ovov)

    # F_mi = e_i d_mi + sum_e t_ie F_me + sum_ne t_ne [2(mi|ne) - (me|ni)]
    #        + sum_nef [2 t_in^ef - t_in^fe] (me|nf)
    Foo = (np.diag(eps_o)
           + einsum("ie,me->mi", t1, Fov)
           + 2.0 * einsum("ne,mine->mi", t1, ooov)
           - einsum("ne,nime->mi", t1, ooov)
           + 2.0 * einsum("inef,menf->mi", t2, ovov)
           - einsum("infe,menf->mi", t2, ovov))

    # F_ae = e_a d_ae - sum_m t_ma F_me + sum_mf t_mf [2(ae|mf) - (af|me)]
    #        - sum_mnf [2 t_mn^af - t_mn^fa] (me|nf)
    Fvv = (np.diag(eps_v)
           - einsum("ma,me->ae", t1, Fov)
           + 2.0 * einsum("mf,mfae->ae", t1, ovvv)
           - einsum("mf,meaf->ae", t1, ovvv)
           - 2.0 * einsum("mnaf,menf->ae", t2, ovov)
           + einsum("mnfa,menf->ae", t2, ovov))

    # W_mnij = (mi|nj) + sum_e t_je (mi|ne) + sum_e t_ie (me|nj) + sum_ef tau_ij^ef (me|nf)
    Woooo = (oooo.transpose(0, 2, 1, 3)
             + einsum("je,mine->mnij", t1, ooov)
             + einsum("ie,njme->mnij", t1, ooov)
             + einsum("ijef,menf->mnij", tau, ovov))

    # W_mnie = (mi|ne) + sum_f t_if (mf|ne)
    Wooov = ooov.transpose(0, 2, 1, 3) + einsum("if,mfne->mnie", t1, ovov)

    # ring parts that only involve bare integrals and T2
    # Q_maej = (me|aj) + sum_nf [(2 t_jn^af - t_jn^fa)(me|nf) - t_jn^af (mf|ne)]
    Qovvo = (ovov.transpose(0, 3, 1, 2)
             + 2.0 * einsum("jnaf,menf->maej", t2, ovov)
             - einsum("jnfa,menf->maej", t2, ovov)
             - einsum("jnaf,mfne->maej", t2, ovov))
    # Q_maje = (mj|ae) - sum_nf t_jn^fa (mf|ne)
    Qovov = (oovv.transpose(0, 2, 1, 3)
             - einsum("jnfa,mfne->maje", t2, ovov))

    # W_maej = Q_maej + sum_f t_jf (me|af) - sum_n t_na (me|nj) - sum_nf t_jf t_na (me|nf)
    Wovvo = (Qovvo
             + einsum("jf,meaf->maej", t1, ovvv)
             - einsum("na,njme->maej", t1, ooov)
             - einsum("jf,na,menf->maej", t1, t1, ovov))
    # W_maje = Q_maje + sum_f t_jf (mf|ae) - sum_n t_na (mj|ne) - sum_nf t_jf t_na (mf|ne)
    Wovov = (Qovov
             + einsum("jf,mfae->maje", t1, ovvv)
             - einsum("na,mjne->maje", t1, ooov)
             - einsum("jf,na,mfne->maje", t1, t1, ovov))

    # W_maij = (mi|aj) + sum_e F_me t_ij^ea - sum_n t_na W_mnij + sum_ef (me|af) tau_ij^ef
    #          + sum_ne [(mi|ne)(2 t_jn^ae - t_jn^ea) - (me|ni) t_jn^ae - (me|nj) t_in^ea]
    #          + sum_e t_ie Q_maej + sum_e t_je Q_maie
    Wovoo = (ooov.transpose(0, 3, 1, 2)
             + einsum("me,ijea->maij", Fov, t2)
             - einsum("na,mnij->maij", t1, Woooo)
             + einsum("meaf,ijef->maij", ovvv, tau)
             + 2.0 * einsum("mine,jnae->maij", ooov, t2)
             - einsum("mine,jnea->maij", ooov, t2)
             - einsum("nime,jnae->maij", ooov, t2)
             - einsum("njme,inea->maij", ooov, t2)
             + einsum("ie,maej->maij", t1, Qovvo)
             + einsum("je,maie->maij", t1, Qovov))

    return {"Fov": Fov, "Foo": Foo, "Fvv": Fvv, "Woooo": Woooo, "Wooov": Wooov,
            "Wovoo": Wovoo, "Wovvo": Wovvo, "Wovov": Wovov, "ovov": ovov,
            "t2": t2, "o": o, "v": sys.n_vir}


# --------------------------------------------------------------------------
# sigma product  sigma = Hbar_N x  (paper, GFCC Workflow and Bottlenecks: O(o^3 v^2) per iteration)
# --------------------------------------------------------------------------

def split(x, o, v):
    """x[..., D] -> (r1[..., o], r2[..., o, o, v])."""
    return x[..., :o], x[..., o:].reshape(x.shape[:-1] + (o, o, v))


def sigma(im, x):
    """Hbar_N applied to x (complex or real), x shape [D] or [nb, D]."""
    o, v = im["o"], im["v"]
    x = np.asarray(x)
    squeeze = x.ndim == 1
    if squeeze:
        x = x[None]
    r1, r2 = split(x, o, v)
    Foo, Fov, Fvv = im["Foo"], im["Fov"], im["Fvv"]
    Wooov, Wovoo, Woooo = im["Wooov"], im["Wovoo"], im["Woooo"]
    Wovvo, Wovov, ovov, t2 = im["Wovvo"], im["Wovov"], im["ovov"], im["t2"]

    # 1h <- 1h, 1h <- 2h1p
    s1 = (-einsum("mi,bm->bi", Foo, r1)
          + 2.0 * einsum("me,bime->bi", Fov, r2)
          - einsum("me,bmie->bi", Fov, r2)
          - 2.0 * einsum("mnie,bmne->bi", Wooov, r2)
          + einsum("nmie,bmne->bi", Wooov, r2))

    # 2h1p <- 1h
    s2 = -einsum("maij,bm->bija", Wovoo, r1)
    # 2h1p <- 2h1p: one-body parts
    s2 += einsum("ae,bije->bija", Fvv, r2)
    s2 -= einsum("mi,bmja->bija", Foo, r2)
    s2 -= einsum("mj,bima->bija", Foo, r2)
    # hole-hole ladder
    s2 += einsum("mnij,bmna->bija", Woooo, r2)
    # ring terms (the O(o^3 v^2) contractions)
    s2 += 2.0 * einsum("maej,bime->bija", Wovvo, r2)
    s2 -= einsum("maje,bime->bija", Wovov, r2)
    s2 -= einsum("maej,bmie->bija", Wovvo, r2)
    s2 -= einsum("maie,bmje->bija", Wovov, r2)
    # three-body term: z_e = sum_mnf [2(me|nf) - (mf|ne)] r_mnf ; s -= sum_e z_e t_ij^ea
    z = 2.0 * einsum("menf,bmnf->be", ovov, r2) - einsum("mfne,bmnf->be", ovov, r2)
    s2 -= einsum("be,ijea->bija", z, t2)

    out = np.concatenate([s1, s2.reshape(x.shape[0], -1)], axis=1)
    return out[0] if squeeze else out


def diagonal(im):
    """Exact diagonal of Hbar_N in the spin-adapted basis."""
    o, v = im["o"], im["v"]
    Foo, Fvv = im["Foo"], im["Fvv"]
    Woooo, Wovvo, Wovov, ovov, t2 = im["Woooo"], im["Wovvo"], im["Wovov"], im["ovov"], im["t2"]
    d1 = -np.diag(Foo).copy()
    io = np.arange(o)
    ia = np.arange(v)
    fo = np.diag(Foo)
    fv = np.diag(Fvv)
    d2 = (fv[None, None, :] - fo[:, None, None] - fo[None, :, None]).copy()
    d2 += einsum("ijij->ij", Woooo)[:, :, None]
    wvo = Wovvo[io[:, None], ia[None, :], ia[None, :], io[:, None]]  # [j,a] W_jaaj
    wov = Wovov[io[:, None], ia[None, :], io[:, None], ia[None, :]]  # [j,a] W_jaja
    d2 += (2.0 * wvo - wov)[None, :, :]          # m = j, e = a
    d2[io, io, :] -= wvo                          # -delta_ij W_iaai
    d2 -= wov[:, None, :]                         # -W_iaia
    # three-body diagonal: -sum_e [2(ie|ja) - (ia|je)] t_ij^ea
    d2 -= 2.0 * einsum("ieja,ijea->ija", ovov, t2) - einsum("iaje,ijea->ija", ovov, t2)
    return np.concatenate([d1, d2.reshape(-1)])


def explicit_matrix(im):
    """Dense Hbar_N assembled block by block from the intermediates.

    Written independently of ``sigma`` (element placement with Kronecker
    deltas rather than contractions), so that comparing the two checks the
    contraction code.
    """
    o, v = im["o"], im["v"]
    D = o + o * o * v
    H = np.zeros((D, D))
    Foo, Fov, Fvv = im["Foo"], im["Fov"], im["Fvv"]
    Wooov, Wovoo, Woooo = im["Wooov"], im["Wovoo"], im["Woooo"]
    Wovvo, Wovov, ovov, t2 = im["Wovvo"], im["Wovov"], im["ovov"], im["t2"]

    def k2(i, j, a):
        return o + (i * o + j) * v + a

    for i in range(o):
        for m in range(o):
            H[i, m] = -Foo[m, i]
        for m in range(o):
            for n in range(o):
                for e in range(v):
                    c = 0.0
                    if m == i:
                        c += 2.0 * Fov[n, e]
                    if n == i:
                        c -= Fov[m, e]
                    c -= 2.0 * Wooov[m, n, i, e] - Wooov[n, m, i, e]
                    H[i, k2(m, n, e)] += c
    d = np.eye(o)
    dv = np.eye(v)
    for i in range(o):
        for j in range(o):
            for a in range(v):
                row = k2(i, j, a)
                for m in range(o):
                    H[row, m] = -Wovoo[m, a, i, j]
                # block over (m, n, e): build the full coefficient tensor
                C = np.zeros((o, o, v))
                C[i, j, :] += Fvv[a, :]
                C[:, j, a] -= Foo[:, i]
                C[i, :, a] -= Foo[:, j]
                C[:, :, a] += Woooo[:, :, i, j]
                C[i, :, :] += 2.0 * Wovvo[:, a, :, j] - Wovov[:, a, j, :]
                C[:, i, :] -= Wovvo[:, a, :, j]
                C[:, j, :] -= Wovov[:, a, i, :]
                # three-body: -sum_e t_ij^ea [2(me|nf) - (mf|ne)]
                te = t2[i, j, :, a]
                C -= 2.0 * np.einsum("e,menf->mnf", te, ovov) - np.einsum("e,mfne->mnf", te, ovov)
                H[row, o:] += C.reshape(-1)
    del d, dv
    return H


# --------------------------------------------------------------------------
# ket and bra of the compact Green's-function expression
# --------------------------------------------------------------------------

def rhs(sys, p):
    """b_p = abar_p |Phi> projected on the 1h + 2h1p space, p in [0, o + v).

    abar_p = e^-T a_p e^T = a_p + [a_p, T]; the next commutator vanishes
    because [a_p, T] only holds occupied annihilators, which commute with T.
    * occupied p: a_p commutes with T, so b_p is the 1h unit vector e_p;
    * virtual p (a = p - o): a_p|Phi> = 0 and [a_p, T]|Phi> gives
      b(1h)[i] = t_i^a and, in the doublet basis, b(2h1p)[i,j,b] = t_ij^ab.
    """
    o, v = sys.n_occ, sys.n_vir
    b = np.zeros(sys.dim)
    if p < o:
        b[p] = 1.0
        return b
    a = p - o
    b[:o] = sys.t1[:, a]
    b[o:] = sys.t2[:, :, a, :].reshape(-1)
    return b


def left_vector(sys, q):
    """c_q[mu] = <Phi|(1 + Lambda) abar_q^+ |mu> (spin-adapted), q in [0, o + v).

    Occupied q: abar_q^+ = a_q^+ - sum_a t_q^a a_a^+ - 1/2 sum_jab t_qj^ab a_a^+ a_b^+ a_j
    (higher commutators vanish).  Spin-summed over the doublet basis:
      c(1h)[i]      = d_qi - sum_a l_ia t_qa - sum_jab (2 l_ij^ab - l_ij^ba) t_qj^ab
      c(2h1p)[k,l,c] = 2 d_qk l_lc - d_ql l_kc - sum_a t_qa (2 l_kl^ac - l_kl^ca)
    Virtual q (a = q - o): a_q^+ commutes with T, so abar_q^+ = a_q^+ and only
    Lambda contributes:
      c(1h)[i] = l_i^a,   c(2h1p)[k,l,c] = 2 l_kl^ac - l_kl^ca
    """
    o, v = sys.n_occ, sys.n_vir
    t1, t2, l1, l2 = sys.t1, sys.t2, sys.l1, sys.l2
    if q >= o:
        a = q - o
        c2 = 2.0 * l2[:, :, a, :] - l2[:, :, :, a]
        return np.concatenate([l1[:, a], c2.reshape(-1)])
    c1 = np.zeros(o)
    c1[q] = 1.0
    c1 -= l1 @ t1[q]
    c1 -= 2.0 * einsum("ijab,jab->i", l2, t2[q]) - einsum("ijba,jab->i", l2, t2[q])
    c2 = np.zeros((o, o, v))
    c2[q, :, :] += 2.0 * l1
    c2[:, q, :] -= l1
    c2 -= 2.0 * einsum("a,klac->klc", t1[q], l2) - einsum("a,klca->klc", t1[q], l2)
    return np.concatenate([c1, c2.reshape(-1)])


# --------------------------------------------------------------------------
# restarted GMRES (Saad & Schultz), complex128, MGS Arnoldi + Givens rotations
# --------------------------------------------------------------------------

def gmres(apply_A, b, tol=1e-12, restart=30, max_iter=2000, precond=None, x0=None,
          history=None):
    """Solve A x = b with right preconditioning ``x = M^-1 u``.

    Convergence is on the true relative residual ``||b - A x|| / ||b||``,
    recomputed at every restart.  Returns ``(x, iters, rel_resid)``.
    ``history`` (a list) receives the Givens residual estimate at each step.
    """
    b = np.asarray(b, dtype=complex)
    n = b.size
    x = np.zeros(n, dtype=complex) if x0 is None else np.array(x0, dtype=complex)
    Minv = (lambda u: u) if precond is None else precond
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    iters = 0
    r = b - apply_A(x)
    beta = np.linalg.norm(r)
    while iters < max_iter:
        if beta / bnorm <= tol:
            break
        m = restart
        V = np.zeros((m + 1, n), dtype=complex)
        Z = np.zeros((m, n), dtype=complex)
        H = np.zeros((m + 1, m), dtype=complex)
        cs = np.zeros(m, dtype=complex)
        sn = np.zeros(m, dtype=complex)
        gvec = np.zeros(m + 1, dtype=complex)
        gvec[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(m):
            Z[k] = Minv(V[k])
            w = apply_A(Z[k])
            for j in range(k + 1):  # modified Gram-Schmidt
                H[j, k] = np.vdot(V[j], w)
                w = w - H[j, k] * V[j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0.0:
                V[k + 1] = w / H[k + 1, k]
            for j in range(k):  # previous rotations
                hj = H[j, k]
                H[j, k] = np.conj(cs[j]) * hj + np.conj(sn[j]) * H[j + 1, k]
                H[j + 1, k] = -sn[j] * hj + cs[j] * H[j + 1, k]
            a, bb = H[k, k], H[k + 1, k]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[k] = a / den if den else 1.0
            sn[k] = bb / den if den else 0.0
            H[k, k] = np.conj(cs[k]) * a + np.conj(sn[k]) * bb
            H[k + 1, k] = 0.0
            gvec[k + 1] = -sn[k] * gvec[k]
            gvec[k] = np.conj(cs[k]) * gvec[k]
            iters += 1
            k_used = k + 1
            if history is not None:
                history.append(abs(gvec[k + 1]) / bnorm)
            if abs(gvec[k + 1]) / bnorm <= tol or iters >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), gvec[:k_used])
        x = x + y @ Z[:k_used]
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
    return x, iters, beta / bnorm


def shifted_operator(im, omega, eta):
    """x -> (omega - i eta) x + Hbar_N x, the operator of the X_p linear system."""
    z = omega - 1j * eta
    return lambda x: z * x + sigma(im, x)


def jacobi(im_diag, omega, eta):
    """Right preconditioner u -> u / (omega - i eta + diag(Hbar_N))."""
    den = (omega - 1j * eta) + im_diag
    return lambda u: u / den


def solve(sys, im, p, omega, eta, tol=1e-12, restart=30, max_iter=5000, precond="jacobi"):
    """X_p(omega) by GMRES; returns (x, iters, rel_resid)."""
    A = shifted_operator(im, omega, eta)
    M = jacobi(diagonal(im), omega, eta) if precond == "jacobi" else None
    return gmres(A, rhs(sys, p), tol=tol, restart=restart, max_iter=max_iter, precond=M)


def greens(sys, im, p, omegas, eta, qs=None, tol=1e-12, restart=30, precond="jacobi"):
    """G[w, k] = c_{q_k}^T X_p(omega_w) (q defaults to [p])."""
    qs = [p] if qs is None else list(qs)
    C = np.stack([left_vector(sys, q) for q in qs])
    out = np.zeros((len(omegas), len(qs)), dtype=complex)
    for w, om in enumerate(omegas):
        x, _, _ = solve(sys, im, p, om, eta, tol=tol, restart=restart, precond=precond)
        out[w] = C @ x
    return out


def spectral_function(G_diag):
    """A(omega) = (1/pi) sum_p Im G_pp for eta > 0 in this sign convention.

    With the operator (omega + Hbar_N - i eta) the retarded poles sit at
    omega = eps - i eta, where Im G > 0; the paper's -(1/pi) Im G refers to the
    +i eta form, so the sign is flipped here to keep A >= 0.
    """
    return np.sum(np.imag(G_diag), axis=-1) / np.pi
