"""O1: Fock-space brute force for the IP part of the GFCCSD Green's function.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Nothing here uses coupled-cluster working equations.  For a tiny closed-shell
system it builds, as dense matrices over Slater determinants,

* the electronic Hamiltonian ``H = sum h_PQ P^+ Q + 1/4 sum <PQ||RS> P^+ Q^+ S R``
  with ``h = f - sum_K <PK||QK>`` so that the Fock operator of the reference
  determinant is ``f = diag(eps)``;
* the cluster operator ``T = T1 + T2`` and ``Lambda = Lambda1 + Lambda2``
  (paper, Theory: T, Lambda truncated at the two-body level, GFCCSD);
* ``exp(+-T)`` by the finite power series (T is nilpotent).

It then forms, for every basis operator ``R_mu`` of the 1h + 2h1p ionised
space (paper, Theory, expansion of X_p: one-hole ``a_i`` and two-hole
one-particle ``a_a^+ a_j a_i`` terms),

* the connected similarity-transformed Hamiltonian matrix
  ``Hbar[mu', mu] = <mu'| [Hbar, R_mu] |Phi>`` with ``Hbar = e^-T H e^T``
  (E0 cancels in the commutator, so this is the normal-product ``Hbar_N``
  of the paper acting on the ionised space),
* the ket ``b_p[mu] = <mu| e^-T a_p e^T |Phi>`` (right-hand side of the
  linear system for X_p),
* the bra ``c_q[mu] = <Phi| (1 + Lambda) e^-T a_q^+ e^T |mu>`` (the
  left vector of the compact Green's-function expression).

Spin orbitals: index ``P`` has spatial orbital ``P % n`` and spin ``P // n``
(0 = alpha, 1 = beta).  The ionised space removes one alpha electron.  The
spin-adapted basis used by the matrix-free oracle is reached through the
explicit maps ``embed``/``extract`` below (doublet states):

* ``r_i``      <-> coefficient of ``a_{i alpha}``
* ``r_ija``    <-> coefficient of ``a^+_{a beta} a_{j beta} a_{i alpha}``
* the same-spin component is ``r_ija - r_jia`` on ``a^+_{a alpha} a_{j alpha} a_{i alpha}`` (i < j).
"""
from __future__ import annotations

from itertools import combinations

import numpy as np


def _parity_below(det: int, P: int) -> int:
    return -1 if bin(det & ((1 << P) - 1)).count("1") & 1 else 1


def apply_string(ops, det):
    """Apply operators right-to-left as listed in ``ops`` (application order).

    ``ops`` is a sequence of ``(dagger, P)``.  Returns ``(sign, det)`` or
    ``(0, None)`` if the result vanishes.
    """
    sign = 1
    for dag, P in ops:
        bit = 1 << P
        if dag:
            if det & bit:
                return 0, None
            sign *= _parity_below(det, P)
            det |= bit
        else:
            if not det & bit:
                return 0, None
            sign *= _parity_below(det, P)
            det ^= bit
    return sign, det


def sector(n: int, n_alpha: int, n_beta: int):
    """All determinants with the given alpha/beta electron counts."""
    dets = []
    for a in combinations(range(n), n_alpha):
        amask = sum(1 << p for p in a)
        for b in combinations(range(n), n_beta):
            dets.append(amask | sum(1 << (n + p) for p in b))
    dets.sort()
    return dets, {d: k for k, d in enumerate(dets)}


def op_matrix(terms, dets_in, idx_out):
    """Dense matrix of ``sum coef * string`` from sector ``dets_in`` to ``idx_out``."""
    M = np.zeros((len(idx_out), len(dets_in)))
    for col, d in enumerate(dets_in):
        for coef, ops in terms:
            s, d2 = apply_string(ops, d)
            if s:
                M[idx_out[d2], col] += s * coef
    return M


class SpinOrbitalSystem:
    """Spin-orbital integrals and amplitudes built from the spatial inputs."""

    def __init__(self, o, v, eps, L, t1, t2, l1, l2):
        self.o, self.v, self.n = o, v, o + v
        n = self.n
        N = 2 * n
        g = np.einsum("Qpq,Qrs->pqrs", L, L)  # chemist (pq|rs), spatial
        spat = np.arange(N) % n
        spin = np.arange(N) // n
        same = spin[:, None] == spin[None, :]
        # <PQ|RS> = (PR|QS) delta(sP,sR) delta(sQ,sS)
        phys = g[np.ix_(spat, spat, spat, spat)].transpose(0, 2, 1, 3)
        phys = phys * same[:, None, :, None] * same[None, :, None, :]
        self.A = phys - phys.transpose(0, 1, 3, 2)  # <PQ||RS>
        occ = [P for P in range(N) if spat[P] < o]
        f = np.diag(eps[spat])
        self.h = f - sum(self.A[:, K, :, K] for K in occ)
        self.occ_so = occ
        self.vir_so = [P for P in range(N) if spat[P] >= o]

        def t1so(I, A_):
            if spin[I] != spin[A_]:
                return 0.0
            return t1[spat[I], spat[A_] - o]

        def t2so(amp, I, J, A_, B):
            val = 0.0
            i, j, a, b = spat[I], spat[J], spat[A_] - o, spat[B] - o
            if spin[I] == spin[A_] and spin[J] == spin[B]:
                val += amp[i, j, a, b]
            if spin[I] == spin[B] and spin[J] == spin[A_]:
                val -= amp[i, j, b, a]
            return val

        self.t1so, self.t2so = t1so, t2so
        self.t1, self.t2, self.l1, self.l2 = t1, t2, l1, l2
        self.spin, self.spat = spin, spat

    def hamiltonian(self, dets, idx):
        """Dense H over one sector (one- and two-body parts, exact)."""
        N = 2 * self.n
        H = np.zeros((len(dets), len(dets)))
        h, A = self.h, self.A
        for col, d in enumerate(dets):
            occ = [P for P in range(N) if d >> P & 1]
            for Q in occ:
                s1, d1 = apply_string([(False, Q)], d)
                for P in range(N):
                    if h[P, Q] == 0.0:
                        continue
                    s2, d2 = apply_string([(True, P)], d1)
                    if s2:
                        H[idx[d2], col] += s1 * s2 * h[P, Q]
            for R, S in combinations(occ, 2):
                s1, d2 = apply_string([(False, R), (False, S)], d)
                free = [P for P in range(N) if not d2 >> P & 1]
                for P, Q in combinations(free, 2):
                    val = A[P, Q, R, S]
                    if val == 0.0:
                        continue
                    s2, d4 = apply_string([(True, Q), (True, P)], d2)
                    H[idx[d4], col] += s1 * s2 * val
        return H

    def cluster_terms(self, which="T"):
        """Operator strings of T (excitation) or Lambda (de-excitation)."""
        terms = []
        amp1 = self.t1 if which == "T" else self.l1
        amp2 = self.t2 if which == "T" else self.l2
        spin, spat, o = self.spin, self.spat, self.o
        for I in self.occ_so:
            for A_ in self.vir_so:
                if spin[I] != spin[A_]:
                    continue
                c = amp1[spat[I], spat[A_] - o]
                if c != 0.0:
                    if which == "T":  # t_I^A A^+ I
                        terms.append((c, [(False, I), (True, A_)]))
                    else:  # lambda_A^I I^+ A
                        terms.append((c, [(False, A_), (True, I)]))
        for I, J in combinations(self.occ_so, 2):
            for A_, B in combinations(self.vir_so, 2):
                c = self.t2so(amp2, I, J, A_, B)
                if c != 0.0:
                    if which == "T":  # t_IJ^AB A^+ B^+ J I
                        terms.append((c, [(False, I), (False, J), (True, B), (True, A_)]))
                    else:  # lambda_AB^IJ I^+ J^+ B A
                        terms.append((c, [(False, A_), (False, B), (True, J), (True, I)]))
        return terms


def _expm_nilpotent(T):
    E = np.eye(T.shape[0])
    term = np.eye(T.shape[0])
    k = 1
    while True:
        term = term @ T / k
        if not np.any(term):
            return E
        E = E + term
        k += 1
        if k > 64:
            raise RuntimeError("cluster operator is not nilpotent")


class IPBruteForce:
    """Dense IP-GFCCSD quantities for one tiny system (o <= 3, v <= 5 advised)."""

    def __init__(self, sysobj):
        o, v = sysobj.n_occ, sysobj.n_vir
        n = o + v
        self.o, self.v, self.n = o, v, n
        so = SpinOrbitalSystem(o, v, sysobj.eps, sysobj.L, sysobj.t1, sysobj.t2,
                               sysobj.l1, sysobj.l2)
        self.so = so
        detsN, idxN = sector(n, o, o)
        detsM, idxM = sector(n, o - 1, o)
        self.detsN, self.idxN, self.detsM, self.idxM = detsN, idxN, detsM, idxM
        phi_det = sum(1 << p for p in range(o)) | sum(1 << (n + p) for p in range(o))
        phi = np.zeros(len(detsN))
        phi[idxN[phi_det]] = 1.0

        HN = so.hamiltonian(detsN, idxN)
        HM = so.hamiltonian(detsM, idxM)
        Tt = so.cluster_terms("T")
        TN = op_matrix(Tt, detsN, idxN)
        TM = op_matrix(Tt, detsM, idxM)
        LamN = op_matrix(so.cluster_terms("L"), detsN, idxN)
        eTN, emTN = _expm_nilpotent(TN), _expm_nilpotent(-TN)
        eTM, emTM = _expm_nilpotent(TM), _expm_nilpotent(-TM)
        HbN = emTN @ HN @ eTN
        HbM = emTM @ HM @ eTM

        # ionised basis: 1h (i alpha) then 2h1p in two spin blocks
        basis = [("1h", i) for i in range(o)]
        basis += [("aaa", i, j, a) for i in range(o) for j in range(i + 1, o) for a in range(v)]
        basis += [("abb", i, j, a) for i in range(o) for j in range(o) for a in range(v)]
        self.basis = basis
        ops = []
        for b in basis:
            if b[0] == "1h":
                ops.append([(False, b[1])])
            elif b[0] == "aaa":
                _, i, j, a = b
                ops.append([(False, i), (False, j), (True, o + a)])
            else:
                _, i, j, a = b
                ops.append([(False, i), (False, n + j), (True, n + o + a)])
        Rmats = [op_matrix([(1.0, s)], detsN, idxM) for s in ops]
        evec = np.stack([R @ phi for R in Rmats], axis=1)  # [dimM, Dso], +-unit columns
        self.evec = evec
        HbNphi = HbN @ phi
        Dso = len(basis)
        Hso = np.zeros((Dso, Dso))
        for mu, R in enumerate(Rmats):
            sig = HbM @ evec[:, mu] - R @ HbNphi
            Hso[:, mu] = evec.T @ sig
        self.Hso = Hso

        # b_p and c_q for every alpha spin orbital (occupied p < o, virtual p >= o)
        self.b_so = np.zeros((n, Dso))
        self.c_so = np.zeros((n, Dso))
        for p in range(n):
            Ap = op_matrix([(1.0, [(False, p)])], detsN, idxM)
            self.b_so[p] = evec.T @ (emTM @ Ap @ eTN @ phi)
            Aqd = op_matrix([(1.0, [(True, p)])], detsM, idxN)
            row = phi @ (np.eye(len(detsN)) + LamN) @ emTN @ Aqd @ eTM
            self.c_so[p] = row @ evec

        # spin-adaptation maps
        D = o + o * o * v
        E = np.zeros((Dso, D))
        X = np.zeros((D, Dso))
        for mu, b in enumerate(basis):
            if b[0] == "1h":
                E[mu, b[1]] = 1.0
                X[b[1], mu] = 1.0
            elif b[0] == "abb":
                _, i, j, a = b
                k = o + (i * o + j) * v + a
                E[mu, k] = 1.0
                X[k, mu] = 1.0
            else:
                _, i, j, a = b
                E[mu, o + (i * o + j) * v + a] += 1.0
                E[mu, o + (j * o + i) * v + a] -= 1.0
        self.E, self.X = E, X
        self.Hsa = X @ Hso @ E
        self.b_sa = self.b_so @ X.T
        self.c_sa = self.c_so @ E

    def doublet_leak(self) -> float:
        """max |(1 - E X) Hso E|: zero iff the doublet space is Hbar-invariant."""
        P = self.E @ self.X
        return float(np.max(np.abs(self.Hso @ self.E - P @ self.Hso @ self.E)))

    def greens_so(self, omega, eta, p, q):
        """G_qp(omega) = c_q^T (omega - i eta + Hbar)^-1 b_p in the spin-orbital space."""
        A = (omega - 1j * eta) * np.eye(self.Hso.shape[0]) + self.Hso
        return self.c_so[q] @ np.linalg.solve(A, self.b_so[p])

    def greens_sa(self, omega, eta, p, q):
        A = (omega - 1j * eta) * np.eye(self.Hsa.shape[0]) + self.Hsa
        return self.c_sa[q] @ np.linalg.solve(A, self.b_sa[p])


class EABruteForce:
    """Dense EA-GFCCSD quantities (the advanced, electron-attached term of G) for one tiny
    system, from the same determinant matrices as the IP part.

    Paper, Theory: the second term of the GFCC Green's function,
    ``G^EA_pq = <Phi|(1 + Lambda) abar_p (omega - Hbar_N + i eta)^-1 abar_q^+ |Phi>``, solved
    through ``(omega - Hbar_N + i eta) Y_q |Phi> = abar_q^+ |Phi>`` with Y_q expanded in
    one-particle ``a_a^+`` and two-particle one-hole ``a_a^+ a_b^+ a_i`` operators.
    For every basis operator ``R_mu`` of the 1p + 2p1h space (one extra alpha electron):

    * ``Hbar[mu', mu] = <mu'| [Hbar, R_mu] |Phi>`` (connected form),
    * ``b_q[mu] = <mu| e^-T a_q^+ e^T |Phi>``,
    * ``c_p[mu] = <Phi| (1 + Lambda) e^-T a_p e^T |mu>``.

    Spin-adapted basis (doublet, reached through ``E``/``X``):

    * ``y_a``      <-> coefficient of ``a^+_{a alpha}``
    * ``y_jab``    <-> coefficient of ``a^+_{a alpha} a^+_{b beta} a_{j beta}``
    * the same-spin component is ``y_jab - y_jba`` on ``a^+_{a alpha} a^+_{b alpha} a_{j alpha}`` (a < b).
    Layout: ``y[0:v] = y_a``, ``y[v + (j*v + a)*v + b] = y_jab``.
    """

    def __init__(self, sysobj):
        o, v = sysobj.n_occ, sysobj.n_vir
        n = o + v
        self.o, self.v, self.n = o, v, n
        so = SpinOrbitalSystem(o, v, sysobj.eps, sysobj.L, sysobj.t1, sysobj.t2, sysobj.l1, sysobj.l2)
        self.so = so
        detsN, idxN = sector(n, o, o)
        detsP, idxP = sector(n, o + 1, o)
        phi_det = sum(1 << p for p in range(o)) | sum(1 << (n + p) for p in range(o))
        phi = np.zeros(len(detsN))
        phi[idxN[phi_det]] = 1.0
        HN = so.hamiltonian(detsN, idxN)
        HP = so.hamiltonian(detsP, idxP)
        Tt = so.cluster_terms("T")
        TN = op_matrix(Tt, detsN, idxN)
        TP = op_matrix(Tt, detsP, idxP)
        LamN = op_matrix(so.cluster_terms("L"), detsN, idxN)
        eTN, emTN = _expm_nilpotent(TN), _expm_nilpotent(-TN)
        eTP, emTP = _expm_nilpotent(TP), _expm_nilpotent(-TP)
        HbN = emTN @ HN @ eTN
        HbP = emTP @ HP @ eTP

        basis = [("1p", a) for a in range(v)]
        basis += [("aaa", j, a, b) for j in range(o) for a in range(v) for b in range(a + 1, v)]
        basis += [("abb", j, a, b) for j in range(o) for a in range(v) for b in range(v)]
        self.basis = basis
        ops = []
        for bb in basis:
            if bb[0] == "1p":
                ops.append([(True, o + bb[1])])
            elif bb[0] == "aaa":
                _, j, a, b = bb
                ops.append([(False, j), (True, o + b), (True, o + a)])
            else:
                _, j, a, b = bb
                ops.append([(False, n + j), (True, n + o + b), (True, o + a)])
        Rmats = [op_matrix([(1.0, sq)], detsN, idxP) for sq in ops]
        evec = np.stack([R @ phi for R in Rmats], axis=1)
        HbNphi = HbN @ phi
        Dso = len(basis)
        Hso = np.zeros((Dso, Dso))
        for mu, R in enumerate(Rmats):
            sig = HbP @ evec[:, mu] - R @ HbNphi
            Hso[:, mu] = evec.T @ sig
        self.Hso = Hso

        self.b_so = np.zeros((n, Dso))
        self.c_so = np.zeros((n, Dso))
        for p in range(n):
            Cq = op_matrix([(1.0, [(True, p)])], detsN, idxP)
            self.b_so[p] = evec.T @ (emTP @ Cq @ eTN @ phi)
            Ap = op_matrix([(1.0, [(False, p)])], detsP, idxN)
            row = phi @ (np.eye(len(detsN)) + LamN) @ emTN @ Ap @ eTP
            self.c_so[p] = row @ evec

        D = v + o * v * v
        E = np.zeros((Dso, D))
        X = np.zeros((D, Dso))
        for mu, bb in enumerate(basis):
            if bb[0] == "1p":
                E[mu, bb[1]] = 1.0
                X[bb[1], mu] = 1.0
            elif bb[0] == "abb":
                _, j, a, b = bb
                k = v + (j * v + a) * v + b
                E[mu, k] = 1.0
                X[k, mu] = 1.0
            else:
                _, j, a, b = bb
                E[mu, v + (j * v + a) * v + b] += 1.0
                E[mu, v + (j * v + b) * v + a] -= 1.0
        self.E, self.X = E, X
        self.Hsa = X @ Hso @ E
        self.b_sa = self.b_so @ X.T
        self.c_sa = self.c_so @ E

    def doublet_leak(self) -> float:
        P = self.E @ self.X
        return float(np.max(np.abs(self.Hso @ self.E - P @ self.Hso @ self.E)))

    def greens_so(self, omega, eta, p, q):
        """G^EA_pq(omega) = c_p^T (omega + i eta - Hbar)^-1 b_q in the spin-orbital space."""
        A = (omega + 1j * eta) * np.eye(self.Hso.shape[0]) - self.Hso
        return self.c_so[p] @ np.linalg.solve(A, self.b_so[q])

    def greens_sa(self, omega, eta, p, q):
        A = (omega + 1j * eta) * np.eye(self.Hsa.shape[0]) - self.Hsa
        return self.c_sa[p] @ np.linalg.solve(A, self.b_sa[q])
