"""Seeded synthetic closed-shell systems for the IP-GFCCSD linear-solve path.

This module is the ONLY code shared by the CPU oracle (``oracle/``) and the
GPU library's tests/benchmarks.  It draws random numbers and forms the MP2
amplitudes that stand in for converged CCSD amplitudes; it contains none of
the Green's-function arithmetic (no similarity-transformed Hamiltonian, no
sigma product, no left vectors, no solver).

Recipe (one ``numpy.random.Generator(PCG64(seed))`` stream, drawn in this
order):

1. ``eps_occ ~ U(-1.2, -0.3)`` (n_occ values), ``eps_vir ~ U(0.1, 2.0)``
   (n_vir values), each block sorted ascending.
2. Cholesky vectors ``L[Q, p, q]`` symmetric in (p, q): the upper triangle
   including the diagonal is drawn i.i.d. ``N(0, sigma_L^2)`` and mirrored.
3. ``T1[i, a] ~ N(0, sigma_T1^2)``.
4. ``T2[i, j, a, b] = (ia|jb) / (e_i + e_j - e_a - e_b)`` with chemist
   integrals ``(pq|rs) = sum_Q L[Q,p,q] L[Q,r,s]`` (MP2 amplitudes; pair
   symmetric ``T2[i,j,a,b] = T2[j,i,b,a]``).
5. ``Lambda = T^dagger``: ``l1 = T1``, ``l2 = T2`` (same index layout).
6. Frequencies ``omega = linspace(w_min, w_max, n_omega)`` (both ends).

Orbital energies are Hartree.  The Fock matrix of the reference is
``diag(eps)``; occupied orbitals come first.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 2010_04768


@dataclasses.dataclass
class System:
    """One synthetic closed-shell system (all arrays float64, C-contiguous)."""

    n_occ: int
    n_vir: int
    n_chol: int
    eps: np.ndarray  # [n_occ + n_vir]
    L: np.ndarray  # [n_chol, n, n]
    t1: np.ndarray  # [n_occ, n_vir]
    t2: np.ndarray  # [n_occ, n_occ, n_vir, n_vir]
    l1: np.ndarray  # [n_occ, n_vir]
    l2: np.ndarray  # [n_occ, n_occ, n_vir, n_vir]
    seed: int

    @property
    def n(self) -> int:
        return self.n_occ + self.n_vir

    @property
    def dim(self) -> int:
        """Dimension of the spin-adapted 1h + 2h1p space: o + o*o*v."""
        return self.n_occ + self.n_occ * self.n_occ * self.n_vir


def make_system(n_occ: int, n_vir: int, n_chol: int, seed: int, *,
                sigma_L: float = 0.05, sigma_t1: float = 1e-3,
                occ_range=(-1.2, -0.3), vir_range=(0.1, 2.0),
                t1: bool = True, t2: bool = True, lam: bool = True,
                L_zero: bool = False) -> System:
    """Draw one system.  Switches zero whole amplitude classes (for pins)."""
    o, v, Q = int(n_occ), int(n_vir), int(n_chol)
    n = o + v
    rng = np.random.Generator(np.random.PCG64(seed))
    e_occ = np.sort(rng.uniform(occ_range[0], occ_range[1], size=o))
    e_vir = np.sort(rng.uniform(vir_range[0], vir_range[1], size=v))
    eps = np.concatenate([e_occ, e_vir])

    iu, ju = np.triu_indices(n)
    L = np.zeros((Q, n, n))
    vals = rng.normal(0.0, sigma_L, size=(Q, iu.size))
    L[:, iu, ju] = vals
    L[:, ju, iu] = vals
    del vals
    if L_zero:
        L[:] = 0.0

    T1 = rng.normal(0.0, sigma_t1, size=(o, v))
    if not t1:
        T1[:] = 0.0

    if t2:
        Lov = np.ascontiguousarray(L[:, :o, o:]).reshape(Q, o * v)
        iajb = (Lov.T @ Lov).reshape(o, v, o, v)
        den = (e_occ[:, None, None, None] + e_occ[None, None, :, None]
               - e_vir[None, :, None, None] - e_vir[None, None, None, :])
        T2 = np.ascontiguousarray((iajb / den).transpose(0, 2, 1, 3))
        del iajb, den
    else:
        T2 = np.zeros((o, o, v, v))

    if lam:
        l1 = T1.copy()
        l2 = T2.copy()
    else:
        l1 = np.zeros_like(T1)
        l2 = np.zeros_like(T2)
    return System(o, v, Q, eps, L, T1, T2, l1, l2, seed)


def make_system_device(n_occ: int, n_vir: int, n_chol: int, seed: int, device, *,
                       sigma_L: float = 0.05, sigma_t1: float = 1e-3,
                       occ_range=(-1.2, -0.3), vir_range=(0.1, 2.0), chunk_bytes: float = 2e9):
    """The recipe of ``make_system`` (same draws, same order) with the large arrays formed
    as torch tensors on ``device``: the random numbers come from the same numpy PCG64 stream,
    L is assembled from them on the device and T2 is formed there in blocks of occupied i
    (the 120/600/3000 system's T2 is 41.5 GB).  Lambda = T^dagger.  Returns a dict with
    float64 tensors eps, L, t1, t2 and the dimensions."""
    import torch
    o, v, Q = int(n_occ), int(n_vir), int(n_chol)
    n = o + v
    rng = np.random.Generator(np.random.PCG64(seed))
    e_occ = np.sort(rng.uniform(occ_range[0], occ_range[1], size=o))
    e_vir = np.sort(rng.uniform(vir_range[0], vir_range[1], size=v))
    eps = np.concatenate([e_occ, e_vir])
    iu, ju = np.triu_indices(n)
    vals = rng.normal(0.0, sigma_L, size=(Q, iu.size))
    T1 = rng.normal(0.0, sigma_t1, size=(o, v))
    dev = torch.device(device)
    L = torch.zeros((Q, n, n), dtype=torch.float64, device=dev)
    iu_t = torch.as_tensor(iu, device=dev)
    ju_t = torch.as_tensor(ju, device=dev)
    q0 = 0
    qc = max(1, int(chunk_bytes // max(1, iu.size * 8)))
    while q0 < Q:  # upload the draws in blocks of Q
        q1 = min(Q, q0 + qc)
        blk = torch.from_numpy(vals[q0:q1]).to(dev)
        L[q0:q1, iu_t, ju_t] = blk
        L[q0:q1, ju_t, iu_t] = blk
        q0 = q1
        del blk
    del vals
    eo = torch.from_numpy(e_occ).to(dev)
    ev = torch.from_numpy(e_vir).to(dev)
    Lov = L[:, :o, o:].reshape(Q, o * v)
    T2 = torch.empty((o, o, v, v), dtype=torch.float64, device=dev)
    ci = max(1, int(chunk_bytes // max(1, v * o * v * 8 * 3)))
    for i0 in range(0, o, ci):  # T2[i, j, a, b] = (ia|jb) / (e_i + e_j - e_a - e_b)
        i1 = min(o, i0 + ci)
        iajb = (Lov[:, i0 * v:i1 * v].T @ Lov).reshape(i1 - i0, v, o, v)
        den = (eo[i0:i1, None, None, None] + eo[None, None, :, None]
               - ev[None, :, None, None] - ev[None, None, None, :])
        T2[i0:i1] = (iajb / den).permute(0, 2, 1, 3)
        del iajb, den
    return dict(n_occ=o, n_vir=v, n_chol=Q, seed=seed,
                eps=torch.from_numpy(eps).to(dev), L=L, t1=torch.from_numpy(T1).to(dev), t2=T2)


@dataclasses.dataclass
class Workload:
    """A named workload: one or more systems plus the (p, omega) grid."""

    name: str
    systems: List[System]
    omegas: List[np.ndarray]
    p_lists: List[np.ndarray]
    eta: float
    tol: float
    restart: int

    @property
    def n_rhs(self) -> int:
        return int(sum(len(w) * len(p) for w, p in zip(self.omegas, self.p_lists)))


def _highest(n_occ: int, k: int) -> np.ndarray:
    return np.arange(max(0, n_occ - k), n_occ, dtype=np.int64)


# Workload shapes (o, v, Q, n_omega, omega range, eta, p selection, tol).
WORKLOADS = {
    "tiny-o4v16": dict(shapes=[(4, 16, 48)], n_omega=6, w=(-1.0, -0.2), eta=0.01,
                       p="all", tol=1e-10, restart=30, seed_off=[1]),
    "plain-o40v200": dict(shapes=[(40, 200, 800)], n_omega=64, w=(-1.2, -0.3), eta=0.01,
                          p="all", tol=1e-8, restart=30, seed_off=[2]),
    "mixed-3sys": dict(shapes=[(20, 100, 400), (40, 180, 720), (60, 300, 1200)], n_omega=128,
                       w=(-1.2, -0.3), eta=0.01, p="all", tol=1e-8, restart=30,
                       seed_off=[31, 32, 33]),
    "learned-o90v420": dict(shapes=[(90, 420, 1800)], n_omega=256, w=(-1.2, -0.3), eta=0.005,
                            p=30, tol=1e-8, restart=30, seed_off=[4]),
    # supplementary variant of the 90/420/1800 system (not a substitute for it): sigma_L scaled by
    # (o v^2 Q / 49152)^(-1/4), which keeps the dressing of the occupied Fock block at the level of
    # the 4/16/48 system, so that restarted GMRES converges and preconditioners can be compared
    "learned-o90v420-scaled": dict(shapes=[(90, 420, 1800)], n_omega=256, w=(-1.2, -0.3), eta=0.005,
                                   p=30, tol=1e-8, restart=30, seed_off=[4],
                                   sigma_L=0.05 * (90 * 420 ** 2 * 1800 / 49152) ** -0.25),
    "c60-o120v600": dict(shapes=[(120, 600, 3000)], n_omega=400, w=(-1.2, -0.3), eta=0.005,
                         p=30, tol=1e-8, restart=30, seed_off=[5]),
}


def make_workload(name: str, n_omega: Optional[int] = None,
                  shapes: Optional[Sequence] = None) -> Workload:
    """Build a named workload; ``n_omega``/``shapes`` override for reduced tests."""
    spec = WORKLOADS[name]
    shp = list(shapes) if shapes is not None else spec["shapes"]
    nw = spec["n_omega"] if n_omega is None else int(n_omega)
    systems, omegas, plists = [], [], []
    for (o, v, Q), off in zip(shp, spec["seed_off"]):
        systems.append(make_system(o, v, Q, BASE_SEED + off, sigma_L=spec.get("sigma_L", 0.05)))
        omegas.append(np.linspace(spec["w"][0], spec["w"][1], nw))
        plists.append(np.arange(o, dtype=np.int64) if spec["p"] == "all"
                      else _highest(o, spec["p"]))
    return Workload(name, systems, omegas, plists, spec["eta"], spec["tol"], spec["restart"])


def random_vectors(n_vec: int, dim: int, seed: int) -> np.ndarray:
    """Complex128 test vectors [n_vec, dim] with N(0,1) real and imaginary parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=(n_vec, dim)) + 1j * rng.normal(size=(n_vec, dim))


# ------------------------------------------------------------------ open-shell (spin-unrestricted) systems

@dataclasses.dataclass
class OpenShellSystem:
    """One synthetic spin-unrestricted system in spin blocks (float64, C-contiguous).

    n spatial orbitals per spin; n_occ_a alpha and n_occ_b beta electrons (n_occ_a >= n_occ_b).
    Chemist integrals between orbitals of spins s and s' are (pq|rs) = sum_Q L_s[Q,p,q] L_s'[Q,r,s].
    Amplitudes: t1a [oa][va], t1b [ob][vb], t2aa [oa][oa][va][va] and t2bb (antisymmetric in the
    occupied and in the virtual pair), t2ab [oa][ob][va][vb] (t_{i alpha j beta}^{a alpha b beta});
    the l's in the same layouts."""

    n: int
    n_occ_a: int
    n_occ_b: int
    n_chol: int
    eps_a: np.ndarray
    eps_b: np.ndarray
    La: np.ndarray
    Lb: np.ndarray
    t1a: np.ndarray
    t1b: np.ndarray
    t2aa: np.ndarray
    t2ab: np.ndarray
    t2bb: np.ndarray
    l1a: np.ndarray
    l1b: np.ndarray
    l2aa: np.ndarray
    l2ab: np.ndarray
    l2bb: np.ndarray
    seed: int

    @property
    def n_vir_a(self) -> int:
        return self.n - self.n_occ_a

    @property
    def n_vir_b(self) -> int:
        return self.n - self.n_occ_b

    @property
    def n_occ(self) -> int:
        """Occupied spin orbitals."""
        return self.n_occ_a + self.n_occ_b

    @property
    def n_vir(self) -> int:
        """Virtual spin orbitals."""
        return self.n_vir_a + self.n_vir_b

    @property
    def dim(self) -> int:
        """Spin-orbital 1h + 2h1p space with both (i, j) orders stored: o + o*o*v."""
        return self.n_occ + self.n_occ * self.n_occ * self.n_vir


def make_open_shell_system(n: int, n_occ_a: int, n_occ_b: int, n_chol: int, seed: int, *,
                           sigma_L: float = 0.05, sigma_dL: float = 0.02, sigma_t1: float = 1e-3,
                           occ_range=(-1.2, -0.3), vir_range=(0.1, 2.0),
                           t1: bool = True, t2: bool = True, lam: bool = True,
                           L_zero: bool = False) -> OpenShellSystem:
    """Draw one open-shell system.  Recipe (one PCG64(seed) stream, in this order):

    1. eps_a: n_occ_a occupied ~ U(occ_range), n - n_occ_a virtual ~ U(vir_range), each sorted;
       eps_b likewise with n_occ_b.
    2. La symmetric in (p, q), upper triangle i.i.d. N(0, sigma_L^2); Lb = La + a symmetric
       N(0, sigma_dL^2) perturbation (the beta orbitals differ from the alpha ones).
    3. t1a ~ N(0, sigma_t1^2), then t1b.
    4. T2 = MP2 amplitudes <ij||ab> / (e_i + e_j - e_a - e_b) per spin block:
       aa: (ia|jb) - (ib|ja) from La; bb from Lb; ab: (ia|jb) with (ia) from La, (jb) from Lb.
    5. Lambda = T^dagger (the l's are copies)."""
    if not (1 <= n_occ_b <= n_occ_a < n):
        raise ValueError("need 1 <= n_occ_b <= n_occ_a < n")
    oa, ob, Q = int(n_occ_a), int(n_occ_b), int(n_chol)
    va, vb = n - oa, n - ob
    rng = np.random.Generator(np.random.PCG64(seed))

    def energies(o):
        eo = np.sort(rng.uniform(occ_range[0], occ_range[1], size=o))
        ev = np.sort(rng.uniform(vir_range[0], vir_range[1], size=n - o))
        return np.concatenate([eo, ev])

    eps_a = energies(oa)
    eps_b = energies(ob)
    iu, ju = np.triu_indices(n)

    def sym(sig):
        M = np.zeros((Q, n, n))
        vals = rng.normal(0.0, sig, size=(Q, iu.size))
        M[:, iu, ju] = vals
        M[:, ju, iu] = vals
        return M

    La = sym(sigma_L)
    Lb = La + sym(sigma_dL)
    if L_zero:
        La[:] = 0.0
        Lb[:] = 0.0
    T1a = rng.normal(0.0, sigma_t1, size=(oa, va))
    T1b = rng.normal(0.0, sigma_t1, size=(ob, vb))
    if not t1:
        T1a[:] = 0.0
        T1b[:] = 0.0

    def ovov(L1, o1, L2, o2):
        A = L1[:, :o1, o1:].reshape(Q, -1)
        B = L2[:, :o2, o2:].reshape(Q, -1)
        return (A.T @ B).reshape(o1, n - o1, o2, n - o2)  # (ia|jb)

    def denom(e1, o1, e2, o2):
        return (e1[:o1, None, None, None] + e2[None, None, :o2, None]
                - e1[None, o1:, None, None] - e2[None, None, None, o2:])  # [i, a, j, b]

    if t2:
        g = ovov(La, oa, La, oa)
        T2aa = ((g - g.transpose(0, 3, 2, 1)) / denom(eps_a, oa, eps_a, oa)).transpose(0, 2, 1, 3)
        g = ovov(Lb, ob, Lb, ob)
        T2bb = ((g - g.transpose(0, 3, 2, 1)) / denom(eps_b, ob, eps_b, ob)).transpose(0, 2, 1, 3)
        g = ovov(La, oa, Lb, ob)
        T2ab = (g / denom(eps_a, oa, eps_b, ob)).transpose(0, 2, 1, 3)
    else:
        T2aa = np.zeros((oa, oa, va, va))
        T2bb = np.zeros((ob, ob, vb, vb))
        T2ab = np.zeros((oa, ob, va, vb))
    T2aa, T2ab, T2bb = (np.ascontiguousarray(x) for x in (T2aa, T2ab, T2bb))
    amps = [T1a, T1b, T2aa, T2ab, T2bb]
    lams = [x.copy() for x in amps] if lam else [np.zeros_like(x) for x in amps]
    return OpenShellSystem(n, oa, ob, Q, eps_a, eps_b, La, Lb, *amps, *lams, seed)
