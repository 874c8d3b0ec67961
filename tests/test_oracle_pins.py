"""Pins of the CPU oracle against things other than itself (no GPU).

* O1 (Fock-space brute force) against closed forms at T = Lambda = L = 0.
* O2 (derived spin-adapted equations) against O1, one amplitude class at a
  time, for the similarity-transformed Hamiltonian, its diagonal, the left
  vectors (with Lambda independent of T) and G itself.
* Closed forms / invariants: G_ii = 1/(omega - eps_i - i eta) at T = Lambda = L = 0;
  fourth-order onset of the self-energy in L; G(-eta) = conj G(eta); linearity
  of G in Lambda; Lambda = 0 gives c_q = e_q; Schur-complement identity.
* GMRES against a dense direct solve; residual monotone within a cycle and
  convergence in at most dim steps without restart (paper, GFCC Workflow and Bottlenecks).
"""
import numpy as np
import pytest

from synth import make_system, make_workload
from oracle import ipgfcc as O
from oracle.fockspace import IPBruteForce


def _dense(im):
    D = im["o"] + im["o"] ** 2 * im["v"]
    return O.sigma(im, np.eye(D)).T


def _sys(o, v, seed, **kw):
    return make_system(o, v, 5, seed, sigma_L=0.3, sigma_t1=0.08, **kw)


CLASSES = {
    "bare": dict(t1=False, t2=False, lam=False),
    "t1": dict(t2=False),
    "t2": dict(t1=False),
    "t1t2": dict(),
}


@pytest.fixture(scope="module")
def bf_cache():
    return {}


def _bf(cache, key, s):
    if key not in cache:
        cache[key] = IPBruteForce(s)
    return cache[key]


# ---------------------------------------------------------------- O1 closed forms

def test_bruteforce_free_particles():
    """T = Lambda = L = 0: Hbar is diagonal with -eps_i (1h) and eps_a - eps_i - eps_j (2h1p)."""
    o, v = 3, 3
    s = make_system(o, v, 4, 11, t1=False, t2=False, lam=False, L_zero=True)
    bf = IPBruteForce(s)
    e = s.eps
    ref = [-e[i] for i in range(o)]
    ref += [e[o + a] - e[i] - e[j] for i in range(o) for j in range(o) for a in range(v)]
    assert np.allclose(bf.Hsa, np.diag(ref), atol=1e-13, rtol=0)
    for p in range(o):
        for q in range(o):
            g = bf.greens_sa(-0.7, 0.02, p, q)
            want = 1.0 / (-0.7 - e[p] - 0.02j) if p == q else 0.0
            assert abs(g - want) < 1e-12


def test_bruteforce_doublet_space_invariant_and_rhs():
    s = _sys(3, 3, 2)
    bf = IPBruteForce(s)
    assert bf.doublet_leak() < 1e-12
    assert np.allclose(bf.b_sa[:3], np.eye(3, s.dim), atol=1e-14)  # occupied p: b_p = e_p
    # spin-orbital and spin-adapted Green's functions agree
    for p, q in [(0, 0), (1, 2), (2, 1)]:
        assert abs(bf.greens_so(-0.4, 0.01, p, q) - bf.greens_sa(-0.4, 0.01, p, q)) < 1e-11


# ---------------------------------------------------------------- O2 vs O1

@pytest.mark.parametrize("shape", [(2, 3), (3, 2), (3, 3)])
@pytest.mark.parametrize("cls", list(CLASSES))
def test_hbar_matches_bruteforce(bf_cache, shape, cls):
    o, v = shape
    s = _sys(o, v, 3, **CLASSES[cls])
    bf = _bf(bf_cache, (shape, cls), s)
    im = O.intermediates(s)
    H = _dense(im)
    scale = np.abs(bf.Hsa).max()
    assert np.abs(H - bf.Hsa).max() < 1e-12 * scale
    assert np.abs(O.diagonal(im) - np.diag(bf.Hsa)).max() < 1e-12 * scale


def test_hbar_matches_bruteforce_zero_integrals(bf_cache):
    """L = 0 with T2 != 0: only the Fock parts and Lambda-dressed bra survive."""
    s = _sys(3, 3, 4, L_zero=True)
    rng = np.random.default_rng(1)
    t2 = rng.normal(0, 0.05, s.t2.shape)
    s.t2 = t2 + t2.transpose(1, 0, 3, 2)
    s.l2 = s.t2.copy()
    bf = IPBruteForce(s)
    im = O.intermediates(s)
    assert np.abs(_dense(im) - bf.Hsa).max() < 1e-13
    c = np.stack([O.left_vector(s, q) for q in range(6)])  # occupied and virtual q
    assert np.abs(c - bf.c_sa).max() < 1e-13


@pytest.mark.parametrize("shape", [(2, 3), (3, 2), (3, 4)])
def test_left_vectors_independent_lambda(bf_cache, shape):
    """Lambda drawn independently of T so that a lambda<->t role swap fails."""
    o, v = shape
    s = _sys(o, v, 7)
    rng = np.random.default_rng(5)
    s.l1 = rng.normal(0, 0.1, s.t1.shape)
    l2 = rng.normal(0, 0.1, s.t2.shape)
    s.l2 = l2 + l2.transpose(1, 0, 3, 2)
    bf = IPBruteForce(s)
    c = np.stack([O.left_vector(s, q) for q in range(o + v)])
    assert np.abs(c - bf.c_sa).max() < 1e-13
    im = O.intermediates(s)
    assert np.abs(_dense(im) - bf.Hsa).max() < 1e-12 * np.abs(bf.Hsa).max()
    # full G through GMRES against the brute-force dense solve
    for p, q, w in [(0, o - 1, -0.4), (o - 1, 0, -0.9), (1, 1, -0.25)]:
        x, _, res = O.solve(s, im, p, w, 0.02, tol=1e-13)
        g = O.left_vector(s, q) @ x
        gref = bf.greens_so(w, 0.02, p, q)
        assert abs(g - gref) < 1e-10 * max(1.0, abs(gref))


@pytest.mark.parametrize("shape", [(2, 3), (3, 4)])
def test_virtual_orbitals_rhs_left_and_greens(bf_cache, shape):
    """Virtual p and q: b_p = [a_p, T]|Phi> and c_q from Lambda alone, against the
    brute force (Lambda independent of T), and G_qp for every occupied/virtual pairing."""
    o, v = shape
    s = _sys(o, v, 9)
    rng = np.random.default_rng(6)
    s.l1 = rng.normal(0, 0.1, s.t1.shape)
    l2 = rng.normal(0, 0.1, s.t2.shape)
    s.l2 = l2 + l2.transpose(1, 0, 3, 2)
    bf = IPBruteForce(s)
    for p in range(o, o + v):
        b = O.rhs(s, p)
        assert np.abs(b).max() > 1e-3  # correlation gives virtual orbitals an ionised component
        assert np.abs(b - bf.b_sa[p]).max() < 1e-13
        assert np.abs(O.left_vector(s, p) - bf.c_sa[p]).max() < 1e-13
    im = O.intermediates(s)
    for p, q, w in [(o, 0, -0.6), (0, o + v - 1, -0.35), (o + v - 1, o, -0.8)]:
        x, _, _ = O.solve(s, im, p, w, 0.02, tol=1e-13)
        g = O.left_vector(s, q) @ x
        gref = bf.greens_sa(w, 0.02, p, q)
        assert abs(g - gref) < 1e-10 * max(1e-3, abs(gref)), (p, q)
        assert abs(gref - bf.greens_so(w, 0.02, p, q)) < 1e-12 * max(1e-3, abs(gref))


def test_lambda_zero_left_vector_is_unit():
    s = _sys(3, 4, 8, lam=False)
    for q in range(3):
        c = O.left_vector(s, q)
        assert np.array_equal(c, np.eye(s.dim)[q])


# ---------------------------------------------------------------- closed forms on O2

def test_closed_form_free_particles_o2():
    o, v = 4, 16
    s = make_system(o, v, 48, 21, t1=False, t2=False, lam=False, L_zero=True)
    im = O.intermediates(s)
    for eta in (0.01, -0.01):
        G = O.greens(s, im, 2, [-1.0, -0.6, -0.2], eta, qs=[0, 1, 2, 3], tol=1e-14)
        for w, om in enumerate([-1.0, -0.6, -0.2]):
            want = np.zeros(4, complex)
            want[2] = 1.0 / (om - s.eps[2] - 1j * eta)
            assert np.abs(G[w] - want).max() < 1e-12


def test_spectral_function_free_particles():
    """T = Lambda = L = 0: A(omega) is a sum of Lorentzians of width eta at the occupied orbital
    energies, (1/pi) sum_i eta / ((omega - eps_i)^2 + eta^2) (Theory section, the spectral function
    as the trace of Im G), positive, and each Lorentzian carries unit weight."""
    o, v = 4, 16
    s = make_system(o, v, 48, 22, t1=False, t2=False, lam=False, L_zero=True)
    im = O.intermediates(s)
    eta = 0.02
    ws = np.array([-1.1, -0.7, -0.45, -0.3])
    Gd = np.stack([O.greens(s, im, p, ws, eta, tol=1e-14)[:, 0] for p in range(o)], axis=1)  # [omega][p]
    A = O.spectral_function(Gd)
    want = np.array([np.sum(eta / ((w - s.eps[:o]) ** 2 + eta ** 2)) / np.pi for w in ws])
    assert np.abs(A - want).max() < 1e-10 * want.max()
    assert np.all(A > 0)
    # unit weight per occupied orbital: the closed form integrates to o over a wide window
    grid = np.linspace(-60.0, 60.0, 2_400_001)
    dense = np.sum(eta / ((grid[:, None] - s.eps[None, :o]) ** 2 + eta ** 2), axis=1) / np.pi
    assert abs(np.trapezoid(dense, grid) - o) < 2e-3


def test_self_energy_fourth_order_in_L():
    """T = Lambda = 0, L -> sL: G - G0 = O(s^4) (ERIs are quadratic in L)."""
    o, v = 3, 6
    base = make_system(o, v, 8, 31, t1=False, t2=False, lam=False, sigma_L=0.2)
    om, eta, p = -0.8, 0.01, 1
    g0 = 1.0 / (om - base.eps[p] - 1j * eta)
    diffs = []
    for s_ in (0.2, 0.1):
        sy = make_system(o, v, 8, 31, t1=False, t2=False, lam=False, sigma_L=0.2)
        sy.L = base.L * s_
        im = O.intermediates(sy)
        G = O.greens(sy, im, p, [om], eta, tol=1e-14)[0, 0]
        diffs.append(abs(G - g0))
    ratio = diffs[0] / diffs[1]
    assert 14.0 < ratio < 18.0, ratio  # 2^4 = 16


def test_schur_complement_identity():
    """G_pp equals 1/(z - F_pp - Sigma_pp) with the 1h/2h1p block Schur complement."""
    s = _sys(3, 4, 9)
    im = O.intermediates(s)
    H = O.explicit_matrix(im)
    o = 3
    z = -0.5 - 0.02j
    A11 = z * np.eye(o) + H[:o, :o]
    A12, A21 = H[:o, o:], H[o:, :o]
    A22 = z * np.eye(H.shape[0] - o) + H[o:, o:]
    S = A11 - A12 @ np.linalg.solve(A22, A21)
    Ginv = np.linalg.inv(S)
    for p in range(o):
        x, _, _ = O.solve(s, im, p, z.real, -z.imag, tol=1e-14)
        g = O.left_vector(s, p) @ x
        c = O.left_vector(s, p)
        # c^T A^-1 e_p through the block inverse
        y1 = Ginv[:, p]
        y2 = -np.linalg.solve(A22, A21 @ y1)
        assert abs(g - (c[:o] @ y1 + c[o:] @ y2)) < 1e-12


def test_conjugation_symmetry():
    s = _sys(3, 4, 10)
    im = O.intermediates(s)
    Gp = O.greens(s, im, 1, [-0.7, -0.3], 0.01, qs=[0, 1, 2], tol=1e-14)
    Gm = O.greens(s, im, 1, [-0.7, -0.3], -0.01, qs=[0, 1, 2], tol=1e-14)
    assert np.abs(Gm - np.conj(Gp)).max() < 1e-12 * np.abs(Gp).max()


def test_linear_in_lambda():
    s = _sys(3, 4, 12)
    im = O.intermediates(s)
    x, _, _ = O.solve(s, im, 0, -0.6, 0.01, tol=1e-14)

    def g_with(scale):
        s.l1, s.l2 = scale * s.t1, scale * s.t2
        return np.array([O.left_vector(s, q) @ x for q in range(3)])

    g0, g1, g07 = g_with(0.0), g_with(1.0), g_with(0.7)
    assert np.abs(g07 - (g0 + 0.7 * (g1 - g0))).max() < 1e-13


def test_sigma_real_and_linear():
    s = _sys(3, 4, 13)
    im = O.intermediates(s)
    rng = np.random.default_rng(0)
    x = rng.normal(size=s.dim)
    y = rng.normal(size=s.dim) + 1j * rng.normal(size=s.dim)
    sx = O.sigma(im, x)
    assert np.isrealobj(sx)
    lhs = O.sigma(im, 2.0 * x + 3j * y)
    assert np.abs(lhs - (2.0 * sx + 3j * O.sigma(im, y))).max() < 1e-12 * np.abs(lhs).max()


# ---------------------------------------------------------------- tiny workload (o=4, v=16)

@pytest.fixture(scope="module")
def tiny():
    wl = make_workload("tiny-o4v16")
    s = wl.systems[0]
    im = O.intermediates(s)
    return wl, s, im


def test_matrix_free_equals_explicit(tiny):
    _, s, im = tiny
    H1 = _dense(im)
    H2 = O.explicit_matrix(im)
    assert s.dim == 260
    assert np.abs(H1 - H2).max() < 1e-12 * np.abs(H2).max()
    assert np.abs(np.diag(H2) - O.diagonal(im)).max() < 1e-12 * np.abs(H2).max()


def test_gmres_vs_direct_tiny(tiny):
    wl, s, im = tiny
    H = O.explicit_matrix(im)
    eta = wl.eta
    for p in wl.p_lists[0]:
        c = O.left_vector(s, p)
        for om in wl.omegas[0]:
            A = (om - 1j * eta) * np.eye(s.dim) + H
            xd = np.linalg.solve(A, O.rhs(s, p))
            for pc in ("jacobi", None):
                x, it, res = O.solve(s, im, p, om, eta, tol=wl.tol, precond=pc)
                assert res <= wl.tol
                gd, g = c @ xd, c @ x
                assert abs(g - gd) <= 1e-8 * abs(gd)


def test_gmres_residual_monotone_and_finite_termination(tiny):
    _, s, im = tiny
    A = O.shifted_operator(im, -0.55, 0.01)
    hist = []
    x, it, res = O.gmres(A, O.rhs(s, 3), tol=1e-13, restart=s.dim, max_iter=s.dim, history=hist)
    assert it <= s.dim and res <= 1e-12
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))


@pytest.mark.slow
def test_gmres_vs_direct_scaled_down():
    """o = 8, v = 40 (dim 2568): a scaled-down version of the 40/200 workload."""
    s = make_system(8, 40, 160, 2010_04768 + 2)
    im = O.intermediates(s)
    H = O.explicit_matrix(im)
    for p, om in [(7, -0.3), (0, -1.2), (4, -0.75)]:
        A = (om - 0.01j) * np.eye(s.dim) + H
        xd = np.linalg.solve(A, O.rhs(s, p))
        x, it, res = O.solve(s, im, p, om, 0.01, tol=1e-12)
        c = O.left_vector(s, p)
        assert abs(c @ x - c @ xd) <= 1e-10 * abs(c @ xd)


def test_golden_bruteforce_fixture():
    """O2 reproduces the stored brute-force G values (tests/golden/make_golden.py)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "bruteforce_o3v4.json")
    with open(path) as f:
        gold = json.load(f)
    sp = gold["system"]
    s = make_system(sp["n_occ"], sp["n_vir"], sp["n_chol"], sp["seed"],
                    sigma_L=sp["sigma_L"], sigma_t1=sp["sigma_t1"])
    im = O.intermediates(s)
    cache = {}
    for row in gold["G_qp"]:
        key = (row["omega"], row["p"])
        if key not in cache:
            cache[key] = O.solve(s, im, row["p"], row["omega"], gold["eta"], tol=1e-14)[0]
        g = O.left_vector(s, row["q"]) @ cache[key]
        want = row["re"] + 1j * row["im"]
        assert abs(g - want) <= 1e-11 * max(1.0, abs(want))
