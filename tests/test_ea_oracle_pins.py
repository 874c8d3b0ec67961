"""Pins of the EA (electron-attached) oracle against things other than itself (no GPU).

* The Fock-space brute force in the N+1 sector against the closed form at T = Lambda = L = 0.
* The derived spin-adapted EA equations (``oracle.eagfcc``) against the brute force, one
  amplitude class at a time and block by block, for Hbar_N, its diagonal, the right-hand
  sides abar_q^+|Phi> and the left vectors (Lambda independent of T).
* G^EA through GMRES on the shifted operator (omega -> -omega, b -> -b) against the
  brute-force dense solve; G(-eta) = conj G(eta); the full G = G^IP + G^EA of a free system.
"""
import numpy as np
import pytest

from synth import make_system
from oracle import eagfcc as E
from oracle import ipgfcc as O
from oracle.fockspace import EABruteForce, IPBruteForce


def _sys(o, v, seed, **kw):
    return make_system(o, v, 5, seed, sigma_L=0.3, sigma_t1=0.08, **kw)


CLASSES = {
    "bare": dict(t1=False, t2=False, lam=False),
    "t1": dict(t2=False),
    "t2": dict(t1=False),
    "t1t2": dict(),
}


def _dense(eim):
    D = eim["v"] + eim["o"] * eim["v"] ** 2
    return E.sigma(eim, np.eye(D)).T


def _blocks(o, v):
    D = v + o * v * v
    return {"1p<-1p": (slice(0, v), slice(0, v)), "1p<-2p1h": (slice(0, v), slice(v, D)),
            "2p1h<-1p": (slice(v, D), slice(0, v)), "2p1h<-2p1h": (slice(v, D), slice(v, D))}


@pytest.fixture(scope="module")
def bf_cache():
    return {}


def _bf(cache, key, s):
    if key not in cache:
        cache[key] = EABruteForce(s)
    return cache[key]


def test_bruteforce_free_particles():
    """T = Lambda = L = 0: Hbar is diagonal with eps_a (1p) and eps_a + eps_b - eps_j (2p1h),
    b_q = e_q for virtual q, zero for occupied q, and G^EA_ab = d_ab / (omega + i eta - eps_a)."""
    o, v = 2, 3
    s = make_system(o, v, 4, 12, t1=False, t2=False, lam=False, L_zero=True)
    bf = EABruteForce(s)
    e = s.eps
    ref = [e[o + a] for a in range(v)]
    ref += [e[o + a] + e[o + b] - e[j] for j in range(o) for a in range(v) for b in range(v)]
    assert np.allclose(bf.Hsa, np.diag(ref), atol=1e-13, rtol=0)
    assert bf.doublet_leak() < 1e-13
    assert np.abs(bf.b_sa[:o]).max() == 0.0
    assert np.allclose(bf.b_sa[o:], np.eye(v, bf.Hsa.shape[0]), atol=1e-14)
    for a in range(v):
        for b in range(v):
            g = bf.greens_sa(0.9, 0.02, o + a, o + b)
            want = 1.0 / (0.9 + 0.02j - e[o + a]) if a == b else 0.0
            assert abs(g - want) < 1e-12
            assert abs(bf.greens_so(0.9, 0.02, o + a, o + b) - g) < 1e-12


def test_bruteforce_doublet_space_invariant():
    s = _sys(2, 3, 2)
    bf = EABruteForce(s)
    assert bf.doublet_leak() < 1e-12
    for p, q in [(0, 0), (1, 3), (3, 4), (4, 1)]:
        assert abs(bf.greens_so(0.6, 0.01, p, q) - bf.greens_sa(0.6, 0.01, p, q)) < 1e-11


@pytest.mark.parametrize("shape", [(2, 3), (3, 2), (2, 4)])
@pytest.mark.parametrize("cls", list(CLASSES))
def test_hbar_matches_bruteforce(bf_cache, shape, cls):
    """Block by block so that a dropped term names its block."""
    o, v = shape
    s = _sys(o, v, 3, **CLASSES[cls])
    if cls in ("t2", "t1t2"):
        s.t2 = s.t2 * 3.0  # make the T2 terms large enough that a dropped one cannot hide
    bf = _bf(bf_cache, (shape, cls), s)
    eim = E.intermediates(s)
    H = _dense(eim)
    scale = np.abs(bf.Hsa).max()
    for name, b in _blocks(o, v).items():
        assert np.abs(H[b] - bf.Hsa[b]).max() < 1e-12 * scale, name
    assert np.abs(E.diagonal(eim) - np.diag(bf.Hsa)).max() < 1e-12 * scale
    assert np.abs(E.explicit_matrix(eim) - H).max() < 1e-12 * scale


def test_hbar_matches_bruteforce_zero_integrals():
    """L = 0 with T2 != 0: only the Fock parts and the three-body term's T2 dressing vanish
    with L, so the 2p1h block reduces to the orbital energies."""
    s = _sys(2, 3, 4, L_zero=True)
    rng = np.random.default_rng(1)
    t2 = rng.normal(0, 0.05, s.t2.shape)
    s.t2 = t2 + t2.transpose(1, 0, 3, 2)
    s.l2 = s.t2.copy()
    bf = EABruteForce(s)
    eim = E.intermediates(s)
    assert np.abs(_dense(eim) - bf.Hsa).max() < 1e-13
    b = np.stack([E.rhs(s, q) for q in range(5)])
    c = np.stack([E.left_vector(s, p) for p in range(5)])
    assert np.abs(b - bf.b_sa).max() < 1e-13
    assert np.abs(c - bf.c_sa).max() < 1e-13


@pytest.mark.parametrize("shape", [(2, 3), (3, 2), (2, 4)])
def test_rhs_and_left_vectors_independent_lambda(shape):
    """Lambda drawn independently of T so that a lambda<->t role swap fails; every occupied
    and virtual index on both sides."""
    o, v = shape
    s = _sys(o, v, 7)
    rng = np.random.default_rng(5)
    s.l1 = rng.normal(0, 0.1, s.t1.shape)
    l2 = rng.normal(0, 0.1, s.t2.shape)
    s.l2 = l2 + l2.transpose(1, 0, 3, 2)
    bf = EABruteForce(s)
    n = o + v
    b = np.stack([E.rhs(s, q) for q in range(n)])
    c = np.stack([E.left_vector(s, p) for p in range(n)])
    assert np.abs(b - bf.b_sa).max() < 1e-13
    assert np.abs(c - bf.c_sa).max() < 1e-13
    eim = E.intermediates(s)
    assert np.abs(_dense(eim) - bf.Hsa).max() < 1e-12 * np.abs(bf.Hsa).max()
    # G^EA through GMRES on (-omega - i eta + Hbar) Y = -b against the dense solve
    for p, q, w in [(o, o, 0.7), (n - 1, o, 1.3), (0, n - 1, 0.45), (o - 1, 0, 1.1)]:
        g = E.greens(s, eim, q, [w], 0.02, ps=[p], tol=1e-13)[0, 0]
        gref = bf.greens_so(w, 0.02, p, q)
        assert abs(g - gref) < 1e-10 * max(1.0, abs(gref)), (p, q, g, gref)


def test_lambda_zero_left_vector():
    """Lambda = 0: c_p = <Phi|abar_p e^T restricted to the space; for virtual p that is e_p
    minus nothing (the T terms of abar_p reach only the N-1 sector), for occupied p zero."""
    s = _sys(2, 3, 8, lam=False)
    for p in range(2):
        assert np.abs(E.left_vector(s, p)).max() == 0.0
    for a in range(3):
        c = E.left_vector(s, 2 + a)
        want = np.zeros_like(c)
        want[a] = 1.0
        assert np.abs(c - want).max() == 0.0


def test_closed_form_free_particles():
    """T = Lambda = L = 0 through the derived equations and GMRES."""
    o, v = 2, 5
    s = make_system(o, v, 4, 21, t1=False, t2=False, lam=False, L_zero=True)
    eim = E.intermediates(s)
    for a in range(v):
        g = E.greens(s, eim, o + a, [0.5, 1.7], 0.03, ps=range(o + v), tol=1e-14)
        for k, w in enumerate([0.5, 1.7]):
            want = np.zeros(o + v, complex)
            want[o + a] = 1.0 / (w + 0.03j - s.eps[o + a])
            assert np.abs(g[k] - want).max() < 1e-12


def test_conjugation_symmetry():
    s = _sys(2, 3, 9)
    eim = E.intermediates(s)
    g1 = E.greens(s, eim, 3, [0.8], 0.02, ps=[1, 3, 4], tol=1e-14)
    g2 = E.greens(s, eim, 3, [0.8], -0.02, ps=[1, 3, 4], tol=1e-14)
    assert np.abs(g1 - np.conj(g2)).max() < 1e-11 * np.abs(g1).max()


def test_full_greens_free_particles_both_terms():
    """Free particles: G = G^IP + G^EA is diag(1/(omega + i eta sgn - eps_p)) over all
    orbitals (occupied from the IP term with -i eta, virtual from the EA term with +i eta)."""
    o, v = 2, 3
    s = make_system(o, v, 4, 31, t1=False, t2=False, lam=False, L_zero=True)
    ip = IPBruteForce(s)
    ea = EABruteForce(s)
    w, eta = 0.3, 0.05
    for p in range(o + v):
        g = ip.greens_sa(w, eta, p, p) + ea.greens_sa(w, eta, p, p)
        e = s.eps[p]
        want = 1.0 / (w - e - 1j * eta) if p < o else 1.0 / (w - e + 1j * eta)
        assert abs(g - want) < 1e-12


def test_sigma_real_linear_batched():
    """The sigma product is real-linear and acts the same on a batch as on single vectors."""
    s = _sys(3, 4, 10)
    eim = E.intermediates(s)
    D = 4 + 3 * 16
    rng = np.random.default_rng(3)
    Y = rng.normal(size=(3, D)) + 1j * rng.normal(size=(3, D))
    S = E.sigma(eim, Y)
    for k in range(3):
        assert np.abs(S[k] - (E.sigma(eim, Y[k].real) + 1j * E.sigma(eim, Y[k].imag))).max() < 1e-13
    assert np.abs(E.sigma(eim, 2.0 * Y[0] - Y[1]) - (2.0 * S[0] - S[1])).max() < 1e-12
