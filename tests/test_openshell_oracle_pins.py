"""Pins of the open-shell (spin-unrestricted) IP oracle against things other than itself (no GPU).

* The brute force in both ionised sectors (an alpha or a beta electron removed) against the
  closed form at T = Lambda = L = 0.
* The spin-orbital working equations (``oracle.openshell``) against the brute force, one
  amplitude class at a time and block by block, for Hbar_N, its diagonal, b_p and c_q (Lambda
  independent of T), and G through GMRES.
* A link between two independent derivations: with identical alpha and beta spins the
  spin-orbital G equals the closed-shell spin-adapted G of ``oracle.ipgfcc``.
* G(-eta) = conj G(eta); spin selection (G between alpha and beta orbitals vanishes).
"""
import numpy as np
import pytest

from synth import make_open_shell_system, make_system
from oracle import ipgfcc as IP
from oracle import openshell as OS


def _sys(n, oa, ob, seed, **kw):
    return make_open_shell_system(n, oa, ob, 5, seed, sigma_L=0.3, sigma_dL=0.1, sigma_t1=0.08, **kw)


CLASSES = {
    "bare": dict(t1=False, t2=False, lam=False),
    "t1": dict(t2=False),
    "t2": dict(t1=False),
    "t1t2": dict(),
}
SHAPES = [(4, 2, 1), (5, 3, 2), (4, 2, 2), (5, 3, 1)]


def _H(bf, im):
    Dk = bf.H.shape[0]
    H = np.zeros((Dk, Dk))
    for mu in range(Dk):
        e = np.zeros(Dk)
        e[mu] = 1.0
        H[:, mu] = bf.unique(OS.sigma(im, bf.full(e)))
    return H


@pytest.fixture(scope="module")
def bf_cache():
    return {}


def test_bruteforce_free_particles():
    n, oa, ob = 4, 2, 1
    s = make_open_shell_system(n, oa, ob, 4, 11, t1=False, t2=False, lam=False, L_zero=True)
    bf = OS.OpenShellBruteForce(s)
    so = OS.so_arrays(s)
    e = so["eps"]
    o = so["o"]
    want = []
    for bb in bf.basis:
        if bb[0] == "1h":
            want.append(-e[bb[1]])
        else:
            _, i, j, a = bb
            want.append(e[o + a] - e[i] - e[j])
    assert np.allclose(bf.H, np.diag(want), atol=1e-13, rtol=0)
    # both sectors present: alpha and beta holes, and the alpha-beta 2h1p states
    assert {bb[1] for bb in bf.basis if bb[0] == "1h"} == set(range(o))
    for p in range(o):
        for q in range(o):
            g = bf.greens(-0.7, 0.02, p, q)
            ref = 1.0 / (-0.7 - e[p] - 0.02j) if p == q else 0.0
            assert abs(g - ref) < 1e-12


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("cls", list(CLASSES))
def test_hbar_matches_bruteforce(bf_cache, shape, cls):
    n, oa, ob = shape
    s = _sys(n, oa, ob, 3, **CLASSES[cls])
    if cls in ("t2", "t1t2"):
        for nm in ("t2aa", "t2ab", "t2bb"):
            setattr(s, nm, getattr(s, nm) * 3.0)
    key = (shape, cls)
    if key not in bf_cache:
        bf_cache[key] = OS.OpenShellBruteForce(s)
    bf = bf_cache[key]
    im = OS.intermediates(s)
    H = _H(bf, im)
    n1 = sum(1 for bb in bf.basis if bb[0] == "1h")
    Dk = H.shape[0]
    scale = np.abs(bf.H).max()
    for name, (r, c) in {"1h<-1h": (slice(0, n1), slice(0, n1)), "1h<-2h1p": (slice(0, n1), slice(n1, Dk)),
                         "2h1p<-1h": (slice(n1, Dk), slice(0, n1)),
                         "2h1p<-2h1p": (slice(n1, Dk), slice(n1, Dk))}.items():
        assert np.abs(H[r, c] - bf.H[r, c]).max() < 1e-12 * scale, name
    assert np.abs(bf.unique(OS.diagonal(im)) - np.diag(bf.H)).max() < 1e-12 * scale
    # sigma keeps vectors antisymmetric in the hole pair
    x = bf.full(np.random.default_rng(1).normal(size=Dk))
    y = OS.sigma(im, x)
    o, v = im["o"], im["v"]
    y2 = y[o:].reshape(o, o, v)
    assert np.abs(y2 + y2.transpose(1, 0, 2)).max() < 1e-13 * np.abs(y2).max()


@pytest.mark.parametrize("shape", [(4, 2, 1), (5, 3, 2), (5, 3, 1)])
def test_rhs_left_and_greens_independent_lambda(shape):
    n, oa, ob = shape
    s = _sys(n, oa, ob, 7)
    rng = np.random.default_rng(5)
    s.l1a = rng.normal(0, 0.1, s.t1a.shape)
    s.l1b = rng.normal(0, 0.1, s.t1b.shape)

    def anti(x):
        return x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)

    s.l2aa = anti(rng.normal(0, 0.05, s.t2aa.shape))
    s.l2bb = anti(rng.normal(0, 0.05, s.t2bb.shape))
    s.l2ab = rng.normal(0, 0.05, s.t2ab.shape)
    bf = OS.OpenShellBruteForce(s)
    im = OS.intermediates(s)
    so = im["so"]
    norb = so["o"] + so["v"]
    Dk = bf.H.shape[0]
    X = bf.full(rng.normal(size=(3, Dk)))
    for p in range(norb):
        assert np.abs(bf.unique(OS.rhs(so, p)) - bf.b[p]).max() < 1e-14, p
        c = OS.left_vector(so, p)
        assert np.abs(X @ c - bf.unique(X) @ bf.c[p]).max() < 1e-13, p
    o = so["o"]
    for p, q, w in [(0, 0, -0.5), (o - 1, o - 1, -0.8), (1, 0, -0.3), (o, 0, -0.6), (0, o + 1, -0.9)]:
        g = OS.greens(im, so, p, [w], 0.02, qs=[q], tol=1e-13)[0, 0]
        ref = bf.greens(w, 0.02, p, q)
        assert abs(g - ref) < 1e-10 * max(1.0, abs(ref)), (p, q)


def test_spin_selection_and_conjugation():
    s = _sys(5, 3, 2, 9)
    im = OS.intermediates(s)
    so = im["so"]
    oa, ob = s.n_occ_a, s.n_occ_b
    g = OS.greens(im, so, 0, [-0.6], 0.02, qs=list(range(so["o"])), tol=1e-13)[0]
    assert np.abs(g[oa:]).max() == 0.0  # an alpha hole has no beta component
    assert abs(g[0]) > 0.1
    g2 = OS.greens(im, so, 0, [-0.6], -0.02, qs=list(range(so["o"])), tol=1e-13)[0]
    assert np.abs(g - np.conj(g2)).max() < 1e-11


@pytest.mark.parametrize("o,v", [(2, 3), (3, 4)])
def test_closed_shell_limit_equals_spin_adapted_oracle(o, v):
    """Identical spins: the spin-orbital G of an alpha hole equals the closed-shell spin-adapted G
    of the independently derived ``oracle.ipgfcc`` (and the beta one equals it too)."""
    cs = make_system(o, v, 5, 21 + o, sigma_L=0.3, sigma_t1=0.08)
    rng = np.random.default_rng(3)
    cs.l1 = rng.normal(0, 0.05, cs.t1.shape)
    l2 = rng.normal(0, 0.05, cs.t2.shape)
    cs.l2 = l2 + l2.transpose(1, 0, 3, 2)
    os_ = OS.from_closed_shell(cs)
    im = OS.intermediates(os_)
    so = im["so"]
    imc = IP.intermediates(cs)
    for p, q, w in [(0, 0, -0.5), (o - 1, 0, -0.8), (1, o + 1, -0.4)]:
        xc, _, _ = IP.solve(cs, imc, p, w, 0.02, tol=1e-13)
        gc = IP.left_vector(cs, q) @ xc
        # closed-shell orbital p -> alpha spin orbital p; q likewise (virtual q -> alpha virtual)
        qa = q if q < o else so["o"] + (q - o)
        g = OS.greens(im, so, p, [w], 0.02, qs=[qa], tol=1e-13)[0, 0]
        assert abs(g - gc) < 1e-10 * max(1.0, abs(gc)), (p, q, g, gc)
        pb, qb = o + p, (o + q if q < o else so["o"] + v + (q - o))  # the beta copies
        gb = OS.greens(im, so, pb, [w], 0.02, qs=[qb], tol=1e-13)[0, 0]
        assert abs(gb - gc) < 1e-10 * max(1.0, abs(gc))


def test_closed_form_free_particles_gmres():
    s = make_open_shell_system(6, 3, 2, 4, 13, t1=False, t2=False, lam=False, L_zero=True)
    im = OS.intermediates(s)
    so = im["so"]
    for p in range(so["o"]):
        g = OS.greens(im, so, p, [-0.9, -0.4], 0.03, qs=[p], tol=1e-14)[:, 0]
        ref = 1.0 / (np.array([-0.9, -0.4]) - so["eps"][p] - 0.03j)
        assert np.abs(g - ref).max() < 1e-12
