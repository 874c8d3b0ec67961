"""Pins of the learned-preconditioner oracle (CPU, FP64)."""
import numpy as np

from oracle import ipgfcc as O
from oracle import mlp as M
from synth import make_system


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = M.init_params(12, seed=3)
    p["W3"] = rng.normal(0, 0.3, p["W3"].shape)  # non-zero output layer so every path is exercised
    p["b3"] = rng.normal(0, 0.1, 2)
    X = rng.normal(size=(40, M.N_FEAT))
    T = rng.normal(size=(40, 2))
    L, g = M.loss_and_grad(p, X, T)
    flat = M.flatten(p)
    gflat = M.flatten(g)
    h = 1e-6
    idx = rng.choice(flat.size, size=60, replace=False)
    for k in idx:
        e = np.zeros_like(flat)
        e[k] = h
        Lp, _ = M.loss_and_grad(M.unflatten(flat + e, 12), X, T)
        Lm, _ = M.loss_and_grad(M.unflatten(flat - e, 12), X, T)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gflat[k]) <= 1e-7 * max(1.0, abs(fd)), (k, fd, gflat[k])


def test_zero_output_layer_is_jacobi_and_perfect_output_is_exact():
    s = make_system(3, 5, 6, 5, sigma_L=0.2, sigma_t1=0.02)
    im = O.intermediates(s)
    d = O.diagonal(im)
    sD = np.mean(np.abs(d))
    rng = np.random.default_rng(1)
    r = rng.normal(size=s.dim) + 1j * rng.normal(size=s.dim)
    p = M.init_params(16, seed=1)
    u = M.apply(p, r, d, -0.6, 0.01, s.n_occ, sD)
    assert np.allclose(u, r / (-0.6 - 0.01j + d), rtol=1e-14, atol=0)
    # the target makes the correction exact: jacobi + t * n / sD == A^-1 r
    H = O.explicit_matrix(im)
    e = np.linalg.solve((-0.6 - 0.01j) * np.eye(s.dim) + H, r)
    t = M.targets(r, e, d, -0.6, 0.01, sD)
    n = np.linalg.norm(r) / np.sqrt(s.dim)
    rebuilt = r / (-0.6 - 0.01j + d) + (t[:, 0] + 1j * t[:, 1]) * n / sD
    assert np.allclose(rebuilt, e, rtol=1e-12, atol=1e-14)


def test_features_scale_free():
    s = make_system(3, 5, 6, 5)
    im = O.intermediates(s)
    d = O.diagonal(im)
    rng = np.random.default_rng(2)
    r = rng.normal(size=s.dim) + 1j * rng.normal(size=s.dim)
    X1, n1 = M.features(r, d, -0.5, 0.01, 3, 10.0)
    X2, n2 = M.features(7.5 * r, d, -0.5, 0.01, 3, 10.0)
    assert np.allclose(X1, X2) and np.isclose(n2, 7.5 * n1)
    assert np.all(X1[:3, 6] == 1) and np.all(X1[3:, 6] == 0)


def test_adam_decreases_loss_on_a_fit():
    rng = np.random.default_rng(3)
    p = M.init_params(16, seed=2)
    X = rng.normal(size=(256, M.N_FEAT))
    T = np.stack([np.sin(X[:, 0]), X[:, 1] * X[:, 2]], axis=1)
    st = {}
    L0, _ = M.loss_and_grad(p, X, T)
    for _ in range(300):
        L, g = M.loss_and_grad(p, X, T)
        M.adam_step(p, g, st, 1e-2)
    assert L < 0.3 * L0
