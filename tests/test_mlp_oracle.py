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


# ---- Adam (Kingma & Ba, Algorithm 1: biased moments m, v; bias corrections
# 1 - beta^t; step lr * mhat / (sqrt(vhat) + eps)).  Pins independent of the
# oracle's own formula: a two-step example worked by hand, and two closed forms.

def _adam_run(p0, grads, lr, **kw):
    p = {"w": np.array(p0, dtype=float)}
    st = {}
    for g in grads:
        M.adam_step(p, {"w": np.array(g, dtype=float)}, st, lr, **kw)
    return p["w"], st


def test_adam_two_steps_worked_by_hand():
    """p0 = 1, gradients 0.5 then -0.25, lr = 0.1, beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
    Step 1: m = 0.05, v = 0.00025, mhat = 0.5, vhat = 0.25,
            p1 = 1 - 0.1 * 0.5 / (0.5 + 1e-8) = 0.90000000199999996000...
    Step 2: m = 0.9*0.05 - 0.1*0.25 = 0.02, v = 0.999*0.00025 + 0.001*0.0625 = 0.00031225,
            mhat = 0.02 / 0.19, vhat = 0.00031225 / 0.001999,
            p2 = 0.87336629870784616255937..."""
    w1, st1 = _adam_run([1.0], [[0.5]], 0.1)
    assert abs(st1["m_w"][0] - 0.05) <= 4e-15 * 0.05 and abs(st1["v_w"][0] - 0.00025) <= 4e-15 * 0.00025
    assert abs(w1[0] - 0.90000000199999996000) <= 1e-15
    w2, st2 = _adam_run([1.0], [[0.5], [-0.25]], 0.1)
    assert abs(st2["m_w"][0] - 0.02) <= 4e-15 * 0.02 and abs(st2["v_w"][0] - 0.00031225) <= 4e-15 * 0.00031225
    assert st2["t"] == 2
    assert abs(w2[0] - 0.87336629870784616256) <= 1e-15


def test_adam_first_step_is_lr_times_sign_like():
    """The bias corrections make the first step exactly lr * g / (|g| + eps) for every
    parameter, whatever the betas.  eps = 0.1 so that eps inside the square root, or a
    missing or misplaced bias correction, changes the result by far more than rounding."""
    rng = np.random.default_rng(11)
    g = rng.normal(size=50) * np.exp(rng.uniform(-3, 3, size=50))
    p0 = rng.normal(size=50)
    for b1, b2 in ((0.9, 0.999), (0.5, 0.9)):
        w, _ = _adam_run(p0, [g], 0.03, b1=b1, b2=b2, eps=0.1)
        assert np.allclose(w, p0 - 0.03 * g / (np.abs(g) + 0.1), rtol=0, atol=1e-15)


def test_adam_constant_gradient_moves_linearly():
    """With a constant gradient the bias-corrected moments equal g and g^2 at every step,
    so t steps move each parameter by t * lr * g / (|g| + eps)."""
    rng = np.random.default_rng(12)
    g = rng.normal(size=20)
    p0 = rng.normal(size=20)
    w, st = _adam_run(p0, [g] * 7, 0.01, eps=0.05)
    assert np.allclose(w, p0 - 7 * 0.01 * g / (np.abs(g) + 0.05), rtol=0, atol=1e-14)
    # the biased first moment after t steps is (1 - beta1^t) g
    assert np.allclose(st["m_w"], (1 - 0.9 ** 7) * g, rtol=1e-14, atol=0)
