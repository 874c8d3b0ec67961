"""Pins of the model-order-reduction oracle (``oracle/mor.py``).

* the level bound against the worked example of the GFCC Workflow and
  Bottlenecks section (a [-0.8, -0.4] window at 0.01 resolution allows at most
  five levels) and the per-level counts summing within the grid;
* a full basis (S = identity) reproduces the dense direct solve at every omega;
* Galerkin interpolation: the model is exact at every omega whose solutions are
  in the span of S (independent of how S was orthonormalised);
* the model G does not depend on the choice of orthonormal basis of the span;
* Gram-Schmidt: orthonormal columns, span keeps every accepted candidate,
  dependent candidates dropped;
* the level loop: schedule shape, level bound, and the final model within the
  tolerance of direct solves on the whole grid.
"""
import numpy as np
import pytest

from oracle import ipgfcc as O
from oracle import mor as M
from synth import make_system


@pytest.fixture(scope="module")
def tiny():
    s = make_system(4, 16, 48, 2010_04768 + 1)
    return s, O.intermediates(s)


def _direct(s, im, p, w, eta):
    A = (w - 1j * eta) * np.eye(s.dim) + O.explicit_matrix(im)
    return np.linalg.solve(A, O.rhs(s, p))


def test_level_bound_worked_example():
    assert M.lmax_bound(-0.8, -0.4, 0.01) == 5
    n_tot = len(M.grid(-0.8, -0.4, 0.01))
    assert n_tot == 41
    assert sum(M.n_max_omega(L) for L in range(1, 6)) <= n_tot
    assert sum(M.n_max_omega(L) for L in range(1, 7)) > n_tot
    assert [M.n_max_omega(L) for L in (1, 2, 3, 4)] == [3, 2, 4, 8]


def test_full_basis_equals_direct_solve(tiny):
    s, im = tiny
    S = np.eye(s.dim)
    H = M.project(im, S)
    assert np.abs(H - O.explicit_matrix(im)).max() < 1e-12 * np.abs(H).max()
    ws = np.array([-1.0, -0.55, -0.2])
    G = M.model_greens(s, S, H, [0, 3], ws, 0.01)
    for k, w in enumerate(ws):
        for i, p in enumerate((0, 3)):
            g = O.left_vector(s, p) @ _direct(s, im, p, w, 0.01)
            assert abs(G[k, i, i] - g) <= 1e-11 * abs(g)


def test_galerkin_exact_at_basis_frequencies(tiny):
    s, im = tiny
    ws = [-0.9, -0.5]
    X = [_direct(s, im, p, w, 0.01) for w in ws for p in range(4)]
    S, kept = M.extend_basis(np.zeros((s.dim, 0)), M.candidates(np.stack(X, axis=1)))
    assert len(kept) == 16
    H = M.project(im, S)
    G = M.model_greens(s, S, H, list(range(4)), np.array(ws), 0.01, q_list=[0, 1, 2, 3])
    for k, w in enumerate(ws):
        for p in range(4):
            x = X[k * 4 + p]
            for q in range(4):
                g = O.left_vector(s, q) @ x
                assert abs(G[k, p, q] - g) <= 1e-9 * max(abs(g), 1e-3), (k, p, q)
    # away from the basis frequencies the model is an approximation, not exact
    G2 = M.model_greens(s, S, H, [0], np.array([-0.2]), 0.01)
    g2 = O.left_vector(s, 0) @ _direct(s, im, 0, -0.2, 0.01)
    assert abs(G2[0, 0, 0] - g2) > 1e-14 * abs(g2)


def test_model_independent_of_basis_choice(tiny):
    s, im = tiny
    X = [_direct(s, im, p, -0.7, 0.01) for p in range(4)]
    S, _ = M.extend_basis(np.zeros((s.dim, 0)), M.candidates(np.stack(X, axis=1)))
    Q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(S.shape[1], S.shape[1])))
    S2 = S @ Q
    ws = np.array([-1.0, -0.3])
    G1 = M.model_greens(s, S, M.project(im, S), [0, 2], ws, 0.01)
    G2 = M.model_greens(s, S2, M.project(im, S2), [0, 2], ws, 0.01)
    assert np.abs(G1 - G2).max() <= 1e-11 * np.abs(G1).max()


def test_gram_schmidt_orthonormal_and_drops_dependent():
    rng = np.random.default_rng(5)
    V = rng.normal(size=(50, 6))
    V = np.concatenate([V, V[:, :2] @ rng.normal(size=(2, 3))], axis=1)  # 3 dependent columns
    S, kept = M.extend_basis(np.zeros((50, 0)), V)
    assert kept == [0, 1, 2, 3, 4, 5]
    assert np.abs(S.T @ S - np.eye(6)).max() < 1e-13
    assert np.abs(S @ (S.T @ V) - V).max() < 1e-12 * np.abs(V).max()
    S2, kept2 = M.extend_basis(S, rng.normal(size=(50, 2)))
    assert kept2 == [0, 1] and np.abs(S2[:, :6] - S).max() == 0.0
    assert np.abs(S2.T @ S2 - np.eye(8)).max() < 1e-13


def test_level_loop_schedule_and_accuracy(tiny):
    s, im = tiny
    ws = M.grid(-1.0, -0.2, 0.01)
    out = M.levels(s, im, [0, 1, 2, 3], ws, 0.01, tol=1e-8)
    sched = out["levels"]
    assert sched[0] == [0, 40, 80]
    assert len(sched) <= M.lmax_bound(-1.0, -0.2, 0.01)
    for L, pts in enumerate(sched, start=1):
        assert len(pts) <= M.n_max_omega(L)
    for k in range(0, len(ws), 7):
        for i, p in enumerate(range(4)):
            g = O.left_vector(s, p) @ _direct(s, im, p, ws[k], 0.01)
            assert abs(out["G"][k, i] - g) <= 1e-7 * abs(g), (k, p)
