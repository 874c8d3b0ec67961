"""Oracle of model-order reduction (MOR) over frequency levels, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What it computes (paper, Theory section, eq. ``model``; GFCC Workflow and
Bottlenecks, the level loop of Algorithm 1 and eq. ``Lmax``):

* an orthonormal basis S of the span of solved vectors X_p(omega_k);
* the projected operator ``Hhat = S^T Hbar_N S``, ``bhat = S^T b_p`` and
  ``chat_q = S^T c_q``;
* the model systems ``(omega - i eta + Hhat) Xhat = bhat`` and the model
  Green's function ``Ghat_qp(omega) = chat_q^T Xhat`` on a fine frequency grid;
* the level schedule: level 1 solves the two ends and the middle of the grid,
  every later level solves the midpoints of the intervals that are not yet
  converged, so level L solves at most 3 (L = 1) or 2^(L-1) (L > 1) points and
  the number of levels is bounded by ``log2((w_max - w_min) / dw)``.

Readings (the paper states the projection, not its details):

* S is real.  The real and imaginary parts of every solved X_p(omega) are
  separate basis candidates, so Hhat is real and one projection serves every
  omega (the span contains the complex span of the X).
* Gram-Schmidt is classical with one reorthogonalisation; a candidate whose
  norm after orthogonalisation falls below ``drop_tol`` times its norm before
  is dropped as linearly dependent.
* An interval is converged when the model built from the levels so far
  predicts G at its midpoint within ``tol`` (relative, every requested p) of
  the directly solved value; otherwise both halves stay open.  An interval
  with no grid point inside is closed.
"""
from __future__ import annotations

import math

import numpy as np

from . import ipgfcc as O


def n_max_omega(level):
    """Largest number of frequencies solved at ``level`` (1-based)."""
    return 3 if level == 1 else 2 ** (level - 1)


def lmax_bound(w_min, w_max, dw):
    """Upper bound on the number of levels for a grid of resolution ``dw``."""
    return int(math.floor(math.log2((w_max - w_min) / dw)))


def grid(w_min, w_max, dw):
    n = int(round((w_max - w_min) / dw)) + 1
    return np.linspace(w_min, w_max, n)


def extend_basis(S, V, drop_tol=1e-10):
    """Append the Gram-Schmidt orthonormalised real columns of V to S.

    S: [D, m] with orthonormal columns (m may be 0); V: [D, k] real.
    Returns (S_new, kept) where ``kept`` lists the accepted columns of V.
    """
    cols = [S[:, j] for j in range(S.shape[1])]
    kept = []
    for c in range(V.shape[1]):
        v = np.array(V[:, c], dtype=float)
        n0 = np.linalg.norm(v)
        if n0 == 0.0:
            continue
        for _ in range(2):
            for s in cols:
                v = v - (s @ v) * s
        n1 = np.linalg.norm(v)
        if n1 <= drop_tol * n0:
            continue
        cols.append(v / n1)
        kept.append(c)
    S_new = np.stack(cols, axis=1) if cols else np.zeros((V.shape[0], 0))
    return S_new, kept


def candidates(X):
    """Real basis candidates [Re x_1, Im x_1, Re x_2, ...] of complex columns X [D, n]."""
    X = np.asarray(X, dtype=complex)
    out = np.empty((X.shape[0], 2 * X.shape[1]))
    out[:, 0::2] = X.real
    out[:, 1::2] = X.imag
    return out


def project(im, S):
    """Hhat = S^T Hbar_N S, through the matrix-free sigma on each basis column."""
    HS = np.stack([O.sigma(im, S[:, j]).real for j in range(S.shape[1])], axis=1)
    return S.T @ HS


def model_greens(sys, S, Hhat, p_list, omegas, eta, q_list=None):
    """Ghat[w, p, q] = chat_q^T (omega - i eta + Hhat)^-1 bhat_p."""
    q_list = list(p_list) if q_list is None else list(q_list)
    B = np.stack([S.T @ O.rhs(sys, p) for p in p_list], axis=1)
    C = np.stack([S.T @ O.left_vector(sys, q) for q in q_list], axis=1)
    m = S.shape[1]
    G = np.empty((len(omegas), len(p_list), len(q_list)), dtype=complex)
    for k, w in enumerate(omegas):
        Xh = np.linalg.solve((w - 1j * eta) * np.eye(m) + Hhat, B)
        G[k] = Xh.T @ C
    return G


def levels(sys, im, p_list, omegas, eta, tol=1e-8, solve_tol=1e-12, drop_tol=1e-10, max_levels=None,
           solver=None):
    """Adaptive midpoint level loop on the grid ``omegas`` (uniform, ascending).

    ``solver(p, omega) -> X_p(omega)`` defaults to the oracle's GMRES.
    Returns dict(G=[n_omega, n_p] model diagonal G, levels=[list of grid indices per level],
    S=basis, Hhat, direct={index: [G_pp direct per p]}).
    """
    if solver is None:
        def solver(p, w):
            return O.solve(sys, im, p, w, eta, tol=solve_tol, restart=60, max_iter=4000)[0]
    n = len(omegas)
    dw = (omegas[-1] - omegas[0]) / (n - 1)
    lmax = max(1, lmax_bound(omegas[0], omegas[-1], dw))
    if max_levels is not None:
        lmax = min(lmax, max_levels)
    S = np.zeros((sys.dim, 0))
    direct = {}

    def solve_points(todo):
        X = []
        for k in todo:
            xs = [solver(int(p), float(omegas[k])) for p in p_list]
            direct[k] = np.array([O.left_vector(sys, int(p)) @ x for p, x in zip(p_list, xs)])
            X.extend(xs)
        return candidates(np.stack(X, axis=1))

    # level 1: both ends and the middle; no model exists yet to test
    mid = (n - 1) // 2
    todo = sorted({0, mid, n - 1})
    sched = [todo]
    S, _ = extend_basis(S, solve_points(todo), drop_tol)
    Hhat = project(im, S)
    open_iv = [(a, b) for a, b in ((0, mid), (mid, n - 1)) if b - a > 1]
    level = 1
    while open_iv and level < lmax:
        level += 1
        mids = [(a + b) // 2 for a, b in open_iv]
        todo = sorted(set(mids))
        sched.append(todo)
        Gm = model_greens(sys, S, Hhat, p_list, omegas[todo], eta)
        V = solve_points(todo)
        err = {k: float(np.max(np.abs(np.diagonal(Gm[i]) - direct[k]) / np.abs(direct[k])))
               for i, k in enumerate(todo)}
        nxt = []
        for (a, b), c in zip(open_iv, mids):
            if err[c] > tol:
                nxt.extend([(a, c), (c, b)])
        open_iv = [(a, b) for a, b in nxt if b - a > 1]
        S, _ = extend_basis(S, V, drop_tol)
        Hhat = project(im, S)
    G = model_greens(sys, S, Hhat, p_list, omegas, eta)
    Gd = np.stack([np.diagonal(G[k]) for k in range(n)])
    return dict(G=Gd, levels=sched, S=S, Hhat=Hhat, direct=direct)
