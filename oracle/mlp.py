"""Oracle of the learned residual->correction preconditioner (TEST INFRASTRUCTURE ONLY).

The paper uses GMRES with the inverse diagonal of the Hamiltonian as the
classic preconditioner (GFCC Workflow and Bottlenecks).  The learned variant
used as a flexible right preconditioner adds an elementwise correction to that
Jacobi step; this module states it plainly in FP64 so that the library's
kernels can be checked against it.

Per element d of a complex vector r (shift z = omega - i*eta, exact diagonal D
of Hbar_N, per-system scale sD = mean |D|, rms n = ||r|| / sqrt(dim)):

    rh = r / n                      (scale-free residual)
    jh = rh * sD / (z + D)          (scale-free Jacobi step)
    features x_d = [Re rh, Im rh, Re jh, Im jh, D/sD - 1, omega, [d < o], 100 eta]
    y_d = W3 tanh(W2 tanh(W1 x_d + b1) + b2) + b3          (2 outputs)
    M(r)_d = r_d / (z + D_d) + (y_d0 + i y_d1) * n / sD

Training target for a pair (r, e) with A e = r:  t_d = e_d * sD / n - jh_d, so
the network learns the part of the exact correction the Jacobi step misses;
loss = mean over sampled elements of |y - t|^2.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 8


def init_params(width, seed=0):
    """Xavier-uniform hidden layers, zero output layer (starts as plain Jacobi)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def xavier(n_out, n_in):
        lim = np.sqrt(6.0 / (n_in + n_out))
        return rng.uniform(-lim, lim, size=(n_out, n_in))

    return {"W1": xavier(width, N_FEAT), "b1": np.zeros(width),
            "W2": xavier(width, width), "b2": np.zeros(width),
            "W3": np.zeros((2, width)), "b3": np.zeros(2)}


def flatten(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]])


def unflatten(v, width):
    W = width
    sizes = [("W1", (W, N_FEAT)), ("b1", (W,)), ("W2", (W, W)), ("b2", (W,)), ("W3", (2, W)), ("b3", (2,))]
    out, k = {}, 0
    for name, shp in sizes:
        n = int(np.prod(shp))
        out[name] = np.asarray(v[k:k + n]).reshape(shp)
        k += n
    return out


def n_params(width):
    return width * N_FEAT + width + width * width + width + 2 * width + 2


def features(r, diag, omega, eta, n_occ, sD):
    """Feature matrix [dim, 8] for one complex vector r."""
    r = np.asarray(r, dtype=complex)
    dim = r.size
    n = np.linalg.norm(r) / np.sqrt(dim)
    rh = r / n
    z = omega - 1j * eta
    jh = rh * sD / (z + diag)
    X = np.zeros((dim, N_FEAT))
    X[:, 0], X[:, 1] = rh.real, rh.imag
    X[:, 2], X[:, 3] = jh.real, jh.imag
    X[:, 4] = diag / sD - 1.0
    X[:, 5] = omega
    X[:n_occ, 6] = 1.0
    X[:, 7] = 100.0 * eta
    return X, n


def forward(p, X):
    H1 = np.tanh(X @ p["W1"].T + p["b1"])
    H2 = np.tanh(H1 @ p["W2"].T + p["b2"])
    Y = H2 @ p["W3"].T + p["b3"]
    return Y, (H1, H2)


def loss_and_grad(p, X, T):
    """L = mean_n sum_k (Y - T)^2 and its gradient (dict like p)."""
    N = X.shape[0]
    Y, (H1, H2) = forward(p, X)
    dY = 2.0 * (Y - T) / N
    L = float(np.sum((Y - T) ** 2) / N)
    g = {"W3": dY.T @ H2, "b3": dY.sum(0)}
    dH2 = (dY @ p["W3"]) * (1.0 - H2 ** 2)
    g["W2"], g["b2"] = dH2.T @ H1, dH2.sum(0)
    dH1 = (dH2 @ p["W2"]) * (1.0 - H1 ** 2)
    g["W1"], g["b1"] = dH1.T @ X, dH1.sum(0)
    return L, g


def apply(p, r, diag, omega, eta, n_occ, sD):
    """M(r): Jacobi step plus the network's correction."""
    X, n = features(r, diag, omega, eta, n_occ, sD)
    Y, _ = forward(p, X)
    z = omega - 1j * eta
    return np.asarray(r) / (z + diag) + (Y[:, 0] + 1j * Y[:, 1]) * n / sD


def targets(r, e, diag, omega, eta, sD):
    """t_d = e_d sD / n - jh_d for a pair with A e = r."""
    r = np.asarray(r, dtype=complex)
    n = np.linalg.norm(r) / np.sqrt(r.size)
    z = omega - 1j * eta
    t = np.asarray(e) * sD / n - (r / n) * sD / (z + diag)
    return np.stack([t.real, t.imag], axis=1)


def adam_step(p, g, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in place; `state` holds m, v and the step count."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
