"""GPU parity of multi-shift GMRES (gfcc_solve_shifts): one real Krylov basis per
orbital serves every frequency.

* tiny system: G for occupied and virtual p, off-diagonal and virtual q, against
  dense direct solves with the oracle's b_p and c_q; the oracle's true residual
  of the returned X; the reported residuals;
* equality with the restarted solver (gfcc_solve_batch, FP64) at a tight tolerance;
* orbital window smaller than the request (refill) equals the full window;
* max_dim too small: status 1 without a fallback, converged G with it;
* estimate-only acceptance (verify = 0); b_p = 0; argument errors;
* the 40/200/800 system on the benchmark's frequency grid: every (p, omega)
  converged, sampled G against FP64 restarted solves, sampled X against the
  oracle's true residual.
"""
import numpy as np
import pytest

from oracle import ipgfcc as O
from synth import make_system, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_04768_amd import gfcc  # noqa: E402

ETA = 0.01
WS = np.linspace(-1.0, -0.2, 6)


@pytest.fixture(scope="module")
def tiny():
    s = make_system(4, 16, 48, 2010_04768 + 3, sigma_t1=0.03)
    im = O.intermediates(s)
    A = O.explicit_matrix(im)
    ctx = gfcc.Context.from_system(s)

    def direct(p, w):
        return np.linalg.solve((w - 1j * ETA) * np.eye(s.dim) + A, O.rhs(s, p))

    yield s, im, ctx, direct
    ctx.close()


def test_shifts_match_direct(tiny):
    s, im, ctx, direct = tiny
    o, v = s.n_occ, s.n_vir
    P = [0, 1, 2, 3, o, o + 9]
    Q = [0, 3, o, o + v - 1]
    tol = 1e-10
    G, info, X = ctx.solve_shifts(P, WS, ETA, q=Q, tol=tol, want_x=True)
    G = G.cpu().numpy()
    X = X.cpu().numpy()
    C = np.stack([O.left_vector(s, q) for q in Q])
    for i, p in enumerate(P):
        b = O.rhs(s, p)
        for k, w in enumerate(WS):
            assert info[i][k]["status"] == 0 and info[i][k]["true_rel_resid"] <= tol, (p, w, info[i][k])
            res = b - O.shifted_operator(im, w, ETA)(X[i, k])
            assert np.linalg.norm(res) <= 1.05 * tol * np.linalg.norm(b), (p, w)
            g = C @ X[i, k]
            assert np.abs(G[i, k] - g).max() <= 1e-12 * np.abs(g).max(), (p, w)
            gd = C @ direct(p, w)  # within the conditioning of the shifted operator (1 / eta)
            assert np.abs(G[i, k] - gd).max() <= 1e3 * tol * np.abs(gd).max(), (p, w)
    # one basis per orbital: every frequency of an orbital used at most the same basis size
    assert max(info[i][k]["iters"] for i in range(len(P)) for k in range(len(WS))) <= s.dim


def test_shifts_equal_restarted_solver(tiny):
    s, im, ctx, direct = tiny
    P = [0, 2, 3]
    G, info, _ = ctx.solve_shifts(P, WS, ETA, tol=1e-12)
    Gr, inr, _ = ctx.solve(np.repeat(P, len(WS)), np.tile(WS, len(P)), ETA, tol=1e-12, precision="fp64")
    G = G.cpu().numpy()[:, :, 0]
    Gr = Gr.cpu().numpy()[:, 0].reshape(len(P), len(WS))
    assert np.abs(G - Gr).max() <= 1e-9 * np.abs(Gr).max()


def test_shifts_window_refill(tiny):
    s, im, ctx, direct = tiny
    P = [3, 0, 1, 2, 3]
    G1, i1, _ = ctx.solve_shifts(P, WS, ETA, tol=1e-11)
    G2, i2, _ = ctx.solve_shifts(P, WS, ETA, tol=1e-11, batch=2)
    G1 = G1.cpu().numpy()
    G2 = G2.cpu().numpy()
    assert np.abs(G1 - G2).max() <= 1e-10 * np.abs(G1).max()
    assert np.array_equal(G1[0], G1[4])  # the same orbital twice in one window


def test_shifts_max_dim_and_fallback(tiny):
    s, im, ctx, direct = tiny
    P = [0, 3]
    G, info, _ = ctx.solve_shifts(P, WS, ETA, tol=1e-10, max_dim=4)
    assert all(x["status"] == 1 and x["iters"] == 4 for row in info for x in row)
    G, info, X = ctx.solve_shifts(P, WS, ETA, tol=1e-10, max_dim=4, want_x=True,
                                  fallback=dict(precond="jacobi", precision="fp64", tol=1e-10))
    G = G.cpu().numpy()[:, :, 0]
    for i, p in enumerate(P):
        for k, w in enumerate(WS):
            assert info[i][k]["status"] == 0 and info[i][k]["restarts"] >= 1
            g = O.left_vector(s, p) @ direct(p, w)
            assert abs(G[i, k] - g) <= 1e3 * 1e-10 * abs(g)
            b = O.rhs(s, p)
            res = b - O.shifted_operator(im, w, ETA)(X[i, k].cpu().numpy())
            assert np.linalg.norm(res) <= 1.05e-10 * np.linalg.norm(b)


def test_shifts_estimate_only(tiny):
    s, im, ctx, direct = tiny
    G, info, _ = ctx.solve_shifts([1], WS, ETA, tol=1e-10, verify=False)
    G = G.cpu().numpy()[0, :, 0]
    for k, w in enumerate(WS):
        g = O.left_vector(s, 1) @ direct(1, w)
        assert abs(G[k] - g) <= 1e3 * 1e-10 * abs(g)


def test_shifts_zero_rhs_and_errors():
    s = make_system(3, 6, 10, 2010_04768 + 4, t1=False, t2=False)
    im = O.intermediates(s)
    ctx = gfcc.Context.from_system(s)
    try:
        o = s.n_occ
        G, info, X = ctx.solve_shifts([o, 1, o + 4], WS, ETA, q=[0, 1, 2], tol=1e-12, want_x=True)
        G = G.cpu().numpy()
        X = X.cpu().numpy()
        assert not np.any(G[0]) and not np.any(G[2]) and not np.any(X[0]) and not np.any(X[2])
        assert all(x["status"] == 0 and x["iters"] == 0 for x in info[0] + info[2])
        for k, w in enumerate(WS):
            x, _, _ = O.solve(s, im, 1, w, ETA, tol=1e-13)
            g = np.array([O.left_vector(s, q) @ x for q in (0, 1, 2)])
            assert np.abs(G[1, k] - g).max() <= 1e-10 * np.abs(g).max()
        with pytest.raises(gfcc.GfccError):
            ctx.solve_shifts([0], WS, ETA, max_dim=513)
        with pytest.raises(gfcc.GfccError):
            ctx.solve_shifts([o + 6], WS, ETA)
        with pytest.raises(gfcc.GfccError):
            ctx.solve_shifts([0], [float("nan")], ETA)
    finally:
        ctx.close()


def test_shifts_benchmark_shape():
    """40/200/800 system, 64 frequencies on [-1.2, -0.3], five orbitals."""
    wl = make_workload("plain-o40v200", n_omega=64)
    s, ws = wl.systems[0], wl.omegas[0]
    ps = [0, 13, 20, 39, 40]  # 40 is the lowest virtual orbital
    ctx = gfcc.Context.from_system(s)
    try:
        G, info, _ = ctx.solve_shifts(ps, ws, wl.eta, tol=wl.tol)
        iters = [x["iters"] for row in info for x in row]
        print("multi-shift basis sizes per orbital", [max(x["iters"] for x in row) for row in info])
        assert all(x["status"] == 0 and x["true_rel_resid"] <= wl.tol for row in info for x in row)
        assert max(iters) <= 160
        G = G.cpu().numpy()[:, :, 0]
        ks = [0, 21, 63]
        P = np.repeat(ps, len(ks))
        W = np.tile(ws[ks], len(ps))
        Gr, inr, Xr = ctx.solve(P, W, wl.eta, tol=1e-11, precision="fp64", max_iter=3000)
        assert all(x["status"] == 0 for x in inr)
        Gr = Gr.cpu().numpy()[:, 0].reshape(len(ps), len(ks))
        err = np.abs(G[:, ks] - Gr) / np.abs(Gr)
        print("multi-shift G max rel err vs FP64 restarted", err.max())
        assert err.max() <= 1e-7
        # the oracle's own residual of two multi-shift solutions
        G1, info1, X1 = ctx.solve_shifts([39, 40], ws[[5, 50]], wl.eta, tol=wl.tol, want_x=True)
        im = O.intermediates(s)
        for i, p in enumerate([39, 40]):
            w = ws[[5, 50]][i]
            x = X1[i, i].cpu().numpy()
            b = O.rhs(s, p)
            res = b - O.shifted_operator(im, w, wl.eta)(x)
            assert np.linalg.norm(res) <= 1.05 * wl.tol * np.linalg.norm(b)
    finally:
        ctx.close()


def test_spectral_function(tiny):
    """A(omega) on the GPU from the multi-shift G_pp equals the oracle's spectral function of the
    oracle's G, and is unchanged when eta changes sign (G -> conj G)."""
    s, im, ctx, direct = tiny
    P = [0, 1, 2, 3]
    Go = np.array([[O.left_vector(s, p) @ direct(p, w) for p in P] for w in WS])  # [omega][p]
    Ao = O.spectral_function(Go)
    G, info, _ = ctx.solve_shifts(P, WS, ETA, tol=1e-12)
    A = gfcc.spectral(G, ETA).cpu().numpy()
    assert np.abs(A - Ao).max() <= 1e-9 * np.abs(Ao).max()
    Gm, _, _ = ctx.solve_shifts(P, WS, -ETA, tol=1e-12)
    Am = gfcc.spectral(Gm, -ETA).cpu().numpy()
    assert np.abs(Am - Ao).max() <= 1e-9 * np.abs(Ao).max()
    assert np.all(A > 0)
