"""GPU parity of model-order reduction (gfcc_mor_*) against the oracle.

* basis: orthonormal, spans every accepted candidate; Hhat equals the oracle's
  projection through its own sigma on the GPU basis;
* model G equals the oracle's model on the same basis, is independent of the
  basis choice (oracle's own Gram-Schmidt) and exact at the basis frequencies;
* extending in two calls equals extending once;
* the level loop reproduces the oracle's schedule (including a split level)
  and its G on the whole grid; at the benchmark shape the model G matches
  direct FP64 solves at frequencies that were never solved;
* error paths: empty basis, non-uniform grid.
"""
import numpy as np
import pytest

from oracle import ipgfcc as O
from oracle import mor as M
from synth import make_system, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_04768_amd import gfcc  # noqa: E402

ETA = 0.01


@pytest.fixture(scope="module")
def tiny():
    s = make_system(4, 16, 48, 2010_04768 + 1)
    im = O.intermediates(s)
    A = O.explicit_matrix(im)
    ctx = gfcc.Context.from_system(s)

    def direct(p, w):
        return np.linalg.solve((w - 1j * ETA) * np.eye(s.dim) + A, O.rhs(s, p))

    yield s, im, ctx, direct
    ctx.close()


def _X(direct, ws, ps):
    return np.stack([direct(p, w) for w in ws for p in ps])


def test_basis_and_projection(tiny):
    s, im, ctx, direct = tiny
    X = _X(direct, [-0.9, -0.5], range(4))
    ctx.mor_reset()
    m = ctx.mor_extend(torch.from_numpy(X))
    assert m == 16
    S = ctx.mor_export("BASIS").cpu().numpy().T
    assert np.abs(S.T @ S - np.eye(m)).max() < 1e-12
    C = M.candidates(X.T)
    assert np.abs(S @ (S.T @ C) - C).max() < 1e-10 * np.abs(C).max()
    H = ctx.mor_export("HHAT").cpu().numpy()
    Ho = M.project(im, S)
    assert np.abs(H - Ho).max() < 1e-12 * np.abs(Ho).max()


def test_model_matches_oracle(tiny):
    s, im, ctx, direct = tiny
    ws_b = [-0.9, -0.5]
    X = _X(direct, ws_b, range(4))
    ctx.mor_reset()
    ctx.mor_extend(torch.from_numpy(X))
    S = ctx.mor_export("BASIS").cpu().numpy().T
    ws = np.array([-1.0, -0.9, -0.63, -0.5, -0.2])
    G = ctx.mor_model([0, 1, 2, 3], ws, ETA, q=[0, 1, 2, 3]).cpu().numpy()
    Go = M.model_greens(s, S, M.project(im, S), [0, 1, 2, 3], ws, ETA)
    assert np.abs(G - Go).max() < 1e-11 * np.abs(Go).max()
    So, _ = M.extend_basis(np.zeros((s.dim, 0)), M.candidates(X.T))
    Go2 = M.model_greens(s, So, M.project(im, So), [0, 1, 2, 3], ws, ETA)
    assert np.abs(G - Go2).max() < 1e-9 * np.abs(Go2).max()
    for k in (1, 3):  # basis frequencies: exact
        for p in range(4):
            x = direct(p, ws[k])
            for q in range(4):
                g = O.left_vector(s, q) @ x
                assert abs(G[k, p, q] - g) <= 1e-9 * max(abs(g), 1e-3)
    Gd = ctx.mor_model([0, 2], ws, ETA).cpu().numpy()
    assert np.abs(Gd - np.stack([G[:, 0, 0], G[:, 2, 2]], axis=1)).max() < 1e-13 * np.abs(Gd).max()


def test_two_extends_equal_one(tiny):
    s, im, ctx, direct = tiny
    X = _X(direct, [-0.9, -0.5, -0.3], range(4))
    ws = np.linspace(-1.0, -0.2, 9)
    ctx.mor_reset()
    ctx.mor_extend(torch.from_numpy(X))
    G1 = ctx.mor_model([0, 1, 2, 3], ws, ETA).cpu().numpy()
    ctx.mor_reset()
    ctx.mor_extend(torch.from_numpy(X[:5]))
    m = ctx.mor_extend(torch.from_numpy(X[5:]))
    assert m == 24
    G2 = ctx.mor_model([0, 1, 2, 3], ws, ETA).cpu().numpy()
    assert np.abs(G1 - G2).max() < 1e-10 * np.abs(G1).max()


@pytest.mark.parametrize("tol", [1e-8, 2e-11])
def test_level_loop_matches_oracle(tiny, tol):
    s, im, ctx, direct = tiny
    ws = M.grid(-1.0, -0.2, 0.01)
    out = M.levels(s, im, [0, 1, 2, 3], ws, ETA, tol=tol, solver=direct)
    G, rep, lev = ctx.mor_greens([0, 1, 2, 3], ws, ETA, tol=tol, solve_tol=1e-13, precision="fp64")
    print("oracle levels", out["levels"], "gpu report", rep)
    want = np.zeros(len(ws), dtype=np.int32)
    for L, pts in enumerate(out["levels"], start=1):
        want[pts] = L
    assert np.array_equal(lev, want)
    assert rep["levels"] == len(out["levels"]) and rep["m"] == out["S"].shape[1]
    assert rep["per_level"] == [len(x) for x in out["levels"]]
    G = G.cpu().numpy()
    assert np.abs(G - out["G"]).max() <= 1e-9 * np.abs(out["G"]).max()
    for k in range(0, len(ws), 5):
        for p in range(4):
            g = O.left_vector(s, p) @ direct(p, ws[k])
            assert abs(G[k, p] - g) <= 1e-8 * abs(g)


def test_errors(tiny):
    s, im, ctx, direct = tiny
    ctx.mor_reset()
    with pytest.raises(gfcc.GfccError):
        ctx.mor_model([0], [-0.5], ETA)
    with pytest.raises(gfcc.GfccError):
        ctx.mor_greens([0], np.array([-1.0, -0.7, -0.2]), ETA)
    with pytest.raises(gfcc.GfccError):
        ctx.mor_model([7], [-0.5], ETA)


def test_level_loop_benchmark_shape():
    """40/200/800 system on the benchmark's 64-point grid, three p: model G at
    frequencies never solved directly against direct FP64 solves (tol 1e-11)."""
    wl = make_workload("plain-o40v200", n_omega=64)
    s, ws = wl.systems[0], wl.omegas[0]
    ps = [0, 20, 39]
    ctx = gfcc.Context.from_system(s)
    try:
        G, rep, lev = ctx.mor_greens(ps, ws, wl.eta, tol=1e-9, solve_tol=1e-10, precision="bf16")
        print("benchmark-shape MOR report", rep, "solved", np.nonzero(lev)[0].tolist())
        assert rep["all_solves_converged"]
        G = G.cpu().numpy()
        ks = [k for k in (5, 17, 27, 45, 58) if lev[k] == 0]
        assert ks
        P = np.repeat(ps, len(ks))
        W = np.tile(ws[ks], len(ps))
        Gr, info, _ = ctx.solve(P, W, wl.eta, tol=1e-11, precision="fp64", max_iter=3000)
        Gr = Gr.cpu().numpy()[:, 0].reshape(len(ps), len(ks))
        err = np.abs(G[ks][:, :].T - Gr) / np.abs(Gr)
        print("MOR max rel err at unsolved frequencies", err.max())
        assert err.max() <= 1e-8
    finally:
        ctx.close()


def test_level_loop_degenerate_grids(tiny):
    """One or two frequencies: no level structure, every point solved directly."""
    s, im, ctx, direct = tiny
    for ws in (np.array([-0.55]), np.array([-0.9, -0.3])):
        G, rep, lev = ctx.mor_greens([0, 2], ws, ETA, tol=1e-8, solve_tol=1e-13, precision="fp64")
        assert rep["levels"] == 1 and list(lev) == [1] * len(ws)
        G = G.cpu().numpy()
        for k, w in enumerate(ws):
            for i, p in enumerate((0, 2)):
                g = O.left_vector(s, p) @ direct(p, w)
                assert abs(G[k, i] - g) <= 1e-10 * abs(g)
