"""Parity at the full 40-occupied / 200-virtual / 800-Cholesky workload, in the
launch configuration the benchmark times (128-slot window, BF16 GMRES-IR).

* every exported FP64 block and the exact diagonal against the oracle (1e-12
  relative to the block's magnitude);
* sigma on random complex vectors against the oracle (1e-12);
* sampled solutions: the oracle's own true residual of the GPU solution
  X_gpu is <= tol (a property that holds at any size), and the GPU G equals
  c_q^T X_gpu with the oracle's left vector.
"""
import numpy as np
import pytest

from oracle import ipgfcc as O
from synth import make_workload, random_vectors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_04768_amd import gfcc  # noqa: E402


@pytest.fixture(scope="module")
def full():
    wl = make_workload("plain-o40v200", n_omega=4)
    s = wl.systems[0]
    im = O.intermediates(s)
    ctx = gfcc.Context.from_system(s)
    yield wl, s, im, ctx
    ctx.close()


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


def test_fullsize_blocks(full):
    wl, s, im, ctx = full
    for blk, key in [("FOO", "Foo"), ("FVV", "Fvv"), ("FOV", "Fov"), ("WOOOO", "Woooo"), ("WOOOV", "Wooov"),
                     ("WOVOO", "Wovoo"), ("WOVVO", "Wovvo"), ("WOVOV", "Wovov")]:
        assert _rel(ctx.export(blk).cpu().numpy(), im[key]) < 1e-12, blk
    assert _rel(ctx.export("DIAG").cpu().numpy(), O.diagonal(im)) < 1e-12
    q = [0, 17, 39]
    C = ctx.export("LEFT").cpu().numpy()
    for qq in q:
        assert _rel(C[qq], O.left_vector(s, qq)) < 1e-12


def test_fullsize_sigma(full):
    wl, s, im, ctx = full
    X = random_vectors(2, s.dim, seed=11)
    Y = ctx.sigma(torch.from_numpy(X)).cpu().numpy()
    assert _rel(Y, O.sigma(im, X)) < 1e-12


def test_fullsize_solve_bench_configuration(full):
    """The benchmark's launch configuration: automatic window (512 slots once 640 right-hand sides
    are queued), BF16-IR, graph replay of the inner iteration; sampled solutions checked with the
    oracle's own residual and left vectors."""
    wl, s, im, ctx = full
    ws = np.linspace(wl.omegas[0][0], wl.omegas[0][-1], 16)
    P = np.repeat(wl.p_lists[0], len(ws))
    W = np.tile(ws, len(wl.p_lists[0]))  # 640 right-hand sides -> the 512-slot window
    G, info, X = ctx.solve(P, W, wl.eta, tol=wl.tol, precision="bf16", use_graph=True, want_x=True)
    assert all(i["status"] == 0 for i in info)
    G = G.cpu().numpy()[:, 0]
    for r in (0, 311, 639):
        x = X[r].cpu().numpy()
        res = O.rhs(s, P[r]) - O.shifted_operator(im, W[r], wl.eta)(x)
        assert np.linalg.norm(res) <= 1.05 * wl.tol, np.linalg.norm(res)
        g_or = O.left_vector(s, P[r]) @ x
        assert abs(G[r] - g_or) <= 1e-12 * abs(g_or)


def test_fullsize_virtual_orbitals(full):
    """Virtual p (b_p = [a_p, T]|Phi>) and virtual q at the full size, BF16 GMRES-IR:
    the oracle's true residual of X_gpu relative to |b_p|, and G against c_q^T X_gpu."""
    wl, s, im, ctx = full
    o, v = s.n_occ, s.n_vir
    P = [o, o + 117, o + v - 1, 5]
    W = [-0.62, -0.5, -0.71, -0.55]
    Q = [5, o, o + 117]
    G, info, X = ctx.solve(P, W, wl.eta, q=Q, tol=wl.tol, precision="bf16", batch=128, want_x=True)
    assert all(i["status"] == 0 for i in info), info
    G = G.cpu().numpy()
    C = np.stack([O.left_vector(s, q) for q in Q])
    for r in (0, 1, 3):
        x = X[r].cpu().numpy()
        b = O.rhs(s, P[r])
        res = b - O.shifted_operator(im, W[r], wl.eta)(x)
        assert np.linalg.norm(res) <= 1.05 * wl.tol * np.linalg.norm(b), np.linalg.norm(res)
        g = C @ x
        assert np.abs(G[r] - g).max() <= 1e-12 * np.abs(g).max()
