"""Several systems in one persistent solve (gfcc_solve_multi): one lane of slots
per system, all systems advancing together, the ring GEMMs of the systems in
grouped launches.

* three small systems of different shapes, interleaved in one queue: G equals
  each system's own gfcc_solve_batch and the oracle's dense direct solve, in
  FP64 and BF16 GMRES-IR, with a window smaller than the queue (refill) and
  with the inner iteration replayed as a hipGraph;
* uneven work: one system with many right-hand sides, one with a single one;
* the three-system mixed-precision workload (20/100/400, 40/180/720,
  60/300/1200): a sample of every system in one call, BF16 GMRES-IR against
  FP64 solves of each system to 1e-8;
* virtual p in the queue, and the resume file;
* argument errors.
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
SHAPES = [(4, 16, 48), (5, 7, 9), (3, 12, 20)]


@pytest.fixture(scope="module")
def three():
    out = []
    for k, (o, v, Q) in enumerate(SHAPES):
        s = make_system(o, v, Q, 2010_04768 + 20 + k, sigma_L=0.08, sigma_t1=0.02)
        im = O.intermediates(s)
        A = O.explicit_matrix(im)
        out.append((s, A, gfcc.Context.from_system(s)))
    yield out
    for _, _, c in out:
        c.close()


def _queue(three, per_sys, seed=0):
    rng = np.random.default_rng(seed)
    S, P, W = [], [], []
    for k, (s, _, _) in enumerate(three):
        for _ in range(per_sys[k]):
            S.append(k)
            P.append(int(rng.integers(0, s.n_occ)))
            W.append(float(rng.uniform(-1.0, -0.2)))
    perm = rng.permutation(len(S))
    return np.array(S)[perm], np.array(P)[perm], np.array(W)[perm]


def _direct(s, A, p, w):
    x = np.linalg.solve((w - 1j * ETA) * np.eye(s.dim) + A, O.rhs(s, p))
    return O.left_vector(s, p) @ x


@pytest.mark.parametrize("prec,tol,graph", [("fp64", 1e-11, False), ("bf16", 1e-10, False), ("fp64", 1e-11, True),
                                           ("fp16", 1e-10, True)])
def test_multi_matches_single_and_direct(three, prec, tol, graph):
    S, P, W = _queue(three, [9, 7, 8])
    ctxs = [c for _, _, c in three]
    G, info = gfcc.solve_multi(ctxs, S, P, W, ETA, tol=tol, batch=9, precision=prec, use_graph=graph)
    assert all(x["status"] == 0 and x["true_rel_resid"] <= tol for x in info), info
    G = G.cpu().numpy()[:, 0]
    for k, (s, A, c) in enumerate(three):
        idx = np.nonzero(S == k)[0]
        Gs, inf, _ = c.solve(P[idx], W[idx], ETA, tol=tol, precision=prec)
        Gs = Gs.cpu().numpy()[:, 0]
        assert np.abs(G[idx] - Gs).max() <= 1e2 * tol * np.abs(Gs).max(), k
        for r in idx[:3]:
            g = _direct(s, A, P[r], W[r])
            assert abs(G[r] - g) <= 1e3 * tol * abs(g), (k, r)


def test_multi_uneven_and_offdiagonal(three):
    S, P, W = _queue(three, [14, 1, 0], seed=3)
    ctxs = [c for _, _, c in three]
    Q = [0, 1, 2]
    G, info = gfcc.solve_multi(ctxs, S, P, W, ETA, q=Q, tol=1e-11, batch=4)
    assert all(x["status"] == 0 for x in info)
    G = G.cpu().numpy()
    for r in range(len(S)):
        s, A, _ = three[S[r]]
        x = np.linalg.solve((W[r] - 1j * ETA) * np.eye(s.dim) + A, O.rhs(s, P[r]))
        g = np.array([O.left_vector(s, q) @ x for q in Q])
        assert np.abs(G[r] - g).max() <= 1e-8 * np.abs(g).max(), r


def test_multi_errors(three):
    ctxs = [c for _, _, c in three]
    with pytest.raises(gfcc.GfccError):
        gfcc.solve_multi([ctxs[0], ctxs[0]], [0], [0], [-0.5], ETA)
    with pytest.raises(gfcc.GfccError):
        gfcc.solve_multi(ctxs, [3], [0], [-0.5], ETA)
    with pytest.raises(gfcc.GfccError):
        gfcc.solve_multi(ctxs, [1], [12], [-0.5], ETA)  # system 1 has 5 + 7 orbitals
    with pytest.raises(gfcc.GfccError):
        gfcc.solve_multi(ctxs, [0], [0], [-0.5], ETA, q=[14])  # valid for system 0, not for system 1
    G, info = gfcc.solve_multi(ctxs, [], [], [], ETA)
    assert G.shape[0] == 0


def test_multi_three_system_workload():
    """The mixed-precision workload's three systems in one call: BF16-IR G of every system
    within 1e-8 of that system's FP64 solve (tol 1e-11)."""
    wl = make_workload("mixed-3sys", n_omega=128)
    ctxs = [gfcc.Context.from_system(s) for s in wl.systems]
    try:
        S, P, W = [], [], []
        for k, s in enumerate(wl.systems):
            o = s.n_occ
            for p in (0, o // 2, o - 1):
                for w in wl.omegas[k][::32]:
                    S.append(k)
                    P.append(p)
                    W.append(w)
        S, P, W = np.array(S), np.array(P), np.array(W)
        G, info = gfcc.solve_multi(ctxs, S, P, W, wl.eta, tol=wl.tol, precision="bf16", use_graph=True)
        assert all(x["status"] == 0 for x in info)
        G = G.cpu().numpy()[:, 0]
        for k, c in enumerate(ctxs):
            idx = np.nonzero(S == k)[0]
            Gr, inf, _ = c.solve(P[idx], W[idx], wl.eta, tol=1e-11, precision="fp64", max_iter=3000)
            Gr = Gr.cpu().numpy()[:, 0]
            err = np.abs(G[idx] - Gr) / np.abs(Gr)
            print("system", k, "max rel G error BF16-IR (one launch) vs FP64", err.max())
            assert err.max() <= 1e-8
    finally:
        for c in ctxs:
            c.close()


def test_multi_virtual_orbitals_and_resume(three, tmp_path):
    """Virtual p in a multi-system queue (b_p = [a_p, T]|Phi>) against dense direct solves, and the
    resume file: a repeated request restores every row bit for bit."""
    ctxs = [c for _, _, c in three]
    S = np.array([0, 1, 2, 0, 1, 2])
    P = np.array([4, 5, 3, 19, 11, 1])  # virtual except the last
    W = np.array([-0.7, -0.5, -0.3, -0.9, -0.4, -0.6])
    ck = str(tmp_path / "multi.ckpt")
    G, info = gfcc.solve_multi(ctxs, S, P, W, ETA, tol=1e-11, batch=4, checkpoint=ck)
    assert all(x["status"] == 0 for x in info)
    G = G.cpu().numpy()[:, 0]
    for r in range(len(S)):
        s, A, _ = three[S[r]]
        x = np.linalg.solve((W[r] - 1j * ETA) * np.eye(s.dim) + A, O.rhs(s, P[r]))
        g = O.left_vector(s, P[r]) @ x
        assert abs(G[r] - g) <= 1e-8 * max(abs(g), 1e-4), r
    G2, info2 = gfcc.solve_multi(ctxs, S, P, W, ETA, tol=1e-11, batch=4, checkpoint=ck)
    assert np.array_equal(G2.cpu().numpy()[:, 0], G) and info2 == info
