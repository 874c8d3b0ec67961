"""GPU tests of the runtime pieces: hipGraph replay of the inner iteration and
the ring-GEMM tile autotuner (neither may change results beyond roundoff)."""
import json
import os

import numpy as np
import pytest

from synth import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_04768_amd import gfcc  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    s = make_system(10, 48, 60, 777, sigma_L=0.1, sigma_t1=0.01)
    c = gfcc.Context.from_system(s)
    yield s, c
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_graph_replay_matches_eager(ctx, prec):
    """Graph replays (many, with eager cycle-finishing work between them) give
    the same G as eager launches, bit for bit."""
    s, c = ctx
    rng = np.random.default_rng(1)
    p = rng.integers(0, s.n_occ, size=24)
    w = rng.uniform(-1.2, -0.3, size=24)
    Ge, ie, _ = c.solve(p, w, 0.01, tol=1e-10, batch=8, precision=prec, use_graph=False)
    c.prof_enable(False)  # clears the counters
    Gg, ig, _ = c.solve(p, w, 0.01, tol=1e-10, batch=8, precision=prec, use_graph=True)
    assert all(i["status"] == 0 for i in ie + ig)
    assert [i["iters"] for i in ie] == [i["iters"] for i in ig]
    assert torch.equal(Ge, Gg)
    # the capture is kept across cycle finishing (no buffer is reallocated there): a few window
    # shapes are captured once each and the rest of the iterations are replays
    cap, rep = c.prof_get("graph_capture")["count"], c.prof_get("graph_replay")["count"]
    print(f"[graph] {prec}: {cap} captures, {rep} replays")
    assert 1 <= cap <= 8 and rep >= 4 * cap  # measured: 1 capture, 35 (FP64) and 40 (BF16) replays


def _counters(c):
    return {k: c.prof_get(k)["count"] for k in ("host_sync", "loop_sync", "inner_iter", "slot_iter")}


@pytest.mark.parametrize("prec,graph", [("fp64", False), ("bf16", True), ("fp16", False)])
def test_runs_between_synchronisations(ctx, prec, graph):
    """Runs of several inner iterations between host synchronisations: a slot whose cycle stops
    inside a run is frozen on the device, so G, the iteration counts and the true residuals are
    the same bits as with a synchronisation after every iteration; the automatic run length cuts
    the inner-loop synchronisations at least threefold (measured 3.5-4x) and all host
    synchronisations of the solve at least twofold.  (FP16: the per-call vector scale is taken
    over every plane of the batch, frozen ones included, so a scale can differ by a power of two and
    move which tiny entries are subnormal: G agrees to the solve tolerance instead of bitwise.)"""
    s, c = ctx
    rng = np.random.default_rng(11)
    p = rng.integers(0, s.n_occ, size=40)
    w = rng.uniform(-1.2, -0.3, size=40)
    runs = {}
    for se in (1, 0, 5):
        c.prof_enable(False)  # clears the counters
        G, info, _ = c.solve(p, w, 0.01, tol=1e-10, restart=30, batch=16, precision=prec, use_graph=graph,
                             sync_every=se)
        runs[se] = (G, info, _counters(c))
    G1, i1, k1 = runs[1]
    assert all(i["status"] == 0 for i in i1)
    assert k1["loop_sync"] == k1["inner_iter"]
    for se in (0, 5):
        G, info, k = runs[se]
        print(f"[sync] {prec} sync_every={se}: {k} (every iteration: {k1})")
        if prec == "fp16":
            assert all(i["status"] == 0 and i["true_rel_resid"] <= 1e-10 for i in info)
            assert ((G - G1).abs() / G1.abs()).max().item() < 1e-8
            continue
        assert torch.equal(G, G1), se
        assert info == i1, se
        assert k["slot_iter"] >= k1["slot_iter"]
    k0 = runs[0][2]
    assert 3 * k0["loop_sync"] <= k1["loop_sync"], (k0, k1)
    assert 2 * k0["host_sync"] <= k1["host_sync"], (k0, k1)
    # the price: sigma planes of frozen slots (right-hand-side iterations launched)
    assert k0["slot_iter"] <= 1.5 * k1["slot_iter"], (k0, k1)


def test_runs_between_synchronisations_several_systems(ctx):
    """The same bit identity for several systems in one persistent solve (lanes of different size
    and convergence), eager and with graph replay."""
    s, c = ctx
    s2 = make_system(6, 20, 30, 779, sigma_L=0.1, sigma_t1=0.01)
    c2 = gfcc.Context.from_system(s2)
    try:
        rng = np.random.default_rng(13)
        sys_ = np.array([0, 1] * 15)
        p = np.array([int(rng.integers(0, 10)) if k == 0 else int(rng.integers(0, 6)) for k in sys_])
        w = rng.uniform(-1.2, -0.3, size=30)
        for graph in (False, True):
            M1, i1 = gfcc.solve_multi([c, c2], sys_, p, w, 0.01, tol=1e-10, batch=12, precision="bf16",
                                      use_graph=graph, sync_every=1)
            M0, i0 = gfcc.solve_multi([c, c2], sys_, p, w, 0.01, tol=1e-10, batch=12, precision="bf16",
                                      use_graph=graph, sync_every=0)
            assert all(x["status"] == 0 for x in i1)
            assert torch.equal(M0, M1) and i0 == i1, graph
    finally:
        c2.close()


def test_runs_respect_the_iteration_budget(ctx):
    """max_iter is an exact budget also inside runs of iterations (status 1, iters == max_iter)."""
    s, c = ctx
    p = [0, 3, 7]
    w = [-0.5, -0.8, -1.1]
    for se in (0, 6):
        G, info, _ = c.solve(p, w, 0.01, tol=1e-15, restart=30, max_iter=13, batch=3, sync_every=se)
        assert [i["status"] for i in info] == [1, 1, 1]
        assert [i["iters"] for i in info] == [13, 13, 13]


def test_autotuner_cache_and_results(ctx, tmp_path):
    s, c = ctx
    cache = str(tmp_path / "tune.json")
    p = list(range(s.n_occ)) * 2
    w = list(np.linspace(-1.1, -0.4, s.n_occ)) * 2
    G0, _, _ = c.solve(p, w, 0.01, tol=1e-11, batch=16)
    G1, _, _ = c.solve(p, w, 0.01, tol=1e-11, batch=16, tune_cache=cache)
    assert os.path.exists(cache)
    ent = json.load(open(cache))["entries"]
    assert ent and all(0 <= e["cfg"] < 21 for e in ent)
    rel = (torch.abs(G1 - G0) / torch.abs(G0)).max().item()
    assert rel < 1e-10


def test_repeat_runs_are_bitwise_identical(ctx):
    """Determinism: the same request twice gives the same bits (restarted solver in FP64 and
    BF16-IR, multi-shift solver, several systems in one solve with and without graph replay)."""
    s, c = ctx
    rng = np.random.default_rng(5)
    p = rng.integers(0, s.n_occ, size=12)
    w = rng.uniform(-1.2, -0.3, size=12)
    for prec in ("fp64", "bf16"):
        G1, _, _ = c.solve(p, w, 0.01, tol=1e-10, batch=5, precision=prec)
        G2, _, _ = c.solve(p, w, 0.01, tol=1e-10, batch=5, precision=prec)
        assert torch.equal(G1, G2), prec
    S1, _, _ = c.solve_shifts([0, 3, 9], w[:6], 0.01, tol=1e-10)
    S2, _, _ = c.solve_shifts([0, 3, 9], w[:6], 0.01, tol=1e-10)
    assert torch.equal(S1, S2)
    s2 = make_system(6, 20, 30, 778, sigma_L=0.1, sigma_t1=0.01)
    c2 = gfcc.Context.from_system(s2)
    try:
        sys_ = np.array([0, 1] * 6)
        pp = np.array([int(x) % 6 for x in p])
        M1, _ = gfcc.solve_multi([c, c2], sys_, pp, w, 0.01, tol=1e-10, batch=6, precision="bf16")
        M2, _ = gfcc.solve_multi([c, c2], sys_, pp, w, 0.01, tol=1e-10, batch=6, precision="bf16")
        M3, _ = gfcc.solve_multi([c, c2], sys_, pp, w, 0.01, tol=1e-10, batch=6, precision="bf16", use_graph=True)
        assert torch.equal(M1, M2) and torch.equal(M1, M3)
    finally:
        c2.close()


HDR = 24  # resume-file header: magic, version, record size, request fingerprint


def test_checkpoint_resume(ctx, tmp_path):
    """Resume file: every finished right-hand side is appended after the header; a repeated
    request restores all of them without solving (same bits, same info, zero X rows); a
    truncated file restores its rows and solves the rest; records of other (p, omega) pairs
    of the same request are ignored."""
    s, c = ctx
    rng = np.random.default_rng(9)
    p = rng.integers(0, s.n_occ, size=16)
    w = rng.uniform(-1.2, -0.3, size=16)
    ck = str(tmp_path / "ck.bin")
    G0, i0, _ = c.solve(p, w, 0.01, tol=1e-10, batch=4, checkpoint=ck)
    size = os.path.getsize(ck)
    assert (size - HDR) % 16 == 0
    rec = (size - HDR) // 16
    X = torch.full((16, c.dim), 7.0 + 1.0j, dtype=torch.complex128, device=c.device)
    G1, i1, X1 = c.solve(p, w, 0.01, tol=1e-10, batch=4, checkpoint=ck, want_x=True, x_out=X)
    assert torch.equal(G0, G1) and i0 == i1
    assert torch.count_nonzero(X1).item() == 0  # restored rows carry no solution: zeros, not stale data
    assert os.path.getsize(ck) == size  # nothing was solved again
    ck2 = str(tmp_path / "ck2.bin")
    with open(ck, "rb") as f, open(ck2, "wb") as g:
        g.write(f.read(HDR + 6 * rec + rec // 2))  # header, six whole records and a torn one
    G2, i2, _ = c.solve(p, w, 0.01, tol=1e-10, batch=4, checkpoint=ck2)
    assert all(x["status"] == 0 for x in i2)
    assert (torch.abs(G2 - G0) / torch.abs(G0)).max().item() < 1e-8
    G3, i3, _ = c.solve(p, w + 0.01, 0.01, tol=1e-10, batch=4, checkpoint=ck)
    assert all(x["iters"] > 0 for x in i3)
    assert os.path.getsize(ck) == 2 * size - HDR


def test_checkpoint_refuses_foreign_and_mismatched_files(ctx, tmp_path):
    """A file that is not a resume file, or one written for another system, tolerance,
    precision or q list, is refused with an argument error and left byte for byte unchanged."""
    s, c = ctx
    p = [0, 1, 2, 3]
    w = [-1.0, -0.8, -0.6, -0.4]
    foreign = tmp_path / "results.txt"
    foreign.write_bytes(b"omega G\n-1.0 0.5\n" * 40)
    before = foreign.read_bytes()
    with pytest.raises(gfcc.GfccError, match="not a resume file"):
        c.solve(p, w, 0.01, tol=1e-10, checkpoint=str(foreign))
    assert foreign.read_bytes() == before
    ck = tmp_path / "ck.bin"
    c.solve(p, w, 0.01, tol=1e-10, checkpoint=str(ck))
    good = ck.read_bytes()
    for kw in (dict(tol=1e-9), dict(tol=1e-10, precision="bf16"), dict(tol=1e-10, q=[0, 1]),
               dict(tol=1e-10, restart=20)):
        with pytest.raises(gfcc.GfccError, match="different request"):
            c.solve(p, w, 0.01, checkpoint=str(ck), **kw)
        assert ck.read_bytes() == good
    s2 = make_system(10, 48, 60, 779, sigma_L=0.1, sigma_t1=0.01)  # same shape, other system
    c2 = gfcc.Context.from_system(s2)
    try:
        with pytest.raises(gfcc.GfccError, match="different request"):
            c2.solve(p, w, 0.01, tol=1e-10, checkpoint=str(ck))
        assert ck.read_bytes() == good
    finally:
        c2.close()
