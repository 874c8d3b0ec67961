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
    Gg, ig, _ = c.solve(p, w, 0.01, tol=1e-10, batch=8, precision=prec, use_graph=True)
    assert all(i["status"] == 0 for i in ie + ig)
    assert [i["iters"] for i in ie] == [i["iters"] for i in ig]
    assert torch.equal(Ge, Gg)


def test_autotuner_cache_and_results(ctx, tmp_path):
    s, c = ctx
    cache = str(tmp_path / "tune.json")
    p = list(range(s.n_occ)) * 2
    w = list(np.linspace(-1.1, -0.4, s.n_occ)) * 2
    G0, _, _ = c.solve(p, w, 0.01, tol=1e-11, batch=16)
    G1, _, _ = c.solve(p, w, 0.01, tol=1e-11, batch=16, tune_cache=cache)
    assert os.path.exists(cache)
    ent = json.load(open(cache))["entries"]
    assert ent and all(0 <= e["cfg"] < 13 for e in ent)
    rel = (torch.abs(G1 - G0) / torch.abs(G0)).max().item()
    assert rel < 1e-10
