"""The GEMM tiles that load operands straight into LDS stages (global_load_lds) against the
register-staged tiles of the same precision: the same K order of the MFMA steps, so sigma is the
same to the bit in BF16, FP16 (against the 16-wave 256x256 tile), FP64 and FP32 (against the
double-buffered 256x128 tile), on shapes with ragged M, N and K (a K remainder below one stage, K
below one stage) and one that fills several tiles.  The tile is forced through GFCC_TILE_<prec>."""
import numpy as np
import pytest

from synth import make_system, random_vectors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_04768_amd import gfcc  # noqa: E402

DMA_TILES = {"bf16": ["dma3_256x256", "dma4_256x256", "dma3_256x256w8", "dma3_256x256w8t", "dma2k64_256x256"],
             "fp64": ["dma3_256x128", "dma2_256x128", "dma2_128x256"]}
DMA_TILES["fp16"] = DMA_TILES["bf16"]
DMA_TILES["fp32"] = ["dma3_256x128", "dma2_256x128"]
REF_TILE = {"bf16": "db32_256x256w16", "fp16": "db32_256x256w16", "fp64": "db256x128", "fp32": "db256x128"}


@pytest.mark.parametrize("shape,nvec", [((5, 7, 9), 3), ((12, 45, 50), 5), ((20, 100, 400), 64)])
@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp64", "fp32"])
def test_dma_tiles_match_register_staged_tile(monkeypatch, shape, nvec, prec):
    o, v, Q = shape
    s = make_system(o, v, Q, 606 + o, sigma_L=0.1, sigma_t1=0.01)
    c = gfcc.Context.from_system(s)
    try:
        X = torch.from_numpy(random_vectors(nvec, c.dim, seed=2)).cuda()
        var = "GFCC_TILE_" + prec.upper()
        monkeypatch.setenv(var, REF_TILE[prec])
        ref = c.sigma(X, precision=prec)
        assert torch.isfinite(ref).all()
        for tile in DMA_TILES[prec]:
            monkeypatch.setenv(var, tile)
            Y = c.sigma(X, precision=prec)
            assert torch.equal(Y, ref), (tile, shape, prec)
        # and the default choice (no override) gives the same bits too
        monkeypatch.delenv(var)
        assert torch.equal(c.sigma(X, precision=prec), ref)
    finally:
        c.close()


def test_dma_tile_in_the_solver(monkeypatch):
    """BF16-IR solves (BF16 inner and FP64 true-residual products) with the direct-to-LDS tiles give
    the same G bits as with the register-staged tiles (the ring products run as grouped launches)."""
    s = make_system(10, 48, 60, 777, sigma_L=0.1, sigma_t1=0.01)
    c = gfcc.Context.from_system(s)
    try:
        p = [0, 3, 7, 9, 2]
        w = [-0.5, -0.8, -1.1, -0.4, -0.6]
        monkeypatch.setenv("GFCC_TILE_BF16", "db32_256x256w16")
        monkeypatch.setenv("GFCC_TILE_FP64", "db256x128")
        G0, i0, _ = c.solve(p, w, 0.01, tol=1e-10, precision="bf16")
        monkeypatch.setenv("GFCC_TILE_BF16", "dma2k64_256x256")
        monkeypatch.setenv("GFCC_TILE_FP64", "dma2_256x128")
        G1, i1, _ = c.solve(p, w, 0.01, tol=1e-10, precision="bf16")
        assert all(i["status"] == 0 for i in i1)
        assert torch.equal(G0, G1) and i0 == i1
    finally:
        c.close()
