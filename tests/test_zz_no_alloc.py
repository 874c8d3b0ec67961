"""The allocation-free Green's-function entry point (gfcc_greens_noalloc, fixed device
scratch) against gfcc_greens through the C ABI: two calls in a row, the second with a
smaller input, in the list and diagonal forms, on a small system (also against the oracle's
left vectors) and on the 40/200/800 system; requests beyond the fixed scratch are refused."""
import numpy as np
import pytest

from oracle import ipgfcc as O
from synth import make_system, make_workload, random_vectors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_04768_amd import gfcc  # noqa: E402


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_noalloc_greens_small_system():
    s = make_system(6, 21, 30, 4243, sigma_L=0.12, sigma_t1=0.02)
    ctx = gfcc.Context.from_system(s)
    try:
        o = s.n_occ
        for n, q, seed in ((5, [0, 3, o + 2, o + 20], 1), (2, [4, o], 2)):  # second call smaller
            X = random_vectors(n, s.dim, seed=seed)
            Xt = torch.from_numpy(X)
            G0 = ctx.greens(Xt, q).cpu().numpy()
            G1 = ctx.greens(Xt, q, noalloc=True).cpu().numpy()
            C = np.stack([O.left_vector(s, qq) for qq in q])
            assert _rel(G1, G0) < 1e-12
            assert _rel(G1, X @ C.T) < 1e-12
            pd = [(3 * r + 1) % (o + s.n_vir) for r in range(n)]
            D0 = ctx.greens(Xt, p=pd).cpu().numpy()
            D1 = ctx.greens(Xt, p=pd, noalloc=True).cpu().numpy()
            assert _rel(D1, D0) < 1e-12
            want = np.array([O.left_vector(s, pd[r]) @ X[r] for r in range(n)])
            assert _rel(D1[:, 0], want) < 1e-12
    finally:
        ctx.close()


def test_noalloc_greens_benchmark_system():
    """40/200/800 (2.56 MB per plane): many vectors go through the 64 MiB array in chunks;
    a q list whose left rows alone exceed it is refused with E_ARG."""
    wl = make_workload("plain-o40v200")
    s = wl.systems[0]
    ctx = gfcc.Context.from_system(s)
    try:
        gen = torch.Generator(device="cuda").manual_seed(5)
        for n, q in ((12, [0, 7, 39, 40, 100, 239]), (3, [20, 39])):  # second call smaller
            X = torch.randn((n, ctx.dim), dtype=torch.complex128, device="cuda", generator=gen)
            G0 = ctx.greens(X, q).cpu().numpy()
            G1 = ctx.greens(X, q, noalloc=True).cpu().numpy()
            assert _rel(G1, G0) < 1e-12
            pd = list(range(n))
            D0 = ctx.greens(X, p=pd).cpu().numpy()
            D1 = ctx.greens(X, p=pd, noalloc=True).cpu().numpy()
            assert _rel(D1, D0) < 1e-12
        X = torch.randn((1, ctx.dim), dtype=torch.complex128, device="cuda", generator=gen)
        with pytest.raises(gfcc.GfccError, match="fixed scratch"):
            ctx.greens(X, list(range(40)), noalloc=True)  # 40 rows x 2.56 MB > 64 MiB
    finally:
        ctx.close()
