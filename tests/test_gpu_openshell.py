"""GPU parity of the open-shell (spin-unrestricted) IP term against its oracle (oracle.openshell,
pinned to the brute force over both ionised sectors and, for identical spins, to the
spin-adapted closed-shell oracle).

* sigma on antisymmetric spin-orbital vectors elementwise at 1e-12 of its scale (several
  shapes, alpha/beta occupations, Lambda = T^dagger and independent);
* diagonal and one-body blocks at 1e-12;
* G_qp through GMRES at 1e-10 against the oracle for alpha, beta and virtual p and q, with
  the spin selection (alpha-beta elements exactly zero);
* identical spins: the open-shell context's G of an alpha (and a beta) hole equals the
  closed-shell context's G at 1e-10;
* entry points that need the closed-shell operands refuse the context.
"""
import numpy as np
import pytest

from oracle import ipgfcc as IP
from oracle import openshell as OS
from synth import make_open_shell_system, make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_04768_amd import gfcc  # noqa: E402

ETA = 0.01


def _indep_lambda(s, seed):
    rng = np.random.default_rng(seed)
    s.l1a = rng.normal(0, 0.05, s.t1a.shape)
    s.l1b = rng.normal(0, 0.05, s.t1b.shape)

    def anti(x):
        return x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)

    s.l2aa = anti(rng.normal(0, 0.03, s.t2aa.shape))
    s.l2bb = anti(rng.normal(0, 0.03, s.t2bb.shape))
    s.l2ab = rng.normal(0, 0.03, s.t2ab.shape)
    return s


SHAPES = [(4, 2, 1, 5, "t"), (6, 3, 2, 8, "indep"), (12, 6, 4, 20, "t"), (20, 9, 7, 30, "indep")]


@pytest.fixture(scope="module", params=SHAPES, ids=lambda p: f"n{p[0]}a{p[1]}b{p[2]}Q{p[3]}-{p[4]}")
def sysos(request):
    n, oa, ob, Q, lam = request.param
    print(f"\n[uhf] building n={n} oa={oa} ob={ob} Q={Q} lambda={lam}", flush=True)
    s = make_open_shell_system(n, oa, ob, Q, 2010_04768 + 60 + n, sigma_L=0.1, sigma_dL=0.03, sigma_t1=0.03)
    if lam == "indep":
        s = _indep_lambda(s, 4)
    im = OS.intermediates(s)
    ctx = gfcc.Context.open_shell(s, lam=(lam == "indep"))
    yield s, im, ctx
    ctx.close()


def _antisym(rng, k, o, v):
    r1 = rng.normal(size=(k, o)) + 1j * rng.normal(size=(k, o))
    r2 = rng.normal(size=(k, o, o, v)) + 1j * rng.normal(size=(k, o, o, v))
    r2 = r2 - r2.transpose(0, 2, 1, 3)
    return np.concatenate([r1, r2.reshape(k, -1)], axis=1)


def test_dims(sysos):
    s, im, ctx = sysos
    o, v = s.n_occ, s.n_vir
    assert (ctx.n_occ, ctx.n_vir, ctx.dim) == (o, v, o + o * o * v)


def test_sigma_matches_oracle(sysos):
    s, im, ctx = sysos
    o, v = im["o"], im["v"]
    X = _antisym(np.random.default_rng(3), 4, o, v)
    got = ctx.sigma(torch.from_numpy(X)).cpu().numpy()
    want = OS.sigma(im, X)
    scale = np.abs(want).max()
    err = np.abs(got - want).max()
    print(f"[uhf] sigma max err {err:.3e} (scale {scale:.3e})")
    assert err <= 1e-12 * scale
    g2 = got[:, o:].reshape(-1, o, o, v)
    assert np.abs(g2 + g2.transpose(0, 2, 1, 3)).max() <= 1e-12 * scale


def test_diagonal_and_one_body_blocks(sysos):
    s, im, ctx = sysos
    d = ctx.export("DIAG").cpu().numpy()
    dref = OS.diagonal(im)
    assert np.abs(d - dref).max() <= 1e-12 * np.abs(dref).max()
    for name, key in [("FOO", "Foo"), ("FVV", "Fvv"), ("FOV", "Fov")]:
        got = ctx.export(name).cpu().numpy()
        assert np.abs(got - im[key]).max() <= 1e-12 * max(1.0, np.abs(im[key]).max()), name


def test_greens_matches_oracle(sysos):
    s, im, ctx = sysos
    so = im["so"]
    o, v = so["o"], so["v"]
    oa = s.n_occ_a
    ps = [0, oa - 1, oa, o - 1, o, o + v - 1]  # alpha holes, beta holes, virtual alpha and beta
    ws = [-0.45, -0.8, -0.55, -1.0, -0.35, -0.7]
    qs = sorted(set(ps + [1 % o, oa + (1 % max(1, s.n_occ_b))]))
    G, info, _ = ctx.solve(ps, ws, ETA, q=qs, tol=1e-12, restart=40, max_iter=4000)
    G = G.cpu().numpy()
    for r, (p, w) in enumerate(zip(ps, ws)):
        b = OS.rhs(so, p)
        if not np.any(b):
            assert info[r]["status"] == 0 and np.abs(G[r]).max() == 0.0
            continue
        assert info[r]["status"] == 0 and info[r]["true_rel_resid"] <= 1e-12, info[r]
        ref = OS.greens(im, so, p, [w], ETA, qs=qs, tol=1e-13, restart=60)[0]
        assert np.abs(G[r] - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max()), (p, w)
        # spin selection
        sp = 0 if (p < oa or (o <= p < o + s.n_vir_a)) else 1
        for k, q in enumerate(qs):
            sq = 0 if (q < oa or (o <= q < o + s.n_vir_a)) else 1
            if sq != sp:
                assert G[r, k] == 0.0


def test_identical_spins_match_closed_shell_context():
    o, v = 4, 10
    cs = make_system(o, v, 16, 91, sigma_L=0.1, sigma_t1=0.03)
    os_ = OS.from_closed_shell(cs)
    ipc = gfcc.Context.from_system(cs)
    uhf = gfcc.Context.open_shell(os_, lam=False)
    ps = [0, o - 1, 1]
    ws = [-0.5, -0.9, -0.35]
    Gc, _, _ = ipc.solve(ps, ws, ETA, q=[0, 1, o - 1, o + 2], tol=1e-12)
    # alpha copies: same index for holes; virtual q = o + a -> 2o + a; beta copies: o + i
    Ga, _, _ = uhf.solve(ps, ws, ETA, q=[0, 1, o - 1, 2 * o + 2], tol=1e-12)
    Gb, _, _ = uhf.solve([o + p for p in ps], ws, ETA, q=[o, o + 1, 2 * o - 1, 2 * o + v + 2], tol=1e-12)
    Gc, Ga, Gb = (x.cpu().numpy() for x in (Gc, Ga, Gb))
    scale = np.abs(Gc).max()
    assert np.abs(Ga - Gc).max() <= 1e-10 * scale
    assert np.abs(Gb - Gc).max() <= 1e-10 * scale
    ipc.close()
    uhf.close()


def test_multishift_matches_oracle(sysos):
    """Multi-shift GMRES on the open-shell context against the oracle's GMRES at 1e-10."""
    s, im, ctx = sysos
    so = im["so"]
    o = so["o"]
    ps = [0, o - 1, o]
    ws = [-1.0, -0.6, -0.35]
    qs = [0, o - 1, o]
    G, info, _ = ctx.solve_shifts(ps, ws, ETA, q=qs, tol=1e-11, max_dim=400,
                                  fallback=dict(precond="jacobi", precision="fp64", tol=1e-11, restart=60,
                                                max_iter=6000))
    G = G.cpu().numpy()
    for i, p in enumerate(ps):
        if not np.any(OS.rhs(so, p)):
            assert np.abs(G[i]).max() == 0.0
            continue
        ref = OS.greens(im, so, p, ws, ETA, qs=qs, tol=1e-13, restart=60)
        for k in range(len(ws)):
            assert info[i][k]["status"] in (0, 4), info[i][k]
            assert np.abs(G[i, k] - ref[k]).max() <= 1e-10 * max(1.0, np.abs(ref[k]).max()), (p, ws[k])


def test_closed_shell_only_entry_points_refuse(sysos):
    s, im, ctx = sysos
    with pytest.raises(RuntimeError, match="open-shell"):
        ctx.sigma(torch.zeros(1, ctx.dim, dtype=torch.complex128), precision="bf16")
    with pytest.raises(RuntimeError):
        ctx.solve([0], [-0.5], ETA, precond="mlp")
    with pytest.raises(RuntimeError, match="open-shell"):
        ctx.sigma(torch.zeros(1, ctx.dim, dtype=torch.complex128), precision="fp16")
    with pytest.raises(RuntimeError, match="open-shell"):
        ctx.export("WOVVO")
