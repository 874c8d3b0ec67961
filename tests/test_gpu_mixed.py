"""Mixed precision on the three-system workload: (n_occ, n_vir, N_chol) =
(20,100,400), (40,180,720), (60,300,1200), eta = 0.01, omega on [-1.2, -0.3].

For each system a sample of (p, omega) right-hand sides is solved three ways
in the persistent batched solver: FP64 throughout (tol 1e-11, the reference),
FP32 sigma with FP64 refinement and BF16 sigma with FP64 refinement (both to
the workload's tol 1e-8).  The G error of each reduced-precision form against
the FP64 solve is printed per system and must stay within 1e-8 relative; the
FP64 solve of the smallest system is itself checked against the oracle.
"""
import numpy as np
import pytest

from oracle import ipgfcc as O
from synth import make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_04768_amd import gfcc  # noqa: E402


@pytest.fixture(scope="module")
def workload():
    return make_workload("mixed-3sys", n_omega=128)


def _sample(wl, k):
    o = wl.systems[k].n_occ
    ps = np.array([0, o // 2, o - 1], dtype=np.int64)
    ws = wl.omegas[k][::16]
    return np.repeat(ps, len(ws)), np.tile(ws, len(ps))


@pytest.mark.parametrize("k", [0, 1, 2])
def test_mixed_precision_per_system_error(workload, k):
    wl = workload
    s = wl.systems[k]
    P, W = _sample(wl, k)
    ctx = gfcc.Context.from_system(s)
    try:
        Gr, ir, _ = ctx.solve(P, W, wl.eta, tol=1e-11, restart=wl.restart, precision="fp64", max_iter=3000)
        assert all(i["status"] == 0 for i in ir)
        Gr = Gr.cpu().numpy()[:, 0]
        errs = {}
        for form in ("fp32", "bf16", "fp16"):
            G, info, _ = ctx.solve(P, W, wl.eta, tol=wl.tol, restart=wl.restart, precision=form, max_iter=3000)
            assert all(i["status"] == 0 and i["true_rel_resid"] <= wl.tol for i in info), form
            G = G.cpu().numpy()[:, 0]
            errs[form] = float(np.max(np.abs(G - Gr) / np.abs(Gr)))
            its = np.mean([i["iters"] for i in info])
            print(f"system o={s.n_occ} v={s.n_vir}: {form}-IR max G rel err vs FP64 {errs[form]:.2e}, "
                  f"mean iters {its:.1f}, FP64 iters {np.mean([i['iters'] for i in ir]):.1f}")
            assert errs[form] <= 1e-8, (form, errs[form])
        if k == 0:
            im = O.intermediates(s)
            for r in (0, len(P) - 1):
                x, _, _ = O.solve(s, im, int(P[r]), float(W[r]), wl.eta, tol=1e-12, restart=60, max_iter=600)
                g = O.left_vector(s, int(P[r])) @ x
                assert abs(Gr[r] - g) <= 1e-10 * abs(g)
    finally:
        ctx.close()


def test_oracle_true_residual_of_fp64_solutions(workload):
    """The 40/180/720 system: the oracle's own true residual ||b - (omega - i eta + Hbar) x|| / ||b||
    of GPU FP64 solutions (tol 1e-11) at two (p, omega), evaluated with the oracle's sigma."""
    wl = workload
    s = wl.systems[1]
    ctx = gfcc.Context.from_system(s)
    try:
        P = np.array([0, s.n_occ - 1], dtype=np.int64)
        W = np.array([wl.omegas[1][5], wl.omegas[1][100]])
        G, info, X = ctx.solve(P, W, wl.eta, tol=1e-11, restart=wl.restart, precision="fp64", max_iter=3000,
                               want_x=True)
        X = X.cpu().numpy()
        print("[mixed] oracle intermediates of the 40/180/720 system", flush=True)
        im = O.intermediates(s)
        Y = O.sigma(im, X)
        for r in range(2):
            b = O.rhs(s, int(P[r]))
            res = b - ((W[r] - 1j * wl.eta) * X[r] + Y[r])
            rel = np.linalg.norm(res) / np.linalg.norm(b)
            print(f"[mixed] p={P[r]} omega={W[r]:.4f}: oracle true residual {rel:.2e}, "
                  f"library {info[r]['true_rel_resid']:.2e}")
            assert rel <= 2e-11
            g = O.left_vector(s, int(P[r])) @ X[r]
            assert abs(G.cpu().numpy()[r, 0] - g) <= 1e-12 * abs(g)
    finally:
        ctx.close()
