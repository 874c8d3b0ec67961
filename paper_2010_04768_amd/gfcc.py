"""ctypes binding of libgfcc.so (argument marshalling only).

Every computation runs in the library's HIP kernels; PyTorch supplies device
memory (complex128 tensors are interleaved (re, im) FP64, the layout the C ABI
expects) and the current HIP stream.  Importing this module does not touch
the GPU; the library is loaded on first use and a missing build raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfcc.so")

FP64, FP32_IR, BF16_IR, FP16_IR = 0, 1, 2, 3
PC_NONE, PC_JACOBI, PC_MLP = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32_IR, "bf16": BF16_IR, "fp16": FP16_IR}
PRECONDS = {"none": PC_NONE, "jacobi": PC_JACOBI, "mlp": PC_MLP}
BLOCKS = ["FOO", "FVV", "FOV", "WOOOO", "WOOOV", "WOVOO", "WOVVO", "WOVOV", "DIAG", "LEFT"]

# exported symbols of include/gfcc.h
SYMBOLS = ["gfcc_build_intermediates", "gfcc_dims", "gfcc_export", "gfcc_sigma", "gfcc_solve_batch",
           "gfcc_greens", "gfcc_prof_enable", "gfcc_prof_get", "gfcc_destroy", "gfcc_strerror",
           "gfcc_last_error", "gfcc_mlp_train", "gfcc_mlp_set_weights", "gfcc_mlp_get_weights",
           "gfcc_mlp_forward", "gfcc_mlp_loss_grad", "gfcc_mlp_features", "gfcc_mlp_apply",
           "gfcc_mor_reset", "gfcc_mor_extend", "gfcc_mor_model", "gfcc_mor_export", "gfcc_mor_greens",
           "gfcc_solve_shifts", "gfcc_spectral", "gfcc_solve_multi", "gfcc_mlp_adam_step",
           "gfcc_greens_noalloc", "gfcc_plan_memory", "gfcc_build_ea_intermediates",
           "gfcc_build_uhf_intermediates"]


class GfccSystem(ctypes.Structure):
    _fields_ = [("n_occ", ctypes.c_int64), ("n_vir", ctypes.c_int64), ("n_chol", ctypes.c_int64),
                ("eps", ctypes.c_void_p), ("L", ctypes.c_void_p), ("t1", ctypes.c_void_p),
                ("t2", ctypes.c_void_p), ("l1", ctypes.c_void_p), ("l2", ctypes.c_void_p)]


class UhfSystem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_occ_a", ctypes.c_int64), ("n_occ_b", ctypes.c_int64),
                ("n_chol", ctypes.c_int64)] + [(nm, ctypes.c_void_p) for nm in
                                               ("eps_a", "eps_b", "La", "Lb", "t1a", "t1b", "t2aa", "t2ab", "t2bb",
                                                "l1a", "l1b", "l2aa", "l2ab", "l2bb")]


class SolveOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("tol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("batch", ctypes.c_int32), ("precond", ctypes.c_int),
                ("precision", ctypes.c_int), ("use_graph", ctypes.c_int32), ("tune_cache", ctypes.c_char_p),
                ("ir_inner_rtol", ctypes.c_double), ("checkpoint", ctypes.c_char_p),
                ("sync_every", ctypes.c_int32)]


class RhsInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("true_rel_resid", ctypes.c_double)]


class ShiftOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("tol", ctypes.c_double), ("max_dim", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("verify", ctypes.c_int32), ("use_fallback", ctypes.c_int32),
                ("fallback", SolveOpts), ("tune_cache", ctypes.c_char_p)]


class MlpOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("width", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("pair_restart", ctypes.c_int32), ("lr", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("max_pairs", ctypes.c_int32), ("data_max_iter", ctypes.c_int32),
                ("data_tol", ctypes.c_double), ("data_precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("xstar_ratio", ctypes.c_double)]


class MlpReport(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("steps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("loss_first", ctypes.c_double), ("loss_final", ctypes.c_double),
                ("data_seconds", ctypes.c_double), ("train_seconds", ctypes.c_double)]


class MorOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("tol", ctypes.c_double), ("drop_tol", ctypes.c_double),
                ("max_levels", ctypes.c_int32), ("reserved", ctypes.c_int32), ("solve", SolveOpts)]


class MorReport(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("m", ctypes.c_int32), ("n_solved", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("per_level", ctypes.c_int32 * 16),
                ("max_mid_err", ctypes.c_double), ("t_solve", ctypes.c_double), ("t_basis", ctypes.c_double),
                ("t_project", ctypes.c_double), ("t_model", ctypes.c_double)]


class MemoryPlan(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t)] + [(n, ctypes.c_double) for n in (
        "input_L", "input_t2", "input_l2", "ring", "ladder", "wovoo", "wooov", "cholesky", "rows_1h", "left",
        "vectors", "small", "context_fp64", "context_lowp", "build_fixed", "build_chunk_min", "per_slot",
        "sigma_workspace", "total", "build_peak")]


class GfccError(RuntimeError):
    pass


_lib = None


def load():
    """Load libgfcc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GfccError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    L.gfcc_build_intermediates.argtypes = [ctypes.POINTER(GfccSystem), vp, ctypes.POINTER(vp)]
    L.gfcc_build_ea_intermediates.argtypes = [ctypes.POINTER(GfccSystem), vp, ctypes.POINTER(vp)]
    L.gfcc_build_ea_intermediates.restype = ctypes.c_int
    L.gfcc_build_uhf_intermediates.argtypes = [ctypes.POINTER(UhfSystem), vp, ctypes.POINTER(vp)]
    L.gfcc_build_uhf_intermediates.restype = ctypes.c_int
    L.gfcc_dims.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.gfcc_export.argtypes = [vp, ctypes.c_int, vp, vp]
    L.gfcc_sigma.argtypes = [vp, i64, vp, vp, ctypes.c_int, vp]
    L.gfcc_solve_batch.argtypes = [vp, i64, vp, vp, dbl, i64, vp, ctypes.POINTER(SolveOpts), vp, vp,
                                   ctypes.POINTER(RhsInfo), vp]
    L.gfcc_greens.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp]
    L.gfcc_greens_noalloc.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp]
    L.gfcc_greens_noalloc.restype = ctypes.c_int
    L.gfcc_plan_memory.argtypes = [i64, i64, i64, ctypes.c_int, ctypes.c_int32, ctypes.c_int32, i64, ctypes.c_int32,
                                   ctypes.POINTER(MemoryPlan)]
    L.gfcc_plan_memory.restype = ctypes.c_int
    L.gfcc_prof_enable.argtypes = [vp, ctypes.c_int]
    L.gfcc_prof_get.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.gfcc_destroy.argtypes = [vp]
    L.gfcc_strerror.restype = ctypes.c_char_p
    L.gfcc_strerror.argtypes = [ctypes.c_int]
    L.gfcc_last_error.restype = ctypes.c_char_p
    for name in ["gfcc_build_intermediates", "gfcc_dims", "gfcc_export", "gfcc_sigma", "gfcc_solve_batch",
                 "gfcc_greens", "gfcc_prof_enable", "gfcc_prof_get", "gfcc_destroy"]:
        getattr(L, name).restype = ctypes.c_int
    L.gfcc_mlp_train.argtypes = [vp, i64, vp, vp, dbl, ctypes.POINTER(MlpOpts), ctypes.POINTER(MlpReport), vp]
    L.gfcc_mlp_set_weights.argtypes = [vp, ctypes.c_int32, vp, vp]
    L.gfcc_mlp_get_weights.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp, vp]
    L.gfcc_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
    L.gfcc_mlp_adam_step.argtypes = [vp, vp, dbl, vp]
    L.gfcc_mlp_loss_grad.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.gfcc_mlp_features.argtypes = [vp, i64, vp, vp, dbl, vp, vp]
    L.gfcc_mlp_apply.argtypes = [vp, i64, vp, vp, dbl, vp, vp]
    for name in ["gfcc_mlp_train", "gfcc_mlp_set_weights", "gfcc_mlp_get_weights", "gfcc_mlp_forward", "gfcc_mlp_adam_step",
                 "gfcc_mlp_loss_grad", "gfcc_mlp_features", "gfcc_mlp_apply"]:
        getattr(L, name).restype = ctypes.c_int
    L.gfcc_solve_shifts.argtypes = [vp, i64, vp, i64, vp, dbl, i64, vp, ctypes.POINTER(ShiftOpts), vp, vp,
                                    ctypes.POINTER(RhsInfo), vp]
    L.gfcc_solve_shifts.restype = ctypes.c_int
    L.gfcc_solve_multi.argtypes = [ctypes.c_int32, vp, i64, vp, vp, vp, dbl, i64, vp, ctypes.POINTER(SolveOpts),
                                   vp, ctypes.POINTER(RhsInfo), vp]
    L.gfcc_solve_multi.restype = ctypes.c_int
    L.gfcc_spectral.argtypes = [i64, i64, vp, i64, dbl, vp, vp]
    L.gfcc_spectral.restype = ctypes.c_int
    L.gfcc_mor_reset.argtypes = [vp]
    L.gfcc_mor_extend.argtypes = [vp, i64, vp, dbl, ctypes.POINTER(i64), vp]
    L.gfcc_mor_model.argtypes = [vp, i64, vp, i64, vp, i64, vp, dbl, vp, vp]
    L.gfcc_mor_export.argtypes = [vp, ctypes.c_int32, vp, ctypes.POINTER(i64), vp]
    L.gfcc_mor_greens.argtypes = [vp, i64, vp, i64, vp, dbl, ctypes.POINTER(MorOpts), vp, vp,
                                  ctypes.POINTER(MorReport), vp]
    for name in ["gfcc_mor_reset", "gfcc_mor_extend", "gfcc_mor_model", "gfcc_mor_export", "gfcc_mor_greens"]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st, what):
    if st < 0:
        L = load()
        raise GfccError(f"{what}: {L.gfcc_strerror(st).decode()}: {L.gfcc_last_error().decode()}")
    return st


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def plan_memory(n_occ, n_vir, n_chol, precision="bf16", restart=30, flexible=False, window=0, lambda_given=False):
    """Device-memory plan (bytes per operand) of one system; host arithmetic only, no GPU needed."""
    p = MemoryPlan()
    p.struct_size = ctypes.sizeof(MemoryPlan)
    _check(load().gfcc_plan_memory(n_occ, n_vir, n_chol, PRECISIONS[precision], restart, int(flexible), window,
                                   int(lambda_given), ctypes.byref(p)), "gfcc_plan_memory")
    return {n: getattr(p, n) for n, _ in MemoryPlan._fields_[1:]}


def spectral(G, eta):
    """A[k] = sgn(eta)/pi * sum_p Im G[p, k] on the GPU; G: [np, n_omega] (or [np, n_omega, 1]) complex
    device tensor of diagonal elements G_pp(omega_k).  Returns a float64 device tensor [n_omega]."""
    import torch
    G = G.reshape(G.shape[0], -1).to(dtype=torch.complex128).contiguous()
    A = torch.empty(G.shape[1], dtype=torch.float64, device=G.device)
    _check(load().gfcc_spectral(G.shape[0], G.shape[1], _ptr(G), G.shape[1], float(eta), _ptr(A), _stream()),
           "gfcc_spectral")
    return A


def solve_multi(ctxs, sys, p, omega, eta, q=None, tol=1e-8, restart=30, max_iter=2000, batch=0,
                precond="jacobi", precision="fp64", use_graph=False, ir_inner_rtol=0.0, tune_cache=None,
                checkpoint=None, sync_every=0):
    """Right-hand sides of several systems (contexts) in one persistent solve: right-hand side r
    belongs to ctxs[sys[r]].  Returns (G [nrhs, nq] complex128 device tensor, info list).
    `checkpoint`: resume file (finished rows are appended; rows it already holds are restored).
    `sync_every`: as in Context.solve."""
    import torch
    s_h = np.ascontiguousarray(np.asarray(sys, dtype=np.int32))
    p_h = np.ascontiguousarray(np.asarray(p, dtype=np.int64))
    w_h = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
    assert s_h.shape == p_h.shape == w_h.shape
    n = p_h.size
    if q is None:
        q_h, nq = None, 1
    else:
        q_h = np.ascontiguousarray(np.asarray(q, dtype=np.int64))
        nq = q_h.size
    G = torch.zeros((n, nq), dtype=torch.complex128, device=ctxs[0].device)
    info = (RhsInfo * max(n, 1))()
    handles = (ctypes.c_void_p * len(ctxs))(*[c._h.value for c in ctxs])
    opts = SolveOpts(ctypes.sizeof(SolveOpts), tol, restart, max_iter, batch, PRECONDS[precond],
                     PRECISIONS[precision], int(use_graph), tune_cache.encode() if tune_cache else None,
                     ir_inner_rtol, checkpoint.encode() if checkpoint else None, sync_every)
    st = load().gfcc_solve_multi(len(ctxs), handles, n, s_h.ctypes.data_as(ctypes.c_void_p),
                                 p_h.ctypes.data_as(ctypes.c_void_p), w_h.ctypes.data_as(ctypes.c_void_p), eta, nq,
                                 q_h.ctypes.data_as(ctypes.c_void_p) if q_h is not None else None,
                                 ctypes.byref(opts), _ptr(G), info, _stream())
    _check(st, "gfcc_solve_multi")
    infos = [dict(status=info[r].status, iters=info[r].iters, restarts=info[r].restarts,
                  true_rel_resid=info[r].true_rel_resid) for r in range(n)]
    return G, infos


class Context:
    """Owns one gfcc_ctx (per-system intermediates on the current device).

    ``sector="ip"`` builds the ionisation (retarded) term on 1h + 2h1p; ``sector="ea"`` the
    electron-attached (advanced) term on 1p + 2p1h, whose ``solve`` returns
    G[r][k] = G^EA_{q[k] p[r]} (see gfcc_build_ea_intermediates)."""

    def __init__(self, eps, L, t1, t2, l1=None, l2=None, sector="ip"):
        import torch
        self._lib = load()
        dev = torch.device("cuda", torch.cuda.current_device())

        def dev_f64(a):
            if a is None:
                return None
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            return t.to(device=dev, dtype=torch.float64).contiguous()

        self._keep = [dev_f64(x) for x in (eps, L, t1, t2, l1, l2)]
        e, Lc, a1, a2, b1, b2 = self._keep
        self.n_occ, self.n_vir = a1.shape
        sysd = GfccSystem(self.n_occ, self.n_vir, Lc.shape[0], e.data_ptr(), Lc.data_ptr(), a1.data_ptr(),
                          a2.data_ptr(), b1.data_ptr() if b1 is not None else None,
                          b2.data_ptr() if b2 is not None else None)
        h = ctypes.c_void_p()
        if sector not in ("ip", "ea"):
            raise ValueError("sector must be 'ip' or 'ea'")
        self.sector = sector
        build = "gfcc_build_intermediates" if sector == "ip" else "gfcc_build_ea_intermediates"
        _check(getattr(self._lib, build)(ctypes.byref(sysd), _stream(), ctypes.byref(h)), build)
        self._h = h
        # the context borrows t2 (and l2) until it is destroyed; eps, L, t1, l1 were read by the build
        self._keep = [a2, b2]
        D = ctypes.c_int64()
        _check(self._lib.gfcc_dims(self._h, ctypes.byref(D), None, None), "gfcc_dims")
        self.dim = D.value
        self.device = dev

    @classmethod
    def from_system(cls, s, sector="ip"):
        return cls(s.eps, s.L, s.t1, s.t2, s.l1, s.l2, sector=sector)

    @classmethod
    def open_shell(cls, s, lam=True):
        """IP context of an open-shell system (synth.OpenShellSystem layout, spin blocks); lam=False
        takes Lambda = T^dagger.  Orbital indices run over spin orbitals, occupied [alpha, beta]
        then virtual [alpha, beta]."""
        import torch
        self = cls.__new__(cls)
        self._lib = load()
        dev = torch.device("cuda", torch.cuda.current_device())

        def d(a):
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            return t.to(device=dev, dtype=torch.float64).contiguous()

        names = ["eps_a", "eps_b", "La", "Lb", "t1a", "t1b", "t2aa", "t2ab", "t2bb"]
        if lam:
            names += ["l1a", "l1b", "l2aa", "l2ab", "l2bb"]
        keep = {nm: d(getattr(s, nm)) for nm in names}
        sysd = UhfSystem(s.n, s.n_occ_a, s.n_occ_b, s.n_chol,
                         *[keep[nm].data_ptr() if nm in keep else None for nm in
                           ("eps_a", "eps_b", "La", "Lb", "t1a", "t1b", "t2aa", "t2ab", "t2bb",
                            "l1a", "l1b", "l2aa", "l2ab", "l2bb")])
        h = ctypes.c_void_p()
        _check(self._lib.gfcc_build_uhf_intermediates(ctypes.byref(sysd), _stream(), ctypes.byref(h)),
               "gfcc_build_uhf_intermediates")
        self._h = h
        self._keep = None  # the build read every input
        self.sector = "uhf"
        D, no, nv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.gfcc_dims(self._h, ctypes.byref(D), ctypes.byref(no), ctypes.byref(nv)), "gfcc_dims")
        self.dim, self.n_occ, self.n_vir = D.value, no.value, nv.value
        self.device = dev
        return self

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.gfcc_destroy(self._h)
            self._h = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- blocks
    def export(self, name):
        import torch
        o, v, D = self.n_occ, self.n_vir, self.dim
        shapes = {"FOO": (o, o), "FVV": (v, v), "FOV": (o, v), "WOOOO": (o, o, o, o), "WOOOV": (o, o, o, v),
                  "WOVOO": (o, v, o, o), "WOVVO": (o, v, v, o), "WOVOV": (o, v, o, v), "DIAG": (D,),
                  "LEFT": (o, D)}
        out = torch.empty(shapes[name], dtype=torch.float64, device=self.device)
        _check(self._lib.gfcc_export(self._h, BLOCKS.index(name), _ptr(out), _stream()), "gfcc_export")
        return out

    # ---------------------------------------------------------------- sigma
    def sigma(self, X, precision="fp64"):
        import torch
        X = X.to(device=self.device, dtype=torch.complex128).contiguous()
        squeeze = X.dim() == 1
        if squeeze:
            X = X[None]
        assert X.shape[-1] == self.dim
        Y = torch.empty_like(X)
        _check(self._lib.gfcc_sigma(self._h, X.shape[0], _ptr(X), _ptr(Y), PRECISIONS[precision], _stream()),
               "gfcc_sigma")
        return Y[0] if squeeze else Y

    # ---------------------------------------------------------------- solve
    def solve(self, p: Sequence[int], omega: Sequence[float], eta: float, q: Optional[Sequence[int]] = None,
              tol=1e-8, restart=30, max_iter=2000, batch=0, precond="jacobi", precision="fp64",
              use_graph=False, want_x=False, ir_inner_rtol=0.0, tune_cache=None, checkpoint=None, x_out=None,
              sync_every=0):
        """Returns (G [nrhs, nq] complex128 device tensor, info list of dicts, X or None).
        `x_out`: caller buffer [nrhs, D] complex128 for X (with want_x; default: a new zero tensor).
        `sync_every`: inner iterations between host synchronisations (0: sized from the predicted
        end of the next cycle; 1: after every iteration)."""
        import torch
        p_h = np.ascontiguousarray(np.asarray(p, dtype=np.int64))
        w_h = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        assert p_h.shape == w_h.shape
        n = p_h.size
        if q is None:
            q_h, nq = None, 1
        else:
            q_h = np.ascontiguousarray(np.asarray(q, dtype=np.int64))
            nq = q_h.size
        G = torch.zeros((n, nq), dtype=torch.complex128, device=self.device)
        X = None
        if want_x:
            X = x_out if x_out is not None else torch.zeros((n, self.dim), dtype=torch.complex128, device=self.device)
            assert X.shape == (n, self.dim) and X.dtype == torch.complex128 and X.is_contiguous()
        info = (RhsInfo * max(n, 1))()
        opts = SolveOpts(ctypes.sizeof(SolveOpts), tol, restart, max_iter, batch, PRECONDS[precond],
                         PRECISIONS[precision], int(use_graph),
                         tune_cache.encode() if tune_cache else None, ir_inner_rtol,
                         checkpoint.encode() if checkpoint else None, sync_every)
        st = self._lib.gfcc_solve_batch(
            self._h, n, p_h.ctypes.data_as(ctypes.c_void_p), w_h.ctypes.data_as(ctypes.c_void_p), eta, nq,
            q_h.ctypes.data_as(ctypes.c_void_p) if q_h is not None else None, ctypes.byref(opts), _ptr(G),
            _ptr(X), info, _stream())
        _check(st, "gfcc_solve_batch")
        infos = [dict(status=info[r].status, iters=info[r].iters, restarts=info[r].restarts,
                      true_rel_resid=info[r].true_rel_resid) for r in range(n)]
        return G, infos, X

    def solve_shifts(self, p: Sequence[int], omega: Sequence[float], eta: float,
                     q: Optional[Sequence[int]] = None, tol=1e-8, max_dim=160, batch=0, verify=True,
                     want_x=False, fallback: Optional[dict] = None, tune_cache=None):
        """Multi-shift GMRES: one Krylov basis per orbital for all frequencies.

        Returns (G [np, n_omega, nq] complex128 device tensor, info [np][n_omega] dicts, X
        [np, n_omega, D] or None).  `fallback`: keyword arguments of `solve` (tol, restart,
        max_iter, batch, precond, precision, use_graph, ir_inner_rtol) for the (p, omega) that
        do not converge within max_dim basis vectors; None leaves them with status 1."""
        import torch
        p_h = np.ascontiguousarray(np.asarray(p, dtype=np.int64))
        w_h = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        npp, nw = p_h.size, w_h.size
        if q is None:
            q_h, nq = None, 1
        else:
            q_h = np.ascontiguousarray(np.asarray(q, dtype=np.int64))
            nq = q_h.size
        G = torch.zeros((npp, nw, nq), dtype=torch.complex128, device=self.device)
        X = torch.zeros((npp, nw, self.dim), dtype=torch.complex128, device=self.device) if want_x else None
        info = (RhsInfo * max(npp * nw, 1))()
        f = dict(tol=tol, restart=30, max_iter=2000, batch=0, precond="jacobi", precision="fp64",
                 use_graph=False, ir_inner_rtol=0.0)
        if fallback:
            f.update(fallback)
        fo = SolveOpts(ctypes.sizeof(SolveOpts), f["tol"], f["restart"], f["max_iter"], f["batch"],
                       PRECONDS[f["precond"]], PRECISIONS[f["precision"]], int(f["use_graph"]), None,
                       f["ir_inner_rtol"])
        opts = ShiftOpts(ctypes.sizeof(ShiftOpts), tol, max_dim, batch, int(verify), int(fallback is not None), fo,
                         tune_cache.encode() if tune_cache else None)
        st = self._lib.gfcc_solve_shifts(
            self._h, npp, p_h.ctypes.data_as(ctypes.c_void_p), nw, w_h.ctypes.data_as(ctypes.c_void_p), eta, nq,
            q_h.ctypes.data_as(ctypes.c_void_p) if q_h is not None else None, ctypes.byref(opts), _ptr(G), _ptr(X),
            info, _stream())
        _check(st, "gfcc_solve_shifts")
        infos = [[dict(status=info[i * nw + k].status, iters=info[i * nw + k].iters,
                       restarts=info[i * nw + k].restarts, true_rel_resid=info[i * nw + k].true_rel_resid)
                  for k in range(nw)] for i in range(npp)]
        return G, infos, X

    def greens(self, X, q=None, p=None, noalloc=False):
        """G [nrhs, nq] = c_q^T X for a list q, or with q None the diagonal form G[r, 0] = c_{p[r]}^T X[r].
        noalloc=True calls the allocation-free entry point (fixed device scratch)."""
        import torch
        X = X.to(device=self.device, dtype=torch.complex128).contiguous()
        if q is None:
            p_h = np.ascontiguousarray(np.asarray(p, dtype=np.int64))
            q_h, nq = None, 1
        else:
            p_h = None
            q_h = np.ascontiguousarray(np.asarray(q, dtype=np.int64))
            nq = q_h.size
        G = torch.empty((X.shape[0], nq), dtype=torch.complex128, device=self.device)
        fn, name = ((self._lib.gfcc_greens_noalloc, "gfcc_greens_noalloc") if noalloc
                    else (self._lib.gfcc_greens, "gfcc_greens"))
        _check(fn(self._h, X.shape[0], p_h.ctypes.data_as(ctypes.c_void_p) if p_h is not None else None, _ptr(X),
                  nq, q_h.ctypes.data_as(ctypes.c_void_p) if q_h is not None else None, _ptr(G), _stream()), name)
        return G

    # ---------------------------------------------------------------- timing
    def prof_enable(self, on=True):
        _check(self._lib.gfcc_prof_enable(self._h, int(on)), "gfcc_prof_enable")

    def prof_get(self, name):
        c, ms, fl, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self._lib.gfcc_prof_get(self._h, name.encode(), ctypes.byref(c), ctypes.byref(ms), ctypes.byref(fl),
                                       ctypes.byref(by)), "gfcc_prof_get")
        return dict(count=c.value, ms=ms.value, flops=fl.value, bytes=by.value)

    # ---------------------------------------------------------------- learned preconditioner
    def mlp_train(self, p, omega, eta, width=256, steps=1000, batch=8192, pair_restart=4, lr=1e-3, seed=0,
                  max_pairs=512, data_tol=0.0, data_max_iter=0, data_precision="fp64", xstar_ratio=0.0):
        p_h = np.ascontiguousarray(np.asarray(p, dtype=np.int64))
        w_h = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        o = MlpOpts(ctypes.sizeof(MlpOpts), width, steps, batch, pair_restart, lr, seed, max_pairs, data_max_iter,
                    data_tol, PRECISIONS[data_precision], 0, xstar_ratio)
        rep = MlpReport()
        _check(self._lib.gfcc_mlp_train(self._h, p_h.size, p_h.ctypes.data_as(ctypes.c_void_p),
                                        w_h.ctypes.data_as(ctypes.c_void_p), eta, ctypes.byref(o),
                                        ctypes.byref(rep), _stream()), "gfcc_mlp_train")
        return dict(n_pairs=rep.n_pairs, steps=rep.steps, loss_first=rep.loss_first, loss_final=rep.loss_final,
                    data_seconds=rep.data_seconds, train_seconds=rep.train_seconds)

    def mlp_set_weights(self, width, params):
        import torch
        t = torch.as_tensor(np.asarray(params, dtype=np.float64)).to(self.device).contiguous()
        _check(self._lib.gfcc_mlp_set_weights(self._h, width, _ptr(t), _stream()), "gfcc_mlp_set_weights")

    def mlp_get_weights(self):
        import torch
        w = ctypes.c_int32()
        _check(self._lib.gfcc_mlp_get_weights(self._h, ctypes.byref(w), None, _stream()), "gfcc_mlp_get_weights")
        W = w.value
        n = W * 8 + W + W * W + W + 2 * W + 2
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        _check(self._lib.gfcc_mlp_get_weights(self._h, ctypes.byref(w), _ptr(out), _stream()), "gfcc_mlp_get_weights")
        return W, out

    def mlp_adam_step(self, grad, lr):
        """One Adam step on the network weights with the flat gradient `grad` (device or host)."""
        import torch
        g = torch.as_tensor(np.asarray(grad, dtype=np.float64) if not isinstance(grad, torch.Tensor) else grad)
        g = g.to(self.device, torch.float64).contiguous()
        _check(self._lib.gfcc_mlp_adam_step(self._h, _ptr(g), float(lr), _stream()), "gfcc_mlp_adam_step")

    def mlp_forward(self, X):
        import torch
        X = torch.as_tensor(X).to(self.device, torch.float64).contiguous()
        Y = torch.empty((X.shape[0], 2), dtype=torch.float64, device=self.device)
        _check(self._lib.gfcc_mlp_forward(self._h, X.shape[0], _ptr(X), _ptr(Y), _stream()), "gfcc_mlp_forward")
        return Y

    def mlp_loss_grad(self, X, T):
        import torch
        X = torch.as_tensor(X).to(self.device, torch.float64).contiguous()
        T = torch.as_tensor(T).to(self.device, torch.float64).contiguous()
        W, _ = self.mlp_get_weights()
        n = W * 8 + W + W * W + W + 2 * W + 2
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        grad = torch.empty(n, dtype=torch.float64, device=self.device)
        _check(self._lib.gfcc_mlp_loss_grad(self._h, X.shape[0], _ptr(X), _ptr(T), _ptr(loss), _ptr(grad),
                                            _stream()), "gfcc_mlp_loss_grad")
        return loss, grad

    def mlp_features(self, R, omega, eta):
        import torch
        R = torch.as_tensor(R).to(self.device, torch.complex128).contiguous()
        w_h = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        X = torch.empty((R.shape[0] * self.dim, 8), dtype=torch.float64, device=self.device)
        _check(self._lib.gfcc_mlp_features(self._h, R.shape[0], _ptr(R), w_h.ctypes.data_as(ctypes.c_void_p), eta,
                                           _ptr(X), _stream()), "gfcc_mlp_features")
        return X

    def mlp_apply(self, R, omega, eta):
        import torch
        R = torch.as_tensor(R).to(self.device, torch.complex128).contiguous()
        w_h = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        U = torch.empty_like(R)
        _check(self._lib.gfcc_mlp_apply(self._h, R.shape[0], _ptr(R), w_h.ctypes.data_as(ctypes.c_void_p), eta,
                                        _ptr(U), _stream()), "gfcc_mlp_apply")
        return U

    # ---------------------------------------------------------------- model-order reduction
    def mor_reset(self):
        _check(self._lib.gfcc_mor_reset(self._h), "gfcc_mor_reset")

    def mor_extend(self, X, drop_tol=1e-10):
        """Gram-Schmidt Re/Im of complex vectors X [n, D] into the basis; returns the basis size."""
        import torch
        X = torch.as_tensor(X).to(self.device, torch.complex128).contiguous()
        m = ctypes.c_int64()
        _check(self._lib.gfcc_mor_extend(self._h, X.shape[0], _ptr(X), drop_tol, ctypes.byref(m), _stream()),
               "gfcc_mor_extend")
        return m.value

    def mor_model(self, p, omega, eta, q=None):
        """Model G: [n_omega, np] (q None: diagonal) or [n_omega, np, nq] complex128 device tensor."""
        import torch
        p_h = np.ascontiguousarray(np.asarray(p, dtype=np.int64))
        w_h = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        if q is None:
            q_h, nq, shape = None, p_h.size, (w_h.size, p_h.size)
        else:
            q_h = np.ascontiguousarray(np.asarray(q, dtype=np.int64))
            nq, shape = q_h.size, (w_h.size, p_h.size, q_h.size)
        G = torch.empty(shape, dtype=torch.complex128, device=self.device)
        _check(self._lib.gfcc_mor_model(self._h, p_h.size, p_h.ctypes.data_as(ctypes.c_void_p), nq,
                                        q_h.ctypes.data_as(ctypes.c_void_p) if q_h is not None else None, w_h.size,
                                        w_h.ctypes.data_as(ctypes.c_void_p), eta, _ptr(G), _stream()),
               "gfcc_mor_model")
        return G

    def mor_export(self, which="HHAT"):
        import torch
        wi = {"HHAT": 0, "BASIS": 1}[which]
        m = ctypes.c_int64()
        _check(self._lib.gfcc_mor_export(self._h, wi, None, ctypes.byref(m), _stream()), "gfcc_mor_export")
        shape = (m.value, m.value) if wi == 0 else (m.value, self.dim)
        out = torch.empty(shape, dtype=torch.float64, device=self.device)
        if m.value > 0:
            _check(self._lib.gfcc_mor_export(self._h, wi, _ptr(out), ctypes.byref(m), _stream()), "gfcc_mor_export")
        return out

    def mor_greens(self, p, omega, eta, tol=1e-8, drop_tol=1e-10, max_levels=0, solve_tol=1e-10, restart=30,
                   max_iter=3000, batch=0, precond="jacobi", precision="fp64", use_graph=False, tune_cache=None,
                   ir_inner_rtol=0.0):
        """Level loop on the uniform grid omega; returns (G [n_omega, np] device, report dict, level_of)."""
        import torch
        p_h = np.ascontiguousarray(np.asarray(p, dtype=np.int64))
        w_h = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        so = SolveOpts(ctypes.sizeof(SolveOpts), solve_tol, restart, max_iter, batch, PRECONDS[precond],
                       PRECISIONS[precision], int(use_graph), tune_cache.encode() if tune_cache else None,
                       ir_inner_rtol)
        o = MorOpts(ctypes.sizeof(MorOpts), tol, drop_tol, max_levels, 0, so)
        rep = MorReport()
        lev = np.zeros(w_h.size, dtype=np.int32)
        G = torch.zeros((w_h.size, p_h.size), dtype=torch.complex128, device=self.device)
        st = self._lib.gfcc_mor_greens(self._h, p_h.size, p_h.ctypes.data_as(ctypes.c_void_p), w_h.size,
                                       w_h.ctypes.data_as(ctypes.c_void_p), eta, ctypes.byref(o), _ptr(G),
                                       lev.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rep), _stream())
        _check(st, "gfcc_mor_greens")
        report = dict(levels=rep.levels, m=rep.m, n_solved=rep.n_solved, converged=bool(rep.converged),
                      per_level=[rep.per_level[i] for i in range(min(rep.levels, 16))],
                      max_mid_err=rep.max_mid_err, t_solve=rep.t_solve, t_basis=rep.t_basis,
                      t_project=rep.t_project, t_model=rep.t_model, all_solves_converged=(st == 0))
        return G, report, lev
