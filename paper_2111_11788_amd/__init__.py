"""Python binding of the MI355X MLMC finite-element library (libmlmc.so).

Argument marshalling only: every step of the hot path runs in the HIP kernels
behind the C-ABI declared in include/mlmc.h.  PyTorch supplies the device
memory (one arena tensor per context, plus the input/output tensors of the
step-level calls) and the stream.  There is no CPU fallback: if the shared
library is missing the first use raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlmc.so")

MLMC_OK, MLMC_PENDING = 0, 1
ERRORS = {-1: "MLMC_E_INVALID", -2: "MLMC_E_NOMEM", -3: "MLMC_E_BUDGET", -4: "MLMC_E_NOCONV",
          -5: "MLMC_E_NONFINITE", -6: "MLMC_E_DEVICE"}
KERNELS = ["XI", "FIELD", "APPLY", "CHEB_ZERO", "CHEB", "CHEB_XO", "RESIDUAL", "RESTRICT", "PROLONG",
           "COARSEST", "COARSEN", "PCG_APPLY", "PCG_UPDATE", "PCG_DOT", "PCG_DIRECTION", "TRUE_RESIDUAL",
           "REDUCE", "QOI", "MISC", "CHEB_PROLONG", "PCG_UPDATE_ZERO",
           "RESIDUAL_RESTRICT", "SOLVE_SMALL"]
# MLMC_FUSE_* bits of the tuning's `fuse` field
FUSE_PROLONG, FUSE_UPDATE, FUSE_REFINE, FUSE_RESTRICT = 1, 2, 4, 8
FUSE_PRESMOOTH, FUSE_DIRECTION, FUSE_RUPDATE, FUSE_SOLVE, FUSE_PACK = 16, 32, 64, 128, 256

# exported symbols of include/mlmc.h (checked by the CPU test suite)
SYMBOLS = ["mlmc_create", "mlmc_destroy", "mlmc_last_error", "mlmc_grid_stride", "mlmc_workspace_bytes",
           "mlmc_modes", "mlmc_kl_modes", "mlmc_draw_xi", "mlmc_field", "mlmc_apply", "mlmc_apply_f32", "mlmc_jacobi", "mlmc_vcycle",
           "mlmc_vcycle_f32", "mlmc_solve", "mlmc_qoi", "mlmc_qoi_noalloc", "mlmc_fold_stats", "mlmc_last_plan",
           "mlmc_sample_level", "mlmc_estimate", "mlmc_estimate_adaptive", "mlmc_get_estimate", "mlmc_reset_stats",
           "mlmc_node_map", "mlmc_pause_model", "mlmc_forcing",
           "mlmc_set_profiling", "mlmc_kernel_time", "mlmc_get_tuning", "mlmc_set_tuning", "mlmc_autotune",
           "mlmc_serve_start", "mlmc_serve_stop", "mlmc_submit", "mlmc_submit_batch", "mlmc_poll", "mlmc_drain",
           "mlmc_serve_stats"]


class MLMCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int32), ("levels", ctypes.c_int32), ("sigma2", ctypes.c_double),
                ("corr_len", ctypes.c_double), ("n_modes", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("qoi", ctypes.c_int32), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("solver", ctypes.c_int32), ("cheb_degree", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("forcing", ctypes.c_int32), ("arena", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_size_t),
                ("stream", ctypes.c_void_p)]


class LevelStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("mean", ctypes.c_double), ("m2", ctypes.c_double),
                ("var", ctypes.c_double), ("cost", ctypes.c_double), ("nonfinite", ctypes.c_uint64)]


class PlanTask(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("n", ctypes.c_int32), ("first", ctypes.c_uint64),
                ("count", ctypes.c_int32), ("lane", ctypes.c_int32), ("task", ctypes.c_int32)]


class SampleResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("level", ctypes.c_int32), ("sample", ctypes.c_uint64),
                ("y", ctypes.c_double), ("q_fine", ctypes.c_double), ("q_coarse", ctypes.c_double),
                ("iters", ctypes.c_int32), ("latency_s", ctypes.c_double), ("queue_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# the same record as a NumPy dtype (C alignment), for draining many results at once
SAMPLE_RESULT_DTYPE = np.dtype([("ticket", np.uint64), ("status", np.int32), ("level", np.int32),
                                ("sample", np.uint64), ("y", np.float64), ("q_fine", np.float64),
                                ("q_coarse", np.float64), ("iters", np.int32), ("latency_s", np.float64),
                                ("queue_s", np.float64)], align=True)
assert SAMPLE_RESULT_DTYPE.itemsize == ctypes.sizeof(SampleResult)


class ServeStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("sample_dofs", ctypes.c_double), ("busy_seconds", ctypes.c_double),
                ("queued", ctypes.c_int32), ("running", ctypes.c_int32), ("slots", ctypes.c_int32 * 16),
                ("occupied", ctypes.c_int32 * 16), ("slot_busy_s", ctypes.c_double * 16),
                ("slot_bytes", ctypes.c_double * 16), ("uptime_s", ctypes.c_double), ("lends", ctypes.c_uint64),
                ("reclaims", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("zvar_fp32", ctypes.c_int32), ("zvar_fp64", ctypes.c_int32), ("vsmall_fp32", ctypes.c_int32),
                ("vsmall_fp64", ctypes.c_int32), ("cheb_degree", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("graph_batch", ctypes.c_int32), ("fuse", ctypes.c_int32), ("field", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EstimateOpts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("n_pilot", ctypes.c_int32), ("cost_model", ctypes.c_int32),
                ("extra_fraction", ctypes.c_double), ("max_rounds", ctypes.c_int32), ("n_fixed", ctypes.c_void_p)]


class AdaptiveOpts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("l0", ctypes.c_int32), ("n_pilot", ctypes.c_int32),
                ("cost_model", ctypes.c_int32), ("max_rounds", ctypes.c_int32), ("extra_fraction", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("beta0", ctypes.c_double)]


class AdaptiveInfo(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("rounds", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("bias", ctypes.c_double), ("err", ctypes.c_double)]


class PauseOpts(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("counts", ctypes.c_void_p), ("widths", ctypes.c_void_p),
                ("mu_us", ctypes.c_double), ("sigma_us", ctypes.c_double), ("capacity", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("min_step_us", ctypes.c_double)]


class PauseOut(ctypes.Structure):
    _fields_ = [("tasks", ctypes.c_int64), ("steps", ctypes.c_int64), ("clock_mhz", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("active_slot_s", ctypes.c_double), ("ratio", ctypes.c_double),
                ("ideal_ratio", ctypes.c_double), ("measured_slot_s", ctypes.c_double)]


class EstimateOut(ctypes.Structure):
    _fields_ = [("qtilde", ctypes.c_double), ("var_qtilde", ctypes.c_double), ("levels", ctypes.c_int32),
                ("level", LevelStats * 16), ("lanes", ctypes.c_int32), ("active_ratio", ctypes.c_double)]


_lib = None


def lib():
    """The loaded C-ABI library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "mlmc_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(P)]),
        "mlmc_destroy": (None, [P]),
        "mlmc_last_error": (ctypes.c_char_p, [P]),
        "mlmc_grid_stride": (ctypes.c_size_t, [I32]),
        "mlmc_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config), I32, I32]),
        "mlmc_modes": (ctypes.c_int, [P, P, P]),
        "mlmc_kl_modes": (ctypes.c_int, [D, D, I32, P, P, P, I32, P]),
        "mlmc_draw_xi": (ctypes.c_int, [P, I32, U64, I64, P]),
        "mlmc_field": (ctypes.c_int, [P, I32, I64, P, P, P]),
        "mlmc_apply": (ctypes.c_int, [P, I32, I64, P, P, P]),
        "mlmc_apply_f32": (ctypes.c_int, [P, I32, I64, P, P, P]),
        "mlmc_jacobi": (ctypes.c_int, [P, I32, I64, P, P, D, P]),
        "mlmc_vcycle": (ctypes.c_int, [P, I32, I64, P, P, P]),
        "mlmc_vcycle_f32": (ctypes.c_int, [P, I32, I64, P, P, P]),
        "mlmc_fold_stats": (ctypes.c_int, [P, I32, P, U64]),
        "mlmc_last_plan": (ctypes.c_int, [P, P, I32, ctypes.POINTER(I32)]),
        "mlmc_solve": (ctypes.c_int, [P, I32, I64, P, P, P]),
        "mlmc_qoi": (ctypes.c_int, [P, I32, I64, P, P]),
        "mlmc_qoi_noalloc": (ctypes.c_int, [P, I32, I64, P, P]),
        "mlmc_sample_level": (ctypes.c_int, [P, I32, U64, U64, P, P, P, P]),
        "mlmc_get_estimate": (ctypes.c_int, [P, ctypes.POINTER(EstimateOut)]),
        "mlmc_estimate": (ctypes.c_int, [P, ctypes.POINTER(EstimateOpts), P, ctypes.POINTER(EstimateOut)]),
        "mlmc_estimate_adaptive": (ctypes.c_int, [P, ctypes.POINTER(AdaptiveOpts), P, ctypes.POINTER(AdaptiveInfo),
                                                  ctypes.POINTER(EstimateOut)]),
        "mlmc_reset_stats": (ctypes.c_int, [P]),
        "mlmc_node_map": (ctypes.c_int, [P, I32, P]),
        "mlmc_forcing": (ctypes.c_int, [P, I32, I32, U64, I64, P, P]),
        "mlmc_pause_model": (ctypes.c_int, [P, ctypes.POINTER(PauseOpts), P, P, ctypes.POINTER(PauseOut)]),
        "mlmc_set_profiling": (ctypes.c_int, [P, I32]),
        "mlmc_get_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "mlmc_set_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "mlmc_autotune": (ctypes.c_int, [P, I32, I32, ctypes.POINTER(Tuning)]),
        "mlmc_serve_start": (ctypes.c_int, [P, P]),
        "mlmc_serve_stop": (ctypes.c_int, [P]),
        "mlmc_submit": (ctypes.c_int, [P, I32, U64, ctypes.POINTER(U64)]),
        "mlmc_poll": (ctypes.c_int, [P, U64, ctypes.POINTER(SampleResult)]),
        "mlmc_submit_batch": (ctypes.c_int, [P, I32, P, P, P]),
        "mlmc_drain": (ctypes.c_int, [P, P, I32, ctypes.POINTER(I32), D]),
        "mlmc_serve_stats": (ctypes.c_int, [P, ctypes.POINTER(ServeStats)]),
        "mlmc_kernel_time": (ctypes.c_int, [P, I32, I32, ctypes.POINTER(I64), ctypes.POINTER(D),
                                            ctypes.POINTER(D)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def grid_stride(n: int) -> int:
    return int(lib().mlmc_grid_stride(n))


def make_config(wl, arena_ptr: int = 0, arena_bytes: int = 0, stream: int = 0, **over) -> Config:
    """mlmc_config from a workloads.Workload (fields may be overridden)."""
    v = dict(n0=wl.n0, levels=wl.levels, sigma2=wl.sigma2, corr_len=wl.corr_len, n_modes=wl.n_modes,
             seed=wl.seed, qoi=wl.qoi, rtol=wl.rtol, max_iter=wl.max_iter, precision=wl.precision,
             solver=wl.solver, cheb_degree=0, max_batch=max(1, wl.batch or 64),
             forcing=getattr(wl, "forcing", 0))
    v.update(over)
    return Config(v["n0"], v["levels"], v["sigma2"], v["corr_len"], v["n_modes"], v["seed"], v["qoi"],
                  v["rtol"], v["max_iter"], v["precision"], v["solver"], v["cheb_degree"], v["max_batch"],
                  v["forcing"], arena_ptr, arena_bytes, stream)


def kl_modes(corr_len: float, sigma2: float, n_modes: int):
    """The library's KLE mode selection without a context (host only):
    (triples [M, 3] int32, lambda [M], omega of the 1D modes used)."""
    tri = np.zeros((n_modes, 3), dtype=np.int32)
    lam = np.zeros(n_modes)
    k1 = ctypes.c_int32()
    rc = lib().mlmc_kl_modes(corr_len, sigma2, n_modes, tri.ctypes.data, lam.ctypes.data, None, 0, ctypes.byref(k1))
    if rc != MLMC_OK:
        raise MLMCError(rc, "mlmc_kl_modes: bad arguments")
    om = np.zeros(max(1, k1.value))
    lib().mlmc_kl_modes(corr_len, sigma2, n_modes, None, None, om.ctypes.data, k1.value, None)
    return tri, lam, om[:k1.value]


def workspace_bytes(cfg: Config, level: int, batch: int) -> int:
    return int(lib().mlmc_workspace_bytes(ctypes.byref(cfg), level, batch))


def _ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


class Context:
    """One library context on cuda:0 with its own arena tensor."""

    def __init__(self, wl, arena_bytes: Optional[int] = None, **over):
        import torch
        self.torch = torch
        self.wl = wl
        probe = make_config(wl, **over)
        if arena_bytes is None:
            need = max(workspace_bytes(probe, l, probe.max_batch) for l in range(probe.levels))
            fp64 = make_config(wl, **dict(over, precision=0, solver=0))
            need = max(need, max(workspace_bytes(fp64, l, probe.max_batch) for l in range(probe.levels)))
            arena_bytes = need + (1 << 20)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
        self.stream = torch.cuda.current_stream()
        self.cfg = make_config(wl, self.arena.data_ptr(), arena_bytes, self.stream.cuda_stream, **over)
        h = ctypes.c_void_p()
        rc = lib().mlmc_create(ctypes.byref(self.cfg), ctypes.byref(h))
        if rc:
            raise MLMCError(rc, lib().mlmc_last_error(None).decode())
        self.h = h
        self.M = self.cfg.n_modes

    def close(self):
        if getattr(self, "h", None):
            lib().mlmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, allow=()):
        if rc and rc not in allow:
            raise MLMCError(rc, lib().mlmc_last_error(self.h).decode())
        return rc

    # --- step-level calls (device tensors) -----------------------------------
    def modes(self):
        tri = np.zeros((self.M, 3), dtype=np.int32)
        lam = np.zeros(self.M)
        self._check(lib().mlmc_modes(self.h, tri.ctypes.data, lam.ctypes.data))
        return tri, lam

    def draw_xi(self, level: int, first: int, count: int):
        xi = self.torch.empty((count, self.M), dtype=self.torch.float64, device="cuda")
        self._check(lib().mlmc_draw_xi(self.h, level, first, count, _ptr(xi)))
        return xi

    def field(self, n: int, xi, want32: bool = False):
        B = xi.shape[0]
        k = self.torch.empty((B, n ** 3), dtype=self.torch.float64, device="cuda")
        k32 = self.torch.empty((B, n ** 3), dtype=self.torch.float32, device="cuda") if want32 else None
        self._check(lib().mlmc_field(self.h, n, B, _ptr(xi.contiguous()), _ptr(k), _ptr(k32)))
        return (k, k32) if want32 else k

    def apply(self, n: int, kappa, u_grid):
        y = self.torch.zeros_like(u_grid)
        self._check(lib().mlmc_apply(self.h, n, u_grid.shape[0], _ptr(kappa), _ptr(u_grid), _ptr(y)))
        return y

    def jacobi(self, n: int, kappa, b_grid, c: float = 1.0):
        """mlmc_jacobi: z = c D^-1 b (fp64, grid layout)."""
        z = self.torch.zeros_like(b_grid)
        self._check(lib().mlmc_jacobi(self.h, n, b_grid.shape[0], _ptr(kappa), _ptr(b_grid), c, _ptr(z)))
        return z

    def vcycle(self, n: int, kappa, r_grid):
        z = self.torch.zeros_like(r_grid)
        self._check(lib().mlmc_vcycle(self.h, n, r_grid.shape[0], _ptr(kappa), _ptr(r_grid), _ptr(z)))
        return z

    def apply_f32(self, n: int, kappa32, u_grid32):
        """mlmc_apply_f32: fp32 kappa and u (grid layout) -> fp32 y."""
        y = self.torch.zeros_like(u_grid32)
        self._check(lib().mlmc_apply_f32(self.h, n, u_grid32.shape[0], _ptr(kappa32), _ptr(u_grid32), _ptr(y)))
        return y

    def vcycle_f32(self, n: int, kappa32, r_grid32):
        """mlmc_vcycle_f32: the fp32 V-cycle of the mixed-precision inner solve."""
        z = self.torch.zeros_like(r_grid32)
        self._check(lib().mlmc_vcycle_f32(self.h, n, r_grid32.shape[0], _ptr(kappa32), _ptr(r_grid32), _ptr(z)))
        return z

    def fold_stats(self, level: int, y, allow_nonfinite: bool = False):
        """mlmc_fold_stats: fold device fp64 values into a level's running statistics."""
        rc = lib().mlmc_fold_stats(self.h, level, _ptr(y), y.numel())
        self._check(rc, allow=(-5,) if allow_nonfinite else ())
        return rc

    def last_plan(self):
        """Parts of the tasks of the last sampling round: list of dicts (level, n, first, count, lane, task)."""
        n = ctypes.c_int32()
        self._check(lib().mlmc_last_plan(self.h, None, 0, ctypes.byref(n)))
        buf = (PlanTask * max(1, n.value))()
        self._check(lib().mlmc_last_plan(self.h, buf, n.value, ctypes.byref(n)))
        return [{k: getattr(buf[i], k) for k, _ in PlanTask._fields_} for i in range(n.value)]

    def solve(self, n: int, kappa, allow_noconv: bool = False):
        B = kappa.shape[0]
        u = self.torch.zeros((B, grid_stride(n)), dtype=self.torch.float64, device="cuda")
        it = np.zeros(B, dtype=np.int32)
        rc = lib().mlmc_solve(self.h, n, B, _ptr(kappa), _ptr(u), it.ctypes.data)
        self._check(rc, allow=(-4,) if allow_noconv else ())
        return u, it

    def qoi(self, n: int, u_grid):
        q = self.torch.empty(u_grid.shape[0], dtype=self.torch.float64, device="cuda")
        self._check(lib().mlmc_qoi(self.h, n, u_grid.shape[0], _ptr(u_grid), _ptr(q)))
        return q

    def qoi_noalloc(self, n: int, u_grid, q=None):
        """mlmc_qoi_noalloc: the QoI with its partial sums in the library's static scratch (q may be given)."""
        if q is None:
            q = self.torch.empty(u_grid.shape[0], dtype=self.torch.float64, device="cuda")
        self._check(lib().mlmc_qoi_noalloc(self.h, n, u_grid.shape[0], _ptr(u_grid), _ptr(q)))
        return q

    # --- whole path (host outputs) -------------------------------------------
    def sample_level(self, level: int, first: int, count: int, allow=()):
        """(Y, Q_fine, Q_coarse, fine iterations) of samples first.. of a level; `allow`: error codes
        returned instead of raised (the outputs are filled)."""
        y = np.zeros(count)
        qf = np.zeros(count)
        qc = np.zeros(count)
        it = np.zeros(count, dtype=np.int32)
        self.last_rc = self._check(lib().mlmc_sample_level(self.h, level, first, count, y.ctypes.data,
                                                           qf.ctypes.data, qc.ctypes.data, it.ctypes.data), allow)
        return y, qf, qc, it

    @staticmethod
    def _estimate_dict(out):
        lv = [dict(n=out.level[l].n, mean=out.level[l].mean, m2=out.level[l].m2, var=out.level[l].var,
                   cost=out.level[l].cost, nonfinite=out.level[l].nonfinite) for l in range(out.levels)]
        return dict(qtilde=out.qtilde, var_qtilde=out.var_qtilde, levels=lv, lanes=out.lanes,
                    active_ratio=out.active_ratio)

    def get_estimate(self):
        out = EstimateOut()
        self._check(lib().mlmc_get_estimate(self.h, ctypes.byref(out)))
        return self._estimate_dict(out)

    def estimate(self, eps: float, n_pilot: int = 32, cost_model: int = 0, extra_fraction: float = 0.0,
                 max_rounds: int = 3, n_fixed=None, allow=()):
        """Pilot + optimal allocation + top-up (mlmc_estimate), or plain MLMC with n_fixed;
        returns (N_l, estimate dict)."""
        fixed = None if n_fixed is None else np.ascontiguousarray(n_fixed, dtype=np.uint64)
        opts = EstimateOpts(eps, n_pilot, cost_model, extra_fraction, max_rounds,
                            None if fixed is None else fixed.ctypes.data)
        nl = np.zeros(self.cfg.levels, dtype=np.uint64)
        out = EstimateOut()
        self.last_rc = self._check(lib().mlmc_estimate(self.h, ctypes.byref(opts), nl.ctypes.data,
                                                       ctypes.byref(out)), allow)
        return nl, self._estimate_dict(out)

    def estimate_adaptive(self, eps: float, l0: int = 1, n_pilot: int = 32, cost_model: int = 0,
                          max_rounds: int = 10, extra_fraction: float = 0.0, alpha0: float = 0.0,
                          beta0: float = 0.0):
        """Adaptive MLMC (mlmc_estimate_adaptive); returns (N_l, info dict, estimate dict)."""
        opts = AdaptiveOpts(eps, l0, n_pilot, cost_model, max_rounds, extra_fraction, alpha0, beta0)
        nl = np.zeros(self.cfg.levels, dtype=np.uint64)
        info = AdaptiveInfo()
        out = EstimateOut()
        self._check(lib().mlmc_estimate_adaptive(self.h, ctypes.byref(opts), nl.ctypes.data, ctypes.byref(info),
                                                 ctypes.byref(out)))
        inf = dict(L=info.L, rounds=info.rounds, alpha=info.alpha, beta=info.beta, bias=info.bias, err=info.err)
        return nl, inf, self._estimate_dict(out)

    def reset_stats(self):
        self._check(lib().mlmc_reset_stats(self.h))

    def forcing(self, n: int, level: int, first: int, count: int):
        """Random forcing of samples first.. of a level on mesh n (mlmc_forcing): (f [count, n^3], b [count, stride])."""
        t = self.torch
        f = t.empty((count, n ** 3), dtype=t.float64, device="cuda")
        b = t.empty((count, grid_stride(n)), dtype=t.float64, device="cuda")
        self._check(lib().mlmc_forcing(self.h, n, level, first, count, _ptr(f), _ptr(b)))
        return f, b

    def node_map(self, n: int) -> np.ndarray:
        """The device's interior-unknown number at every grid position of mesh n (-1: none)."""
        out = np.empty(grid_stride(n), dtype=np.int32)
        self._check(lib().mlmc_node_map(self.h, n, out.ctypes.data))
        return out

    def pause_model(self, counts, widths, mu_us: float, sigma_us: float, capacity: int, batch: int = 1,
                    min_step_us: float = 0.0):
        """Pause-model scheduler stress (mlmc_pause_model); returns (summary dict, ticks, done_step).

        ticks and done_step are per sample, level-major (all samples of level 0 first)."""
        c = np.ascontiguousarray(counts, dtype=np.int64)
        w = np.ascontiguousarray(widths, dtype=np.int32)
        if c.shape != w.shape or c.ndim != 1:
            raise ValueError("counts and widths need one entry per level")
        opts = PauseOpts(len(c), c.ctypes.data, w.ctypes.data, mu_us, sigma_us, capacity, batch, min_step_us)
        total = int(c.sum()) if len(c) else 0
        ticks = np.zeros(max(total, 1), dtype=np.int64)
        done = np.zeros(max(total, 1), dtype=np.int64)
        out = PauseOut()
        self._check(lib().mlmc_pause_model(self.h, ctypes.byref(opts), ticks.ctypes.data, done.ctypes.data,
                                           ctypes.byref(out)))
        summary = {k: getattr(out, k) for k, _ in PauseOut._fields_}
        return summary, ticks[:total], done[:total]

    def tuning(self) -> dict:
        t = Tuning()
        self._check(lib().mlmc_get_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning()
        self._check(lib().mlmc_get_tuning(self.h, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, v)
        self._check(lib().mlmc_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, level: int, batch: int) -> dict:
        t = Tuning()
        self._check(lib().mlmc_autotune(self.h, level, batch, ctypes.byref(t)))
        return t.as_dict()

    # --- serving (continuous batching) ----------------------------------------
    def serve_start(self, slots_per_mesh=None):
        arr = None
        if slots_per_mesh is not None:
            arr = np.ascontiguousarray(slots_per_mesh, dtype=np.int32)
        self._check(lib().mlmc_serve_start(self.h, None if arr is None else arr.ctypes.data))
        self._slots = arr

    def serve_stop(self):
        self._check(lib().mlmc_serve_stop(self.h))

    def submit(self, level: int, sample: int) -> int:
        t = ctypes.c_uint64()
        self._check(lib().mlmc_submit(self.h, level, sample, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """None while pending, else the result dict."""
        r = SampleResult()
        rc = lib().mlmc_poll(self.h, ticket, ctypes.byref(r))
        if rc == MLMC_PENDING:
            return None
        self._check(rc)
        return r.as_dict()

    def serve_stats(self) -> dict:
        s = ServeStats()
        self._check(lib().mlmc_serve_stats(self.h, ctypes.byref(s)))
        return dict(completed=s.completed, sample_dofs=s.sample_dofs, busy_seconds=s.busy_seconds,
                    queued=s.queued, running=s.running, slots=list(s.slots), occupied=list(s.occupied),
                    slot_busy_s=list(s.slot_busy_s), slot_bytes=list(s.slot_bytes), uptime_s=s.uptime_s,
                    lends=s.lends, reclaims=s.reclaims)

    def submit_batch(self, levels, samples):
        lv = np.ascontiguousarray(levels, dtype=np.int32)
        sm = np.ascontiguousarray(samples, dtype=np.uint64)
        tk = np.zeros(len(lv), dtype=np.uint64)
        self._check(lib().mlmc_submit_batch(self.h, len(lv), lv.ctypes.data, sm.ctypes.data, tk.ctypes.data))
        return tk

    def drain(self, max_results: int = 4096, timeout: float = 0.05):
        """Finished results (completion order), waiting up to `timeout` s for the first."""
        buf = (SampleResult * max_results)()
        n = ctypes.c_int32()
        self._check(lib().mlmc_drain(self.h, buf, max_results, ctypes.byref(n), timeout))
        return [buf[i].as_dict() for i in range(n.value)]

    def drain_array(self, max_results: int = 16384, timeout: float = 0.0) -> np.ndarray:
        """Like drain, as a structured array of SAMPLE_RESULT_DTYPE (no per-result Python objects)."""
        buf = np.empty(max_results, dtype=SAMPLE_RESULT_DTYPE)
        n = ctypes.c_int32()
        self._check(lib().mlmc_drain(self.h, buf.ctypes.data, max_results, ctypes.byref(n), timeout))
        return buf[:n.value].copy()

    def wait(self, tickets, timeout: float = 120.0):
        """Drain until every ticket is done; returns {ticket: result}."""
        import time
        want = set(int(t) for t in tickets)
        out = {}
        t0 = time.monotonic()
        while want:
            for r in self.drain(timeout=0.05):
                if r["ticket"] in want:
                    want.discard(r["ticket"])
                out[r["ticket"]] = r
            if want and time.monotonic() - t0 > timeout:
                raise TimeoutError(f"{len(want)} requests still pending")
        return out

    def set_profiling(self, on: bool):
        self._check(lib().mlmc_set_profiling(self.h, 1 if on else 0))

    def kernel_time(self, name: str, precision: int = 0):
        """(launches, total ms, algorithmic bytes) of one kernel; precision 0 fp64, 1 fp32."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        self._check(lib().mlmc_kernel_time(self.h, KERNELS.index(name), precision, ctypes.byref(n),
                                           ctypes.byref(ms), ctypes.byref(by)))
        return n.value, ms.value, by.value


# --- layout marshalling (index bookkeeping only) ------------------------------

def interior_positions(n: int) -> np.ndarray:
    """Grid-layout position of every interior node, in canonical order
    g = (i-1) + (n-1)((j-1) + (n-1)(k-1)); position = i + n j + n^2 k."""
    m = n - 1
    g = np.arange(m ** 3)
    i, j, k = g % m + 1, (g // m) % m + 1, g // (m * m) + 1
    return i + n * j + n * n * k


def to_grid(v, n: int):
    """[B, (n-1)^3] canonical (torch, cuda) -> [B, stride] grid layout with zero boundary."""
    import torch
    pos = torch.as_tensor(interior_positions(n), device=v.device)
    out = torch.zeros((v.shape[0], grid_stride(n)), dtype=v.dtype, device=v.device)
    out[:, pos] = v
    return out


def from_grid(g, n: int):
    import torch
    pos = torch.as_tensor(interior_positions(n), device=g.device)
    return g[:, pos]
