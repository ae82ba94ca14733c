"""Python binding of libparareal.so (the C ABI in include/parareal.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Device buffers are passed as torch CUDA tensors (float64,
contiguous) or raw integer device pointers.  The binding refuses to run if
the compiled library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libparareal.so")

PR_OK = 0
PR_EINVAL = -1
PR_EUNSTABLE = -2
PR_ENOMEM = -3
PR_EHIP = -4
PR_ENOTCONV = -5
PR_ENORESIDENT = -6
PR_ETIMEOUT = -7

PR_COARSE_AUTO = 0
PR_COARSE_THOMAS = 1
PR_COARSE_CG = 2

PR_ASYNC_FREE = 0
PR_ASYNC_EXACT = 1
PR_ASYNC_REPLAY = 2
PR_ASYNC_PIPELINED = 3
PR_FINE_EXPLICIT = 0
PR_FINE_BACKWARD_EULER = 1
PR_FINE_TRAPEZOIDAL = 2


class pr_config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int), ("nu", ctypes.c_double),
        ("T", ctypes.c_double), ("nslices", ctypes.c_int), ("dt_nominal", ctypes.c_double),
        ("coarse", ctypes.c_int), ("cg_tol", ctypes.c_double), ("cg_maxit", ctypes.c_int),
        ("eps", ctypes.c_double), ("kmax", ctypes.c_int), ("tb_depth", ctypes.c_int),
        ("tile_rows", ctypes.c_int), ("coarse_increment", ctypes.c_int),
        ("fine_xpts", ctypes.c_int), ("fine", ctypes.c_int), ("cg_precond", ctypes.c_int),
    ]


class pr_info(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int), ("dt", ctypes.c_double), ("dT", ctypes.c_double),
        ("h", ctypes.c_double), ("r", ctypes.c_double), ("s", ctypes.c_double),
        ("npts", ctypes.c_longlong), ("offset", ctypes.c_longlong),
        ("tb_depth", ctypes.c_int), ("tile_rows", ctypes.c_int),
        ("xpts", ctypes.c_int), ("sliding", ctypes.c_int), ("cg_precond", ctypes.c_int),
    ]


class pr_stats(ctypes.Structure):
    _fields_ = [
        ("k_per_slice", ctypes.POINTER(ctypes.c_int)),
        ("deltas", ctypes.POINTER(ctypes.c_double)),
        ("deltas_cap", ctypes.c_int),
        ("iters", ctypes.c_int), ("kappa", ctypes.c_int), ("converged", ctypes.c_int),
        ("last_delta", ctypes.c_double), ("wall_ms", ctypes.c_double),
        ("fine_ms", ctypes.c_double), ("coarse_ms", ctypes.c_double),
        ("fine_lups", ctypes.c_double), ("cg_iters", ctypes.c_longlong),
        ("g_solves", ctypes.c_longlong), ("g_skipped", ctypes.c_longlong),
        ("kernel_ms", ctypes.c_double), ("kernel_cg_iters", ctypes.c_longlong),
        ("kernel_updates", ctypes.c_longlong),
        ("teams", ctypes.c_int), ("copy_retries", ctypes.c_longlong),
        ("idle_rounds", ctypes.c_longlong),
        ("team_fine_ms", ctypes.c_double), ("team_copy_ms", ctypes.c_double),
        ("team_coarse_ms", ctypes.c_double), ("team_corr_ms", ctypes.c_double),
        ("team_total_ms", ctypes.c_double), ("fine_cg_iters", ctypes.c_longlong),
    ]


class pr_async_opts(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int), ("teams", ctypes.c_int), ("max_local_iters", ctypes.c_int),
        ("schedule", ctypes.POINTER(ctypes.c_int)), ("delay_spins", ctypes.POINTER(ctypes.c_int)),
        ("time_limit_s", ctypes.c_double), ("latency_us", ctypes.c_double),
        ("slice_blocks", ctypes.c_int),
        ("drop_every", ctypes.POINTER(ctypes.c_int)), ("reset_after", ctypes.POINTER(ctypes.c_int)),
    ]


EXPORTS = [
    "pr_create", "pr_destroy", "pr_last_error", "pr_get_info", "pr_solve_sync",
    "pr_set_async_options", "pr_solve_async", "pr_solve_fine", "pr_grad",
    "pr_apply_fine", "pr_apply_coarse", "pr_fine_shape_count", "pr_fine_shape_get",
    "pr_set_fine_shape", "pr_autotune", "pr_set_graph", "pr_apply_coarse_static",
]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libparareal.so (built by paper_2110_10762_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2110_10762_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.pr_create.argtypes = [ctypes.POINTER(pr_config), ctypes.c_int, ctypes.c_int, P, ctypes.POINTER(P)]
    lib.pr_destroy.argtypes = [P]
    lib.pr_destroy.restype = None
    lib.pr_last_error.restype = ctypes.c_char_p
    lib.pr_get_info.argtypes = [P, ctypes.c_int, ctypes.POINTER(pr_info)]
    for name in ("pr_solve_sync", "pr_solve_async", "pr_solve_fine"):
        getattr(lib, name).argtypes = [P, P, P, ctypes.POINTER(pr_stats)]
    lib.pr_set_async_options.argtypes = [P, ctypes.POINTER(pr_async_opts)]
    lib.pr_grad.argtypes = [P, P, P, P, ctypes.POINTER(ctypes.c_double)]
    lib.pr_apply_fine.argtypes = [P, P, P, ctypes.c_int, ctypes.c_int]
    lib.pr_apply_coarse.argtypes = [P, P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
    lib.pr_fine_shape_count.argtypes = [ctypes.c_int]
    lib.pr_fine_shape_get.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 4
    lib.pr_set_fine_shape.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.pr_autotune.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_double)]
    lib.pr_set_graph.argtypes = [P, ctypes.c_int]
    lib.pr_apply_coarse_static.argtypes = [ctypes.POINTER(pr_config), ctypes.c_int, P, P, P, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_longlong)]
    _lib = lib
    return lib


class PRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc: int, allow=()):
    if rc != PR_OK and rc not in allow:
        raise PRError(rc, load_library().pr_last_error().decode())
    return rc


def _ptr(x, numel: Optional[int] = None, at_least: bool = False) -> int:
    """Device pointer of a torch tensor (float64, contiguous, on a GPU) or an int.

    numel: the element count the library will read or write through the
    pointer; a tensor of another size (fewer elements, with at_least) is
    refused before any kernel sees it.  Raw integer pointers are the caller's
    responsibility."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a torch tensor or an integer device pointer")
    if not x.is_cuda:
        raise ValueError("buffers must live in GPU memory")
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError("buffers must be contiguous float64")
    if numel is not None:
        bad = x.numel() < numel if at_least else x.numel() != numel
        if bad:
            raise ValueError(f"buffer holds {x.numel()} values, the call needs "
                             f"{'at least ' if at_least else ''}{numel}")
    return x.data_ptr()


def make_config(dim, n, nu, T, nslices, dt_nominal, coarse=PR_COARSE_AUTO, cg_tol=1e-12,
                cg_maxit=0, eps=1e-10, kmax=0, tb_depth=0, tile_rows=0,
                coarse_increment=0, fine_xpts=0, fine=0, cg_precond=0) -> pr_config:
    return pr_config(dim, n, nu, T, nslices, dt_nominal, coarse, cg_tol, cg_maxit, eps, kmax,
                     tb_depth, tile_rows, coarse_increment, fine_xpts, fine, cg_precond)


def config_of(problem, **over) -> pr_config:
    """pr_config for a workloads.Problem (keyword overrides allowed)."""
    kw = dict(dim=problem.dim, n=problem.n, nu=problem.nu, T=problem.T,
              nslices=problem.nslices, dt_nominal=problem.dt_nominal,
              cg_tol=problem.cg_tol, eps=problem.eps)
    kw.update(over)
    return make_config(**kw)


class Stats:
    """Host-side view of pr_stats with optional per-slice and per-iteration arrays."""

    def __init__(self, nslices: int = 0, deltas_cap: int = 0):
        self.raw = pr_stats()
        self._k = (ctypes.c_int * nslices)() if nslices else None
        self._d = (ctypes.c_double * deltas_cap)() if deltas_cap else None
        if self._k is not None:
            self.raw.k_per_slice = ctypes.cast(self._k, ctypes.POINTER(ctypes.c_int))
        if self._d is not None:
            self.raw.deltas = ctypes.cast(self._d, ctypes.POINTER(ctypes.c_double))
            self.raw.deltas_cap = deltas_cap

    @property
    def k_per_slice(self):
        return list(self._k) if self._k is not None else None

    @property
    def deltas(self):
        if self._d is None:
            return None
        return list(self._d)[: max(0, min(self.raw.iters, len(self._d)))]

    def __getattr__(self, name):
        return getattr(self.raw, name)

    def as_dict(self):
        d = {f: getattr(self.raw, f) for f, _ in pr_stats._fields_ if f not in ("k_per_slice", "deltas")}
        if self._k is not None:
            d["k_per_slice"] = self.k_per_slice
        if self._d is not None:
            d["deltas"] = self.deltas
        return d


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    """Destroys every handle still open while the interpreter can still make
    HIP calls (before profilers and the runtime tear down)."""
    for p in list(_live):
        try:
            p.close()
        except Exception:
            pass


class Problem:
    """Owns one library handle (one problem, or a batch when given several configs)."""

    def __init__(self, cfgs, device: int = 0, stream: Optional[int] = None):
        lib = load_library()
        if isinstance(cfgs, pr_config):
            cfgs = [cfgs]
        arr = (pr_config * len(cfgs))(*cfgs)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        _check(lib.pr_create(arr, len(cfgs), device, ctypes.c_void_p(stream), ctypes.byref(h)))
        self.h = h
        self.lib = lib
        self.nproblems = len(cfgs)
        self.cfgs = list(cfgs)
        self.npts = [c.n ** c.dim for c in self.cfgs]
        self.state_numel = sum(self.npts)
        self.iterate_numel = sum((c.nslices + 1) * q for c, q in zip(self.cfgs, self.npts))
        _live.add(self)

    def close(self):
        """Waits for the handle's work and frees it (idempotent)."""
        if getattr(self, "h", None) and self.h.value:
            self.lib.pr_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP call once the interpreter is shutting down: the runtime (and
        # any profiler attached to it) may already be gone (module globals
        # such as `sys` may be gone too, hence the bound default)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def info(self, problem: int = 0) -> pr_info:
        out = pr_info()
        _check(self.lib.pr_get_info(self.h, problem, ctypes.byref(out)))
        return out

    def _solve(self, fn, u0, lam, stats: Optional[Stats], allow=()):
        st = stats.raw if stats is not None else None
        return _check(fn(self.h, _ptr(u0, self.state_numel), _ptr(lam, self.iterate_numel),
                         ctypes.byref(st) if st is not None else None), allow)

    def solve_sync(self, u0, lam, stats: Optional[Stats] = None, allow_notconv=False):
        return self._solve(self.lib.pr_solve_sync, u0, lam, stats, (PR_ENOTCONV,) if allow_notconv else ())

    def solve_async(self, u0, lam, stats: Optional[Stats] = None, allow_notconv=False):
        return self._solve(self.lib.pr_solve_async, u0, lam, stats, (PR_ENOTCONV,) if allow_notconv else ())

    def solve_fine(self, u0, lam, stats: Optional[Stats] = None):
        return self._solve(self.lib.pr_solve_fine, u0, lam, stats)

    def set_async_options(self, mode=PR_ASYNC_FREE, teams=0, max_local_iters=0,
                          schedule: Optional[Sequence[int]] = None,
                          delay_spins: Optional[Sequence[int]] = None,
                          time_limit_s: float = 0.0, latency_us: float = 0.0, slice_blocks: int = 0,
                          drop_every: Optional[Sequence[int]] = None,
                          reset_after: Optional[Sequence[int]] = None):
        o = pr_async_opts()
        o.mode, o.teams, o.max_local_iters = mode, teams, max_local_iters
        o.time_limit_s = time_limit_s
        o.latency_us = latency_us
        o.slice_blocks = slice_blocks
        keep = []
        if schedule is not None:
            arr = (ctypes.c_int * len(schedule))(*schedule)
            keep.append(arr)
            o.schedule = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int))
        if delay_spins is not None:
            arr = (ctypes.c_int * len(delay_spins))(*delay_spins)
            keep.append(arr)
            o.delay_spins = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int))
        for name, vals in (("drop_every", drop_every), ("reset_after", reset_after)):
            if vals is not None:
                n = self.cfgs[0].nslices
                if len(vals) != n:
                    raise ValueError(f"{name} needs one entry per slice ({n})")
                arr = (ctypes.c_int * n)(*vals)
                keep.append(arr)
                setattr(o, name, ctypes.cast(arr, ctypes.POINTER(ctypes.c_int)))
        _check(self.lib.pr_set_async_options(self.h, ctypes.byref(o)))

    def grad(self, lam, gT, dldu0) -> float:
        out = ctypes.c_double()
        _check(self.lib.pr_grad(self.h, _ptr(lam, self.iterate_numel), _ptr(gT, self.state_numel),
                                _ptr(dldu0, self.state_numel), ctypes.byref(out)))
        return out.value

    def apply_fine(self, x, y, count: int, steps: int = 0):
        q = max(count, 0) * self.npts[0]
        _check(self.lib.pr_apply_fine(self.h, _ptr(x, q, True), _ptr(y, q, True), count, steps))

    def apply_coarse(self, x, y, count: int) -> int:
        it = ctypes.c_longlong()
        q = max(count, 0) * self.npts[0]
        _check(self.lib.pr_apply_coarse(self.h, _ptr(x, q, True), _ptr(y, q, True), count, ctypes.byref(it)))
        return it.value

    def set_fine_shape(self, tb_depth: int, tile_rows: int, xpts: int = 0, problem: int = 0):
        _check(self.lib.pr_set_fine_shape(self.h, problem, tb_depth, tile_rows, xpts))

    def autotune(self, problem: int = 0, reps: int = 3):
        """Runs the library's autotuner; returns (tb_depth, tile_rows, xpts, best_ms)."""
        d, r, x, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(self.lib.pr_autotune(self.h, problem, reps, ctypes.byref(d), ctypes.byref(r), ctypes.byref(x),
                                    ctypes.byref(ms)))
        return d.value, r.value, x.value, ms.value

    def set_graph(self, enable: bool):
        _check(self.lib.pr_set_graph(self.h, 1 if enable else 0))

    def solve_batch(self, u0, lam, allow_notconv=False):
        """Batched synchronous solve; returns one Stats per problem."""
        arr = (pr_stats * self.nproblems)()
        rc = _check(self.lib.pr_solve_sync(self.h, _ptr(u0, self.state_numel), _ptr(lam, self.iterate_numel), arr),
                    (PR_ENOTCONV,) if allow_notconv else ())
        return rc, [arr[b] for b in range(self.nproblems)]


def fine_shapes(dim: int):
    """[(tb_depth, tile_rows, xpts, sliding)] of every fine-kernel shape."""
    lib = load_library()
    out = []
    for i in range(lib.pr_fine_shape_count(dim)):
        d, r, x, sw = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.pr_fine_shape_get(dim, i, ctypes.byref(d), ctypes.byref(r), ctypes.byref(x), ctypes.byref(sw)))
        out.append((d.value, r.value, x.value, sw.value))
    return out


# ---------------------------------------------------------------------- autograd

def _torch_function():
    import torch

    class HeatPararealFn(torch.autograd.Function):
        """u(T) = Parareal solution of the heat problem from u0 with diffusivity nu.

        forward: synchronous (default), asynchronous or serial-fine solve;
        the slice-boundary values lambda_0..lambda_N are kept as checkpoints.
        backward: pr_grad (adjoint of the fine integration with in-slice
        recomputation) gives dL/du0 and dL/dnu for the upstream dL/du(T).
        The fine step dt is fixed by the slicing, independent of nu."""

        @staticmethod
        def forward(ctx, u0, nu, dim, n, T, nslices, dt_nominal, eps, driver):
            if u0.numel() != n ** dim:
                raise ValueError(f"u0 holds {u0.numel()} values, a {dim}D grid of side {n} has {n ** dim}")
            cfg = make_config(dim, n, float(nu), T, nslices, dt_nominal, eps=eps)
            prob = Problem(cfg, device=u0.device.index or 0)
            lam = torch.empty((nslices + 1,) + tuple(u0.shape), dtype=torch.float64, device=u0.device)
            u = u0.detach().contiguous()
            if driver == "sync":
                prob.solve_sync(u, lam)
            elif driver == "async":
                prob.solve_async(u, lam)
            elif driver == "fine":
                prob.solve_fine(u, lam)
            else:
                raise ValueError("driver must be 'sync', 'async' or 'fine'")
            ctx.prob = prob
            ctx.nu_shape = nu.shape
            ctx.save_for_backward(lam)
            return lam[-1].clone()

        @staticmethod
        def backward(ctx, gT):
            (lam,) = ctx.saved_tensors
            d0 = torch.empty_like(gT, dtype=torch.float64).contiguous()
            dnu = ctx.prob.grad(lam, gT.to(torch.float64).contiguous(), d0)
            gnu = torch.full(ctx.nu_shape, dnu, dtype=torch.float64, device=gT.device)
            return d0, gnu, None, None, None, None, None, None, None

    return HeatPararealFn


_HPF = None


def heat_parareal(u0, nu, dim, n, T, nslices, dt_nominal, eps=1e-10, driver="sync"):
    """Differentiable u(T) (see HeatPararealFn)."""
    global _HPF
    if _HPF is None:
        _HPF = _torch_function()
    return _HPF.apply(u0, nu, dim, n, T, nslices, dt_nominal, eps, driver)
