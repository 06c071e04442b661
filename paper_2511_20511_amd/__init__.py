"""MI355X (gfx950) pilot assignment: K-means-seeded elitist 2D genetic algorithm.

Thin ctypes binding over ``libpa_amd.so`` (C ABI declared in ``include/pa.h``).
The functions keep the C names; they only marshal arguments (torch tensors
for device buffers, numpy arrays for host buffers) and raise ``PaError`` on a
nonzero status.  Every step of the method runs in the library's HIP kernels;
there is no CPU fallback: without the built library every call raises.

torch is imported before the library is loaded so both use the same HIP
runtime (``libamdhip64.so.7``) and torch's device pointers and streams are
valid inside the library.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "PaError", "GaParams", "Result", "lib", "library_path",
    "pa_context_create", "pa_context_destroy", "pa_instance_create", "pa_instance_destroy",
    "pa_kmeans_init", "pa_fitness", "pa_fitness_shaped", "pa_ga_step", "pa_solve",
    "pa_solve_plain", "pa_solve_batch", "pa_solve_begin", "pa_solve_next", "pa_solve_state",
    "pa_solve_shape", "pa_solve_batch_begin", "pa_solve_batch_next", "pa_solve_batch_state",
    "pa_solve_population", "pa_solve_resume", "pa_device_peaks", "pa_solve_noalloc", "pa_population_kmeans", "pa_island_step",
    "pa_island_solve", "release_all", "pa_server_create", "pa_server_submit", "pa_server_poll", "pa_server_stats",
    "pa_server_destroy", "pa_server_cancel", "Server", "pa_exhaustive",
    "pa_instance_kmeans_state", "pa_problem_check", "pa_params_check",
    "pa_status_string", "pa_last_error", "pa_version",
    "SE_ASYMPTOTIC", "SE_FINITE_M",
]

SE_ASYMPTOTIC = 0
SE_FINITE_M = 1
OBJ_SUM_SE = 0
OBJ_MIN_SINR = 1
OBJ_INTERCLUSTER = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libpa_amd.so")


class PaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("K", ctypes.c_int32), ("tau", ctypes.c_int32),
                ("T", ctypes.c_int32), ("M", ctypes.c_int32), ("rho", ctypes.c_double),
                ("se_mode", ctypes.c_int32), ("beta", ctypes.c_void_p),
                ("user_xy", ctypes.c_void_p), ("bs_xy", ctypes.c_void_p),
                ("objective", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_int32), ("gens", ctypes.c_int32), ("elite", ctypes.c_int32),
                ("p_cross", ctypes.c_double), ("p_mut", ctypes.c_double),
                ("kmeans_frac", ctypes.c_double), ("p_init", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("instance_id", ctypes.c_uint32)]


class _Result(ctypes.Structure):
    _fields_ = [("best", ctypes.c_void_p), ("best_fit", ctypes.c_float),
                ("best_index", ctypes.c_int32), ("trace", ctypes.c_void_p),
                ("device_ms", ctypes.c_double)]


@dataclass
class GaParams:
    pop: int = 50
    gens: int = 100
    elite: int = 2
    p_cross: float = 0.8
    p_mut: float = 0.05
    kmeans_frac: float = 0.5
    p_init: float = 0.1
    seed: int = 1
    instance_id: int = 0

    def to_c(self) -> _Params:
        return _Params(self.pop, self.gens, self.elite, self.p_cross, self.p_mut,
                       self.kmeans_frac, self.p_init, self.seed & ((1 << 64) - 1),
                       self.instance_id & 0xFFFFFFFF)


class _ServerCfg(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("max_L", ctypes.c_int32), ("max_K", ctypes.c_int32),
                ("max_pop", ctypes.c_int32), ("max_gens", ctypes.c_int32),
                ("hbm_budget", ctypes.c_double)]


class _PeakRates(ctypes.Structure):
    _fields_ = [("lds_b32", ctypes.c_double), ("lds_b128", ctypes.c_double),
                ("valu_f32", ctypes.c_double), ("clock_mhz", ctypes.c_double),
                ("cus", ctypes.c_int32)]


class _ServerCounters(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("resident", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("submitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("ticks", ctypes.c_uint64),
                ("slot_bytes", ctypes.c_double), ("max_tasks_per_workgroup", ctypes.c_int32),
                ("max_resident", ctypes.c_int32), ("cancelled", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("arena_bytes", ctypes.c_double),
                ("arena_peak_bytes", ctypes.c_double)]


@dataclass
class Result:
    best: np.ndarray
    best_fit: float
    best_index: int
    trace: np.ndarray
    device_ms: float


_lib = None
# every live handle, so that release_all() can free them in order at exit
_live = {"servers": weakref.WeakSet(), "instances": weakref.WeakSet(),
         "contexts": weakref.WeakSet()}


def release_all():
    """Destroys every live server, instance and context (in that order), so no
    plan, graph, stream, event or device buffer of the library outlives the
    interpreter's orderly shutdown.  Registered with atexit when the library
    is loaded; callable at any time (the handles become closed)."""
    for kind in ("servers", "instances", "contexts"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


def lib():
    """Loads libpa_amd.so (after torch, so the HIP runtime is shared)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads torch's libamdhip64 first)
    if not os.path.exists(library_path):
        raise RuntimeError(f"{library_path} is not built: run `python -m paper_2511_20511_amd.build`")
    L = ctypes.CDLL(library_path)
    vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32
    sig = {
        "pa_context_create": (st, [i32, ctypes.POINTER(vp)]),
        "pa_context_destroy": (None, [vp]),
        "pa_instance_create": (st, [vp, ctypes.POINTER(_Problem), ctypes.POINTER(vp)]),
        "pa_instance_destroy": (None, [vp]),
        "pa_kmeans_init": (st, [vp, ctypes.POINTER(_Params), vp, vp]),
        "pa_fitness": (st, [vp, vp, i32, vp, vp]),
        "pa_fitness_shaped": (st, [vp, vp, i32, vp, i32, i32, i32, vp]),
        "pa_ga_step": (st, [vp, ctypes.POINTER(_Params), i32, vp, vp, vp, vp]),
        "pa_solve": (st, [vp, ctypes.POINTER(_Params), ctypes.POINTER(_Result), vp]),
        "pa_solve_plain": (st, [vp, ctypes.POINTER(_Params), ctypes.POINTER(_Result), vp]),
        "pa_solve_batch": (st, [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(_Params),
                                ctypes.POINTER(_Result), vp]),
        "pa_instance_kmeans_state": (st, [vp, vp, vp, vp, vp]),
        "pa_solve_begin": (st, [vp, ctypes.POINTER(_Params), vp]),
        "pa_solve_next": (st, [vp, i32, vp]),
        "pa_solve_state": (st, [vp, ctypes.POINTER(_Result), ctypes.POINTER(i32), vp]),
        "pa_solve_shape": (st, [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "pa_solve_batch_begin": (st, [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(_Params), vp]),
        "pa_solve_batch_next": (st, [vp, i32, vp]),
        "pa_solve_batch_state": (st, [vp, ctypes.POINTER(_Result), ctypes.POINTER(i32), vp]),
        "pa_solve_population": (st, [vp, vp, i32, vp, vp, ctypes.POINTER(i32), vp]),
        "pa_solve_resume": (st, [vp, ctypes.POINTER(_Params), i32, vp, vp, vp, vp]),
        "pa_server_create": (st, [vp, ctypes.POINTER(_ServerCfg), ctypes.POINTER(vp)]),
        "pa_server_submit": (st, [vp, ctypes.POINTER(_Problem), ctypes.POINTER(_Params),
                                  ctypes.POINTER(ctypes.c_uint64)]),
        "pa_server_poll": (st, [vp, ctypes.c_uint64, ctypes.POINTER(_Result), i32]),
        "pa_server_stats": (st, [vp, ctypes.POINTER(_ServerCounters)]),
        "pa_server_cancel": (st, [vp, ctypes.c_uint64]),
        "pa_server_destroy": (None, [vp]),
        "pa_exhaustive": (st, [vp, ctypes.c_int64, ctypes.POINTER(_Result),
                               ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), vp]),
        "pa_device_peaks": (st, [vp, ctypes.POINTER(_PeakRates)]),
        "pa_solve_noalloc": (st, [vp, ctypes.POINTER(_Params), vp, vp, vp, vp]),
        "pa_population_kmeans": (st, [vp, i32, i32, vp, vp, i32, vp, vp]),
        "pa_island_step": (st, [vp, ctypes.POINTER(_Params), i32, i32, vp, vp, vp, vp, vp]),
        "pa_island_solve": (st, [vp, ctypes.POINTER(_Params), i32, i32, i32,
                                 ctypes.POINTER(_Result), vp, vp]),
        "pa_problem_check": (st, [ctypes.POINTER(_Problem)]),
        "pa_params_check": (st, [ctypes.POINTER(_Problem), ctypes.POINTER(_Params)]),
        "pa_status_string": (ctypes.c_char_p, [st]),
        "pa_last_error": (ctypes.c_char_p, []),
        "pa_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    atexit.register(release_all)
    return L


def _check(status: int):
    if status != 0:
        raise PaError(status, lib().pa_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda) torch tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


class _Host:
    """Keeps the host arrays of a pa_problem alive while the C struct points at them."""

    def __init__(self, beta, user_xy, bs_xy, T, M, rho, se_mode, objective=0):
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        L, L2, K = self.beta.shape
        if L != L2:
            raise ValueError("beta must be [L][L][K]")
        self.user_xy = None if user_xy is None else np.ascontiguousarray(user_xy, dtype=np.float64)
        self.bs_xy = None if bs_xy is None else np.ascontiguousarray(bs_xy, dtype=np.float64)
        self.c = _Problem(L, K, K, int(T), int(M), float(rho), int(se_mode),
                          self.beta.ctypes.data,
                          None if self.user_xy is None else self.user_xy.ctypes.data,
                          None if self.bs_xy is None else self.bs_xy.ctypes.data,
                          int(objective))
        self.L, self.K = L, K


def pa_version() -> str:
    return lib().pa_version().decode()


def pa_status_string(status: int) -> str:
    return lib().pa_status_string(status).decode()


def pa_last_error() -> str:
    return lib().pa_last_error().decode()


def pa_problem_check(beta, user_xy=None, bs_xy=None, T=0, M=1, rho=1.0, se_mode=SE_ASYMPTOTIC):
    """Host-only validation of a problem; returns the status (0 = valid)."""
    h = _Host(beta, user_xy, bs_xy, T, M, rho, se_mode)
    return int(lib().pa_problem_check(ctypes.byref(h.c)))


def pa_params_check(beta, params: GaParams, user_xy=None, bs_xy=None, T=0, M=1, rho=1.0,
                    se_mode=SE_ASYMPTOTIC):
    h = _Host(beta, user_xy, bs_xy, T, M, rho, se_mode)
    p = params.to_c()
    return int(lib().pa_params_check(ctypes.byref(h.c), ctypes.byref(p)))


class Context:
    def __init__(self, device: int = 0):
        self.h = ctypes.c_void_p()
        _check(lib().pa_context_create(device, ctypes.byref(self.h)))
        _live["contexts"].add(self)

    def close(self):
        if self.h:
            lib().pa_context_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Instance:
    def __init__(self, ctx: Context, beta, user_xy=None, bs_xy=None, T=0, M=1, rho=1.0,
                 se_mode=SE_ASYMPTOTIC, objective=0):
        self.ctx = ctx
        host = _Host(beta, user_xy, bs_xy, T, M, rho, se_mode, objective)
        self.L, self.K = host.L, host.K
        self.h = ctypes.c_void_p()
        _check(lib().pa_instance_create(ctx.h, ctypes.byref(host.c), ctypes.byref(self.h)))
        _live["instances"].add(self)

    def close(self):
        if self.h:
            lib().pa_instance_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pa_context_create(device: int = 0) -> Context:
    return Context(device)


def pa_context_destroy(ctx: Context):
    ctx.close()


def pa_instance_create(ctx: Context, beta, user_xy=None, bs_xy=None, T=0, M=1, rho=1.0,
                       se_mode=SE_ASYMPTOTIC, objective=0) -> Instance:
    return Instance(ctx, beta, user_xy, bs_xy, T, M, rho, se_mode, objective)


def pa_instance_destroy(inst: Instance):
    inst.close()


def pa_kmeans_init(inst: Instance, params: GaParams, d_pop, stream=None):
    import torch
    p = params.to_c()
    _check(lib().pa_kmeans_init(inst.h, ctypes.byref(p), _dev(d_pop, torch.uint8), _stream(stream)))


def pa_fitness(inst: Instance, d_pop, n: int, d_fit, stream=None):
    import torch
    _check(lib().pa_fitness(inst.h, _dev(d_pop, torch.uint8), int(n), _dev(d_fit, torch.float32),
                            _stream(stream)))


def pa_fitness_shaped(inst: Instance, d_pop, n: int, d_fit, block=0, grid_cap=0, generic=0,
                      stream=None):
    import torch
    _check(lib().pa_fitness_shaped(inst.h, _dev(d_pop, torch.uint8), int(n),
                                   _dev(d_fit, torch.float32), int(block), int(grid_cap),
                                   int(generic), _stream(stream)))


def pa_ga_step(inst: Instance, params: GaParams, gen: int, d_pop_in, d_fit_in, d_pop_out,
               stream=None):
    import torch
    p = params.to_c()
    _check(lib().pa_ga_step(inst.h, ctypes.byref(p), int(gen), _dev(d_pop_in, torch.uint8),
                            _dev(d_fit_in, torch.float32), _dev(d_pop_out, torch.uint8),
                            _stream(stream)))


def _solve(fn, inst: Instance, params: GaParams, stream) -> Result:
    best = np.zeros((inst.L, inst.K), dtype=np.uint8)
    trace = np.zeros(params.gens + 1, dtype=np.float32)
    r = _Result(best.ctypes.data, 0.0, 0, trace.ctypes.data, 0.0)
    p = params.to_c()
    _check(fn(inst.h, ctypes.byref(p), ctypes.byref(r), _stream(stream)))
    return Result(best, float(r.best_fit), int(r.best_index), trace, float(r.device_ms))


def pa_solve(inst: Instance, params: GaParams, stream=None) -> Result:
    return _solve(lib().pa_solve, inst, params, stream)


def pa_solve_plain(inst: Instance, params: GaParams, stream=None) -> Result:
    return _solve(lib().pa_solve_plain, inst, params, stream)


def pa_solve_batch(ctx: Context, insts, params, stream=None) -> list:
    """Solves many instances in one graph-captured batch; one Result per instance."""
    n = len(insts)
    if len(params) != n:
        raise ValueError("one GaParams per instance")
    handles = (ctypes.c_void_p * max(n, 1))(*[i.h for i in insts])
    cp = (_Params * max(n, 1))(*[p.to_c() for p in params])
    bests = [np.zeros((i.L, i.K), dtype=np.uint8) for i in insts]
    traces = [np.zeros(p.gens + 1, dtype=np.float32) for p in params]
    cr = (_Result * max(n, 1))(*[_Result(b.ctypes.data, 0.0, 0, t.ctypes.data, 0.0)
                                 for b, t in zip(bests, traces)])
    _check(lib().pa_solve_batch(ctx.h, n, handles, cp, cr, _stream(stream)))
    return [Result(bests[i], float(cr[i].best_fit), int(cr[i].best_index), traces[i],
                   float(cr[i].device_ms)) for i in range(n)]


def pa_solve_batch_begin(ctx: Context, insts, params, stream=None):
    """Stepwise batch: seeding and initial fitness of every instance."""
    n = len(insts)
    if len(params) != n:
        raise ValueError("one GaParams per instance")
    handles = (ctypes.c_void_p * max(n, 1))(*[i.h for i in insts])
    cp = (_Params * max(n, 1))(*[p.to_c() for p in params])
    _check(lib().pa_solve_batch_begin(ctx.h, n, handles, cp, _stream(stream)))
    ctx._batch = ([(i.L, i.K) for i in insts], [p.gens for p in params],
                  [p.pop for p in params])


def pa_solve_batch_next(ctx: Context, ngens: int = 1, stream=None):
    _check(lib().pa_solve_batch_next(ctx.h, int(ngens), _stream(stream)))


def pa_solve_batch_state(ctx: Context, stream=None):
    """(list of Result, generations done) of a stepwise batch."""
    shapes, gens, _ = ctx._batch
    n = len(shapes)
    bests = [np.zeros(s, dtype=np.uint8) for s in shapes]
    traces = [np.zeros(g + 1, dtype=np.float32) for g in gens]
    cr = (_Result * max(n, 1))(*[_Result(b.ctypes.data, 0.0, 0, t.ctypes.data, 0.0)
                                 for b, t in zip(bests, traces)])
    done = ctypes.c_int32(0)
    _check(lib().pa_solve_batch_state(ctx.h, cr, ctypes.byref(done), _stream(stream)))
    d = int(done.value)
    return [Result(bests[i], float(cr[i].best_fit), int(cr[i].best_index),
                   traces[i][:min(d, gens[i]) + 1], float(cr[i].device_ms))
            for i in range(n)], d


def pa_solve_population(ctx: Context | None, inst: Instance | None, index: int, L: int, K: int,
                        N: int, stream=None):
    """(population [N][L][K] uint8, fitness [N] float32, generation) of one
    instance of a plan (inst's pa_solve plan, or the context's batch plan)."""
    pop = np.zeros((N, L, K), dtype=np.uint8)
    fit = np.zeros(N, dtype=np.float32)
    gen = ctypes.c_int32(0)
    _check(lib().pa_solve_population(ctx.h if ctx is not None else None,
                                     inst.h if inst is not None else None, int(index),
                                     pop.ctypes.data, fit.ctypes.data, ctypes.byref(gen),
                                     _stream(stream)))
    return pop, fit, int(gen.value)


def pa_solve_resume(inst: Instance, params: GaParams, gen: int, pop, fit=None, trace=None,
                    stream=None):
    """Continue a stepwise solve from a saved state: pop [N][L][K] uint8 of
    generation gen (host), its fitness [N] float32 (None: recomputed) and the
    trace of generations 0..gen-1 (None: NaN).  pa_solve_next and
    pa_solve_state follow as in an uninterrupted solve."""
    inst._gens = params.gens
    pop = np.ascontiguousarray(pop, dtype=np.uint8)
    if pop.shape != (params.pop, inst.L, inst.K):
        raise ValueError(f"population shape {pop.shape} != {(params.pop, inst.L, inst.K)}")
    if fit is not None:
        fit = np.ascontiguousarray(fit, dtype=np.float32)
        if fit.shape != (params.pop,):
            raise ValueError(f"fitness shape {fit.shape} != {(params.pop,)}")
    if trace is not None:
        trace = np.ascontiguousarray(trace, dtype=np.float32)
        if trace.ndim != 1 or trace.shape[0] < gen:
            raise ValueError(f"trace holds {trace.shape} entries, needs {gen}")
    p = params.to_c()
    _check(lib().pa_solve_resume(inst.h, ctypes.byref(p), int(gen), pop.ctypes.data,
                                 None if fit is None else fit.ctypes.data,
                                 None if trace is None else trace.ctypes.data,
                                 _stream(stream)))


def pa_solve_noalloc(inst: Instance, params: GaParams, d_best, d_best_fit, d_trace=None,
                     stream=None):
    """pa_solve without any device allocation (async): best chromosome, its
    fitness and (optionally) the trace into the caller's device tensors
    (uint8 [L][K], float32 [1], float32 [gens+1])."""
    import torch
    p = params.to_c()
    _check(lib().pa_solve_noalloc(inst.h, ctypes.byref(p), _dev(d_best, torch.uint8),
                                  _dev(d_best_fit, torch.float32),
                                  None if d_trace is None else _dev(d_trace, torch.float32),
                                  _stream(stream)))


def pa_population_kmeans(inst: Instance, clusters: int, d_pop, d_fit, n: int, d_labels,
                         kmeans_iters: int = 20, stream=None):
    """K-means of a device population into islands (Alg. 2); labels into d_labels."""
    import torch
    _check(lib().pa_population_kmeans(inst.h, int(clusters), int(kmeans_iters),
                                      _dev(d_pop, torch.uint8), _dev(d_fit, torch.float32),
                                      int(n), _dev(d_labels, torch.int32), _stream(stream)))


def pa_island_step(inst: Instance, params: GaParams, clusters: int, gen: int, d_labels,
                   d_pop_in, d_fit_in, d_pop_out, stream=None):
    """One generation of every island (Alg. 2 loop body)."""
    import torch
    p = params.to_c()
    _check(lib().pa_island_step(inst.h, ctypes.byref(p), int(clusters), int(gen),
                                _dev(d_labels, torch.int32), _dev(d_pop_in, torch.uint8),
                                _dev(d_fit_in, torch.float32), _dev(d_pop_out, torch.uint8),
                                _stream(stream)))


def pa_island_solve(inst: Instance, params: GaParams, clusters: int, recluster_every: int = 3,
                    kmeans_iters: int = 20, stream=None):
    """The PK-means GA (Alg. 2): (Result, labels of the last partition)."""
    best = np.zeros((inst.L, inst.K), dtype=np.uint8)
    trace = np.zeros(params.gens + 1, dtype=np.float32)
    labels = np.zeros(params.pop, dtype=np.int32)
    r = _Result(best.ctypes.data, 0.0, 0, trace.ctypes.data, 0.0)
    p = params.to_c()
    _check(lib().pa_island_solve(inst.h, ctypes.byref(p), int(clusters), int(recluster_every),
                                 int(kmeans_iters), ctypes.byref(r), labels.ctypes.data,
                                 _stream(stream)))
    return Result(best, float(r.best_fit), int(r.best_index), trace, float(r.device_ms)), labels


def pa_solve_begin(inst: Instance, params: GaParams, stream=None):
    inst._gens = params.gens
    p = params.to_c()
    _check(lib().pa_solve_begin(inst.h, ctypes.byref(p), _stream(stream)))


def pa_solve_next(inst: Instance, ngens: int = 1, stream=None):
    _check(lib().pa_solve_next(inst.h, int(ngens), _stream(stream)))


def pa_solve_state(inst: Instance, stream=None):
    """(Result, generations done) of a stepwise solve."""
    gens = getattr(inst, "_gens", 0)
    best = np.zeros((inst.L, inst.K), dtype=np.uint8)
    trace = np.zeros(gens + 1, dtype=np.float32)
    r = _Result(best.ctypes.data, 0.0, 0, trace.ctypes.data, 0.0)
    done = ctypes.c_int32(0)
    _check(lib().pa_solve_state(inst.h, ctypes.byref(r), ctypes.byref(done), _stream(stream)))
    return Result(best, float(r.best_fit), int(r.best_index), trace[:done.value + 1],
                  float(r.device_ms)), int(done.value)


def pa_solve_shape(ctx: Context | None = None, inst: Instance | None = None) -> dict:
    """Execution form of the solve plan of `inst` (or of the context's batch
    plan when inst is None): persistent, block, children_per_task, workgroups."""
    vals = [ctypes.c_int32(0) for _ in range(4)]
    _check(lib().pa_solve_shape(ctx.h if ctx is not None else None,
                                inst.h if inst is not None else None,
                                *[ctypes.byref(v) for v in vals]))
    return dict(zip(("persistent", "block", "children_per_task", "workgroups"),
                    (int(v.value) for v in vals)))


def pa_instance_kmeans_state(inst: Instance):
    seed = np.zeros((inst.L, inst.K), dtype=np.uint8)
    cent = np.zeros((inst.K, 2), dtype=np.int32)
    labels = np.zeros(inst.L * inst.K, dtype=np.int32)
    iters = np.zeros(1, dtype=np.int32)
    _check(lib().pa_instance_kmeans_state(inst.h, seed.ctypes.data, cent.ctypes.data,
                                          labels.ctypes.data, iters.ctypes.data))
    return seed, cent, labels, int(iters[0])


def pa_exhaustive(inst: Instance, max_count: int = 0, stream=None):
    """Exhaustive search: (Result with best and best_fit, best enumeration rank, count)."""
    best = np.zeros((inst.L, inst.K), dtype=np.uint8)
    r = _Result(best.ctypes.data, 0.0, 0, None, 0.0)
    rank, cnt = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().pa_exhaustive(inst.h, int(max_count), ctypes.byref(r), ctypes.byref(rank),
                               ctypes.byref(cnt), _stream(stream)))
    return (Result(best, float(r.best_fit), int(r.best_index), np.zeros(0, np.float32),
                   float(r.device_ms)), int(rank.value), int(cnt.value))


def pa_device_peaks(ctx: Context) -> dict:
    """Measured peak rates of the device (LDS gathers per clock and CU with
    ds_read_b32 and ds_read_b128, FP32 VALU issue, shader clock)."""
    r = _PeakRates()
    _check(lib().pa_device_peaks(ctx.h, ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in r._fields_}


# ---- continuous-batching server ---------------------------------------------

PA_EAGAIN = -4


class Server:
    """Handle of a pa_server; remembers (L, K, gens) of every pending ticket so
    that poll can size the result arrays."""

    def __init__(self, ctx: Context, max_slots=0, max_queue=0, max_L=0, max_K=0, max_pop=0,
                 max_gens=0, hbm_budget=0.0):
        cfg = _ServerCfg(int(max_slots), int(max_queue), int(max_L), int(max_K), int(max_pop),
                         int(max_gens), float(hbm_budget))
        self.h = ctypes.c_void_p()
        _check(lib().pa_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(self.h)))
        _live["servers"].add(self)
        self.ctx = ctx
        self._shape = {}

    def close(self):
        if self.h:
            lib().pa_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pa_server_create(ctx: Context, **cfg) -> Server:
    return Server(ctx, **cfg)


def pa_server_destroy(srv: Server):
    srv.close()


def pa_server_submit(srv: Server, beta, user_xy=None, bs_xy=None, params: GaParams = None, T=0,
                     M=1, rho=1.0, se_mode=SE_ASYMPTOTIC, objective=0) -> int:
    """Queues one solve; returns its ticket (the arrays are copied)."""
    host = _Host(beta, user_xy, bs_xy, T, M, rho, se_mode, objective)
    p = params.to_c()
    t = ctypes.c_uint64(0)
    _check(lib().pa_server_submit(srv.h, ctypes.byref(host.c), ctypes.byref(p), ctypes.byref(t)))
    srv._shape[t.value] = (host.L, host.K, params.gens)
    return int(t.value)


def pa_server_poll(srv: Server, ticket: int, block: bool = True):
    """Result of a ticket (device_ms = submit-to-result time in ms), or None
    while it runs (block=False)."""
    L, K, G = srv._shape[ticket]
    best = np.zeros((L, K), dtype=np.uint8)
    trace = np.zeros(G + 1, dtype=np.float32)
    r = _Result(best.ctypes.data, 0.0, 0, trace.ctypes.data, 0.0)
    st = lib().pa_server_poll(srv.h, ctypes.c_uint64(ticket), ctypes.byref(r), 1 if block else 0)
    if st == PA_EAGAIN and not block:
        return None
    _check(st)
    del srv._shape[ticket]
    return Result(best, float(r.best_fit), int(r.best_index), trace, float(r.device_ms))


def pa_server_cancel(srv: Server, ticket: int):
    """Cancels a queued or resident request; polling it then raises PaError
    with status PA_ECANCELED (-5)."""
    _check(lib().pa_server_cancel(srv.h, ctypes.c_uint64(ticket)))


def pa_server_stats(srv: Server) -> dict:
    c = _ServerCounters()
    _check(lib().pa_server_stats(srv.h, ctypes.byref(c)))
    return {f: getattr(c, f) for f, _ in c._fields_}
