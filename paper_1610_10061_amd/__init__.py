"""Python binding of the gfx950 p-median library (include/pmp.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libpmp.so.  PyTorch provides device memory and streams.  The binding loads
the library after torch so that both share one HIP runtime; if the library
is missing the import fails (there is no CPU fallback).

Functions carry the C names; pass torch CUDA tensors for device buffers
(the call then runs on `stream`, default torch's current stream) or numpy
arrays for host buffers.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime libpmp.so binds to)

__all__ = [
    "PmpError", "lib", "pmp_preprocess", "pmp_instance_info",
    "pmp_instance_tables", "pmp_eval_population", "pmp_eval_population_noalloc",
    "pmp_instance_check",
    "pmp_instance_destroy", "pmp_ga_create", "pmp_ga_step", "pmp_ga_best",
    "pmp_ga_state", "pmp_ga_destroy", "pmp_solve", "pmp_ga_profile",
    "pmp_ga_profile_read", "pmp_ga_autotune", "pmp_batch_create",
    "pmp_batch_step", "pmp_batch_check", "pmp_batch_destroy",
    "pmp_batch_profile", "pmp_batch_profile_read", "pmp_batch_autotune",
    "pmp_ga_step_batch", "pmp_features", "pmp_model_create", "pmp_model_get",
    "pmp_model_set", "pmp_model_forward", "pmp_model_grad", "pmp_model_train",
    "pmp_model_destroy", "pmp_ga_set_model", "pmp_ga_replay", "pmp_exhaustive",
    "pmp_apsp", "pmp_hbp_reduce", "pmp_hbp_info", "pmp_hbp_terms", "pmp_hbp_eval",
    "pmp_hbp_destroy", "Instance", "GA", "Hbp",
    "Batch", "Model", "LearnParams", "EXPORTS", "MLP_PARAMS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmp.so")

PMP_OK, PMP_EINVAL, PMP_ENOMEM, PMP_EDEVICE, PMP_EINFEASIBLE, PMP_EUNSUPPORTED = range(6)
PMP_ON_DEVICE = 1
PMP_ASYNC = 2
PMP_EVAL_PER_CHROMOSOME = 4
PMP_EVAL_PER_CLIENT = 8
PMP_NOALLOC_CELLS = 1 << 19
EVAL_SCHEMES = {"tiled": 0, "per_chromosome": PMP_EVAL_PER_CHROMOSOME,
                "per_client": PMP_EVAL_PER_CLIENT}

EXPORTS = [
    "pmp_preprocess", "pmp_instance_info", "pmp_instance_tables",
    "pmp_eval_population", "pmp_instance_check", "pmp_instance_destroy",
    "pmp_ga_create", "pmp_ga_step", "pmp_ga_best", "pmp_ga_state",
    "pmp_ga_destroy", "pmp_solve", "pmp_ga_profile", "pmp_ga_profile_read",
    "pmp_status_str", "pmp_last_error", "pmp_ga_autotune", "pmp_batch_create",
    "pmp_batch_step", "pmp_batch_check", "pmp_batch_destroy", "pmp_ga_step_batch",
    "pmp_features", "pmp_model_create", "pmp_model_get", "pmp_model_set",
    "pmp_model_forward", "pmp_model_grad", "pmp_model_train", "pmp_model_destroy",
    "pmp_ga_set_model", "pmp_ga_replay", "pmp_exhaustive", "pmp_apsp",
    "pmp_hbp_reduce", "pmp_hbp_info", "pmp_hbp_terms", "pmp_hbp_eval", "pmp_hbp_destroy",
    "pmp_eval_population_noalloc", "pmp_batch_profile", "pmp_batch_profile_read",
    "pmp_batch_autotune",
]

FEATURES = 16
MLP_INPUTS = 32
MLP_PARAMS = 20865


class PmpError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class GaParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("population", C.c_int32),
                ("group_size", C.c_int32), ("generations", C.c_int32),
                ("saturation", C.c_int32), ("crossover_iters", C.c_int32),
                ("mutation_iters", C.c_int32), ("migration", C.c_int32),
                ("init", C.c_int32)]


class GaStats(C.Structure):
    _fields_ = [(name, C.c_int64) for name in (
        "generations", "saturation_count", "done", "best_cost",
        "chromosome_evals", "crossover_fail", "crossover_taken",
        "mutation_taken", "scan_total", "pair_evals", "swap_tried",
        "swap_taken", "speculative_evals")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class LearnParams(C.Structure):
    _fields_ = [("candidates", C.c_int32), ("learned_iters", C.c_int32),
                ("explore_permille", C.c_int32), ("history", C.c_int32),
                ("train_every", C.c_int32), ("lr", C.c_float),
                ("reserved", C.c_int32 * 2)]


class Profile(C.Structure):
    _fields_ = [("eval_ms", C.c_double), ("eval_launches", C.c_int64),
                ("eval_bytes", C.c_int64), ("eval_pairs", C.c_int64)]


_lib = None
_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_u32 = C.c_uint32


def lib():
    """Load libpmp.so (built in place by build.py); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python paper_1610_10061_amd/build.py` (there is no fallback)")
    L = C.CDLL(LIB_PATH)
    L.pmp_preprocess.argtypes = [_vp, _i64, _i32, _i32, _i32, _u32, _vp, C.POINTER(_vp)]
    L.pmp_instance_info.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.pmp_instance_tables.argtypes = [_vp, _vp, _vp, _vp, _u32, _vp]
    L.pmp_eval_population.argtypes = [_vp, _vp, _i32, _vp, _vp, _u32, _vp]
    L.pmp_eval_population_noalloc.argtypes = [_vp, _vp, _i32, _vp, _vp, _u32, _vp]
    L.pmp_instance_check.argtypes = [_vp, _vp]
    L.pmp_instance_destroy.argtypes = [_vp]
    L.pmp_instance_destroy.restype = None
    L.pmp_ga_create.argtypes = [_vp, C.POINTER(GaParams), C.POINTER(_vp)]
    L.pmp_ga_step.argtypes = [_vp, _i32, _vp]
    L.pmp_ga_best.argtypes = [_vp, _vp, C.POINTER(_i64), C.POINTER(GaStats), _vp]
    L.pmp_ga_state.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.pmp_ga_destroy.argtypes = [_vp]
    L.pmp_ga_destroy.restype = None
    L.pmp_solve.argtypes = [_vp, _i32, _i32, _i32, C.POINTER(GaParams), _vp,
                            C.POINTER(_i64), C.POINTER(GaStats)]
    L.pmp_ga_profile.argtypes = [_vp, _i32]
    L.pmp_ga_profile_read.argtypes = [_vp, C.POINTER(Profile), _vp]
    L.pmp_ga_autotune.argtypes = [_vp, C.POINTER(_i32), C.POINTER(_i32), _vp]
    L.pmp_batch_create.argtypes = [C.POINTER(_vp), _i32, C.POINTER(_vp)]
    L.pmp_batch_step.argtypes = [_vp, _i32, _vp]
    L.pmp_batch_check.argtypes = [_vp, C.POINTER(_i32), _vp]
    L.pmp_batch_autotune.argtypes = [_vp, C.POINTER(_i32), _vp]
    L.pmp_batch_destroy.argtypes = [_vp]
    L.pmp_batch_destroy.restype = None
    L.pmp_batch_profile.argtypes = [_vp, _i32]
    L.pmp_batch_profile_read.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(_i64), _vp]
    L.pmp_ga_step_batch.argtypes = [C.POINTER(_vp), _i32, _i32, _vp]
    L.pmp_features.argtypes = [_vp, _vp, _i32, C.c_float, _vp, _u32, _vp]
    L.pmp_model_create.argtypes = [C.c_uint64, C.POINTER(_vp)]
    L.pmp_model_get.argtypes = [_vp, _vp, _u32, _vp]
    L.pmp_model_set.argtypes = [_vp, _vp, _u32, _vp]
    L.pmp_model_forward.argtypes = [_vp, _vp, _i32, _vp, _u32, _vp]
    L.pmp_model_grad.argtypes = [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _u32, _vp]
    L.pmp_model_train.argtypes = [_vp, _vp, _vp, _vp, _i32, C.c_float, _i32, _vp, _u32,
                                  _vp]
    L.pmp_model_destroy.argtypes = [_vp]
    L.pmp_model_destroy.restype = None
    L.pmp_ga_set_model.argtypes = [_vp, _vp, C.POINTER(LearnParams)]
    L.pmp_ga_replay.argtypes = [_vp, C.POINTER(_i32), _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.pmp_exhaustive.argtypes = [_vp, _vp, C.POINTER(_i64), C.POINTER(_i64), _vp]
    L.pmp_apsp.argtypes = [_vp, _i64, _i32, _vp, _i64, _u32, _vp]
    L.pmp_hbp_reduce.argtypes = [_vp, _vp, C.POINTER(_vp)]
    L.pmp_hbp_info.argtypes = [_vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i32),
                               C.POINTER(_i32)]
    L.pmp_hbp_terms.argtypes = [_vp, _vp, _vp, _vp, _vp, _u32, _vp]
    L.pmp_hbp_eval.argtypes = [_vp, _vp, _i32, _vp, _vp, _u32, _vp]
    L.pmp_hbp_destroy.argtypes = [_vp]
    L.pmp_hbp_destroy.restype = None
    L.pmp_status_str.argtypes = [_i32]
    L.pmp_status_str.restype = C.c_char_p
    L.pmp_last_error.argtypes = []
    L.pmp_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("pmp_instance_destroy", "pmp_ga_destroy", "pmp_model_destroy",
                        "pmp_batch_destroy", "pmp_status_str", "pmp_last_error"):
            getattr(L, name).restype = _i32
    _lib = L
    return L


def _check(status: int, where: str):
    if status != PMP_OK:
        detail = lib().pmp_last_error().decode(errors="replace")
        raise PmpError(status, where, detail)


def _stream(stream):
    if stream is None:
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return _vp(stream.cuda_stream)
    return _vp(int(stream))


def _buf(x, dtype_np, dtype_t):
    """(pointer, on_device) for a numpy array or a CUDA tensor."""
    if x is None:
        return None, None
    if isinstance(x, torch.Tensor):
        if not x.is_cuda or not x.is_contiguous() or x.dtype != dtype_t:
            raise ValueError(f"need a contiguous CUDA {dtype_t} tensor")
        return _vp(x.data_ptr()), True
    if not (isinstance(x, np.ndarray) and x.dtype == dtype_np and x.flags.c_contiguous):
        raise ValueError(f"need a C-contiguous numpy {dtype_np} array")
    return x.ctypes.data_as(_vp), False


# --------------------------------------------------------------- C names
def pmp_preprocess(d, p: int, stream=None, asynchronous=False):
    """Section 2.1 tables of d (n x m int32, numpy or CUDA tensor);
    asynchronous (CUDA tensors only): returns before the tables are made, its
    errors reported by pmp_instance_check."""
    ptr, dev = _buf(d, np.int32, torch.int32)
    n, m = d.shape
    out = _vp()
    flags = PMP_ON_DEVICE if dev else 0
    if asynchronous:
        flags |= PMP_ASYNC
    _check(lib().pmp_preprocess(ptr, m, n, m, p, flags,
                                _stream(stream) if dev else None, C.byref(out)),
           "pmp_preprocess")
    return out


def pmp_instance_info(inst):
    v = [_i32() for _ in range(5)]
    _check(lib().pmp_instance_info(inst, *[C.byref(x) for x in v]), "pmp_instance_info")
    return tuple(x.value for x in v)  # n, m, p, K, W


def pmp_instance_tables(inst):
    n, m, p, K, W = pmp_instance_info(inst)
    pi = np.zeros((n, K), np.uint16)
    de = np.zeros((n, K), np.int32)
    ds = np.zeros((n, K), np.int32)
    _check(lib().pmp_instance_tables(inst, pi.ctypes.data_as(_vp), de.ctypes.data_as(_vp),
                                     ds.ctypes.data_as(_vp), 0, None), "pmp_instance_tables")
    return pi, de, ds


def pmp_eval_population(inst, masks, fitness, scan_total=None, stream=None,
                        asynchronous=False, scheme="tiled"):
    """Eq. (6) for every row of masks (P x W uint64) into fitness (P int64).
    scheme: "tiled" (default), "per_chromosome" or "per_client" (the thread
    mappings the paper compares; same results)."""
    mp, dev = _buf(masks, np.uint64, torch.uint64)
    fp, fdev = _buf(fitness, np.int64, torch.int64)
    sp, sdev = _buf(scan_total, np.int64, torch.int64)
    if fdev != dev or (sp is not None and sdev != dev):
        raise ValueError("all buffers must be host arrays or all CUDA tensors")
    P = masks.shape[0]
    flags = (PMP_ON_DEVICE | (PMP_ASYNC if asynchronous else 0)) if dev else 0
    flags |= EVAL_SCHEMES[scheme]
    _check(lib().pmp_eval_population(inst, mp, P, fp, sp, flags,
                                     _stream(stream) if dev else None),
           "pmp_eval_population")


def pmp_eval_population_noalloc(inst, masks, fitness, scan_total=None, stream=None,
                                asynchronous=False):
    """pmp_eval_population on CUDA tensors without any allocation: the
    library's fixed workspace holds the partial sums (P up to
    PMP_NOALLOC_CELLS; calls on one GPU must not overlap)."""
    mp, dev = _buf(masks, np.uint64, torch.uint64)
    fp, fdev = _buf(fitness, np.int64, torch.int64)
    sp, sdev = _buf(scan_total, np.int64, torch.int64)
    if not dev or not fdev or (sp is not None and not sdev):
        raise ValueError("pmp_eval_population_noalloc takes CUDA tensors only")
    flags = PMP_ON_DEVICE | (PMP_ASYNC if asynchronous else 0)
    _check(lib().pmp_eval_population_noalloc(inst, mp, masks.shape[0], fp, sp, flags,
                                             _stream(stream)),
           "pmp_eval_population_noalloc")


def pmp_apsp(w, d=None, stream=None):
    """Shortest path lengths of the graph with arc weights w (n x n int32,
    negative = no arc; numpy or CUDA tensor) into d (same kind; allocated
    when None); -1 where there is no path.  Returns d."""
    n = w.shape[0]
    if w.shape != (n, n):
        raise ValueError("w must be square")
    if d is None:
        d = (torch.empty((n, n), dtype=torch.int32, device=w.device)
             if isinstance(w, torch.Tensor) else np.empty((n, n), np.int32))
    wp, wdev = _buf(w, np.int32, torch.int32)
    dp, ddev = _buf(d, np.int32, torch.int32)
    if wdev != ddev:
        raise ValueError("w and d must both be host arrays or both CUDA tensors")
    _check(lib().pmp_apsp(wp, n, n, dp, n, PMP_ON_DEVICE if wdev else 0,
                          _stream(stream) if wdev else None), "pmp_apsp")
    return d


def pmp_hbp_reduce(inst, stream=None):
    """The reduced polynomial of an instance (a handle)."""
    out = _vp()
    _check(lib().pmp_hbp_reduce(inst, _stream(stream), C.byref(out)), "pmp_hbp_reduce")
    return out


def pmp_hbp_info(h):
    c, t = _i64(), _i64()
    r, k = _i32(), _i32()
    _check(lib().pmp_hbp_info(h, C.byref(c), C.byref(t), C.byref(r), C.byref(k)),
           "pmp_hbp_info")
    return c.value, t.value, r.value, k.value  # constant, monomials, rows, max_len


def pmp_hbp_terms(h, n):
    """(row, degree, coefficient) arrays of the monomials and K_i of the n
    client rows."""
    _, T, _, _ = pmp_hbp_info(h)
    row = np.zeros(T, np.int32)
    deg = np.zeros(T, np.int32)
    coef = np.zeros(T, np.int64)
    rl = np.zeros(n, np.int32)
    _check(lib().pmp_hbp_terms(h, row.ctypes.data_as(_vp), deg.ctypes.data_as(_vp),
                               coef.ctypes.data_as(_vp), rl.ctypes.data_as(_vp), 0, None),
           "pmp_hbp_terms")
    return row, deg, coef, rl


def pmp_hbp_eval(h, masks, fitness, scan_total=None, stream=None, asynchronous=False):
    """The reduced polynomial at every row of masks into fitness."""
    mp, dev = _buf(masks, np.uint64, torch.uint64)
    fp, fdev = _buf(fitness, np.int64, torch.int64)
    sp, sdev = _buf(scan_total, np.int64, torch.int64)
    if fdev != dev or (sp is not None and sdev != dev):
        raise ValueError("all buffers must be host arrays or all CUDA tensors")
    flags = (PMP_ON_DEVICE | (PMP_ASYNC if asynchronous else 0)) if dev else 0
    _check(lib().pmp_hbp_eval(h, mp, masks.shape[0], fp, sp, flags,
                              _stream(stream) if dev else None), "pmp_hbp_eval")


def pmp_hbp_destroy(h):
    lib().pmp_hbp_destroy(h)


def pmp_instance_check(inst, stream=None):
    _check(lib().pmp_instance_check(inst, _stream(stream)), "pmp_instance_check")


def pmp_instance_destroy(inst):
    lib().pmp_instance_destroy(inst)


def pmp_ga_create(inst, population, group_size, generations, seed,
                  saturation=0, crossover_iters=0, mutation_iters=0, migration=0, init=0):
    prm = GaParams(seed, population, group_size, generations, saturation,
                   crossover_iters, mutation_iters, migration, init)
    out = _vp()
    _check(lib().pmp_ga_create(inst, C.byref(prm), C.byref(out)), "pmp_ga_create")
    return out


def pmp_ga_step(ga, generations, stream=None):
    _check(lib().pmp_ga_step(ga, generations, _stream(stream)), "pmp_ga_step")


def pmp_ga_best(ga, W, stream=None):
    mask = np.zeros(W, np.uint64)
    cost = _i64()
    st = GaStats()
    _check(lib().pmp_ga_best(ga, mask.ctypes.data_as(_vp), C.byref(cost),
                             C.byref(st), _stream(stream)), "pmp_ga_best")
    return mask, cost.value, st.as_dict()


def pmp_ga_state(ga, P, NB, W, stream=None):
    pop = np.zeros((P, W), np.uint64)
    fit = np.zeros(P, np.int64)
    gm = np.zeros((NB, W), np.uint64)
    gc = np.zeros(NB, np.int64)
    _check(lib().pmp_ga_state(ga, pop.ctypes.data_as(_vp), fit.ctypes.data_as(_vp),
                              gm.ctypes.data_as(_vp), gc.ctypes.data_as(_vp),
                              _stream(stream)), "pmp_ga_state")
    return pop, fit, gm, gc


def pmp_ga_destroy(ga):
    lib().pmp_ga_destroy(ga)


def pmp_ga_profile(ga, enable: bool):
    _check(lib().pmp_ga_profile(ga, 1 if enable else 0), "pmp_ga_profile")


def pmp_ga_profile_read(ga, stream=None):
    pr = Profile()
    _check(lib().pmp_ga_profile_read(ga, C.byref(pr), _stream(stream)),
           "pmp_ga_profile_read")
    return {"eval_ms": pr.eval_ms, "eval_launches": pr.eval_launches,
            "eval_bytes": pr.eval_bytes, "eval_pairs": pr.eval_pairs}


def pmp_solve(d, p, population, group_size, generations, seed, saturation=0,
              crossover_iters=0, mutation_iters=0, migration=0, init=0):
    d = np.ascontiguousarray(d, dtype=np.int32)
    n, m = d.shape
    prm = GaParams(seed, population, group_size, generations, saturation,
                   crossover_iters, mutation_iters, migration, init)
    open_ = np.zeros(m, np.uint8)
    cost = _i64()
    st = GaStats()
    _check(lib().pmp_solve(d.ctypes.data_as(_vp), n, m, p, C.byref(prm),
                           open_.ctypes.data_as(_vp), C.byref(cost), C.byref(st)),
           "pmp_solve")
    return open_, cost.value, st.as_dict()


def pmp_ga_autotune(ga, stream=None):
    """Returns (clients per workgroup, waves per workgroup)."""
    out, wv = _i32(), _i32()
    _check(lib().pmp_ga_autotune(ga, C.byref(out), C.byref(wv), _stream(stream)),
           "pmp_ga_autotune")
    return out.value, wv.value


def _handles(gas):
    arr = (_vp * len(gas))(*[g.value if isinstance(g, _vp) else g for g in gas])
    return arr


def pmp_batch_create(gas):
    out = _vp()
    _check(lib().pmp_batch_create(_handles(gas), len(gas), C.byref(out)),
           "pmp_batch_create")
    return out


def pmp_batch_step(batch, generations, stream=None):
    _check(lib().pmp_batch_step(batch, generations, _stream(stream)), "pmp_batch_step")


def pmp_batch_check(batch, stream=None):
    grid = _i32()
    _check(lib().pmp_batch_check(batch, C.byref(grid), _stream(stream)), "pmp_batch_check")
    return grid.value


def pmp_batch_autotune(batch, stream=None):
    """Time the batch evaluation's client tilings; returns the chosen common
    count of clients per workgroup (0: every run keeps its own tuning)."""
    clients = _i32()
    _check(lib().pmp_batch_autotune(batch, C.byref(clients), _stream(stream)),
           "pmp_batch_autotune")
    return clients.value


def pmp_batch_destroy(batch):
    lib().pmp_batch_destroy(batch)


def pmp_batch_profile(batch, enable: bool):
    _check(lib().pmp_batch_profile(batch, 1 if enable else 0), "pmp_batch_profile")


def pmp_batch_profile_read(batch, stream=None):
    """(milliseconds, launches) of the batch evaluation launches since the
    last enable or read."""
    ms = C.c_double()
    n = _i64()
    _check(lib().pmp_batch_profile_read(batch, C.byref(ms), C.byref(n), _stream(stream)),
           "pmp_batch_profile_read")
    return ms.value, n.value


def pmp_ga_step_batch(gas, generations, stream=None):
    _check(lib().pmp_ga_step_batch(_handles(gas), len(gas), generations, _stream(stream)),
           "pmp_ga_step_batch")


def _same_side(*bufs):
    """All given (pointer, on_device) pairs on one side; returns on_device."""
    sides = {dev for ptr, dev in bufs if ptr is not None}
    if len(sides) > 1:
        raise ValueError("all buffers must be host arrays or all CUDA tensors")
    return sides.pop() if sides else False


def pmp_features(inst, masks, gen_frac=0.0, out=None, stream=None):
    """The 16 features of every facility of every chromosome: P x m x 16."""
    n, m, p, K, W = pmp_instance_info(inst)
    P = masks.shape[0]
    if out is None:
        out = (torch.empty((P, m, FEATURES), dtype=torch.float32, device=masks.device)
               if isinstance(masks, torch.Tensor) else np.zeros((P, m, FEATURES), np.float32))
    mb = _buf(masks, np.uint64, torch.uint64)
    ob = _buf(out, np.float32, torch.float32)
    dev = _same_side(mb, ob)
    _check(lib().pmp_features(inst, mb[0], P, float(gen_frac), ob[0],
                              PMP_ON_DEVICE if dev else 0, _stream(stream) if dev else None),
           "pmp_features")
    return out


def pmp_model_create(seed=0):
    out = _vp()
    _check(lib().pmp_model_create(seed, C.byref(out)), "pmp_model_create")
    return out


def pmp_model_get(model, params=None, stream=None):
    if params is None:
        params = np.zeros(MLP_PARAMS, np.float32)
    pb = _buf(params, np.float32, torch.float32)
    _check(lib().pmp_model_get(model, pb[0], PMP_ON_DEVICE if pb[1] else 0,
                               _stream(stream) if pb[1] else None), "pmp_model_get")
    return params


def pmp_model_set(model, params, stream=None):
    pb = _buf(params, np.float32, torch.float32)
    _check(lib().pmp_model_set(model, pb[0], PMP_ON_DEVICE if pb[1] else 0,
                               _stream(stream) if pb[1] else None), "pmp_model_set")


def pmp_model_forward(model, x, y=None, stream=None):
    """Scores of rows x (rows x 32 float32)."""
    rows = x.shape[0]
    if y is None:
        y = (torch.empty(rows, dtype=torch.float32, device=x.device)
             if isinstance(x, torch.Tensor) else np.zeros(rows, np.float32))
    xb, yb = _buf(x, np.float32, torch.float32), _buf(y, np.float32, torch.float32)
    dev = _same_side(xb, yb)
    _check(lib().pmp_model_forward(model, xb[0], rows, yb[0], PMP_ON_DEVICE if dev else 0,
                                   _stream(stream) if dev else None), "pmp_model_forward")
    return y


def pmp_model_grad(model, x, t, w=None, stream=None):
    """(gradient, loss) of rows (x, t, w) on the host."""
    rows = x.shape[0]
    grad = np.zeros(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    xb, tb = _buf(x, np.float32, torch.float32), _buf(t, np.float32, torch.float32)
    wb = _buf(w, np.float32, torch.float32)
    if _same_side(xb, tb, wb):
        raise ValueError("pmp_model_grad binding takes host arrays")
    _check(lib().pmp_model_grad(model, xb[0], tb[0], wb[0], rows, grad.ctypes.data_as(_vp),
                                loss.ctypes.data_as(_vp), 0, None), "pmp_model_grad")
    return grad, float(loss[0])


def pmp_model_train(model, x, t, w=None, lr=1e-3, steps=1, stream=None):
    """`steps` Adam steps on host rows; returns the loss before the last."""
    rows = x.shape[0]
    loss = np.zeros(1, np.float32)
    xb, tb = _buf(x, np.float32, torch.float32), _buf(t, np.float32, torch.float32)
    wb = _buf(w, np.float32, torch.float32)
    if _same_side(xb, tb, wb):
        raise ValueError("pmp_model_train binding takes host arrays")
    _check(lib().pmp_model_train(model, xb[0], tb[0], wb[0], rows, float(lr), steps,
                                 loss.ctypes.data_as(_vp), 0, None), "pmp_model_train")
    return float(loss[0])


def pmp_model_destroy(model):
    lib().pmp_model_destroy(model)


def pmp_ga_set_model(ga, model, candidates=0, learned_iters=0, explore_permille=0,
                     history=0, train_every=0, lr=0.0):
    prm = LearnParams(candidates, learned_iters, explore_permille, history, train_every,
                      lr)
    _check(lib().pmp_ga_set_model(ga, model, C.byref(prm)), "pmp_ga_set_model")


def pmp_ga_replay(ga, population, candidates, stream=None):
    """The training ring: dict of x (rows x 32 uint16 BF16 bits), target,
    weight, swap (rows x 2), delta (rows x 2: change, parent cost), and the
    last generation's candidate scores (population x candidates)."""
    rows = _i32()
    _check(lib().pmp_ga_replay(ga, C.byref(rows), None, None, None, None, None, None,
                               _stream(stream)), "pmp_ga_replay")
    R = rows.value
    out = {"x": np.zeros((R, MLP_INPUTS), np.uint16), "target": np.zeros(R, np.float32),
           "weight": np.zeros(R, np.float32), "swap": np.zeros((R, 2), np.int32),
           "delta": np.zeros((R, 2), np.int64),
           "scores": np.zeros((population, candidates), np.float32)}
    _check(lib().pmp_ga_replay(ga, C.byref(rows), *[out[k].ctypes.data_as(_vp) for k in
                                                     ("x", "target", "weight", "swap",
                                                      "delta", "scores")], _stream(stream)),
           "pmp_ga_replay")
    return out


def pmp_exhaustive(inst, stream=None):
    """(best cost, best mask (W words), C(m, p)) by GPU enumeration."""
    n, m, p, K, W = pmp_instance_info(inst)
    mask = np.zeros(W, np.uint64)
    cost, cnt = _i64(), _i64()
    _check(lib().pmp_exhaustive(inst, mask.ctypes.data_as(_vp), C.byref(cost), C.byref(cnt),
                                _stream(stream)), "pmp_exhaustive")
    return cost.value, mask, cnt.value


# ------------------------------------------------------- small conveniences
class Instance:
    """Owning wrapper of a pmp_instance handle."""

    def __init__(self, d, p: int, stream=None, asynchronous=False):
        self.handle = pmp_preprocess(d, p, stream, asynchronous)
        self.n, self.m, self.p, self.K, self.W = pmp_instance_info(self.handle)

    def tables(self):
        return pmp_instance_tables(self.handle)

    def eval(self, masks, fitness=None, scan_total=None, stream=None,
             asynchronous=False):
        if fitness is None:
            if isinstance(masks, torch.Tensor):
                fitness = torch.empty(masks.shape[0], dtype=torch.int64,
                                      device=masks.device)
            else:
                fitness = np.zeros(masks.shape[0], np.int64)
        pmp_eval_population(self.handle, masks, fitness, scan_total, stream,
                            asynchronous)
        return fitness

    def check(self, stream=None):
        pmp_instance_check(self.handle, stream)

    def close(self):
        if self.handle:
            pmp_instance_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hbp:
    """Owning wrapper of a reduced-polynomial handle (its instance must stay
    open while it is used)."""

    def __init__(self, inst: "Instance", stream=None):
        self.inst = inst
        self.handle = pmp_hbp_reduce(inst.handle, stream)

    def info(self):
        """(constant, monomials, kept rows, longest kept row)."""
        return pmp_hbp_info(self.handle)

    def terms(self):
        return pmp_hbp_terms(self.handle, pmp_instance_info(self.inst.handle)[0])

    def eval(self, masks, fitness=None, scan_total=None, stream=None, asynchronous=False):
        if fitness is None:
            if isinstance(masks, torch.Tensor):
                fitness = torch.empty(masks.shape[0], dtype=torch.int64, device=masks.device)
            else:
                fitness = np.zeros(masks.shape[0], np.int64)
        pmp_hbp_eval(self.handle, masks, fitness, scan_total, stream, asynchronous)
        return fitness

    def close(self):
        if self.handle:
            pmp_hbp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GA:
    """Owning wrapper of a pmp_ga handle (the instance must outlive it)."""

    def __init__(self, inst: Instance, population, group_size, generations,
                 seed, saturation=0, crossover_iters=0, mutation_iters=0, migration=0,
                 init=0):
        self.inst = inst
        self.P, self.NT = population, group_size
        self.NB = population // group_size
        self.handle = pmp_ga_create(inst.handle, population, group_size,
                                    generations, seed, saturation,
                                    crossover_iters, mutation_iters, migration, init)

    def step(self, generations, stream=None):
        pmp_ga_step(self.handle, generations, stream)

    def best(self, stream=None):
        return pmp_ga_best(self.handle, self.inst.W, stream)

    def state(self, stream=None):
        return pmp_ga_state(self.handle, self.P, self.NB, self.inst.W, stream)

    def profile(self, enable=True):
        pmp_ga_profile(self.handle, enable)

    def autotune(self, stream=None):
        return pmp_ga_autotune(self.handle, stream)

    def set_model(self, model, **kw):
        """Attach a Model (keyword arguments: LearnParams fields)."""
        pmp_ga_set_model(self.handle, model.handle if model is not None else None, **kw)
        self.model = model
        self.candidates = (kw.get("candidates") or 64) if model is not None else 0

    def replay(self, stream=None):
        return pmp_ga_replay(self.handle, self.P, self.candidates, stream)

    def profile_read(self, stream=None):
        return pmp_ga_profile_read(self.handle, stream)

    def close(self):
        if self.handle:
            pmp_ga_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owning wrapper of a pmp_batch handle over GA objects (which must
    outlive it)."""

    def __init__(self, gas):
        self.gas = list(gas)
        self.handle = pmp_batch_create([g.handle for g in self.gas])

    def step(self, generations, stream=None):
        pmp_batch_step(self.handle, generations, stream)

    def check(self, stream=None):
        return pmp_batch_check(self.handle, stream)

    def autotune(self, stream=None):
        return pmp_batch_autotune(self.handle, stream)

    def profile(self, enable=True):
        pmp_batch_profile(self.handle, enable)

    def profile_read(self, stream=None):
        return pmp_batch_profile_read(self.handle, stream)

    def close(self):
        if self.handle:
            pmp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """Owning wrapper of a pmp_model handle."""

    def __init__(self, seed=0):
        self.handle = pmp_model_create(seed)

    def params(self):
        return pmp_model_get(self.handle)

    def set_params(self, params):
        pmp_model_set(self.handle, np.ascontiguousarray(params, dtype=np.float32))

    def forward(self, x, y=None, stream=None):
        return pmp_model_forward(self.handle, x, y, stream)

    def grad(self, x, t, w=None):
        return pmp_model_grad(self.handle, x, t, w)

    def train(self, x, t, w=None, lr=1e-3, steps=1):
        return pmp_model_train(self.handle, x, t, w, lr, steps)

    def close(self):
        if self.handle:
            pmp_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
