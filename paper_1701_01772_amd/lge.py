"""Thin Python binding of liblge.so (include/lge.h).

Argument marshalling only: every step of the estimate runs in the HIP
library.  Names mirror the C ABI.  Results come back as dicts with Python
ints for the exact integer fields (``csum``, ``zsum`` signed, ``qsum``,
``exact``; lists indexed by graphlet number 0..17, slot 0 unused) and float
lists for ``estimate``, ``variance``, ``lower95``, ``upper95``.

The library must be built (``python -m paper_1701_01772_amd.build``); there
is no fallback: importing a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblge.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lge.h")

LGE_OK = 0
LGE_EINVAL = -1
LGE_ENOMEM = -2
LGE_EGRAPH = -3
LGE_EDEVICE = -4
LGE_ERANGE = -5
LGE_EBUSY = -6
LGE_ETIMEDOUT = -7
LGE_ECANCELED = -8
LGE_ENOTFOUND = -9
LGE_EINTERNAL = -10
LGE_MICRO_COLS = 17
LGE_WEIGHT_DEGREE = 1
LGE_WEIGHT_KCORE = 2
LGE_WEIGHT_CLASSES = 16
LGE_FLAG_TRUSTED = 1
LGE_FLAG_COMPACT = 2
LGE_FLAG_NO_TABLES = 4
LGE_OPT_SORT_HUB = 1
LGE_OPT_XCD_LOCAL = 2


class LgeError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, lge_strerror(code), code))


class U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64), ("p", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("sampled_edges", ctypes.c_uint64),
        ("csum", U128 * 18), ("z", U128 * 18), ("q", U128 * 18), ("exact", U128 * 18),
        ("estimate", ctypes.c_double * 18), ("variance", ctypes.c_double * 18),
        ("lower95", ctypes.c_double * 18), ("upper95", ctypes.c_double * 18),
    ]


class Opts(ctypes.Structure):
    _fields_ = [("wave_max_deg", ctypes.c_int32), ("block_max_deg", ctypes.c_int32),
                ("probe_ratio", ctypes.c_int32), ("grid_per_cu", ctypes.c_int32),
                ("global_chunk", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("max_list_mib", ctypes.c_int32), ("grid_share", ctypes.c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_float), ("sample_ms", ctypes.c_float), ("count_ms", ctypes.c_float * 3),
                ("global_prep_ms", ctypes.c_float),
                ("class_edges", ctypes.c_uint64 * 3), ("words_read", ctypes.c_uint64 * 3),
                ("launches", ctypes.c_uint64), ("micro_ms", ctypes.c_float), ("host_waits", ctypes.c_uint32),
                ("alg_bytes", ctypes.c_uint64 * 3)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("max_deg", ctypes.c_int32), ("ranked", ctypes.c_int32),
                ("rows", ctypes.c_int32), ("rows_floor", ctypes.c_int32), ("rows_width", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("state_bytes", ctypes.c_uint64), ("build_ms", ctypes.c_double)]


class WeightInfo(ctypes.Structure):
    _fields_ = [("p_level", ctypes.c_double * 16), ("edges", ctypes.c_uint64 * 16),
                ("sampled", ctypes.c_uint64 * 16), ("max_core", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32),
                ("vtx_off", ctypes.POINTER(ctypes.c_int64)), ("nnz_off", ctypes.POINTER(ctypes.c_int64)),
                ("row_ptr", ctypes.POINTER(ctypes.c_int32)), ("col", ctypes.POINTER(ctypes.c_int32)),
                ("p", ctypes.POINTER(ctypes.c_double)), ("seed", ctypes.POINTER(ctypes.c_uint64)),
                ("flags", ctypes.c_uint32)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("min_chunk_edges", ctypes.c_int64),
                ("target_step_us", ctypes.c_int64), ("workers", ctypes.c_int32), ("short_us", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("canceled", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("steps", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("running", ctypes.c_uint64), ("busy_s", ctypes.c_double), ("workspace_bytes", ctypes.c_uint64)]


class AdaptiveCfg(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("t_max", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("phi0", ctypes.c_double)]


class AdaptiveTrace(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("pad", ctypes.c_int32), ("p", ctypes.c_double * 64),
                ("delta", ctypes.c_double * 64), ("sampled", ctypes.c_uint64 * 64)]


_lib = None
_VP = ctypes.c_void_p


def load():
    """Load liblge.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblge.so is not built (%s); run `python -m paper_1701_01772_amd.build`" % LIB_PATH)
    # PyTorch-ROCm ships its own HIP/HSA runtime under the same sonames as the
    # system one.  Loading torch first makes liblge.so bind to that already
    # loaded runtime, so the process has one runtime and device pointers and
    # streams from torch are valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "lge_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "lge_opts_default": ([ctypes.POINTER(Opts)], ctypes.c_int),
        "lge_open": ([ctypes.c_int, ctypes.POINTER(_VP)], ctypes.c_int),
        "lge_close": ([_VP], ctypes.c_int),
        "lge_validate_csr_host": ([ctypes.c_int64, i32p, i32p], ctypes.c_int),
        "lge_graph_create_host": ([_VP, ctypes.c_int64, i32p, i32p, ctypes.c_uint32, ctypes.POINTER(_VP)],
                                  ctypes.c_int),
        "lge_graph_create_device": ([_VP, ctypes.c_int64, _VP, _VP, _VP, ctypes.c_uint32, ctypes.POINTER(_VP)],
                                    ctypes.c_int),
        "lge_graph_destroy": ([_VP], ctypes.c_int),
        "lge_graph_n": ([_VP], ctypes.c_int64),
        "lge_graph_m": ([_VP], ctypes.c_int64),
        "lge_estimate": ([_VP, _VP, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(Opts), ctypes.POINTER(Result)],
                         ctypes.c_int),
        "lge_estimate_noalloc": ([_VP, _VP, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(Result)], ctypes.c_int),
        "lge_graph_query": ([_VP, ctypes.POINTER(GraphInfo)], ctypes.c_int),
        "lge_estimate_range": ([_VP, _VP, ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                ctypes.POINTER(Opts), ctypes.POINTER(Result)], ctypes.c_int),
        "lge_estimate_async": ([_VP, _VP, ctypes.c_double, ctypes.c_uint64, _VP, ctypes.POINTER(Result),
                                ctypes.POINTER(_VP)], ctypes.c_int),
        "lge_event_wait": ([_VP], ctypes.c_int),
        "lge_count_batch": ([_VP, ctypes.POINTER(Batch), ctypes.POINTER(Opts), ctypes.POINTER(Result)], ctypes.c_int),
        "lge_estimate_many": ([_VP, ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32, ctypes.POINTER(Opts),
                               ctypes.POINTER(Result)], ctypes.c_int),
        "lge_last_timing": ([_VP, ctypes.POINTER(Timing)], ctypes.c_int),
        "lge_autotune": ([_VP, _VP, ctypes.c_double, ctypes.POINTER(Opts)], ctypes.c_int),
        "lge_autotune_reset": ([_VP], ctypes.c_int),
        "lge_set_table_budget": ([_VP, ctypes.c_uint64, ctypes.c_uint64], ctypes.c_int),
        "lge_set_build_scratch": ([_VP, ctypes.c_uint64], ctypes.c_int),
        "lge_adaptive_cfg_default": ([ctypes.POINTER(AdaptiveCfg)], ctypes.c_int),
        "lge_estimate_adaptive": ([_VP, _VP, ctypes.c_uint64, ctypes.POINTER(AdaptiveCfg), ctypes.POINTER(Result),
                                   ctypes.POINTER(AdaptiveTrace)], ctypes.c_int),
        "lge_micro": ([_VP, _VP, ctypes.c_int64, ctypes.c_int64, _VP, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "lge_estimate_weighted": ([_VP, _VP, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(Opts),
                                   ctypes.POINTER(Result), ctypes.POINTER(WeightInfo)], ctypes.c_int),
        "lge_core_numbers": ([_VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "lge_estimate_fixed_k": ([_VP, _VP, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(Opts),
                                  ctypes.POINTER(Result)], ctypes.c_int),
        "lge_server_cfg_default": ([ctypes.POINTER(ServerCfg)], ctypes.c_int),
        "lge_server_create": ([_VP, ctypes.POINTER(ServerCfg), ctypes.POINTER(_VP)], ctypes.c_int),
        "lge_server_add_graph": ([_VP, _VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "lge_submit": ([_VP, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)],
                       ctypes.c_int),
        "lge_wait": ([_VP, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(Result)], ctypes.c_int),
        "lge_cancel": ([_VP, ctypes.c_uint64], ctypes.c_int),
        "lge_server_get_stats": ([_VP, ctypes.POINTER(ServerStats)], ctypes.c_int),
        "lge_server_destroy": ([_VP], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def header_symbols():
    """Every function the public header declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^LGE_API\s+[\w\s\*]*?\b(lge_\w+)\(", txt, flags=re.M)))


def _check(rc: int, where: str):
    if rc != LGE_OK:
        raise LgeError(rc, where)


def lge_strerror(code: int) -> str:
    return load().lge_strerror(code).decode()


def lge_opts_default() -> Opts:
    o = Opts()
    _check(load().lge_opts_default(ctypes.byref(o)), "lge_opts_default")
    return o


def make_opts(**kw) -> Opts:
    o = lge_opts_default()
    for k, v in kw.items():
        setattr(o, k, int(v))
    return o


def opts_dict(o: Opts) -> dict:
    """The tuning fields of an Opts as a plain dict."""
    return {k: getattr(o, k) for k, _ in Opts._fields_}


def lge_open(device: int = 0):
    ctx = _VP()
    _check(load().lge_open(device, ctypes.byref(ctx)), "lge_open")
    return ctx


def lge_close(ctx):
    _check(load().lge_close(ctx), "lge_close")


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a


def lge_validate_csr_host(row_ptr, col) -> int:
    rp, cl = _i32(row_ptr), _i32(col)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    return load().lge_validate_csr_host(rp.shape[0] - 1, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


def lge_graph_create_host(ctx, row_ptr, col, flags: int = 0):
    rp, cl = _i32(row_ptr), _i32(col)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    g = _VP()
    _check(load().lge_graph_create_host(ctx, rp.shape[0] - 1, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), flags, ctypes.byref(g)),
           "lge_graph_create_host")
    return g


def lge_graph_create_device(ctx, n: int, row_ptr_ptr: int, col_ptr: int, stream_ptr: int = 0, flags: int = 0):
    """Adopt device buffers (e.g. ``tensor.data_ptr()`` of int32 tensors)."""
    g = _VP()
    _check(load().lge_graph_create_device(ctx, n, _VP(row_ptr_ptr), _VP(col_ptr), _VP(stream_ptr or None), flags,
                                          ctypes.byref(g)), "lge_graph_create_device")
    return g


def lge_graph_destroy(g):
    _check(load().lge_graph_destroy(g), "lge_graph_destroy")


def _u(x) -> int:
    return (int(x.hi) << 64) | int(x.lo)


def _s(x) -> int:
    v = _u(x)
    return v - (1 << 128) if v >> 127 else v


def result_dict(r: Result) -> dict:
    return {
        "n": r.n, "m": r.m, "p": r.p, "seed": r.seed, "sampled": int(r.sampled_edges),
        "csum": [_u(r.csum[i]) for i in range(18)],
        "zsum": [_s(r.z[i]) for i in range(18)],
        "qsum": [_u(r.q[i]) for i in range(18)],
        "exact": [_u(r.exact[i]) for i in range(18)],
        "estimate": list(r.estimate), "variance": list(r.variance),
        "lower95": list(r.lower95), "upper95": list(r.upper95),
    }


def lge_estimate(ctx, g, p: float, seed: int, opts: Opts | None = None, raw: bool = False,
                 out: Result | None = None):
    """Result as a dict of Python numbers, or (raw=True) the lge_result
    struct itself (``out`` when given), skipping the conversion."""
    r = out if out is not None else Result()
    _check(load().lge_estimate(ctx, g, float(p), int(seed), ctypes.byref(opts) if opts is not None else None,
                               ctypes.byref(r)), "lge_estimate")
    return r if raw else result_dict(r)


def lge_graph_query(g) -> dict:
    i = GraphInfo()
    _check(load().lge_graph_query(g, ctypes.byref(i)), "lge_graph_query")
    return {k: getattr(i, k) for k, _ in GraphInfo._fields_ if k != "pad"}


def lge_estimate_noalloc(ctx, g, p: float, seed: int, raw: bool = False, out: Result | None = None):
    """lge_estimate through the allocation-free entry point (graphs of at
    most 2^18 edges; workspace in the library's fixed device array)."""
    r = out if out is not None else Result()
    _check(load().lge_estimate_noalloc(ctx, g, float(p), int(seed), ctypes.byref(r)), "lge_estimate_noalloc")
    return r if raw else result_dict(r)


def lge_estimate_range(ctx, g, p: float, seed: int, e0: int, e1: int, opts: Opts | None = None) -> dict:
    r = Result()
    _check(load().lge_estimate_range(ctx, g, float(p), int(seed), int(e0), int(e1),
                                     ctypes.byref(opts) if opts is not None else None, ctypes.byref(r)),
           "lge_estimate_range")
    return result_dict(r)


def lge_estimate_async(ctx, g, p: float, seed: int, stream_ptr: int = 0):
    """Returns (event, Result); call lge_event_wait(event) then result_dict."""
    r = Result()
    ev = _VP()
    _check(load().lge_estimate_async(ctx, g, float(p), int(seed), _VP(stream_ptr or None), ctypes.byref(r),
                                     ctypes.byref(ev)), "lge_estimate_async")
    return ev, r


def lge_event_wait(ev):
    _check(load().lge_event_wait(ev), "lge_event_wait")


def pack_batch(graphs):
    """Concatenated CSR arrays (vtx_off, nnz_off, row_ptr, col) of (row_ptr, col) pairs."""
    vtx = [0]
    nnz = [0]
    rps, cols = [], []
    for rp, cl in graphs:
        rp = _i32(rp)
        cl = _i32(cl)
        vtx.append(vtx[-1] + rp.shape[0] - 1)
        nnz.append(nnz[-1] + cl.shape[0])
        rps.append(rp)
        cols.append(cl)
    return (np.asarray(vtx, dtype=np.int64), np.asarray(nnz, dtype=np.int64),
            np.concatenate(rps) if rps else np.zeros(0, np.int32),
            np.concatenate(cols) if cols else np.zeros(0, np.int32))


def lge_count_batch(ctx, graphs, p, seed, flags: int = 0, opts: Opts | None = None):
    """graphs: list of (row_ptr, col); p, seed: scalars or per-graph lists."""
    G = len(graphs)
    vtx, nnz, rp, cl = pack_batch(graphs)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    ps = np.asarray(p if np.ndim(p) else [p] * G, dtype=np.float64)
    ss = np.asarray(seed if np.ndim(seed) else [seed] * G, dtype=np.uint64)
    b = Batch(G, vtx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nnz.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
              rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
              ps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ss.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
              flags)
    outs = (Result * max(G, 1))()
    _check(load().lge_count_batch(ctx, ctypes.byref(b), ctypes.byref(opts) if opts is not None else None, outs),
           "lge_count_batch")
    return [result_dict(outs[i]) for i in range(G)]


def lge_estimate_many(ctx, graphs, p, seed, opts: Opts | None = None, raw: bool = False):
    """graphs: list of graph handles on ctx; p, seed: scalars or per-graph
    lists.  Dicts, or (raw=True) the array of lge_result structs."""
    G = len(graphs)
    arr = (_VP * max(G, 1))(*graphs)
    ps = np.ascontiguousarray(p if np.ndim(p) else [p] * G, dtype=np.float64)
    ss = np.ascontiguousarray(seed if np.ndim(seed) else [seed] * G, dtype=np.uint64)
    outs = (Result * max(G, 1))()
    _check(load().lge_estimate_many(ctx, arr, ps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ss.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), G,
                                    ctypes.byref(opts) if opts is not None else None, outs), "lge_estimate_many")
    return outs if raw else [result_dict(outs[i]) for i in range(G)]


def lge_last_timing(ctx) -> dict:
    t = Timing()
    _check(load().lge_last_timing(ctx, ctypes.byref(t)), "lge_last_timing")
    return {"total_ms": t.total_ms, "sample_ms": t.sample_ms, "count_ms": list(t.count_ms),
            "global_prep_ms": t.global_prep_ms,
            "class_edges": [int(x) for x in t.class_edges], "words_read": [int(x) for x in t.words_read],
            "launches": int(t.launches), "micro_ms": t.micro_ms, "host_waits": int(t.host_waits),
            "alg_bytes": [int(x) for x in t.alg_bytes]}


def lge_autotune(ctx, g, p: float) -> Opts:
    o = Opts()
    _check(load().lge_autotune(ctx, g, float(p), ctypes.byref(o)), "lge_autotune")
    return o


def lge_autotune_reset(ctx):
    _check(load().lge_autotune_reset(ctx), "lge_autotune_reset")


def lge_set_table_budget(ctx, codeg_bytes: int = 0, rows_bytes: int = 0):
    _check(load().lge_set_table_budget(ctx, int(codeg_bytes), int(rows_bytes)), "lge_set_table_budget")


def lge_set_build_scratch(ctx, nbytes: int = 0):
    _check(load().lge_set_build_scratch(ctx, int(nbytes)), "lge_set_build_scratch")


def lge_estimate_adaptive(ctx, g, seed: int, beta: float = 0.01, t_max: int = 20, phi0: float = 0.0):
    """Returns (result dict, trace dict with lists p, delta, sampled)."""
    cfg = AdaptiveCfg(float(beta), int(t_max), 0, float(phi0))
    r = Result()
    tr = AdaptiveTrace()
    _check(load().lge_estimate_adaptive(ctx, g, int(seed), ctypes.byref(cfg), ctypes.byref(r), ctypes.byref(tr)),
           "lge_estimate_adaptive")
    k = tr.rounds
    return result_dict(r), {"rounds": k, "p": list(tr.p[:k]), "delta": list(tr.delta[:k]),
                            "sampled": [int(x) for x in tr.sampled[:k]]}


def lge_micro(ctx, g, e0: int = 0, e1: int | None = None, out=None, device: str = "cuda:0"):
    """Micro-level graphlet statistics of the edges [e0, e1): returns (rows,
    colmax) with rows a (e1-e0) x 17 int64 torch tensor on the device (the
    one given as ``out`` if any) and colmax the 18 column maxima (index i =
    graphlet G_i)."""
    import torch
    if e1 is None:
        e1 = int(load().lge_graph_m(g))
    nrows = max(int(e1) - int(e0), 0)
    if out is None:
        out = torch.empty((nrows, LGE_MICRO_COLS), dtype=torch.int64, device=device)
    elif (out.dtype != torch.int64 or not out.is_cuda or not out.is_contiguous()
          or tuple(out.shape) != (nrows, LGE_MICRO_COLS)):
        raise ValueError("out must be a contiguous (e1-e0) x 17 int64 device tensor")
    torch.cuda.synchronize(out.device)  # the library works on its own stream
    cm = (ctypes.c_int64 * 18)()
    _check(load().lge_micro(ctx, g, int(e0), int(e1), ctypes.c_void_p(out.data_ptr() if nrows else 0), cm),
           "lge_micro")
    return out, list(cm)


def lge_estimate_weighted(ctx, g, mode: int, p_mean: float, seed: int, opts: Opts | None = None):
    """Returns (result dict, info dict with p_level, edges, sampled per class
    and max_core)."""
    r = Result()
    info = WeightInfo()
    _check(load().lge_estimate_weighted(ctx, g, int(mode), float(p_mean), int(seed),
                                        ctypes.byref(opts) if opts is not None else None, ctypes.byref(r),
                                        ctypes.byref(info)), "lge_estimate_weighted")
    return result_dict(r), {"p_level": list(info.p_level), "edges": [int(x) for x in info.edges],
                            "sampled": [int(x) for x in info.sampled], "max_core": int(info.max_core)}


def lge_core_numbers(ctx, g, device: str = "cuda:0"):
    """Returns (int32 torch tensor of the n core numbers on the device, max core)."""
    import torch
    n = int(load().lge_graph_n(g))
    out = torch.empty(max(n, 0), dtype=torch.int32, device=device)
    mc = ctypes.c_int32()
    torch.cuda.synchronize(out.device)
    _check(load().lge_core_numbers(ctx, g, ctypes.c_void_p(out.data_ptr() if n else 0), ctypes.byref(mc)),
           "lge_core_numbers")
    return out, mc.value


def lge_estimate_fixed_k(ctx, g, k: int, seed: int, opts: Opts | None = None) -> dict:
    r = Result()
    _check(load().lge_estimate_fixed_k(ctx, g, int(k), int(seed), ctypes.byref(opts) if opts is not None else None,
                                       ctypes.byref(r)), "lge_estimate_fixed_k")
    return result_dict(r)


def lge_server_cfg_default() -> ServerCfg:
    c = ServerCfg()
    _check(load().lge_server_cfg_default(ctypes.byref(c)), "lge_server_cfg_default")
    return c


def lge_server_create(ctx, cfg: ServerCfg | None = None):
    s = _VP()
    _check(load().lge_server_create(ctx, ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(s)),
           "lge_server_create")
    return s


def lge_server_add_graph(srv, g) -> int:
    gid = ctypes.c_int32()
    _check(load().lge_server_add_graph(srv, g, ctypes.byref(gid)), "lge_server_add_graph")
    return gid.value


def lge_submit(srv, gid: int, p: float, seed: int) -> int:
    """Returns the ticket; raises LgeError (e.g. LGE_EBUSY)."""
    t = ctypes.c_uint64()
    _check(load().lge_submit(srv, int(gid), float(p), int(seed), ctypes.byref(t)), "lge_submit")
    return t.value


def lge_wait(srv, ticket: int, timeout_us: int = -1) -> dict:
    r = Result()
    _check(load().lge_wait(srv, int(ticket), int(timeout_us), ctypes.byref(r)), "lge_wait")
    return result_dict(r)


def lge_wait_rc(srv, ticket: int, timeout_us: int = -1):
    """(code, result-or-None) without raising."""
    r = Result()
    rc = load().lge_wait(srv, int(ticket), int(timeout_us), ctypes.byref(r))
    return rc, (result_dict(r) if rc == LGE_OK else None)


def lge_cancel(srv, ticket: int) -> int:
    return load().lge_cancel(srv, int(ticket))


def lge_server_get_stats(srv) -> dict:
    st = ServerStats()
    _check(load().lge_server_get_stats(srv, ctypes.byref(st)), "lge_server_get_stats")
    return {k: getattr(st, k) for k, _ in ServerStats._fields_}


def lge_server_destroy(srv):
    _check(load().lge_server_destroy(srv), "lge_server_destroy")


class Context:
    """RAII helper around lge_open / lge_close."""

    def __init__(self, device: int = 0):
        self.ctx = lge_open(device)

    def close(self):
        if self.ctx:
            lge_close(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def graph(self, row_ptr, col, flags: int = 0):
        return lge_graph_create_host(self.ctx, row_ptr, col, flags)

    def estimate(self, g, p: float, seed: int, opts: Opts | None = None) -> dict:
        return lge_estimate(self.ctx, g, p, seed, opts)
