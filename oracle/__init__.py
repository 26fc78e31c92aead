"""ORACLE — test infrastructure only.

A plain single-thread CPU implementation of the edge-centric graphlet
estimator (``lge_oracle.c``) plus a brute-force enumerator of all 3- and
4-vertex subsets (``bruteforce.py``).  Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import this package; the product path
never does, and this package imports nothing from the product.

Pins (each checked by a ``-m "not gpu"`` test, see tests/test_oracle_*.py):
  * exact counts == brute-force classification of every 3-/4-subset, the
    classes identified by the Table 1 properties (edges, max degree,
    components) stored in tests/golden/table1_graphlets.txt;
  * closed forms on complete, complete bipartite, star, cycle and empty
    graphs; trace identities tr(A^3)/6 and the closed-4-walk identity;
  * exact unbiasedness of X and of the variance estimate by enumerating every
    sample outcome on tiny graphs (Sec. 2.4);
  * Philox4x32-10 known-answer vectors and a cross-check against an
    independent Philox implementation;
  * micro rows (``micro``) against a per-edge brute-force enumeration and
    edge-weighted census sums;
  * the adaptive loop (``adaptive.py``), the weighted and fixed-size designs
    and k-core numbers (``designs.py``): schedule closed forms, brute-force
    cores, exact unbiasedness by enumerating every sample outcome, planted
    mistakes caught.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lge_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

GRAPHLET_NAMES = [
    None, "edge", "2-node-independent", "triangle", "2-star", "3-node-1-edge",
    "3-node-independent", "4-clique", "chordal-cycle", "tailed-triangle", "4-cycle",
    "3-star", "4-path", "4-node-1-triangle", "4-node-2-star", "4-node-2-edge",
    "4-node-1-edge", "4-node-independent",
]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class _Result(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64), ("p", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("sampled", ctypes.c_uint64),
        ("csum", _U128 * 18), ("zsum", _U128 * 18), ("qsum", _U128 * 18), ("exact", _U128 * 18),
        ("estimate", ctypes.c_double * 18), ("variance", ctypes.c_double * 18),
        ("lower95", ctypes.c_double * 18), ("upper95", ctypes.c_double * 18),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.oracle_philox4x32_10.restype = None
        lib.oracle_edge_sampled.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double]
        lib.oracle_edge_sampled.restype = ctypes.c_int
        lib.oracle_estimate.argtypes = [ctypes.c_int64, i32p, i32p, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(_Result)]
        lib.oracle_estimate.restype = ctypes.c_int
        lib.oracle_edge_local.argtypes = [ctypes.c_int64, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_edge_local.restype = ctypes.c_int
        lib.oracle_sample_mask.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_sample_mask.restype = ctypes.c_uint64
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_micro.argtypes = [ctypes.c_int64, i32p, i32p, i32p, i32p, ctypes.c_int64, i64p]
        lib.oracle_micro.restype = ctypes.c_int
        lib.oracle_philox_keys.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_philox_keys.restype = None
        lib.oracle_finalize_sums.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                             ctypes.c_uint64, _U128 * 17, _U128 * 18, ctypes.POINTER(_Result)]
        lib.oracle_finalize_sums.restype = ctypes.c_int
        lib.oracle_i128_to_double.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_i128_to_double.restype = ctypes.c_double
        _lib = lib
    return _lib


def _u(x: _U128) -> int:
    return (x.hi << 64) | x.lo


def _s(x: _U128) -> int:
    v = _u(x)
    return v - (1 << 128) if v >> 127 else v


def philox4x32_10(ctr, key):
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def edge_sampled(seed: int, eid: int, p: float) -> bool:
    return bool(_load().oracle_edge_sampled(seed, eid, p))


def sample_count(seed: int, p: float, e0: int, e1: int) -> int:
    """Number of canonical edge ids in [e0, e1) that the sampler keeps."""
    return int(_load().oracle_sample_mask(seed, p, e0, e1, None))


def sample_mask(seed: int, p: float, m: int, e0: int = 0, e1: int | None = None) -> np.ndarray:
    """uint8[m] mask of the sampled edges whose id lies in [e0, e1)."""
    e1 = m if e1 is None else e1
    mask = np.zeros(max(m, 1), dtype=np.uint8)
    if e1 > e0:
        sub = np.zeros(e1 - e0, dtype=np.uint8)
        _load().oracle_sample_mask(seed, p, e0, e1, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        mask[e0:e1] = sub
    return mask[:m] if m > 0 else mask


def philox_keys(seed: int, m: int) -> np.ndarray:
    """uint64[m]: the 64-bit Philox output (x1:x0) of every edge id."""
    out = np.zeros(max(m, 1), dtype=np.uint64)
    if m > 0:
        _load().oracle_philox_keys(seed, 0, m, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out[:m]


def i128_to_double(x: int) -> float:
    """The oracle's int128 -> double conversion (round to nearest, ties to even)."""
    if not -(1 << 127) <= x < (1 << 127):
        raise ValueError("not a signed 128-bit value")
    v = x & ((1 << 128) - 1)
    return float(_load().oracle_i128_to_double(v & ((1 << 64) - 1), v >> 64))


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    return rp, cl


def estimate(row_ptr, col, p: float, seed: int = 0, mask=None) -> dict:
    """Run the oracle.  Returns a dict with Python ints for every integer field
    (``csum``, ``zsum`` signed, ``qsum``, ``exact``: lists indexed by graphlet
    number 0..17, slot 0 unused) and float lists for the FP64 fields."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    n = rp.shape[0] - 1
    res = _Result()
    mptr = None
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        if mk.size == 0:
            mk = np.zeros(1, dtype=np.uint8)
        mptr = mk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    rc = lib.oracle_estimate(n, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(p), int(seed),
                             mptr, ctypes.byref(res))
    if rc != 0:
        raise RuntimeError("oracle_estimate failed: %d" % rc)
    return _result_dict(res)


def _result_dict(res) -> dict:
    return {
        "n": res.n, "m": res.m, "p": res.p, "seed": res.seed, "sampled": res.sampled,
        "csum": [_u(res.csum[i]) for i in range(18)],
        "zsum": [_s(res.zsum[i]) for i in range(18)],
        "qsum": [_u(res.qsum[i]) for i in range(18)],
        "exact": [_u(res.exact[i]) for i in range(18)],
        "estimate": list(res.estimate), "variance": list(res.variance),
        "lower95": list(res.lower95), "upper95": list(res.upper95),
    }


def _limbs(x: int) -> _U128:
    v = x & ((1 << 128) - 1)
    return _U128(v & ((1 << 64) - 1), v >> 64)


def estimate_threads(row_ptr, col, p: float, seed: int = 0, threads: int = 8, mask=None) -> dict:
    """``estimate`` over the same sample, split round-robin by sampled edge
    over ``threads`` host threads (the C oracle is reentrant and ctypes drops
    the GIL during a call).  Each thread's integer sums come from the plain
    oracle on its share; their exact totals are finalised once, as one call
    would.  The result equals ``estimate`` bit for bit (the sums do not
    depend on the order of the edges).  Also returns the per-thread results
    under ``"parts"``."""
    from concurrent.futures import ThreadPoolExecutor
    rp, cl = _csr(row_ptr, col)
    n = rp.shape[0] - 1
    m = int(rp[-1]) // 2
    if mask is None:
        mask = sample_mask(seed, p, m)
    ids = np.nonzero(np.asarray(mask, dtype=np.uint8)[:m])[0]
    threads = max(1, min(int(threads), max(1, ids.size)))
    masks = []
    for i in range(threads):
        mk = np.zeros(max(m, 1), dtype=np.uint8)
        mk[ids[i::threads]] = 1
        masks.append(mk)
    with ThreadPoolExecutor(max_workers=threads) as pool:
        parts = list(pool.map(lambda mk: estimate(rp, cl, p, seed, mask=mk), masks))
    sampled = sum(x["sampled"] for x in parts)
    csum = [sum(x["csum"][i] for x in parts) for i in range(17)]
    qsum = [sum(x["qsum"][i] for x in parts) for i in range(18)]
    cs = (_U128 * 17)(*[_limbs(v) for v in csum])
    qs = (_U128 * 18)(*[_limbs(v) for v in qsum])
    res = _Result()
    rc = _load().oracle_finalize_sums(n, m, float(p), int(seed), sampled, cs, qs, ctypes.byref(res))
    if rc != 0:
        raise RuntimeError("oracle_finalize_sums failed: %d" % rc)
    out = _result_dict(res)
    out["parts"] = parts
    return out


def edge_local(row_ptr, col, u: int, v: int) -> dict:
    """Per-edge local quantities of Alg. 2-4 with u as the classified side."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    out = (ctypes.c_int64 * 7)()
    rc = lib.oracle_edge_local(rp.shape[0] - 1, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(u), int(v), out)
    if rc != 0:
        raise RuntimeError("oracle_edge_local failed")
    keys = ["t", "su", "sv", "r", "clique", "cycle", "f"]
    return {k: int(out[i]) for i, k in enumerate(keys)}


def canonical_edges(row_ptr, col):
    """(us, vs) of every edge u < v, in canonical id order (row-major)."""
    rp, cl = _csr(row_ptr, col)
    cl = cl[:int(rp[-1])]
    deg = np.diff(rp)
    src = np.repeat(np.arange(rp.shape[0] - 1, dtype=np.int32), deg)
    keep = cl > src
    return src[keep], cl[keep]


def micro(row_ptr, col, eids=None) -> np.ndarray:
    """Micro-level graphlet statistics (Sec. 3, Alg. 7 with p_e = 1): one row
    of 17 int64 per edge id in ``eids`` (default: every edge), column i-1 =
    number of induced G_i containing both ends of the edge."""
    lib = _load()
    rp, cl = _csr(row_ptr, col)
    us, vs = canonical_edges(rp, cl)
    if eids is not None:
        idx = np.asarray(eids, dtype=np.int64)
        us, vs = us[idx], vs[idx]
    us = np.ascontiguousarray(us, dtype=np.int32)
    vs = np.ascontiguousarray(vs, dtype=np.int32)
    out = np.zeros((us.shape[0], 17), dtype=np.int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    rc = lib.oracle_micro(rp.shape[0] - 1, rp.ctypes.data_as(i32p), cl.ctypes.data_as(i32p),
                          us.ctypes.data_as(i32p), vs.ctypes.data_as(i32p), us.shape[0],
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RuntimeError("oracle_micro failed")
    return out
