"""Seeded synthetic input graphs (int32 CSR, sorted adjacency, simple, undirected).

Input generation only: this module draws graphs with the shapes of the
workloads and holds none of the graphlet-counting arithmetic, so both the CPU
oracle and the GPU path can consume its output.  The generators themselves
are C (``graphgen.c``) because R-MAT scale 22 needs 67M endpoint draws.

Workload recipes (all seeds explicit):

* ``erdos_renyi(n, q)``: every pair i.i.d. Bernoulli(q).
* ``chung_lu(n, avg_deg, gamma, cap)``: weights w_i ~ (i+1)^(-1/(gamma-1)),
  scaled by bisection so the capped mean is ``avg_deg``; round(n*avg_deg/2)
  endpoint pairs drawn proportional to w; loops dropped, duplicates merged.
* ``rmat(scale, edge_factor, a, b, c)``: Graph500-style recursive quadrants
  without noise, seeded vertex relabelling; loops dropped, duplicates merged.
* ``batch_graphs``: mixed small ER / Chung-Lu graphs, log-uniform sizes.
* ``serving_graphs``: mixed Chung-Lu / R-MAT-shaped graphs, log-uniform edge
  counts.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile graphgen.c into libgraphgen.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32p, dbl, u64 = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_double, ctypes.c_uint64
        lib.gg_erdos_renyi.argtypes = [i64, dbl, u64, i32p, i32p, i64]
        lib.gg_chung_lu.argtypes = [i64, dbl, dbl, dbl, u64, i32p, i32p, i64]
        lib.gg_rmat.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, ctypes.c_int, u64, i32p, i32p, i64]
        lib.gg_from_pairs.argtypes = [i64, i64, i32p, i32p, i32p, i32p, i64]
        for f in (lib.gg_erdos_renyi, lib.gg_chung_lu, lib.gg_rmat, lib.gg_from_pairs):
            f.restype = i64
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class Graph:
    """An undirected simple graph as int32 CSR (both directions stored)."""

    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[2m], strictly increasing within each row
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0] // 2)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _finish(n: int, fn, cap: int, name: str) -> Graph:
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.empty(max(cap, 1), dtype=np.int32)
    nnz = fn(row_ptr, col, cap)
    if nnz < 0:
        raise RuntimeError("graph generator failed with code %d (%s)" % (nnz, name))
    return Graph(row_ptr, col[:nnz].copy(), name)


def erdos_renyi(n: int, q: float, seed: int) -> Graph:
    exp = q * n * (n - 1) / 2.0
    cap = int(2 * (exp + 12 * math.sqrt(exp + 1) + 64))
    lib = _load()
    return _finish(n, lambda rp, c, k: lib.gg_erdos_renyi(n, q, seed, _p32(rp), _p32(c), k), cap,
                   "er(n=%d,q=%g,seed=%d)" % (n, q, seed))


def chung_lu(n: int, avg_deg: float, gamma: float, cap: float, seed: int) -> Graph:
    draws = int(round(n * avg_deg / 2.0))
    lib = _load()
    return _finish(n, lambda rp, c, k: lib.gg_chung_lu(n, avg_deg, gamma, cap, seed, _p32(rp), _p32(c), k),
                   2 * draws, "chung_lu(n=%d,d=%g,gamma=%g,cap=%g,seed=%d)" % (n, avg_deg, gamma, cap, seed))


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int, relabel: bool = True) -> Graph:
    n = 1 << scale
    draws = edge_factor * n
    lib = _load()
    return _finish(n, lambda rp, cc, k: lib.gg_rmat(scale, edge_factor, a, b, c, int(relabel), seed,
                                                     _p32(rp), _p32(cc), k),
                   2 * draws, "rmat(scale=%d,ef=%d,seed=%d)" % (scale, edge_factor, seed))


def from_edges(n: int, edges) -> Graph:
    """CSR of the simple graph on n vertices spanned by the given pairs."""
    e = np.asarray(list(edges), dtype=np.int32).reshape(-1, 2)
    pa = np.ascontiguousarray(e[:, 0])
    pb = np.ascontiguousarray(e[:, 1])
    lib = _load()
    return _finish(n, lambda rp, c, k: lib.gg_from_pairs(n, len(pa), _p32(pa), _p32(pb), _p32(rp), _p32(c), k),
                   2 * len(pa), "pairs(n=%d)" % n)


# ---------------------------------------------------------------------------
# Workload presets with the sizes of the measured configurations.
# ---------------------------------------------------------------------------

def er_2000(seed: int = 20000) -> Graph:
    """G(n=2000, q=0.005)."""
    return erdos_renyi(2000, 0.005, seed)


def chung_lu_1m(seed: int = 1000000) -> Graph:
    """Chung-Lu n=1,000,000, mean expected degree 16, exponent 2.1, cap 50,000."""
    return chung_lu(1_000_000, 16.0, 2.1, 50_000.0, seed)


def rmat_22(seed: int = 22) -> Graph:
    """R-MAT scale 22, edge factor 16, (a,b,c,d) = (0.57,0.19,0.19,0.05)."""
    return rmat(22, 16, 0.57, 0.19, 0.19, seed)


def batch_graphs(count: int = 4096, seed: int = 4096, n_lo: int = 50, n_hi: int = 5000):
    """Mixed batch: n log-uniform in [n_lo, n_hi]; even index ER with mean degree
    log-uniform in [4, 32]; odd index Chung-Lu with exponent U[2.1, 2.8], mean
    degree log-uniform in [4, 32], cap n-1."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(10 ** rng.uniform(math.log10(n_lo), math.log10(n_hi))))
        d = float(10 ** rng.uniform(math.log10(4.0), math.log10(32.0)))
        gseed = int(rng.integers(0, 2**62))
        if i % 2 == 0:
            q = min(1.0, d / max(n - 1, 1))
            out.append(erdos_renyi(n, q, gseed))
        else:
            gamma = float(rng.uniform(2.1, 2.8))
            out.append(chung_lu(n, min(d, n - 1), gamma, float(n - 1), gseed))
    return out


def serving_graphs(count: int = 64, seed: int = 64, m_lo: float = 1e3, m_hi: float = 5e7, threads: int = 1):
    """Mixed resident set: target edge counts log-uniform in [m_lo, m_hi];
    even index Chung-Lu (mean degree 16, exponent 2.1, cap n/20), odd index
    R-MAT-shaped (edge factor 16, scale chosen for the target).  With
    threads > 1 the graphs are drawn in parallel (the C generator releases
    the interpreter lock); the result does not depend on it."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        m_t = 10 ** rng.uniform(math.log10(m_lo), math.log10(m_hi))
        gseed = int(rng.integers(0, 2**62))
        specs.append((i, m_t, gseed))

    def make(spec):
        i, m_t, gseed = spec
        if i % 2 == 0:
            n = max(64, int(round(m_t / 8.0)))
            return chung_lu(n, 16.0, 2.1, max(16.0, n / 20.0), gseed)
        scale = max(6, int(round(math.log2(max(m_t / 16.0 * 1.12, 64)))))
        return rmat(scale, 16, 0.57, 0.19, 0.19, gseed)

    if threads <= 1:
        return [make(sp) for sp in specs]
    from concurrent.futures import ThreadPoolExecutor
    _load()
    # largest first, so the longest draws start early
    order = sorted(range(count), key=lambda k: -specs[k][1])
    out = [None] * count
    with ThreadPoolExecutor(max_workers=threads) as pool:
        for k, g in zip(order, pool.map(lambda k: make(specs[k]), order)):
            out[k] = g
    return out
