"""Writes the whole-graph oracle goldens of the full-size configurations.

Each golden is one JSON file holding the oracle's estimate of a seeded
synthetic graph (every integer as a decimal string, every double as its
hexadecimal form) together with a SHA-256 fingerprint of the graph's CSR, so
that a test first checks it regenerated the same input.  Only ``oracle`` (the
threaded plain oracle, whose per-thread integer sums add up exactly) and the
seeded input generators are called; nothing here touches the GPU library.

    python tests/golden/make_goldens.py [--threads 8] [name ...]

Names: chung_lu_1m_p1, chung_lu_1m_p0.1, chung_lu_1m_p0.01,
rmat_s22_p0.01.  The Chung-Lu and R-MAT graphs are the full-size
workloads (n = 10^6, mean expected degree 16, exponent 2.1, cap 5*10^4,
generator seed 10^6; R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19,
0.05), generator seed 22); the sampler seed is 2024 (2025 for R-MAT).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDENS = {
    "chung_lu_1m_p1": ("chung_lu_1m", 1.0, 2024),
    "chung_lu_1m_p0.1": ("chung_lu_1m", 0.1, 2024),
    "chung_lu_1m_p0.01": ("chung_lu_1m", 0.01, 2024),
    "rmat_s22_p0.01": ("rmat_22", 0.01, 2025),
}


def graph_fingerprint(g) -> str:
    h = hashlib.sha256()
    h.update(g.row_ptr.astype("<i4").tobytes())
    h.update(g.col.astype("<i4").tobytes())
    return h.hexdigest()


def path_of(name: str) -> str:
    return os.path.join(HERE, "%s.json" % name)


def load(name: str) -> dict:
    """The stored golden as an oracle-style result dict (Python ints and
    floats) plus its ``graph`` fingerprint and ``maker`` name."""
    with open(path_of(name)) as fh:
        d = json.load(fh)
    out = {k: d[k] for k in ("n", "m", "p", "seed", "graph_sha256", "maker")}
    out["p"] = float.fromhex(out["p"])
    out["sampled"] = int(d["sampled"])
    for k in ("csum", "zsum", "qsum", "exact"):
        out[k] = [int(x) for x in d[k]]
    for k in ("estimate", "variance", "lower95", "upper95"):
        out[k] = [float.fromhex(x) for x in d[k]]
    return out


def write(name: str, threads: int) -> None:
    import oracle
    from paper_1701_01772_amd import inputs
    maker, p, seed = GOLDENS[name]
    g = getattr(inputs, maker)()
    t0 = time.perf_counter()
    r = oracle.estimate_threads(g.row_ptr, g.col, p, seed, threads=threads)
    dt = time.perf_counter() - t0
    parts = r.pop("parts")
    # the per-thread integer sums add up to the finalised totals
    assert sum(x["sampled"] for x in parts) == r["sampled"]
    for k in ("csum", "qsum"):
        for i in range(18):
            assert sum(x[k][i] for x in parts) == r[k][i], (k, i)
    d = {
        "maker": maker, "n": g.n, "m": g.m, "p": float(p).hex(), "seed": seed,
        "graph_sha256": graph_fingerprint(g),
        "sampled": str(r["sampled"]),
        "oracle_threads": len(parts), "oracle_seconds": round(dt, 1),
    }
    for k in ("csum", "zsum", "qsum", "exact"):
        d[k] = [str(int(x)) for x in r[k]]
    for k in ("estimate", "variance", "lower95", "upper95"):
        d[k] = [float(x).hex() for x in r[k]]
    with open(path_of(name), "w") as fh:
        json.dump(d, fh, indent=1)
        fh.write("\n")
    print("%s: n=%d m=%d p=%g sampled=%d in %.1f s on %d threads" % (
        name, g.n, g.m, p, r["sampled"], dt, len(parts)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("names", nargs="*")
    args = ap.parse_args()
    for name in args.names or sorted(GOLDENS):
        write(name, args.threads)


if __name__ == "__main__":
    main()
