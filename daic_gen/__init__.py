"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This module builds graphs and plain random draws only; it contains none of the
solver arithmetic. Every draw is a pure function of (seed, counter), so results
do not depend on the thread count.

Workload recipes (shapes of the paper's evaluation, Sec. 6.1.2, at one-GPU
scale; the Google Webgraph and the paper's 100M-2B node graphs are not
available, so these stand in for them):

* ``powerlaw_10k``   -- 10,000 vertices, out-degree floor(LogNormal(2, 1))
  capped at 500, targets drawn preferentially by in-degree (+1), no self-loop,
  no duplicate per source; seed 1.
* ``rmat(scale, ef)`` -- RMAT a/b/c/d = .57/.19/.19/.05, no noise, no vertex
  permutation, duplicates and self-loops kept; rows sorted ascending.
* ``paper_lognormal`` -- the paper's own variant: in-degree
  floor(LogNormal(-0.5, 2.3)), sources uniform.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdaicgen.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the generator library with g++ (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        import subprocess

        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               os.path.join(_HERE, "gen.cpp"), "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.gen_draw_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _u64p]
        lib.gen_uniform_u32.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_uint32, _u32p]
        lib.gen_lognormal_f64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                          ctypes.c_double, _f64p]
        lib.gen_rmat.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, _u64p, _u32p]
        lib.gen_rmat.restype = ctypes.c_int
        lib.gen_lognormal_outdeg.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_uint64, ctypes.c_uint64, _u64p]
        lib.gen_lognormal_outdeg.restype = ctypes.c_uint64
        lib.gen_pref_targets.argtypes = [ctypes.c_uint64, _u64p, ctypes.c_uint64, _u32p]
        lib.gen_indeg_lognormal_count.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_uint64, _u64p]
        lib.gen_indeg_lognormal_count.restype = ctypes.c_uint64
        lib.gen_indeg_lognormal_edges.argtypes = [ctypes.c_uint64, _u64p, ctypes.c_uint64, _u64p, _u32p]
        lib.gen_ppr_seeds.argtypes = [ctypes.c_uint64, _u64p, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_uint32, ctypes.c_uint32, _u32p, _u32p]
        lib.gen_ppr_seeds.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


@dataclass
class Graph:
    """Directed graph in CSR form: row_ptr[n+1] (uint64), col[m] (uint32)."""

    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def outdeg(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def draw_u64(seed: int, count: int, first: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    if count:
        _get().gen_draw_u64(seed, first, count, _p(out, _u64p))
    return out


def uniform_u32(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    if count:
        _get().gen_uniform_u32(seed, count, lo, hi, _p(out, _u32p))
    return out


def lognormal_f64(seed: int, count: int, mu: float, sigma: float) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    if count:
        _get().gen_lognormal_f64(seed, count, mu, sigma, _p(out, _f64p))
    return out


def rmat(scale: int, edgefactor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19) -> Graph:
    n = 1 << scale
    m = edgefactor * n
    row_ptr = np.empty(n + 1, dtype=np.uint64)
    col = np.empty(m, dtype=np.uint32)
    rc = _get().gen_rmat(scale, edgefactor, a, b, c, seed, _p(row_ptr, _u64p), _p(col, _u32p))
    if rc != 0:
        raise ValueError("rmat: bad scale")
    return Graph(row_ptr, col, f"rmat{scale}_ef{edgefactor}_s{seed}")


def powerlaw(n: int = 10000, mu: float = 2.0, sigma: float = 1.0, cap: int = 500,
             seed: int = 1) -> Graph:
    outdeg = np.empty(n, dtype=np.uint64)
    m = _get().gen_lognormal_outdeg(n, mu, sigma, cap, seed, _p(outdeg, _u64p))
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(outdeg, out=row_ptr[1:])
    col = np.empty(int(m), dtype=np.uint32)
    _get().gen_pref_targets(n, _p(row_ptr, _u64p), seed ^ 0x5EED, _p(col, _u32p))
    return Graph(row_ptr, col, f"powerlaw{n}_s{seed}")


def paper_lognormal(n: int, seed: int, mu: float = -0.5, sigma: float = 2.3) -> Graph:
    indeg = np.empty(n, dtype=np.uint64)
    m = _get().gen_indeg_lognormal_count(n, mu, sigma, seed, _p(indeg, _u64p))
    row_ptr = np.empty(n + 1, dtype=np.uint64)
    col = np.empty(int(m), dtype=np.uint32)
    _get().gen_indeg_lognormal_edges(n, _p(indeg, _u64p), seed, _p(row_ptr, _u64p), _p(col, _u32p))
    return Graph(row_ptr, col, f"paperlognormal{n}_s{seed}")


def ppr_seeds(g: Graph, seed: int, rhs_base: int, n_rhs: int, max_k: int = 32):
    """Seed sets for personalized PageRank right-hand sides.

    Returns (counts[n_rhs], seeds[n_rhs, max_k]) with unused slots = 2**32-1.
    """
    counts = np.empty(n_rhs, dtype=np.uint32)
    seeds = np.empty((n_rhs, max_k), dtype=np.uint32)
    rp = np.ascontiguousarray(g.row_ptr)
    _get().gen_ppr_seeds(g.n, _p(rp, _u64p), seed, rhs_base, n_rhs, max_k,
                         _p(counts, _u32p), _p(seeds, _u32p))
    return counts, seeds


def from_edges(n: int, src, dst) -> Graph:
    """CSR from an explicit edge list (rows sorted ascending); for small tests."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.uint64)
    return Graph(row_ptr, dst.astype(np.uint32), "edges")


# ---------------------------------------------------------------------------
# Named workloads.
# ---------------------------------------------------------------------------

def batch_scales(n_graphs: int = 64, seed: int = 5, lo: int = 12, hi: int = 20) -> np.ndarray:
    """Per-graph RMAT scales for the batched personalized-PageRank workload."""
    return uniform_u32(seed, n_graphs, lo, hi).astype(np.int64)


def sssp_weights(m: int, seed: int = 3) -> np.ndarray:
    """Integer edge weights uniform on 1..255."""
    return uniform_u32(seed, m, 1, 255)
