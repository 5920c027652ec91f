"""Seeded synthetic inputs shared by the CPU oracle and the GPU solver.

Input construction only: graphs in CSR form (row_ptr u64[n+1], col u32[m],
w u32[m], rows sorted by target id), source vertices and raw counter-stream
numbers. Nothing here evaluates a shortest-path criterion or relaxes an edge.
The generators themselves live in ``gen.c`` (SplitMix64 as a counter-based
generator) and are compiled on first use with the host C compiler.

Workload families follow the paper's simulation and benchmark sections:
fixed-out-degree uniform random digraphs (stand-in for G(n, p)), R-MAT with
the Graph 500 initiator (a, b, c, d) = (.57, .19, .19, .05) (stand-in for the
Kronecker graphs), and 4-neighbour grids with an independent weight per
directed edge (stand-in for the road networks).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c into libgraphgen.so next to it (gcc -O2)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            u32, u64 = ctypes.c_uint32, ctypes.c_uint64
            lib.gg_er.argtypes = [u32, u32, u32, u32, u64, P, P, P]
            lib.gg_rmat.argtypes = [u32, u32, u32, u32, u32, u32, u32, u64, ctypes.c_int, P, P, P, P]
            lib.gg_grid.argtypes = [u32, u32, u32, u32, u64, P, P, P]
            lib.gg_sources.argtypes = [u32, P, u32, u64, P]
            lib.gg_u64.argtypes = [u64, u64, u64, u64, P]
            lib.gg_u64.restype = None
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """Directed graph in CSR form. Unreachable = no path; weights >= 0 (uint32)."""
    n: int
    row_ptr: np.ndarray  # uint64[n+1]
    col: np.ndarray      # uint32[m]
    w: np.ndarray        # uint32[m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])

    def outdeg(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def er(n: int, k: int, wlo: int, whi: int, seed: int) -> Graph:
    """n vertices, each with exactly k distinct uniform targets other than itself."""
    rp = np.empty(n + 1, np.uint64)
    col = np.empty(n * k, np.uint32)
    w = np.empty(n * k, np.uint32)
    rc = _L().gg_er(n, k, wlo, whi, seed, _p(rp), _p(col), _p(w))
    if rc != 0:
        raise ValueError("gg_er failed (%d): need 2 <= n and k < n" % rc)
    return Graph(n, rp, col, w, "er_n%d_k%d" % (n, k), dict(kind="er", k=k, wlo=wlo, whi=whi, seed=seed))


def rmat(scale: int, ef: int, wlo: int, whi: int, seed: int,
         abc=(0.57, 0.19, 0.19), permute: bool = True) -> Graph:
    """R-MAT with ef * 2^scale sampled edges; self-loops dropped, duplicates merged."""
    n = 1 << scale
    ms = ef << scale
    a16, b16, c16 = (int(round(x * 65536)) for x in abc)
    rp = np.empty(n + 1, np.uint64)
    col = np.empty(ms, np.uint32)
    w = np.empty(ms, np.uint32)
    m = ctypes.c_uint64(0)
    rc = _L().gg_rmat(scale, ef, a16, b16, c16, wlo, whi, seed, int(permute),
                      _p(rp), _p(col), _p(w), ctypes.byref(m))
    if rc != 0:
        raise ValueError("gg_rmat failed (%d)" % rc)
    mm = int(m.value)
    return Graph(n, rp, col[:mm].copy(), w[:mm].copy(), "rmat_s%d_ef%d" % (scale, ef),
                 dict(kind="rmat", scale=scale, ef=ef, wlo=wlo, whi=whi, seed=seed))


def grid(W: int, H: int, wlo: int, whi: int, seed: int) -> Graph:
    """W x H 4-neighbour grid; each directed edge has its own weight."""
    n = W * H
    m = 2 * (2 * W * H - W - H)
    rp = np.empty(n + 1, np.uint64)
    col = np.empty(max(m, 1), np.uint32)
    w = np.empty(max(m, 1), np.uint32)
    rc = _L().gg_grid(W, H, wlo, whi, seed, _p(rp), _p(col), _p(w))
    if rc != 0:
        raise ValueError("gg_grid failed")
    return Graph(n, rp, col[:m].copy(), w[:m].copy(), "grid_%dx%d" % (W, H),
                 dict(kind="grid", W=W, H=H, wlo=wlo, whi=whi, seed=seed))


def sources(g: Graph, count: int, seed: int) -> np.ndarray:
    """count sources uniform over vertices with out-degree >= 1."""
    out = np.empty(count, np.uint32)
    if _L().gg_sources(g.n, _p(g.row_ptr), count, seed, _p(out)) != 0:
        raise ValueError("graph has no out-edges")
    return out


def u64_stream(seed: int, tag: int, count: int, start: int = 0) -> np.ndarray:
    out = np.empty(count, np.uint64)
    _L().gg_u64(seed, tag, start, count, _p(out))
    return out


def uniform01(seed: int, tag: int, count: int) -> np.ndarray:
    """float64 in [0, 1) from the counter stream (53 high bits)."""
    return (u64_stream(seed, tag, count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def from_edges(n: int, edges, name: str = "edges") -> Graph:
    """CSR from an explicit list of (u, v, c) triples (kept in (u, v) order).

    Self-loops and parallel edges are kept as given.
    """
    e = sorted(((int(u), int(v), int(c)) for (u, v, c) in edges), key=lambda t: (t[0], t[1]))
    rp = np.zeros(n + 1, np.uint64)
    for u, _, _ in e:
        rp[u + 1] += 1
    rp = np.cumsum(rp).astype(np.uint64)
    col = np.array([v for _, v, _ in e], dtype=np.uint32)
    w = np.array([c for _, _, c in e], dtype=np.uint32)
    return Graph(n, rp, col, w, name)


def random_small(n: int, m: int, wmax: int, seed: int, zero_ok: bool = True,
                 self_loops: bool = True) -> Graph:
    """Tiny random multigraph (parallel edges, self-loops, zero weights allowed)."""
    x = u64_stream(seed, 77, 3 * m)
    us = (x[0::3] % np.uint64(n)).astype(np.int64)
    vs = (x[1::3] % np.uint64(n)).astype(np.int64)
    lo = 0 if zero_ok else 1
    cs = (x[2::3] % np.uint64(wmax - lo + 1)).astype(np.int64) + lo
    edges = [(u, v, c) for u, v, c in zip(us, vs, cs) if self_loops or u != v]
    return from_edges(n, edges, "small_n%d_m%d_s%d" % (n, m, seed))


def path(n: int, weights) -> Graph:
    return from_edges(n, [(i, i + 1, weights[i]) for i in range(n - 1)], "path%d" % n)


def out_star(k: int, weights) -> Graph:
    return from_edges(k + 1, [(0, i + 1, weights[i]) for i in range(k)], "star%d" % k)


# Named workloads ------------------------------------------------------------

def config_small(seed: int = 1) -> Graph:
    """16384 vertices, 8 distinct out-targets each, weights uniform in [1, 1000]."""
    return er(16384, 8, 1, 1000, seed)


def config_er_large(seed: int = 1, log2n: int = 22) -> Graph:
    """2^22 vertices, out-degree 16, weights uniform in [1, 2^20)."""
    return er(1 << log2n, 16, 1, (1 << 20) - 1, seed)


def config_rmat(seed: int = 1, scale: int = 22) -> Graph:
    """R-MAT scale 22, edge factor 16, (.57,.19,.19,.05), weights [1, 2^20)."""
    return rmat(scale, 16, 1, (1 << 20) - 1, seed)


def config_grid(seed: int = 1, side: int = 2048) -> Graph:
    """side x side 4-neighbour grid, weights uniform in [1, 2^16]."""
    return grid(side, side, 1, 1 << 16, seed)


def batch_workload(seed: int = 7, n_graphs: int = 64, q_per_graph: int = 8, max_log2: int = 18):
    """Uneven graph mix: ER 2^12..2^18 deg 4..32, grids 64^2..512^2, R-MAT 12..18 ef 16.

    Weights uniform in [1, 2^16]; q_per_graph random sources per graph.
    Returns (graphs, [(graph_index, source), ...]).
    """
    r = u64_stream(seed, 91, 4 * n_graphs)
    graphs, queries = [], []
    lo = 12
    for i in range(n_graphs):
        kind = i % 3
        gs = seed * 1000 + i
        if kind == 0:
            lg = lo + int(r[4 * i] % np.uint64(max_log2 - lo + 1))
            deg = 4 + int(r[4 * i + 1] % np.uint64(29))
            g = er(1 << lg, deg, 1, 1 << 16, gs)
        elif kind == 1:
            side_max = 1 << ((max_log2 + 1) // 2)
            side = 64 + int(r[4 * i + 2] % np.uint64(side_max - 64 + 1))
            g = grid(side, side, 1, 1 << 16, gs)
        else:
            sc = lo + int(r[4 * i + 3] % np.uint64(max_log2 - lo + 1))
            g = rmat(sc, 16, 1, 1 << 16, gs)
        graphs.append(g)
        for s in sources(g, q_per_graph, gs + 17):
            queries.append((i, int(s)))
    return graphs, queries
