"""CPU oracle for the phased SSSP path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU product path never links or calls it, and the
oracle imports nothing from the product package: the two share only the
seeded input generators in ``graphgen``.

The arithmetic lives in ``oracle.c`` (plain C, compiled on first use with
gcc); this module only marshals numpy arrays. Criterion bit values follow
the disjunction convention of Section 3 (a set of bits = their OR).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

INF = np.uint64(0xFFFFFFFFFFFFFFFF)
INF_INT = 0xFFFFFFFFFFFFFFFF

DIJK, IN_STATIC, OUT_STATIC, IN_SIMPLE, OUT_SIMPLE, IN_FULL, OUT_WEAK, OUT_FULL = (1 << i for i in range(8))
IN_APPROX, OUT_APPROX = 1 << 8, 1 << 9  # approximate criteria (Section 3, last paragraphs); see phased()
BIT_NAMES = ["DIJK", "IN_STATIC", "OUT_STATIC", "IN_SIMPLE", "OUT_SIMPLE", "IN_FULL", "OUT_WEAK", "OUT_FULL"]
CRIT = {name: 1 << i for i, name in enumerate(BIT_NAMES)}
STATIC_OR = IN_STATIC | OUT_STATIC
SIMPLE_OR = IN_SIMPLE | OUT_SIMPLE
FULL_OR = IN_FULL | OUT_FULL


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_SAN_SRC = os.path.join(_HERE, "sanitize_main.c")
_GEN_SRC = os.path.join(os.path.dirname(_HERE), "graphgen", "gen.c")
SANITIZED_EXE = os.path.join(_HERE, "orc_sanitize")


def build_sanitized(exe: str = SANITIZED_EXE) -> str:
    """The stdin-driven sanitizer driver: oracle.c + graphgen/gen.c + sanitize_main.c, host code
    built by gcc with AddressSanitizer and UndefinedBehaviorSanitizer."""
    tmp = exe + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-g", "-O1", _SRC, _GEN_SRC, _SAN_SRC, "-lm", "-o", tmp])
    os.replace(tmp, exe)
    return exe


class _Stats(ctypes.Structure):
    _fields_ = [("phases", ctypes.c_uint32), ("pad", ctypes.c_uint32), ("sum_f", ctypes.c_uint64),
                ("n_reach", ctypes.c_uint64), ("m_reach", ctypes.c_uint64),
                ("relax_edges", ctypes.c_uint64), ("improving", ctypes.c_uint64)]


class _DStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint32), ("buckets", ctypes.c_uint32),
                ("light_relax", ctypes.c_uint64), ("heavy_relax", ctypes.c_uint64),
                ("sum_frontier", ctypes.c_uint64)]


def _L():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P, u32, u64, i = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
            lib.orc_validate.argtypes = [u32, P, P]
            lib.orc_dijkstra.argtypes = [u32, P, P, P, u32, P, P]
            lib.orc_dijkstra.restype = ctypes.c_int64
            lib.orc_bellman_ford.argtypes = [u32, P, P, P, u32, P]
            lib.orc_static_minima.argtypes = [u32, P, P, P, P, P]
            lib.orc_phased.argtypes = [u32, P, P, P, u32, u32, P, u32, i, P, P,
                                       ctypes.POINTER(_Stats), u32, P, P, P, P, P, P, P, P, P, u32, u32, u32]
            lib.orc_delta_step.argtypes = [u32, P, P, P, u32, P, u32, P, ctypes.POINTER(_DStats), u32, P, P]
            lib.orc_features.argtypes = [P, ctypes.c_double, i, P]
            lib.orc_features.restype = None
            lib.orc_mlp_choice.argtypes = [P, P, i, P]
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    return (int(g.n), np.ascontiguousarray(g.row_ptr, np.uint64), np.ascontiguousarray(g.col, np.uint32),
            np.ascontiguousarray(g.w, np.uint32))


def validate(g) -> bool:
    n, rp, col, _ = _csr(g)
    return _L().orc_validate(n, _p(rp), _p(col) if col.size else None) == 0


def dijkstra(g, src: int):
    """(dist u64[n] with INF for unreachable, hops u32[n]) -- Section 2."""
    n, rp, col, w = _csr(g)
    dist = np.empty(n, np.uint64)
    hops = np.empty(n, np.uint32)
    rc = _L().orc_dijkstra(n, _p(rp), _p(col), _p(w), src, _p(dist), _p(hops))
    if rc < 0:
        raise RuntimeError("orc_dijkstra failed: %d" % rc)
    return dist, hops


def bellman_ford(g, src: int) -> np.ndarray:
    n, rp, col, w = _csr(g)
    dist = np.empty(n, np.uint64)
    rc = _L().orc_bellman_ford(n, _p(rp), _p(col), _p(w), src, _p(dist))
    if rc != 0:
        raise RuntimeError("orc_bellman_ford failed: %d" % rc)
    return dist


def static_minima(g):
    """(minIn u32[n], minOut u32[n]); 0xFFFFFFFF where a vertex has no such edge."""
    n, rp, col, w = _csr(g)
    mi = np.empty(n, np.uint32)
    mo = np.empty(n, np.uint32)
    if _L().orc_static_minima(n, _p(rp), _p(col), _p(w), _p(mi), _p(mo)) != 0:
        raise RuntimeError("orc_static_minima failed")
    return mi, mo


@dataclass
class PhasedResult:
    dist: np.ndarray
    phases: int
    sum_f: int
    n_reach: int
    m_reach: int
    relax_edges: int
    improving: int
    trace_f: np.ndarray
    trace_s: np.ndarray
    trace_mind: np.ndarray
    trace_counts: np.ndarray | None
    phase_of: np.ndarray
    trace_crit: np.ndarray | None = None
    trace_union: np.ndarray | None = None
    trace_feat: np.ndarray | None = None


class OracleError(RuntimeError):
    pass


_ERRS = {-1: "invalid argument", -2: "out of memory", -10: "unsound: certified vertex not correct",
         -11: "incomplete: a minimum-distance vertex was not certified", -12: "strength chain violated",
         -13: "final distances differ from the reference"}


def phased(g, src: int, crit: int, crit_seq=None, check: bool = False, dist_ref=None,
           trace_cap: int | None = None, mlp_w=None, commit: int = 0, approx_k: int = 0,
           checkpoint: bool = False) -> PhasedResult:
    """Generic phased algorithm of Section 3 with the given criterion bits.

    mlp_w: float32[5382] selector weights; the criterion of each phase is then the selector's
    choice (crit is ignored). commit = K > 0: the choice made for phase K is kept from then on.
    IN_APPROX / OUT_APPROX: the approximate criteria, minima recomputed at the evaluation of a vertex
    with at least approx_k counted changes (0: never).
    checkpoint=True (with mlp_w, crit = STATIC_OR): the learned checkpoint mode -- static phases, the
    selector evaluated after every 16th phase k on checkpoint features (trace_feat row k // 16), and
    the first choice c != 0 at phase k switches every phase from k + 17 on to CHOICE_CRIT[c]."""
    n, rp, col, w = _csr(g)
    mw = None if mlp_w is None else np.ascontiguousarray(mlp_w, np.float32)
    cap = n if trace_cap is None else trace_cap
    dist = np.empty(n, np.uint64)
    tf = np.zeros(cap, np.uint32)
    ts = np.zeros(cap, np.uint32)
    tm = np.zeros(cap, np.uint64)
    tc = np.zeros(8 * cap, np.uint32) if check else None
    seq = None if crit_seq is None else np.ascontiguousarray(crit_seq, np.uint32)
    po = np.zeros(n, np.uint32)
    tcr = np.zeros(cap, np.uint32)
    tun = np.zeros(3 * cap, np.uint32) if check else None
    tft = np.zeros(12 * cap, np.float32) if mw is not None else None
    st = _Stats()
    rc = _L().orc_phased(n, _p(rp), _p(col), _p(w), src, crit, _p(seq), 0 if seq is None else len(seq),
                         int(check), _p(None if dist_ref is None else np.ascontiguousarray(dist_ref, np.uint64)),
                         _p(dist), ctypes.byref(st), cap, _p(tf), _p(ts), _p(tm), _p(tc), _p(po), _p(mw), _p(tcr),
                         _p(tun), _p(tft), int(commit), int(approx_k), int(checkpoint))
    if rc != 0:
        raise OracleError("orc_phased: %s (%d)" % (_ERRS.get(rc, "?"), rc))
    k = min(st.phases, cap)
    return PhasedResult(dist, int(st.phases), int(st.sum_f), int(st.n_reach), int(st.m_reach),
                        int(st.relax_edges), int(st.improving), tf[:k], ts[:k], tm[:k],
                        None if tc is None else tc[:8 * k].reshape(k, 8), po, tcr[:k],
                        None if tun is None else tun[:3 * k].reshape(k, 3),
                        None if tft is None else tft[:12 * k].reshape(k, 12))


@dataclass
class DeltaResult:
    dist: np.ndarray
    rounds: int
    buckets: int
    light_relax: int
    heavy_relax: int
    sum_frontier: int
    trace_delta: np.ndarray


def delta_step(g, src: int, deltas, trace_cap: int = 0, mlp_w=None) -> DeltaResult:
    """Delta-stepping; bucket b uses deltas[min(b, len-1)], or the selector's choice when mlp_w is given."""
    n, rp, col, w = _csr(g)
    ds = np.ascontiguousarray(np.atleast_1d(deltas if deltas is not None else [1]), np.uint64)
    mw = None if mlp_w is None else np.ascontiguousarray(mlp_w, np.float32)
    dist = np.empty(n, np.uint64)
    td = np.zeros(max(trace_cap, 1), np.uint64)
    st = _DStats()
    rc = _L().orc_delta_step(n, _p(rp), _p(col), _p(w), src, _p(ds), len(ds), _p(dist), ctypes.byref(st),
                             trace_cap, _p(td), _p(mw))
    if rc != 0:
        raise OracleError("orc_delta_step: %s (%d)" % (_ERRS.get(rc, "?"), rc))
    return DeltaResult(dist, int(st.rounds), int(st.buckets), int(st.light_relax), int(st.heavy_relax),
                       int(st.sum_frontier), td[:min(trace_cap, st.buckets)])


def reach_stats(g, dist):
    """(n_reach, m_reach): reachable vertices and the out-edges they own."""
    reach = dist != INF
    return int(reach.sum()), int(np.diff(g.row_ptr)[reach].sum())


MLP_NPARAM = 64 * 12 + 64 + 64 * 64 + 64 + 6 * 64 + 6
CHOICE_CRIT = [STATIC_OR, SIMPLE_OR, IN_SIMPLE | OUT_STATIC]


def features(ints, Wm: float, delta_mode: int = 0) -> np.ndarray:
    """The 12 selector features of one state; ints = (n m F S R a t SD DG Fp D Sp Ip Op k);
    delta_mode 0: phased solver, 1: Delta-stepping bucket start, 2: checkpoint (x5 = floor(log2 n)/32,
    x6 = min(m/n, 64)/64, x7 = x8 = 0)."""
    a = np.ascontiguousarray(ints, np.uint64)
    x = np.zeros(12, np.float32)
    _L().orc_features(_p(a), float(Wm), int(delta_mode), _p(x))
    return x


def mlp_choice(wts, x, lo: int = 0):
    """FP32 forward pass of the selector; (argmax over outputs lo..lo+2, logits)."""
    wv = np.ascontiguousarray(wts, np.float32)
    xv = np.ascontiguousarray(x, np.float32)
    z = np.zeros(6, np.float32)
    c = _L().orc_mlp_choice(_p(wv), _p(xv), lo, _p(z))
    return int(c), z
