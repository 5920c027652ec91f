"""ctypes binding of libsssp.so (the C ABI declared in include/sssp.h).

Argument marshalling only: every step of every solve runs in the library's
HIP kernels. PyTorch provides device memory and the stream. If the library is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsssp.so")

# Criterion bits (include/sssp.h)
DIJK, IN_STATIC, OUT_STATIC, IN_SIMPLE, OUT_SIMPLE, IN_FULL, OUT_WEAK, OUT_FULL = (1 << i for i in range(8))
CRIT_NAMES = ["DIJK", "IN_STATIC", "OUT_STATIC", "IN_SIMPLE", "OUT_SIMPLE", "IN_FULL", "OUT_WEAK", "OUT_FULL"]
CRIT = {name: 1 << i for i, name in enumerate(CRIT_NAMES)}
STATIC_OR = IN_STATIC | OUT_STATIC
SIMPLE_OR = IN_SIMPLE | OUT_SIMPLE
FULL_OR = IN_FULL | OUT_FULL
IN_APPROX, OUT_APPROX = 1 << 8, 1 << 9  # approximate criteria (sssp_solve_approx)

SYMBOLS = ["sssp_graph_create", "sssp_graph_destroy", "sssp_set_stream", "sssp_graph_minima", "sssp_solve",
           "sssp_solve_ex", "sssp_delta_step", "sssp_delta_step_ex", "sssp_solve_batch", "sssp_last_error",
           "sssp_profile_enable", "sssp_profile_get", "sssp_profile_phases", "sssp_solve_oracle",
           "sssp_get_launch", "sssp_set_launch",
           "sssp_solve_batch_ex", "sssp_batch_set_config", "sssp_batch_get_config", "sssp_autotune",
           "sssp_autotune_batch", "sssp_selector_create", "sssp_selector_destroy", "sssp_selector_get_weights",
           "sssp_selector_set_weights", "sssp_selector_forward", "sssp_selector_grad", "sssp_selector_train",
           "sssp_solve_learned", "sssp_delta_step_learned", "sssp_trace_learned",
           "sssp_solve_learned_commit", "sssp_measure_atomic_min", "sssp_solve_switch",
           "sssp_solve_learned_switch", "sssp_solve_approx", "sssp_solve_noalloc",
           "sssp_solve_schedule", "sssp_solve_learned_checkpoint"]

ERRORS = {-1: "SSSP_ERR_INVALID", -2: "SSSP_ERR_OOM", -3: "SSSP_ERR_DEVICE", -4: "SSSP_ERR_UNSUPPORTED",
          -5: "SSSP_ERR_INTERNAL"}


class SsspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("phases", ctypes.c_uint32), ("buckets", ctypes.c_uint32), ("sum_f", ctypes.c_uint64),
                ("n_reach", ctypes.c_uint64), ("m_reach", ctypes.c_uint64), ("relax_edges", ctypes.c_uint64),
                ("improving", ctypes.c_uint64), ("precompute_ns", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class KernelProfile(ctypes.Structure):
    _fields_ = [("phases", ctypes.c_uint32), ("term_ms", ctypes.c_float), ("identify_ms", ctypes.c_float),
                ("relax_ms", ctypes.c_float)]

    def as_dict(self):
        return {k: (int(getattr(self, k)) if k == "phases" else float(getattr(self, k))) for k, _ in self._fields_}


class LaunchCfg(ctypes.Structure):
    _fields_ = [("scan_blocks", ctypes.c_uint32), ("relax_blocks", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("queue", ctypes.c_uint32), ("single", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class BatchCfg(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("split", ctypes.c_uint32), ("blocks", ctypes.c_uint32),
                ("team_edges", ctypes.c_uint32), ("team_size", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


PHASE_REC = np.dtype([("min_d", np.uint64), ("fringe", np.uint32), ("settled", np.uint32),
                      ("criterion", np.uint32), ("edges", np.uint32)])

_lib = None


def load(path: str = LIB_PATH):
    """Load libsssp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsssp.so not built (%s); run paper_1903_12085_amd.build.build()" % path)
    # torch first: its HIP runtime is then the one libsssp resolves to, so device memory, streams
    # and the library's kernels all live in one runtime of the process
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, u32, u64, i = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.sssp_graph_create.argtypes = [u32, u64, P, P, P, i, P, ctypes.POINTER(P)]
    lib.sssp_graph_destroy.argtypes = [P]
    lib.sssp_set_stream.argtypes = [P, P]
    lib.sssp_graph_minima.argtypes = [P, P, P]
    lib.sssp_solve.argtypes = [P, u32, u32, P, P]
    lib.sssp_solve_noalloc.argtypes = [P, u32, u32, P, P]
    lib.sssp_solve_schedule.argtypes = [P, u32, u32, u32, u32, P, ctypes.POINTER(Stats), P, P, u32]
    lib.sssp_solve_learned_checkpoint.argtypes = [P, u32, P, P, ctypes.POINTER(Stats), P, P, u32, P]
    lib.sssp_solve_approx.argtypes = [P, u32, u32, u32, P, ctypes.POINTER(Stats), P, P, u32]
    lib.sssp_solve_ex.argtypes = [P, u32, u32, P, ctypes.POINTER(Stats), P, P, u32]
    lib.sssp_delta_step.argtypes = [P, u32, u64, P, P]
    lib.sssp_solve_oracle.argtypes = [P, u32, P, P, ctypes.POINTER(Stats), P]
    lib.sssp_delta_step_ex.argtypes = [P, u32, P, u32, P, ctypes.POINTER(Stats), P, u32]
    lib.sssp_solve_batch.argtypes = [P, P, u32, u32, P, P]
    lib.sssp_profile_enable.argtypes = [P, i]
    lib.sssp_profile_get.argtypes = [P, ctypes.POINTER(KernelProfile)]
    lib.sssp_profile_phases.argtypes = [P, P, u32, ctypes.POINTER(ctypes.c_uint32)]
    lib.sssp_get_launch.argtypes = [P, ctypes.POINTER(LaunchCfg)]
    lib.sssp_set_launch.argtypes = [P, ctypes.POINTER(LaunchCfg)]
    lib.sssp_solve_batch_ex.argtypes = [P, P, u32, u32, P, P, ctypes.POINTER(BatchCfg)]
    lib.sssp_batch_set_config.argtypes = [ctypes.POINTER(BatchCfg)]
    lib.sssp_batch_get_config.argtypes = [ctypes.POINTER(BatchCfg)]
    lib.sssp_autotune.argtypes = [P, u32, u32, ctypes.POINTER(LaunchCfg), ctypes.POINTER(ctypes.c_float)]
    lib.sssp_autotune_batch.argtypes = [P, P, u32, u32, P, ctypes.POINTER(BatchCfg), ctypes.POINTER(ctypes.c_float)]
    f32p = ctypes.POINTER(ctypes.c_float)
    lib.sssp_selector_create.argtypes = [P, ctypes.POINTER(P)]
    lib.sssp_selector_destroy.argtypes = [P]
    lib.sssp_selector_get_weights.argtypes = [P, P]
    lib.sssp_selector_set_weights.argtypes = [P, P]
    lib.sssp_selector_forward.argtypes = [P, P, u32, P]
    lib.sssp_selector_grad.argtypes = [P, P, P, u32, f32p, P]
    lib.sssp_selector_train.argtypes = [P, P, P, u32, u32, u32, ctypes.c_float, u64, f32p]
    lib.sssp_solve_learned.argtypes = [P, u32, P, P, ctypes.POINTER(Stats), P, P, u32]
    lib.sssp_solve_learned_commit.argtypes = [P, u32, P, u32, P, ctypes.POINTER(Stats), P, P, u32]
    lib.sssp_delta_step_learned.argtypes = [P, u32, P, P, ctypes.POINTER(Stats), P, u32]
    lib.sssp_trace_learned.argtypes = [P, u32, P, i, P, ctypes.POINTER(Stats), u32, P, P, P]
    lib.sssp_solve_switch.argtypes = [P, u32, u32, u32, u32, u32, P, ctypes.POINTER(Stats), P, P, u32]
    lib.sssp_solve_learned_switch.argtypes = [P, u32, P, u32, u32, u32, u32, P, ctypes.POINTER(Stats), P, P, u32]
    lib.sssp_measure_atomic_min.argtypes = [P, ctypes.c_uint64, u32, u32, P, ctypes.POINTER(ctypes.c_float)]
    lib.sssp_last_error.restype = ctypes.c_char_p
    lib.sssp_last_error.argtypes = []
    for name in SYMBOLS:
        getattr(lib, name)
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise SsspError(rc, load().sssp_last_error().decode(errors="replace"))


def _stream_ptr():
    """torch's current HIP stream (NULL stream when torch sees no GPU: argument checks only)."""
    import torch
    if not torch.cuda.is_available():
        return None
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class DeviceGraph:
    """A graph resident on the GPU (library-owned buffers)."""

    def __init__(self, n, row_ptr, col, w, device_ptrs: bool = False):
        lib = load()
        self.n = int(n)
        self._h = ctypes.c_void_p()
        if device_ptrs:
            m = int(col.numel())
            ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (row_ptr, col, w)]
        else:
            row_ptr = np.ascontiguousarray(row_ptr, np.uint64)
            col = np.ascontiguousarray(col, np.uint32)
            w = np.ascontiguousarray(w, np.uint32)
            m = int(col.size)
            ptrs = [_np_ptr(row_ptr), _np_ptr(col) if m else None, _np_ptr(w) if m else None]
        self.m = m
        _check(lib.sssp_graph_create(self.n, m, ptrs[0], ptrs[1], ptrs[2], int(device_ptrs), _stream_ptr(),
                                     ctypes.byref(self._h)))

    @classmethod
    def from_graph(cls, g):
        return cls(g.n, g.row_ptr, g.col, g.w)

    def close(self):
        if self._h:
            load().sssp_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _bind_stream(self):
        load().sssp_set_stream(self._h, _stream_ptr())

    def profile(self, enable: bool):
        _check(load().sssp_profile_enable(self._h, int(enable)))

    def last_profile(self) -> dict:
        p = KernelProfile()
        _check(load().sssp_profile_get(self._h, ctypes.byref(p)))
        return p.as_dict()

    def phase_times(self) -> np.ndarray:
        """Per-phase kernel milliseconds of the last phased solve run with profile(True)."""
        cnt = ctypes.c_uint32(0)
        _check(load().sssp_profile_phases(self._h, None, 0, ctypes.byref(cnt)))
        ms = np.zeros(cnt.value, np.float32)
        _check(load().sssp_profile_phases(self._h, _np_ptr(ms), cnt.value, ctypes.byref(cnt)))
        return ms

    def launch(self) -> dict:
        c = LaunchCfg()
        _check(load().sssp_get_launch(self._h, ctypes.byref(c)))
        return c.as_dict()

    def set_launch(self, **kw):
        c = LaunchCfg()
        _check(load().sssp_get_launch(self._h, ctypes.byref(c)))
        for k, v in kw.items():
            setattr(c, k, int(v))
        _check(load().sssp_set_launch(self._h, ctypes.byref(c)))

    def minima(self):
        import torch
        mi = torch.empty(self.n, dtype=torch.int32, device="cuda")
        mo = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self._bind_stream()
        _check(load().sssp_graph_minima(self._h, ctypes.c_void_p(mi.data_ptr()), ctypes.c_void_p(mo.data_ptr())))
        return mi, mo


def new_dist(n):
    """Device buffer for n uint64 distances (int64 storage, reinterpret on the host)."""
    import torch
    return torch.empty(n, dtype=torch.int64, device="cuda")


def to_u64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


@dataclass
class SolveResult:
    dist: object            # torch int64 device tensor holding uint64 bits
    phases: int
    stats: dict | None = None
    phase_of: object = None
    trace: np.ndarray | None = None

    def dist_u64(self) -> np.ndarray:
        return to_u64(self.dist)


def solve(g: DeviceGraph, source: int, criterion: int, dist=None) -> SolveResult:
    dist = new_dist(g.n) if dist is None else dist
    ph = ctypes.c_uint32(0)
    g._bind_stream()
    _check(load().sssp_solve(g.handle, source, criterion, ctypes.c_void_p(dist.data_ptr()), ctypes.byref(ph)))
    return SolveResult(dist, int(ph.value))


def solve_noalloc(g: DeviceGraph, source: int, criterion: int, dist=None) -> SolveResult:
    """sssp_solve_noalloc: the static-criterion solve with the library's fixed scratch array
    (dist, if given, is the caller's device output; otherwise one is made here)."""
    dist = new_dist(g.n) if dist is None else dist
    ph = ctypes.c_uint32(0)
    g._bind_stream()
    _check(load().sssp_solve_noalloc(g.handle, source, criterion, ctypes.c_void_p(dist.data_ptr()),
                                     ctypes.byref(ph)))
    return SolveResult(dist, int(ph.value))


def solve_ex(g: DeviceGraph, source: int, criterion: int, dist=None, phase_of: bool = False,
             trace_cap: int = 0) -> SolveResult:
    import torch
    dist = new_dist(g.n) if dist is None else dist
    po = torch.empty(g.n, dtype=torch.int32, device="cuda") if phase_of else None
    tr = np.zeros(trace_cap, PHASE_REC) if trace_cap else None
    st = Stats()
    g._bind_stream()
    _check(load().sssp_solve_ex(g.handle, source, criterion, ctypes.c_void_p(dist.data_ptr()), ctypes.byref(st),
                                ctypes.c_void_p(po.data_ptr()) if po is not None else None,
                                _np_ptr(tr), trace_cap))
    if tr is not None:
        tr = tr[:min(st.phases, trace_cap)]
    return SolveResult(dist, int(st.phases), st.as_dict(), po, tr)


def solve_approx(g: DeviceGraph, source: int, criterion: int, k: int, dist=None, phase_of: bool = False,
                 trace_cap: int = 0) -> SolveResult:
    """sssp_solve_approx: the approximate criteria (criterion made of DIJK, IN_APPROX, OUT_APPROX),
    minima recomputed after k counted changes (0: never)."""
    import torch
    dist = new_dist(g.n) if dist is None else dist
    po = torch.empty(g.n, dtype=torch.int32, device="cuda") if phase_of else None
    tr = np.zeros(trace_cap, PHASE_REC) if trace_cap else None
    st = Stats()
    g._bind_stream()
    _check(load().sssp_solve_approx(g.handle, source, criterion, k, ctypes.c_void_p(dist.data_ptr()),
                                    ctypes.byref(st), ctypes.c_void_p(po.data_ptr()) if po is not None else None,
                                    _np_ptr(tr), trace_cap))
    if tr is not None:
        tr = tr[:min(st.phases, trace_cap)]
    return SolveResult(dist, int(st.phases), st.as_dict(), po, tr)


def solve_oracle(g: DeviceGraph, source: int, dist_ref, dist=None, phase_of: bool = True) -> SolveResult:
    """Phased solve with the clairvoyant ORACLE criterion; dist_ref = dist(source, .) as a device
    uint64/int64 tensor (or anything torch.as_tensor accepts, copied to the device)."""
    import torch
    ref = torch.as_tensor(np.asarray(dist_ref).view(np.int64) if not torch.is_tensor(dist_ref) else dist_ref)
    ref = ref.to(device="cuda", dtype=torch.int64).contiguous()
    if ref.numel() != g.n:
        raise ValueError("dist_ref needs %d entries" % g.n)
    dist = new_dist(g.n) if dist is None else dist
    po = torch.empty(g.n, dtype=torch.int32, device="cuda") if phase_of else None
    st = Stats()
    g._bind_stream()
    _check(load().sssp_solve_oracle(g.handle, source, ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                                    ctypes.byref(st), ctypes.c_void_p(po.data_ptr()) if po is not None else None))
    return SolveResult(dist, int(st.phases), st.as_dict(), po, None)


def delta_step(g: DeviceGraph, source: int, delta: int, dist=None) -> SolveResult:
    dist = new_dist(g.n) if dist is None else dist
    ph = ctypes.c_uint32(0)
    g._bind_stream()
    _check(load().sssp_delta_step(g.handle, source, int(delta), ctypes.c_void_p(dist.data_ptr()), ctypes.byref(ph)))
    return SolveResult(dist, int(ph.value))


def delta_step_ex(g: DeviceGraph, source: int, deltas, dist=None, trace_cap: int = 0) -> SolveResult:
    dist = new_dist(g.n) if dist is None else dist
    ds = np.ascontiguousarray(np.atleast_1d(deltas), np.uint64)
    tr = np.zeros(trace_cap, PHASE_REC) if trace_cap else None
    st = Stats()
    g._bind_stream()
    _check(load().sssp_delta_step_ex(g.handle, source, _np_ptr(ds), len(ds), ctypes.c_void_p(dist.data_ptr()),
                                     ctypes.byref(st), _np_ptr(tr), trace_cap))
    if tr is not None:
        tr = tr[:min(st.phases, trace_cap)]
    return SolveResult(dist, int(st.phases), st.as_dict(), None, tr)


def _batch_args(graphs, sources, dists):
    nq = len(sources)
    if dists is None:
        dists = [new_dist(g.n) for g in graphs]
    handles = (ctypes.c_void_p * nq)(*[g.handle.value for g in graphs])
    srcs = np.ascontiguousarray(sources, np.uint32)
    outs = (ctypes.c_void_p * nq)(*[d.data_ptr() for d in dists])
    graphs[0]._bind_stream()
    return nq, dists, handles, srcs, outs


def solve_batch(graphs, sources, criterion: int, dists=None, cfg: dict | None = None):
    """graphs: list of DeviceGraph (may repeat), sources: list of ints. Returns (dists, phases)."""
    nq, dists, handles, srcs, outs = _batch_args(graphs, sources, dists)
    phases = np.zeros(nq, np.uint32)
    if cfg is None:
        _check(load().sssp_solve_batch(handles, _np_ptr(srcs), nq, criterion, outs, _np_ptr(phases)))
    else:
        c = BatchCfg(**{k: int(v) for k, v in cfg.items()})
        _check(load().sssp_solve_batch_ex(handles, _np_ptr(srcs), nq, criterion, outs, _np_ptr(phases),
                                          ctypes.byref(c)))
    return dists, phases


def batch_config() -> dict:
    c = BatchCfg()
    _check(load().sssp_batch_get_config(ctypes.byref(c)))
    return c.as_dict()


def set_batch_config(**kw):
    c = BatchCfg(**{k: int(v) for k, v in kw.items()})
    _check(load().sssp_batch_set_config(ctypes.byref(c)))


def autotune(g: DeviceGraph, source: int, criterion: int):
    c, ms = LaunchCfg(), ctypes.c_float(0)
    g._bind_stream()
    _check(load().sssp_autotune(g.handle, source, criterion, ctypes.byref(c), ctypes.byref(ms)))
    return c.as_dict(), float(ms.value)


def autotune_batch(graphs, sources, criterion: int, dists=None):
    nq, dists, handles, srcs, outs = _batch_args(graphs, sources, dists)
    c, ms = BatchCfg(), ctypes.c_float(0)
    _check(load().sssp_autotune_batch(handles, _np_ptr(srcs), nq, criterion, outs, ctypes.byref(c), ctypes.byref(ms)))
    return c.as_dict(), float(ms.value)


SELECTOR_PARAMS = 5382
CHOICE_CRIT = [STATIC_OR, SIMPLE_OR, IN_SIMPLE | OUT_STATIC]
CHOICE_DELTA = [1 << 12, 1 << 14, 1 << 16]


class Selector:
    """The per-phase selector network (device weights owned by the library)."""

    def __init__(self, weights=None):
        self._h = ctypes.c_void_p()
        w = None if weights is None else np.ascontiguousarray(weights, np.float32)
        if w is not None and w.size != SELECTOR_PARAMS:
            raise ValueError("selector needs %d weights" % SELECTOR_PARAMS)
        _check(load().sssp_selector_create(_np_ptr(w), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            load().sssp_selector_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def weights(self) -> np.ndarray:
        w = np.zeros(SELECTOR_PARAMS, np.float32)
        _check(load().sssp_selector_get_weights(self._h, _np_ptr(w)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        _check(load().sssp_selector_set_weights(self._h, _np_ptr(w)))

    def forward(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, np.float32).reshape(-1, 12)
        z = np.zeros((x.shape[0], 6), np.float32)
        _check(load().sssp_selector_forward(self._h, _np_ptr(x), x.shape[0], _np_ptr(z)))
        return z

    def grad(self, x, y):
        x = np.ascontiguousarray(x, np.float32).reshape(-1, 12)
        y = np.ascontiguousarray(y, np.int32)
        g = np.zeros(SELECTOR_PARAMS, np.float32)
        loss = ctypes.c_float(0)
        _check(load().sssp_selector_grad(self._h, _np_ptr(x), _np_ptr(y), x.shape[0], ctypes.byref(loss), _np_ptr(g)))
        return float(loss.value), g

    def train(self, x, y, epochs=20, batch=256, lr=3e-3, seed=0) -> float:
        x = np.ascontiguousarray(x, np.float32).reshape(-1, 12)
        y = np.ascontiguousarray(y, np.int32)
        loss = ctypes.c_float(0)
        _check(load().sssp_selector_train(self._h, _np_ptr(x), _np_ptr(y), x.shape[0], epochs, batch, lr, seed,
                                          ctypes.byref(loss)))
        return float(loss.value)


def solve_learned(g: DeviceGraph, source: int, sel: Selector, dist=None, phase_of: bool = False,
                  trace_cap: int = 0, commit: int = 0, switch=None) -> SolveResult:
    """commit = 0: the selector chooses every phase (sssp_solve_learned); commit = K >= 1: it
    chooses phases 0 .. K - 1, then phase K's choice holds (sssp_solve_learned_commit); with
    switch = (crit_then, num, den) as well, a committed static choice switches to crit_then once
    |F| has fallen to num/den of its peak (sssp_solve_learned_switch)."""
    import torch
    dist = new_dist(g.n) if dist is None else dist
    po = torch.empty(g.n, dtype=torch.int32, device="cuda") if phase_of else None
    tr = np.zeros(trace_cap, PHASE_REC) if trace_cap else None
    st = Stats()
    g._bind_stream()
    po_p = ctypes.c_void_p(po.data_ptr()) if po is not None else None
    if switch is not None:
        _check(load().sssp_solve_learned_switch(g.handle, source, sel.handle, int(commit), int(switch[0]),
                                                int(switch[1]), int(switch[2]), ctypes.c_void_p(dist.data_ptr()),
                                                ctypes.byref(st), po_p, _np_ptr(tr), trace_cap))
    elif commit:
        _check(load().sssp_solve_learned_commit(g.handle, source, sel.handle, int(commit),
                                                ctypes.c_void_p(dist.data_ptr()), ctypes.byref(st), po_p,
                                                _np_ptr(tr), trace_cap))
    else:
        _check(load().sssp_solve_learned(g.handle, source, sel.handle, ctypes.c_void_p(dist.data_ptr()),
                                         ctypes.byref(st), po_p, _np_ptr(tr), trace_cap))
    if tr is not None:
        tr = tr[:min(st.phases, trace_cap)]
    return SolveResult(dist, int(st.phases), st.as_dict(), po, tr)


def solve_switch(g: DeviceGraph, source: int, crit_first: int, crit_then: int, drop=(1, 2), dist=None,
                 phase_of: bool = False, trace_cap: int = 0) -> SolveResult:
    """crit_first until |F| falls to drop[0]/drop[1] of its peak, then crit_then (sssp_solve_switch)."""
    import torch
    dist = new_dist(g.n) if dist is None else dist
    po = torch.empty(g.n, dtype=torch.int32, device="cuda") if phase_of else None
    tr = np.zeros(trace_cap, PHASE_REC) if trace_cap else None
    st = Stats()
    g._bind_stream()
    _check(load().sssp_solve_switch(g.handle, source, crit_first, crit_then, int(drop[0]), int(drop[1]),
                                    ctypes.c_void_p(dist.data_ptr()), ctypes.byref(st),
                                    ctypes.c_void_p(po.data_ptr()) if po is not None else None, _np_ptr(tr),
                                    trace_cap))
    if tr is not None:
        tr = tr[:min(st.phases, trace_cap)]
    return SolveResult(dist, int(st.phases), st.as_dict(), po, tr)


def solve_schedule(g: DeviceGraph, source: int, crit_first: int, crit_then: int, switch_phase: int, dist=None,
                   phase_of: bool = False, trace_cap: int = 0) -> SolveResult:
    """crit_first for phases 0 .. switch_phase - 1, crit_then afterwards (sssp_solve_schedule)."""
    import torch
    dist = new_dist(g.n) if dist is None else dist
    po = torch.empty(g.n, dtype=torch.int32, device="cuda") if phase_of else None
    tr = np.zeros(trace_cap, PHASE_REC) if trace_cap else None
    st = Stats()
    g._bind_stream()
    _check(load().sssp_solve_schedule(g.handle, source, crit_first, crit_then, int(switch_phase),
                                      ctypes.c_void_p(dist.data_ptr()), ctypes.byref(st),
                                      ctypes.c_void_p(po.data_ptr()) if po is not None else None, _np_ptr(tr),
                                      trace_cap))
    if tr is not None:
        tr = tr[:min(st.phases, trace_cap)]
    return SolveResult(dist, int(st.phases), st.as_dict(), po, tr)


def solve_checkpoint(g: DeviceGraph, source: int, sel: Selector, dist=None, phase_of: bool = False,
                     trace_cap: int = 0, features: bool = False):
    """The learned checkpoint solve (sssp_solve_learned_checkpoint). With features=True, returns
    (result, feature rows of the checkpoints) and needs trace_cap >= the number of checkpoints."""
    import torch
    dist = new_dist(g.n) if dist is None else dist
    po = torch.empty(g.n, dtype=torch.int32, device="cuda") if phase_of else None
    tr = np.zeros(trace_cap, PHASE_REC) if trace_cap else None
    feat = np.zeros((trace_cap, 12), np.float32) if features else None
    st = Stats()
    g._bind_stream()
    _check(load().sssp_solve_learned_checkpoint(g.handle, source, sel.handle, ctypes.c_void_p(dist.data_ptr()),
                                                ctypes.byref(st),
                                                ctypes.c_void_p(po.data_ptr()) if po is not None else None,
                                                _np_ptr(tr), trace_cap, _np_ptr(feat)))
    if tr is not None:
        tr = tr[:min(st.phases, trace_cap)]
    r = SolveResult(dist, int(st.phases), st.as_dict(), po, tr)
    if features:
        return r, feat[:min(st.phases // 16, trace_cap)]
    return r


def delta_step_learned(g: DeviceGraph, source: int, sel: Selector, dist=None, trace_cap: int = 0) -> SolveResult:
    dist = new_dist(g.n) if dist is None else dist
    tr = np.zeros(trace_cap, PHASE_REC) if trace_cap else None
    st = Stats()
    g._bind_stream()
    _check(load().sssp_delta_step_learned(g.handle, source, sel.handle, ctypes.c_void_p(dist.data_ptr()),
                                          ctypes.byref(st), _np_ptr(tr), trace_cap))
    if tr is not None:
        tr = tr[:min(st.phases, trace_cap)]
    return SolveResult(dist, int(st.phases), st.as_dict(), None, tr)


def trace_learned(g: DeviceGraph, source: int, sel: Selector, delta_mode: bool = False, cap: int = 1 << 16):
    """(result, features[k][12], counts[k][3] or None): a learned solve that records training data."""
    dist = new_dist(g.n)
    tr = np.zeros(cap, PHASE_REC)
    feat = np.zeros((cap, 12), np.float32)
    cnt = None if delta_mode else np.zeros((cap, 3), np.uint32)
    st = Stats()
    g._bind_stream()
    _check(load().sssp_trace_learned(g.handle, source, sel.handle, int(delta_mode), ctypes.c_void_p(dist.data_ptr()),
                                     ctypes.byref(st), cap, _np_ptr(tr), _np_ptr(feat), _np_ptr(cnt)))
    k = min(st.phases, cap)
    kb = min(st.buckets, cap) if delta_mode else k
    res = SolveResult(dist, int(st.phases), st.as_dict(), None, tr[:k])
    return res, feat[:kb], (None if cnt is None else cnt[:k])


def measure_atomic_min(slots: int, blocks: int, iters: int) -> float:
    """Returning 64-bit atomicMin operations per second (sssp_measure_atomic_min) on `slots`
    distinct addresses, on torch's current stream."""
    import torch
    buf = torch.full((slots,), -1, dtype=torch.int64, device="cuda")
    ms = ctypes.c_float(0)
    _check(load().sssp_measure_atomic_min(ctypes.c_void_p(buf.data_ptr()), slots, blocks, iters,
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                          ctypes.byref(ms)))
    return blocks * 256.0 * iters / (ms.value * 1e-3)
