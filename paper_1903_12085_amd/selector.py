"""Training pipeline of the per-phase selector (host logic; every solve and every training step
runs in libsssp's HIP kernels).

Data comes from the solver itself: `trace_learned` runs a phased solve under a fixed policy and, on
every phase's snapshot, records the 12 features and how many queued vertices each of the three
criteria (IN-STATIC|OUT-STATIC, IN-SIMPLE|OUT-SIMPLE, IN|OUT) would certify. Labels come from a cost
model measured on the GPU: for each criterion c, a phase costs alpha_c + beta_c * |F|, fitted by
least squares to the times of fixed-criterion solves of the training graphs (time = alpha_c *
phases + beta_c * sum of |F|). The label of a phase is the criterion that settles the most
vertices per unit of time, argmax_c count_c / (alpha_c + beta_c * |F|). For Delta-stepping, every
bucket start of a graph is labelled with the width (2^12, 2^14 or 2^16) whose fixed run was
fastest on that graph.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B


def constant_weights(choice: int) -> np.ndarray:
    """Weights of a network whose output `choice` always wins (a fixed policy)."""
    w = np.zeros(B.SELECTOR_PARAMS, np.float32)
    w[-6 + choice] = 10.0
    return w


def he_init(seed: int) -> np.ndarray:
    """He-uniform weights and zero biases (numpy PCG64 stream of `seed`)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in ((64, 12), (64,), (64, 64), (64,), (6, 64), (6,)):
        if len(shape) == 2:
            lim = np.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def _timed(fn, reps: int = 2) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def measure_costs(dg, src: int, reps: int = 2) -> dict:
    """Fixed-criterion solves of one graph: time, phases and summed |F| per criterion; total time
    per bucket width."""
    dist = B.new_dist(dg.n)
    out = {"time": [], "phases": [], "sum_f": [], "delta_time": []}
    for crit in B.CHOICE_CRIT:
        st = B.solve_ex(dg, src, crit, dist).stats
        out["phases"].append(st["phases"])
        out["sum_f"].append(st["sum_f"])
        out["time"].append(_timed(lambda: B.solve(dg, src, crit, dist), reps))
    for delta in B.CHOICE_DELTA:
        out["delta_time"].append(_timed(lambda: B.delta_step(dg, src, delta, dist), reps))
    return out


def fit_cost_model(measured) -> np.ndarray:
    """[3][2] = (alpha_c, beta_c) per criterion: time = alpha * phases + beta * sum|F| (least squares,
    clipped at zero)."""
    model = np.zeros((3, 2))
    for c in range(3):
        A = np.array([[m["phases"][c], m["sum_f"][c]] for m in measured], np.float64)
        t = np.array([m["time"][c] for m in measured], np.float64)
        coef, *_ = np.linalg.lstsq(A, t, rcond=None)
        model[c] = np.maximum(coef, [1e-7, 0.0])
    return model


def collect(dg, src: int, costs: dict, model: np.ndarray, cap: int = 1 << 16):
    """Training rows (features, label) of one graph: phased traces under each fixed policy, and the
    bucket starts of Delta-stepping under the fastest width."""
    X, y = [], []
    for policy in range(3):
        sel = B.Selector(constant_weights(policy))
        r, feat, cnt = B.trace_learned(dg, src, sel, cap=cap)
        fringe = r.trace["fringe"].astype(np.float64)
        cost = model[None, :, 0] + model[None, :, 1] * fringe[:, None]
        rate = cnt.astype(np.float64) / cost
        X.append(feat)
        y.append(np.argmax(rate, axis=1).astype(np.int32))
    best = int(np.argmin(costs["delta_time"]))
    _, feat, _ = B.trace_learned(dg, src, B.Selector(constant_weights(3 + best)), delta_mode=True, cap=cap)
    X.append(feat)
    y.append(np.full(feat.shape[0], 3 + best, np.int32))
    return np.concatenate(X), np.concatenate(y)


def training_graphs():
    """Training workloads (seeds distinct from every evaluation graph): random graphs 2^14..2^20,
    R-MAT 14..18, grids 128^2..512^2."""
    import graphgen as G
    return [G.er(1 << 14, 8, 1, 1000, 101), G.er(1 << 16, 16, 1, (1 << 20) - 1, 102),
            G.er(1 << 20, 16, 1, (1 << 20) - 1, 103), G.rmat(14, 16, 1, (1 << 20) - 1, 104),
            G.rmat(18, 16, 1, (1 << 20) - 1, 105), G.grid(128, 128, 1, 1 << 16, 106),
            G.grid(512, 512, 1, 1 << 16, 107)]


def build_training_set(graphs=None, log=None):
    """(X, y, cost model) from traces of the training graphs."""
    import graphgen as G
    graphs = training_graphs() if graphs is None else graphs
    dgs = [B.DeviceGraph.from_graph(g) for g in graphs]
    srcs = [int(G.sources(g, 1, 5)[0]) for g in graphs]
    measured = [measure_costs(dg, s) for dg, s in zip(dgs, srcs)]
    model = fit_cost_model(measured)
    Xs, ys = [], []
    for g, dg, s, m in zip(graphs, dgs, srcs, measured):
        X, y = collect(dg, s, m, model)
        Xs.append(X)
        ys.append(y)
        if log:
            log("trace %s: %d rows, labels %s" % (g.name, len(y), np.bincount(y, minlength=6).tolist()))
    return np.concatenate(Xs), np.concatenate(ys), model


def train(X, y, seed: int = 0, epochs: int = 60, batch: int = 256, lr: float = 3e-3):
    """A selector trained with the library's HIP kernels (Adam, shuffled minibatches)."""
    sel = B.Selector(he_init(seed))
    loss = sel.train(X, y, epochs=epochs, batch=min(batch, len(y)), lr=lr, seed=seed)
    return sel, loss


def evaluate(sel, dg, src: int, reps: int = 2) -> dict:
    """Learned solves against the fixed criteria / widths on one graph (times in ms)."""
    dist = B.new_dist(dg.n)
    res = {}
    ph = []
    res["learned_ms"] = 1e3 * _timed(lambda: ph.append(B.solve_learned(dg, src, sel, dist).phases), reps)
    res["learned_phases"] = ph[-1]
    for name, crit in zip(("static_or", "simple_or", "full_or"), B.CHOICE_CRIT):
        ph = []
        res[name + "_ms"] = 1e3 * _timed(lambda: ph.append(B.solve(dg, src, crit, dist).phases), reps)
        res[name + "_phases"] = ph[-1]
    ph = []
    res["learned_delta_ms"] = 1e3 * _timed(lambda: ph.append(B.delta_step_learned(dg, src, sel, dist).phases), reps)
    res["learned_delta_rounds"] = ph[-1]
    for delta in B.CHOICE_DELTA:
        res["delta_%d_ms" % delta] = 1e3 * _timed(lambda: B.delta_step(dg, src, delta, dist), reps)
    return res
