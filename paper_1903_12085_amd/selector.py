"""Training pipeline of the per-phase selector (host logic; every solve and every training step
runs in libsssp's HIP kernels).

Data comes from the solver itself: `trace_learned` runs a phased solve under a fixed policy and
records, for every phase, the 12 features its choice is made from. Each training graph is solved
with each fixed criterion (IN-STATIC|OUT-STATIC, IN-SIMPLE|OUT-SIMPLE, IN|OUT), and every phase of
its three fixed-policy traces is labelled with the criterion whose fixed solve of that graph was
fastest on the GPU; the network learns which criterion suits the state it sees. For
Delta-stepping, every bucket start of a graph is labelled with the width (2^12, 2^14 or 2^16) whose
fixed run was fastest on that graph.
"""
from __future__ import annotations

import os
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


def measure(dg, src: int, reps: int = 3) -> dict:
    """Per criterion: the fixed-policy trace (features, counts, |F| per phase), the kernel time
    of every phase of the same fixed-criterion solve, and its total time (best of reps); per bucket
    width: fixed Delta-stepping time."""
    dist = B.new_dist(dg.n)
    out = {"n": dg.n, "time": [], "trace": [], "delta_time": []}
    for c, crit in enumerate(B.CHOICE_CRIT):
        r, feat, cnt = B.trace_learned(dg, src, B.Selector(constant_weights(c)), cap=dg.n + 2)
        fringe = r.trace["fringe"].astype(np.float64)
        dg.profile(True)
        try:
            ph = B.solve(dg, src, crit, dist).phases
            ms = dg.phase_times().astype(np.float64)
        finally:
            dg.profile(False)
        if ph != len(fringe) or len(ms) != len(fringe):
            raise RuntimeError("fixed solve and fixed-policy trace disagree on the phase count")
        settled = r.trace["settled"].astype(np.float64)
        out["trace"].append((feat, cnt, fringe, ms * 1e-3, settled, float(r.stats["n_reach"])))
        out["time"].append(_timed(lambda: B.solve(dg, src, crit, dist), reps))
    for delta in B.CHOICE_DELTA:
        out["delta_time"].append(_timed(lambda: B.delta_step(dg, src, delta, dist), reps))
    return out


def collect(m: dict):
    """Training rows (features, label) of one graph: the phases of its three fixed-policy traces,
    each labelled with the criterion whose fixed solve of this graph was fastest."""
    best = int(np.argmin(m["time"]))
    X = [tr[0] for tr in m["trace"]]
    y = [np.full(len(tr[0]), best, np.int32) for tr in m["trace"]]
    return X, y, best


def collect_delta(dg, src: int, measured: dict):
    best = int(np.argmin(measured["delta_time"]))
    _, feat, _ = B.trace_learned(dg, src, B.Selector(constant_weights(3 + best)), delta_mode=True, cap=dg.n + 2)
    return feat, np.full(feat.shape[0], 3 + best, np.int32)


def training_graphs():
    """Training workloads (seeds distinct from every evaluation graph) at the evaluation scales and
    below: random graphs 2^16..2^21, R-MAT 16..20, grids 256^2..1024^2."""
    import graphgen as G
    return [G.er(1 << 16, 16, 1, (1 << 20) - 1, 102), G.er(1 << 18, 8, 1, (1 << 20) - 1, 108),
            G.er(1 << 20, 16, 1, (1 << 20) - 1, 103), G.er(1 << 21, 16, 1, (1 << 20) - 1, 113),
            G.rmat(16, 16, 1, (1 << 20) - 1, 109), G.rmat(18, 16, 1, (1 << 20) - 1, 105),
            G.rmat(20, 16, 1, (1 << 20) - 1, 114),
            G.grid(256, 256, 1, 1 << 16, 111), G.grid(512, 512, 1, 1 << 16, 107),
            G.grid(1024, 1024, 1, 1 << 16, 115)]


def build_training_set(graphs=None, sources_per_graph: int = 1, log=None):
    """(X, y) from traces of the training graphs."""
    import graphgen as G
    graphs = training_graphs() if graphs is None else graphs
    Xs, ys = [], []
    for g in graphs:
        dg = B.DeviceGraph.from_graph(g)
        for s in G.sources(g, sources_per_graph, 5):
            m = measure(dg, int(s))
            X, y, model = collect(m)
            Xd, yd = collect_delta(dg, int(s), m)
            Xs += X + [Xd]
            ys += y + [yd]
            if log:
                lab = np.bincount(np.concatenate(y + [yd]), minlength=6).tolist()
                log("trace %s src %d: fixed ms %s, labels %s" % (g.name, s, [round(t * 1e3, 2) for t in m["time"]], lab))
        del dg
    return np.concatenate(Xs), np.concatenate(ys)


def train(X, y, seed: int = 0, epochs: int = 60, batch: int = 256, lr: float = 3e-3):
    """A selector trained with the library's HIP kernels (Adam, shuffled minibatches)."""
    sel = B.Selector(he_init(seed))
    loss = sel.train(X, y, epochs=epochs, batch=min(batch, len(y)), lr=lr, seed=seed)
    return sel, loss


# Phases the selector chooses one by one in committed mode before its choice is kept.
COMMIT_PHASES = 32
# After a committed static choice: IN_SIMPLE | OUT_STATIC once |F| has fallen to half its peak.
SWITCH = (B.IN_SIMPLE | B.OUT_STATIC, 1, 2)


def evaluate(sel, dg, src: int, reps: int = 2) -> dict:
    """Learned solves (per phase, and committed after COMMIT_PHASES phases) against the fixed
    criteria / widths on one graph (times in ms)."""
    dist = B.new_dist(dg.n)
    res = {}
    ph = []
    res["learned_ms"] = 1e3 * _timed(lambda: ph.append(B.solve_learned(dg, src, sel, dist).phases), reps)
    res["learned_phases"] = ph[-1]
    ph = []
    res["learned_commit_ms"] = 1e3 * _timed(
        lambda: ph.append(B.solve_learned(dg, src, sel, dist, commit=COMMIT_PHASES).phases), reps)
    res["learned_commit_phases"] = ph[-1]
    ph = []
    res["learned_switch_ms"] = 1e3 * _timed(
        lambda: ph.append(B.solve_learned(dg, src, sel, dist, commit=COMMIT_PHASES, switch=SWITCH).phases), reps)
    res["learned_switch_phases"] = ph[-1]
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


WEIGHTS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.npy")


def evaluation_graphs():
    """Held-out workloads (seeds used by no training graph): random graph 2^22 out-degree 16,
    R-MAT 20, grid 1024^2."""
    import graphgen as G
    return [G.er(1 << 22, 16, 1, (1 << 20) - 1, 2), G.rmat(20, 16, 1, (1 << 20) - 1, 2),
            G.grid(1024, 1024, 1, 1 << 16, 2)]


def load_trained() -> "B.Selector":
    """The selector trained by `python -m paper_1903_12085_amd.selector` (weights file in the package)."""
    return B.Selector(np.load(WEIGHTS_FILE))


def main(argv=None):
    import argparse
    import json
    import graphgen as G
    ap = argparse.ArgumentParser(description="train the per-phase selector on the GPU and save its weights")
    ap.add_argument("--out", default=WEIGHTS_FILE)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-eval", action="store_true")
    args = ap.parse_args(argv)
    t = time.time()
    X, y = build_training_set(log=print)
    sel, loss = train(X, y, seed=args.seed)
    acc = float((sel.forward(X).argmax(1) == y).mean())
    print("trained on %d phases in %.1fs: loss %.4f, accuracy %.3f" % (len(y), time.time() - t, loss, acc))
    np.save(args.out, sel.weights())
    if not args.no_eval:
        for g in evaluation_graphs():
            dg = B.DeviceGraph.from_graph(g)
            print(g.name, json.dumps({k: (round(v, 3) if isinstance(v, float) else v)
                                      for k, v in evaluate(sel, dg, int(G.sources(g, 1, 5)[0])).items()}))


if __name__ == "__main__":
    main()
