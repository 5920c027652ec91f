"""Training pipeline of the selector (host logic; every solve and every training step runs in
libsssp's HIP kernels).

The network is used at checkpoints (sssp_solve_learned_checkpoint): a plain IN-STATIC|OUT-STATIC
solve asks it after every 16th phase whether to keep the static criterion (output 0) or to switch,
for the rest of the solve, to IN-SIMPLE|OUT-SIMPLE (1) or IN-SIMPLE|OUT-STATIC (2). The stronger
criteria of Section 3 certify far more per phase once most vertices are settled, but cost more per
phase while the queue is large, so the best switch point depends on the graph and on its state.

Labels come from the solver itself, per checkpoint. For a training graph, fixed two-stage schedules
(sssp_solve_schedule: static until phase c, then criterion X) are timed on the GPU for candidate
switch phases c that a checkpoint can produce (c = 16 (j + 2) for checkpoint j) and both stronger
criteria, next to the plain static solve. With (c*, X*) the fastest schedule, checkpoint j is
labelled X* if 16 (j + 2) >= c*, else 0 (all 0 when no schedule beats the plain static solve): its
label is the choice that leads to the fastest remaining solve among those that switch at or after
it. The checkpoint features come from a checkpoint solve whose network always answers 0. For
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


def candidate_checkpoints(phases: int, most: int = 24) -> list:
    """Checkpoints j (switch phase 16 (j + 2) < phases) whose schedules are timed: all of them for
    short solves, else a geometric subset."""
    last = (phases - 1) // 16 - 2
    if last < 0:
        return []
    if last + 1 <= most:
        return list(range(last + 1))
    pts = np.unique(np.round(np.geomspace(1, last + 1, most)).astype(int) - 1)
    return [int(x) for x in pts]


def measure(dg, src: int, reps: int = 2) -> dict:
    """Plain static time and phases, the checkpoint features of the static solve, the times of the
    two-stage schedules at the candidate checkpoints, and the fixed Delta-stepping times."""
    dist = B.new_dist(dg.n)
    static = B.STATIC_OR
    t_static = _timed(lambda: B.solve(dg, src, static, dist), reps)
    phases = B.solve(dg, src, static, dist).phases
    r, feat = B.solve_checkpoint(dg, src, B.Selector(constant_weights(0)), dist, trace_cap=phases // 16 + 2,
                                 features=True)
    if r.phases != phases:
        raise RuntimeError("checkpoint solve with a static-only network took a different number of phases")
    sched = {}
    for j in candidate_checkpoints(phases):
        for x in (1, 2):
            sched[(j, x)] = _timed(lambda: B.solve_schedule(dg, src, static, B.CHOICE_CRIT[x], 16 * (j + 2), dist),
                                   reps)
    out = {"n": dg.n, "phases": phases, "static": t_static, "features": feat, "schedules": sched,
           "delta_time": [_timed(lambda: B.delta_step(dg, src, d, dist), reps) for d in B.CHOICE_DELTA]}
    return out


# A schedule must beat the plain static solve by this fraction to label a switch (timing noise).
LABEL_MARGIN = 0.02


def collect(m: dict):
    """Training rows (checkpoint features, label) of one graph and source: checkpoint j is labelled
    with the second criterion of the fastest schedule if that schedule switches at or before
    16 (j + 2) and beats the static solve by LABEL_MARGIN, else 0 (keep static)."""
    best_t, best = m["static"] * (1.0 - LABEL_MARGIN), None
    for key, t in m["schedules"].items():
        if t < best_t:
            best_t, best = t, key
    if best is None:
        best_t = m["static"]
    feat = m["features"]
    y = np.zeros(len(feat), np.int32)
    if best is not None:
        j_star, x_star = best
        y[j_star:] = x_star
    return feat, y, best, best_t


def collect_delta(dg, src: int, measured: dict):
    best = int(np.argmin(measured["delta_time"]))
    _, feat, _ = B.trace_learned(dg, src, B.Selector(constant_weights(3 + best)), delta_mode=True, cap=dg.n + 2)
    return feat, np.full(feat.shape[0], 3 + best, np.int32)


def training_graphs():
    """Training workloads (seeds distinct from every evaluation graph), one at a time, at and below
    the evaluation scales: random graphs 2^16..2^22, R-MAT 16..21, grids 256^2..2048^2."""
    import graphgen as G
    yield G.er(1 << 16, 16, 1, (1 << 20) - 1, 102)
    yield G.er(1 << 18, 8, 1, (1 << 20) - 1, 108)
    yield G.er(1 << 20, 16, 1, (1 << 20) - 1, 103)
    yield G.er(1 << 21, 16, 1, (1 << 20) - 1, 113)
    yield G.er(1 << 22, 16, 1, (1 << 20) - 1, 117)
    yield G.rmat(16, 16, 1, (1 << 20) - 1, 109)
    yield G.rmat(18, 16, 1, (1 << 20) - 1, 105)
    yield G.rmat(20, 16, 1, (1 << 20) - 1, 114)
    yield G.rmat(21, 16, 1, (1 << 20) - 1, 118)
    yield G.grid(256, 256, 1, 1 << 16, 111)
    yield G.grid(512, 512, 1, 1 << 16, 107)
    yield G.grid(1024, 1024, 1, 1 << 16, 115)
    yield G.grid(2048, 2048, 1, 1 << 16, 116)


def build_training_set(graphs=None, sources_per_graph: int = 1, log=None):
    """(X, y) from the training graphs: checkpoint rows and Delta-stepping bucket rows."""
    import graphgen as G
    graphs = training_graphs() if graphs is None else graphs
    Xs, ys, groups = [], [], []
    for g in graphs:
        dg = B.DeviceGraph.from_graph(g)
        for s in G.sources(g, sources_per_graph, 5):
            m = measure(dg, int(s))
            X, y, best, best_t = collect(m)
            Xd, yd = collect_delta(dg, int(s), m)
            Xs += [X, Xd]
            ys += [y, yd]
            groups.append((X, y))
            groups.append((Xd, yd))
            if log:
                log("trace %s src %d: %d phases, static %.2f ms, best schedule %s %.2f ms, labels %s"
                    % (g.name, s, m["phases"], m["static"] * 1e3,
                       None if best is None else (16 * (best[0] + 2), best[1]), best_t * 1e3,
                       np.bincount(np.concatenate([y, yd]), minlength=6).tolist()))
        del dg
    return balance([x for x, _ in groups], [y for _, y in groups])


def balance(Xs, ys, per: int = 512, seed: int = 0):
    """Each group of rows (one graph and source, or its bucket starts) repeated or subsampled to
    `per` rows, so that long solves (grids: hundreds of checkpoints) do not drown short ones."""
    rng = np.random.default_rng(seed)
    X, y = [], []
    for a, b in zip(Xs, ys):
        if len(b) == 0:
            continue
        idx = rng.choice(len(b), per, replace=len(b) < per)
        X.append(a[idx])
        y.append(b[idx])
    return np.concatenate(X), np.concatenate(y)


def train(X, y, seed: int = 0, epochs: int = 60, batch: int = 256, lr: float = 3e-3):
    """A selector trained with the library's HIP kernels (Adam, shuffled minibatches)."""
    sel = B.Selector(he_init(seed))
    loss = sel.train(X, y, epochs=epochs, batch=min(batch, len(y)), lr=lr, seed=seed)
    return sel, loss


# Phases the selector chooses one by one in committed mode before its choice is kept.
COMMIT_PHASES = 32
# After a committed static choice: IN_SIMPLE | OUT_STATIC once |F| has fallen to half its peak.
SWITCH = (B.IN_SIMPLE | B.OUT_STATIC, 1, 2)


def evaluate(sel, dg, src: int, reps: int = 2, per_phase: bool = True) -> dict:
    """On one graph (times in ms, best of reps): the network-only checkpoint solve against the plain
    static solve, the hand-set switch (SWITCH) and the two stronger criteria from the start; the
    per-phase learned solve and learned Delta-stepping against the fixed widths. The switch phase
    of the checkpoint solve comes from one more, traced run (tracing is outside the timed runs)."""
    dist = B.new_dist(dg.n)
    res = {}

    def t(name, fn):
        box = []
        res[name + "_ms"] = 1e3 * _timed(lambda: box.append(fn()), reps)
        res[name + "_phases"] = box[-1].phases
        return box[-1]

    t("static_or", lambda: B.solve(dg, src, B.STATIC_OR, dist))
    t("hand_switch", lambda: B.solve_switch(dg, src, B.STATIC_OR, SWITCH[0], SWITCH[1:], dist))
    t("simple_or", lambda: B.solve(dg, src, B.SIMPLE_OR, dist))
    t("in_simple_out_static", lambda: B.solve(dg, src, B.CHOICE_CRIT[2], dist))
    r = t("checkpoint", lambda: B.solve_checkpoint(dg, src, sel, dist))
    rt = B.solve_checkpoint(dg, src, sel, dist, trace_cap=r.phases + 16)
    crit = [int(c) for c in rt.trace["criterion"]]
    sw = next((k for k, c in enumerate(crit) if c != B.STATIC_OR), None)
    res["checkpoint_switch_phase"] = sw
    res["checkpoint_switch_to"] = None if sw is None else B.CHOICE_CRIT.index(crit[sw])
    if per_phase:
        t("learned", lambda: B.solve_learned(dg, src, sel, dist))
    t("learned_delta", lambda: B.delta_step_learned(dg, src, sel, dist))
    for delta in B.CHOICE_DELTA:
        res["delta_%d_ms" % delta] = 1e3 * _timed(lambda: B.delta_step(dg, src, delta, dist), reps)
    res["checkpoint_over_static"] = res["checkpoint_ms"] / res["static_or_ms"]
    res["checkpoint_over_hand_switch"] = res["checkpoint_ms"] / res["hand_switch_ms"]
    return res


WEIGHTS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.npy")


def evaluation_graphs():
    """Held-out workloads (seeds used by no training graph), one at a time: random graph 2^23
    out-degree 16, R-MAT 23, grid 4096^2 (weights as in training)."""
    import graphgen as G
    yield G.er(1 << 23, 16, 1, (1 << 20) - 1, 2)
    yield G.rmat(23, 16, 1, (1 << 20) - 1, 2)
    yield G.grid(4096, 4096, 1, 1 << 16, 2)


def load_trained() -> "B.Selector":
    """The selector trained by `python -m paper_1903_12085_amd.selector` (weights file in the package)."""
    return B.Selector(np.load(WEIGHTS_FILE))


def main(argv=None):
    import argparse
    import json
    import graphgen as G
    ap = argparse.ArgumentParser(description="train the selector on the GPU and save its weights")
    ap.add_argument("--out", default=WEIGHTS_FILE)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--data", default=None, help="save (or, with --reuse, load) the training rows here (.npz)")
    ap.add_argument("--reuse", action="store_true", help="train on the rows in --data instead of measuring")
    ap.add_argument("--weights", default=None, help="evaluate these weights instead of training")
    ap.add_argument("--no-eval", action="store_true")
    args = ap.parse_args(argv)
    t = time.time()
    if args.weights:
        sel = B.Selector(np.load(args.weights))
    else:
        if args.reuse:
            z = np.load(args.data)
            X, y = z["X"], z["y"]
        else:
            X, y = build_training_set(log=lambda *a: print(*a, flush=True))
            if args.data:
                np.savez(args.data, X=X, y=y)
        sel, loss = train(X, y, seed=args.seed)
        acc = float((sel.forward(X).argmax(1) == y).mean())
        print("trained on %d rows in %.1fs: loss %.4f, accuracy %.3f, labels %s"
              % (len(y), time.time() - t, loss, acc, np.bincount(y, minlength=6).tolist()), flush=True)
        np.save(args.out, sel.weights())
    if not args.no_eval:
        for g in evaluation_graphs():
            dg = B.DeviceGraph.from_graph(g)
            print(g.name, json.dumps({k: (round(v, 3) if isinstance(v, float) else v)
                                      for k, v in evaluate(sel, dg, int(G.sources(g, 1, 5)[0])).items()}),
                  flush=True)
            del dg


if __name__ == "__main__":
    main()
