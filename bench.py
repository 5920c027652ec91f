#!/usr/bin/env python3
"""Benchmark: GTEPS and phases per SSSP solve on one MI355X.

Workload (the headline configuration): directed random graph, n = 2^22 vertices, each with 16
distinct uniform random out-neighbours, uint32 weights uniform in [1, 2^20), source 0, seed 1;
plain phased solver with the combined IN-STATIC | OUT-STATIC criterion, uint64 distances.
A step = one whole solve (every phase: identify, compaction, relaxation) with the graph already
resident in HBM. GTEPS = out-edges of reachable vertices / solve time.

Also reported (outside the timed region): the other criteria and Delta-stepping on the same
graph, the batched form (512 queries over 64 uneven graphs in one launch), the learned per-phase
selector (headline graph plus held-out R-MAT and grid graphs), the dominant kernel's roofline
fraction (algorithmic bytes / HIP-event kernel time vs the 8 TB/s HBM peak), the whole-solve
fraction of each form (all algorithmic bytes of a solve / its time), the same plain measurement on
the largest random graph (2^23 vertices), switched solves (static criteria, then a stronger one
once the queue has shrunk), R-MAT scale 22 and the 2048^2 grid (plain against Delta-stepping),
and the CPU oracle (binary-heap Dijkstra, one core) timed on the host.

usage: python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu] [--no-extra] [--no-batch]
                      [--no-learned] [--no-c3]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GTEPS + phases per SSSP; plain vs batched/learned on 1 GPU, distances exact"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


GOLDEN = os.path.join(ROOT, "tests", "golden", "full")


def golden(graph, what, src):
    """The oracle's stored expectations for a full-size run (written by tests/golden/make_full_size.py,
    which calls only the oracle and the input generators), or None."""
    path = os.path.join(GOLDEN, "%s_%s_s%d.json" % (graph, what.replace("|", "_"), src))
    return json.load(open(path)) if os.path.exists(path) else None


def dist_sha(d):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(d).astype("<u8").tobytes()).hexdigest()


def exact_vs_golden(graph, src, d):
    """Distances equal to the oracle's for this graph and source (SHA-256 of the uint64 array), or
    None when no stored expectation exists."""
    rec = golden(graph, "dist", src)
    return None if rec is None else dist_sha(d) == rec["sha256"]


def median_time(torch, fn, reps=3):
    """Median wall time (s) of reps calls after one untimed call, and the last result."""
    fn()
    torch.cuda.synchronize()
    ts, r = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], r


class CpuBaseline:
    """The oracle's binary-heap Dijkstra timed on the host, single-threaded per solve: `reps` solves
    of the same graph and source one after the other on one background thread (the C oracle releases
    the interpreter lock), started after the headline's timed region so that it overlaps the later
    GPU legs rather than lengthening the run. Reports the median solve."""

    def __init__(self, g, src, reps=10):
        import threading
        self.g, self.src, self.reps = g, src, reps
        self.times, self.dist, self.err = [], None, None
        self.th = threading.Thread(target=self._run, daemon=True)
        self.th.start()

    def _run(self):
        try:
            import oracle as O
            for _ in range(self.reps):
                t0 = time.perf_counter()
                d, _ = O.dijkstra(self.g, self.src)
                self.times.append(time.perf_counter() - t0)
                self.dist = d
        except Exception as e:  # reported in the JSON line
            self.err = repr(e)

    def result(self, m_reach):
        self.th.join()
        if self.err or not self.times:
            return {"error": self.err or "no solve finished"}
        med = sorted(self.times)[len(self.times) // 2]
        return {"value": round(m_reach / med / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
                "seconds_median": round(med, 3), "seconds_min": round(min(self.times), 3),
                "seconds_max": round(max(self.times), 3), "solves": len(self.times),
                "host_nproc": os.cpu_count(),
                "sample": "%d full solves of the same graph and source with the oracle's binary-heap Dijkstra, one "
                          "thread, one solve at a time on a background thread while the later GPU legs ran; "
                          "median" % len(self.times)}


def alg_bytes(kernel, st, phases):
    """Algorithmic bytes per launch of a phase kernel (per-unit figures from the design notes)."""
    if kernel == "identify":
        return 24.0 * st["sum_f"] / phases  # id 4 + d 8 + minIn 4 + minOut 4 + compacted write 4 per queued vertex
    # relax: per S' vertex 16 B (row range 8, id + snapshot distance 8); per out-edge of S' 16 B
    # (target+weight 8, target distance 8); per improving relaxation 8 B (the atomic write)
    return (16.0 * st["n_reach"] + 16.0 * st["m_reach"] + 8.0 * st["improving"]) / phases


def solve_bytes(st, n):
    """Algorithmic bytes of one whole phased solve: both kernels' per-unit figures summed over the
    phases (every queued vertex once per phase it waits, every reachable vertex and out-edge once,
    every improving relaxation once), plus 16 B per vertex of initialisation (distance, state)."""
    return (24.0 * st["sum_f"] + 16.0 * st["n_reach"] + 16.0 * st["m_reach"] + 8.0 * st["improving"] +
            16.0 * n)


def device_ceilings(B, torch):
    """Measured ceilings of this device: a 1 GiB device-to-device copy (bytes read + written per
    second, median of three) and returning 64-bit atomicMin throughput on random distinct
    addresses (2^22 slots, the size of the headline distance array), on 32 slots and on one."""
    src = torch.empty(1 << 27, dtype=torch.int64, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    copy_gbs = 2.0 * (1 << 30) / (sorted(ts)[1] * 1e-3) / 1e9
    del src, dst
    atom = {"random_2^22_slots_Gops": B.measure_atomic_min(1 << 22, 1024, 64) / 1e9,
            "32_slots_Gops": B.measure_atomic_min(32, 64, 32) / 1e9,
            "1_slot_Gops": B.measure_atomic_min(1, 16, 16) / 1e9}
    return round(copy_gbs, 1), {k: round(v, 3) for k, v in atom.items()}


def solve_frac(st, ms, n):
    """Whole-solve algorithmic bytes per second as a fraction of the 8 TB/s HBM peak."""
    return round(solve_bytes(st, n) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)


def measure_plain(B, torch, dg, src, crit, steps, warmup, record):
    """Timed plain solves (steps after warmup) and the dominant kernel's roofline from a separate
    HIP-event pass over the same solve."""
    dist = B.new_dist(dg.n)
    for _ in range(warmup):
        B.solve(dg, src, crit, dist)
    torch.cuda.synchronize()
    phases = None
    t0 = time.perf_counter()
    for _ in range(steps):
        phases = B.solve(dg, src, crit, dist).phases
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = B.solve_ex(dg, src, crit, dist).stats
    # per-kernel HIP-event timing on the solve stream (same workload, separate pass)
    dg.profile(True)
    for _ in range(max(1, min(steps, 3))):
        B.solve(dg, src, crit, dist)
    torch.cuda.synchronize()
    prof = dg.last_profile()
    dg.profile(False)
    kern = "identify" if prof["identify_ms"] >= prof["relax_ms"] else "relax"
    # with queue arrays on (static criteria) identify runs as k_identify_queue
    kname = "k_identify_queue" if kern == "identify" and dg.launch()["queue"] else "k_" + kern
    per_launch = alg_bytes(kern, st, prof["phases"])
    avg_us = prof[kern + "_ms"] * 1e3 / prof["phases"]
    achieved = per_launch / (avg_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kname, record, dg.launch()),
                "kernel": kname,
                "alg_bytes_per_launch": round(per_launch), "avg_launch_us": round(avg_us, 2),
                "launches": prof["phases"], "identify_ms": round(prof["identify_ms"], 3),
                "relax_ms": round(prof["relax_ms"], 3)}
    return ms, phases, st, roofline, prof, dist


def measured_traffic(kern, record, launch):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE records, or None when the
    kernel source changed since the counters were taken, or no record is for this kernel, size and
    launch shape."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_identify_%s.json" % record)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in ("paper_1903_12085_amd/csrc/phased.hip", "paper_1903_12085_amd/csrc/common.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"] or rec["kernel"] != kern:
        return None
    shape = "%d,%d,%d,%d,%d" % tuple(launch[k] for k in ("scan_blocks", "relax_blocks", "chunk", "use_graph", "queue"))
    for r in rec["by_launch"]:
        if r["launch"] == shape:
            return r["traffic_bytes_per_launch"]
    return None


def bench_batched(B, torch, G):
    """512 queries over 64 uneven graphs: one persistent batched launch vs the same queries one by one."""
    t = time.time()
    graphs, queries = G.batch_workload(seed=7)
    dgs = [B.DeviceGraph.from_graph(g) for g in graphs]
    torch.cuda.synchronize()
    log("batch workload: %d graphs, %d queries, %.1fs" % (len(graphs), len(queries), time.time() - t))
    qg = [dgs[i] for i, _ in queries]
    qs = [s for _, s in queries]
    dists = [B.new_dist(graphs[i].n) for i, _ in queries]
    tuned, tuned_ms = B.autotune_batch(qg, qs, B.STATIC_OR, dists)
    log("batch autotune", tuned, "%.2f ms" % tuned_ms)
    reps = []
    for _ in range(3):
        torch.cuda.synchronize()
        tt = time.perf_counter()
        _, bph = B.solve_batch(qg, qs, B.STATIC_OR, dists)
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - tt)
    tb = sorted(reps)[1]
    m_reach = 0
    for (i, _), d in zip(queries, dists):
        reach = B.to_u64(d) != np.uint64(0xFFFFFFFFFFFFFFFF)
        m_reach += int(np.diff(graphs[i].row_ptr)[reach].sum())
    # the same queries through the plain solver, one call each
    pd = [B.new_dist(graphs[i].n) for i, _ in queries]
    for dg in dgs:  # warm each graph's scratch once
        B.solve(dg, 0, B.STATIC_OR)
    torch.cuda.synchronize()
    tt = time.perf_counter()
    pph = [B.solve(dg, s, B.STATIC_OR, d).phases for dg, s, d in zip(qg, qs, pd)]
    torch.cuda.synchronize()
    tp = time.perf_counter() - tt
    # algorithmic bytes of the same queries, from the plain solver's counts (same phases and F sets)
    qbytes = 0.0
    for dg, s_, d in zip(qg, qs, pd):
        qbytes += solve_bytes(B.solve_ex(dg, s_, B.STATIC_OR, d).stats, dg.n)
    same = all(np.array_equal(B.to_u64(a), B.to_u64(b)) for a, b in zip(dists, pd)) and list(bph) == pph
    gpath = os.path.join(GOLDEN, "batch_c4.json")
    exact = phases_ok = None
    if os.path.exists(gpath):  # every query against the oracle's stored distances and phase count
        grec = json.load(open(gpath))["queries"]
        exact = all(dist_sha(B.to_u64(d)) == q["sha256"] for d, q in zip(dists, grec))
        phases_ok = [int(x) for x in bph] == [q["phases"] for q in grec]
    res = {"workload": "64 graphs (random 2^12..2^18 deg 4..32, grids 64^2..512^2, R-MAT 12..18 ef 16), "
                       "8 sources each, weights [1, 2^16], IN_STATIC|OUT_STATIC",
           "queries": len(queries), "m_reach_total": m_reach, "batched_ms": round(tb * 1e3, 3),
           "batched_gteps": round(m_reach / tb / 1e9, 4), "plain_ms": round(tp * 1e3, 3),
           "plain_gteps": round(m_reach / tp / 1e9, 4), "speedup_vs_plain": round(tp / tb, 2),
           "batched_solve_hbm_frac": round(qbytes / tb / 1e9 / HBM_PEAK_GBS, 4),
           "phases_total": int(sum(pph)), "max_phases": int(max(pph)), "autotuned": tuned,
           "batched_equals_plain": bool(same), "distances_exact": exact, "phases_equal_oracle": phases_ok}
    log("batched", res)
    return res


SWITCHES = (("IN_SIMPLE|OUT_STATIC", 1, 2), ("SIMPLE_OR", 1, 3))


def bench_switched(B, torch, dg, src, m_reach, plain_ms, ref):
    """Switched solves (IN_STATIC|OUT_STATIC until |F| falls to a fraction of its peak, then a
    stronger criterion) against the plain solver on the same graph; distances checked against ref."""
    crits = {"IN_SIMPLE|OUT_STATIC": B.IN_SIMPLE | B.OUT_STATIC, "SIMPLE_OR": B.SIMPLE_OR}
    out = {}
    dist = B.new_dist(dg.n)
    for name, num, den in SWITCHES:
        fn = lambda: B.solve_switch(dg, src, B.STATIC_OR, crits[name], (num, den), dist)
        fn()
        torch.cuda.synchronize()
        ts, r = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = sorted(ts)[1]
        out["then %s at %d/%d of peak F" % (name, num, den)] = {
            "ms": round(t * 1e3, 3), "phases": r.phases, "gteps": round(m_reach / t / 1e9, 4),
            "over_plain": round(t * 1e3 / plain_ms, 3), "distances_exact": bool(np.array_equal(B.to_u64(r.dist), ref))}
    return out


def bench_c1(B, torch, G):
    """The small random graph (n = 16384, out-degree 8, weights [1, 1000], source 0) with
    IN_STATIC|OUT_STATIC: latency-bound (about a hundred short phases), so reported per phase, for
    the grid-wide kernels and the one-workgroup launch option; median of 11 solves."""
    g = G.config_small(seed=1)
    dg = B.DeviceGraph.from_graph(g)
    dist = B.new_dist(g.n)
    st = B.solve_ex(dg, 0, B.STATIC_OR, dist).stats
    rec = golden("er16k", "STATIC_OR", 0)
    res = {"workload": "er_n16384_outdeg8_w1-1000_src0", "n": g.n, "m": g.m, "m_reach": st["m_reach"]}
    for single in (0, 1):
        dg.set_launch(single=single)
        dt, r = median_time(torch, lambda: B.solve(dg, 0, B.STATIC_OR, dist), reps=11)
        res["single" if single else "plain"] = {
            "ms": round(dt * 1e3, 4), "phases": r.phases, "us_per_phase": round(dt * 1e6 / r.phases, 2),
            "gteps": round(st["m_reach"] / dt / 1e9, 4),
            "distances_exact": exact_vs_golden("er16k", 0, B.to_u64(dist)),
            "phases_equal_oracle": None if rec is None else r.phases == rec["phases"]}
    log("c1", res)
    return res


def bench_c3(B, torch, G, tuned):
    """R-MAT scale 22 and the 2048^2 grid, the 8 seeded sources each: the plain solver with
    IN_STATIC|OUT_STATIC against Delta-stepping (2^12, 2^14, 2^16), median of three solves per
    source, with the launch shape tuned on the headline graph; distances, phase and round counts
    against the oracle's stored values. The grid is latency-bound (thousands of phases with a small
    F), so its plain figure is also given per phase, with the one-workgroup launch option beside it."""
    res = {}
    for name, gname, make in (("rmat_s22_ef16", "rmat22", lambda: G.config_rmat(seed=1)),
                              ("grid_2048x2048", "grid2048", lambda: G.config_grid(seed=1))):
        t = time.time()
        g = make()
        dg = B.DeviceGraph.from_graph(g)
        dg.set_launch(**tuned)
        srcs = [int(x) for x in G.sources(g, 8, 11)]
        dist = B.new_dist(g.n)
        sts = [B.solve_ex(dg, s_, B.STATIC_OR, dist).stats for s_ in srcs]
        m_reach = sum(x["m_reach"] for x in sts)
        n_reach = sum(x["n_reach"] for x in sts)
        checks = {"distances_exact": True, "phases_equal_oracle": True, "rounds_equal_oracle": True}

        def check(key, ok):
            checks[key] = checks[key] and ok is not None and bool(ok)

        def run(fn, kind=None):
            tot, ph = 0.0, 0
            for s_ in srcs:
                dt, r = median_time(torch, lambda: fn(s_))
                tot += dt
                ph += r.phases
                check("distances_exact", exact_vs_golden(gname, s_, B.to_u64(dist)))
                if kind is not None:
                    rec = golden(gname, kind, s_)
                    key = "rounds" if kind.startswith("delta") else "phases"
                    check(key + "_equal_oracle", None if rec is None else r.phases == rec[key])
            return tot, ph

        nsrc = len(srcs)
        tp, php = run(lambda s_: B.solve(dg, s_, B.STATIC_OR, dist), "STATIC_OR")
        e = {"n": g.n, "m": g.m, "sources": nsrc, "m_reach_total": m_reach, "plain_ms": round(tp * 1e3 / nsrc, 3),
             "plain_phases": round(php / nsrc, 1), "plain_gteps": round(m_reach / tp / 1e9, 4),
             "plain_us_per_phase": round(tp * 1e6 / php, 2)}
        if n_reach <= 4096 * php:
            # few vertices settled per phase (the autotuner's rule): also the one-workgroup form
            dg.set_launch(single=1)
            ts, phs = run(lambda s_: B.solve(dg, s_, B.STATIC_OR, dist), "STATIC_OR")
            dg.set_launch(single=0)
            e["single_ms"] = round(ts * 1e3 / nsrc, 3)
            e["single_gteps"] = round(m_reach / ts / 1e9, 4)
            e["single_us_per_phase"] = round(ts * 1e6 / phs, 2)
        for k in (12, 14, 16):
            td, rd = run(lambda s_: B.delta_step(dg, s_, 1 << k, dist), "delta%d" % k)
            e["delta_2^%d" % k] = {"ms": round(td * 1e3 / nsrc, 3), "rounds": round(rd / nsrc, 1),
                                   "gteps": round(m_reach / td / 1e9, 4)}
        e.update(checks)
        if name.startswith("rmat"):
            s0 = srcs[0]
            tp0, rp = median_time(torch, lambda: B.solve(dg, s0, B.STATIC_OR, dist))
            e["switched_src0"] = bench_switched(B, torch, dg, s0, sts[0]["m_reach"], tp0 * 1e3, B.to_u64(rp.dist))
            # the dominant kernel's roofline on the first source, as for the headline graph
            rms, _, rst, rroof, _, _ = measure_plain(B, torch, dg, s0, B.STATIC_OR, 3, 1, gname)
            e["roofline_src0"] = rroof
            e["solve_hbm_frac_src0"] = solve_frac(rst, rms, g.n)
        res[name] = e
        log("c3", name, e, "%.1fs" % (time.time() - t))
        del dg, dist, g
    return res


def bench_learned(B, torch, G, dg, src, m_reach, plain_ms):
    """The learned selector (weights trained on training seeds by the package's training script) on
    the headline graph and on the held-out evaluation graphs (random 2^23, R-MAT 23, grid 4096^2):
    the network-only checkpoint solve against the plain static solve, the hand-set switch and the
    stronger criteria from the start; the per-phase learned solve; learned Delta-stepping against
    every fixed width. Distances of every learned form are checked against the plain solver's."""
    from paper_1903_12085_amd import selector as S
    sel = S.load_trained()
    res = {"weights": "selector_weights.npy (trained on random 2^16..2^21, R-MAT 16..20, grids 256^2..1024^2; "
                      "other seeds)"}
    exact = True

    def one(name, h, s, mr, per_phase):
        nonlocal exact
        e = S.evaluate(sel, h, s, reps=3, per_phase=per_phase)
        ref = B.to_u64(B.solve(h, s, B.STATIC_OR).dist)
        ok = (np.array_equal(B.to_u64(B.solve_checkpoint(h, s, sel).dist), ref) and
              np.array_equal(B.to_u64(B.delta_step_learned(h, s, sel).dist), ref) and
              (not per_phase or np.array_equal(B.to_u64(B.solve_learned(h, s, sel).dist), ref)))
        e["distances_exact"] = bool(ok)
        exact = exact and e["distances_exact"]
        e["checkpoint_gteps"] = mr / (e["checkpoint_ms"] * 1e6)
        e["static_or_gteps"] = mr / (e["static_or_ms"] * 1e6)
        e["best_fixed_delta_ms"] = min(e["delta_%d_ms" % d] for d in B.CHOICE_DELTA)
        e["learned_delta_over_best_fixed"] = e["learned_delta_ms"] / e["best_fixed_delta_ms"]
        res[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in e.items()}
        log("learned", name, res[name])

    one("headline", dg, src, m_reach, True)
    res["headline"]["plain_ms_timed_run"] = round(plain_ms, 3)
    for g in S.evaluation_graphs():
        h = B.DeviceGraph.from_graph(g)
        s = int(G.sources(g, 1, 5)[0])
        mr = B.solve_ex(h, s, B.STATIC_OR).stats["m_reach"]
        one(g.name, h, s, mr, False)
        del h
    res["distances_exact"] = exact
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=22)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the R-MAT 22 / 2048^2 grid section")
    ap.add_argument("--profile-run", action="store_true",
                    help="one solve with the default launch shape, for rocprofv3 (no tuning, no extra passes)")
    ap.add_argument("--profile-graph", default="er", choices=("er", "rmat", "grid"),
                    help="with --profile-run: the random graph of --log2n (source 0), or R-MAT scale 22 or the "
                         "2048^2 grid (the first of their 8 benchmark sources)")
    ap.add_argument("--launch", default=None,
                    help="with --profile-run: scan_blocks,relax_blocks,chunk,use_graph[,queue[,single]] (e.g. the "
                         "shape the autotuner picks for the timed run)")
    ap.add_argument("--profile-batch", default=None,
                    help="one batched solve of the 512-query workload with the given launch shape "
                         "block,split,blocks,team_edges (for rocprofv3; no tuning, no other legs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy kernel (known bytes) for counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single device "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen as G
    from paper_1903_12085_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    B.load()
    if args.copy_calibration:
        src_t = torch.empty(1 << 27, dtype=torch.int64, device="cuda").fill_(1)  # 1 GiB
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 1 << 30}))
        return
    if args.profile_batch:
        graphs, queries = G.batch_workload(seed=7)
        dgs = [B.DeviceGraph.from_graph(g) for g in graphs]
        qg = [dgs[i] for i, _ in queries]
        qs = [s for _, s in queries]
        dists = [B.new_dist(graphs[i].n) for i, _ in queries]
        f = [int(x) for x in args.profile_batch.split(",")]
        cfg = dict(zip(("block", "split", "blocks", "team_edges"), f), team_size=0)
        torch.cuda.synchronize()
        _, ph = B.solve_batch(qg, qs, B.STATIC_OR, dists, cfg=cfg)
        torch.cuda.synchronize()
        print(json.dumps({"profile_batch": True, "queries": len(queries), "phases_total": int(ph.sum()), "cfg": cfg}))
        return
    if args.profile_run:
        if args.profile_graph in ("rmat", "grid"):
            g = G.config_rmat(seed=1) if args.profile_graph == "rmat" else G.config_grid(seed=1)
            psrc = int(G.sources(g, 8, 11)[0])
        else:
            g = G.config_er_large(seed=1, log2n=args.log2n)
            psrc = 0
        dg = B.DeviceGraph.from_graph(g)
        if args.launch:
            f = [int(x) for x in args.launch.split(",")]
            keys = ("scan_blocks", "relax_blocks", "chunk", "use_graph", "queue", "single")
            dg.set_launch(**dict(zip(keys, f)))
        r = B.solve(dg, psrc, B.STATIC_OR)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "phases": r.phases, "launch": dg.launch()}))
        return
    seed, src = 1, 0
    t = time.time()
    g = G.config_er_large(seed=seed, log2n=args.log2n)
    log("graph n=%d m=%d generated in %.1fs" % (g.n, g.m, time.time() - t))
    t = time.time()
    dg = B.DeviceGraph.from_graph(g)
    torch.cuda.synchronize()
    log("device graph ready in %.1fs" % (time.time() - t))
    crit = B.STATIC_OR
    tuned, tuned_ms = B.autotune(dg, src, crit)  # one-time launch-shape search (untimed)
    log("autotuned launch shape", tuned, "%.3f ms" % tuned_ms)

    ms, phases, st, roofline, prof, dist = measure_plain(B, torch, dg, src, crit, args.steps, args.warmup,
                                                         "er%d" % args.log2n)
    log("timed %d steps: %.3f ms/step, %d phases" % (args.steps, ms, phases))
    gteps = st["m_reach"] / (ms * 1e-3) / 1e9
    log("profile", prof)
    copy_gbs, atomics = device_ceilings(B, torch)
    roofline["stream_copy_GBs"] = copy_gbs
    roofline["frac_vs_copy"] = round(roofline["achieved"] / copy_gbs, 4)
    log("device ceilings: copy %.1f GB/s, atomicMin %s" % (copy_gbs, atomics))

    out = {
        "metric": METRIC, "value": round(gteps, 4), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "er_n%d_outdeg16_w1-2^20_src0" % g.n, "n": g.n, "m": g.m, "seed": seed,
                   "source": src, "criterion": "IN_STATIC|OUT_STATIC", "form": "plain", "launch": tuned},
        "phases": phases, "sum_f": st["sum_f"], "m_reach": st["m_reach"], "n_reach": st["n_reach"],
        "relax_edges": st["relax_edges"], "improving": st["improving"],
        "us_per_phase": round(ms * 1e3 / phases, 2), "precompute_ms": round(st["precompute_ns"] / 1e6, 3),
        "gteps_incl_precompute": round(st["m_reach"] / ((ms + st["precompute_ns"] / 1e6) * 1e-3) / 1e9, 4),
        "roofline": roofline,
        "solve_hbm_frac": solve_frac(st, ms, g.n),
        "atomic_min": atomics,
    }

    gname = "er%d" % args.log2n
    out["distances_exact"] = exact_vs_golden(gname, src, B.to_u64(dist))
    cpu = None if args.no_cpu else CpuBaseline(g, src)

    if not args.no_extra:
        # the other criteria and Delta-stepping on the same graph: median of three solves after one
        # untimed one, distances and phase / round counts against the oracle's stored values
        forms = {}
        for name, c in [("IN_STATIC", B.IN_STATIC), ("OUT_STATIC", B.OUT_STATIC), ("SIMPLE_OR", B.SIMPLE_OR),
                        ("IN_FULL|OUT_WEAK", B.IN_FULL | B.OUT_WEAK), ("FULL_OR", B.FULL_OR)]:
            dt, r = median_time(torch, lambda: B.solve(dg, src, c, dist))
            rec = golden(gname, name, src)
            forms[name] = {"phases": r.phases, "ms": round(dt * 1e3, 3), "gteps": round(st["m_reach"] / dt / 1e9, 4),
                           "distances_exact": exact_vs_golden(gname, src, B.to_u64(dist)),
                           "phases_equal_oracle": None if rec is None else r.phases == rec["phases"]}
            log("criterion", name, forms[name])
        for k in (12, 14, 16):
            dt, r = median_time(torch, lambda: B.delta_step(dg, src, 1 << k, dist))
            rec = golden(gname, "delta%d" % k, src)
            forms["delta_2^%d" % k] = {"rounds": r.phases, "ms": round(dt * 1e3, 3),
                                       "gteps": round(st["m_reach"] / dt / 1e9, 4),
                                       "distances_exact": exact_vs_golden(gname, src, B.to_u64(dist)),
                                       "rounds_equal_oracle": None if rec is None else r.phases == rec["rounds"]}
            log("delta", k, forms["delta_2^%d" % k])
        out["forms"] = forms
        out["c1"] = bench_c1(B, torch, G)

    if not args.no_extra and args.log2n == 22:
        # the largest random graph of the workloads (2^23 vertices, same out-degree and weights),
        # with the launch shape tuned above
        gl = G.config_er_large(seed=seed, log2n=23)
        dl = B.DeviceGraph.from_graph(gl)
        dl.set_launch(**tuned)
        lms, lph, lst, lroof, _, ldist = measure_plain(B, torch, dl, src, crit, 3, 1, "er23")
        rec = golden("er23", "STATIC_OR", src)
        out["largest"] = {"workload": "er_n%d_outdeg16_w1-2^20_src0" % gl.n, "n": gl.n, "m": gl.m,
                          "solve_hbm_frac": solve_frac(lst, lms, gl.n),
                          "launch": tuned, "ms": round(lms, 3), "phases": lph,
                          "gteps": round(lst["m_reach"] / (lms * 1e-3) / 1e9, 4),
                          "distances_exact": exact_vs_golden("er23", src, B.to_u64(ldist)),
                          "phases_equal_oracle": None if rec is None else lph == rec["phases"],
                          "roofline": lroof}
        lroof["stream_copy_GBs"] = copy_gbs
        lroof["frac_vs_copy"] = round(lroof["achieved"] / copy_gbs, 4)
        log("largest", out["largest"])
        del dl, ldist, gl

    if not args.no_extra:
        out["switched"] = bench_switched(B, torch, dg, src, st["m_reach"], ms, B.to_u64(dist))
        log("switched", out["switched"])

    if not args.no_extra and not args.no_c3:
        out["c3"] = bench_c3(B, torch, G, tuned)

    if not args.no_batch:
        out["batched"] = bench_batched(B, torch, G)

    if not args.no_learned:
        out["learned"] = bench_learned(B, torch, G, dg, src, st["m_reach"], ms)

    if cpu is not None:
        out["cpu_baseline"] = cpu.result(st["m_reach"])
        if cpu.dist is not None:
            out["distances_equal_cpu_oracle"] = bool(np.array_equal(B.to_u64(dist), cpu.dist))
        log("cpu oracle", out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
