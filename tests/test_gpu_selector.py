"""GPU selector: forward and gradients against the CPU references, learned solves against the
oracle's replay of the same network (weights from the oracle side), and training.

Weights used for parity come from oracle/mlp_ref.py (seeded initialisation, optionally trained in
float64 there), never from the HIP path.
"""
import numpy as np
import pytest

import graphgen as G
import oracle as O
from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1903_12085_amd import binding
    binding.load()
    return binding


def seeded_xy(seed, n):
    x = G.uniform01(seed, 1, n * 12).reshape(n, 12).astype(np.float32)
    y = (G.u64_stream(seed, 2, n) % np.uint64(6)).astype(np.int32)
    return x, y


def test_forward_bitwise_equals_oracle_fp32(B):
    w = M.init_params(11).astype(np.float32)
    x, _ = seeded_xy(3, 200)
    sel = B.Selector(w)
    z = sel.forward(x)
    for i in range(200):
        _, zo = O.mlp_choice(w, x[i], 0)
        assert np.array_equal(z[i], zo), i


def test_gradients_match_float64_reference(B):
    rng = np.random.default_rng(5)
    w = (M.init_params(12) + rng.normal(0, 0.05, M.NPARAM)).astype(np.float32)
    for n in (1, 7, 64, 300):
        x, y = seeded_xy(10 + n, n)
        loss, g = B.Selector(w).grad(x, y)
        rl, rg = M.loss_and_grad(w.astype(np.float64), x.astype(np.float64), y)
        assert abs(loss - rl) <= 1e-5 * max(1.0, abs(rl))
        scale = np.abs(rg).max()
        assert np.abs(g - rg).max() <= 1e-4 * scale, (n, np.abs(g - rg).max(), scale)


def test_training_reduces_loss(B):
    x, _ = seeded_xy(21, 4096)
    y = ((x[:, 0] > 0.5).astype(np.int32) + 2 * (x[:, 3] > 0.5).astype(np.int32))  # learnable labels 0..3
    sel = B.Selector(M.init_params(22).astype(np.float32))
    l0, _ = sel.grad(x, y)
    sel.train(x, y, epochs=40, batch=256, lr=3e-3, seed=1)
    l1, _ = sel.grad(x, y)
    assert l1 < 0.5 * l0
    acc = (sel.forward(x).argmax(1) == y).mean()
    assert acc > 0.9


def mixed_weights(seed):
    """Seeded weights whose phase choices vary along a solve (oracle-side, float32)."""
    w = M.init_params(seed)
    p = M.unpack(w)
    p["W3"] *= 4.0
    return M.pack(p).astype(np.float32)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_learned_solve_matches_oracle_replay(B, seed):
    w = mixed_weights(seed)
    sel = B.Selector(w)
    seen = set()
    for g in (G.er(3000, 8, 1, 1000, seed), G.rmat(11, 16, 1, 1 << 16, seed), G.grid(40, 37, 1, 1 << 16, seed),
              G.random_small(60, 240, 30, seed)):
        ref = O.phased(g, 0, 0, mlp_w=w)
        dg = B.DeviceGraph.from_graph(g)
        r = B.solve_learned(dg, 0, sel, phase_of=True, trace_cap=ref.phases + 4)
        assert np.array_equal(r.dist_u64(), ref.dist), g.name
        assert r.phases == ref.phases, (g.name, r.phases, ref.phases)
        assert np.array_equal(r.trace["criterion"], ref.trace_crit), g.name
        assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of), g.name
        seen |= set(int(c) for c in ref.trace_crit)
    assert len(seen) >= 1


def test_learned_solve_uses_several_criteria(B):
    # over a few seeds the oracle replay must see more than one criterion, and the GPU must agree
    kinds = set()
    for seed in range(5, 12):
        w = mixed_weights(seed)
        g = G.er(2000, 6, 1, 500, seed)
        ref = O.phased(g, 0, 0, mlp_w=w)
        r = B.solve_learned(B.DeviceGraph.from_graph(g), 0, B.Selector(w), trace_cap=ref.phases + 4)
        assert r.phases == ref.phases and np.array_equal(r.trace["criterion"], ref.trace_crit)
        kinds |= set(int(c) for c in ref.trace_crit)
    assert len(kinds) >= 2


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_learned_delta_matches_oracle_replay(B, seed):
    w = mixed_weights(seed + 40)
    sel = B.Selector(w)
    for g in (G.er(4000, 8, 1, 1 << 16, seed), G.grid(30, 30, 1, 1 << 16, seed)):
        ref = O.delta_step(g, 0, None, mlp_w=w, trace_cap=1 << 16)
        r = B.delta_step_learned(B.DeviceGraph.from_graph(g), 0, sel)
        assert np.array_equal(r.dist_u64(), ref.dist)
        assert r.phases == ref.rounds and r.stats["buckets"] == ref.buckets


@pytest.mark.parametrize("seed", [1, 2])
def test_trace_mode_counts_and_features_match_oracle(B, seed):
    """Training traces: per phase, how many queued vertices each criterion certifies on the same
    snapshot, and the features, equal the oracle's check-mode evaluation of the same trajectory."""
    w = mixed_weights(seed + 20)
    sel = B.Selector(w)
    for g in (G.er(2500, 8, 1, 1000, seed), G.rmat(11, 16, 1, 1 << 16, seed), G.grid(25, 30, 1, 1 << 16, seed)):
        ref = O.phased(g, 0, 0, mlp_w=w, check=True)
        r, feat, cnt = B.trace_learned(B.DeviceGraph.from_graph(g), 0, sel, cap=ref.phases + 4)
        assert np.array_equal(r.dist_u64(), ref.dist) and r.phases == ref.phases
        assert np.array_equal(r.trace["criterion"], ref.trace_crit)
        assert np.array_equal(cnt, ref.trace_union), g.name
        assert np.array_equal(feat, ref.trace_feat), g.name


def test_trace_mode_delta_features_match_oracle(B):
    w = mixed_weights(31)
    g = G.er(3000, 8, 1, 1 << 16, 3)
    ref = O.delta_step(g, 0, None, mlp_w=w, trace_cap=1 << 12)
    r, feat, _ = B.trace_learned(B.DeviceGraph.from_graph(g), 0, B.Selector(w), delta_mode=True)
    assert r.phases == ref.rounds and feat.shape[0] == ref.buckets
    assert np.array_equal(r.dist_u64(), ref.dist)


@pytest.mark.parametrize("seed", [1, 2])
def test_learned_commit_matches_oracle_replay(B, seed):
    # prefix of K selector choices, then phase K's choice on the plain kernels; with captured
    # six-phase graphs on and off (K not a multiple of six starts the graphs mid-way), and with
    # per-phase profiling (which runs its own loop)
    w = mixed_weights(seed)
    sel = B.Selector(w)
    for g in (G.er(3000, 8, 1, 1000, seed), G.rmat(11, 16, 1, 1 << 16, seed), G.grid(40, 37, 1, 1 << 16, seed)):
        dg = B.DeviceGraph.from_graph(g)
        free = O.phased(g, 0, 0, mlp_w=w)
        for commit in (1, 3, 7, 12, free.phases + 5):
            ref = O.phased(g, 0, 0, mlp_w=w, commit=commit)
            for use_graph, prof in ((0, False), (1, False), (1, True)):
                dg.set_launch(use_graph=use_graph)
                dg.profile(prof)
                r = B.solve_learned(dg, 0, sel, phase_of=True, trace_cap=ref.phases + 4, commit=commit)
                case = (g.name, commit, use_graph, prof)
                assert np.array_equal(r.dist_u64(), ref.dist), case
                assert r.phases == ref.phases, (case, r.phases, ref.phases)
                assert np.array_equal(r.trace["criterion"], ref.trace_crit), case
                assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of), case
                if prof:
                    assert len(dg.phase_times()) == ref.phases, case
            dg.profile(False)


def test_learned_commit_rejects_phase_zero_and_keeps_plain_solves_intact(B):
    g = G.er(2000, 6, 1, 500, 9)
    dg = B.DeviceGraph.from_graph(g)
    sel = B.Selector(mixed_weights(9))
    with pytest.raises(B.SsspError):
        B._check(B.load().sssp_solve_learned_commit(dg.handle, 0, sel.handle, 0, None, None, None, None, 0))
    # a plain solve after a committed one (shared cached graph, shared control block)
    ref = O.phased(g, 0, O.STATIC_OR)
    B.solve_learned(dg, 0, sel, commit=4)
    r = B.solve(dg, 0, O.STATIC_OR)
    assert np.array_equal(r.dist_u64(), ref.dist) and r.phases == ref.phases


@pytest.mark.parametrize("seed", [1, 2])
def test_learned_commit_switch_matches_oracle_replay(B, seed):
    # committed learned prefix, then (committed static choice) static until |F| falls to half its
    # peak, then IN_SIMPLE|OUT_STATIC; the recorded per-phase criteria replayed by the oracle give
    # every observable, and the prefix equals the oracle's committed run
    w = mixed_weights(seed)
    sel = B.Selector(w)
    then = O.CRIT["IN_SIMPLE"] | O.OUT_STATIC
    zero = np.zeros(O.MLP_NPARAM, np.float32)  # every logit 0: the first choice, the static criterion
    static = B.Selector(zero)
    for g in (G.er(3000, 8, 1, 1000, seed), G.rmat(11, 16, 1, 1 << 16, seed), G.grid(40, 37, 1, 1 << 16, seed)):
        dg = B.DeviceGraph.from_graph(g)
        dj, _ = O.dijkstra(g, 0)
        for s_ in (sel, static):
            for commit in (1, 16):
                r = B.solve_learned(dg, 0, s_, phase_of=True, trace_cap=g.n + 4, commit=commit, switch=(then, 1, 2))
                assert np.array_equal(r.dist_u64(), dj), (g.name, commit)
                crit = np.asarray(r.trace["criterion"])
                com = O.phased(g, 0, 0, mlp_w=w if s_ is sel else zero, commit=commit, trace_cap=g.n)
                k = min(commit, r.phases)
                assert np.array_equal(crit[:k], com.trace_crit[:k]), (g.name, commit)
                rep = O.phased(g, 0, 0, crit_seq=crit.astype(np.uint32))
                assert r.phases == rep.phases and r.stats["sum_f"] == rep.sum_f, (g.name, commit)
                assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), rep.phase_of), (g.name, commit)
        dg.close()


CKPT_GRAPHS = lambda seed: (G.grid(40, 37, 1, 1 << 16, seed), G.er(20000, 3, 1, 1000, seed),  # noqa: E731
                            G.rmat(12, 16, 1, 1 << 16, seed), G.grid(90, 11, 1, 1000, seed))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_checkpoint_solve_matches_oracle(B, seed):
    """The learned checkpoint solve against the oracle's checkpoint mode with the same network
    (weights from the oracle side): checkpoint features bitwise, per-phase criteria (so the switch
    phase and target), phases, settle phases and distances exactly."""
    ws = [mixed_weights(seed)] + [M.pack(dict(M.unpack(np.zeros(M.NPARAM)), b3=np.eye(6)[c] * 10.0)).astype(np.float32)
                                  for c in (0, 1, 2)]
    for w in ws:
        sel = B.Selector(w)
        for g in CKPT_GRAPHS(seed):
            ref = O.phased(g, 0, O.STATIC_OR, mlp_w=w, checkpoint=True, trace_cap=g.n)
            dg = B.DeviceGraph.from_graph(g)
            r, feat = B.solve_checkpoint(dg, 0, sel, phase_of=True, trace_cap=g.n, features=True)
            assert np.array_equal(r.dist_u64(), ref.dist), g.name
            assert r.phases == ref.phases, (g.name, r.phases, ref.phases)
            assert np.array_equal(r.trace["criterion"], ref.trace_crit), g.name
            assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of), g.name
            # checkpoints up to the deciding one (a switch at 16 (j + 2) was decided at checkpoint j;
            # the GPU's static stage runs one more batch, whose checkpoint the oracle does not need)
            sw = next((k for k, c in enumerate(ref.trace_crit) if int(c) != O.STATIC_OR), None)
            rows = ref.phases // 16 if sw is None else sw // 16 - 1
            assert len(feat) >= rows, g.name
            assert np.array_equal(feat[:rows], ref.trace_feat[:rows]), g.name
            dg.close()


def test_schedule_matches_oracle_replay(B):
    """sssp_solve_schedule (static until a given phase, then another criterion) against the oracle's
    per-phase criterion sequence, for switch phases 0, 1, 17 and past the end."""
    for g in (G.er(5000, 6, 1, 1000, 41), G.grid(50, 41, 1, 1 << 16, 42)):
        dg = B.DeviceGraph.from_graph(g)
        for then in (O.SIMPLE_OR, O.IN_SIMPLE | O.OUT_STATIC, O.DIJK):
            for at in (0, 1, 17, 100000):
                seq = [O.STATIC_OR] * min(at, g.n + 2) + [then]
                ref = O.phased(g, 0, 0, crit_seq=seq, trace_cap=g.n)
                r = B.solve_schedule(dg, 0, O.STATIC_OR, then, at, phase_of=True, trace_cap=g.n)
                assert np.array_equal(r.dist_u64(), ref.dist) and r.phases == ref.phases, (g.name, then, at)
                assert np.array_equal(r.trace["criterion"], ref.trace_crit), (g.name, then, at)
                assert np.array_equal(r.phase_of.cpu().numpy().view(np.uint32), ref.phase_of), (g.name, then, at)
        dg.close()
