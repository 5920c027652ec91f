"""Pins for the selector side of the oracle (no GPU).

* The float64 network reference is pinned by central finite differences and by a per-sample loop
  forward pass written separately.
* The oracle's FP32 forward pass agrees with the float64 reference wherever the top two logits are
  clearly apart.
* Learned-mode replay with a network that always prefers one output equals the fixed criterion
  (or the fixed bucket width) exactly.
* The 12 features the oracle computes equal an independent pure-Python re-simulation of the phased
  algorithm on small graphs.
"""
import numpy as np
import pytest

import graphgen as G
import oracle as O
from oracle import mlp_ref as M


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    w = M.init_params(1) + rng.normal(0, 0.05, M.NPARAM)
    X = rng.uniform(0, 1, (9, 12))
    y = rng.integers(0, 6, 9)
    _, g = M.loss_and_grad(w, X, y)
    idx = rng.choice(M.NPARAM, 120, replace=False)
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = 1e-6
        fd = (M.loss_and_grad(w + e, X, y)[0] - M.loss_and_grad(w - e, X, y)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_forward_matches_per_sample_loops():
    rng = np.random.default_rng(2)
    w = M.init_params(3)
    p = M.unpack(w)
    X = rng.uniform(0, 1, (5, 12))
    z, _ = M.forward(w, X)
    for s in range(5):
        h1 = [max(0.0, p["b1"][j] + sum(p["W1"][j][i] * X[s][i] for i in range(12))) for j in range(64)]
        h2 = [max(0.0, p["b2"][j] + sum(p["W2"][j][i] * h1[i] for i in range(64))) for j in range(64)]
        out = [p["b3"][j] + sum(p["W3"][j][i] * h2[i] for i in range(64)) for j in range(6)]
        assert np.allclose(out, z[s], rtol=1e-12, atol=1e-12)


def test_fp32_forward_agrees_with_reference():
    rng = np.random.default_rng(4)
    w = M.init_params(5)
    checked = 0
    for _ in range(300):
        x = rng.uniform(0, 1, 12).astype(np.float32)
        z64, _ = M.forward(w, x[None, :].astype(np.float64))
        for lo in (0, 3):
            seg = np.sort(z64[0, lo:lo + 3])
            if seg[-1] - seg[-2] < 1e-4:
                continue
            c, z32 = O.mlp_choice(w.astype(np.float32), x, lo)
            assert c == lo + int(np.argmax(z64[0, lo:lo + 3]))
            assert np.allclose(z32, z64[0], rtol=1e-4, atol=1e-4)
            checked += 1
    assert checked > 400


def constant_net(choice):
    w = np.zeros(M.NPARAM, np.float32)
    w[-6 + choice] = 10.0  # b3: this output always wins
    return w


@pytest.mark.parametrize("choice", [0, 1, 2])
def test_learned_replay_with_constant_choice_equals_fixed_criterion(choice):
    for g in (G.er(600, 5, 1, 300, 2), G.rmat(9, 8, 1, 1000, 3), G.grid(12, 9, 1, 40, 4)):
        ref = O.phased(g, 0, O.CHOICE_CRIT[choice])
        lr = O.phased(g, 0, 0, mlp_w=constant_net(choice), check=True)
        assert lr.phases == ref.phases and np.array_equal(lr.phase_of, ref.phase_of)
        assert (lr.trace_crit == O.CHOICE_CRIT[choice]).all()


@pytest.mark.parametrize("choice", [3, 4, 5])
def test_learned_delta_with_constant_choice_equals_fixed_width(choice):
    g = G.er(2000, 6, 1, 1 << 16, 5)
    delta = 1 << (12 + 2 * (choice - 3))
    ref = O.delta_step(g, 0, [delta])
    lr = O.delta_step(g, 0, None, mlp_w=constant_net(choice), trace_cap=64)
    assert lr.rounds == ref.rounds and np.array_equal(lr.dist, ref.dist)
    assert (lr.trace_delta == delta).all()


def python_features(g, src):
    """Independent re-simulation of IN-STATIC|OUT-STATIC with the feature definitions: row 0 is the
    state {s} before any evaluation, row k+1 is phase k's snapshot with phase k's own outcome."""
    n, m = g.n, g.m
    rp, col, w = [int(x) for x in g.row_ptr], [int(x) for x in g.col], [int(x) for x in g.w]
    INF = O.INF_INT
    min_in = [INF] * n
    min_out = [INF] * n
    for u in range(n):
        for e in range(rp[u], rp[u + 1]):
            min_out[u] = min(min_out[u], w[e])
            min_in[col[e]] = min(min_in[col[e]], w[e])
    Wm = (float(sum(w)) / float(m)) if m else 1.0

    def feat(F, S, R, a, t, SD, DG, Fp, D, Sp, Ip, Op):
        x = [0.0] * 12
        x[0] = F / n
        x[1] = S / n
        x[2] = Sp / D if D else 0.0
        x[3] = min(F / 4194304.0, 4.0) / 4.0
        x[4] = 1.0 if t == INF else min((t - a) / Wm, 64.0) / 64.0
        x[5] = min(max((SD / F - a) / Wm, 0.0), 256.0) / 256.0
        x[6] = min((DG / F) / (m / n), 8.0) / 8.0
        x[7] = Ip / D if D else 0.0
        x[8] = Op / D if D else 0.0
        x[9] = min(F / Fp, 4.0) / 4.0 if Fp else 0.0
        x[10] = (n - R) / n
        x[11] = min(a / Wm, 4096.0) / 4096.0
        return np.array(x, np.float64).astype(np.float32)

    d = [INF] * n
    st = [0] * n
    d[src] = 0
    st[src] = 1
    settled = 0
    prevF = 0
    out = [feat(1, 0, 1, 0, min_out[src], 0, rp[src + 1] - rp[src], 0, 0, 0, 0, 0)]
    while True:
        Fs = [v for v in range(n) if st[v] == 1]
        if not Fs:
            break
        F = len(Fs)
        a = min(d[v] for v in Fs)
        t = min((d[v] + min_out[v]) if min_out[v] != INF else INF for v in Fs)
        SD = sum(d[v] for v in Fs)
        DG = sum(rp[v + 1] - rp[v] for v in Fs)
        ins = [v for v in Fs if min_in[v] == INF or d[v] <= a + min_in[v]]
        outs = [v for v in Fs if d[v] <= t]
        S = sorted(set(ins) | set(outs))
        out.append(feat(F, settled, F + settled, a, t, SD, DG, prevF, F, len(S), len(ins), len(outs)))
        for v in S:
            st[v] = 2
        for u in S:
            for e in range(rp[u], rp[u + 1]):
                x_ = col[e]
                if st[x_] != 2 and d[u] + w[e] < d[x_]:
                    d[x_] = d[u] + w[e]
                    st[x_] = 1
        prevF = F
        settled += len(S)
    return np.array(out[:-1])  # the row after the last phase chooses for no phase


def test_features_match_independent_simulation():
    for g in (G.er(300, 4, 1, 500, 7), G.random_small(40, 150, 9, 8), G.grid(7, 6, 1, 30, 9)):
        ref = python_features(g, 0)
        lr = O.phased(g, 0, 0, mlp_w=constant_net(0))
        assert lr.trace_feat.shape == ref.shape
        assert np.array_equal(lr.trace_feat, ref)


def mixed_net(seed):
    """Float64-reference initialisation with large output biases jittered so that several
    criteria win on different states."""
    w = M.init_params(seed).astype(np.float32)
    rng = np.random.default_rng(seed)
    w[-6:-3] = rng.normal(0, 0.5, 3).astype(np.float32)
    return w


@pytest.mark.parametrize("commit", [1, 5, 12])
def test_commit_keeps_the_choice_of_phase_k(commit):
    for seed, g in enumerate((G.er(800, 6, 1, 500, 21), G.grid(20, 15, 1, 40, 22), G.rmat(10, 8, 1, 1000, 23))):
        w = mixed_net(seed + 3)
        free = O.phased(g, 0, 0, mlp_w=w, trace_cap=g.n)
        com = O.phased(g, 0, 0, mlp_w=w, commit=commit, trace_cap=g.n)
        k = min(commit, com.phases)
        # phases before K choose exactly as without commit; from K on, phase K's choice stays
        assert np.array_equal(com.trace_crit[:k], free.trace_crit[:k])
        if com.phases > commit:
            assert (com.trace_crit[commit:] == com.trace_crit[commit]).all()
        # the run equals the fixed per-phase sequence it recorded (the crit_seq path)
        seq = O.phased(g, 0, 0, crit_seq=com.trace_crit)
        assert seq.phases == com.phases and np.array_equal(seq.dist, com.dist)
        assert np.array_equal(seq.phase_of, com.phase_of)


def python_checkpoint_features(g, src):
    """Checkpoint features (delta_mode 2) from an independent re-simulation of IN-STATIC|OUT-STATIC:
    after every 16th phase k (k + 1 divisible by 16), phase k's F, S, minD, OUT-STATIC threshold and
    |S'|, and |F| at the previous checkpoint; x5 = floor(log2 n)/32 and x6 = min(m/n, 64)/64 (size and
    mean degree), x7 = x8 = 0."""
    n, m = g.n, g.m
    rp, col, w = [int(x) for x in g.row_ptr], [int(x) for x in g.col], [int(x) for x in g.w]
    INF = O.INF_INT
    min_in, min_out = [INF] * n, [INF] * n
    for u in range(n):
        for e in range(rp[u], rp[u + 1]):
            min_out[u] = min(min_out[u], w[e])
            min_in[col[e]] = min(min_in[col[e]], w[e])
    Wm = (float(sum(w)) / float(m)) if m else 1.0
    d, st = [INF] * n, [0] * n
    d[src], st[src] = 0, 1
    settled, fprev, k, rows = 0, 0, 0, []
    while True:
        Fs = [v for v in range(n) if st[v] == 1]
        if not Fs:
            break
        F = len(Fs)
        a = min(d[v] for v in Fs)
        t = min((d[v] + min_out[v]) if min_out[v] != INF else INF for v in Fs)
        S = [v for v in Fs if min_in[v] == INF or d[v] <= a + min_in[v] or d[v] <= t]
        if (k + 1) % 16 == 0:
            x = [0.0] * 12
            x[0] = F / n
            x[1] = settled / n
            x[2] = len(S) / F
            x[3] = min(F / 4194304.0, 4.0) / 4.0
            x[4] = 1.0 if t == INF else min((t - a) / Wm, 64.0) / 64.0
            x[5] = (n.bit_length() - 1) / 32.0
            x[6] = min(m / n, 64.0) / 64.0
            x[9] = min(F / fprev, 4.0) / 4.0 if fprev else 0.0
            x[10] = (n - (F + settled)) / n
            x[11] = min(a / Wm, 4096.0) / 4096.0
            rows.append(np.array(x, np.float64).astype(np.float32))
            fprev = F
        for v in S:
            st[v] = 2
        for u in S:
            for e in range(rp[u], rp[u + 1]):
                x_ = col[e]
                if st[x_] != 2 and d[u] + w[e] < d[x_]:
                    d[x_] = d[u] + w[e]
                    st[x_] = 1
        settled += len(S)
        k += 1
    return np.array(rows)


CKPT_GRAPHS = (G.grid(20, 15, 1, 40, 31), G.grid(33, 9, 1, 1000, 32), G.er(4000, 2, 1, 1000, 33))


def test_checkpoint_features_match_independent_simulation():
    for g in CKPT_GRAPHS:
        ref = python_checkpoint_features(g, 0)
        assert len(ref) >= 2, g.name
        lr = O.phased(g, 0, O.STATIC_OR, mlp_w=constant_net(0), checkpoint=True, trace_cap=g.n)
        assert np.array_equal(lr.trace_feat[:len(ref)], ref), g.name


@pytest.mark.parametrize("choice", [0, 1, 2])
def test_checkpoint_constant_choice_switches_at_phase_32(choice):
    """A network that always chooses c: c = 0 keeps the static criterion throughout; otherwise the
    first checkpoint (after phase 15) switches every phase from 32 on (two batch boundaries later)."""
    for g in CKPT_GRAPHS:
        r = O.phased(g, 0, O.STATIC_OR, mlp_w=constant_net(choice), checkpoint=True, trace_cap=g.n, check=True)
        seq = [O.STATIC_OR] * 32 + [O.CHOICE_CRIT[choice]] * g.n
        ref = O.phased(g, 0, 0, crit_seq=seq, trace_cap=g.n)
        assert r.phases == ref.phases and np.array_equal(r.phase_of, ref.phase_of), (g.name, choice)
        assert list(r.trace_crit) == list(ref.trace_crit), (g.name, choice)


def test_checkpoint_mixed_network_replays_as_its_schedule():
    for seed, g in enumerate(CKPT_GRAPHS):
        w = mixed_net(seed + 11)
        r = O.phased(g, 0, O.STATIC_OR, mlp_w=w, checkpoint=True, trace_cap=g.n)
        crit = [int(c) for c in r.trace_crit]
        # static up to a multiple of 16 (>= 32), one criterion after it
        sw = next((i for i, c in enumerate(crit) if c != O.STATIC_OR), len(crit))
        assert sw == len(crit) or (sw >= 32 and sw % 16 == 0 and len(set(crit[sw:])) == 1)
        seq = O.phased(g, 0, 0, crit_seq=r.trace_crit, trace_cap=g.n)
        assert seq.phases == r.phases and np.array_equal(seq.dist, r.dist) and np.array_equal(seq.phase_of, r.phase_of)
