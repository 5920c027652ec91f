"""Gain of the trained checkpoint selector on held-out graphs (seeds no training graph uses).

The selector's weights are the package's trained ones. The network alone decides, at every 16th
phase of a plain IN-STATIC|OUT-STATIC solve, whether to keep the static criterion or to switch to
IN-SIMPLE|OUT-SIMPLE or IN-SIMPLE|OUT-STATIC for the rest of the solve. On each family the
checkpoint solve must keep distances exact (against the oracle's Dijkstra) and must not lose more
than a few per cent to the plain static solve (its fallback and judge; a solve that never
switches pays one small launch per 16 phases). Over the families the geometric mean of its time
over the plain static solve's must be below 0.98, and on at least two families it must be within
3 % of the hand-set switch (static until |F| falls to half its peak, then IN-SIMPLE|OUT-STATIC) or
faster. Times are the best of five on the GPU; the per-family results are printed for the record.
"""
import numpy as np
import pytest

import graphgen as G
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1903_12085_amd import binding
    binding.load()
    return binding


def held_out():
    return (G.er(1 << 18, 16, 1, (1 << 20) - 1, 3), G.rmat(17, 16, 1, (1 << 20) - 1, 3),
            G.grid(384, 384, 1, 1 << 16, 3))


def test_checkpoint_selector_gain_on_held_out_graphs(B):
    from paper_1903_12085_amd import selector as S
    sel = S.load_trained()
    ratios, vs_hand = [], []
    for g in held_out():
        dg = B.DeviceGraph.from_graph(g)
        src = int(G.sources(g, 1, 5)[0])
        ref, _ = O.dijkstra(g, src)
        assert np.array_equal(B.solve_checkpoint(dg, src, sel).dist_u64(), ref), g.name
        assert np.array_equal(B.solve_learned(dg, src, sel).dist_u64(), ref), g.name
        assert np.array_equal(B.delta_step_learned(dg, src, sel).dist_u64(), ref), g.name
        e = S.evaluate(sel, dg, src, reps=5, per_phase=False)
        print(g.name, {k: round(v, 3) if isinstance(v, float) else v for k, v in e.items()}, flush=True)
        assert e["checkpoint_ms"] <= 1.05 * e["static_or_ms"], (g.name, e)
        ratios.append(e["checkpoint_over_static"])
        vs_hand.append(e["checkpoint_over_hand_switch"])
        dg.close()
    gm = float(np.exp(np.mean(np.log(ratios))))
    print("checkpoint / static per family", [round(r, 3) for r in ratios], "geometric mean %.3f" % gm,
          "checkpoint / hand switch", [round(r, 3) for r in vs_hand], flush=True)
    assert gm < 0.98, ratios
    assert sum(r <= 1.03 for r in vs_hand) >= 2, vs_hand
