"""The launch-shape autotuner picks a valid shape, results stay oracle-exact under it,
and the per-process cache returns the same shape without timing."""
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qmc():
    import __graft_entry__ as g
    g._ensure_built()
    import torch
    import paper_2305_19768_amd as q
    torch.cuda.set_device(0)
    return q


def test_autotune_picks_a_valid_shape_and_keeps_parity(qmc):
    prob = W.two_loop_integral(seed=3, n_sectors=6, n_scale=0.01, m=8)
    plan = qmc.Plan(prob)
    best = plan.autotune(reps=1, use_cache=False)
    print("best", best, flush=True)
    assert best["ms"] > 0 and best["block"] in (64, 128, 256)
    assert prob.m % best["shift_tile"] == 0 and best["shift_tile"] % best["shifts_per_pass"] == 0
    assert plan.launch_shape()["block"] == best["block"]
    q, _, _ = plan.integrate()
    q = q.cpu().numpy()
    for s, sec in enumerate(prob.sectors):
        Q, S = oracle.sector_sums(sec, prob.shifts[s], threads=8)
        assert np.all(np.abs(q[s] - Q) <= 1e-12 * np.maximum(np.abs(Q), S))
    # the same problem shape is served from the cache, without timing
    plan2 = qmc.Plan(prob)
    t0 = time.perf_counter()
    again = plan2.autotune(reps=5, use_cache=True)
    assert time.perf_counter() - t0 < 1.0
    assert {k: again[k] for k in ("block", "shift_tile", "shifts_per_pass", "target_blocks")} == \
        {k: best[k] for k in ("block", "shift_tile", "shifts_per_pass", "target_blocks")}


def test_every_shape_gives_the_same_sums(qmc):
    prob = W.two_loop_integral(seed=4, n_sectors=3, n_scale=0.01, m=8)
    plan = qmc.Plan(prob)
    ref = None
    for blk, tile, spp, tg in [(64, 1, 1, 256), (128, 8, 4, 8192), (256, 4, 2, 32768),
                               (256, 8, 1, 16384)]:
        plan.set_launch_shape(blk, tile, spp, tg)
        q, _, _ = plan.integrate()
        q = q.cpu().numpy()
        if ref is None:
            ref = q
        assert np.allclose(q, ref, rtol=1e-13, atol=0)
