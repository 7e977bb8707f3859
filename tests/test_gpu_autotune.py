"""The tile / bin-depth autotuner on the GPU: it returns one of its
candidates, a plan built with that choice renders the same visibility keys
as the default plan, and a cache file short-cuts a second call."""
import numpy as np
import pytest
import torch

import scenegen as sg
from paper_2308_10896_amd import dsm

pytestmark = pytest.mark.gpu


def test_autotune_choice_cache_and_equivalence(tmp_path):
    batch = sg.config0()
    dev = torch.device('cuda:0')
    ref = dsm.Plan(batch)
    verts, lp, alb, _ = dsm.batch_inputs(batch, dev)
    gimg = torch.as_tensor(np.random.default_rng(5).standard_normal(int(ref.info.image_floats)).astype(np.float32),
                           device=dev)
    cache = str(tmp_path / 'tune.txt')
    tile, scale, ms = dsm.autotune(batch, verts, lp, alb, gimg, reps=1, cache_path=cache)
    print('autotune', tile, scale, ms, flush=True)
    assert tile in (8, 16, 32) and scale in (8, 32) and ms > 0
    lines = open(cache).read().split('\n')
    assert len([x for x in lines if x.strip()]) == 1
    # second call: answered from the cache, no new line
    tile2, scale2, ms2 = dsm.autotune(batch, verts, lp, alb, gimg, reps=1, cache_path=cache)
    assert (tile2, scale2) == (tile, scale) and abs(ms2 - ms) <= 1e-5 * max(1.0, ms)
    assert len([x for x in open(cache).read().split('\n') if x.strip()]) == 1
    # the tuned plan computes the same visibility as the default one
    tuned = dsm.Plan(batch, tile_size=tile, bin_capacity_scale=scale)
    outs = []
    for plan in (ref, tuned):
        saved, scratch = plan.workspace(dev)
        plan.forward(verts, lp, alb, saved, scratch)
        outs.append([plan.view_keys(saved, v).cpu() for v in range(len(plan.view_shapes))])
    torch.cuda.synchronize()
    for a, b in zip(*outs):
        assert torch.equal(a, b)
