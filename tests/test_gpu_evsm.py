"""GPU parity of the alternative pre-filtered maps: exponentially warped
moments and the light-bleeding reduction, alone and together, plain and
warped lights mixed in one batch; forward (keys bit-exact, maps, images)
and backward (light, vertex and albedo gradients) against the oracle."""
import numpy as np
import pytest

import scenegen as sg
from parity_helpers import (assert_image, IMG_ATOL, IMG_RTOL, MAP_ATOL, MAP_RTOL, assert_close, check_gradients,
                            cone_ambiguous, gpu_run, loss_grad, oracle_run, random_grad)

pytestmark = pytest.mark.gpu


def cfg0_warp():
    b = sg.config0()
    b.lights[0].resolution = 200
    b.cameras[0].width, b.cameras[0].height = 250, 190
    b.lights[0].warp_exponent = 40.0
    return b


def cfg1_warp_bleed():
    b = sg.config1()
    b.lights[0].resolution = 300
    b.cameras[0].width, b.cameras[0].height = 280, 232
    b.lights[0].warp_exponent = 20.0
    b.lights[0].bleed_reduction = 0.3
    return b


def cfg1_bleed():
    b = cfg1_warp_bleed()
    b.lights[0].warp_exponent = 0.0
    return b


def cfg2_mixed():
    b = sg.config2(n_scenes=3, resolution=176, with_pose=False)
    b.lights[1].warp_exponent = 35.0
    b.lights[2].warp_exponent = 10.0
    b.lights[2].bleed_reduction = 0.2
    return b


BATCHES = {'cfg0_warp': cfg0_warp, 'cfg1_warp_bleed': cfg1_warp_bleed, 'cfg1_bleed': cfg1_bleed,
           'cfg2_mixed': cfg2_mixed}


@pytest.mark.parametrize('name', list(BATCHES))
def test_forward_matches_oracle(name):
    b = BATCHES[name]()
    g = gpu_run(b)
    o = oracle_run(b)
    for v, (kg, ko) in enumerate(zip(g['keys'], o['keys'])):
        assert not (kg != ko).any(), f'view {v}: keys differ'
    for l in range(len(b.lights)):
        assert_close(f'F0[{l}]', g['F0'][l], o['F0'][l], MAP_RTOL, MAP_ATOL)
        assert_close(f'F1[{l}]', g['F1'][l], o['F1'][l], MAP_RTOL, MAP_ATOL)
        assert_close(f'M[{l}]', g['M'][l], o['M'][l], MAP_RTOL, MAP_ATOL)
    for r in range(len(b.renders)):
        ok = ~cone_ambiguous(b, o, r)[..., None]
        assert_image(f'image[{r}]', g['images'][r], o['images'][r], b, o, r, mask=ok, smoothed=True)


@pytest.mark.parametrize('name', list(BATCHES))
def test_backward_matches_oracle(name):
    b = BATCHES[name]()
    o0 = oracle_run(b)
    G = loss_grad(b, o0['images']) if name != 'cfg2_mixed' else random_grad(b, 5)
    check_gradients(b, G, o0)
