"""GPU parity of the full forward pass (raster keys bit-exact; moments,
smoothed and filtered maps, shaded images within tolerance) and of the
backward pass (gradients w.r.t. vertices, light parameters, albedo, pose)
against the oracle, through the C ABI."""
import numpy as np
import pytest

import scenegen as sg
from parity_helpers import (assert_image, IMG_ATOL, IMG_RTOL, MAP_ATOL, MAP_RTOL, assert_close, check_gradients,
                            cone_ambiguous, gpu_run, loss_grad, oracle_run, random_grad)

pytestmark = pytest.mark.gpu


def cfg0_ragged():
    b = sg.config0()
    b.lights[0].resolution = 200
    b.cameras[0].width, b.cameras[0].height = 250, 190
    return b


def cfg1_small():
    b = sg.config1()
    b.lights[0].resolution = 300
    b.cameras[0].width, b.cameras[0].height = 280, 232
    return b


def cfg2_small(n=3, res=176, with_pose=False):
    return sg.config2(n_scenes=n, resolution=res, with_pose=with_pose)


BATCHES = {'cfg0': sg.config0, 'cfg0_ragged': cfg0_ragged, 'cfg1_small': cfg1_small, 'cfg2_small': cfg2_small}


def check_forward(b, g, o):
    for v, (kg, ko) in enumerate(zip(g['keys'], o['keys'])):
        assert kg.shape == ko.shape
        diff = kg != ko
        assert not diff.any(), f'view {v}: {int(diff.sum())} keys differ'
    for l in range(len(b.lights)):
        assert_close(f'F0[{l}]', g['F0'][l], o['F0'][l], MAP_RTOL, MAP_ATOL)
        assert_close(f'F1[{l}]', g['F1'][l], o['F1'][l], MAP_RTOL, MAP_ATOL)
        assert_close(f'M[{l}]', g['M'][l], o['M'][l], MAP_RTOL, MAP_ATOL)
    for r in range(len(b.renders)):
        ok = ~cone_ambiguous(b, o, r)[..., None]
        assert_image(f'img0[{r}]', g['img0'][r], o['img0'][r], b, o, r, mask=ok)
        assert_image(f'image[{r}]', g['images'][r], o['images'][r], b, o, r, mask=ok, smoothed=True)
    assert g['stats']['culled'] == 0 and o['culled'] == 0
    assert g['stats']['bad_indices'] == 0


@pytest.mark.parametrize('name', list(BATCHES))
def test_forward_matches_oracle(name):
    b = BATCHES[name]()
    g = gpu_run(b)
    o = oracle_run(b)
    check_forward(b, g, o)


@pytest.mark.parametrize('tile,bins', [(8, 0), (32, 0), (16, 1)])
def test_keys_independent_of_tile_and_bin_capacity(tile, bins):
    """Tile size and bin capacity (1 pair per triangle forces most triangles
    through the overflow path) must not change a single key."""
    b = cfg2_small(2, 160)
    ref = gpu_run(b)
    g = gpu_run(b, tile_size=tile, bin_scale=bins)
    for kr, kg in zip(ref['keys'], g['keys']):
        assert np.array_equal(kr, kg)
    for a, c in zip(ref['images'], g['images']):
        assert np.array_equal(a, c)
    if bins == 1:
        assert g['stats']['overflow'] > 0


def test_run_twice_bit_identical_forward():
    b = cfg1_small()
    a = gpu_run(b)
    c = gpu_run(b)
    for x, y in zip(a['keys'], c['keys']):
        assert np.array_equal(x, y)
    for x, y in zip(a['images'], c['images']):
        assert np.array_equal(x, y)


@pytest.mark.parametrize('name', ['cfg0', 'cfg0_ragged', 'cfg1_small'])
def test_backward_matches_oracle_loss_gradient(name):
    b = BATCHES[name]()
    o0 = oracle_run(b)
    check_gradients(b, loss_grad(b, o0['images']), o0)


def test_backward_random_cotangent_cfg0():
    b = sg.config0()
    check_gradients(b, random_grad(b, 3))


def test_pose_forward_and_backward():
    b = cfg2_small(2, 160, with_pose=True)
    o0 = oracle_run(b, pose=True)
    check_forward(b, gpu_run(b, pose=True), o0)
    check_gradients(b, loss_grad(b, o0['images']), o0, pose=True, groups=['gpose', 'glight'])


def cfg3_small():
    """Multi-view: 2 point lights x 3 cameras of one displaced sphere; each
    camera view is shared by two renders, each light by three."""
    return sg.config3(n_lat=20, sm_res=160, view_res=120, n_cams=3, n_lights=2)


def cfg4_small():
    """Complex-scene shape at small size: 4 objects, RGB albedo, 3 point lights
    summed in one render, non-square camera."""
    return sg.config4(sm_res=192, width=200, height=112, n_objects=4, detail=0.15)


@pytest.mark.parametrize('name', ['cfg3_small', 'cfg4_small'])
def test_forward_and_backward_multi_view_and_rgb(name):
    b = {'cfg3_small': cfg3_small, 'cfg4_small': cfg4_small}[name]()
    o0 = oracle_run(b)
    check_forward(b, gpu_run(b), o0)
    check_gradients(b, random_grad(b, 7), o0)
