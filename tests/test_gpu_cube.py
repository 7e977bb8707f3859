"""GPU parity of cube shadow maps for omnidirectional point lights (six
cube-face lights sharing one position; Sec. 3 box of planes, Sec. 5): keys of
all six light views and the camera bit-exact, moment maps, images and the
loss gradients within the tolerances of the other parity tests."""
import numpy as np
import pytest

import scenegen as sg
from parity_helpers import (assert_image, GRAD_ELEM_FRAC, GRAD_FLOOR_ELEM_FRAC, GRAD_FLOOR_TOL, GRAD_TOL, IMG_ATOL, IMG_RTOL, MAP_ATOL, MAP_RTOL, assert_close,
                            check_gradients, cone_ambiguous, gpu_run, normwise, oracle_run, random_grad, loss_grad)

pytestmark = pytest.mark.gpu


def cube_batch(res=136, k=5, filt='box', antialias=True):
    b = sg.cube_light_scene(resolution=res, view=128, k=k, antialias=antialias)
    for L in b.lights:
        L.filter = filt
    b.cameras[0].width, b.cameras[0].height = 144, 112
    return b


def check_forward(b, g, o):
    for v, (kg, ko) in enumerate(zip(g['keys'], o['keys'])):
        assert kg.shape == ko.shape
        diff = kg != ko
        assert not diff.any(), f'view {v}: {int(diff.sum())} keys differ'
    for l in range(len(b.lights)):
        assert_close(f'F0[{l}]', g['F0'][l], o['F0'][l], MAP_RTOL, MAP_ATOL)
        assert_close(f'F1[{l}]', g['F1'][l], o['F1'][l], MAP_RTOL, MAP_ATOL)
        assert_close(f'M[{l}]', g['M'][l], o['M'][l], MAP_RTOL, MAP_ATOL)
    # the +y face sees nothing: its maps hold the far value everywhere (to
    # the rounding of the float32 bilinear weights of its padding)
    assert np.allclose(g['M'][2], 1.0, rtol=0, atol=1e-6)
    for r in range(len(b.renders)):
        # face choice within a 1e-4 relative gap of the two largest |d_a| is a tie
        ok = ~cone_ambiguous(b, o, r, margin=1e-4)[..., None]
        assert ok.mean() > 0.99
        assert_image(f'img0[{r}]', g['img0'][r], o['img0'][r], b, o, r, mask=ok)
        assert_image(f'image[{r}]', g['images'][r], o['images'][r], b, o, r, mask=ok, smoothed=True)
    # triangles behind a face's light plane are dropped in that face alone
    assert g['stats']['culled'] == o['culled'] > 0
    assert g['stats']['bad_indices'] == 0


@pytest.mark.parametrize('res,k,filt', [(136, 5, 'box'), (100, 7, 'gaussian'), (37, 1, 'box'), (64, 9, 'gaussian')])
def test_cube_forward_matches_oracle(res, k, filt):
    b = cube_batch(res, k, filt)
    check_forward(b, gpu_run(b), oracle_run(b))


def test_cube_backward_matches_oracle_loss_gradient():
    b = cube_batch()
    o0 = oracle_run(b)

    def faces(share, g, o):
        # the shared position's gradient is the sum over the six faces
        tol, elem = (GRAD_TOL, GRAD_ELEM_FRAC) if share == 'rest' else (GRAD_FLOOR_TOL, GRAD_FLOOR_ELEM_FRAC)
        if np.any(o['glight']):
            normwise(f'glight, sum over faces ({share})', g['glight'].sum(0), o['glight'].sum(0), tol, elem)
        assert np.all(g['glight'][2] == 0.0)       # the empty +y face

    check_gradients(b, loss_grad(b, o0['images']), o0, extra=faces)


@pytest.mark.parametrize('res,k', [(120, 3), (48, 9)])
def test_cube_backward_random_upstream_without_light_smoothing(res, k):
    b = cube_batch(res, k, 'box', antialias=False)
    # Without light-view smoothing the moment maps keep sharp steps (only the
    # k-box filter), and the light-position gradient, which enters through
    # the map position u = L(x), is steep in u: perturbing the oracle's u by
    # 1, 2 and 4 float32 ulps moves this share of its light gradient by
    # 3.6e-5, 7.2e-5 and 1.4e-4 at 120^2 / k = 3 (1.5e-5 ... 6.1e-5 at
    # 48^2 / k = 9).  The kernels form u with a few ulps of error, so the
    # bound is twice the 4-ulp sensitivity.
    check_gradients(b, random_grad(b, 11), groups=['glight', 'gverts'], rest_tol=3e-4)
