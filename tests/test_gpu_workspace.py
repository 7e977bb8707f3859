"""The saved / scratch contract of the C ABI: dsm_backward reads only what
the matching forward left in `saved`, so any scratch buffer of the plan's
size serves it.  A backward given a fresh zero-filled scratch, or the
forward's scratch overwritten with garbage, returns the gradients of a
backward given the forward's own scratch untouched."""
import ctypes as C

import numpy as np
import pytest
import torch

import scenegen as sg

pytestmark = pytest.mark.gpu


def _p(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _backward(lib, plan, verts, lp, alb, saved, scratch, gimg, stream):
    gv, gl, ga = torch.empty_like(verts), torch.empty_like(lp), torch.empty_like(alb)
    st = lib.dsm_backward(plan.handle, _p(verts), _p(lp), _p(alb), _p(saved), saved.numel(), _p(scratch),
                          scratch.numel(), _p(gimg), _p(gv), _p(gl), _p(ga), C.c_void_p(stream.cuda_stream))
    assert st == 0, st
    stream.synchronize()
    return gv.cpu().numpy(), gl.cpu().numpy(), ga.cpu().numpy()


@pytest.mark.parametrize('make', [lambda: sg.config2(n_scenes=3, resolution=176), sg.config0,
                                  lambda: sg.cube_light_scene(resolution=64, view=96)],
                         ids=['cfg2_small', 'cfg0', 'cube'])
def test_backward_needs_only_saved(make):
    from paper_2308_10896_amd import _lib, dsm
    lib = _lib.lib()
    b = make()
    plan = dsm.Plan(b)
    verts, lp, alb, _ = dsm.batch_inputs(b)
    saved, scratch = plan.workspace()
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(5)
    gimg = torch.as_tensor(rng.standard_normal(int(plan.info.image_floats)).astype(np.float32), device='cuda')
    images = torch.empty(int(plan.info.image_floats), device='cuda')

    def forward():
        st = lib.dsm_forward(plan.handle, _p(verts), _p(lp), _p(alb), _p(saved), saved.numel(), _p(scratch),
                             scratch.numel(), _p(images), C.c_void_p(stream.cuda_stream))
        assert st == 0, st
        stream.synchronize()

    forward()
    ref = _backward(lib, plan, verts, lp, alb, saved, scratch, gimg, stream)

    forward()
    fresh = torch.zeros_like(scratch)
    got_fresh = _backward(lib, plan, verts, lp, alb, saved, fresh, gimg, stream)

    forward()
    scratch.copy_(torch.randint(0, 256, scratch.shape, dtype=torch.uint8, generator=torch.Generator().manual_seed(3))
                  .to(scratch.device))
    got_garbage = _backward(lib, plan, verts, lp, alb, saved, scratch, gimg, stream)

    for got in (got_fresh, got_garbage):
        for name, g, r in zip(('verts', 'light', 'albedo'), got, ref):
            assert np.isfinite(g).all(), name
            n = np.linalg.norm(r)
            err = np.linalg.norm(g - r) / max(n, 1e-30)
            # float atomics in the map-gradient scatter sum in varying order
            assert err <= 1e-5, f'{name}: {err:.2e}'
