"""dsm_forward_static_scratch, the forward for callers that cannot allocate
device memory, called through the C ABI: it returns what dsm_forward
returns with a caller scratch buffer (images, depth keys and filtered maps
bit for bit), on two calls in a row, the second on a smaller plan, and a
backward after it gives dsm_forward's gradients.  Plans whose forward
temporaries exceed the library's static array are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import scenegen as sg

pytestmark = pytest.mark.gpu

DSM_ERR_WORKSPACE_TOO_SMALL = 3
STATIC_BYTES = 64 << 20


def _p(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _case(make):
    from paper_2308_10896_amd import dsm
    b = make()
    plan = dsm.Plan(b)
    verts, lp, alb, _ = dsm.batch_inputs(b)
    return b, plan, verts, lp, alb


def _outputs(plan, saved, images, scratch=None):
    torch.cuda.synchronize()
    keys = [plan.view_keys(saved, v).cpu().numpy() for v in range(len(plan.view_shapes))]
    maps = [plan.light_maps(saved, scratch, l, 2).cpu().numpy() for l in range(plan.num_lights)]
    return images.cpu().numpy(), keys, maps


def _backward(lib, plan, verts, lp, alb, saved, gimg, stream):
    scratch = torch.empty(int(plan.info.scratch_bytes), dtype=torch.uint8, device='cuda')
    gv, gl, ga = torch.empty_like(verts), torch.empty_like(lp), torch.empty_like(alb)
    st = lib.dsm_backward(plan.handle, _p(verts), _p(lp), _p(alb), _p(saved), saved.numel(), _p(scratch),
                          scratch.numel(), _p(gimg), _p(gv), _p(gl), _p(ga), C.c_void_p(stream.cuda_stream))
    assert st == 0, st
    stream.synchronize()
    return gv.cpu().numpy(), gl.cpu().numpy(), ga.cpu().numpy()


def test_static_scratch_forward_matches_forward_twice():
    from paper_2308_10896_amd import _lib
    lib = _lib.lib()
    stream = torch.cuda.Stream()
    cases = [lambda: sg.config2(n_scenes=3, resolution=176),          # first call: 3 scenes at 176^2
             lambda: sg.config0()]                                    # second call: a smaller plan
    sizes = []
    for make in cases:
        b, plan, verts, lp, alb = _case(make)
        fwd_bytes = int(plan.info.forward_scratch_bytes)
        assert 0 < fwd_bytes <= min(int(plan.info.scratch_bytes), STATIC_BYTES)
        sizes.append(fwd_bytes)
        print(f'{b.name}: forward scratch {fwd_bytes} B of {int(plan.info.scratch_bytes)} B', flush=True)

        # reference: dsm_forward with a caller scratch buffer
        saved_a, scratch_a = plan.workspace()
        img_a = torch.empty(int(plan.info.image_floats), device='cuda')
        st = lib.dsm_forward(plan.handle, _p(verts), _p(lp), _p(alb), _p(saved_a), saved_a.numel(), _p(scratch_a),
                             scratch_a.numel(), _p(img_a), C.c_void_p(stream.cuda_stream))
        assert st == 0, st
        stream.synchronize()
        ref = _outputs(plan, saved_a, img_a, scratch_a)

        # the static-scratch forward into a fresh saved buffer (garbage-filled)
        saved_b = torch.randint(0, 256, saved_a.shape, dtype=torch.uint8,
                                generator=torch.Generator().manual_seed(7)).to('cuda')
        img_b = torch.full_like(img_a, float('nan'))
        st = lib.dsm_forward_static_scratch(plan.handle, _p(verts), _p(lp), _p(alb), _p(saved_b), saved_b.numel(),
                                            _p(img_b), C.c_void_p(stream.cuda_stream))
        assert st == 0, st
        stream.synchronize()
        got = _outputs(plan, saved_b, img_b, scratch_a)
        assert np.array_equal(got[0], ref[0]), 'images differ'
        for v, (x, y) in enumerate(zip(got[1], ref[1])):
            assert np.array_equal(x, y), f'keys of view {v} differ'
        for l, (x, y) in enumerate(zip(got[2], ref[2])):
            assert np.array_equal(x, y), f'filtered maps of light {l} differ'

        # backward from either forward's saved state: the same gradients
        rng = np.random.default_rng(5)
        gimg = torch.as_tensor(rng.standard_normal(int(plan.info.image_floats)).astype(np.float32), device='cuda')
        ga = _backward(lib, plan, verts, lp, alb, saved_a, gimg, stream)
        gb = _backward(lib, plan, verts, lp, alb, saved_b, gimg, stream)
        for name, x, y in zip(('verts', 'light', 'albedo'), gb, ga):
            n = np.linalg.norm(y)
            err = np.linalg.norm(x - y) / max(n, 1e-30)
            # the map-gradient scatter adds floats atomically, in varying order
            assert err <= 1e-5, f'{name}: {err:.2e}'
    assert sizes[1] < sizes[0]


def test_static_scratch_refuses_plans_beyond_its_size():
    from paper_2308_10896_amd import _lib, dsm
    lib = _lib.lib()
    b = sg.config0()
    b.lights[0].resolution = 4096            # smoothed maps alone: 2 * 4096^2 floats = 128 MiB
    plan = dsm.Plan(b)
    assert int(plan.info.forward_scratch_bytes) > STATIC_BYTES
    verts, lp, alb, _ = dsm.batch_inputs(b)
    saved = torch.empty(int(plan.info.saved_bytes), dtype=torch.uint8, device='cuda')
    img = torch.empty(int(plan.info.image_floats), device='cuda')
    st = lib.dsm_forward_static_scratch(plan.handle, _p(verts), _p(lp), _p(alb), _p(saved), saved.numel(),
                                        _p(img), None)
    assert st == DSM_ERR_WORKSPACE_TOO_SMALL, st
    # on a plan that fits, a saved buffer below the plan's size is refused
    b = sg.config0()
    plan = dsm.Plan(b)
    verts, lp, alb, _ = dsm.batch_inputs(b)
    saved = torch.empty(int(plan.info.saved_bytes), dtype=torch.uint8, device='cuda')
    img = torch.empty(int(plan.info.image_floats), device='cuda')
    st = lib.dsm_forward_static_scratch(plan.handle, _p(verts), _p(lp), _p(alb), _p(saved), saved.numel() - 256,
                                        _p(img), None)
    assert st == DSM_ERR_WORKSPACE_TOO_SMALL, st
