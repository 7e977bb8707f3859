"""Python binding of libdsm: argument marshalling from torch tensors to the C ABI.

Every step of the render and of its gradient runs in the HIP library; torch
only provides device memory and the current stream.  The functions mirror the
ABI names without the ``dsm_`` prefix.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib

# pipeline stages in launch order (the dsm_stage enum of the C ABI)
STAGES = ('setup', 'bin', 'raster', 'resolve', 'light_aa', 'filter', 'lookup', 'camera_aa', 'bwd_setup',
          'camera_aa_adj', 'lookup_adj', 'filter_adj', 'light_adj', 'vertex_grad', 'light_grad')

__all__ = ['filter_moments', 'version']


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _need_cuda_f32(name, t):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f'{name} must be a contiguous float32 CUDA tensor')


def version() -> str:
    return _lib.lib().dsm_version().decode()


def filter_moments(maps: torch.Tensor, filter: str = 'box', k: int = 5, sigma: float = 0.0,
                   adjoint: bool = False) -> torch.Tensor:
    """Moment filter G (or its transpose) of [n, 2, S, S] maps (Eq. moment1/moment2)."""
    _need_cuda_f32('maps', maps)
    if maps.dim() != 4 or maps.shape[1] != 2 or maps.shape[2] != maps.shape[3]:
        raise ValueError('maps must have shape [n, 2, S, S]')
    out = torch.empty_like(maps)
    _lib.call('dsm_filter_moments', maps.shape[2], maps.shape[0], _lib.FILTERS[filter], k, float(sigma),
              _ptr(maps), _ptr(out), int(adjoint), _stream())
    return out


# ----------------------------------------------------------------------------- plans

def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _cptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class _BatchDesc:
    """Host-side dsm_batch_desc of a batch, with the arrays it points to."""

    def __init__(self, batch):
        L = _lib
        scenes = batch.scenes
        self.num_scenes = len(scenes)
        nv = [len(s.verts) for s in scenes]
        nf = [len(s.faces) for s in scenes]
        self.vert_offsets = _arr(np.concatenate([[0], np.cumsum(nv)]), np.int32)
        self.face_offsets = _arr(np.concatenate([[0], np.cumsum(nf)]), np.int32)
        self.faces = _arr(np.concatenate([s.faces for s in scenes]) if scenes else np.zeros((0, 3)), np.int32)
        self.pose_counts = _arr([getattr(s, 'pose_count', 0) for s in scenes], np.int32)
        self.pose_centers = _arr([getattr(s, 'pose_center', np.zeros(3)) for s in scenes], np.float32)
        self.channels = int(batch.channels)
        lights = (L.LightDesc * max(1, len(batch.lights)))()
        for i, l in enumerate(batch.lights):
            d = lights[i]
            d.type = L.LIGHT_TYPES[l.kind]
            d.scene = l.scene
            d.target[:] = [float(x) for x in l.target]
            d.up[:] = [float(x) for x in l.up]
            d.fov_deg = l.fov_deg
            d.dir_distance = l.dir_distance
            d.ortho_half = l.ortho_half
            d.znear = l.near
            d.zfar = l.far
            d.intensity = l.intensity
            d.resolution = l.resolution
            d.filter = L.FILTERS[l.filter]
            d.k = l.k
            d.sigma = l.sigma
            d.min_variance = l.min_variance
            d.antialias = int(l.antialias)
            d.cube_face = int(getattr(l, 'face', 0))
            d.warp_exponent = float(getattr(l, 'warp_exponent', 0.0))
            d.bleed_reduction = float(getattr(l, 'bleed_reduction', 0.0))
        cams = (L.CameraDesc * max(1, len(batch.cameras)))()
        for i, c in enumerate(batch.cameras):
            d = cams[i]
            d.eye[:] = [float(x) for x in c.eye]
            d.target[:] = [float(x) for x in c.target]
            d.up[:] = [float(x) for x in c.up]
            d.fov_deg = c.fov_deg
            d.znear = c.near
            d.zfar = c.far
            d.width = c.width
            d.height = c.height
            d.scene = c.scene
        rl = []
        rends = (L.RenderDesc * max(1, len(batch.renders)))()
        for i, r in enumerate(batch.renders):
            rends[i].camera = r.camera
            rends[i].light_begin = len(rl)
            rends[i].light_count = len(r.lights)
            rl += list(r.lights)
        self.render_light_list = _arr(rl if rl else [0], np.int32)
        self._keep = (lights, cams, rends)
        desc = L.BatchDesc()
        desc.num_scenes = self.num_scenes
        desc.vert_offsets = _cptr(self.vert_offsets, C.c_int32)
        desc.face_offsets = _cptr(self.face_offsets, C.c_int32)
        desc.faces = _cptr(self.faces, C.c_int32)
        desc.pose_counts = _cptr(self.pose_counts, C.c_int32)
        desc.pose_centers = _cptr(self.pose_centers, C.c_float)
        desc.num_lights = len(batch.lights)
        desc.lights = lights
        desc.num_cameras = len(batch.cameras)
        desc.cameras = cams
        desc.num_renders = len(batch.renders)
        desc.renders = rends
        desc.render_light_list = _cptr(self.render_light_list, C.c_int32)
        desc.channels = self.channels
        desc.camera_antialias = int(getattr(batch, 'antialias_camera', True))
        self.desc = desc


class Plan:
    """A batch of scenes / lights / cameras / renders bound to the HIP library.

    ``batch`` follows the layout of ``scenegen.Batch`` (any object with the
    same attributes works).  The plan owns device copies of faces and
    adjacency; vertices, light parameters and albedo are passed per call."""

    def __init__(self, batch, tile_size: int = 0, bin_capacity_scale: int = 0):
        L = _lib
        bd = _BatchDesc(batch)
        self._desc = bd
        desc = bd.desc
        self.num_scenes = bd.num_scenes
        self.channels = bd.channels
        self.vert_offsets = bd.vert_offsets
        self.face_offsets = bd.face_offsets
        self.faces = bd.faces
        self.pose_counts = bd.pose_counts
        self.pose_centers = bd.pose_centers
        h = C.c_void_p()
        L.call('dsm_plan_create', C.byref(desc), int(tile_size), int(bin_capacity_scale), C.byref(h))
        self.handle = h
        info = L.PlanInfo()
        L.call('dsm_plan_info_get', h, C.byref(info))
        self.info = info
        self.num_lights = len(batch.lights)
        self.render_shapes = [(batch.cameras[r.camera].height, batch.cameras[r.camera].width, self.channels)
                              for r in batch.renders]
        self.view_shapes = [(l.resolution, l.resolution) for l in batch.lights] + \
                           [(c.height, c.width) for c in batch.cameras]
        self.light_res = [l.resolution for l in batch.lights]
        self._scratch = {}

    def __del__(self):
        h = getattr(self, 'handle', None)
        if h is not None and h.value:
            try:
                _lib.lib().dsm_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    # --- memory
    def workspace(self, device='cuda'):
        saved = torch.empty(int(self.info.saved_bytes), dtype=torch.uint8, device=device)
        scratch = torch.empty(int(self.info.scratch_bytes), dtype=torch.uint8, device=device)
        return saved, scratch

    def scratch(self, device='cuda'):
        """The plan's own scratch buffer on `device`, allocated on first use
        and reused by every later call (scratch carries nothing from a forward
        to its backward; calls on one plan are ordered on one stream)."""
        dev = torch.device(device)
        if dev.type == 'cuda' and dev.index is None:
            dev = torch.device('cuda', torch.cuda.current_device())
        t = self._scratch.get(dev)
        if t is None:
            t = torch.empty(int(self.info.scratch_bytes), dtype=torch.uint8, device=dev)
            self._scratch[dev] = t
        return t

    def split_images(self, flat):
        out, o = [], 0
        for (H, W, Cc) in self.render_shapes:
            n = H * W * Cc
            out.append(flat[o:o + n].view(H, W, Cc))
            o += n
        return out

    # --- raw calls (tensors already allocated)
    def forward(self, verts, light_params, albedo, saved, scratch, images=None):
        for n, t in (('verts', verts), ('light_params', light_params), ('albedo', albedo)):
            _need_cuda_f32(n, t)
        if images is None:
            images = torch.empty(int(self.info.image_floats), dtype=torch.float32, device=verts.device)
        _lib.call('dsm_forward', self.handle, _ptr(verts), _ptr(light_params), _ptr(albedo), _ptr(saved),
                  saved.numel(), _ptr(scratch), scratch.numel(), _ptr(images), _stream())
        return images

    def backward(self, verts, light_params, albedo, saved, scratch, grad_images, want_albedo=True):
        _need_cuda_f32('grad_images', grad_images)
        gv = torch.empty_like(verts)
        gl = torch.empty_like(light_params)
        ga = torch.empty_like(albedo) if want_albedo else None
        _lib.call('dsm_backward', self.handle, _ptr(verts), _ptr(light_params), _ptr(albedo), _ptr(saved),
                  saved.numel(), _ptr(scratch), scratch.numel(), _ptr(grad_images), _ptr(gv), _ptr(gl), _ptr(ga),
                  _stream())
        return gv, gl, ga

    def pose_forward(self, local, poses):
        _need_cuda_f32('local', local)
        _need_cuda_f32('poses', poses)
        world = torch.empty_like(local)
        _lib.call('dsm_pose_forward', self.handle, _ptr(local), _ptr(poses), _ptr(world), _stream())
        return world

    def pose_backward(self, local, poses, grad_world):
        gp = torch.empty_like(poses)
        _lib.call('dsm_pose_backward', self.handle, _ptr(local), _ptr(poses), _ptr(grad_world), _ptr(gp), _stream())
        return gp

    # --- stage getters
    def view_keys(self, saved, view):
        H, W = self.view_shapes[view]
        out = torch.empty(H * W, dtype=torch.int64, device=saved.device)
        _lib.call('dsm_get_view_keys', self.handle, _ptr(saved), int(view), _ptr(out), _stream())
        return out.view(H, W)

    def light_maps(self, saved, scratch, light, which):
        S = self.light_res[light]
        out = torch.empty(2, S, S, dtype=torch.float32, device=saved.device)
        _lib.call('dsm_get_light_maps', self.handle, _ptr(saved), _ptr(scratch), int(light), int(which), _ptr(out),
                  _stream())
        return out

    def image0(self, saved, render):
        H, W, Cc = self.render_shapes[render]
        out = torch.empty(H, W, Cc, dtype=torch.float32, device=saved.device)
        _lib.call('dsm_get_render_image0', self.handle, _ptr(saved), int(render), _ptr(out), _stream())
        return out

    def stats(self, saved):
        """Counters of the forward that wrote `saved`."""
        st = _lib.Stats()
        _lib.call('dsm_get_stats', self.handle, _ptr(saved), C.byref(st), _stream())
        return dict(culled=st.culled_triangles, pairs=st.binned_pairs, overflow=st.overflow_triangles,
                    bad_indices=st.bad_indices)

    # --- graphs
    def graph_capture(self, stream, local, poses, verts, light_params, albedo, saved, scratch, images, grad_images,
                      grad_verts, grad_light_params, grad_albedo, grad_poses):
        with torch.cuda.stream(stream):
            _lib.call('dsm_graph_capture', self.handle, _ptr(local), _ptr(poses), _ptr(verts), _ptr(light_params),
                      _ptr(albedo), _ptr(saved), saved.numel(), _ptr(scratch), scratch.numel(), _ptr(images),
                      _ptr(grad_images), _ptr(grad_verts), _ptr(grad_light_params), _ptr(grad_albedo),
                      _ptr(grad_poses), C.c_void_p(stream.cuda_stream))

    def graph_launch(self, stream):
        _lib.call('dsm_graph_launch', self.handle, C.c_void_p(stream.cuda_stream))

    def time_stages(self, stream, verts, light_params, albedo, saved, scratch, images, grad_images, grad_verts,
                    grad_light_params, grad_albedo, reps, flush=None):
        """Mean duration (ms) of every pipeline stage over `reps` eager
        forward + backward passes on `stream`, timed with HIP events.  With
        `flush` (a device tensor, e.g. 1 GiB), the library overwrites it
        before every stage so that each stage starts with cold caches."""
        ms = (C.c_float * len(STAGES))()
        with torch.cuda.stream(stream):
            _lib.call('dsm_time_stages', self.handle, _ptr(verts), _ptr(light_params), _ptr(albedo), _ptr(saved),
                      saved.numel(), _ptr(scratch), scratch.numel(), _ptr(images), _ptr(grad_images),
                      _ptr(grad_verts), _ptr(grad_light_params), _ptr(grad_albedo), int(reps),
                      _ptr(flush), 0 if flush is None else flush.numel() * flush.element_size(), ms,
                      C.c_void_p(stream.cuda_stream))
        return dict(zip(STAGES, (float(x) for x in ms)))


def autotune(batch, verts, light_params, albedo, grad_images, reps: int = 3, cache_path: str | None = None,
             stream=None):
    """Pick the plan's (tile_size, bin_capacity_scale) by timing forward +
    backward for every candidate on these inputs (dsm_autotune).  Returns
    (tile_size, bin_capacity_scale, ms per forward + backward)."""
    for name, t in (('verts', verts), ('light_params', light_params), ('albedo', albedo),
                    ('grad_images', grad_images)):
        _need_cuda_f32(name, t)
    bd = _BatchDesc(batch)
    tile = C.c_int32()
    scale = C.c_int32()
    ms = C.c_float()
    st = stream if stream is not None else torch.cuda.current_stream()
    path = cache_path.encode() if cache_path else None
    _lib.call('dsm_autotune', C.byref(bd.desc), _ptr(verts), _ptr(light_params), _ptr(albedo), _ptr(grad_images),
              int(reps), path, C.c_void_p(st.cuda_stream), C.byref(tile), C.byref(scale), C.byref(ms))
    return int(tile.value), int(scale.value), float(ms.value)


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, verts, light_params, albedo):
        saved = torch.empty(int(plan.info.saved_bytes), dtype=torch.uint8, device=verts.device)
        images = plan.forward(verts, light_params, albedo, saved, plan.scratch(verts.device))
        ctx.plan = plan
        ctx.save_for_backward(verts, light_params, albedo, saved)
        return images

    @staticmethod
    def backward(ctx, grad_images):
        verts, light_params, albedo, saved = ctx.saved_tensors
        gv, gl, ga = ctx.plan.backward(verts, light_params, albedo, saved, ctx.plan.scratch(verts.device),
                                       grad_images.contiguous(),
                                       want_albedo=ctx.needs_input_grad[3])
        return None, gv, gl, ga


class _Pose(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, local, poses):
        ctx.plan = plan
        ctx.save_for_backward(local, poses)
        return plan.pose_forward(local, poses)

    @staticmethod
    def backward(ctx, grad_world):
        local, poses = ctx.saved_tensors
        return None, None, ctx.plan.pose_backward(local, poses, grad_world.contiguous())


def render(plan: Plan, verts, light_params, albedo):
    """Differentiable render of every image of the plan (flat float32 tensor;
    ``plan.split_images`` gives per-render [H, W, C] views)."""
    return _Render.apply(plan, verts, light_params, albedo)


def pose(plan: Plan, local, poses):
    """Differentiable rigid pose of each scene's posed vertex prefix."""
    return _Pose.apply(plan, local, poses)


def batch_inputs(batch, device='cuda'):
    """Concatenated float32 device tensors (verts, light params, albedo, poses) of a batch."""
    verts = torch.as_tensor(np.concatenate([s.verts for s in batch.scenes]).astype(np.float32), device=device)
    lp = torch.as_tensor(np.stack([l.param for l in batch.lights]).astype(np.float32), device=device)
    alb = torch.as_tensor(np.concatenate([s.albedo for s in batch.scenes]).astype(np.float32), device=device)
    poses = torch.as_tensor(np.stack([getattr(s, 'pose', np.zeros(6)) for s in batch.scenes]).astype(np.float32),
                            device=device)
    return verts.contiguous(), lp.contiguous(), alb.contiguous(), poses.contiguous()


__all__ += ['Plan', 'render', 'pose', 'batch_inputs']
