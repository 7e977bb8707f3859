"""ctypes loader for libdsm.so (the C ABI declared in include/dsm.h).

Argument marshalling only.  There is no fallback: if the library is missing
or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libdsm.so')

DSM_OK = 0
STATUS = {0: 'ok', 1: 'invalid argument', 2: 'out of memory', 3: 'workspace too small', 4: 'unsupported',
          5: 'no device', 6: 'HIP error', 7: 'device fault'}

LIGHT_TYPES = {'directional': 0, 'point': 1, 'spot': 2, 'cubeface': 3}
FILTERS = {'box': 0, 'gaussian': 1}


class DSMError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f'{fn} failed: {STATUS.get(status, status)} ({status})')
        self.status = status


class LightDesc(C.Structure):
    _fields_ = [('type', C.c_int32), ('scene', C.c_int32), ('target', C.c_float * 3), ('up', C.c_float * 3),
                ('fov_deg', C.c_float), ('dir_distance', C.c_float), ('ortho_half', C.c_float),
                ('znear', C.c_float), ('zfar', C.c_float), ('intensity', C.c_float),
                ('resolution', C.c_int32), ('filter', C.c_int32), ('k', C.c_int32), ('sigma', C.c_float),
                ('min_variance', C.c_float), ('antialias', C.c_int32), ('cube_face', C.c_int32),
                ('warp_exponent', C.c_float), ('bleed_reduction', C.c_float)]


class CameraDesc(C.Structure):
    _fields_ = [('eye', C.c_float * 3), ('target', C.c_float * 3), ('up', C.c_float * 3),
                ('fov_deg', C.c_float), ('znear', C.c_float), ('zfar', C.c_float),
                ('width', C.c_int32), ('height', C.c_int32), ('scene', C.c_int32)]


class RenderDesc(C.Structure):
    _fields_ = [('camera', C.c_int32), ('light_begin', C.c_int32), ('light_count', C.c_int32)]


class BatchDesc(C.Structure):
    _fields_ = [('num_scenes', C.c_int32), ('vert_offsets', C.POINTER(C.c_int32)),
                ('face_offsets', C.POINTER(C.c_int32)), ('faces', C.POINTER(C.c_int32)),
                ('pose_counts', C.POINTER(C.c_int32)), ('pose_centers', C.POINTER(C.c_float)),
                ('num_lights', C.c_int32), ('lights', C.POINTER(LightDesc)),
                ('num_cameras', C.c_int32), ('cameras', C.POINTER(CameraDesc)),
                ('num_renders', C.c_int32), ('renders', C.POINTER(RenderDesc)),
                ('render_light_list', C.POINTER(C.c_int32)), ('channels', C.c_int32),
                ('camera_antialias', C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [('total_vertices', C.c_int64), ('total_faces', C.c_int64), ('image_floats', C.c_int64),
                ('saved_bytes', C.c_int64), ('scratch_bytes', C.c_int64), ('map_floats', C.c_int64),
                ('tile_size', C.c_int32), ('bin_capacity_scale', C.c_int32),
                ('forward_scratch_bytes', C.c_int64)]


class Stats(C.Structure):
    _fields_ = [('culled_triangles', C.c_uint64), ('binned_pairs', C.c_uint64),
                ('overflow_triangles', C.c_uint64), ('bad_indices', C.c_uint64)]


P = C.c_void_p
I32 = C.c_int32
SZ = C.c_size_t
F32 = C.c_float

_SIGNATURES = {
    'dsm_version': (C.c_char_p, []),
    'dsm_status_string': (C.c_char_p, [C.c_int]),
    'dsm_plan_create': (C.c_int, [C.POINTER(BatchDesc), I32, I32, C.POINTER(P)]),
    'dsm_plan_info_get': (C.c_int, [P, C.POINTER(PlanInfo)]),
    'dsm_plan_destroy': (None, [P]),
    'dsm_forward': (C.c_int, [P, P, P, P, P, SZ, P, SZ, P, P]),
    'dsm_forward_static_scratch': (C.c_int, [P, P, P, P, P, SZ, P, P]),
    'dsm_backward': (C.c_int, [P, P, P, P, P, SZ, P, SZ, P, P, P, P, P]),
    'dsm_pose_forward': (C.c_int, [P, P, P, P, P]),
    'dsm_pose_backward': (C.c_int, [P, P, P, P, P, P]),
    'dsm_graph_capture': (C.c_int, [P, P, P, P, P, P, P, SZ, P, SZ, P, P, P, P, P, P, P]),
    'dsm_graph_launch': (C.c_int, [P, P]),
    'dsm_get_view_keys': (C.c_int, [P, P, I32, P, P]),
    'dsm_get_light_maps': (C.c_int, [P, P, P, I32, I32, P, P]),
    'dsm_get_render_image0': (C.c_int, [P, P, I32, P, P]),
    'dsm_get_stats': (C.c_int, [P, P, C.POINTER(Stats), P]),
    'dsm_filter_moments': (C.c_int, [I32, I32, I32, I32, F32, P, P, I32, P]),
    'dsm_autotune': (C.c_int, [C.POINTER(BatchDesc), P, P, P, P, I32, C.c_char_p, P, C.POINTER(I32),
                               C.POINTER(I32), C.POINTER(C.c_float)]),
    'dsm_time_stages': (C.c_int, [P, P, P, P, P, SZ, P, SZ, P, P, P, P, P, I32, P, SZ, C.POINTER(C.c_float), P]),
}

_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f'{LIB_PATH} is missing: build it with `python -m paper_2308_10896_amd.build`')
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(h, name, None)
            if fn is None:      # reported by the ABI test; calling it raises AttributeError
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def check(fn, status):
    if status != DSM_OK:
        raise DSMError(fn, status)


def call(name, *args):
    check(name, getattr(lib(), name)(*args))
