"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/dsm.h declares, and argument validation
rejects bad input before anything reaches the device."""
import ctypes as C
import os
import re

import pytest

from paper_2308_10896_amd import dsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, 'include', 'dsm.h')).read()
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    return sorted(set(re.findall(r'\b(dsm_[a-z_0-9]+)\s*\(', text)))


def test_library_exports_every_declared_symbol():
    from paper_2308_10896_amd import _lib
    lib = _lib.lib()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib._SIGNATURES), set(names) ^ set(_lib._SIGNATURES)


def test_version_and_status_strings():
    from paper_2308_10896_amd import _lib
    lib = _lib.lib()
    assert b'gfx950' in lib.dsm_version()
    for s in range(8):
        assert lib.dsm_status_string(s)


def test_filter_validation_on_host():
    from paper_2308_10896_amd import _lib
    lib = _lib.lib()
    # even k, k > S, k > 31, negative count: rejected before any device call
    assert lib.dsm_filter_moments(16, 1, 0, 4, 0.0, 1, 2, 0, None) == 1
    assert lib.dsm_filter_moments(4, 1, 0, 5, 0.0, 1, 2, 0, None) == 1
    assert lib.dsm_filter_moments(64, 1, 0, 33, 0.0, 1, 2, 0, None) == 1
    assert lib.dsm_filter_moments(64, -1, 0, 5, 0.0, 1, 2, 0, None) == 1
    assert lib.dsm_filter_moments(64, 1, 7, 5, 0.0, 1, 2, 0, None) == 1
    # null pointers
    assert lib.dsm_filter_moments(64, 1, 0, 5, 0.0, None, 2, 0, None) == 1
    # zero maps is a no-op
    assert lib.dsm_filter_moments(64, 0, 0, 5, 0.0, None, None, 0, None) == 0


def test_stage_names_follow_header_enum():
    text = open(os.path.join(ROOT, 'include', 'dsm.h')).read()
    body = text[text.index('DSM_STAGE_SETUP = 0'):text.index('} dsm_stage;')]
    names = re.findall(r'DSM_STAGE_([A-Z_]+)', body)
    assert names[-1] == 'COUNT'
    assert tuple(n.lower() for n in names[:-1]) == dsm.STAGES


def test_autotune_validation_on_host():
    import ctypes as C
    import scenegen as sg
    from paper_2308_10896_amd import _lib
    lib = _lib.lib()
    t, s, ms = C.c_int32(), C.c_int32(), C.c_float()
    # null description / outputs, bad repetition count: rejected before any device call
    assert lib.dsm_autotune(None, None, None, None, None, 1, None, None, C.byref(t), C.byref(s), None) == 1
    bd = dsm._BatchDesc(sg.config0())
    assert lib.dsm_autotune(C.byref(bd.desc), None, None, None, None, 1, None, None, None, C.byref(s), None) == 1
    assert lib.dsm_autotune(C.byref(bd.desc), None, None, None, None, 0, None, None, C.byref(t), C.byref(s),
                            None) == 1
    # a valid request on a host without a GPU
    import torch
    if not torch.cuda.is_available():
        assert lib.dsm_autotune(C.byref(bd.desc), None, None, None, None, 1, None, None, C.byref(t), C.byref(s),
                                C.byref(ms)) == 5


def test_light_desc_mirror_matches_header():
    """The binding's ctypes mirror of dsm_light_desc lists the header's
    members in order (all 32-bit), so the two agree on size and offsets."""
    from paper_2308_10896_amd import _lib
    text = open(os.path.join(ROOT, 'include', 'dsm.h')).read()
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    body = text[:text.index('} dsm_light_desc;')]
    body = body[body.rindex('typedef struct {') + len('typedef struct {'):]
    names = []
    for decl in body.split(';'):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(None, 1)[1].split(','):
            m = re.match(r'\s*([a-z_0-9]+)\s*(\[(\d+)\])?', part)
            names.append((m.group(1), int(m.group(3) or 1)))
    fields = [(n, C.sizeof(t) // 4) for n, t in _lib.LightDesc._fields_]
    assert fields == names
    assert C.sizeof(_lib.LightDesc) == 4 * sum(k for _, k in names)


def test_cube_face_light_validation_on_host():
    """A cube-face light needs a face index in 0..5; unknown light types are
    rejected; both before any device call."""
    import scenegen as sg
    from paper_2308_10896_amd import _lib
    lib = _lib.lib()
    for face, typ in ((6, 3), (-1, 3), (0, 4)):
        b = sg.cube_light_scene(resolution=32, view=32)
        bd = dsm._BatchDesc(b)
        bd.desc.lights[2].cube_face = face
        bd.desc.lights[2].type = typ
        h = C.c_void_p()
        assert lib.dsm_plan_create(C.byref(bd.desc), 0, 0, C.byref(h)) == 1


def test_cube_group_validation_on_host():
    """The six faces of a cube light must be consecutive lights with faces
    0..5 and one map size and filter; a broken group is rejected before any
    device call."""
    import scenegen as sg
    from paper_2308_10896_amd import _lib
    lib = _lib.lib()

    def create(mutate):
        b = sg.cube_light_scene(resolution=32, view=32)
        mutate(b)
        bd = dsm._BatchDesc(b)
        h = C.c_void_p()
        return lib.dsm_plan_create(C.byref(bd.desc), 0, 0, C.byref(h))

    def five(b):
        b.lights.pop()
        b.renders[0].lights = list(range(5))
    assert create(five) == 1                                                       # five faces
    assert create(lambda b: setattr(b.lights[3], 'resolution', 64)) == 1          # mixed sizes
    assert create(lambda b: setattr(b.lights[4], 'k', 3)) == 1                     # mixed filters
    assert create(lambda b: b.lights.__setitem__(slice(0, 2), b.lights[1::-1])) == 1   # out of order
