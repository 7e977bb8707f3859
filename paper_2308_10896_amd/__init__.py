"""Differentiable pre-filtered shadow mapping for MI355X (gfx950).

The compute path is the HIP library ``libdsm.so`` (C ABI in include/dsm.h);
this package only marshals torch tensors into it.  See ``dsm`` for the
entry points.
"""
from .dsm import *  # noqa: F401,F403
