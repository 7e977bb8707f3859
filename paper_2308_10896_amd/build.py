"""Build the HIP library in-tree with hipcc for gfx950.

Usage: python -m paper_2308_10896_amd.build  (or call build()).
The shared library lands next to this file as libdsm.so.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
INCLUDE = os.path.join(ROOT, 'include')
LIB = os.path.join(HERE, 'libdsm.so')

# -ffp-contract=off: no fused multiply-add anywhere, so the float32
#   transform / snapping / depth arithmetic that decides coverage is exactly
#   the stated operation order (integer outputs are compared bit for bit).
# -fhip-fp32-correctly-rounded-divide-sqrt: IEEE division for the same reason.
# -packed-fp32-ops off: no packed FP32 instructions.
FLAGS = [
    '-O3', '--offload-arch=gfx950', '-fPIC', '-shared', '-std=c++17',
    '-ffp-contract=off', '-fhip-fp32-correctly-rounded-divide-sqrt', '-munsafe-fp-atomics',
    '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
    '-Wno-unused-command-line-argument',
]


def hipcc():
    for c in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if c and os.path.exists(c):
            return c
    raise RuntimeError('hipcc not found')


def sources():
    return sorted(glob.glob(os.path.join(CSRC, '*.hip')))


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libdsm.so (always recompiles)."""
    srcs = sources()
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        procs = []
        for s in srcs:
            o = os.path.join(tmp, os.path.basename(s) + '.o')
            cmd = [hipcc()] + [f for f in FLAGS if f not in ('-shared',)] + ['-c', '-I', INCLUDE, '-I', CSRC, s, '-o', o]
            if verbose:
                print(' '.join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(o)
        for s, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors='replace')
            text = '\n'.join(l for l in text.splitlines() if 'packed-fp32-ops' not in l and l.strip())
            if p.returncode != 0:
                raise RuntimeError(f'hipcc failed on {s}:\n{text}')
            if verbose and text:
                print(text)
        tmp_lib = LIB + '.tmp'
        cmd = [hipcc(), '--offload-arch=gfx950', '-shared', '-fPIC', '-o', tmp_lib] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f'link failed:\n{r.stdout}\n{r.stderr}')
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == '__main__':
    print(build(verbose='-v' in sys.argv))
