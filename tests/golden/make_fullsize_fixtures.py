"""Writes the oracle fixtures of the full-size parity tests of the multi-view
workload (one displaced 99k-triangle sphere, 8 point lights at 1024^2, 16
cameras at 512^2, 128 renders) and the complex scene (about 330k triangles,
3 point lights at 2048^2 summed in one 1920x1080 RGB render).

Only the oracle and the seeded scene generator run here (CPU, float64; about
three minutes and 7 GB for the complex scene).  The oracle renders the
sampled renders of each workload at full size and differentiates them for a
seeded float32 upstream gradient kept on the pixels whose lookup decisions
are clear of their thresholds.  The upstream gradient is split into the
share on pixels whose visibility rests on the variance floor and the rest,
and each share is differentiated on its own.  Stored (npz, no pickles): a
hash of the scene inputs, SHA-256 digests of the full depth|id key maps of
every view involved, sampled filtered-moment texels, sampled image pixels
with their variance-floor flags, the clear-pixel and floor masks (packed
bits), and per share the light gradients and samples of the vertex and
albedo gradients with each group's largest entry and norm.

    python tests/golden/make_fullsize_fixtures.py [multiview] [complex]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import scenegen as sg                                   # noqa: E402
from oracle import pipeline as P                        # noqa: E402
from parity_helpers import decisions_clear, floor_conditioned   # noqa: E402  (oracle outputs only)

N_TEXELS = 4096          # sampled filtered-moment texels per light
N_PIXELS = 8192          # sampled pixels per render
N_GRAD = 2048            # largest-gradient vertices / faces, plus as many seeded others


def scene_hash(batch) -> str:
    """Digest of everything the renderer reads from a batch description."""
    h = hashlib.sha256()
    for sc in batch.scenes:
        for a in (sc.verts, sc.faces, sc.albedo, sc.pose, sc.pose_center):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(str(sc.pose_count).encode())
    for x in list(batch.lights) + list(batch.cameras):
        for k, v in sorted(x.__dict__.items()):
            h.update(k.encode())
            h.update(np.ascontiguousarray(np.asarray(v)).tobytes())
    for r in batch.renders:
        h.update(repr((r.camera, list(r.lights))).encode())
    h.update(repr((batch.channels, batch.antialias_camera)).encode())
    return h.hexdigest()


def key_digest(keys: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(keys, dtype=np.uint64).tobytes()).hexdigest()


def upstream(batch, seed):
    """Seeded float32 upstream gradient, one [H, W, C] array per render."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((batch.cameras[r.camera].height, batch.cameras[r.camera].width, batch.channels))
            .astype(np.float32) for r in batch.renders]


def sub_batch(batch, renders):
    """The lights and cameras that the chosen renders use, and those renders."""
    lights = sorted({l for r in renders for l in batch.renders[r].lights})
    cams = sorted({batch.renders[r].camera for r in renders})
    rs = [sg.Render(cams.index(batch.renders[r].camera), [lights.index(l) for l in batch.renders[r].lights])
          for r in renders]
    return (sg.Batch(batch.name, batch.scenes, [batch.lights[l] for l in lights], [batch.cameras[c] for c in cams],
                     rs, channels=batch.channels, antialias_camera=batch.antialias_camera), lights, cams)


def make(name, batch, renders, seed):
    t0 = time.time()
    sub, lights, cams = sub_batch(batch, renders)
    base, poses, lp, alb = P.scene_leaves(sub, requires_grad=True)
    out = P.render(sub, P.world_vertices(sub, base, poses), lp, alb)
    res = dict(raw=out, flags=out['flags'])
    print(f'{name}: oracle forward {time.time() - t0:.1f} s', flush=True)
    rng = np.random.default_rng(seed + 1)
    rec = dict(scene_hash=np.array(scene_hash(batch)), renders=np.array(renders, np.int64),
               lights=np.array(lights, np.int64), cameras=np.array(cams, np.int64), seed=np.array(seed))
    # keys of every view involved: light views, then camera views
    for q, ls in enumerate(out['lights']):
        rec[f'key_light{q}'] = np.array(key_digest(ls['rv']['key']))
    for q, v in enumerate(out['views']):
        rec[f'key_render{q}'] = np.array(key_digest(v['rv']['key']))
    # filtered moments at sampled texels
    for q, ls in enumerate(out['lights']):
        M = ls['M'].detach().numpy()
        S = M.shape[-1]
        idx = np.sort(rng.choice(S * S, size=min(N_TEXELS, S * S), replace=False))
        rec[f'M{q}_idx'] = idx.astype(np.int64)
        rec[f'M{q}_val'] = M.reshape(2, -1)[:, idx].astype(np.float32)
    # images at sampled pixels, with their variance-floor flags; the upstream
    # gradient kept on clear pixels and split into the floor-conditioned
    # share and the rest
    G = upstream(sub, seed)
    keep_all, shares = [], {'rest': [], 'floor': []}
    for q, v in enumerate(out['views']):
        img = out['images'][q].detach().numpy()
        H, W, C = img.shape
        idx = np.sort(rng.choice(H * W, size=min(N_PIXELS, H * W), replace=False))
        cond = floor_conditioned(sub, res, q, dilate=1)
        rec[f'img{q}_idx'] = idx.astype(np.int64)
        rec[f'img{q}_val'] = img.reshape(H * W, C)[idx].astype(np.float32)
        rec[f'img{q}_floor'] = cond.ravel()[idx]
        keep = decisions_clear(sub, res, q)
        keep_all.append(keep)
        rec[f'keep{q}'] = np.packbits(keep.ravel())
        rec[f'floor{q}'] = np.packbits(cond.ravel())
        g = G[q].astype(np.float64) * keep[..., None]
        shares['rest'].append(g * ~cond[..., None])
        shares['floor'].append(g * cond[..., None])
    dropped = 1.0 - float(np.mean(np.concatenate([k.ravel() for k in keep_all])))
    rec['dropped'] = np.array(dropped)
    # gradients of each share
    leaves = list(base) + list(lp) + list(alb)
    res_g = {}
    for share, Gs in shares.items():
        total = sum((im * torch.as_tensor(g)).sum() for im, g in zip(out['images'], Gs))
        grads = torch.autograd.grad(total, leaves, allow_unused=True, retain_graph=True)
        res_g[share] = dict(
            gverts=np.concatenate([g.numpy() if g is not None else np.zeros(b.shape)
                                   for g, b in zip(grads[:len(base)], base)]),
            glight=np.stack([g.numpy() for g in grads[len(base):len(base) + len(lp)]]),
            galbedo=np.concatenate([g.numpy() for g in grads[len(base) + len(lp):]]))
    for key in ('gverts', 'galbedo'):
        # rows with the largest entries (of both shares) and as many seeded
        # others; each share's largest entry and norm are kept for the checks
        mag = np.maximum(np.abs(res_g['rest'][key]).max(1), np.abs(res_g['floor'][key]).max(1))
        top = np.argsort(-mag)[:N_GRAD]
        rest = np.setdiff1d(np.arange(len(mag)), top)
        other = rng.choice(rest, size=min(N_GRAD, len(rest)), replace=False)
        idx = np.sort(np.concatenate([top, other]))
        rec[f'{key}_idx'] = idx.astype(np.int64)
        for share in shares:
            g = res_g[share][key]
            rec.update({f'{key}_{share}_val': g[idx].astype(np.float32),
                        f'{key}_{share}_absmax': np.array(np.abs(g).max()),
                        f'{key}_{share}_norm': np.array(np.linalg.norm(g))})
    for share in shares:
        rec[f'glight_{share}'] = res_g[share]['glight']
    path = os.path.join(HERE, f'fullsize_{name}.npz')
    np.savez_compressed(path, **rec)
    print(f'{name}: wrote {path} ({os.path.getsize(path) / 1e3:.0f} kB), {100 * dropped:.3f} % of the pixels '
          f'ambiguous, {time.time() - t0:.1f} s', flush=True)


def main(which):
    torch.set_num_threads(os.cpu_count() or 1)
    if 'multiview' in which:
        b = sg.config3()
        # camera 0 with light 0, and a seeded (camera, light) pair
        r2 = int(np.random.default_rng(30).integers(1, len(b.renders)))
        make('multiview', b, [0, r2], seed=31)
    if 'complex' in which:
        make('complex', sg.config4(), [0], seed=41)


if __name__ == '__main__':
    main(sys.argv[1:] or ['multiview', 'complex'])
