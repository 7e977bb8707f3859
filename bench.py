#!/usr/bin/env python3
"""Throughput of differentiable pre-filtered shadow mapping on one MI355X.

Workload (default): the batched pose-estimation batch -- 64 procedural blob
scenes (2k..20k triangles each, seeded) over a ground plane, one directional
light and one 512x512 camera per scene, 512x512 shadow maps with a 5x5 box
moment filter.  One step = for every scene: rigid pose -> light-view raster,
moment resolve, edge smoothing, moment filter -> camera raster, Chebyshev
visibility + Lambert shading, edge smoothing -> and the full backward pass to
pose, light and albedo gradients.  All 64 renders of a step run as one
captured HIP graph (batched path); the plain path runs the same scenes one
plan and one forward/backward call at a time, eagerly.

Prints one JSON line (rank 0).  Inputs are resident in HBM before timing.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shadowed fwd+bwd renders/sec at 512² (batched vs plain, 1 MI355X); % HBM roofline"
HBM_PEAK_GBS = 8000.0

# Counter records per launch of the targeted kernels on this workload, from
# rocprofv3 --pmc passes of this script, one counter group per run
# (profiles/cfg2_counters_pmc.md gives the commands and the tables):
#
# * fetch_kib / write_kib: FETCH_SIZE and WRITE_SIZE (KiB per dispatch).
#   Each is scaled by what it reads for a plain 128 MiB device-to-device copy
#   in the same runs (PMC_COPY): FETCH_SIZE counts a 128-byte read request
#   as 64 bytes, so the copy reads back half its size;
# * rd_bytes / wr_bytes: the same traffic from the per-request-size counters
#   (32 TCC_EA0_RDREQ_32B + 64 TCC_EA0_RDREQ_64B + 128 TCC_EA0_RDREQ_128B;
#   32 (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B) + 64 TCC_EA0_WRREQ_64B), exact
#   for the copy (factor 1.00) and for gathers that mix request sizes;
# * waves, valu_per_wave (SQ_INSTS_VALU / SQ_WAVES), valu_busy
#   (4 SQ_ACTIVE_INST_VALU over the 1024 SIMDs' cycles: a wave64 VALU
#   instruction occupies a 16-lane SIMD for 4 cycles) and occupancy
#   (waves resident per CU, 4 SQ_WAVE_CYCLES / GRBM_GUI_ACTIVE per XCD).
#
# A record is used only while the kernel's sources hash to the value they
# had when the counters were taken (and at tile side 8, where they were).
PMC_COPY = dict(fetch_kib=65547.6, write_kib=131072.0, moved_kib=131072.0)
PMC = {
    'filter': dict(kernel='blur_kernel<false, 2, true>', fetch_kib=65751.8, write_kib=131072.0, rd_bytes=134574259, wr_bytes=134217728, waves=32768, valu_per_wave=716.2, valu_busy=0.585, occupancy=19.8, sources=('blur.hip', 'dsm_internal.h'), sha1='e7468a0f4ddb340f'),
    'filter_adj': dict(kernel='blur_kernel<true, 2, true>', fetch_kib=65621.9, write_kib=131072.0, rd_bytes=134309030, wr_bytes=134217728, waves=32768, valu_per_wave=943.1, valu_busy=0.801, occupancy=20.1, sources=('blur.hip', 'dsm_internal.h'), sha1='e7468a0f4ddb340f'),
    'lookup': dict(kernel='lookup_kernel<2>', fetch_kib=200689.8, write_kib=65536.0, rd_bytes=410704768, wr_bytes=67108864, waves=131072, valu_per_wave=466.0, valu_busy=0.952, occupancy=26.3, sources=('shade.hip', 'dsm_internal.h'), sha1='24a515cac17e6ff0'),
    'lookup_adj': dict(kernel='lookup_backward_kernel_1l<8>', fetch_kib=117285.1, write_kib=120145.4, rd_bytes=239955072, wr_bytes=123028288, waves=262144, valu_per_wave=854.4, valu_busy=0.763, occupancy=14.8, sources=('grad.hip', 'dsm_internal.h'), sha1='8b4f6eb42447484f'),
}

# Issue peak of the vector ALUs: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per
# wave64 instruction.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def pmc_record(stage, tile):
    """The counter record of a stage's kernel, or None when there is none for
    the current kernel sources (and tile side 8)."""
    import hashlib
    rec = PMC.get(stage)
    if rec is None or tile != 8:
        return None
    m = hashlib.sha1()
    for f in rec['sources']:
        with open(os.path.join(ROOT, 'paper_2308_10896_amd', 'csrc', f), 'rb') as fh:
            m.update(fh.read())
    if m.hexdigest()[:16] != rec['sha1']:
        return None
    return rec


def pmc_traffic(rec):
    """HBM bytes per launch: FETCH_SIZE / WRITE_SIZE scaled by the copy."""
    fs = PMC_COPY['moved_kib'] / PMC_COPY['fetch_kib']
    ws = PMC_COPY['moved_kib'] / PMC_COPY['write_kib']
    return 1024.0 * (rec['fetch_kib'] * fs + rec['write_kib'] * ws)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=5)
    ap.add_argument('--scenes', type=int, default=64)
    ap.add_argument('--res', type=int, default=512)
    ap.add_argument('--no-plain', action='store_true')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-seconds', type=float, default=24.0,
                    help='time budget of the oracle baseline (three passes over one sample)')
    ap.add_argument('--stage-reps', type=int, default=10)
    ap.add_argument('--tile', type=int, default=0, help='raster tile side; 0: autotune')
    ap.add_argument('--no-other', action='store_true', help='skip the other configurations')
    ap.add_argument('--no-cold', action='store_true', help='skip the cold-cache stage timing')
    return ap.parse_args()


def progress(msg):
    """One line per finished phase on stderr (the JSON result stays alone on stdout)."""
    print(f'[bench] {msg}', file=sys.stderr, flush=True)


def timed(fn, steps, stream, per_step=None):
    """Seconds for `steps` calls of fn, bracketed by synchronizations and HIP
    events on `stream`; with a list `per_step`, each step's milliseconds
    (events recorded between the steps) are appended to it."""
    import torch
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1 if per_step is not None else 2)]
    ev[0].record(stream)
    for i in range(steps):
        fn()
        if per_step is not None:
            ev[i + 1].record(stream)
    ev[-1].record(stream)
    torch.cuda.synchronize()
    if per_step is not None:
        per_step.extend(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    return ev[0].elapsed_time(ev[-1]) / 1000.0


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({'error': 'this build measures one GPU only; run with --gpus 1',
                          'n_gpus_requested': args.gpus}))
        sys.exit(2)
    import torch
    import scenegen as sg
    from paper_2308_10896_amd import dsm

    dev = torch.device('cuda:0')
    batch = sg.config2(n_scenes=args.scenes, resolution=args.res, with_pose=True)
    tris = [len(s.faces) for s in batch.scenes]
    stream = torch.cuda.Stream()

    # ---------------- tile side and bin depth: given, or chosen by the autotuner
    local, lp, alb, poses = dsm.batch_inputs(batch, dev)
    plan = dsm.Plan(batch)
    rng = np.random.default_rng(0)
    gimg = torch.as_tensor(rng.standard_normal(int(plan.info.image_floats)).astype(np.float32) * 1e-3, device=dev)
    tune = None
    if args.tile == 0:
        with torch.cuda.stream(stream):
            posed = plan.pose_forward(local, poses)
            tile, scale, tune_ms = dsm.autotune(batch, posed, lp, alb, gimg, reps=3, stream=stream)
        tune = {'tile': tile, 'bin_capacity_scale': scale, 'ms_fwd_bwd': round(tune_ms, 4)}
        progress(f'autotuned: tile {tile}, bin scale {scale}')
    else:
        tile, scale = args.tile, 0
    del plan
    # ---------------- batched: one plan, one graph of pose+fwd+bwd+pose^T
    plan = dsm.Plan(batch, tile_size=tile, bin_capacity_scale=scale)
    saved, scratch = plan.workspace(dev)
    verts = torch.empty_like(local)
    images = torch.empty(int(plan.info.image_floats), device=dev)
    gverts = torch.empty_like(local)
    glp = torch.empty_like(lp)
    galb = torch.empty_like(alb)
    gposes = torch.empty_like(poses)
    torch.cuda.synchronize()
    plan.graph_capture(stream, local, poses, verts, lp, alb, saved, scratch, images, gimg, gverts, glp, galb, gposes)
    torch.cuda.synchronize()

    def step_batched():
        plan.graph_launch(stream)

    for _ in range(args.warmup):
        step_batched()
    torch.cuda.synchronize()
    step_ms = []
    t_batched = timed(step_batched, args.steps, stream, step_ms)
    R = len(batch.renders)
    batched_rps = R * args.steps / t_batched
    progress(f'batched: {batched_rps:.1f} renders/s')
    st = plan.stats(saved)
    assert st['culled'] == 0 and st['bad_indices'] == 0, st

    # ---------------- dominant kernels, timed live with HIP events on the plan's stream
    kern = kernel_timings(plan, batch, stream, verts, lp, alb, saved, scratch, images, gimg, gverts, glp, galb,
                          args)
    progress('stage timings done')

    # ---------------- plain: one plan per scene, eager calls, no graph
    plain_rps = None
    if not args.no_plain:
        subs = []
        for i in range(args.scenes):
            b1 = sg.Batch(batch.name, [batch.scenes[i]],
                          [sg.Light(**{**batch.lights[i].__dict__, 'scene': 0})],
                          [sg.Camera(**{**batch.cameras[i].__dict__, 'scene': 0})],
                          [sg.Render(0, [0])], channels=1)
            p1 = dsm.Plan(b1, tile_size=tile, bin_capacity_scale=scale)
            l1, lp1, a1, po1 = dsm.batch_inputs(b1, dev)
            s1, sc1 = p1.workspace(dev)
            g1 = torch.as_tensor(rng.standard_normal(int(p1.info.image_floats)).astype(np.float32) * 1e-3, device=dev)
            subs.append((p1, l1, lp1, a1, po1, s1, sc1, g1))

        def step_plain():
            with torch.cuda.stream(stream):
                for (p1, l1, lp1, a1, po1, s1, sc1, g1) in subs:
                    v1 = p1.pose_forward(l1, po1)
                    p1.forward(v1, lp1, a1, s1, sc1)
                    gv1, _, _ = p1.backward(v1, lp1, a1, s1, sc1, g1)
                    p1.pose_backward(l1, po1, gv1)

        for _ in range(max(1, args.warmup // 2)):
            step_plain()
        torch.cuda.synchronize()
        psteps = max(2, args.steps // 4)
        t_plain = timed(step_plain, psteps, stream)
        plain_rps = R * psteps / t_plain
        progress(f'plain: {plain_rps:.1f} renders/s')

    # ---------------- the other configurations of the method, absolute rates
    other = None
    if not args.no_other:
        other = other_configs(stream)
        progress('other configurations done')

    # ---------------- CPU baseline: the oracle on a bounded sample of scenes
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch, args.cpu_seconds)
        progress(f"oracle baseline: {cpu['value']} renders/s")

    out = {
        'metric': METRIC,
        'value': round(batched_rps, 2),
        'unit': 'renders/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': round(1000 * t_batched / args.steps, 4),
        'ms_per_step_p10_p50_p90': [round(float(np.percentile(step_ms, q)), 4) for q in (10, 50, 90)],
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f32',
        'data': 'synthetic',
        'config': {
            'workload': f'batched pose estimation: {args.scenes} blob scenes x 1 directional light, '
                        f'{args.res}^2 shadow maps (5x5 box) and {args.res}^2 views, fwd+bwd to pose',
            'scenes': args.scenes, 'renders_per_step': R, 'shadow_map': args.res, 'view': args.res,
            'triangles_total': int(sum(tris)), 'triangles_min': int(min(tris)), 'triangles_max': int(max(tris)),
            'path': 'batched: one plan, one HIP graph per step',
            'plain_renders_per_s': None if plain_rps is None else round(plain_rps, 2),
            'batched_over_plain': None if plain_rps is None else round(batched_rps / plain_rps, 3),
            'tile': int(plan.info.tile_size),
            'bin_capacity_scale': int(plan.info.bin_capacity_scale),
            'autotune': tune,
            'stages_us': kern['stages_us'],
            'stages_us_cold': kern['stages_us_cold'],
            'other_configs': other,
        },
        'roofline': kern['roofline'],
        'cpu_baseline': cpu,
    }
    print(json.dumps(out), flush=True)


def kernel_timings(plan, batch, stream, verts, lp, alb, saved, scratch, images, gimg, gverts, glp, galb, args):
    """Durations of the pipeline's kernels, measured live with HIP events on
    `stream` (the stream the kernels are launched on):

    * every stage of forward + backward, eager, via the library's stage
      timer (each targeted stage is one kernel launch);
    * the moment filter forward / transpose again as back-to-back launches
      of the stand-alone filter (the same kernel with both sides
      channel-planar; in the pipeline the filtered side is interleaved) on
      the batch's own smoothed maps;
    * a plain device-to-device copy of the same size, for the achievable
      bandwidth on this GPU.

    Algorithmic bytes per launch follow the per-unit figures: filter 16 S^2
    per map (2 channels read + written, f32); lookup P (4 + 4C) + 8 S^2 per
    light + 12 (F + V) + 4 C F per render; lookup^T P (4 + 4C) + 16 S^2 per
    light + 12 (F + V) + 12 V per render.
    """
    import torch
    from paper_2308_10896_amd import dsm
    stages = plan.time_stages(stream, verts, lp, alb, saved, scratch, images, gimg, gverts, glp, galb,
                              args.stage_reps)
    # the same with the caches (the 256 MB MALL included) evicted before every stage
    stages_cold = None
    if not args.no_cold:
        flush = torch.empty(1 << 28, dtype=torch.float32, device=verts.device)
        stages_cold = plan.time_stages(stream, verts, lp, alb, saved, scratch, images, gimg, gverts, glp, galb,
                                       args.stage_reps, flush=flush)
        del flush
    n, S = len(plan.light_res), plan.light_res[0]
    P = args.res * args.res
    C = 1
    F = np.array([len(sc.faces) for sc in batch.scenes], dtype=np.float64)
    V = np.array([len(sc.verts) for sc in batch.scenes], dtype=np.float64)
    R = len(batch.renders)
    algo = {
        'filter': 16.0 * n * S * S,
        'filter_adj': 16.0 * n * S * S,
        'lookup': float(R * P * (4 + 4 * C) + R * 8.0 * S * S + 12.0 * (F + V).sum() + 4.0 * C * F.sum()),
        'lookup_adj': float(R * P * (4 + 4 * C) + R * 16.0 * S * S + 12.0 * (F + V).sum() + 12.0 * V.sum()),
    }
    kernels = {}
    tile = int(plan.info.tile_size)
    for name, b in algo.items():
        us = 1000.0 * stages[name]
        rec = pmc_record(name, tile)
        tr = None if rec is None else pmc_traffic(rec)
        tx = None if rec is None else rec['rd_bytes'] + rec['wr_bytes']
        kernels[name] = dict(us=round(us, 2), bytes=b, gbs=round(b / (us * 1e-6) / 1e9, 1),
                             frac=round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))
        if stages_cold is not None:
            us_cold = 1000.0 * stages_cold[name]
            kernels[name].update(us_cold=round(us_cold, 2), gbs_cold=round(b / (us_cold * 1e-6) / 1e9, 1),
                                 frac_cold=round(b / (us_cold * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))
        kernels[name].update(traffic=None if tr is None else round(tr),
                             traffic_gbs=None if tr is None else round(tr / (us * 1e-6) / 1e9, 1),
                             traffic_by_request_size=None if tx is None else round(tx),
                             gbs_counter_bytes=None if tx is None else round(tx / (us * 1e-6) / 1e9, 1))
        if rec is not None:
            # counter-measured vector-ALU issue: instructions per launch at
            # the issue peak, against this launch's time
            insts = rec['valu_per_wave'] * rec['waves']
            kernels[name]['valu'] = {
                'insts_per_wave': rec['valu_per_wave'], 'waves': rec['waves'],
                'issue_bound_us': round(insts / VALU_ISSUE_PEAK * 1e6, 1),
                'issue_frac': round(insts / VALU_ISSUE_PEAK / (us * 1e-6), 3),
                'busy': rec['valu_busy'], 'waves_per_cu': rec['occupancy']}
    reps = 20
    with torch.cuda.stream(stream):
        maps = torch.stack([plan.light_maps(saved, scratch, l, 1) for l in range(n)]).contiguous()
        for name, adj in (('filter', False), ('filter_adj', True)):
            for _ in range(3):
                dsm.filter_moments(maps, 'box', 5, 0.0, adj)
            t = timed(lambda: dsm.filter_moments(maps, 'box', 5, 0.0, adj), reps, stream)
            us = 1e6 * t / reps
            kernels[name]['us_back_to_back'] = round(us, 2)
            kernels[name]['gbs_back_to_back'] = round(algo[name] / (us * 1e-6) / 1e9, 1)
        dst = torch.empty_like(maps)
        for _ in range(3):
            dst.copy_(maps)
        t = timed(lambda: dst.copy_(maps), reps, stream)
        copy_gbs = 2.0 * maps.numel() * 4 / (t / reps) / 1e9
    dom = max(kernels, key=lambda k: kernels[k]['us'])
    d = kernels[dom]
    # achieved / frac: algorithmic bytes per launch over the launch time;
    # achieved_counter_bytes: the bytes the counters saw over the same time
    roof = {'kernel': dom, 'bound': 'hbm', 'achieved': d['gbs'], 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
            'frac': d['frac'], 'traffic': d['traffic'],
            'traffic_by_request_size': d['traffic_by_request_size'],
            'achieved_counter_bytes': d['gbs_counter_bytes'], 'valu': d.get('valu'),
            'kernels': kernels,
            'copy_gbs': round(copy_gbs, 1)}
    return {'stages_us': {k: round(1000.0 * v, 2) for k, v in stages.items()},
            'stages_us_cold': None if stages_cold is None else {k: round(1000.0 * v, 2) for k, v in stages_cold.items()},
            'roofline': roof}


def other_configs(stream, steps=10, warmup=3):
    """Forward + backward renders/s of the other workloads (one captured
    graph per step, inputs resident, default tile side 8): the tiny cube
    scene, the icosphere under a spot light, the 128-render multi-view
    sphere, the 330k-triangle complex scene and an omnidirectional point
    light (six 512^2 cube faces) over a ground with four occluders."""
    import torch
    import scenegen as sg
    from paper_2308_10896_amd import dsm
    res = {}
    for name, make in (('tiny cube, 256^2', sg.config0), ('icosphere, spot, 512^2', sg.config1),
                       ('multi-view sphere, 8 lights x 16 cameras, 1024^2 maps', sg.config3),
                       ('complex scene, 330k triangles, 3 lights at 2048^2, 1920x1080', sg.config4),
                       ('omnidirectional light, 6 cube faces at 512^2, 512^2 view',
                        lambda: sg.cube_light_scene(resolution=512, view=512))):
        batch = make()
        dev = torch.device('cuda:0')
        plan = dsm.Plan(batch)
        local, lp, alb, poses = dsm.batch_inputs(batch, dev)
        saved, scratch = plan.workspace(dev)
        verts = torch.empty_like(local)
        images = torch.empty(int(plan.info.image_floats), device=dev)
        gimg = torch.full((int(plan.info.image_floats),), 1e-3, device=dev)
        gv, gl, ga, gp = (torch.empty_like(local), torch.empty_like(lp), torch.empty_like(alb),
                          torch.empty_like(poses))
        torch.cuda.synchronize()
        plan.graph_capture(stream, local, poses, verts, lp, alb, saved, scratch, images, gimg, gv, gl, ga, gp)
        for _ in range(warmup):
            plan.graph_launch(stream)
        t = timed(lambda: plan.graph_launch(stream), steps, stream)
        R = len(batch.renders)
        progress(f'{name}: {R * steps / t:.1f} renders/s')
        res[name] = {'renders_per_s': round(R * steps / t, 2), 'ms_per_step': round(1000 * t / steps, 4),
                     'renders_per_step': R, 'triangles': int(sum(len(sc.faces) for sc in batch.scenes))}
        del plan, saved, scratch
        torch.cuda.synchronize()
    return res


def host_cpu():
    """Model name and logical-CPU counts of this host."""
    model = None
    try:
        with open('/proc/cpuinfo') as f:
            for line in f:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    return {'model': model, 'nproc': os.cpu_count(), 'affinity': len(os.sched_getaffinity(0))}


def _oracle_fwd_bwd(b1):
    from oracle import pipeline as P
    base, poses, lp, alb = P.scene_leaves(b1)
    out = P.render(b1, P.world_vertices(b1, base, poses), lp, alb)
    loss = sum((im ** 2).sum() for im in out['images'])
    loss.backward()


def cpu_baseline(batch, budget_s):
    """The oracle (float64, plain numpy/torch) timed on this host's cores:
    fwd+bwd of the batch's scenes, smallest first and then in a seeded
    order, until about a third of `budget_s` has passed; that sample is then
    timed twice more and the median of the three passes is reported.  The
    tiny-cube and icosphere workloads are timed beside it (median of 3).
    Torch keeps the thread count the environment gives it (OMP_NUM_THREADS,
    the host threads allotted to one GPU)."""
    import torch
    import scenegen as sg
    threads = torch.get_num_threads()
    tris = np.array([len(s.faces) for s in batch.scenes])
    first = int(np.argmin(tris))
    rest = [int(i) for i in np.random.default_rng(1).permutation(len(tris)) if int(i) != first]

    def single(i):
        return sg.Batch(batch.name, [batch.scenes[i]], [sg.Light(**{**batch.lights[i].__dict__, 'scene': 0})],
                        [sg.Camera(**{**batch.cameras[i].__dict__, 'scene': 0})], [sg.Render(0, [0])], channels=1,
                        target_poses=[np.zeros(6, np.float32)])

    done, t0 = [], time.time()
    for i in [first] + rest:
        _oracle_fwd_bwd(single(i))
        done.append(i)
        if time.time() - t0 >= budget_s / 3.0:
            break
    passes = [time.time() - t0]
    for _ in range(2):
        t0 = time.time()
        for i in done:
            _oracle_fwd_bwd(single(i))
        passes.append(time.time() - t0)
    dt = float(np.median(passes))
    other = {}
    for name, make in (('tiny cube, 256^2', sg.config0), ('icosphere, spot, 512^2', sg.config1)):
        b1 = make()
        ts = []
        for _ in range(3):
            t0 = time.time()
            _oracle_fwd_bwd(b1)
            ts.append(time.time() - t0)
        other[name] = {'renders_per_s': round(1.0 / float(np.median(ts)), 4), 'seconds': [round(t, 3) for t in ts]}
    return {'value': round(len(done) / dt, 4), 'unit': 'renders/s', 'cores': int(threads),
            'kind': 'oracle', 'host': host_cpu(),
            'sample': f'{len(done)} of the {len(batch.scenes)} scenes (smallest first, then seeded order; '
                      f'{int(tris[done].sum())} triangles in all), fwd+bwd each in float64; median of 3 passes '
                      f'({", ".join(f"{t:.1f}" for t in passes)} s)',
            'other_configs': other}


if __name__ == '__main__':
    main()
