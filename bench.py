#!/usr/bin/env python3
"""Throughput of the differentiable DVR hot path on one MI355X.

Workload (absorption-only tomography, Sec. 5.3 shapes): a 256^3 grid stored as
bf16 (float32 master), 64 views on a Fibonacci sphere at 512x512, step 0.2
voxel, loss L2 against target images rendered once from a seeded
ground-truth grid of ellipsoids.  One step = one reconstruction iteration:
refresh the bf16 storage copy of the master grid, one fused forward -> L2
gradient -> adjoint pass over all 64 views in a single launch (replayed from a
HIP graph), and a projected gradient-descent update of the master.  Timing
starts after a few untimed iterations from the zero grid (burn-in): at zero
density every ray whose target pixel is empty has an exactly zero residual and
its adjoint is skipped, which only the very first iterations see.

Printed (one JSON line): fwd+adjoint ray-samples/s, the roofline of the fused
kernel (algorithmic bytes per launch / its event-timed duration), the FP64
oracle timed on the host on a bounded pixel sample, and the speedup over the
plain per-view float32 path (one launch per view, direct global gathers and
atomics).
"""
from __future__ import annotations

import argparse

import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Published VALU figure: MI355X's fp32 vector rate, 157.3 TFLOP/s = 256 CUs x
# 128 lanes x 2 flops (FMA) x 2.4 GHz, i.e. two wave64 instructions per CU and
# clock.  Chains of one instruction class (FMA, integer add) issue half that,
# 256 x 64 x 2.4 GHz = 39.3 T lane-instructions/s; some pairs of classes
# (a multiply and a max) dual-issue up to the full rate.
VALU_PUBLISHED_TOPS = 256 * 128 * 2.4e9 / 1e12
VALU_NONPACKED_TOPS = 256 * 64 * 2.4e9 / 1e12
# The ALU roof the benchmark prices against: the issue rate measured on the
# device with the library's own flags (bench.py --calibrate-valu, summary in
# profiles/): the dual-issue figure, with the single-issue one beside it
VALU_CEILING_FILE = os.path.join(ROOT, "profiles", "valu_ceiling.json")
ALG_BYTES_BF16 = 64      # per sample pair: 8 gathers x 2 B (fwd) + 8 x 2 B (adj) + 8 x 4 B scatter
ALG_BYTES_F32 = 96
KERNEL_SOURCES = ["paper_2107_12672_amd/csrc/ddvr_kernels.hip",
                  "paper_2107_12672_amd/csrc/ddvr_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c3_fused.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(sources=None) -> str:
    """Hash of the kernels' code, comments ignored: the key of committed
    counters (they go stale with any change to the code)."""
    from paper_2107_12672_amd import isa_count
    return isa_count.source_hash(sources or KERNEL_SOURCES)


def measured_traffic():
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def valu_ceiling(key="issue_tops"):
    """Committed measurement of the VALU issue ceiling (T lane-instructions/s):
    `issue_tops` the dual-issue figure (the roof), `single_issue_tops` that of
    FMA / integer chains; None if absent."""
    try:
        with open(VALU_CEILING_FILE) as f:
            t = json.load(f)
        return float(t[key])
    except (OSError, ValueError, KeyError, TypeError):
        return None


def valu_probe(mode, blocks, iters, reps=3):
    """Event-timed VALU probe launches: (T lane-ops/s, ms per launch)."""
    import torch
    from paper_2107_12672_amd import ddvr as d
    out = torch.empty(blocks * 256, device="cuda")
    stream = torch.cuda.current_stream()
    ops = d.valu_probe(mode, blocks, iters, out)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        d.valu_probe(mode, blocks, iters, out)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return ops / (ms * 1e-3) / 1e12, ms


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(work, n_views_max, budget_s=12.0, one_core_s=6.0):
    """FP64 oracle (forward + stored-tape adjoint) on every 8th row and column
    of successive views until the time budget is spent, on all the host's
    threads; then the same on one thread for a shorter budget."""
    import oracle
    oracle.build(force=False)
    res = _cpu_baseline_run(work, n_views_max, budget_s)
    nt = oracle.num_threads()
    oracle.set_threads(1)
    try:
        one = _cpu_baseline_run(work, n_views_max, one_core_s)
    finally:
        oracle.set_threads(nt)
    res["one_core"] = {"value": one["value"], "sample": one["sample"]}
    res["cpu_model"] = cpu_model()
    return res


def _cpu_baseline_run(work, n_views_max, budget_s):
    import numpy as np
    import oracle
    import synth
    V = np.zeros(work.volume.shape, np.float64)
    W = H = work.views[0].width
    pix = np.array([y * W + x for y in range(0, H, 8) for x in range(0, W, 8)], np.int32)
    rng = synth.rng_for(3, 7)
    samples = 0
    views = 0
    t0 = time.perf_counter()
    for v in work.views[:n_views_max]:
        cam = oracle.camera_from_sphere(v.yaw, v.pitch, v.dist, v.fovy, W, H)
        out = oracle.render(V, None, cam, W, H, work.step_world, oracle.AO, pix=pix)
        tgt = rng.uniform(0.0, 1.0, size=out["image"].shape)
        g = 2.0 * (out["image"] - tgt) / (len(work.views) * W * H)
        oracle.adjoint(V, None, cam, W, H, work.step_world, oracle.AO, g, pix=pix)
        samples += int(out["nsamp"].sum())
        views += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": samples / dt, "unit": "ray-samples/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"fp64 forward + stored-tape adjoint, every 8th row and column "
                      f"({len(pix)} rays/view) of {views} of the {len(work.views)} views, "
                      f"{samples} samples in {dt:.1f} s"}


def cpu_baseline_color(work, volume_np, budget_s=10.0):
    """FP64 oracle forward + stored-tape adjoint of the colour volume on every
    16th row and column of successive views until the budget is spent."""
    import numpy as np
    import oracle
    import synth
    oracle.build(force=False)
    V = np.asarray(volume_np, np.float64)
    W = H = work.views[0].width
    pix = np.array([y * W + x for y in range(0, H, 16) for x in range(0, W, 16)], np.int32)
    rng = synth.rng_for(9, 8)
    samples = views = 0
    t0 = time.perf_counter()
    for v in work.views:
        cam = oracle.camera_from_sphere(v.yaw, v.pitch, v.dist, v.fovy, W, H)
        out = oracle.render(V, None, cam, W, H, work.step_world, oracle.COLOR, pix=pix)
        g = 2.0 * (out["image"] - rng.uniform(0.0, 1.0, out["image"].shape)) / out["image"].size
        oracle.adjoint(V, None, cam, W, H, work.step_world, oracle.COLOR, g, pix=pix)
        samples += int(out["nsamp"].sum())
        views += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": samples / dt, "unit": "ray-samples/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"fp64 colour-volume forward + stored-tape adjoint, every 16th row and "
                      f"column ({len(pix)} rays/view) of {views} views, {samples} samples in "
                      f"{dt:.1f} s"}


def cpu_baseline_dfc(CV, tf, prev, alpha, ncand, budget_s=10.0):
    """FP64 oracle sweep on growing samples of random voxels until the budget
    is spent."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    nvox = int(np.prod(CV.shape[:3]))
    rng = np.random.default_rng(5)
    done = 0
    t0 = time.perf_counter()
    k = 4096
    while time.perf_counter() - t0 < budget_s and done < nvox:
        sel = rng.choice(nvox, size=min(k, nvox), replace=False)
        oracle.density_from_color(CV, tf, prev, alpha=alpha, beta=1.0, seed=7, iteration=1,
                                  ncand=ncand, voxels=sel)
        done += len(sel)
        k *= 2
    dt = time.perf_counter() - t0
    return {"value": done * ncand / dt, "unit": "candidates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"fp64 sweep of {done} random voxels x {ncand} candidates in {dt:.1f} s"}


def _arch(torch):
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def _timed(fn, steps, warmup, stream, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def secondary(args):
    """The other workloads, one JSON line each (not the headline figure):
      c1  absorption-only 32^3 f32, one 64x64 view, step 0.5 voxel, fused L2
          (launch-bound: timed as a single-view call and as a graph replay);
      c2  emission-absorption 128^3 f32, R=16, one 256x256 view, fused L2 with
          gradients for density, TF, camera and step;
      c4  uneven batch of 16 grids (edges 64-384, f16/f32, R 8-64, images
          128-1024 px) in one persistent launch, forward, minus the opacity
          entropy of each image as the loss, adjoint for camera and step
          gradients;
      c5  emission-absorption 512^3 f16 sparse noise, R=32, 32 views at
          1024x1024, fused L2 with density, TF and step gradients: T-form
          inversion (AUTO) and segment checkpointing (CHECKPOINT);
      viewpoint  the C5 grid and views, gradient w.r.t. (yaw, pitch, dist) of
          every view by forward-mode (delayed / immediate) and by the adjoint;
      color  pre-shaded colour volume 256^3 x (r, g, b, tau) bf16, the C3 views
          (64 at 512x512, step 0.2 voxel), fused L2 with the colour-volume
          gradient: one batched launch per step (and, for comparison, one launch
          per view);
      dfc  density from colour on that volume: R=32 TF, 256 candidates per
          voxel, one Jacobi sweep with the 6-neighbour term per step;
      recon  the whole multi-resolution reconstruction of Sec. 5.3 on the C3
          views of the C3 ground truth: 32^3 -> 256^3, 10 steps per level and
          50 at 256^3, batches of 8 views, fused L1 + 3D prior + Adam."""
    import numpy as np
    import torch
    import synth
    from paper_2107_12672_amd import ddvr as d
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def cams_of(views):
        return [d.camera_from_sphere(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                     math.radians(v.fovy), v.width, v.height) for v in views]

    def stored(vol_np, storage):
        v32 = torch.from_numpy(np.ascontiguousarray(vol_np)).to(dev)
        if storage == "f32":
            return v32
        out = torch.empty_like(v32, dtype=torch.float16 if storage == "f16" else torch.bfloat16)
        d.cast_volume(v32, out)
        return out

    out = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "unit": "ray-samples/s"}
    from paper_2107_12672_amd import autotune
    old_tuning = d.get_tuning()
    if args.workload in ("c1", "c2"):
        key = (autotune.c1_key if args.workload == "c1" else autotune.c2_key)(_arch(torch))
        out["tuning_source"] = "autotuned" if autotune.apply(key) else "default"
    if args.workload == "c1":
        # one small view: the launch and its synchronisation dominate
        w = synth.make_c1()
        v = w.views[0]
        vol = stored(w.volume, "f32")
        cam = cams_of([v])[0]
        # target: the render of the second blob grid (the workload's recipe)
        tgt = torch.from_numpy(np.ascontiguousarray(w.target_volume)).to(dev)
        targets = torch.empty((v.height, v.width), device=dev)
        d.render_forward(tgt, None, cam, w.step_world, d.ABSORPTION, targets)
        image = torch.empty_like(targets)
        dV = torch.zeros(w.volume.shape, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        g = d.grads_desc(dV)
        scale = 1.0 / image.numel()
        b = d.Batch([vol], None, [d.make_view(0, cam, w.step_world, image, target=targets)],
                    d.ABSORPTION, d_volumes=[dV])
        S = b.sample_count()
        ms_single = _timed(lambda: d.render_fused_l2(vol, None, cam, w.step_world, d.ABSORPTION,
                                                     targets, scale, image, None, g,
                                                     loss_out=loss),
                           max(args.steps, 50), args.warmup, stream, torch)
        ms_graph = _timed(lambda: b.run(d.PASS_FUSED, scale, loss, graph=True),
                          max(args.steps, 50), args.warmup, stream, torch)
        b.close()
        log(f"c1: single-view call {ms_single * 1e3:.1f} us, graph replay {ms_graph * 1e3:.1f} us, "
            f"{S} samples")
        out.update({"metric": "fwd+adjoint ray-samples/s (fused forward + L2 + adjoint)",
                    "value": S / (ms_graph * 1e-3), "ms_per_step": ms_graph,
                    "config": {"workload": w.name + ", fused L2, density gradient",
                               "samples_per_step": S, "single_call_ms": ms_single,
                               "launch": "one fused launch, HIP graph replay",
                               "tuning": d.get_tuning()}})
    elif args.workload == "c5":
        res = inversion_c5(d, torch, args, stream)
        out.update({"metric": "fwd+adjoint ray-samples/s (fused forward + L2 + adjoint)",
                    "value": res["auto"]["value"], "ms_per_step": res["auto"]["ms_per_step"],
                    "config": {"workload": res["workload"],
                               "samples_per_step": res["auto"]["samples_per_step"],
                               "tuning": res["tuning"], "tuning_source": res["tuning_source"]},
                    "auto": res["auto"]})
        if "checkpoint" in res:
            out["checkpoint"] = res["checkpoint"]
    elif args.workload == "c2":
        w = synth.make_c2()
        vol = stored(w.volume, w.storage)
        tf = torch.from_numpy(w.tf).to(dev)
        cams = cams_of(w.views)
        nv = len(cams)
        W = H = w.views[0].width
        # targets: the same grid under a TF with seeded +-20% perturbations
        tf_t = torch.from_numpy(w.tf * synth.rng_for(9, 1).uniform(0.8, 1.2, w.tf.shape)
                                .astype(np.float32)).to(dev)
        targets = torch.empty((nv, H, W, 4), device=dev)
        tb = d.Batch([vol], [tf_t], [d.make_view(0, cams[i], w.step_world, targets[i],
                                                 tf_index=0) for i in range(nv)],
                     d.EMISSION_ABSORPTION)
        tb.run(d.PASS_FORWARD)
        torch.cuda.synchronize()
        tb.close()
        images = torch.empty_like(targets)
        trans = torch.empty((nv, H, W), device=dev)
        dV = torch.zeros(w.volume.shape, device=dev)
        dTF = torch.zeros_like(tf)
        dstep = torch.zeros(nv, device=dev)
        dcam = torch.zeros((nv, 12), device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        scale = 1.0 / images.numel()
        res = {}
        for mode, flags in (("auto", 0),):
            views = [d.make_view(0, cams[i], w.step_world, images[i], transmittance=trans[i],
                                 target=targets[i], d_step=dstep[i:i + 1], tf_index=0,
                                 d_camera=dcam[i]) for i in range(nv)]
            b = d.Batch([vol], [tf], views, d.EMISSION_ABSORPTION, flags=flags,
                        d_volumes=[dV], d_tfs=[dTF])
            ws = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32, device=dev)
            S = b.sample_count()
            ms = _timed(lambda: b.run(d.PASS_FUSED, scale, loss, workspace=ws, graph=True),
                        args.steps, args.warmup, stream, torch)
            res[mode] = {"ms_per_step": ms, "value": S / (ms * 1e-3), "samples_per_step": S}
            log(f"{args.workload} {mode}: {ms:.3f} ms, {S / (ms * 1e-3):.4g} ray-samples/s")
            b.close()
        out.update({"metric": "fwd+adjoint ray-samples/s (fused forward + L2 + adjoint)",
                    "value": res["auto"]["value"], "ms_per_step": res["auto"]["ms_per_step"],
                    "config": {"workload": w.name + ", gradients density+TF+camera+step",
                               "samples_per_step": res["auto"]["samples_per_step"],
                               "tuning": d.get_tuning()}})
    elif args.workload == "color":
        w = synth.make_color()
        vol = stored(w.volume, w.storage)
        cams = cams_of(w.views)
        nv = len(cams)
        W = H = w.views[0].width
        rng = synth.rng_for(9, 6)
        targets = torch.from_numpy(rng.uniform(0.0, 1.0, (nv, H, W, 4)).astype(np.float32)).to(dev)
        images = torch.empty_like(targets)
        trans = torch.empty((nv, H, W), device=dev)
        dV = torch.zeros(w.volume.shape, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        scale = 1.0 / images.numel()
        grads = d.grads_desc(dV)
        # samples per step: the sample count depends only on the geometry, so
        # an absorption-only batch over a scalar grid of the same size counts it
        geo = torch.empty(w.volume.shape[:3], dtype=torch.bfloat16, device=dev)
        cb = d.Batch([geo], None, [d.make_view(0, cams[i], w.step_world, images[i, :, :, 0])
                                   for i in range(nv)], d.ABSORPTION)
        S = cb.sample_count()
        cb.close()
        del geo

        def step():
            for i in range(nv):
                d.render_fused_l2(vol, None, cams[i], w.step_world, d.COLOR, targets[i], scale,
                                  images[i], trans[i], grads, loss_out=loss)

        res = {}
        routes = () if args.no_plain else (("auto", d.ADJ_AUTO), ("residual", d.ADJ_RESIDUAL))
        for mode, flags in routes:
            fn = step if flags == 0 else (lambda: [d.render_fused_l2(
                vol, None, cams[i], w.step_world, d.COLOR, targets[i], scale, images[i], trans[i],
                grads, flags=flags, loss_out=loss) for i in range(nv)])
            ms = _timed(fn, args.steps, args.warmup, stream, torch)
            res[mode] = {"ms_per_step": ms, "value": S / (ms * 1e-3)}
            log(f"color {mode}: {ms:.3f} ms, {S / (ms * 1e-3):.4g} ray-samples/s")
        fwd_ms = None
        if not args.no_plain:
            fwd_ms = _timed(lambda: [d.render_forward(vol, None, cams[i], w.step_world, d.COLOR,
                                                      images[i], trans[i]) for i in range(nv)],
                            args.steps, args.warmup, stream, torch)
            log(f"color forward only: {fwd_ms:.3f} ms")
        # the same step as one batched launch per pass, replayed from a HIP graph
        cb = d.Batch([vol], None, [d.make_view(0, cams[i], w.step_world, images[i],
                                               transmittance=trans[i], target=targets[i])
                                   for i in range(nv)], d.COLOR, d_volumes=[dV])
        b_ms = _timed(lambda: cb.run(d.PASS_FUSED, scale, loss, graph=True), args.steps,
                      args.warmup, stream, torch)
        cb.close()
        log(f"color batched (one launch, graph): {b_ms:.3f} ms, {S / (b_ms * 1e-3):.4g} "
            f"ray-samples/s")
        res["batched"] = {"ms_per_step": b_ms, "value": S / (b_ms * 1e-3)}
        # The batched launch against HBM on its measured DRAM bytes (rocprofv3
        # FETCH_SIZE + WRITE_SIZE, committed with the kernel source's hash).
        # Algorithmic bytes per sample pair (8 corner gathers of 4 bf16 channels
        # in the forward and again in the adjoint, 8 x 4 float32 gradient
        # scatters) over the launch are a gather/scatter rate that the LDS
        # bricks serve, reported beside it, not against the HBM peak.
        alg = S * (2 * 8 * 4 * 2 + 8 * 4 * 4)
        c = counters_record("k_color_lds_bf16_fused_color", b_ms)
        tr = None
        t = load_counters("k_color_lds_bf16_fused_color")
        if t:
            tr = t.get("dram_bytes_per_launch")
        out["roofline"] = {"bound": "hbm", "achieved": c.get("dram_gbs"), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": c.get("dram_frac"), "traffic": tr,
                           "kernel": "k_color_lds<bf16, fused> (64 views, one launch)",
                           "kernel_ms": round(b_ms, 4),
                           "counters": c.get("counters"),
                           "note": "DRAM bytes of the launch (rocprofv3, copy-calibrated) over "
                                   "its event-timed duration; the adjoint's device-scope float "
                                   "atomics, carried out past the per-XCD L2, are most of them"}
        if t:
            out["roofline"]["valu_frac"] = c.get("valu_frac")
            out["roofline"]["atomic_requests_per_launch"] = t.get("counters", {}).get(
                "TCC_EA0_ATOMIC_sum")
        out["lds_gather_rate"] = {"achieved": round(alg / (b_ms * 1e-3) / 1e9, 1),
                                  "unit": "GB/s", "alg_bytes_per_launch": alg,
                                  "note": "algorithmic bytes (256 per sample pair) over the "
                                          "launch, served by the LDS bricks: not HBM traffic"}
        if not getattr(args, "no_cpu_baseline", False):
            out["cpu_baseline"] = cpu_baseline_color(w, w.volume)
            log(f"cpu baseline: {out['cpu_baseline']}")
        out.update({"metric": "fwd+adjoint ray-samples/s (fused forward + L2 + adjoint)",
                    "value": res["batched"]["value"], "ms_per_step": res["batched"]["ms_per_step"],
                    "config": {"workload": w.name + ", fused L2, colour-volume gradient",
                               "samples_per_step": S,
                               "launch": "one batched launch per step, HIP graph replay"},
                    "per_view_launches": res.get("auto"), "residual_form": res.get("residual"),
                    "forward_ms_per_view_launches": fwd_ms})
    elif args.workload == "dfc":
        w = synth.make_color()
        vol = stored(w.volume, w.storage)
        rng = synth.rng_for(9, 7)
        tf = torch.from_numpy(synth.random_tf(32, rng, synth.COLOR_TAU_MAX)).to(dev)
        shape = w.volume.shape[:3]
        nvox = int(np.prod(shape))
        ncand = 256
        a = torch.zeros(shape, device=dev)
        b = torch.zeros(shape, device=dev)
        nch = torch.zeros(1, dtype=torch.int32, device=dev)
        alpha = d.density_from_color(vol, tf, a, seed=7, sweep=0, ncand=ncand)
        it = [1]

        def sweep():
            src, dst = (a, b) if it[0] % 2 else (b, a)
            d.density_from_color(vol, tf, dst, d_prev=src, alpha=alpha, beta=1.0, seed=7,
                                 sweep=it[0], ncand=ncand, n_changed=nch)
            it[0] += 1

        ms = _timed(sweep, args.steps, args.warmup, stream, torch)
        log(f"dfc: {ms:.3f} ms per sweep, {nvox * ncand / (ms * 1e-3):.4g} candidates/s")
        if not getattr(args, "no_cpu_baseline", False):
            cv_read = vol.to(torch.float64).cpu().numpy()
            out["cpu_baseline"] = cpu_baseline_dfc(cv_read, tf.cpu().numpy(),
                                                   b.cpu().numpy(), alpha, ncand)
            log(f"cpu baseline: {out['cpu_baseline']}")
        # ALU roofline: VALU lane-operations of the candidate loop (counted in
        # the kernel's assembly) per sweep over its event-timed duration (one
        # launch per sweep, on the timed stream)
        try:
            with open(os.path.join(ROOT, "profiles", "valu_per_candidate_dfc.json")) as f:
                vc = json.load(f)
        except (OSError, ValueError):
            vc = None
        dfc_sha = kernel_source_hash(["paper_2107_12672_amd/csrc/ddvr_dfc.hip",
                                      "paper_2107_12672_amd/csrc/ddvr_internal.h"])
        tr = None
        try:
            with open(os.path.join(ROOT, "profiles", "traffic_dfc.json")) as f:
                t = json.load(f)
            if t.get("kernel_source_sha") == dfc_sha:
                tr = t.get("bytes_per_launch")
        except (OSError, ValueError):
            pass
        if vc and vc.get("kernel_source_sha") == dfc_sha:
            ops = nvox * ncand * vc["valu_per_candidate"]
            a = ops / (ms * 1e-3) / 1e12
            peak = valu_ceiling() or VALU_PUBLISHED_TOPS
            single = valu_ceiling("single_issue_tops")
            out["roofline"] = {"bound": "alu", "achieved": round(a, 3), "peak": peak,
                               "unit": "TOP/s", "frac": round(a / peak, 4),
                               "frac_of_single_issue": round(a / single, 4) if single else None,
                               "peak_source": "measured VALU issue ceiling (dual issue), "
                                              "profiles/valu_ceiling.json",
                               "traffic": tr, "kernel": "k_density_from_color<bf16>",
                               "kernel_ms": round(ms, 4), "ops_per_launch": ops,
                               "ops": "VALU lane-instructions: %d per candidate" %
                                      vc["valu_per_candidate"]}
        else:
            out["roofline"] = None
        out.update({"metric": "candidate evaluations/s (density from colour, one sweep)",
                    "unit": "candidates/s", "value": nvox * ncand / (ms * 1e-3),
                    "ms_per_step": ms,
                    "config": {"workload": f"density from colour: {w.name.split(',')[0]}, "
                                           f"R=32 TF, {ncand} candidates per voxel, "
                                           "6-neighbour term", "voxels": nvox,
                               "candidates": ncand}})
    elif args.workload == "recon":
        from paper_2107_12672_amd import recon
        w = synth.make_c3()
        gt32 = torch.from_numpy(w.target_volume).to(dev)
        gt = torch.empty_like(gt32, dtype=torch.bfloat16)
        d.cast_volume(gt32, gt)
        cams = cams_of(w.views)
        W = H = w.views[0].width
        targets = torch.empty((len(cams), H, W), device=dev)
        tb = d.Batch([gt], None, [d.make_view(0, cams[i], w.step_world, targets[i])
                                  for i in range(len(cams))], d.ABSORPTION)
        tb.run(d.PASS_FORWARD)
        torch.cuda.synchronize()
        tb.close()
        sched = recon.Schedule()
        t0 = time.perf_counter()
        rc = recon.Reconstructor(targets, cams, sched)     # plans every level's batches
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(args.warmup):
            rc.run()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        res = None
        for _ in range(args.steps):
            res = rc.run()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        gpu_ms = ev0.elapsed_time(ev1) / args.steps
        losses = res.losses.cpu().numpy()
        err = float(torch.linalg.vector_norm(res.volume - gt32) / torch.linalg.vector_norm(gt32))
        log(f"recon: {ms:.1f} ms for {res.steps} steps (events {gpu_ms:.1f} ms, setup "
            f"{setup_ms:.0f} ms once), {res.samples} samples, loss "
            f"{losses[0]:.4g} -> {losses[-1]:.4g}, relative volume error {err:.4f}")
        rc.close()
        out.update({"metric": "end-to-end reconstruction ray-samples/s (fused L1 + adjoint, "
                              "3D prior, Adam, resampling)",
                    "value": res.samples / (ms * 1e-3), "ms_per_step": ms,
                    "config": {"workload": "multi-resolution AO reconstruction of the C3 ground "
                                           "truth from 64 views at 512^2: 32^3->256^3, 10 "
                                           "steps per level, 50 at 256^3, batches of 8, "
                                           "lr 0.3, prior 0.5, step 0.2 voxel",
                               "steps": res.steps, "samples": res.samples,
                               "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                               "relative_volume_error": round(err, 4),
                               "setup_ms_once": round(setup_ms, 1)}})
    elif args.workload == "viewpoint":
        # viewpoint gradients (yaw, pitch, dist) of every view of the C5 grid:
        # forward-delayed (one tangent pass per view), forward-immediate
        # (tangent images written), and the adjoint (batched forward + adjoint
        # with camera gradients) -- the comparison of Sec. 5.1
        w = synth.make_c5()
        vol = stored(w.volume, w.storage)
        tf = torch.from_numpy(w.tf).to(dev)
        cams = cams_of(w.views)
        nv = len(cams)
        W = H = w.views[0].width
        rng = synth.rng_for(9, 5)
        gs = torch.from_numpy(rng.normal(size=(nv, H, W, 4)).astype(np.float32)
                              / (H * W)).to(dev)
        dirs = []
        for v in w.views:
            J = d.camera_sphere_tangents(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                         math.radians(v.fovy), W, H)
            dirs.append([J[0] + [0.0], J[1] + [0.0], J[2] + [0.0]])
        images = torch.empty((nv, H, W, 4), device=dev)
        dots = torch.empty((3, H, W, 4), device=dev)
        d_dir = torch.zeros((nv, 3), device=dev)

        def delayed():
            for i in range(nv):
                d.render_tangent(vol, tf, cams[i], w.step_world, d.EMISSION_ABSORPTION, dirs[i],
                                 image=images[i], d_image=gs[i], d_dir=d_dir[i])

        def immediate():
            for i in range(nv):
                d.render_tangent(vol, tf, cams[i], w.step_world, d.EMISSION_ABSORPTION, dirs[i],
                                 image=images[i], image_dot=dots)

        trans = torch.empty((nv, H, W), device=dev)
        dcam = torch.zeros((nv, 12), device=dev)
        views = [d.make_view(0, cams[i], w.step_world, images[i], transmittance=trans[i],
                             d_image=gs[i], d_camera=dcam[i], tf_index=0) for i in range(nv)]
        b = d.Batch([vol], [tf], views, d.EMISSION_ABSORPTION)
        ws = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32, device=dev)
        S = b.sample_count()

        plan = d.Plan(b, d.PLAN_LOSS_GIVEN, workspace=ws)

        def adjoint():
            plan.run()

        res = {}
        for name, fn in (("forward_delayed", delayed), ("forward_immediate", immediate),
                         ("adjoint", adjoint)):
            ms = _timed(fn, args.steps, args.warmup, stream, torch)
            res[name] = {"ms_per_step": ms, "value": S / (ms * 1e-3)}
            log(f"viewpoint {name}: {ms:.3f} ms, {S / (ms * 1e-3):.4g} ray-samples/s")
        out.update({"metric": "ray-samples/s of the viewpoint (yaw, pitch, dist) gradient",
                    "value": res["forward_delayed"]["value"],
                    "ms_per_step": res["forward_delayed"]["ms_per_step"],
                    "config": {"workload": w.name + ", gradient w.r.t. yaw, pitch, dist of "
                                                    "every view (seeded upstream gradients)",
                               "samples_per_step": S},
                    "routes": res})
    else:   # c4
        ws_ = synth.make_c4()
        vols = [stored(w.volume, w.storage) for w in ws_]
        tfs = [torch.from_numpy(w.tf).to(dev) for w in ws_]
        imgs, trs, gs, views = [], [], [], []
        dcam = torch.zeros((len(ws_), 12), device=dev)
        dstep = torch.zeros(len(ws_), device=dev)
        # the loss is minus the opacity entropy of each image; its image
        # gradients live in one buffer, cleared once per step
        gbuf = torch.zeros(sum(w.views[0].height * w.views[0].width * 4 for w in ws_), device=dev)
        off = 0
        for i, w in enumerate(ws_):
            v = w.views[0]
            imgs.append(torch.empty((v.height, v.width, 4), device=dev))
            trs.append(torch.empty((v.height, v.width), device=dev))
            gs.append(gbuf[off:off + v.height * v.width * 4].view(v.height, v.width, 4))
            off += v.height * v.width * 4
            cam = cams_of([v])[0]
            views.append(d.make_view(i, cam, w.step_world, imgs[i], transmittance=trs[i],
                                     d_image=gs[i], d_camera=dcam[i], d_step=dstep[i:i + 1],
                                     tf_index=i))
        # launch shape: the autotuner's choice for the uneven-batch class, if cached
        from paper_2107_12672_amd import autotune
        tuned = autotune.apply(autotune.c4_key(_arch(torch)))
        b = d.Batch(vols, tfs, views, d.EMISSION_ABSORPTION)
        ws = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32, device=dev)
        S = b.sample_count()
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        # the whole step -- forward, entropy of every image and its gradient,
        # adjoint, fallback -- is one recorded graph
        plan = d.Plan(b, d.PLAN_LOSS_NEG_ENTROPY, 1.0, loss, workspace=ws)
        ms = _timed(plan.run, args.steps, args.warmup, stream, torch)
        oe = plan.loss_terms()
        log(f"c4: {ms:.3f} ms, {S / (ms * 1e-3):.4g} ray-samples/s, {S} samples; "
            f"mean OE {sum(oe) / len(oe):.4f}")
        plan.close()
        b.close()
        out.update({"metric": "fwd+adjoint ray-samples/s (forward, -OE loss, adjoint)",
                    "value": S / (ms * 1e-3), "ms_per_step": ms,
                    "config": {"workload": "uneven batch: 16 grids (edges 64-384, f16/f32, "
                                           "EA, R 8-64), one view each at 128-1024 px, "
                                           "loss -OE per image, camera + step gradients, "
                                           "persistent launch",
                               "launch": "one step plan: forward, entropy sums and gradient "
                                         "of all views, adjoint, fallback in one HIP graph",
                               "samples_per_step": S, "tuning": d.get_tuning(),
                               "tuning_source": "autotuned" if tuned else "default"}})
    d.set_tuning(**old_tuning)
    print(json.dumps(out), flush=True)


def inversion_c3(d, torch, vol16, views, dV, scale, loss, S, args, stream):
    """Fused forward + L2 + adjoint of the timed batch with INVERT_T: every
    sample re-gathers its density, recomputes exp(-dt tau) and divides it out
    of the transmittance."""
    b = d.Batch([vol16], None, views, d.ABSORPTION, flags=d.ADJ_INVERT_T, d_volumes=[dV])
    try:
        ms = _timed(lambda: b.run(d.PASS_FUSED, scale, loss, graph=True), args.steps,
                    args.warmup, stream, torch)
        builds = b.graph_builds()
    finally:
        b.close()
    dV.zero_()
    log(f"c3 inversion (INVERT_T): {ms:.3f} ms, {S / (ms * 1e-3):.4g} ray-samples/s")
    rec = {"ms_per_step": round(ms, 4), "value": S / (ms * 1e-3), "unit": "ray-samples/s",
           "samples_per_step": S, "mode": "INVERT_T fused, one launch, HIP graph replay",
           "graph_builds": builds}
    rec.update(counters_record("k_render_ao_bf16_invert_c3", ms))
    return rec


def load_counters(name):
    """Committed rocprofv3 counters of a kernel (profiles/counters_<name>.json),
    if taken on the current kernel source."""
    try:
        with open(os.path.join(ROOT, "profiles", f"counters_{name}.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    return t if t.get("kernel_source_sha") == kernel_source_hash() else None


def counters_record(name, ms):
    """Committed rocprofv3 counters of a kernel (profiles/counters_<name>.json,
    taken on the current kernel source) as rates over `ms` per launch."""
    try:
        with open(os.path.join(ROOT, "profiles", f"counters_{name}.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {"counters": None}
    if t.get("kernel_source_sha") != kernel_source_hash():
        return {"counters": "stale (kernel source changed since they were taken)"}
    out = {"counters": f"profiles/counters_{name}.json"}
    if t.get("dram_bytes_per_launch"):
        gbs = t["dram_bytes_per_launch"] / (ms * 1e-3) / 1e9
        out["dram_gbs"] = round(gbs, 1)
        out["dram_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    if t.get("valu_thread_cycles_per_launch"):
        tops = t["valu_thread_cycles_per_launch"] / (ms * 1e-3) / 1e12
        ceil = valu_ceiling()
        out["valu_active_lane_tops"] = round(tops, 3)
        if ceil:
            out["valu_frac"] = round(tops / ceil, 4)
    return out


def inversion_c5(d, torch, args, stream):
    """Emission-absorption 512^3 f16, 32 views at 1024^2, R=32, step 0.25
    voxel, fused L2 with density, TF and step gradients: the T-form inversion
    (AUTO; opaque rays to the checkpoint fallback) and segment checkpointing
    for every ray."""
    import numpy as np
    import synth
    dev = torch.device("cuda:0")
    w = synth.make_c5()
    v32 = torch.from_numpy(np.ascontiguousarray(w.volume)).to(dev)
    vol = torch.empty_like(v32, dtype=torch.float16)
    d.cast_volume(v32, vol)
    del v32
    tf = torch.from_numpy(w.tf).to(dev)
    cams = [d.camera_from_sphere(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                 math.radians(v.fovy), v.width, v.height) for v in w.views]
    nv = len(cams)
    W = H = w.views[0].width
    tf_t = torch.from_numpy(w.tf * synth.rng_for(9, 1).uniform(0.8, 1.2, w.tf.shape)
                            .astype(np.float32)).to(dev)
    targets = torch.empty((nv, H, W, 4), device=dev)
    tb = d.Batch([vol], [tf_t], [d.make_view(0, cams[i], w.step_world, targets[i], tf_index=0)
                                 for i in range(nv)], d.EMISSION_ABSORPTION)
    tb.run(d.PASS_FORWARD)
    torch.cuda.synchronize()
    tb.close()
    images = torch.empty_like(targets)
    trans = torch.empty((nv, H, W), device=dev)
    dV = torch.zeros(w.volume.shape, device=dev)
    dTF = torch.zeros_like(tf)
    dstep = torch.zeros(nv, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    scale = 1.0 / images.numel()
    res = {"workload": w.name + ", fused L2, gradients density+TF+step"}
    # launch shape: the autotuner's choice for this class, if cached
    from paper_2107_12672_amd import autotune
    old_tuning = d.get_tuning()
    res["tuning_source"] = "autotuned" if autotune.apply(autotune.workload_key(
        _arch(torch), d.EMISSION_ABSORPTION, "f16", w.tf.shape[0], W, w.volume.shape[0],
        "V+TF+step", d.PASS_FUSED)) else "default"
    res["tuning"] = d.get_tuning()
    for mode, flags, steps, warm in (("auto", d.ADJ_AUTO, max(2, min(args.steps, 5)), 1),
                                     ("checkpoint", d.ADJ_CHECKPOINT, args.c5_checkpoint, 0)):
        if steps <= 0:
            continue
        views = [d.make_view(0, cams[i], w.step_world, images[i], transmittance=trans[i],
                             target=targets[i], d_step=dstep[i:i + 1], tf_index=0)
                 for i in range(nv)]
        b = d.Batch([vol], [tf], views, d.EMISSION_ABSORPTION, flags=flags, d_volumes=[dV],
                    d_tfs=[dTF])
        ws = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32, device=dev)
        S = b.sample_count()
        ms = _timed(lambda: b.run(d.PASS_FUSED, scale, loss, workspace=ws, graph=warm > 0),
                    steps, warm, stream, torch)
        b.close()
        del ws
        rec = {"ms_per_step": round(ms, 3), "value": S / (ms * 1e-3), "unit": "ray-samples/s",
               "samples_per_step": S, "steps": steps}
        rec.update(counters_record(f"k_render_ea_f16_{mode}_c5", ms))
        res[mode] = rec
        log(f"c5 {mode}: {ms:.3f} ms, {S / (ms * 1e-3):.4g} ray-samples/s")
    d.set_tuning(**old_tuning)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="grid edge")
    ap.add_argument("--views", type=int, default=64)
    ap.add_argument("--image", type=int, default=512)
    ap.add_argument("--step-vox", type=float, default=0.2)
    ap.add_argument("--workload", default="c3",
                    choices=("c3", "c1", "c2", "c4", "c5", "viewpoint", "color", "dfc", "recon"),
                    help="c3 (default) is the headline tomography step; the others print "
                         "their own line")
    ap.add_argument("--burn-in", type=int, default=4,
                    help="untimed reconstruction iterations from the zero grid before warmup")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-views", type=int, default=0,
                    help="views of the plain path to time (0 = all)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a float32 copy of MIB MiB through the library (3 times), "
                         "to calibrate HBM byte counters, and exit")
    ap.add_argument("--calibrate-valu", action="store_true",
                    help="only time the VALU issue-rate probe (non-packed fp32 FMA and int "
                         "add, 16 independent chains per lane) and exit")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the emission-absorption 512^3 inversion records")
    ap.add_argument("--c5-checkpoint", type=int, default=1,
                    help="timed launches of the C5 segment-checkpoint adjoint (0: skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(views would shard across GPUs with one all-reduce of the gradients). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2107_12672_amd import ddvr as d

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    if args.workload != "c3":
        secondary(args)
        return
    dev = torch.device("cuda:0")
    if args.calibrate_valu:
        props = torch.cuda.get_device_properties(0)
        res = {"device": props.name, "compute_units": props.multi_processor_count}
        for mode, name in ((0, "fma"), (1, "int_add"), (2, "fma_int_add"), (3, "fma_exp2"),
                           (4, "mul_max"), (5, "shift_xor"), (6, "fma_max"),
                           (7, "mul_max_independent")):
            for blocks in (2048, 8192):
                tops, ms = valu_probe(mode, blocks, 16000)
                key = f"{name}_{blocks}wg"
                res[key] = {"tops": round(tops, 3), "ms": round(ms, 4),
                            "wave_instr_per_cu_per_ns": round(
                                tops * 1e12 / 64 / props.multi_processor_count / 1e9, 4)}
                log(f"valu probe {key}: {tops:.3f} T lane-ops/s, {ms:.3f} ms")
        res["fma_tops"] = max(res["fma_2048wg"]["tops"], res["fma_8192wg"]["tops"])
        res["issue_tops"] = max(v["tops"] for v in res.values()
                                if isinstance(v, dict) and "tops" in v)
        res["published_fp32_tops"] = VALU_PUBLISHED_TOPS
        res["nonpacked_nominal_tops"] = VALU_NONPACKED_TOPS
        print(json.dumps(res), flush=True)
        return
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            d.cast_volume(src, dst)
        torch.cuda.synchronize()
        # achievable HBM bandwidth: the same copy timed with events (read + write)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            d.cast_volume(src, dst)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 13,
                          "copy_ms": ms, "copy_gbs": 8 * n / (ms * 1e-3) / 1e9}))
        return
    work = synth.make_c3(args.n, args.views, args.image, args.step_vox)
    W = H = args.image
    nv = len(work.views)
    step = work.step_world
    log(f"workload: {args.n}^3 bf16, {nv} views {W}x{H}, step {args.step_vox} vox")

    # ground truth -> target images (input preparation, untimed)
    gt32 = torch.from_numpy(work.target_volume).to(dev)
    gt16 = torch.empty_like(gt32, dtype=torch.bfloat16)
    d.cast_volume(gt32, gt16)
    cams = [d.camera_from_sphere(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                 math.radians(v.fovy), W, H) for v in work.views]
    targets = torch.empty((nv, H, W), device=dev)
    tviews = [d.make_view(0, cams[i], step, targets[i]) for i in range(nv)]
    tb = d.Batch([gt16], None, tviews, d.ABSORPTION)
    tb.run(d.PASS_FORWARD)
    torch.cuda.synchronize()
    tb.close()
    del gt16

    # launch shape: the autotuner's choice for this workload class, if cached
    from paper_2107_12672_amd import autotune
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    tkey = autotune.workload_key(arch, d.ABSORPTION, "bf16", 0, W, args.n, "V", d.PASS_FUSED)
    tuned = autotune.apply(tkey)
    log(f"tuning ({'autotuned' if tuned else 'default'}): {d.get_tuning()}")

    # reconstruction state: float32 master (zero-initialised), bf16 storage, gradient
    master = torch.zeros((args.n,) * 3, device=dev)
    vol16 = torch.empty_like(master, dtype=torch.bfloat16)
    dV = torch.zeros_like(master)
    images = torch.empty((nv, H, W), device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    scale = 1.0 / (nv * W * H)
    views = [d.make_view(0, cams[i], step, images[i], target=targets[i]) for i in range(nv)]
    batch = d.Batch([vol16], None, views, d.ABSORPTION, d_volumes=[dV])
    S = batch.sample_count()
    log(f"samples per step: {S:.4g}")

    stream = torch.cuda.current_stream()
    lr = [0.0]

    def one_step(ev=None):
        d.cast_volume(master, vol16)
        loss.zero_()
        if ev is not None:
            ev[0].record(stream)
        batch.run(d.PASS_FUSED, scale, loss, graph=True)
        if ev is not None:
            ev[1].record(stream)
        if lr[0] == 0.0:
            # step size fixed once: the first update moves the densest voxel by 0.25
            lr[0] = 0.25 / max(float(dV.abs().max()), 1e-30)
        master.add_(dV, alpha=-lr[0]).clamp_(min=0.0)
        dV.zero_()

    for _ in range(args.burn_in + args.warmup):
        one_step()
    torch.cuda.synchronize()
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for k in range(args.steps):
        one_step(kev[k])
    t_stop.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_stop)
    ms_step = ms_total / args.steps
    k_ms = sum(a.elapsed_time(b) for a, b in kev) / args.steps
    value = S / (ms_step * 1e-3)
    log(f"step {ms_step:.3f} ms, fused kernel {k_ms:.3f} ms, {value:.4g} ray-samples/s")
    # share of pixels whose residual (and so adjoint seed) is non-zero in the timed state
    seeded = float((images != targets).float().mean())
    log(f"pixels with a non-zero residual: {seeded:.4f}, loss {float(loss):.4g}")

    # The fused kernel is bound by VALU issue: rocprofv3's count of VALU
    # lane-instructions per launch (SQ_THREAD_CYCLES_VALU, committed with the
    # kernel source's hash) over the kernel's event-timed duration, against the
    # measured issue ceiling of the same quantity (profiles/valu_ceiling.json:
    # instruction pairs that dual-issue; FMA chains alone reach about half,
    # reported beside it).  The live probe of this run checks the device.
    achieved_gbs = S * ALG_BYTES_BF16 / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    counters = load_counters("k_render_ao_bf16_fused_c3")
    live_tops, _ = valu_probe(4, 8192, 4000)
    ceiling = valu_ceiling()
    single = valu_ceiling("single_issue_tops")
    peak = ceiling if ceiling else live_tops
    log(f"VALU ceiling: committed {ceiling} (single issue {single}), live probe "
        f"{live_tops:.3f} T lane-instructions/s")
    roofline = {"bound": "alu", "achieved": None, "peak": round(peak, 3), "unit": "TOP/s",
                "frac": None, "traffic": traffic, "kernel": "k_render<AO,bf16,4 waves,fused>",
                "kernel_ms": round(k_ms, 4),
                "peak_source": "measured VALU issue ceiling: independent multiply/max pairs "
                               "(dual issue), library flags (profiles/valu_ceiling.json)"
                               if ceiling else "measured live: VALU probe of this run",
                "peak_live": round(live_tops, 3),
                "peak_single_issue": single,
                "peak_published_fp32": VALU_PUBLISHED_TOPS}
    if counters and counters.get("valu_thread_cycles_per_launch"):
        ops = counters["valu_thread_cycles_per_launch"]
        a_tops = ops / (k_ms * 1e-3) / 1e12
        roofline.update({"achieved": round(a_tops, 3), "frac": round(a_tops / peak, 4),
                         "frac_of_single_issue": round(a_tops / single, 4) if single else None,
                         "ops_per_launch": ops,
                         "ops": "VALU lane-instructions per launch (rocprofv3 "
                                "SQ_THREAD_CYCLES_VALU, profiles/counters_"
                                "k_render_ao_bf16_fused_c3.json)",
                         "valu_wave_instr_per_launch":
                             counters.get("valu_wave_instr_per_launch")})
    else:
        roofline["note"] = ("counters missing or taken on another kernel source: "
                            "profiles/counters_k_render_ao_bf16_fused_c3.json")
    roofline_hbm = None
    if traffic:
        gbs = traffic / (k_ms * 1e-3) / 1e9
        roofline_hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "traffic": traffic,
                        "note": "DRAM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                "calibrated on a copy) over the event-timed launch"}
    gather = {"achieved": round(achieved_gbs, 1), "unit": "GB/s",
              "alg_bytes_per_launch": S * ALG_BYTES_BF16,
              "note": "algorithmic bytes (16 s_V + 32 per sample pair) over the launch: a "
                      "gather/scatter rate served by the LDS bricks, not HBM traffic"}

    result = {
        "metric": "fwd+adjoint ray-samples/s (fused forward + L2 + adjoint)",
        "value": value, "unit": "ray-samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"absorption-only tomography: {args.n}^3 grid stored bf16 "
                               f"(f32 master), {nv} Fibonacci views at {W}x{H}, step "
                               f"{args.step_vox} voxel, L2 loss, gradient w.r.t. density",
                   "storage": "bf16", "samples_per_step": S, "views": nv, "image": W,
                   "grid": args.n, "step_vox": args.step_vox,
                   "launch": "one fused launch per step, HIP graph replay",
                   "state": f"after {args.burn_in + args.warmup} gradient-descent iterations "
                            f"from the zero grid",
                   "pixels_with_nonzero_residual": round(seeded, 4),
                   "tuning": d.get_tuning(), "tuning_source": "autotuned" if tuned else "default"},
        "roofline": roofline,
        "roofline_hbm_measured": roofline_hbm,
        "lds_gather_rate": gather,
    }

    # the same batch and state with the paper's inversion on every sample
    # (T-form, eq. inv-blend-forward solved for T^(i)): the AUTO launch above
    # takes the absorption-only closed form of that inversion
    inv = inversion_c3(d, torch, vol16, views, dV, scale, loss, S, args, stream)
    if inv:
        result["inversion_c3"] = inv
    if not args.no_c5:
        result["inversion_c5"] = inversion_c5(d, torch, args, stream)

    if not args.no_plain:
        # the plain per-view float32 path: one launch per view, global atomics
        pv = nv if args.plain_views <= 0 else min(nv, args.plain_views)
        dV32 = torch.zeros_like(master)
        g32 = d.grads_desc(dV32)
        img1 = torch.empty((H, W), device=dev)

        def plain_step(nviews):
            for i in range(nviews):
                d.render_fused_l2(master, None, cams[i], step, d.ABSORPTION, targets[i], scale,
                                  img1, None, g32, flags=d.LAUNCH_PLAIN, loss_out=loss)

        plain_step(min(2, pv))
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plain_step(pv)
        b.record(stream)
        torch.cuda.synchronize()
        plain_ms = a.elapsed_time(b) * nv / pv
        result["plain_fp32_per_view"] = {
            "ms_per_step": plain_ms, "views_timed": pv,
            "speedup": plain_ms / ms_step,
            "path": "float32 grid, one launch per view, direct gathers, global atomics"}
        log(f"plain per-view fp32: {plain_ms:.1f} ms per step -> speedup {plain_ms / ms_step:.2f}x")

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(work, nv)
        log(f"cpu baseline: {result['cpu_baseline']}")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
