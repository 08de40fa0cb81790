"""Autotuner for the launch shape of the render kernels.

For a workload (a function that builds a ``ddvr.Batch`` and a function that
runs one timed pass on it) the tuner tries candidate launch shapes -- waves
per workgroup (tile shape), LDS brick capacity, initial slab length, lane
mapping, batch schedule -- times each with HIP events, checks that every
candidate renders bitwise the same images (the per-ray arithmetic does not
depend on the launch shape), and stores the fastest under a key that
describes the workload class.  ``apply`` looks a key up and sets the
process-wide tuning before a batch is built.

Cache: JSON at $DDVR_TUNING_CACHE, else ``tuning_cache.json`` next to this
file.  Keys: ``arch|model|storage|R<bucket>|img<bucket>|grid<bucket>|grads|pass``
with power-of-two buckets.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from typing import Callable, Dict, Iterable, List, Optional

from . import ddvr as _d

HERE = os.path.dirname(os.path.abspath(__file__))


def cache_path() -> str:
    return os.environ.get("DDVR_TUNING_CACHE", os.path.join(HERE, "tuning_cache.json"))


def _bucket(x: float) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1.0, float(x))))))


def workload_key(arch: str, model: int, storage: str, R: int, image_px: int, grid_edge: int,
                 grads: str, pass_: int) -> str:
    """Key of a workload class: image and grid sizes and R in power-of-two buckets."""
    m = "ea" if model == _d.EMISSION_ABSORPTION else "ao"
    return (f"{arch}|{m}|{storage}|R{_bucket(R) if model == _d.EMISSION_ABSORPTION else 0}|"
            f"img{_bucket(image_px)}|grid{_bucket(grid_edge)}|{grads}|pass{pass_}")


def c4_key(arch: str) -> str:
    """Key of the uneven-batch class: many emission-absorption grids of mixed
    storage and size, one persistent launch per pass, camera and step
    gradients, the whole step as one plan."""
    return f"{arch}|ea|mixed|uneven-batch|cam+step|plan"


def color_key(arch: str, storage: str, image_px: int, grid_edge: int) -> str:
    """Key of a batched colour-volume workload (fused pass, colour gradient)."""
    return f"{arch}|color|{storage}|img{_bucket(image_px)}|grid{_bucket(grid_edge)}|V|pass2"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict], path: Optional[str] = None) -> None:
    path = path or cache_path()
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(key: str, path: Optional[str] = None) -> Optional[dict]:
    entry = load_cache(path).get(key)
    if not entry:
        return None
    t = entry.get("tuning")
    if not isinstance(t, dict) or set(t) != set(_d.TUNING_DEFAULT):
        return None
    return t


def apply(key: str, path: Optional[str] = None) -> bool:
    """Set the tuning cached for `key`; False (tuning unchanged) if none."""
    t = lookup(key, path)
    if t is None:
        return False
    _d.set_tuning(**t)
    return True


def default_candidates() -> List[dict]:
    out = []
    for waves, cap, k, lm, ax in itertools.product((2, 4), (5120, 6144, 7168, 8192, 12288),
                                                   (32, 64), (1, 2), (0, 1)):
        out.append({"waves": waves, "lds_cap": cap, "slab_k": k, "slab_kmax": 256,
                    "cell_acc": 1, "lane_map": lm, "schedule": 0, "slab_axis": ax})
    return out


def tune(key: str, make_batch: Callable[[], "object"], run: Callable[["object"], None],
         images: Callable[[], "object"], candidates: Optional[Iterable[dict]] = None,
         reps: int = 3, path: Optional[str] = None, verbose: bool = False) -> dict:
    """Time every candidate on the workload and cache the fastest.

    make_batch() builds a fresh batch under the current tuning; run(batch)
    enqueues one pass on torch's current stream; images() returns a tensor of
    the rendered images, compared across candidates: a launch shape may change
    only the grouping of float32 sums (absorption-only cell runs end at slab
    boundaries, which depend on the tile and brick size), so they must agree to
    1e-5 of the largest value."""
    import torch
    old = _d.get_tuning()
    results = []
    ref = None
    try:
        for cand in (list(candidates) if candidates is not None else default_candidates()):
            _d.set_tuning(**cand)
            try:
                b = make_batch()
            except _d.DDVRError:
                continue               # e.g. a brick that does not fit the device's LDS
            run(b)
            torch.cuda.synchronize()
            img = images().clone()
            if ref is None:
                ref = img
            elif not bool((img - ref).abs().max() <= 1e-5 * max(1.0, float(ref.abs().max()))):
                raise RuntimeError(f"launch shape {cand} changed the rendered images")
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                run(b)
            z.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(z) / reps
            results.append((ms, cand))
            if verbose:
                print(f"[autotune] {ms:9.3f} ms  {cand}", flush=True)
            b.close()
    finally:
        _d.set_tuning(**old)
    if not results:
        raise RuntimeError("no candidate launch shape could run")
    results.sort(key=lambda x: x[0])
    best_ms, best = results[0]
    cache = load_cache(path)
    cache[key] = {"tuning": best, "ms": best_ms,
                  "runner_up_ms": results[1][0] if len(results) > 1 else None,
                  "candidates": len(results)}
    save_cache(cache, path)
    return {"tuning": best, "ms": best_ms, "all": results}


def uneven_candidates() -> List[dict]:
    """Launch shapes of the persistent uneven-batch launch (its schedule is
    always the queue)."""
    out = []
    for waves, cap, k, lm, ax in itertools.product((2, 4), (4096, 7168, 10240), (32, 64),
                                                   (0, 2), (0, 1)):
        out.append({"waves": waves, "lds_cap": cap, "slab_k": k, "slab_kmax": 256,
                    "cell_acc": 1, "lane_map": lm, "schedule": 2, "slab_axis": ax})
    return out


def small_candidates() -> List[dict]:
    """Launch shapes of single small views (a few hundred tiles or fewer), where
    smaller tiles spread the work over more CUs."""
    out = []
    for waves, cap, k, lm, ax in itertools.product((1, 2, 4), (2048, 4096, 7168), (16, 64),
                                                   (0, 2), (0, 1)):
        out.append({"waves": waves, "lds_cap": cap, "slab_k": k, "slab_kmax": 256,
                    "cell_acc": 1, "lane_map": lm, "schedule": 0, "slab_axis": ax})
    return out


def c1_key(arch: str) -> str:
    """Absorption-only 32^3 f32, one 64^2 view, fused pass (density gradient)."""
    return workload_key(arch, _d.ABSORPTION, "f32", 0, 64, 32, "V", _d.PASS_FUSED)


def c2_key(arch: str) -> str:
    """Emission-absorption 128^3 f32, R=16, one 256^2 view, fused pass with
    density, TF, camera and step gradients."""
    return workload_key(arch, _d.EMISSION_ABSORPTION, "f32", 16, 256, 128, "V+TF+cam+step",
                        _d.PASS_FUSED)


def color_candidates() -> List[dict]:
    """The colour kernel takes 16x16 tiles and one item per workgroup; only its
    brick capacity (lds_cap / 4 vertices of 4 channels) is free."""
    base = dict(_d.TUNING_DEFAULT)
    return [dict(base, lds_cap=c) for c in (4096, 7168, 10240, 14336, 16384)]


def _device_arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def main(argv=None) -> None:
    """Tune a workload class and store the result in the cache:
      c1     absorption-only 32^3 f32, one 64x64 view, fused pass;
      c2     emission-absorption 128^3 f32, R=16, one 256x256 view, fused pass with
             density, TF, camera and step gradients;
      c3     absorption-only tomography (256^3 bf16, 64 views at 512x512, fused pass);
      c4     the uneven batch (16 grids of mixed size and storage, one view each,
             minus the opacity entropy, camera + step gradients, one step plan);
      c5     emission-absorption 512^3 f16, 32 views at 1024x1024, R=32, fused pass
             with density, TF and step gradients (T-form inversion, AUTO);
      color  the colour volume (256^3 x 4 bf16, the c3 views, fused pass)."""
    import argparse
    import sys
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3", choices=("c1", "c2", "c3", "c4", "c5", "color"))
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--views", type=int, default=64)
    ap.add_argument("--image", type=int, default=512)
    ap.add_argument("--step-vox", type=float, default=0.2)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import numpy as np
    import synth
    dev = torch.device("cuda:0")
    if args.workload in ("c1", "c2"):
        w = synth.make_c1() if args.workload == "c1" else synth.make_c2()
        v = w.views[0]
        vol = torch.from_numpy(np.ascontiguousarray(w.volume)).to(dev)
        cam = _d.camera_from_sphere(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                    math.radians(v.fovy), v.width, v.height)
        ea = args.workload == "c2"
        C = 4 if ea else 1
        tf = torch.from_numpy(w.tf).to(dev) if ea else None
        targets = torch.rand((v.height, v.width, C) if ea else (v.height, v.width), device=dev,
                             generator=torch.Generator("cuda").manual_seed(1))
        image = torch.empty_like(targets)
        trans = torch.empty((v.height, v.width), device=dev)
        dV = torch.zeros(w.volume.shape, device=dev)
        dTF = torch.zeros_like(tf) if ea else None
        dcam = torch.zeros(12, device=dev)
        dstep = torch.zeros(1, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        scale = 1.0 / image.numel()
        ws_ = {}

        def make_s():
            view = _d.make_view(0, cam, w.step_world, image, transmittance=trans, target=targets,
                                d_camera=dcam if ea else None, d_step=dstep if ea else None,
                                tf_index=0 if ea else -1)
            b = _d.Batch([vol], [tf] if ea else None, [view],
                         _d.EMISSION_ABSORPTION if ea else _d.ABSORPTION, d_volumes=[dV],
                         d_tfs=[dTF] if ea else None)
            ws_["ws"] = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32,
                                    device=dev)
            return b

        key = c2_key(_device_arch()) if ea else c1_key(_device_arch())
        res = tune(key, make_s, lambda b: b.run(_d.PASS_FUSED, scale, loss, workspace=ws_["ws"]),
                   lambda: image, candidates=small_candidates(), reps=max(args.reps, 20),
                   verbose=True)
        print(json.dumps({"key": key, "best": res["tuning"], "ms": res["ms"]}))
        return
    if args.workload == "c4":
        ws_ = synth.make_c4()
        vols, tfs, imgs, views = [], [], [], []
        for k, w in enumerate(ws_):
            v = w.views[0]
            v32 = torch.from_numpy(w.volume).to(dev)
            if w.storage == "f32":
                vols.append(v32)
            else:
                vols.append(torch.empty_like(v32, dtype=torch.float16))
                _d.cast_volume(v32, vols[-1])
            tfs.append(torch.from_numpy(w.tf).to(dev))
        npx = [w.views[0].width * w.views[0].height for w in ws_]
        flat = torch.empty(4 * sum(npx), device=dev)
        gflat = torch.zeros_like(flat)
        trans = torch.empty(sum(npx), device=dev)
        dcam = torch.zeros((len(ws_), 12), device=dev)
        dstep = torch.zeros(len(ws_), device=dev)
        off = 0
        for k, w in enumerate(ws_):
            v = w.views[0]
            cam = _d.camera_from_sphere(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                        math.radians(v.fovy), v.width, v.height)
            views.append(_d.make_view(k, cam, w.step_world, flat[4 * off:4 * (off + npx[k])],
                                      transmittance=trans[off:off + npx[k]],
                                      d_image=gflat[4 * off:4 * (off + npx[k])],
                                      d_camera=dcam[k], d_step=dstep[k:k + 1], tf_index=k))
            off += npx[k]
        state = {}

        def make():
            b = _d.Batch(vols, tfs, views, _d.EMISSION_ABSORPTION)
            ws = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32, device=dev)
            state["plan"] = _d.Plan(b, _d.PLAN_LOSS_NEG_ENTROPY, 1.0, None, workspace=ws)
            return b

        key = c4_key(_device_arch())
        res = tune(key, make, lambda b: state["plan"].run(), lambda: flat,
                   candidates=uneven_candidates(), reps=args.reps, verbose=True)
        print(json.dumps({"key": key, "best": res["tuning"], "ms": res["ms"]}))
        return
    if args.workload == "c5":
        w = synth.make_c5()
        v32 = torch.from_numpy(np.ascontiguousarray(w.volume)).to(dev)
        vol = torch.empty_like(v32, dtype=torch.float16)
        _d.cast_volume(v32, vol)
        del v32
        tf = torch.from_numpy(w.tf).to(dev)
        W = w.views[0].width
        cams = [_d.camera_from_sphere(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                      math.radians(v.fovy), W, W) for v in w.views]
        nv = len(cams)
        targets = torch.rand((nv, W, W, 4), device=dev,
                             generator=torch.Generator("cuda").manual_seed(1))
        images = torch.empty_like(targets)
        trans = torch.empty((nv, W, W), device=dev)
        dV = torch.zeros(w.volume.shape, device=dev)
        dTF = torch.zeros_like(tf)
        dstep = torch.zeros(nv, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        scale = 1.0 / images.numel()
        ws_ = {}

        def make5():
            views = [_d.make_view(0, cams[i], w.step_world, images[i], transmittance=trans[i],
                                  target=targets[i], d_step=dstep[i:i + 1], tf_index=0)
                     for i in range(nv)]
            b = _d.Batch([vol], [tf], views, _d.EMISSION_ABSORPTION, d_volumes=[dV],
                         d_tfs=[dTF])
            ws_["ws"] = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32,
                                    device=dev)
            return b

        key = workload_key(_device_arch(), _d.EMISSION_ABSORPTION, "f16", w.tf.shape[0], W,
                           w.volume.shape[0], "V+TF+step", _d.PASS_FUSED)
        cands = []
        for waves, cap, k, lm, ax in itertools.product((2, 4), (4096, 5120, 6144, 7168),
                                                       (32, 64), (0, 2), (0, 1)):
            cands.append({"waves": waves, "lds_cap": cap, "slab_k": k, "slab_kmax": 256,
                          "cell_acc": 1, "lane_map": lm, "schedule": 0, "slab_axis": ax})
        res = tune(key, make5, lambda b: b.run(_d.PASS_FUSED, scale, loss, workspace=ws_["ws"]),
                   lambda: images, candidates=cands, reps=args.reps, verbose=True)
        print(json.dumps({"key": key, "best": res["tuning"], "ms": res["ms"]}))
        return
    if args.workload == "color":
        w = synth.make_color()
        v32 = torch.from_numpy(np.ascontiguousarray(w.volume)).to(dev)
        vol = torch.empty_like(v32, dtype=torch.bfloat16)
        _d.cast_volume(v32, vol)
        del v32
        W = w.views[0].width
        cams = [_d.camera_from_sphere(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                      math.radians(v.fovy), W, W) for v in w.views]
        nv = len(cams)
        targets = torch.rand((nv, W, W, 4), device=dev,
                             generator=torch.Generator("cuda").manual_seed(1))
        images = torch.empty_like(targets)
        trans = torch.empty((nv, W, W), device=dev)
        dV = torch.zeros(w.volume.shape, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        scale = 1.0 / images.numel()

        def make_c():
            views = [_d.make_view(0, cams[i], w.step_world, images[i], transmittance=trans[i],
                                  target=targets[i]) for i in range(nv)]
            return _d.Batch([vol], None, views, _d.COLOR, d_volumes=[dV])

        key = color_key(_device_arch(), "bf16", W, w.volume.shape[0])
        res = tune(key, make_c, lambda b: b.run(_d.PASS_FUSED, scale, loss), lambda: images,
                   candidates=color_candidates(), reps=args.reps, verbose=True)
        print(json.dumps({"key": key, "best": res["tuning"], "ms": res["ms"]}))
        return
    w = synth.make_c3(args.n, args.views, args.image, args.step_vox)
    W = args.image
    gt = torch.from_numpy(w.target_volume).to(dev)
    vol = torch.empty_like(gt, dtype=torch.bfloat16)
    _d.cast_volume(gt, vol)
    cams = [_d.camera_from_sphere(math.radians(v.yaw), math.radians(v.pitch), v.dist,
                                  math.radians(v.fovy), W, W) for v in w.views]
    nv = len(cams)
    targets = torch.rand((nv, W, W), device=dev, generator=torch.Generator("cuda").manual_seed(1))
    images = torch.empty((nv, W, W), device=dev)
    dV = torch.zeros_like(gt)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    scale = 1.0 / (nv * W * W)

    def make():
        views = [_d.make_view(0, cams[i], w.step_world, images[i], target=targets[i])
                 for i in range(nv)]
        return _d.Batch([vol], None, views, _d.ABSORPTION, d_volumes=[dV])

    key = workload_key(_device_arch(), _d.ABSORPTION, "bf16", 0, W, args.n, "V", _d.PASS_FUSED)
    res = tune(key, make, lambda b: b.run(_d.PASS_FUSED, scale, loss), lambda: images,
               reps=args.reps, verbose=True)
    print(json.dumps({"key": key, "best": res["tuning"], "ms": res["ms"]}))


if __name__ == "__main__":
    main()
