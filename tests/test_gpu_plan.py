"""Step plans and graph replay (batched form of one optimisation step; no
paper counterpart).  A plan records forward, loss gradient, adjoint and the
checkpoint fallback of a batch into one HIP graph; its replays must equal the
same passes run eagerly, replay after replay, and a batch that alternates
passes under graph replay must record each pass once."""
import math

import numpy as np
import pytest

import oracle
from harness import Problem, device_volume, gpu_camera
from test_gpu_parity import ea_problem

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _uneven():
    """Three views of two grids (f16 and f32), ragged image sizes, EA."""
    probs = [ea_problem(W=40, H=24, seed=71, storage="f16"),
             ea_problem(W=72, H=56, seed=72, yaw=200.0),
             ea_problem(W=33, H=47, seed=71, yaw=-40.0, pitch=30.0, storage="f16")]
    probs[2].volume = probs[0].volume
    return probs, [0, 1, 0]


def _views(d, torch, probs, vidx, imgs, trs, gs, dcam, dstep):
    return [d.make_view(vidx[k], gpu_camera(p), p.step, imgs[k], transmittance=trs[k],
                        d_image=gs[k], d_camera=dcam[k], d_step=dstep[k:k + 1], tf_index=k)
            for k, p in enumerate(probs)]


def test_entropy_plan_replays_equal_the_eager_step():
    import torch
    from paper_2107_12672_amd import ddvr as d
    probs, vidx = _uneven()
    _say("entropy plan vs eager step")
    vols = [device_volume(probs[0]), device_volume(probs[1])]
    tfs = [torch.from_numpy(p.tf).cuda() for p in probs]
    n = len(probs)

    def buffers():
        imgs = [torch.full((p.H * p.W * 4,), float("nan"), device="cuda") for p in probs]
        trs = [torch.zeros(p.H * p.W, device="cuda") for p in probs]
        gs = [torch.full((p.H * p.W * 4,), 7.0, device="cuda") for p in probs]
        return imgs, trs, gs, torch.zeros((n, 12), device="cuda"), torch.zeros(n, device="cuda")

    # eager: forward, entropy of every image, adjoint
    imgs, trs, gs, dcam, dstep = buffers()
    dvs = [torch.zeros(v.shape, device="cuda") for v in vols]
    b = d.Batch(vols, tfs, _views(d, torch, probs, vidx, imgs, trs, gs, dcam, dstep),
                d.EMISSION_ABSORPTION, d_volumes=dvs)
    ws = torch.zeros(b.workspace_size() // 4 + 1, dtype=torch.int32, device="cuda")
    b.run(d.PASS_FORWARD)
    work = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    oe = torch.zeros(n, dtype=torch.float64, device="cuda")
    for k in range(n):
        gs[k].zero_()
        d.opacity_entropy(imgs[k].view(probs[k].H, probs[k].W, 4), work[k], oe[k:k + 1],
                          gs[k], scale=-0.5)
    b.run(d.PASS_ADJOINT, workspace=ws)
    torch.cuda.synchronize()
    ref = ([t.clone() for t in imgs], [t.clone() for t in gs], dcam.clone(), dstep.clone(),
           [t.clone() for t in dvs], oe.cpu().numpy())
    b.close()

    # the plan, replayed three times with eager work in between
    imgs, trs, gs, dcam, dstep = buffers()
    dvs = [torch.zeros(v.shape, device="cuda") for v in vols]
    b = d.Batch(vols, tfs, _views(d, torch, probs, vidx, imgs, trs, gs, dcam, dstep),
                d.EMISSION_ABSORPTION, d_volumes=dvs)
    ws = torch.zeros(b.workspace_size() // 4 + 1, dtype=torch.int32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan = d.Plan(b, d.PLAN_LOSS_NEG_ENTROPY, 0.5, loss, workspace=ws)
    for rep in range(3):
        dcam.zero_()
        dstep.zero_()
        loss.zero_()
        for t in dvs:
            t.zero_()
        plan.run()
        torch.cuda.synchronize()
        terms = np.array(plan.loss_terms())
        _ = torch.ones(8, device="cuda").sum().item()     # eager work between replays
        for k in range(n):
            assert torch.equal(imgs[k], ref[0][k]), (rep, k)
            # the float64 sums are reduced in another order: the seeds agree to
            # float32 rounding, relative to the image's largest seed
            atol = 1e-6 * float(ref[1][k].abs().max())
            assert torch.allclose(gs[k], ref[1][k], rtol=1e-6, atol=atol), (rep, k)
        assert np.allclose(terms, ref[5], rtol=1e-12, atol=0.0)
        assert abs(float(loss) + 0.5 * ref[5].sum()) <= 1e-12 * abs(ref[5].sum())
        e = float((dcam - ref[2]).norm() / ref[2].norm())
        assert e < 1e-5, (rep, e)
        assert torch.allclose(dstep, ref[3], rtol=1e-5, atol=1e-7 * float(ref[3].abs().max()))
        for j in range(2):
            e = float((dvs[j] - ref[4][j]).norm() / ref[4][j].norm())
            assert e < 1e-5, (rep, j, e)
    # the entropy the plan reports is the one of the image it rendered
    for k, p in enumerate(probs):
        a = imgs[k].view(-1, 4)[:, 3].double().cpu().numpy()
        pk = a / a.sum()
        nz = pk > 0
        oe_np = -(pk[nz] * np.log2(pk[nz])).sum() / math.log2(a.size)
        assert abs(terms[k] - oe_np) <= 1e-9, (k, terms[k], oe_np)
    plan.close()
    b.close()


def test_fused_plan_equals_the_batch_fused_pass():
    import torch
    from paper_2107_12672_amd import ddvr as d
    probs, vidx = _uneven()
    _say("fused plan")
    vols = [device_volume(probs[0]), device_volume(probs[1])]
    tfs = [torch.from_numpy(p.tf).cuda() for p in probs]
    rng = np.random.default_rng(5)
    tg = [torch.from_numpy(rng.uniform(0, 1, p.H * p.W * 4).astype(np.float32)).cuda()
          for p in probs]
    outs = []
    for use_plan in (False, True):
        imgs = [torch.zeros(p.H * p.W * 4, device="cuda") for p in probs]
        trs = [torch.zeros(p.H * p.W, device="cuda") for p in probs]
        dvs = [torch.zeros(v.shape, device="cuda") for v in vols]
        dtfs = [torch.zeros_like(t) for t in tfs]
        views = [d.make_view(vidx[k], gpu_camera(p), p.step, imgs[k], transmittance=trs[k],
                             target=tg[k], tf_index=k) for k, p in enumerate(probs)]
        b = d.Batch(vols, tfs, views, d.EMISSION_ABSORPTION, d_volumes=dvs, d_tfs=dtfs)
        ws = torch.zeros(b.workspace_size() // 4 + 1, dtype=torch.int32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        if use_plan:
            plan = d.Plan(b, d.PLAN_LOSS_FUSED, 0.25, loss, workspace=ws)
            plan.run()
        else:
            b.run(d.PASS_FUSED, 0.25, loss, workspace=ws)
        torch.cuda.synchronize()
        outs.append((imgs, dvs, dtfs, float(loss)))
        if use_plan:
            plan.close()
        b.close()
    (i0, v0, t0, l0), (i1, v1, t1, l1) = outs
    for k in range(3):
        assert torch.equal(i0[k], i1[k])
    for j in range(2):
        assert float((v0[j] - v1[j]).norm() / v0[j].norm()) < 1e-5
    for k in range(3):
        assert torch.allclose(t0[k], t1[k], rtol=1e-5, atol=1e-6 * float(t0[k].abs().max()))
    assert abs(l0 - l1) <= 1e-9 * abs(l0)


def test_alternating_graph_passes_record_each_pass_once():
    """Forward and adjoint alternating under graph replay: one recording per
    pass, results equal to eager launches on every round."""
    import torch
    from paper_2107_12672_amd import ddvr as d
    probs, vidx = _uneven()
    _say("alternating graph passes")
    vols = [device_volume(probs[0]), device_volume(probs[1])]
    tfs = [torch.from_numpy(p.tf).cuda() for p in probs]
    rng = np.random.default_rng(9)
    gs = [torch.from_numpy(rng.normal(size=p.H * p.W * 4).astype(np.float32)).cuda()
          for p in probs]
    res = []
    for graph in (False, True):
        imgs = [torch.zeros(p.H * p.W * 4, device="cuda") for p in probs]
        trs = [torch.zeros(p.H * p.W, device="cuda") for p in probs]
        dcam = torch.zeros((3, 12), device="cuda")
        dvs = [torch.zeros(v.shape, device="cuda") for v in vols]
        views = [d.make_view(vidx[k], gpu_camera(p), p.step, imgs[k], transmittance=trs[k],
                             d_image=gs[k], d_camera=dcam[k], tf_index=k)
                 for k, p in enumerate(probs)]
        b = d.Batch(vols, tfs, views, d.EMISSION_ABSORPTION, d_volumes=dvs)
        ws = torch.zeros(b.workspace_size() // 4 + 1, dtype=torch.int32, device="cuda")
        rounds = []
        for r in range(4):
            dcam.zero_()
            for t in dvs:
                t.zero_()
            b.run(d.PASS_FORWARD, graph=graph)
            b.run(d.PASS_ADJOINT, workspace=ws, graph=graph)
            torch.cuda.synchronize()
            rounds.append(([t.clone() for t in imgs], dcam.clone(), [t.clone() for t in dvs]))
        if graph:
            assert b.graph_builds() == 2, b.graph_builds()
        res.append(rounds)
        b.close()
    for r in range(4):
        (ie, ce, ve), (ig, cg, vg) = res[0][r], res[1][r]
        for k in range(3):
            assert torch.equal(ie[k], ig[k]), (r, k)
        assert float((ce - cg).norm() / ce.norm()) < 1e-5
        for j in range(2):
            assert float((ve[j] - vg[j]).norm() / ve[j].norm()) < 1e-5


def test_autotuner_times_candidates_and_caches_the_fastest(tmp_path):
    """tune() on a small batch: every candidate must render the same images
    (tune() raises past float32 rounding; emission-absorption marches one
    sample at a time, so here they are bitwise equal), the fastest is cached
    under the key, and apply() sets it."""
    import torch
    from paper_2107_12672_amd import autotune
    from paper_2107_12672_amd import ddvr as d
    probs, vidx = _uneven()
    _say("autotune")
    vols = [device_volume(probs[0]), device_volume(probs[1])]
    tfs = [torch.from_numpy(p.tf).cuda() for p in probs]
    flat = torch.zeros(sum(p.H * p.W * 4 for p in probs), device="cuda")
    imgs, off = [], 0
    for p in probs:
        imgs.append(flat[off:off + p.H * p.W * 4])
        off += p.H * p.W * 4

    def make():
        views = [d.make_view(vidx[k], gpu_camera(p), p.step, imgs[k], tf_index=k)
                 for k, p in enumerate(probs)]
        return d.Batch(vols, tfs, views, d.EMISSION_ABSORPTION)

    cands = [dict(d.TUNING_DEFAULT, waves=w, lds_cap=c, lane_map=lm, schedule=2)
             for w, c, lm in ((4, 7168, 2), (2, 4096, 0), (4, 2048, 1))]
    path = str(tmp_path / "cache.json")
    old = d.get_tuning()
    try:
        res = autotune.tune("test|key", make, lambda b: b.run(d.PASS_FORWARD), lambda: flat,
                            candidates=cands, reps=2, path=path)
        assert len(res["all"]) == 3
        assert res["tuning"] in cands
        ref = None
        for c in cands:
            d.set_tuning(**c)
            b = make()
            b.run(d.PASS_FORWARD)
            torch.cuda.synchronize()
            b.close()
            if ref is None:
                ref = flat.clone()
            else:
                assert torch.equal(flat, ref), c
        d.set_tuning(**old)
        entry = autotune.load_cache(path)["test|key"]
        assert entry["tuning"] == res["tuning"] and entry["candidates"] == 3
        assert d.get_tuning() == old            # tune() leaves the tuning as it was
        assert autotune.apply("test|key", path)
        assert d.get_tuning() == res["tuning"]
        assert not autotune.apply("absent|key", path)
    finally:
        d.set_tuning(**old)
