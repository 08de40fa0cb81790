"""Multi-resolution density reconstruction from images (Sec. 5.3), driven
entirely through the library's entry points: every step of the loop runs in
the HIP kernels; this module only sequences the calls.

Per optimiser step, on a batch of views:
  1. one fused launch per batch: forward, L1 image loss of eq. (tf-loss) and
     its upstream gradient, adjoint into the density gradient (batch pass 2,
     ``DDVR_LOSS_L1``, replayed from a HIP graph);
  2. the smoothing prior on the densities in 3D (``ddvr_volume_prior``);
  3. one Adam step on the float32 master grid, clamped to [0, inf), fused with
     the bf16 storage copy the renderer reads and the clearing of the
     gradient (``ddvr_adam_step``).
The grid starts at `start`^3 vertices and doubles its resolution per axis
after `steps_per_level` steps (``ddvr_resample_volume``), up to `final`^3,
where `final_steps` steps are taken.

Readings (the paper is silent): an "iteration" of the schedule is one
optimiser step on one batch (the views are visited in order, batch after
batch); Adam's moments restart at every level; densities are clamped at 0.

`Reconstructor` plans every level's batches and allocates its buffers once;
`run()` then executes the schedule from a zero grid.

`optimize_tf` is the TF reconstruction of Sec. 5.2 through the same entry
points: a fused L1 batch pass into the TF gradient, the TF smoothing prior
and Adam on the table, per step.

`reconstruct_via_color` is the pipeline of Sec. 5.4 for non-monotonic TFs:
colour volume from the images, densities from the colour volume, density
optimisation with the TF.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

from . import ddvr as d


@dataclass
class Schedule:
    start: int = 32
    final: int = 256
    steps_per_level: int = 10
    final_steps: int = 50
    batch: int = 8
    lr: float = 0.3
    prior: float = 0.5
    step_vox: float = 0.2

    def levels(self) -> List[int]:
        out, n = [], self.start
        while n < self.final:
            out.append(n)
            n *= 2
        out.append(self.final)
        return out

    def total_steps(self) -> int:
        return self.steps_per_level * (len(self.levels()) - 1) + self.final_steps


@dataclass
class Result:
    steps: int = 0
    samples: int = 0
    losses: object = None      # [steps] float64 device tensor: L1 + prior of every step
    volume: object = None      # the float32 master grid at the end


class _Level:
    def __init__(self, n, targets, cams, sched, stream):
        import torch
        dev = targets.device
        nview, H, W = targets.shape
        shape = (n, n, n)
        self.n = n
        self.master = torch.zeros(shape, dtype=torch.float32, device=dev)
        self.store = torch.zeros(shape, dtype=torch.bfloat16, device=dev)
        self.grad = torch.zeros_like(self.master)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.images = torch.empty((nview, H, W), device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        step_world = sched.step_vox * 2.0 / (n - 1)
        self.batches = []
        for b0 in range(0, nview, sched.batch):
            idx = range(b0, min(nview, b0 + sched.batch))
            views = [d.make_view(0, cams[i], step_world, self.images[i], target=targets[i])
                     for i in idx]
            b = d.Batch([self.store], None, views, d.ABSORPTION, flags=d.LOSS_L1,
                        d_volumes=[self.grad], stream=stream)
            self.batches.append((b, 1.0 / (len(views) * H * W), b.sample_count()))

    def close(self):
        for b, _, _ in self.batches:
            b.close()


class Reconstructor:
    def __init__(self, targets, cams, sched: Schedule, stream=None):
        """targets: [V][H][W] float32 device tensor of absorption-only images;
        cams: their V cameras."""
        self.sched = sched
        self.stream = stream
        self.levels = [_Level(n, targets, cams, sched, stream) for n in sched.levels()]

    def run(self, on_step=None) -> Result:
        import torch
        sched, s = self.sched, self.stream
        res = Result()
        res.losses = torch.zeros(sched.total_steps(), dtype=torch.float64,
                                 device=self.levels[0].master.device)
        prev = None
        for li, L in enumerate(self.levels):
            if prev is None:
                L.master.zero_()
            else:
                d.resample_volume(prev.master, L.master, s)
            d.cast_volume(L.master, L.store, s)
            L.grad.zero_()
            L.m.zero_()
            L.v.zero_()
            steps = sched.final_steps if L.n == sched.final else sched.steps_per_level
            for t in range(1, steps + 1):
                b, scale, samples = L.batches[(t - 1) % len(L.batches)]
                L.loss.zero_()
                b.run(d.PASS_FUSED, scale, L.loss, graph=True, stream=s)
                d.volume_prior(L.master, sched.prior, L.grad, L.loss, s)
                d.adam_step(L.master, L.grad, L.m, L.v, t, sched.lr, lo=0.0, store=L.store,
                            zero_grad=True, stream=s)
                res.losses[res.steps:res.steps + 1].copy_(L.loss)
                res.samples += samples
                res.steps += 1
                if on_step is not None:
                    on_step(li, t, L.loss)
            prev = L
        res.volume = self.levels[-1].master
        return res

    def close(self):
        for L in self.levels:
            L.close()


def reconstruct(targets, cams, sched: Schedule, stream=None, on_step=None) -> Result:
    """Plan, run the schedule once, release the batches."""
    r = Reconstructor(targets, cams, sched, stream)
    try:
        return r.run(on_step)
    finally:
        r.close()


@dataclass
class TFSchedule:
    """TF reconstruction (Sec. 5.2): L1 image loss plus lambda times the
    smoothing prior of eq. (tf-loss), Adam with lr 0.8, all views in one batch
    per step (an "epoch" of the paper's 8 views)."""
    steps: int = 200
    lr: float = 0.8
    prior: float = 0.4


def optimize_tf(volume, tf0, targets, cams, step_world: float, sched: TFSchedule,
                stream=None):
    """volume: stored grid [nz][ny][nx] (device); tf0: [R][4] float32 start;
    targets: [V][H][W][4] emission-absorption images.  Returns (tf, losses):
    the optimised table (clamped to >= 0) and the loss of every step."""
    import torch
    dev = targets.device
    nview, H, W, _ = targets.shape
    tf = tf0.clone().contiguous()
    grad = torch.zeros_like(tf)
    m = torch.zeros_like(tf)
    v = torch.zeros_like(tf)
    images = torch.empty_like(targets)
    trans = torch.empty((nview, H, W), device=dev)
    views = [d.make_view(0, cams[i], step_world, images[i], transmittance=trans[i],
                         target=targets[i], tf_index=0) for i in range(nview)]
    b = d.Batch([volume], [tf], views, d.EMISSION_ABSORPTION, flags=d.LOSS_L1,
                d_tfs=[grad], stream=stream)
    ws = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32, device=dev)
    losses = torch.zeros(sched.steps, dtype=torch.float64, device=dev)
    try:
        for t in range(1, sched.steps + 1):
            loss = losses[t - 1:t]
            b.run(d.PASS_FUSED, 1.0 / targets.numel(), loss, workspace=ws, stream=stream)
            d.tf_prior(tf, sched.prior, grad, loss, stream)
            d.adam_step(tf, grad, m, v, t, sched.lr, lo=0.0, zero_grad=True, stream=stream)
    finally:
        b.close()
    return tf, losses


@dataclass
class ColorPipelineSchedule:
    """The pipeline of Sec. 5.4: a pre-shaded colour volume reconstructed from
    the images, densities estimated from it through the TF, then the density
    optimisation with the TF from that start."""
    color_start: int = 32      # colour volume: first level's grid edge, doubled per level
    color_steps_per_level: int = 10
    color_steps: int = 50      # at the final level
    color_lr: float = 0.05
    dfc_sweeps: int = 10
    dfc_stop: float = 1e-3     # stop once fewer than this fraction of voxels change
    ncand: int = 256
    beta: float = 1.0
    density_steps: int = 100
    density_lr: float = 0.02
    prior: float = 20.0
    seed: int = 0


@dataclass
class ColorPipelineResult:
    color: object = None           # [n][n][n][4] float32: the reconstructed colour volume
    density_init: object = None    # [n][n][n] float32: the estimate from the colour volume
    density: object = None         # [n][n][n] float32: after the density optimisation
    color_losses: object = None    # [all colour steps] float64 (device)
    density_losses: object = None  # [density_steps] float64 (device): L1 + prior
    sweeps: int = 0


def reconstruct_via_color(targets, cams, tf, n: int, step_world: float,
                          sched: ColorPipelineSchedule = None, stream=None) -> ColorPipelineResult:
    """targets: [V][H][W][4] emission-absorption images of an unknown density
    grid under the known TF `tf` ([R][4] float32, device); cams: their V
    cameras; n: edge of the grid to reconstruct (float32 throughout).

    Readings (the paper is silent): the colour volume follows the
    multi-resolution schedule of the density reconstruction (each channel
    resampled on its own between levels, Adam's moments restarted) with the L1
    loss alone, starting from zero and clamped to [0, inf); the densities are
    clamped to [0, 1], the range the TF covers; the TF stays fixed."""
    import torch
    sched = sched or ColorPipelineSchedule()
    dev = targets.device
    nview, H, W, _ = targets.shape
    scale = 1.0 / targets.numel()
    res = ColorPipelineResult()
    images = torch.empty_like(targets)
    trans = torch.empty((nview, H, W), device=dev)

    def views():
        return [d.make_view(0, cams[i], step_world, images[i], transmittance=trans[i],
                            target=targets[i], tf_index=0) for i in range(nview)]

    # 1. the colour volume from the images, coarse to fine
    levels, m = [], min(sched.color_start, n)
    while m < n:
        levels.append(m)
        m *= 2
    levels.append(n)
    total = sched.color_steps_per_level * (len(levels) - 1) + sched.color_steps
    res.color_losses = torch.zeros(total, dtype=torch.float64, device=dev)
    color, k = None, 0
    for m in levels:
        prev, color = color, torch.zeros((m, m, m, 4), device=dev)
        if prev is not None:
            d.resample_volume(prev, color, stream)
        cg, cm, cv = (torch.zeros_like(color) for _ in range(3))
        b = d.Batch([color], None, views(), d.COLOR, flags=d.LOSS_L1, d_volumes=[cg],
                    stream=stream)
        try:
            for t in range(1, (sched.color_steps if m == n else sched.color_steps_per_level) + 1):
                b.run(d.PASS_FUSED, scale, res.color_losses[k:k + 1], stream=stream)
                d.adam_step(color, cg, cm, cv, t, sched.color_lr, lo=0.0, zero_grad=True,
                            stream=stream)
                k += 1
        finally:
            b.close()
    res.color = color
    del cg, cm, cv, prev

    # 2. densities from the colour volume (Jacobi sweeps, alpha = 1/max tau)
    a = torch.zeros((n, n, n), device=dev)
    bb = torch.zeros_like(a)
    nch = torch.zeros(1, dtype=torch.int32, device=dev)
    alpha = d.density_from_color(color, tf, a, seed=sched.seed, sweep=0, ncand=sched.ncand,
                                 stream=stream)
    cur, nxt = a, bb
    res.sweeps = 1
    for s in range(1, sched.dfc_sweeps):
        nch.zero_()
        d.density_from_color(color, tf, nxt, d_prev=cur, alpha=alpha, beta=sched.beta,
                             seed=sched.seed, sweep=s, ncand=sched.ncand, n_changed=nch,
                             stream=stream)
        cur, nxt = nxt, cur
        res.sweeps += 1
        if int(nch.item()) < sched.dfc_stop * cur.numel():
            break
    res.density_init = cur.clone()

    # 3. the density optimisation with the TF, from that start
    dens = cur
    dg, dm, dv = (torch.zeros_like(dens) for _ in range(3))
    res.density_losses = torch.zeros(sched.density_steps, dtype=torch.float64, device=dev)
    b = d.Batch([dens], [tf], views(), d.EMISSION_ABSORPTION, flags=d.LOSS_L1, d_volumes=[dg],
                stream=stream)
    ws = torch.zeros(max(b.workspace_size(), 4) // 4, dtype=torch.int32, device=dev)
    try:
        for t in range(1, sched.density_steps + 1):
            loss = res.density_losses[t - 1:t]
            b.run(d.PASS_FUSED, scale, loss, workspace=ws, stream=stream)
            d.volume_prior(dens, sched.prior, dg, loss, stream)
            d.adam_step(dens, dg, dm, dv, t, sched.density_lr, lo=0.0, hi=1.0, zero_grad=True,
                        stream=stream)
    finally:
        b.close()
    res.density = dens
    return res
