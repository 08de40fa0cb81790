"""Host-side logic of the optimisation drivers (no GPU): the multi-resolution
schedule of Sec. 5.3, the starting poses of Sec. 5.1 and the batched
wrapper's argument checks."""
import math

import pytest


def test_density_schedule_levels_and_step_count():
    from paper_2107_12672_amd import recon
    s = recon.Schedule()                       # 32^3 -> 256^3, 10 per level, 50 at the end
    assert s.levels() == [32, 64, 128, 256]
    assert s.total_steps() == 10 * 3 + 50
    s = recon.Schedule(start=20, final=100, steps_per_level=4, final_steps=7)
    assert s.levels() == [20, 40, 80, 100]     # the last doubling is cut at the final size
    assert s.total_steps() == 4 * 3 + 7
    assert recon.Schedule(start=64, final=64).levels() == [64]


def test_paper_starting_poses_for_viewpoint_selection():
    from paper_2107_12672_amd import viewpoint as vp
    deg = sorted((round(math.degrees(y)), round(math.degrees(p))) for y, p in vp.PAPER_STARTS)
    assert deg == sorted((lon, lat) for lon in (45, 135, 225, 315) for lat in (45, -45))
    s = vp.ViewpointSchedule()
    assert s.iterations == 20
    assert 0.0 < s.pole_margin < 0.5 * math.pi


def test_color_pipeline_schedule_defaults_follow_the_paper():
    from paper_2107_12672_amd import recon
    s = recon.ColorPipelineSchedule()
    assert s.ncand == 256 and s.beta == 1.0 and s.prior == 20.0
    assert s.color_start == 32


def test_batch_wrapper_rejects_bad_arguments_before_any_launch():
    import torch
    from paper_2107_12672_amd import autograd as ag, ddvr as d
    # a CPU grid is refused before any library call
    with pytest.raises(ValueError):
        ag.render_batch(torch.zeros((4, 4, 4)), None, torch.zeros((2, 12)), 0.1, d.ABSORPTION,
                        8, 8)
