"""Launch timing by kind (ga_profile mask) through the C ABI."""
import pytest
import torch

from paper_2102_11536_amd import ga, workloads

pytestmark = pytest.mark.gpu


def test_profile_times_only_the_selected_kinds():
    n, p = 6, 3
    pt = ga.ga_setup_patch(3, n, p, workloads.deformed_cube_ctrl(n, p))
    x = torch.as_tensor(workloads.grf(n, p, seed=5), device="cuda:0")
    y = torch.empty_like(x)
    ga.ga_profile(True, kinds=[ga.PROF_STIFF])
    ga.ga_apply_MK(pt, "M", x, y)
    ga.ga_apply_MK(pt, "K", x, y)
    ga.ga_apply_MK(pt, "K", x, y)
    ga.ga_apply_Pinv(pt, x, y)
    counts = {kd: ga.ga_profile_query(kd)[1] for kd in (ga.PROF_MASS, ga.PROF_STIFF, ga.PROF_PINV)}
    assert counts == {ga.PROF_MASS: 0, ga.PROF_STIFF: 2, ga.PROF_PINV: 0}
    assert ga.ga_profile_query(ga.PROF_STIFF)[0] > 0.0
    ga.ga_profile(True)                       # every kind, totals cleared
    ga.ga_apply_MK(pt, "M", x, y)
    ga.ga_apply_Pinv(pt, x, y)
    counts = {kd: ga.ga_profile_query(kd)[1] for kd in (ga.PROF_MASS, ga.PROF_STIFF, ga.PROF_PINV)}
    assert counts == {ga.PROF_MASS: 1, ga.PROF_STIFF: 0, ga.PROF_PINV: 1}
    ga.ga_profile(False)
    ga.ga_apply_MK(pt, "M", x, y)
    assert ga.ga_profile_query(ga.PROF_MASS)[1] == 0
    torch.cuda.synchronize()
