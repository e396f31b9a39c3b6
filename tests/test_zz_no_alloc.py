"""The allocation-free preconditioner entry point (ga_apply_Pinv_noalloc, for
callers that cannot allocate device memory) against ga_apply_Pinv: two calls in a
row, the second with a smaller input, equal bit for bit (same kernels, no atomics);
sizes beyond the fixed scratch refused; no device memory taken by the calls."""
import sys

import numpy as np
import pytest
import torch

from paper_2102_11536_amd import ga, workloads
from tests.helpers import OracleProblem, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ga.load_library()


def _vec(n, seed):
    return torch.as_tensor(np.random.default_rng(seed).standard_normal(n), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("mode", [ga.GA_PINV_AUTO, ga.GA_PINV_DENSE, ga.GA_PINV_MFMA])
def test_noalloc_equals_pinv_two_calls(mode):
    _say("noalloc mode", mode)
    big = ga.ga_setup_patch(3, (20, 17, 13), 3, workloads.deformed_cube_ctrl((20, 17, 13), 3))
    small = ga.ga_setup_patch(3, 6, 2, workloads.deformed_cube_ctrl(6, 2))
    for pt in (big, small):
        ga.ga_patch_set_pinv(pt, mode)
    calls = [(big, 3, 1), (small, 1, 2)]   # the second call is smaller
    # references (these also build the packed inverses of the matrix-core mode)
    refs = []
    for pt, nr, seed in calls:
        r = _vec(nr * pt.n_free, seed)
        z = torch.empty_like(r)
        ga.ga_apply_Pinv(pt, r, z, nrhs=nr)
        refs.append((r, z))
    # the first call on a device looks up the scratch array's device address (the
    # runtime maps the library's device globals then); the calls measured below
    # must not take any device memory
    w = _vec(small.n_free, 9)
    ga.ga_apply_Pinv_noalloc(small, w, torch.empty_like(w))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    outs = []
    for (pt, nr, _), (r, _) in zip(calls, refs):
        z = torch.full_like(r, np.nan)
        outs.append(z)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for (pt, nr, _), (r, _), z in zip(calls, refs, outs):
        ga.ga_apply_Pinv_noalloc(pt, r, z, nrhs=nr)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    assert free2 == free1, (free0, free1, free2)
    for (r, zref), z in zip(refs, outs):
        assert torch.equal(z, zref)
    # the small patch against the oracle as well
    pr = OracleProblem(3, 6, 2)
    r, _ = refs[1]
    assert rel(outs[1].cpu().numpy(), pr.P.apply(r.cpu().numpy())) < 1e-12
    # in place
    r2 = refs[0][0].clone()
    ga.ga_apply_Pinv_noalloc(big, r2, r2, nrhs=3)
    assert torch.equal(r2, refs[0][1])


def test_noalloc_limits():
    pt = ga.ga_setup_patch(3, 8, 3, workloads.deformed_cube_ctrl(8, 3))
    nr = ga.GA_NOALLOC_MAX_ENTRIES // pt.n_free + 1
    r = torch.zeros(nr * pt.n_free, dtype=torch.float64, device=DEV)
    with pytest.raises(ga.GAError) as e:
        ga.ga_apply_Pinv_noalloc(pt, r, r, nrhs=nr)
    assert e.value.code == ga.GA_EINVAL
    # the largest accepted size
    nr = ga.GA_NOALLOC_MAX_ENTRIES // pt.n_free
    r = _vec(nr * pt.n_free, 5)
    z, zr = torch.empty_like(r), torch.empty_like(r)
    ga.ga_apply_Pinv_noalloc(pt, r, z, nrhs=nr)
    ga.ga_apply_Pinv(pt, r, zr, nrhs=nr)
    assert torch.equal(z, zr)
    # the matrix-core mode before its data exist is refused, afterwards accepted
    pt2 = ga.ga_setup_patch(3, 5, 3, workloads.deformed_cube_ctrl(5, 3))
    ga.ga_patch_set_pinv(pt2, ga.GA_PINV_MFMA)
    r = _vec(pt2.n_free, 6)
    z = torch.empty_like(r)
    with pytest.raises(ga.GAError) as e:
        ga.ga_apply_Pinv_noalloc(pt2, r, z)
    assert e.value.code == ga.GA_EINVAL
    ga.ga_apply_Pinv(pt2, r, z)
    z2 = torch.empty_like(r)
    ga.ga_apply_Pinv_noalloc(pt2, r, z2)
    assert torch.equal(z, z2)
