"""The allocation-free forward entry (ur_simulate_noalloc) against the
ordinary one (ur_simulate), through the C ABI.

Its scratch is one static device array shared by every call on the device,
so the calls below run back to back on the same array: a 256^3 FP32 box
(the largest the array holds) and then a smaller 64^3 box, whose call finds
the first call's contents in the array.  Counts bit-exact; sums, means,
SEMs and totals within 1e-12 relative (the same kernels; the in-block bin
sums are FP64 LDS atomics whose order varies between runs).
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ur():
    import torch
    import paper_2303_13435_amd as ur
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ur


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _same(got, ref, what):
    assert np.array_equal(got["count"], ref["count"]), f"{what}: counts differ"
    pop = ref["count"] > 0
    for k in ("sum", "sumsq", "mean"):
        a, b = got[k][pop], ref[k][pop]
        assert np.all(np.abs(a - b) <= 1e-12 * np.abs(b)), (what, k, float(np.max(np.abs(a - b) / np.abs(b))))
    multi = ref["count"] > 1
    assert np.all(np.abs(got["sem"][multi] - ref["sem"][multi]) <= 1e-12 * np.abs(ref["sem"][multi])), what
    assert np.all(np.isnan(got["mean"][~pop])), what
    for i in (0, 1, 3):
        assert abs(got["totals"][i] - ref["totals"][i]) <= 1e-12 * abs(ref["totals"][i]), (what, i)


def _reference(ur, wl, prec):
    import torch
    plan = ur.Plan(wl.n, wl.voxel, prec)
    plan.set_bins(wl.edges)
    h = ur.Hist(wl.nbins)
    plan.simulate(ur.DeviceCell.from_host(wl.cell), wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    return h.numpy()


def test_noalloc_matches_simulate_two_calls(ur):
    import torch
    cases = [(W.c4(), 0), (W.small(64, c=8, n_atoms=10, seed=7, radius=25.0, nbins=64), 0),
             (W.small(128, c=16, n_atoms=20, seed=8, radius=50.0, nbins=128, prec=1), 1)]
    for wl, prec in cases:
        _say(f"noalloc {wl.n}^3 prec={prec}")
        ref = _reference(ur, wl, prec)
        plan = ur.Plan(wl.n, wl.voxel, prec, workspace=False)      # no workspace attached
        plan.set_bins(wl.edges)
        h = ur.Hist(wl.nbins)
        plan.simulate_noalloc(ur.DeviceCell.from_host(wl.cell), wl.mask, wl.zoom, h)
        torch.cuda.synchronize()
        _same(h.numpy(), ref, f"{wl.n}^3")


def test_noalloc_refuses_boxes_beyond_the_scratch(ur):
    import torch
    wl = W.c2()                                                   # 512^3 FP32: beyond the limit
    plan = ur.Plan(wl.n, wl.voxel, 0, workspace=False)
    plan.set_bins(wl.edges)
    h = ur.Hist(wl.nbins)
    h.sum.fill_(-7.0)
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.simulate_noalloc(ur.DeviceCell.from_host(wl.cell), wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    assert float(h.sum[0].item()) == -7.0                          # nothing was enqueued


def test_noalloc_recorded_without_an_eager_call(ur):
    """Captured into a HIP graph on a plan that never ran eagerly (nothing to
    allocate); every replay, with eager work in between, equals ur_simulate."""
    import torch
    wl = W.small(64, c=8, n_atoms=10, seed=11, radius=27.0, nbins=64)
    ref = _reference(ur, wl, 0)
    plan = ur.Plan(wl.n, wl.voxel, 0, workspace=False)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = ur.Graph(s)
    with torch.cuda.stream(s):
        with g:
            plan.simulate_noalloc(cell, wl.mask, wl.zoom, h, stream=s)
    for rep in range(3):
        h.sum.fill_(-1.0)
        h.mean.fill_(-1.0)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        _same(h.numpy(), ref, f"replay {rep}")
    ur.lib().ur_graph_destroy(g.h)
    g.h = None
