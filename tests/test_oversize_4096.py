"""4096^3 boxes through the out-of-core forward path (the 2D + 1D split of
eq. 2): the density lives in host memory, only its planes are copied,
and the spectrum kept in HBM covers just those planes.

Neither the oracle transform nor its n^3 binning loop fits this size, so the
expected values come from the oracle's O12 functions (per-bin counts taken
axis by axis; the closed form of a two-voxel density) and from direct
summation over the nonzero voxels of a sparse density (eq. 1 at every lattice
point of the low-|Q| bins), all pinned against the n^3 loops and
numpy.fft.fftn at small n in test_oracle_pins.py.  The last test streams the
out-of-core workload itself (truncated octahedron R = 1900, 128-voxel cell of
200 atoms, 2048 log bins): exact counts, Parseval and F(0) against the
oracle's voxel-by-voxel density moments.
"""
import sys

import numpy as np
import pytest

import workloads as W

N = 4096


@pytest.fixture(scope="module")
def ur():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2303_13435_amd as ur
    ur.lib()
    return ur


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="module")
def edges():
    return W.c5(N).edges


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _stream(ur, host, x_lo, x_hi, edges, budget=0, vform=False):
    import torch
    plan = ur.Plan(N, 1.0, ur.UR_F32)
    plan.set_hbm_budget(budget)
    plan.set_voxel_form(vform)
    plan.set_bins(edges)
    h = ur.Hist(len(edges) - 1)
    nbytes = plan.simulate_host(host, x_lo, x_hi, h)
    torch.cuda.synchronize()
    single = (x_hi - x_lo + 1) * N * N * 4
    _say(f"  {nbytes // single} pass(es) over the planes")
    assert nbytes % single == 0 and (nbytes == single) == (budget == 0)
    del plan
    torch.cuda.empty_cache()
    return h.numpy()


def _check_totals(got, s1, s2):
    n3 = float(N) ** 3
    assert abs(got["totals"][0] - s2 / n3) <= 1e-6 * s2 / n3        # Parseval
    assert abs(got["totals"][1] - s1 / n3) <= 1e-6 * s1 / n3        # Re F(0)
    assert abs(got["totals"][2]) <= 1e-6 * s1 / n3                  # Im F(0)
    assert abs(got["totals"][3] - s2) <= 1e-6 * s2                  # sum of rho^2 streamed


@pytest.mark.gpu
def test_in_hbm_calls_refused(ur, edges):
    """A 4096^3 plan runs only the out-of-core path: the in-HBM forward call
    and the adjoint fail with UR_ERR_UNSUPPORTED before any launch."""
    import torch
    wl = W.c5(N)
    plan = ur.Plan(N, 1.0, ur.UR_F32)
    plan.set_bins(edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(len(edges) - 1)
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.simulate(cell, wl.mask, wl.zoom, h)
    g = torch.zeros(len(edges) - 1, dtype=torch.float64, device="cuda")
    ga = torch.zeros(wl.cell.n_atoms, dtype=torch.float64, device="cuda")
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.adjoint(h, g, cell=cell, mask=wl.mask, grad_amp=ga)
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.workspace_size()
    torch.cuda.synchronize()


@pytest.mark.gpu
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_two_voxels_every_bin(ur, orc, edges, axis):
    """rho = 1 at p and 1/2 at p + 5 e_axis: every one of the 2048 bins
    against the closed form (counts bit-exact, means 1e-5 relative); the
    phase 5 t / 4096 takes every value, so a wrong twiddle, index or unpack
    along that axis shows in some bin."""
    import torch
    d, r1, r2 = 5, 1.0, 0.5
    p = np.array([1000, 1234, 2345])
    q = p.copy()
    q[axis] += d
    x_lo, x_hi = int(p[0]), int(q[0])
    _say(f"4096^3 two voxels along axis {axis}, planes [{x_lo}, {x_hi}]")
    host = torch.zeros((x_hi - x_lo + 1, N, N), dtype=torch.float32, pin_memory=True)
    host[p[0] - x_lo, p[1], p[2]] = r1
    host[q[0] - x_lo, q[1], q[2]] = r2
    got = _stream(ur, host, x_lo, x_hi, edges)
    cnt, s = orc.axis_pair_bins(N, 1.0, edges, d, r1, r2)
    assert np.array_equal(got["count"], cnt)
    pop = cnt > 0
    ref = s[pop] / cnt[pop]
    rel = np.abs(got["mean"][pop] - ref) / ref
    _say(f"  {pop.sum()} bins, max rel err {rel.max():.3e}")
    assert rel.max() <= 1e-5
    _check_totals(got, r1 + r2, r1 * r1 + r2 * r2)


@pytest.mark.gpu
@pytest.mark.parametrize("budget,vform", [(0, False), (16 * 10 ** 9, False), (0, True)])
def test_uniform_cube_every_bin(ur, orc, edges, budget, vform):
    """A dense density at 4096^3: a uniform cube of half-width 300 (601
    planes, 37.6 GiB of pageable host memory, generated on the device),
    every one of the 2048 bins against the factorised closed form of eq. 1
    (O13): counts bit-exact, means within 1e-5 or the FP32 transform's
    norm-wise error bound where a bin's mean lies far below the box mean.
    With a 16 GB HBM budget (the x range of the spectrum takes 40.8 GB) the
    second stage runs in three kz passes; with the voxel form factor the
    reference is the continuous cube (O13 with O15)."""
    import math
    import torch
    hw = 300
    wl = W.uniform_cube(N, hw, 2048)
    x_lo, x_hi = N // 2 - hw, N // 2 + hw
    _say(f"4096^3 uniform cube, planes [{x_lo}, {x_hi}]")
    plan = ur.Plan(N, 1.0, ur.UR_F32)
    plan.set_bins(edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    host = torch.empty((x_hi - x_lo + 1, N, N), dtype=torch.float32)
    for a in range(x_lo, x_hi + 1, 64):
        b = min(a + 63, x_hi)
        host[a - x_lo:b - x_lo + 1].copy_(plan.rho_generate(cell, wl.mask, wl.zoom, x_lo=a, x_hi=b))
    torch.cuda.synchronize()
    del plan
    torch.cuda.empty_cache()
    got = _stream(ur, host, x_lo, x_hi, edges, budget, vform)
    del host
    cnt, s = orc.cube_bins(N, 1.0, edges, hw, 1.0, voxel_form_factor=vform)
    assert np.array_equal(got["count"], cnt)
    pop = cnt > 0
    ref = s[pop] / cnt[pop]
    w3 = float(2 * hw + 1) ** 3
    ibar = w3 / float(N) ** 6
    rel = np.abs(got["mean"][pop] - ref) / ref
    # norm-wise FFT rounding error, systematic over a shell for a cube (see
    # bin_bound in test_gpu_path.py)
    bound = np.maximum(1e-5, 8.0 * 2.0 ** -24 * math.sqrt(36.0) * np.sqrt(ibar / ref))
    _say(f"  {pop.sum()} bins, max rel err {rel.max():.3e}, max err/bound {np.max(rel / bound):.3f}, "
         f"bins above 1e-5: {int(np.sum(rel > 1e-5))}")
    assert np.all(rel <= bound)
    if not vform:
        _check_totals(got, w3, w3)


@pytest.mark.gpu
def test_sparse_slab_low_bins(ur, orc, edges):
    """48 random voxels in 16 planes (any y, z): every populated bin below
    n2 = 49^2 (mixing all three axes) against direct
    summation of eq. 1, plus the counts of all bins, Parseval and F(0)."""
    import torch
    x_lo, x_hi = 2040, 2055
    xyz, val = W.sparse_slab(4096, N, x_lo, x_hi - x_lo + 1, 48)
    _say("4096^3 sparse slab, planes [2040, 2055]")
    host = torch.zeros((x_hi - x_lo + 1, N, N), dtype=torch.float32, pin_memory=True)
    v64 = val.astype(np.float64)
    for (x, y, z), v in zip(xyz, val):
        host[x - x_lo, y, z] = float(v)
    got = _stream(ur, host, x_lo, x_hi, edges)
    cnt, _ = orc.axis_pair_bins(N, 1.0, edges, 1, 1.0, 0.0)
    assert np.array_equal(got["count"], cnt)
    bins, c_low, _, mean = orc.sparse_low_bins(N, 1.0, edges, xyz, v64, 49 * 49)
    assert np.array_equal(got["count"][bins], c_low)
    bins, mean = bins[c_low > 0], mean[c_low > 0]
    assert len(bins) > 100
    rel = np.abs(got["mean"][bins] - mean) / mean
    _say(f"  {len(bins)} low bins, max rel err {rel.max():.3e}")
    assert rel.max() <= 1e-5
    _check_totals(got, float(v64.sum()), float(np.sum(v64 * v64)))


@pytest.mark.gpu
def test_out_of_core_workload_4096(ur, orc):
    """The out-of-core workload at its own size: 3399 planes (212 GiB of
    pageable host memory, more than the page-locked memory a process may
    hold here, so the copies go through the plan's pinned bounce slabs)
    generated on the device chunk by chunk, streamed, a 229 GB spectrum in
    HBM; counts of all 2048 bins bit-exact, Parseval and F(0) against the
    oracle's density moments (voxel by voxel)."""
    import torch
    wl = W.c5(N)
    hw = int(wl.mask.p0)
    x_lo, x_hi = N // 2 - hw, N // 2 + hw
    _say(f"4096^3 out-of-core workload, planes [{x_lo}, {x_hi}]")
    host = torch.empty((x_hi - x_lo + 1, N, N), dtype=torch.float32)
    plan = ur.Plan(N, wl.voxel, ur.UR_F32)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    for a in range(x_lo, x_hi + 1, 64):
        b = min(a + 63, x_hi)
        host[a - x_lo:b - x_lo + 1].copy_(plan.rho_generate(cell, wl.mask, wl.zoom, x_lo=a, x_hi=b))
        if (a - x_lo) % 1024 == 0:
            _say(f"  planes {a}..{b} filled")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    _say("  host density filled")
    h = ur.Hist(wl.nbins)
    nbytes = plan.simulate_host(host, x_lo, x_hi, h)
    torch.cuda.synchronize()
    got = h.numpy()
    del plan, host
    torch.cuda.empty_cache()
    assert nbytes == (x_hi - x_lo + 1) * N * N * 4
    _say("  streamed; oracle counts and moments")
    cnt, _ = orc.axis_pair_bins(N, 1.0, wl.edges, 1, 1.0, 0.0)
    assert np.array_equal(got["count"], cnt)
    s1, s2 = orc.density_moments(wl, orc.cell_synth(wl.cell))
    _check_totals(got, s1, s2)
    pop = cnt > 0
    assert np.all(np.isfinite(got["mean"][pop])) and np.all(got["mean"][pop] > 0)
