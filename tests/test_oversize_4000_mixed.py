"""The paper's ED-1 edge, 4000 = 2^5 5^3, through the out-of-core path of a
real mixed-radix plan: slabs of planes from host memory transformed along z
(radices 16, 2, 5, 5, 5; 80 elements per lane, one wavefront per line) and y
into a half spectrum of only the density's planes, then the x pass with the
other planes read as zero.

As at 4096^3, the oracle's transform and n^3 binning do not fit this size:
the expected values come from the oracle's O12 functions (per-bin counts
axis by axis; the closed form of a two-voxel density) and from direct
summation of eq. 1 over the nonzero voxels of a sparse density, all pinned
against the n^3 loops and numpy.fft at small n in test_oracle_pins.py.
"""
import sys

import numpy as np
import pytest

import workloads as W

N = 4000


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


def _stream(ur, host, x_lo, x_hi, edges):
    import torch
    plan = ur.Plan(N, 1.0, ur.UR_F32)
    plan.set_bins(edges)
    h = ur.Hist(len(edges) - 1)
    nbytes = plan.simulate_host(host, x_lo, x_hi, h)
    torch.cuda.synchronize()
    assert nbytes == (x_hi - x_lo + 1) * N * N * 4
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
def test_refusals_at_4000(ur):
    """Edges above 2048 run FP32 real plans only; the in-HBM forward path
    would need the whole 256 GB half spectrum and is left to the caller's
    memory; complex and FP64 plans are refused at creation."""
    with pytest.raises(ur.UltimaError, match="status 2"):
        ur.Plan(N, 1.0, ur.UR_F64)
    with pytest.raises(ur.UltimaError, match="status 2"):
        ur.Plan(N, 1.0, ur.UR_F32, c2c=True)


@pytest.mark.gpu
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_two_voxels_every_bin_4000(ur, orc, edges, axis):
    """rho = 1 at p and 1/2 at p + 5 e_axis: every one of the 2048 bins
    against the closed form (counts bit-exact, means 1e-5 relative); the
    phase 5 t / 4000 takes every value, so a wrong twiddle, index or unpack
    along that axis, radix 16, 2 or 5, shows in some bin."""
    import torch
    d, r1, r2 = 5, 1.0, 0.5
    p = np.array([1001, 1234, 2345])
    q = p.copy()
    q[axis] += d
    x_lo, x_hi = int(p[0]), int(q[0])
    _say(f"4000^3 mixed, two voxels along axis {axis}, planes [{x_lo}, {x_hi}]")
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
def test_sparse_slab_low_bins_4000(ur, orc, edges):
    """48 random voxels in 13 planes that start off a slab boundary: every
    populated bin below n2 = 49^2 (mixing all three axes) against direct
    summation of eq. 1, the counts of all bins, Parseval and F(0)."""
    import torch
    x_lo, x_hi = 1995, 2007
    xyz, val = W.sparse_slab(4000, N, x_lo, x_hi - x_lo + 1, 48)
    _say(f"4000^3 mixed, sparse slab, planes [{x_lo}, {x_hi}]")
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
