"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (stated per comparison):
* bin assignment and voxel counts: bit-exact (integer thresholds on n2);
* FP64 path: bin means within 1e-12 relative; spectra within 1e-12 of max|F|;
* FP32 path: bin means within 1e-5 relative; spectra within 2e-6 of max|F|
  (single-precision butterflies, error ~ eps32 * sqrt(log2 n^3) in norm).
"""
import math
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

F32_BIN = 1e-5
F64_BIN = 1e-12


@pytest.fixture(scope="module")
def ur():
    import torch
    import paper_2303_13435_amd as ur
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ur


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_simulate(ur, wl, prec=None):
    import torch
    p = wl.prec if prec is None else prec
    plan = ur.Plan(wl.n, wl.voxel, p, c2c=(wl.transform == "c2c"))
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    return h.numpy()


def compare_bins(got, ref, tol, what="", n=None):
    """Counts bit-exact; means within `tol` relative.  Bins whose exact mean
    sits at the rounding level of the transform (e.g. exact zeros off the
    Bragg comb of an unmasked lattice) are compared against an absolute floor
    floor = (8 eps)^2 * Ibar, Ibar = mean intensity over the box, eps the unit
    roundoff of the precision the GPU path ran in."""
    assert np.array_equal(got["count"], ref["count"]), f"{what}: counts differ"
    pop = ref["count"] > 0
    m_ref = ref["mean"][pop]
    m_got = got["mean"][pop]
    eps = 6e-8 if tol >= 1e-6 else 1.2e-16
    nvox = float(n) ** 3 if n is not None else float(np.sum(ref["count"]))
    ibar = ref["totals"][0] / nvox
    floor = (8.0 * eps) ** 2 * ibar
    err = np.abs(m_got - m_ref)
    den = np.maximum(np.abs(m_ref), floor)
    rel = np.where(den > 0, err / np.where(den > 0, den, 1.0), 0.0)
    worst = int(np.argmax(rel)) if rel.size else 0
    _say(f"  {what}: {pop.sum()} bins, max rel err {rel.max() if rel.size else 0:.3e}")
    assert rel.size == 0 or rel.max() <= tol, f"{what}: max rel err {rel.max():.3e} at bin {np.flatnonzero(pop)[worst]}"
    # empty bins: NaN mean (both sides)
    assert np.all(np.isnan(got["mean"][~pop])), f"{what}: empty bins must have a NaN mean"
    # SEM of the kernel (one pass over pooled sums) against the oracle's
    # two-pass SEM: relative bound, plus a floor for bins whose intensities
    # are (nearly) equal, where the one-pass difference sumsq - sum*mean is
    # at its rounding level: sqrt(eps * (mean^2 + var)) / sqrt(count)
    c = ref["count"][pop]
    multi = c > 1
    s_ref, s_got = ref["sem"][pop][multi], got["sem"][pop][multi]
    t_rel, t_abs = (1e-5, 1e-5) if tol >= 1e-6 else (1e-9, 3e-8)
    bound = t_rel * s_ref + (t_abs * np.abs(m_ref[multi]) + floor) / np.sqrt(c[multi])
    serr = np.abs(s_got - s_ref)
    assert np.all(serr <= bound), f"{what}: SEM error {np.max(serr / bound):.3g} x bound"
    assert np.all(np.isnan(got["sem"][pop][~multi])), f"{what}: one-voxel bins must have a NaN SEM"
    return rel


# ---------------------------------------------------------------------------
# transform alone
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 32, 64, 128])
@pytest.mark.parametrize("prec", [0, 1])
def test_fft3d_r2c_forward_and_inverse(ur, orc, n, prec):
    import torch
    _say(f"fft3d r2c n={n} prec={prec}")
    rho = W.random_density(1000 + n, n)
    F = orc.forward(rho)                        # eq. 1, full spectrum [u][v][w]
    ref = F[:, :, : n // 2 + 1].transpose(2, 1, 0)
    plan = ur.Plan(n, 1.0, prec)
    dt = torch.float32 if prec == 0 else torch.float64
    x = torch.as_tensor(rho, dtype=dt, device="cuda").contiguous()
    out = plan.fft3d(x)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"  spectrum rel err {err:.3e}")
    assert err <= (2e-6 if prec == 0 else 1e-13)
    back = plan.fft3d(out, direction=+1)
    torch.cuda.synchronize()
    err2 = np.max(np.abs(back.cpu().numpy() - rho)) / np.max(np.abs(rho))
    assert err2 <= (2e-6 if prec == 0 else 1e-13)


def test_fft3d_r2c_2048_sampled(ur, orc):
    """The 2048-point transform (columns over two wavefronts) at full size:
    a 2048^3 FP32 box that is zero except at 64 random voxels, so that every
    coefficient is a sum of 64 plane waves; 516 coefficients (random, plus
    the corners) against eq. 1 by direct summation.  FP32 bound as for the
    small boxes: 2e-6 of max|F|."""
    import torch
    n = 2048
    _say("fft3d r2c n=2048 sampled")
    xyz, val = W.sparse_voxels(2048, n, 64, dtype=np.float32)
    x = torch.zeros((n, n, n), dtype=torch.float32, device="cuda")
    x[torch.as_tensor(xyz[:, 0], device="cuda"), torch.as_tensor(xyz[:, 1], device="cuda"),
      torch.as_tensor(xyz[:, 2], device="cuda")] = torch.as_tensor(val, device="cuda")
    plan = ur.Plan(n, 1.0, 0)
    out = plan.fft3d(x)                                        # [kz][ky][kx]
    del x
    uvw = W.random_frequencies(2049, n, 512)                   # (kx, ky, kz), kz <= n/2
    idx = torch.as_tensor(uvw, device="cuda")
    got = out[idx[:, 2], idx[:, 1], idx[:, 0]].cpu().numpy().astype(np.complex128)
    del out, plan
    torch.cuda.empty_cache()
    ref = orc.dft_points(n, xyz, val.astype(np.float64), uvw)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"  2048 sampled rel err {err:.3e}")
    assert err <= 2e-6


@pytest.mark.parametrize("n", [16, 64])
@pytest.mark.parametrize("prec", [0, 1])
def test_fft3d_c2c(ur, orc, n, prec):
    import torch
    rng = np.random.default_rng(n)
    z = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    F = orc.fft3d(z, -1) / n ** 3
    plan = ur.Plan(n, 1.0, prec, c2c=True)
    dt = torch.complex64 if prec == 0 else torch.complex128
    out = plan.fft3d(torch.as_tensor(z, dtype=dt, device="cuda").contiguous())
    torch.cuda.synchronize()
    err = np.max(np.abs(out.cpu().numpy() - F.transpose(2, 1, 0))) / np.max(np.abs(F))
    assert err <= (2e-6 if prec == 0 else 1e-13)
    back = plan.fft3d(out, direction=+1)
    torch.cuda.synchronize()
    assert np.max(np.abs(back.cpu().numpy() - z)) / np.max(np.abs(z)) <= (2e-6 if prec == 0 else 1e-13)


# ---------------------------------------------------------------------------
# fused forward path
# ---------------------------------------------------------------------------

SMALL_CASES = [
    # (name, workload factory)
    ("sphere64", lambda p: W.small(64, c=8, n_atoms=10, seed=7, radius=25.0, nbins=64, prec=p)),
    ("sphere32_ragged", lambda p: W.small(32, c=4, n_atoms=3, seed=8, radius=11.3, nbins=40, prec=p)),
    ("cube64", lambda p: W.small(64, c=8, n_atoms=5, seed=9, mask=W.cube(17), nbins=64, prec=p)),
    ("troct64", lambda p: W.small(64, c=16, n_atoms=20, seed=10, mask=W.trunc_oct(27.0), nbins=64, prec=p)),
    ("nomask32", lambda p: W.small(32, c=8, n_atoms=4, seed=12, mask=W.no_mask(), nbins=30, prec=p)),
    ("sphere128", lambda p: W.small(128, c=16, n_atoms=40, seed=13, radius=50.0, nbins=128, prec=p)),
    ("tiny16", lambda p: W.small(16, c=4, n_atoms=2, seed=14, radius=5.0, nbins=10, prec=p)),
]


@pytest.mark.parametrize("name,factory", SMALL_CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_simulate_small(ur, orc, name, factory, prec):
    wl = factory(prec)
    _say(f"simulate {name} prec={prec}")
    ref = orc.simulate(wl)
    got = run_simulate(ur, wl)
    compare_bins(got, ref, F32_BIN if prec == 0 else F64_BIN, name, n=wl.n)
    tol = 1e-6 if prec == 0 else 1e-12
    assert abs(got["totals"][0] - ref["totals"][0]) <= tol * ref["totals"][0]          # sum of all I
    assert abs(got["totals"][1] - ref["totals"][1]) <= tol * abs(ref["totals"][1])     # Re F(0)
    assert abs(got["totals"][3] - ref["rho_sumsq"]) <= tol * ref["rho_sumsq"]          # sum rho^2
    # Parseval on the GPU result alone
    assert abs(got["totals"][0] - got["totals"][3] / wl.n ** 3) <= (1e-6 if prec == 0 else 1e-12) * got["totals"][0]


def test_c1_full_complex_fp64(ur, orc):
    wl = W.c1()
    _say("C1 64^3 FP64 c2c")
    ref = orc.simulate(wl)
    got = run_simulate(ur, wl)
    compare_bins(got, ref, F64_BIN, "C1", n=wl.n)


def test_empty_particle(ur, orc):
    wl = W.small(32, c=4, n_atoms=2, mask=W.Mask(W.MASK_SPHERE, -1), nbins=20)
    got = run_simulate(ur, wl)
    ref = orc.simulate(wl)
    assert np.array_equal(got["count"], ref["count"])
    assert np.all(got["sum"] == 0.0) and got["totals"][0] == 0.0


@pytest.mark.parametrize("f,n,n1", [(2, 32, 32), (4, 32, 64), (8, 32, 128), (4, 64, 64)])
def test_simulate_zoom_levels(ur, orc, f, n, n1):
    """ED-2/ED-3 style levels: block sums of a larger ED-1 centred in a box."""
    cell = W.draw_atoms(21, 12, 16 if f <= 4 else 8)
    wl = W.Workload(f"zoom{f}", n, float(f), W.PREC_F64, "r2c", cell, W.sphere(0.42 * n1), W.Zoom(n1, f),
                    W.default_log_edges(n, float(f), 48))
    _say(f"zoom f={f} n={n} n1={n1}")
    ref = orc.simulate(wl)
    got = run_simulate(ur, wl)
    compare_bins(got, ref, F64_BIN, f"zoom f={f}", n=n)
    assert abs(got["totals"][3] - ref["rho_sumsq"]) <= 1e-12 * ref["rho_sumsq"]
    got32 = run_simulate(ur, wl, prec=0)
    compare_bins(got32, ref, F32_BIN, f"zoom f={f} fp32", n=n)


def test_simulate_rho_and_intensity_bin(ur, orc):
    import torch
    wl = W.small(64, c=8, n_atoms=9, seed=31, radius=22.0, nbins=50, prec=1)
    ref = orc.simulate(wl, return_fields=True)
    plan = ur.Plan(wl.n, wl.voxel, 1)
    plan.set_bins(wl.edges)
    rho = torch.as_tensor(ref["rho"], device="cuda").contiguous()
    h = ur.Hist(wl.nbins)
    plan.simulate_rho(rho, h)
    torch.cuda.synchronize()
    compare_bins(h.numpy(), ref, F64_BIN, "simulate_rho", n=wl.n)
    spec = torch.as_tensor(np.ascontiguousarray(ref["F"][:, :, : wl.n // 2 + 1].transpose(2, 1, 0)), device="cuda")
    h2 = ur.Hist(wl.nbins)
    plan.intensity_bin(spec, h2)
    torch.cuda.synchronize()
    compare_bins(h2.numpy(), ref, F64_BIN, "intensity_bin", n=wl.n)


def test_rho_generate_matches_oracle_density(ur, orc):
    import torch
    for (n, f, n1) in [(64, 1, 64), (32, 4, 64)]:
        cell = W.draw_atoms(41, 7, 8)
        wl = W.Workload("g", n, 1.0, 1, "r2c", cell, W.trunc_oct(0.4 * n1), W.Zoom(n1, f), W.default_log_edges(n, 1.0, 8))
        ref = orc.density(wl)
        plan = ur.Plan(n, 1.0, 1)
        got = plan.rho_generate(ur.DeviceCell.from_host(cell), wl.mask, wl.zoom)
        torch.cuda.synchronize()
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
        cg = plan.cell_synth(ur.DeviceCell.from_host(cell))
        torch.cuda.synchronize()
        assert np.max(np.abs(cg.cpu().numpy() - orc.cell_synth(cell))) <= 1e-14 * np.max(orc.cell_synth(cell))


@pytest.mark.parametrize("prec", [0, 1])
def test_c4_size_256(ur, orc, prec):
    wl = W.c4()
    if prec == 1:
        wl = W.Workload(wl.name, wl.n, wl.voxel, 1, wl.transform, wl.cell, wl.mask, wl.zoom, wl.edges)
    _say(f"C4 256^3 prec={prec}")
    ref = orc.simulate(wl)
    got = run_simulate(ur, wl)
    compare_bins(got, ref, F32_BIN if prec == 0 else F64_BIN, "C4", n=wl.n)


# ---------------------------------------------------------------------------
# rotated lattice (cell sampled at u = R d, trilinear, periodic)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,prec,interp,c", [(64, 0, 1, 8), (64, 1, 1, 8), (128, 0, 1, 8), (64, 0, 3, 8), (64, 1, 3, 8),
                                              (128, 0, 3, 8), (64, 1, 1, 32), (64, 0, 3, 32)])
def test_rotated_lattice(ur, orc, n, prec, interp, c):
    """A lattice oriented by a general rotation, the cell sampled trilinearly
    or by the cubic B-spline (cells of 8^3, read from LDS, and of 32^3, read
    through the caches): the fused forward path against the whole
    oracle (O2r, then O4-O8), the generated density voxel by voxel (the
    cubic case's spline coefficients, stored in the working precision, are
    up to 2.4 times the cell's largest value here: same bounds); amplitude
    gradients of the 32^3 cell are refused (cell edges up to 16)."""
    import torch
    from dataclasses import replace
    base = W.small(n, c=c, n_atoms=9, seed=71, radius=0.4 * n, nbins=60, prec=prec)
    wl = replace(base, cell=base.cell.with_rot(W.rotation([1.0, 2.0, 3.0], 0.7), interp))
    _say(f"rotated lattice {n}^3 prec={prec} interp={interp} cell {c}^3")
    ref = orc.simulate(wl)
    got = run_simulate(ur, wl)
    compare_bins(got, ref, F32_BIN if prec == 0 else F64_BIN, "rotated", n=n)
    tol = 1e-6 if prec == 0 else 1e-12
    assert abs(got["totals"][3] - ref["rho_sumsq"]) <= tol * ref["rho_sumsq"]
    plan = ur.Plan(n, 1.0, prec)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    rho = plan.rho_generate(cell, wl.mask, wl.zoom)
    torch.cuda.synchronize()
    want = orc.density(wl)
    err = np.max(np.abs(rho.cpu().numpy().astype(np.float64) - want)) / np.max(np.abs(want))
    _say(f"  density max rel err {err:.3e}")
    assert err <= (1e-6 if prec == 0 else 1e-14)
    h = ur.Hist(wl.nbins)
    g = torch.zeros(wl.nbins, dtype=torch.float64, device="cuda")
    ga = torch.zeros(wl.cell.n_atoms, dtype=torch.float64, device="cuda")
    if c > 16:
        with pytest.raises(ur.UltimaError, match="status 2"):
            plan.adjoint(h, g, cell=cell, mask=wl.mask, grad_amp=ga)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,interp,grains", [(0, 1, False), (1, 1, False), (0, 3, False), (1, 3, True),
                                                (0, 1, True)])
def test_rotated_zoom_levels(ur, orc, prec, interp, grains):
    """Zoom levels of an oriented lattice (64^3 by 2 and 32^3 by 4 from a
    128^3 ED-1; one orientation, or 5 grains): the fused forward path against
    the oracle (O2r/O2g, block sums O3, then O4-O8), the level's density from
    ur_rho_generate voxel by voxel, and Sum rho^2; the allocation-free entry
    refuses such levels."""
    import torch
    from dataclasses import replace
    R = W.rotation([1.0, 2.0, 3.0], 0.7)
    seeds, rots = W.random_grains(77, 5, 0.35 * 128)
    for wl in W.zoom_levels(128, 8, 9, 73, 50.0, [(64, 2), (32, 4)], 40, decades=2.0):
        cell_h = wl.cell.with_grains(seeds, rots, interp) if grains else wl.cell.with_rot(R, interp)
        wl = replace(wl, prec=prec, cell=cell_h)
        _say(f"rotated zoom level {wl.n}^3 f={wl.zoom.factor} prec={prec} interp={interp} grains={grains}")
        ref = orc.simulate(wl, return_fields=True)
        got = run_simulate(ur, wl)
        compare_bins(got, ref, F32_BIN if prec == 0 else F64_BIN, "rotated zoom level", n=wl.n)
        assert abs(got["totals"][3] - ref["rho_sumsq"]) <= (1e-6 if prec == 0 else 1e-12) * ref["rho_sumsq"]
        plan = ur.Plan(wl.n, wl.voxel, prec)
        plan.set_bins(wl.edges)
        cell = ur.DeviceCell.from_host(wl.cell)
        rho = plan.rho_generate(cell, wl.mask, wl.zoom)
        torch.cuda.synchronize()
        want = ref["rho"]
        err = np.max(np.abs(rho.cpu().numpy().astype(np.float64) - want)) / np.max(np.abs(want))
        _say(f"  level density max rel err {err:.3e}")
        assert err <= (2e-6 if prec == 0 else 1e-13)
        if prec == 0:
            h = ur.Hist(wl.nbins)
            with pytest.raises(ur.UltimaError, match="status 2"):
                plan.simulate_noalloc(cell, wl.mask, wl.zoom, h)
        torch.cuda.synchronize()


@pytest.mark.parametrize("n,prec,interp,c", [(64, 0, 1, 8), (64, 1, 1, 8), (64, 0, 3, 8), (64, 1, 3, 8), (128, 0, 3, 8),
                                              (64, 1, 3, 32), (64, 0, 1, 32)])
def test_polycrystalline_grains(ur, orc, n, prec, interp, c):
    """A polycrystalline particle: 7 grains (random integer seeds inside the
    sphere, random orientations), every inside voxel sampling the cell in
    its nearest seed's orientation; the fused forward path against the
    oracle (O2g, then O4-O8) and the generated density voxel by voxel.
    Grains with a lattice rotation, more than 16 grains and seeds that are not
    integers are refused."""
    import ctypes
    import torch
    from dataclasses import replace
    base = W.small(n, c=c, n_atoms=9, seed=72, radius=0.4 * n, nbins=60, prec=prec)
    seeds, rots = W.random_grains(73, 7, 0.35 * n)
    wl = replace(base, cell=base.cell.with_grains(seeds, rots, interp))
    _say(f"grains {n}^3 prec={prec} interp={interp} cell {c}^3")
    ref = orc.simulate(wl)
    got = run_simulate(ur, wl)
    compare_bins(got, ref, F32_BIN if prec == 0 else F64_BIN, "grains", n=n)
    tol = 1e-6 if prec == 0 else 1e-12
    assert abs(got["totals"][3] - ref["rho_sumsq"]) <= tol * ref["rho_sumsq"]
    plan = ur.Plan(n, 1.0, prec)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    rho = plan.rho_generate(cell, wl.mask, wl.zoom)
    torch.cuda.synchronize()
    want = orc.density(wl)
    err = np.max(np.abs(rho.cpu().numpy().astype(np.float64) - want)) / np.max(np.abs(want))
    _say(f"  density max rel err {err:.3e}")
    assert err <= (1e-6 if prec == 0 else 1e-14)
    h = ur.Hist(wl.nbins)
    for bad in (replace(cell, rot=np.eye(3).reshape(9)),
                replace(cell, grain_seed=np.zeros(51), grain_rot=np.tile(np.eye(3).reshape(9), 17)),
                replace(cell, grain_seed=cell.grain_seed + 0.5)):
        with pytest.raises(ur.UltimaError, match="status 1"):
            plan.simulate(bad, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# voxel form factor (intensities of the voxel-uniform density)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", [0, 1])
def test_voxel_form_factor(ur, orc, prec):
    """With the voxel form factor on: the fused path, ur_simulate_rho and
    ur_intensity_bin against the oracle with O15 applied; off again gives the
    plain curve (its adjoint is checked in test_gpu_path)."""
    import torch
    wl = W.small(64, c=8, n_atoms=9, seed=33, radius=22.0, nbins=50, prec=prec)
    _say(f"voxel form factor prec={prec}")
    ref_v = orc.simulate(wl, return_fields=True, voxel_form_factor=True)
    plan = ur.Plan(wl.n, wl.voxel, prec)
    plan.set_bins(wl.edges)
    plan.set_voxel_form(True)
    cell = ur.DeviceCell.from_host(wl.cell)
    tol = F32_BIN if prec == 0 else F64_BIN
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    compare_bins(h.numpy(), ref_v, tol, "simulate + voxel form", n=wl.n)
    rho = torch.as_tensor(ref_v["rho"], dtype=plan.real_dtype, device="cuda").contiguous()
    h1 = ur.Hist(wl.nbins)
    plan.simulate_rho(rho, h1)
    torch.cuda.synchronize()
    compare_bins(h1.numpy(), ref_v, tol, "simulate_rho + voxel form", n=wl.n)
    spec = torch.as_tensor(np.ascontiguousarray(ref_v["F"][:, :, : wl.n // 2 + 1].transpose(2, 1, 0)),
                           dtype=plan.complex_dtype, device="cuda")
    h2 = ur.Hist(wl.nbins)
    plan.intensity_bin(spec, h2)
    torch.cuda.synchronize()
    compare_bins(h2.numpy(), ref_v, tol, "intensity_bin + voxel form", n=wl.n)
    plan.set_voxel_form(False)
    h3 = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h3)
    torch.cuda.synchronize()
    compare_bins(h3.numpy(), orc.simulate(wl), tol, "voxel form off", n=wl.n)


# ---------------------------------------------------------------------------
# block-transfer correction of zoom levels (O18)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", [0, 1])
def test_block_transfer_correction(ur, orc, prec):
    """Zoom levels 64^3 by 2 and by 4 of a 128^3 ED-1 with the block
    transfer removed: the fused path and ur_intensity_bin against the
    oracle with O18 applied, alone and with the voxel form factor; a level of
    another factor, the adjoint and a mixed-radix plan are refused; factor 0
    restores the plain curve."""
    import torch
    from dataclasses import replace
    levels = W.zoom_levels(128, 8, 10, 41, 50.0, [(64, 2), (64, 4)], 48, decades=2.0)
    tol = F32_BIN if prec == 0 else F64_BIN
    for wl in levels:
        wl = replace(wl, prec=prec)
        f = wl.zoom.factor
        _say(f"block transfer f={f} prec={prec}")
        ref = orc.simulate(wl, return_fields=True, block_transfer_removed=True)
        plan = ur.Plan(wl.n, wl.voxel, prec)
        plan.set_bins(wl.edges)
        plan.set_block_transfer(f)
        cell = ur.DeviceCell.from_host(wl.cell)
        h = ur.Hist(wl.nbins)
        plan.simulate(cell, wl.mask, wl.zoom, h)
        torch.cuda.synchronize()
        compare_bins(h.numpy(), ref, tol, f"simulate, block transfer f={f}", n=wl.n)
        spec = torch.as_tensor(np.ascontiguousarray(ref["F"][:, :, : wl.n // 2 + 1].transpose(2, 1, 0)),
                               dtype=plan.complex_dtype, device="cuda")
        h2 = ur.Hist(wl.nbins)
        plan.intensity_bin(spec, h2)
        torch.cuda.synchronize()
        compare_bins(h2.numpy(), ref, tol, f"intensity_bin, block transfer f={f}", n=wl.n)
        # with the voxel form factor as well: the weights multiply
        plan.set_voxel_form(True)
        h3 = ur.Hist(wl.nbins)
        plan.simulate(cell, wl.mask, wl.zoom, h3)
        torch.cuda.synchronize()
        compare_bins(h3.numpy(), orc.simulate(wl, voxel_form_factor=True, block_transfer_removed=True), tol,
                     f"simulate, block transfer f={f} + voxel form", n=wl.n)
        plan.set_voxel_form(False)
        # refusals: another factor, the adjoint
        other = replace(wl, zoom=replace(wl.zoom, factor=2 if f != 2 else 4))
        with pytest.raises(ur.UltimaError, match="status 1"):
            plan.simulate(cell, other.mask, other.zoom, h)
        g = torch.zeros(wl.nbins, dtype=torch.float64, device="cuda")
        ga = torch.zeros(wl.cell.n_atoms, dtype=torch.float64, device="cuda")
        with pytest.raises(ur.UltimaError, match="status 2"):
            plan.adjoint(h, g, cell=cell, mask=wl.mask, grad_amp=ga)
        # off again: the plain curve
        plan.set_block_transfer(0)
        h4 = ur.Hist(wl.nbins)
        plan.simulate(cell, wl.mask, wl.zoom, h4)
        torch.cuda.synchronize()
        compare_bins(h4.numpy(), orc.simulate(wl), tol, f"block transfer off f={f}", n=wl.n)
        # the correction raises every populated bin away from q = 0
        pop = (ref["count"] > 0) & (h4.numpy()["count"] > 0)
        assert np.all(h.numpy()["mean"][pop] >= h4.numpy()["mean"][pop] * (1 - 1e-6))
    mplan = ur.Plan(40, 1.0, prec, c2c=True)
    with pytest.raises(ur.UltimaError, match="status 2"):
        mplan.set_block_transfer(2)


# ---------------------------------------------------------------------------
# Ewald-sphere detector image
# ---------------------------------------------------------------------------

EWALD_GEOS = {
    "beam_z": W.detector(np.eye(3), pixel=5.0, nu=41, nv=33, cu=20, cv=16),
    "tilted_spread": W.detector(W.rotation([0.3, -0.5, 0.8], 1.1), rel_spread=0.05, n_lambda=16,
                                pixel=5.0, nu=37, nv=29, cu=11.0, cv=20.0),
    "wide_offcentre": W.detector(W.rotation([1.0, 1.0, 0.0], 2.0), rel_spread=0.02, n_lambda=5,
                                 distance=300.0, pixel=4.0, nu=64, nv=48, cu=-10.5, cv=60.25),
}


@pytest.mark.parametrize("geo_name", sorted(EWALD_GEOS))
@pytest.mark.parametrize("prec,c2c,n", [(0, False, 64), (1, False, 64), (1, True, 32), (0, True, 32)])
def test_ewald_image(ur, orc, geo_name, prec, c2c, n):
    """ur_ewald_image on the transform of ur_fft3d_exec against the oracle's
    image of the full FP64 spectrum: real boxes read the missing half of the
    spectrum through F(-q) = F(q)*; the detectors reach several times past
    the Nyquist frequency (periodic grid).  Bound per pixel: each spectrum
    value is off by at most eps_F max|F| (2e-6 in FP32, 1e-13 in FP64, as
    for the transform alone), so an interpolated intensity (weights summing
    to 1) is off by at most 2 eps_F max|F| sqrt(I) + (eps_F max|F|)^2, plus
    FP64 rounding of the interpolation (1e-14 max|F|^2)."""
    import torch
    geo = EWALD_GEOS[geo_name]
    _say(f"ewald {geo_name} n={n} prec={prec} c2c={c2c}")
    if c2c:
        rng = np.random.default_rng(700 + n)
        rho = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
        dt = torch.complex64 if prec == 0 else torch.complex128
    else:
        rho = W.random_density(700 + n, n)
        dt = torch.float32 if prec == 0 else torch.float64
    voxel = 1.0
    F = orc.forward(rho)
    ref = orc.ewald_image(F, voxel, geo)
    plan = ur.Plan(n, voxel, prec, c2c=c2c)
    spec = plan.fft3d(torch.as_tensor(rho, dtype=dt, device="cuda").contiguous())
    img = plan.ewald_image(spec, geo)
    torch.cuda.synchronize()
    got = img.cpu().numpy()
    fmax = float(np.max(np.abs(F)))
    eps_f = 2e-6 if prec == 0 else 1e-13
    bound = 2.0 * eps_f * fmax * np.sqrt(ref) + (eps_f * fmax) ** 2 + 1e-14 * fmax ** 2
    ratio = np.abs(got - ref) / bound
    _say(f"  max rel err {np.max(np.abs(got - ref) / ref):.3e}, max err/bound {ratio.max():.3f}")
    assert np.all(ratio <= 1.0)


def test_ewald_image_refusals(ur):
    """Axes that are not orthonormal, a non-positive wavelength or pixel,
    an out-of-range node count and a spectrum of the wrong size are refused
    before any launch."""
    import dataclasses
    import torch
    n = 16
    plan = ur.Plan(n, 1.0, 1)
    spec = torch.zeros((n // 2 + 1, n, n), dtype=torch.complex128, device="cuda")
    good = W.detector(np.eye(3), nu=8, nv=8)
    plan.ewald_image(spec, good)
    for bad in (dataclasses.replace(good, du=(1.0, 0.1, 0.0)), dataclasses.replace(good, wavelength=0.0),
                dataclasses.replace(good, pixel=-1.0), dataclasses.replace(good, rel_spread=0.1, n_lambda=65),
                dataclasses.replace(good, rel_spread=0.5)):
        with pytest.raises(ur.UltimaError, match="status 1"):
            plan.ewald_image(spec, bad)
    with pytest.raises(ur.UltimaError, match="elements"):
        plan.ewald_image(spec[:4], good)
    torch.cuda.synchronize()


def test_ewald_image_1024_sampled(ur, orc):
    """The Ewald image at the headline box size: a 1024^3 FP32 box that is
    zero but at 64 voxels, its r2c spectrum from ur_fft3d_exec, a tilted
    256 x 192 detector with a 2 % wavelength spread (8 nodes) reaching past
    the Nyquist frequency; 60 random pixels against the oracle with every
    corner coefficient summed directly over the 64 voxels.  Bound as for the
    small boxes, with max|F| <= sum(rho)/n^3."""
    import torch
    n = 1024
    _say("ewald 1024 sampled")
    xyz, val = W.sparse_voxels(4096, n, 64, dtype=np.float32)
    x = torch.zeros((n, n, n), dtype=torch.float32, device="cuda")
    x[torch.as_tensor(xyz[:, 0], device="cuda"), torch.as_tensor(xyz[:, 1], device="cuda"),
      torch.as_tensor(xyz[:, 2], device="cuda")] = torch.as_tensor(val, device="cuda")
    plan = ur.Plan(n, 1.0, 0)
    spec = plan.fft3d(x)
    del x
    geo = W.detector(W.rotation([0.3, -0.5, 0.8], 1.1), rel_spread=0.02, n_lambda=8, distance=300.0,
                     pixel=0.5, nu=256, nv=192, cu=100.0, cv=60.0)
    img = plan.ewald_image(spec, geo)
    torch.cuda.synchronize()
    del spec, plan
    torch.cuda.empty_cache()
    rng = np.random.default_rng(61)
    iv, iu = rng.integers(0, geo.nv, 60), rng.integers(0, geo.nu, 60)
    got = img.cpu().numpy()[iv, iu]
    ref = orc.ewald_pixels_sparse(n, 1.0, geo, iv, iu, xyz, val.astype(np.float64))
    fmax = float(np.sum(val.astype(np.float64))) / float(n) ** 3
    bound = 2.0 * 2e-6 * fmax * np.sqrt(ref) + (2e-6 * fmax) ** 2 + 1e-14 * fmax ** 2
    ratio = np.abs(got - ref) / bound
    _say(f"  max rel err {np.max(np.abs(got - ref) / ref):.3e}, max err/bound {ratio.max():.3f}")
    assert np.all(ratio <= 1.0)


def test_grains_1024_forward_matches_generated_density(ur):
    """16 grains at 1024^3 FP32 (the benchmarked polycrystal): the fused
    forward path (grains generated inside the z pass) against
    ur_simulate_rho of the whole box from ur_rho_generate (checked voxel by
    voxel against the oracle in the sampled test); the two generators must
    agree on every voxel, so the curves agree to the transform's rounding."""
    import torch
    wl = W.m1024()
    seeds, rots = W.random_grains(16, 16, 0.35 * wl.n)
    cell = ur.DeviceCell.from_host(wl.cell.with_grains(seeds, rots, 1))
    _say("grains 1024 forward vs generated density")
    plan = ur.Plan(wl.n, wl.voxel, 0)
    plan.set_bins(wl.edges)
    h1 = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h1)
    rho = plan.rho_generate(cell, wl.mask, wl.zoom)
    h2 = ur.Hist(wl.nbins)
    plan.simulate_rho(rho, h2)
    torch.cuda.synchronize()
    a, b = h1.numpy(), h2.numpy()
    assert np.array_equal(a["count"], b["count"])
    pop = a["count"] > 0
    rel = np.abs(a["mean"][pop] - b["mean"][pop]) / np.abs(b["mean"][pop])
    _say(f"  max rel diff {rel.max():.3e}")
    assert rel.max() <= 1e-6
    del rho
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", ["trilinear", "cubic", "grains16"])
def test_oriented_density_1024_sampled(ur, orc, kind):
    """The rotated samplers at the size the benchmark times them: the 1024^3
    FP32 headline particle with its lattice rotated (trilinear or cubic) or
    split into 16 grains; ur_rho_generate over the 8 central planes, 4000
    random voxels of them against the oracle evaluated voxel by voxel.
    Bound: 16 eps32 times the largest cell value or spline coefficient (the
    weights are nonnegative and sum to 1; they and the cell table are
    rounded to FP32)."""
    import torch
    wl = W.m1024()
    R = W.rotation([1.0, 2.0, 3.0], 0.7)
    if kind == "grains16":
        seeds, rots = W.random_grains(16, 16, 0.35 * wl.n)
        cellh = wl.cell.with_grains(seeds, rots, 1)
        interp = 1
    else:
        interp = 3 if kind == "cubic" else 1
        cellh = wl.cell.with_rot(R, interp)
        seeds, rots = np.zeros((1, 3)), R[None]
    _say(f"oriented density 1024 {kind}")
    plan = ur.Plan(wl.n, wl.voxel, 0)
    x_lo, x_hi = wl.n // 2 - 4, wl.n // 2 + 3
    rho = plan.rho_generate(ur.DeviceCell.from_host(cellh), wl.mask, wl.zoom, x_lo=x_lo, x_hi=x_hi)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1024)
    pts = np.stack([rng.integers(x_lo, x_hi + 1, 4000), rng.integers(0, wl.n, 4000), rng.integers(0, wl.n, 4000)], axis=1)
    got = rho.cpu().numpy()[pts[:, 0] - x_lo, pts[:, 1], pts[:, 2]].astype(np.float64)
    cg = orc.cell_synth(wl.cell)
    ref = orc.oriented_points(wl.n, cg, wl.mask, pts, seeds, rots, interp)
    big = np.max(np.abs(orc.bspline_coefficients(cg) if interp == 3 else cg))
    err = np.max(np.abs(got - ref))
    _say(f"  {np.count_nonzero(ref)} inside, max abs err {err:.3e} = {err / (2.0 ** -24 * big):.2f} eps32 x max")
    assert np.count_nonzero(ref) > 1000
    assert err <= 16 * 2.0 ** -24 * big
