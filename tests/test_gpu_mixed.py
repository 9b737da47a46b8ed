"""Boxes whose edge is not a power of two (n = 2^a 3^b 5^c: the paper's 250 ...
2000 family of ED-1 and zoom boxes, and 2^a 3): the mixed-radix path
(radix 2/4/8 then 3 then 5 Stockham stages, one axis at a time, in place,
natural-order spectrum) through the C ABI against the FP64 oracle, whose
transform takes odd lengths by the DFT sum itself (pinned against brute force
and numpy.fft in test_oracle_pins.py).

Tolerances as for the power-of-two transforms: spectra within 2e-6 (FP32)
or 1e-13 (FP64) of max|F|; bin counts bit-exact and means within 1e-5 /
1e-12 relative (compare_bins).
"""
import sys

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import F32_BIN, F64_BIN, compare_bins

pytestmark = pytest.mark.gpu

_SPECTRA = {}


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
    print(msg, file=sys.stderr, flush=True)


def _spectrum(orc, n):
    if n not in _SPECTRA:
        rng = np.random.default_rng(900 + n)
        z = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
        _SPECTRA[n] = (z, orc.fft3d(z, -1) / float(n) ** 3)
    return _SPECTRA[n]


@pytest.mark.parametrize("n", [40, 48, 96, 100, 160, 200, 250])
@pytest.mark.parametrize("prec", [0, 1])
def test_mixed_fft3d_forward_and_inverse(ur, orc, n, prec):
    """Every coefficient of a random complex box (radix sequences 2,2,2,5 /
    2,2,2,2,3 / 2,2,2,2,2,3 / 2,2,5,5 / 2,2,2,2,2,5 / 2,2,2,5,5 / 2,5,5,5),
    and the inverse transform back to the input."""
    import torch
    _say(f"mixed fft3d n={n} prec={prec}")
    z, F = _spectrum(orc, n)
    plan = ur.Plan(n, 1.0, prec, c2c=True)
    dt = torch.complex64 if prec == 0 else torch.complex128
    out = plan.fft3d(torch.as_tensor(z, dtype=dt, device="cuda").contiguous())
    torch.cuda.synchronize()
    err = np.max(np.abs(out.cpu().numpy() - F)) / np.max(np.abs(F))
    _say(f"  spectrum rel err {err:.3e}")
    assert err <= (2e-6 if prec == 0 else 1e-13)
    back = plan.fft3d(out, direction=+1)
    torch.cuda.synchronize()
    err2 = np.max(np.abs(back.cpu().numpy() - z)) / np.max(np.abs(z))
    assert err2 <= (2e-6 if prec == 0 else 1e-13)


@pytest.mark.parametrize("n,prec", [(400, 0), (500, 0), (384, 1), (768, 0), (1000, 0), (1000, 1), (1536, 0), (2000, 0)])
def test_mixed_fft3d_sampled(ur, orc, n, prec):
    """Large mixed-radix boxes (up to 2000^3 FP32, 64 GB each way): zero
    except at 64 random voxels, 516 coefficients over the whole spectrum
    against eq. 1 by direct summation."""
    import torch
    _say(f"mixed fft3d sampled n={n} prec={prec}")
    xyz, val = W.sparse_voxels(3000 + n, n, 64, dtype=np.float32 if prec == 0 else np.float64)
    dt = torch.complex64 if prec == 0 else torch.complex128
    x = torch.zeros((n, n, n), dtype=dt, device="cuda")
    idx = [torch.as_tensor(xyz[:, i], device="cuda") for i in range(3)]
    x[idx[0], idx[1], idx[2]] = torch.as_tensor(val, device="cuda").to(dt)
    plan = ur.Plan(n, 1.0, prec, c2c=True)
    out = plan.fft3d(x)
    del x
    uvw = W.random_frequencies(3001 + n, n, 512, half_z=False)
    q = torch.as_tensor(uvw, device="cuda")
    got = out[q[:, 0], q[:, 1], q[:, 2]].cpu().numpy().astype(np.complex128)
    del out, plan
    torch.cuda.empty_cache()
    ref = orc.dft_points(n, xyz, val.astype(np.float64), uvw)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"  sampled rel err {err:.3e}")
    assert err <= (2e-6 if prec == 0 else 1e-13)


@pytest.mark.parametrize("n,prec", [(40, 0), (40, 1), (100, 0), (100, 1), (200, 1), (250, 0)])
def test_mixed_simulate(ur, orc, n, prec):
    """The whole forward path on a mixed-radix box (lattice of Gaussian atoms
    in a sphere): ur_simulate, ur_simulate_rho and ur_intensity_bin against
    the oracle; ur_rho_generate voxel by voxel."""
    import torch
    wl = W.mixed(n, prec, nbins=64)
    _say(f"mixed simulate n={n} prec={prec}")
    ref = orc.simulate(wl, return_fields=True)
    plan = ur.Plan(n, wl.voxel, prec, c2c=True)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    tol = F32_BIN if prec == 0 else F64_BIN
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    got = h.numpy()
    compare_bins(got, ref, tol, "mixed simulate", n=n)
    rt = 1e-6 if prec == 0 else 1e-12
    assert abs(got["totals"][3] - np.sum(ref["rho"] ** 2)) <= rt * np.sum(ref["rho"] ** 2)
    assert abs(got["totals"][1] - ref["totals"][1]) <= rt * abs(ref["totals"][1])
    rho = plan.rho_generate(cell, wl.mask, wl.zoom)
    torch.cuda.synchronize()
    assert np.max(np.abs(rho.cpu().numpy() - ref["rho"])) <= (1e-6 if prec == 0 else 1e-14) * np.max(np.abs(ref["rho"]))
    z = torch.as_tensor(ref["rho"], dtype=plan.complex_dtype, device="cuda").contiguous()
    h1 = ur.Hist(wl.nbins)
    plan.simulate_rho(z, h1)
    torch.cuda.synchronize()
    got1 = h1.numpy()
    compare_bins(got1, ref, tol, "mixed simulate_rho", n=n)
    assert abs(got1["totals"][3] - np.sum(ref["rho"] ** 2)) <= rt * np.sum(ref["rho"] ** 2)
    spec = torch.as_tensor(ref["F"], dtype=plan.complex_dtype, device="cuda").contiguous()
    h2 = ur.Hist(wl.nbins)
    plan.intensity_bin(spec, h2)
    torch.cuda.synchronize()
    compare_bins(h2.numpy(), ref, tol, "mixed intensity_bin", n=n)


@pytest.mark.parametrize("n,prec", [(40, 0), (40, 1), (100, 0), (100, 1), (250, 0), (250, 1)])
def test_mixed_real_boxes(ur, orc, n, prec):
    """Real mixed-radix plans (two real pencils per complex z line, the half
    spectrum kz in [0, n/2] in natural order [kx][ky][kz], kz in (0, n/2)
    binned twice): ur_simulate, ur_simulate_rho, ur_fft3d_exec (every
    coefficient of the half spectrum), ur_intensity_bin and the Ewald image
    of the half spectrum against the oracle; a zoom level (40^3 by 4 of a
    160^3 ED-1); the inverse transform and oriented lattices are refused."""
    import torch
    from dataclasses import replace
    wl = replace(W.mixed(n, prec, nbins=64), transform="r2c")
    _say(f"mixed real n={n} prec={prec}")
    ref = orc.simulate(wl, return_fields=True)
    plan = ur.Plan(n, wl.voxel, prec)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    tol = F32_BIN if prec == 0 else F64_BIN
    rt = 1e-6 if prec == 0 else 1e-12
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    got = h.numpy()
    compare_bins(got, ref, tol, "mixed real simulate", n=n)
    assert abs(got["totals"][3] - np.sum(ref["rho"] ** 2)) <= rt * np.sum(ref["rho"] ** 2)
    assert abs(got["totals"][1] - ref["totals"][1]) <= rt * abs(ref["totals"][1])
    rho = torch.as_tensor(ref["rho"], dtype=plan.real_dtype, device="cuda").contiguous()
    h1 = ur.Hist(wl.nbins)
    plan.simulate_rho(rho, h1)
    torch.cuda.synchronize()
    compare_bins(h1.numpy(), ref, tol, "mixed real simulate_rho", n=n)
    nh = n // 2 + 1
    half = np.ascontiguousarray(ref["F"][:, :, :nh])
    spec = plan.fft3d(rho)
    torch.cuda.synchronize()
    assert tuple(spec.shape) == (n, n, nh)
    err = np.max(np.abs(spec.cpu().numpy() - half)) / np.max(np.abs(half))
    _say(f"  half spectrum rel err {err:.3e}")
    assert err <= (2e-6 if prec == 0 else 1e-13)
    h2 = ur.Hist(wl.nbins)
    plan.intensity_bin(torch.as_tensor(half, dtype=plan.complex_dtype, device="cuda"), h2)
    torch.cuda.synchronize()
    compare_bins(h2.numpy(), ref, tol, "mixed real intensity_bin", n=n)
    if n == 40:
        geo = W.detector(W.rotation([0.3, -0.5, 0.8], 1.1), rel_spread=0.05, n_lambda=8, pixel=5.0,
                         nu=31, nv=23, cu=11.0, cv=12.0)
        img = plan.ewald_image(torch.as_tensor(half, dtype=plan.complex_dtype, device="cuda"), geo)
        torch.cuda.synchronize()
        want = orc.ewald_image(ref["F"], wl.voxel, geo)
        fmax = float(np.max(np.abs(ref["F"])))
        eps = 2e-6 if prec == 0 else 1e-13
        assert np.max(np.abs(img.cpu().numpy() - want)) <= 2 * eps * fmax * np.sqrt(np.max(want)) + (eps * fmax) ** 2
        zl = replace(W.mixed_zoom(40, 160, 4, prec), transform="r2c")
        zref = orc.simulate(zl)
        zp = ur.Plan(zl.n, zl.voxel, prec)
        zp.set_bins(zl.edges)
        hz = ur.Hist(zl.nbins)
        zp.simulate(ur.DeviceCell.from_host(zl.cell), zl.mask, zl.zoom, hz)
        torch.cuda.synchronize()
        compare_bins(hz.numpy(), zref, tol, "mixed real zoom level", n=zl.n)
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.fft3d(spec, direction=+1)
    rcell = ur.DeviceCell.from_host(wl.cell.with_rot(W.rotation([1.0, 2.0, 3.0], 0.7), 1))
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.simulate(rcell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,prec,pinned", [(100, 1, True), (250, 0, False), (40, 0, True)])
def test_mixed_out_of_core(ur, orc, n, prec, pinned):
    """Real mixed-radix boxes streamed from host memory (page-locked, or
    pageable through the bounce slabs): slabs of planes transformed along z
    and y as they arrive into a box of only the particle's planes, then the
    x pass with the other planes read as zero; against the whole oracle,
    and against the in-HBM real plan; a truncated octahedron whose planes do
    not start at a slab boundary."""
    import torch
    from dataclasses import replace
    wl = replace(W.mixed(n, prec, nbins=60), mask=W.trunc_oct(0.37 * n), transform="r2c")
    _say(f"mixed out-of-core n={n} prec={prec} pinned={pinned}")
    ref = orc.simulate(wl, return_fields=True)
    rho = ref["rho"]
    nz = np.flatnonzero(np.any(rho != 0.0, axis=(1, 2)))
    x_lo, x_hi = int(nz.min()), int(nz.max())
    host = torch.empty((x_hi - x_lo + 1, n, n), dtype=torch.float32 if prec == 0 else torch.float64, pin_memory=pinned)
    host.copy_(torch.as_tensor(rho[x_lo:x_hi + 1]))
    plan = ur.Plan(n, wl.voxel, prec)
    plan.set_bins(wl.edges)
    h = ur.Hist(wl.nbins)
    nbytes = plan.simulate_host(host, x_lo, x_hi, h)
    torch.cuda.synchronize()
    got = h.numpy()
    assert nbytes == (x_hi - x_lo + 1) * n * n * host.element_size()
    tol = F32_BIN if prec == 0 else F64_BIN
    compare_bins(got, ref, tol, "mixed out-of-core", n=n)
    rt = 1e-6 if prec == 0 else 1e-12
    assert abs(got["totals"][3] - ref["rho_sumsq"]) <= rt * ref["rho_sumsq"]
    assert abs(got["totals"][1] - ref["totals"][1]) <= rt * abs(ref["totals"][1])
    p2 = ur.Plan(n, wl.voxel, prec)
    p2.set_bins(wl.edges)
    h2 = ur.Hist(wl.nbins)
    p2.simulate(ur.DeviceCell.from_host(wl.cell), wl.mask, wl.zoom, h2)
    torch.cuda.synchronize()
    b = h2.numpy()
    pop = ref["count"] > 0
    assert np.array_equal(got["count"], b["count"])
    assert np.allclose(got["mean"][pop], b["mean"][pop], rtol=1e-12 if prec == 1 else 1e-6, atol=0.0)
    cplan = ur.Plan(n, wl.voxel, prec, c2c=True)
    cplan.set_bins(wl.edges)
    with pytest.raises(ur.UltimaError, match="status 2"):
        cplan.simulate_host(host, x_lo, x_hi, h)
    torch.cuda.synchronize()


def test_mixed_2000_counts_and_moments(ur, orc):
    """The 2000^3 FP32 box of the family (64 GB complex box in HBM): counts of
    all 256 bins bit-exact (O12 counts, axis by axis), Parseval, F(0) and the
    sum of rho^2 against the oracle's voxel-by-voxel density moments, and the
    curve finite and positive."""
    import torch
    wl = W.mixed(2000, 0, nbins=256)
    _say("mixed simulate n=2000")
    plan = ur.Plan(wl.n, wl.voxel, 0, c2c=True)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    got = h.numpy()
    del plan
    torch.cuda.empty_cache()
    cnt, _ = orc.axis_pair_bins(wl.n, wl.voxel, wl.edges, 1, 1.0, 0.0)
    assert np.array_equal(got["count"], cnt)
    s1, s2 = orc.density_moments(wl, orc.cell_synth(wl.cell))
    n3 = float(wl.n) ** 3
    assert abs(got["totals"][0] - s2 / n3) <= 1e-6 * s2 / n3
    assert abs(got["totals"][1] - s1 / n3) <= 1e-6 * s1 / n3
    assert abs(got["totals"][2]) <= 1e-6 * s1 / n3
    assert abs(got["totals"][3] - s2) <= 1e-6 * s2
    pop = cnt > 0
    assert np.all(np.isfinite(got["mean"][pop])) and np.all(got["mean"][pop] > 0)


def test_mixed_ewald_and_refusals(ur, orc):
    """The Ewald image reads the natural-order spectrum of a mixed-radix plan;
    zoom levels whose n1 the factor does not divide (or a
    factor that is not positive), the adjoint and the voxel form factor are
    refused on such plans, and edges outside the compiled set at creation."""
    import torch
    n = 40
    z, F = _spectrum(orc, n)
    geo = W.detector(W.rotation([0.3, -0.5, 0.8], 1.1), rel_spread=0.05, n_lambda=16, pixel=5.0,
                     nu=37, nv=29, cu=11.0, cv=20.0)
    ref = orc.ewald_image(F, 1.0, geo)
    plan = ur.Plan(n, 1.0, 1, c2c=True)
    img = plan.ewald_image(plan.fft3d(torch.as_tensor(z, device="cuda").contiguous()), geo)
    torch.cuda.synchronize()
    fmax = float(np.max(np.abs(F)))
    assert np.max(np.abs(img.cpu().numpy() - ref)) <= 1e-12 * fmax ** 2
    with pytest.raises(ur.UltimaError, match="status 1"):
        ur.Plan(120, 1.0, 0, c2c=True)
    wl = W.mixed(n, 1, nbins=16)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.simulate(cell, wl.mask, W.Zoom(3 * n + 1, 3), h)          # n1 not divisible by the factor
    with pytest.raises(ur.UltimaError, match="status 1"):
        plan.simulate(cell, wl.mask, W.Zoom(3 * n, 0), h)              # factor not positive
    plan.simulate(cell, wl.mask, wl.zoom, h)
    g = torch.zeros(wl.nbins, dtype=torch.float64, device="cuda")
    ga = torch.zeros(wl.cell.n_atoms, dtype=torch.float64, device="cuda")
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.adjoint(h, g, cell=cell, mask=wl.mask, grad_amp=ga)
    plan.set_voxel_form(True)
    with pytest.raises(ur.UltimaError, match="status 2"):
        plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()


def test_mixed_simulate_and_ewald_in_one_graph(ur, orc):
    """A mixed-radix box (200^3 FP32: density generated in the z pass, |F|^2
    binned in the x pass, the finalize) and an Ewald image of a power-of-two
    box's spectrum, recorded in one HIP graph; three replays, with eager work
    and synchronisation between them, each against the eager results (curve
    to rounding, the image exactly)."""
    import torch
    wl = W.mixed(200, 0, nbins=64)
    plan = ur.Plan(wl.n, wl.voxel, 0, c2c=True)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    p2 = ur.Plan(64, 1.0, 0)
    rho = torch.as_tensor(W.random_density(5, 64), dtype=torch.float32, device="cuda").contiguous()
    spec = p2.fft3d(rho)
    geo = W.detector(W.rotation([0.3, -0.5, 0.8], 1.1), rel_spread=0.05, n_lambda=8, pixel=5.0, nu=48, nv=40)
    img = torch.empty((geo.nv, geo.nu), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()

    def run():
        plan.simulate(cell, wl.mask, wl.zoom, h, stream=s)
        p2.ewald_image(spec, geo, out=img, stream=s)

    with torch.cuda.stream(s):
        run()
    torch.cuda.synchronize()
    m_e, i_e = h.mean.cpu().numpy(), img.cpu().numpy()
    g = ur.Graph(s)
    with torch.cuda.stream(s):
        with g:
            run()
    for rep in range(3):
        h.mean.fill_(0.0)
        img.fill_(0.0)
        junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        m_g = h.mean.cpu().numpy()
        ok = ~np.isnan(m_e)
        assert np.array_equal(np.isnan(m_g), np.isnan(m_e))
        assert np.max(np.abs(m_g[ok] - m_e[ok]) / np.abs(m_e[ok])) <= 1e-12
        assert np.array_equal(img.cpu().numpy(), i_e)
        del junk
    ref = orc.simulate(wl)
    compare_bins(h.numpy(), ref, F32_BIN, "mixed in a graph", n=wl.n)


@pytest.mark.parametrize("n,prec,c", [(200, 1, 21), (250, 0, 105), (100, 0, 7)])
def test_mixed_any_cell_edge(ur, orc, n, prec, c):
    """Cells whose edge is not a power of two (the paper's block-reduced cell
    is 105^3) on mixed-radix boxes, whose generator wraps the cell index by
    a modulo: the whole forward path against the oracle.  The generators of
    the other paths wrap with a bit mask and refuse such cells."""
    import torch
    wl = W.mixed(n, prec, nbins=64, c=c)
    _say(f"mixed simulate n={n} prec={prec} cell {c}^3")
    ref = orc.simulate(wl)
    plan = ur.Plan(n, wl.voxel, prec, c2c=True)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    got = h.numpy()
    compare_bins(got, ref, F32_BIN if prec == 0 else F64_BIN, f"mixed, cell {c}^3", n=n)
    rt = 1e-6 if prec == 0 else 1e-12
    assert abs(got["totals"][3] - ref["rho_sumsq"]) <= rt * ref["rho_sumsq"]
    with pytest.raises(ur.UltimaError, match="status 1"):
        plan.rho_generate(cell, wl.mask, wl.zoom)
    p2 = ur.Plan(128, 1.0, prec)
    p2.set_bins(W.default_log_edges(128, 1.0, 16))
    with pytest.raises(ur.UltimaError, match="status 1"):
        p2.simulate(cell, W.sphere(40.0), W.Zoom(128, 1), ur.Hist(16))
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,n1,f,prec", [(40, 160, 4, 1), (100, 800, 8, 0), (250, 1000, 4, 0),
                                         (40, 200, 5, 1), (100, 300, 3, 0), (40, 1000, 25, 0)])
def test_mixed_zoom_level(ur, orc, n, n1, f, prec):
    """Zoom levels on mixed-radix boxes (the paper's ED-2: its ED-1 block-summed
    by 16 into a 250^3 box; its ED-3 factor 125 = 5^3 is not a power of two,
    here 5, 3 and 25, whose blocks are summed pencil by pencil): the level's
    density (block sums of ED-1 over f^3 voxels, centred) and its curve
    against the oracle (O3 then O4-O8)."""
    import torch
    wl = W.mixed_zoom(n, n1, f, prec)
    _say(f"mixed zoom level {n}^3 from {n1}^3 / {f} prec={prec}")
    ref = orc.simulate(wl, return_fields=True)
    plan = ur.Plan(n, wl.voxel, prec, c2c=True)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    got = h.numpy()
    compare_bins(got, ref, F32_BIN if prec == 0 else F64_BIN, "mixed zoom level", n=n)
    rt = 1e-6 if prec == 0 else 1e-12
    assert abs(got["totals"][3] - ref["rho_sumsq"]) <= rt * ref["rho_sumsq"]
    rho = plan.rho_generate(cell, wl.mask, wl.zoom)
    torch.cuda.synchronize()
    err = np.max(np.abs(rho.cpu().numpy().astype(np.float64) - ref["rho"])) / np.max(np.abs(ref["rho"]))
    assert err <= (1e-6 if prec == 0 else 1e-14)


@pytest.mark.parametrize("n,transform", [(40, "c2c"), (40, "r2c"), (32, "r2c"), (32, "c2c")])
def test_maximum_bin_count(ur, orc, n, transform):
    """4096 bins, the most a plan accepts: the binning x passes then keep
    82 KB of histogram and thresholds in LDS (beside the mixed-radix tile,
    beside the power-of-two columns), and most bins of a small box are
    empty.  ur_simulate and ur_intensity_bin against the oracle."""
    import torch
    from dataclasses import replace
    wl = replace(W.mixed(n, 0, nbins=4096), transform=transform)
    _say(f"maximum bin count n={n} {transform}")
    ref = orc.simulate(wl, return_fields=True)
    plan = ur.Plan(n, wl.voxel, 0, c2c=transform == "c2c")
    plan.set_bins(wl.edges)
    h = ur.Hist(wl.nbins)
    plan.simulate(ur.DeviceCell.from_host(wl.cell), wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    got = h.numpy()
    assert np.count_nonzero(got["count"]) < wl.nbins
    compare_bins(got, ref, F32_BIN, "4096 bins simulate", n=n)
    F = ref["F"] if transform == "c2c" else ref["F"][:, :, :n // 2 + 1]
    if n & (n - 1) == 0:                               # power-of-two plans: [kz][ky][kx]
        F = np.transpose(F, (2, 1, 0))
    F = np.ascontiguousarray(F)
    h2 = ur.Hist(wl.nbins)
    plan.intensity_bin(torch.as_tensor(F, dtype=plan.complex_dtype, device="cuda"), h2)
    torch.cuda.synchronize()
    compare_bins(h2.numpy(), ref, F32_BIN, "4096 bins intensity_bin", n=n)


@pytest.mark.parametrize("transform", ["r2c", "c2c"])
@pytest.mark.parametrize("shape", ["one_voxel", "no_mask", "cube_to_faces", "trunc_oct"])
def test_mixed_pruning_edges(ur, orc, transform, shape):
    """The pruned mixed-radix passes (tiles of pencils outside the particle
    skipped, the y pass over the particle's planes with rows outside each
    plane's range read as zero, the x pass over those planes) at the edges of
    the region: a single voxel (one plane, one row), no mask (every plane and
    row), a cube reaching both faces of the box, a truncated octahedron;
    ur_simulate against the oracle at 40^3, FP32 and FP64."""
    import torch
    from dataclasses import replace
    masks = {"one_voxel": W.sphere(0.5), "no_mask": W.no_mask(), "cube_to_faces": W.cube(20),
             "trunc_oct": W.trunc_oct(15.0)}
    for prec in (0, 1):
        wl = replace(W.mixed(40, prec, nbins=64), transform=transform, mask=masks[shape])
        _say(f"pruning edges {shape} {transform} prec={prec}")
        ref = orc.simulate(wl)
        plan = ur.Plan(40, wl.voxel, prec, c2c=transform == "c2c")
        plan.set_bins(wl.edges)
        h = ur.Hist(wl.nbins)
        plan.simulate(ur.DeviceCell.from_host(wl.cell), wl.mask, wl.zoom, h)
        torch.cuda.synchronize()
        compare_bins(h.numpy(), ref, F32_BIN if prec == 0 else F64_BIN, f"pruning {shape}", n=40)
