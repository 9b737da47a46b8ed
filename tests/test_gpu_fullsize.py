"""Full-size parity: every bin of the benchmarked boxes against the whole
FP64 oracle, and the adjoint at the sizes it is timed.

* M1024 (the headline 1024^3 box, 512 log bins), FP32 and FP64;
* the C3 zoom levels ED-2 (1024^3, block factor 4) and ED-3 (512^3, factor
  16) of the 2048^3 ED-1 particle (whose own 2048^3 spectrum exceeds the
  oracle's host memory and keeps its counts / moments / low-frequency checks);
* the mixed-radix M1000 box (1000^3, complex), FP32 and FP64;
* C4 (256^3): the voxel gradient at every voxel and the gradient of all 40
  atom amplitudes against the oracle, and central finite differences
  (h = 1e-3, FP64) on 32 seeded voxels and all 40 amplitudes;
* 1024^3: the adjoint through both entry points (recomputing and reusing the
  forward's y-pass output), FP32 and FP64, with finite differences of all 40
  amplitudes and the dot-product identity of the linearised map.

Tolerances: counts bit-exact; FP32 bin means 1e-5 relative and FP64 1e-12
(a bin whose mean lies far below the box-mean intensity is held to the
transform's rounding bound instead, and listed); Parseval 1e-6 (FP32) /
1e-12 (FP64) against the oracle's sum of rho^2.

The oracle's per-bin results of the largest boxes come from
tests/golden/fullsize_*.npz when those were written (by make_fullsize.py,
which calls only the oracle) from the current oracle and workload sources;
otherwise the oracle runs here.
"""
import importlib.util
import math
import os
import sys
import time
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    spec = importlib.util.spec_from_file_location("make_fullsize", os.path.join(HERE, "golden", "make_fullsize.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


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


_CACHE = {}


def oracle_result(orc, name):
    """The oracle's per-bin statistics of a full-size workload: the stored
    result of make_fullsize.py when it matches the current sources, else a
    live oracle run."""
    if name in _CACHE:
        return _CACHE[name]
    g = _golden()
    r = g.load(name)
    if r is None:
        _say(f"  {name}: running the whole oracle ...")
        t0 = time.perf_counter()
        r = g.compute(name)
        _say(f"  {name}: oracle {time.perf_counter() - t0:.1f} s on {orc.num_threads()} threads")
    else:
        _say(f"  {name}: oracle result stored for the current sources")
    _CACHE[name] = r
    return r


def run_box(ur, wl, prec):
    import torch
    plan = ur.Plan(wl.n, wl.voxel, prec, c2c=(wl.transform == "c2c"))
    plan.set_bins(wl.edges)
    h = ur.Hist(wl.nbins)
    plan.simulate(ur.DeviceCell.from_host(wl.cell), wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    got = h.numpy()
    del plan
    torch.cuda.empty_cache()
    return got


def check_every_bin(got, ref, prec, n, what):
    """Counts bit-exact; every populated bin's mean within 1e-5 (FP32) /
    1e-12 (FP64) relative, or within the transform's rounding bound where a
    bin's mean lies far below the box-mean intensity (listed); SEM; Parseval
    against the oracle's sum of rho^2; F(0) against its sum of rho."""
    assert np.array_equal(got["count"], ref["count"]), f"{what}: counts differ"
    pop = ref["count"] > 0
    assert np.all(np.isnan(got["mean"][~pop]))
    eps, tol = (2.0 ** -24, 1e-5) if prec == 0 else (2.0 ** -53, 1e-12)
    n3 = float(n) ** 3
    ibar = ref["totals"][0] / n3
    m_ref, m_got = ref["mean"][pop], got["mean"][pop]
    rel = np.abs(m_got - m_ref) / np.abs(m_ref)
    bound = np.maximum(tol, 8.0 * eps * math.sqrt(3.0 * math.log2(n)) * np.sqrt(ibar / np.abs(m_ref)))
    above = np.flatnonzero(rel > tol)
    _say(f"  {what} prec={prec}: {pop.sum()} bins, max rel err {rel.max():.3e} (median {np.median(rel):.3e}), "
         f"{above.size} bins above {tol:g}")
    for i in above[np.argsort(-rel[above])][:8]:
        _say(f"    bin {np.flatnonzero(pop)[i]}: count {ref['count'][pop][i]:.0f}, I/Ibar {m_ref[i] / ibar:.3e}, "
             f"rel err {rel[i]:.3e}, bound {bound[i]:.3e}")
    assert np.all(rel <= bound), f"{what}: max err/bound {np.max(rel / bound):.3f}"
    # SEM (one pass over pooled sums on the GPU, two passes in the oracle)
    c = ref["count"][pop]
    multi = c > 1
    s_ref, s_got = ref["sem"][pop][multi], got["sem"][pop][multi]
    t_rel, t_abs = (1e-5, 1e-5) if prec == 0 else (1e-9, 3e-8)
    floor = (8.0 * (6e-8 if prec == 0 else 1.2e-16)) ** 2 * ibar
    sb = t_rel * s_ref + (t_abs * np.abs(m_ref[multi]) + floor) / np.sqrt(c[multi])
    serr = np.abs(s_got - s_ref)
    _say(f"    SEM: max rel err {np.max(serr / s_ref):.3e}, max err/bound {np.max(serr / sb):.3f}")
    if not np.all(serr <= sb):
        idx = np.flatnonzero(pop)[multi]
        for i in np.argsort(-serr / sb)[:6]:
            _say(f"    bin {idx[i]}: count {c[multi][i]:.0f}, mean {m_ref[multi][i]:.4e}, SEM ref {s_ref[i]:.6e} "
                 f"got {s_got[i]:.6e}, spread sqrt(c) SEM / mean {s_ref[i] * np.sqrt(c[multi][i]) / m_ref[multi][i]:.3e}")
    assert np.all(serr <= sb), f"{what}: SEM error {np.max(serr / sb):.3g} x bound"
    # Parseval: sum of I over the box = sum rho^2 / n^3 (eq. 1 carries 1/n^3)
    pt = 1e-6 if prec == 0 else 1e-12
    pars = abs(got["totals"][0] - ref["rho_sumsq"] / n3) / (ref["rho_sumsq"] / n3)
    f0 = abs(got["totals"][1] - ref["rho_sum"] / n3) / abs(ref["rho_sum"] / n3)
    _say(f"    Parseval rel err {pars:.3e}, F(0) rel err {f0:.3e}")
    assert pars <= pt and f0 <= pt


# ---------------------------------------------------------------------------
# every bin of the benchmarked boxes
# ---------------------------------------------------------------------------

@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec", [0, 1])
def test_m1024_every_bin(ur, orc, prec):
    """The headline box in the launch configuration the benchmark times."""
    ref = oracle_result(orc, "M1024")
    wl = W.m1024(prec)
    check_every_bin(run_box(ur, wl, prec), ref, prec, wl.n, "M1024")


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("level", ["C3-ED2", "C3-ED3"])
@pytest.mark.parametrize("prec", [0, 1])
def test_c3_zoom_levels_every_bin(ur, orc, level, prec):
    """The C3 zoom levels (block sums of the 2048^3 ED-1 by 4 and 16,
    centred in 1024^3 and 512^3 boxes), 1024 log bins over four decades."""
    ref = oracle_result(orc, level)
    wl = {w.name: w for w in W.c3_levels()}[level]
    check_every_bin(run_box(ur, wl, prec), ref, prec, wl.n, level)


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec,transform", [(0, "c2c"), (1, "c2c"), (0, "r2c"), (1, "r2c")])
def test_m1000_mixed_every_bin(ur, orc, prec, transform):
    """The benchmarked mixed-radix box (1000^3, density generated in the
    first pass and |F|^2 binned in the last; complex, or real with two real
    pencils per z line and the half spectrum) against the oracle, whose
    transform takes the odd factor 125 by the DFT sum (the curve does not
    depend on the transform the GPU uses)."""
    ref = oracle_result(orc, "M1000")
    wl = replace(W.mixed(1000, prec, nbins=512), transform=transform)
    check_every_bin(run_box(ur, wl, prec), ref, prec, wl.n, f"M1000 {transform}")


# ---------------------------------------------------------------------------
# adjoint at the sizes it is timed
# ---------------------------------------------------------------------------

def _target(orc, wl):
    """Target curve of the chi^2 misfit: the same box with the atom
    amplitudes perturbed by 5 % (seed 41), from the oracle; empty bins 1."""
    tgt = replace(wl, cell=wl.cell.with_amp(W.perturbed_amplitudes(wl.cell, 41, 0.05)), prec=W.PREC_F64)
    r = orc.simulate(tgt)
    return np.where(r["count"] > 0, r["mean"], 1.0)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [1, 0])
def test_c4_adjoint_every_voxel_and_amplitude(ur, orc, prec):
    """C4 (256^3): grad rho at every voxel and grad amp of all 40 atoms from
    the adjoint kernels (recomputing, and from the held forward output)
    against the oracle's gradients for the same g_b (FP32 1e-4, FP64 1e-10
    of the largest entry)."""
    import torch
    wl = replace(W.c4(), prec=prec)
    T = _target(orc, wl)
    _say(f"C4 adjoint prec={prec}: oracle ...")
    ref = orc.simulate(wl, return_fields=True)
    gb = orc.chi2_bin_grad(ref["mean"], ref["count"], T)
    grho_ref = orc.grad_rho(ref["F"], wl.voxel, wl.edges, ref["count"], gb)
    gamp_ref = orc.grad_amp(grho_ref, wl.cell, wl.mask)
    plan = ur.Plan(wl.n, wl.voxel, prec)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    fwd = ur.Hist(wl.nbins)
    g = torch.as_tensor(gb, device="cuda")
    n = wl.n
    grho = torch.empty((n, n, n), dtype=plan.real_dtype, device="cuda")
    gamp = torch.empty(wl.cell.n_atoms, dtype=torch.float64, device="cuda")
    plan.simulate(cell, wl.mask, wl.zoom, fwd)
    plan.adjoint(fwd, g, cell=cell, mask=wl.mask, grad_rho=grho, grad_amp=gamp)
    gamp_keep = torch.empty_like(gamp)
    plan.simulate(cell, wl.mask, wl.zoom, fwd)
    plan.adjoint_reuse(fwd, g, cell, wl.mask, gamp_keep)
    torch.cuda.synchronize()
    assert np.array_equal(fwd.numpy()["count"], ref["count"])
    tol = 1e-10 if prec == 1 else 1e-4
    e_rho = np.max(np.abs(grho.cpu().numpy().astype(np.float64) - grho_ref)) / np.max(np.abs(grho_ref))
    e_amp = np.max(np.abs(gamp.cpu().numpy() - gamp_ref)) / np.max(np.abs(gamp_ref))
    e_keep = np.max(np.abs(gamp_keep.cpu().numpy() - gamp_ref)) / np.max(np.abs(gamp_ref))
    _say(f"  grad_rho ({n}^3 voxels) rel err {e_rho:.3e}; grad_amp (40 atoms) {e_amp:.3e}, from the held output {e_keep:.3e}")
    assert e_rho <= tol and e_amp <= tol and e_keep <= tol


def _fd_loss(ur, plan, nbins, T, count):
    import torch
    from paper_2303_13435_amd.autograd import chi2
    Tt = torch.as_tensor(T, device="cuda")
    cnt = torch.as_tensor(count, device="cuda")

    def loss_of_rho(r):
        h = ur.Hist(nbins)
        plan.simulate_rho(r.contiguous(), h)
        return float(chi2(torch.nan_to_num(h.mean, nan=0.0), Tt, cnt).item())
    return loss_of_rho


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", ["rot1", "grains3"])
def test_c4_oriented_amplitudes_fd(ur, orc, kind):
    """C4 recipe in FP64 (256^3) with the lattice rotated (trilinear) or as 8
    grains (cubic B-spline): d chi^2 / d amp of all 40 atoms through the
    autograd function (the oriented samplers' transpose) against central
    differences (h = 1e-3) of the GPU forward path."""
    import torch
    from paper_2303_13435_amd.autograd import BinnedIntensity, chi2
    wl0 = replace(W.c4(), prec=W.PREC_F64)
    T = _target(orc, wl0)
    if kind == "rot1":
        cell_h = wl0.cell.with_rot(W.rotation([1.0, 2.0, 3.0], 0.7), 1)
    else:
        seeds, rots = W.random_grains(97, 8, 0.35 * wl0.n)
        cell_h = wl0.cell.with_grains(seeds, rots, 3)
    wl = replace(wl0, cell=cell_h)
    _say(f"C4 FP64 oriented ({kind}) amplitude gradients against central differences")
    plan = ur.Plan(wl.n, wl.voxel, 1)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    count = orc.bin_counts(wl.n, wl.voxel, wl.edges)
    Tt = torch.as_tensor(T, device="cuda")
    cnt = torch.as_tensor(count, device="cuda")
    amp = torch.as_tensor(wl.cell.amp, device="cuda").clone().requires_grad_(True)
    chi2(BinnedIntensity.apply(amp, plan, cell, wl.mask, wl.zoom), Tt, cnt).backward()
    ga = amp.grad.cpu().numpy()
    h = 1e-3
    worst = 0.0
    for a_i in range(wl.cell.n_atoms):
        def La(d):
            a2 = amp.detach().clone()
            a2[a_i] += d
            return float(chi2(BinnedIntensity.apply(a2, plan, cell, wl.mask, wl.zoom), Tt, cnt).item())
        fd = (La(h) - La(-h)) / (2 * h)
        worst = max(worst, abs(fd - ga[a_i]) / max(1.0, abs(fd)))
        assert abs(fd - ga[a_i]) <= 1e-6 * max(1.0, abs(fd)), (a_i, fd, ga[a_i])
    _say(f"  40 amplitudes: max |fd - adjoint| / max(1, |fd|) = {worst:.3e}")


@pytest.mark.timeout(600)
def test_c4_finite_differences(ur, orc):
    """C4 recipe in FP64 (256^3): d chi^2 / d rho at the 32 seeded voxels
    (seed 42) and d chi^2 / d amp of all 40 atoms, from the adjoint kernels,
    against central differences (h = 1e-3) of the GPU forward path."""
    import torch
    from paper_2303_13435_amd.autograd import BinnedIntensity, BinnedIntensityRho, chi2
    wl = replace(W.c4(), prec=W.PREC_F64)
    T = _target(orc, wl)
    plan = ur.Plan(wl.n, wl.voxel, 1)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    count = orc.bin_counts(wl.n, wl.voxel, wl.edges)
    Tt = torch.as_tensor(T, device="cuda")
    cnt = torch.as_tensor(count, device="cuda")
    # voxels
    rho0 = plan.rho_generate(cell, wl.mask, wl.zoom)
    rho = rho0.clone().requires_grad_(True)
    chi2(BinnedIntensityRho.apply(rho, plan), Tt, cnt).backward()
    g = rho.grad.cpu().numpy()
    L = _fd_loss(ur, plan, wl.nbins, T, count)
    h = 1e-3
    worst = 0.0
    for (x, y, z) in W.random_voxels(42, wl.n, 32):
        r2 = rho0.clone()
        r2[x, y, z] += h
        lp = L(r2)
        r2[x, y, z] -= 2 * h
        lm = L(r2)
        fd = (lp - lm) / (2 * h)
        worst = max(worst, abs(fd - g[x, y, z]) / max(1.0, abs(fd)))
        assert abs(fd - g[x, y, z]) <= 1e-5 * max(1.0, abs(fd)), (x, y, z, fd, g[x, y, z])
    _say(f"  32 voxels: max |fd - adjoint| / max(1, |fd|) = {worst:.3e}")
    # amplitudes
    amp = torch.as_tensor(wl.cell.amp, device="cuda").clone().requires_grad_(True)
    chi2(BinnedIntensity.apply(amp, plan, cell, wl.mask, wl.zoom), Tt, cnt).backward()
    ga = amp.grad.cpu().numpy()
    worst = 0.0
    for a_i in range(wl.cell.n_atoms):
        def La(d):
            a2 = amp.detach().clone()
            a2[a_i] += d
            return float(chi2(BinnedIntensity.apply(a2, plan, cell, wl.mask, wl.zoom), Tt, cnt).item())
        fd = (La(h) - La(-h)) / (2 * h)
        worst = max(worst, abs(fd - ga[a_i]) / max(1.0, abs(fd)))
        assert abs(fd - ga[a_i]) <= 1e-6 * max(1.0, abs(fd)), (a_i, fd, ga[a_i])
    _say(f"  40 amplitudes: max |fd - adjoint| / max(1, |fd|) = {worst:.3e}")


@pytest.mark.timeout(900)
def test_adjoint_1024(ur, orc):
    """The adjoint at 1024^3 (the box the forward+adjoint timing uses; its
    column groups are wave-uniform there).  FP64: all 40 amplitude
    gradients against central differences (h = 1e-3) of the FP64 forward,
    the recomputing and the reusing entry points against each other, and the
    dot-product identity <dI/drho . v, g> = <v, adjoint(g)> of the voxel
    gradient.  FP32: both entry points' amplitude gradients and the voxel
    gradient against the FP64 adjoint (1e-4 of the largest entry)."""
    import torch
    from paper_2303_13435_amd.autograd import BinnedIntensity, chi2
    wl = W.m1024(W.PREC_F64)
    n = wl.n
    count = orc.bin_counts(n, wl.voxel, wl.edges)
    cnt = torch.as_tensor(count, device="cuda")
    cell = ur.DeviceCell.from_host(wl.cell)
    tcell = ur.DeviceCell.from_host(wl.cell.with_amp(W.perturbed_amplitudes(wl.cell, 41, 0.05)))
    p64 = ur.Plan(n, wl.voxel, 1)
    p64.set_bins(wl.edges)
    th = ur.Hist(wl.nbins)
    p64.simulate(tcell, wl.mask, wl.zoom, th)              # target from the FP64 path
    Tt = torch.where(cnt > 0, torch.nan_to_num(th.mean, nan=1.0), torch.ones_like(th.mean))
    fwd = ur.Hist(wl.nbins)
    p64.simulate(cell, wl.mask, wl.zoom, fwd)
    m = torch.nan_to_num(fwd.mean, nan=0.0)
    gb = torch.where(cnt > 0, 2.0 * (m - Tt) / (0.01 * Tt) ** 2, torch.zeros_like(m))
    ga_re = torch.empty(wl.cell.n_atoms, dtype=torch.float64, device="cuda")
    ga_keep = torch.empty_like(ga_re)
    p64.adjoint(fwd, gb, cell=cell, mask=wl.mask, grad_amp=ga_re)
    p64.simulate(cell, wl.mask, wl.zoom, fwd)
    p64.adjoint_reuse(fwd, gb, cell, wl.mask, ga_keep)
    torch.cuda.synchronize()
    a_re, a_keep = ga_re.cpu().numpy(), ga_keep.cpu().numpy()
    assert np.max(np.abs(a_re - a_keep)) <= 1e-12 * np.max(np.abs(a_re))
    # finite differences of chi^2 over every amplitude (FP64 forward)
    amp = torch.as_tensor(wl.cell.amp, device="cuda")
    h = 1e-3
    worst = 0.0
    for a_i in range(wl.cell.n_atoms):
        def La(d):
            a2 = amp.clone()
            a2[a_i] += d
            return float(chi2(BinnedIntensity.apply(a2, p64, cell, wl.mask, wl.zoom), Tt, cnt).item())
        fd = (La(h) - La(-h)) / (2 * h)
        worst = max(worst, abs(fd - a_re[a_i]) / max(1.0, abs(fd)))
        assert abs(fd - a_re[a_i]) <= 1e-6 * max(1.0, abs(fd)), (a_i, fd, a_re[a_i])
    _say(f"  1024^3 FP64: 40 amplitudes, max |fd - adjoint| / max(1, |fd|) = {worst:.3e}")
    # voxel gradient and the dot-product identity (FP64); the forward map is
    # quadratic in rho, so the central difference along v is exact up to rounding
    rho = p64.rho_generate(cell, wl.mask, wl.zoom)
    h0 = ur.Hist(wl.nbins)
    p64.simulate_rho(rho, h0)
    g64 = torch.empty_like(rho)
    p64.adjoint(h0, gb, rho=rho, grad_rho=g64)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    v = torch.randn(rho.shape, dtype=torch.float64, device="cuda", generator=gen)
    eps = 1e-4

    def means(r):
        hh = ur.Hist(wl.nbins)
        p64.simulate_rho(r, hh)
        return torch.nan_to_num(hh.mean, nan=0.0)
    mp = means((rho + eps * v).contiguous())
    mm = means((rho - eps * v).contiguous())
    lhs = float(torch.sum((mp - mm) / (2 * eps) * gb).item())
    rhs = float(torch.sum(g64 * v).item())
    _say(f"  1024^3 FP64 dot test: lhs {lhs:.12e} rhs {rhs:.12e} rel {abs(lhs - rhs) / abs(rhs):.3e}")
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), abs(rhs))
    del v, mp, mm
    # FP32 adjoint against the FP64 one at the same g_b
    p32 = ur.Plan(n, wl.voxel, 0)
    p32.set_bins(wl.edges)
    f32 = ur.Hist(wl.nbins)
    ga32 = torch.empty_like(ga_re)
    ga32k = torch.empty_like(ga_re)
    p32.simulate(cell, wl.mask, wl.zoom, f32)
    p32.adjoint(f32, gb, cell=cell, mask=wl.mask, grad_amp=ga32)
    p32.simulate(cell, wl.mask, wl.zoom, f32)
    p32.adjoint_reuse(f32, gb, cell, wl.mask, ga32k)
    rho32 = rho.float().contiguous()
    del rho
    g32 = torch.empty_like(rho32)
    p32.adjoint(f32, gb, rho=rho32, grad_rho=g32)
    torch.cuda.synchronize()
    sc = np.max(np.abs(a_re))
    e_a, e_k = np.max(np.abs(ga32.cpu().numpy() - a_re)) / sc, np.max(np.abs(ga32k.cpu().numpy() - a_re)) / sc
    e_r = float(torch.max(torch.abs(g32.double() - g64)).item() / torch.max(torch.abs(g64)).item())
    _say(f"  1024^3 FP32 vs FP64 adjoint: grad_amp {e_a:.3e} (reuse {e_k:.3e}), grad_rho {e_r:.3e}")
    assert e_a <= 1e-4 and e_k <= 1e-4 and e_r <= 1e-4
