#!/usr/bin/env python3
"""Benchmark of the fused ED-generation -> 3D FFT -> |F|^2 -> |Q|-bin path.

Workload (default): the 1024^3 FP32 headline box -- a 16-voxel cubic unit
cell holding 40 seeded Gaussian atoms, tiled and masked by a sphere of radius
400 voxels, r2c transform, 512 log-spaced |Q| bins.  Synthetic data stands in
for the paper's DFT electron density of a ZIF-8 unit cell.

A step is one call of the fused forward path on inputs already resident in
HBM: cell synthesis from the atoms, the generating z pass, the y pass, the x
pass with |F|^2 and binning, and the fixed-order finalize.  The line printed
also carries, for the same box, the FP64 path and the forward+adjoint time,
the roofline of the dominant kernel (per-pass HIP events on the launch
stream, algorithmic bytes from the pruned geometry) and the FP64 CPU oracle
timed on this host on a bounded sample of the workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
PROFILES = os.path.join(ROOT, "profiles")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("ur_kernels.hip", "ur_device.hpp", "ur_geom.hpp", "ur_kernels.hpp", "ur_tuned.hpp"):
        with open(os.path.join(ROOT, "paper_2303_13435_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when absent or taken from different kernel sources."""
    path = os.path.join(PROFILES, f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def cpu_baseline(wl, got32=None, got64=None):
    """The FP64 oracle, as it stands, on the benchmarked box itself (density
    -> eq. 1 -> binning of the whole 1024^3 box; FFT lines on every OpenMP
    thread, binning on one), reported as voxels/s; the same path on C4
    (256^3) with one thread; and, from the oracle's result, the accuracy of
    the GPU curves of the same box (FP32 and FP64): max relative error over
    the populated bins, Parseval and F(0) errors."""
    import numpy as np
    import oracle
    import workloads as W
    oracle.lib()
    nthr = oracle.num_threads()
    t0 = time.perf_counter()
    ref = oracle.simulate(wl)
    dt = time.perf_counter() - t0
    note(f"oracle {wl.name}: {dt:.1f} s on {nthr} threads")
    c4 = W.c4()
    oracle.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.simulate(c4)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(nthr)
    note(f"oracle C4 on 1 thread: {dt1:.1f} s")
    n3 = float(wl.n) ** 3
    acc = {}
    for tag, got in (("f32", got32), ("f64", got64)):
        if got is None:
            continue
        pop = ref["count"] > 0
        rel = np.abs(got["mean"][pop] - ref["mean"][pop]) / np.abs(ref["mean"][pop])
        acc[tag] = {"counts_equal": bool(np.array_equal(got["count"], ref["count"])),
                    "max_rel_err": float(rel.max()), "median_rel_err": float(np.median(rel)),
                    "bins_above_1e-5": int(np.sum(rel > 1e-5)), "bins": int(pop.sum()),
                    "parseval_rel_err": float(abs(got["totals"][0] - ref["rho_sumsq"] / n3) / (ref["rho_sumsq"] / n3)),
                    "f0_rel_err": float(abs(got["totals"][1] - ref["rho_sum"] / n3) / abs(ref["rho_sum"] / n3))}
    return {"value": wl.n ** 3 / dt, "unit": "voxels/s", "cores": nthr, "kind": "oracle",
            "sample": f"the whole {wl.name} box ({wl.n}^3, 512 log bins): density, eq. 1 by recursive radix-2 "
                      f"lines on {nthr} OpenMP threads, binning on one thread; {dt:.1f} s",
            "one_thread": {"workload": "C4 256^3 whole path", "s": round(dt1, 2),
                           "voxels_per_s": c4.n ** 3 / dt1},
            "gpu_accuracy_vs_oracle": acc,
            "host": host_info()}


def host_info():
    """CPU model, logical CPUs and memory of the host the oracle ran on."""
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def c3_batch(ur, W, torch, reps):
    """The multi-zoom batch (ED-1 2048^3, ED-2 1024^3 by 4, ED-3 512^3 by 16
    and the merge) recorded in one HIP graph and replayed: the two coarse
    levels run on a second stream beside the ED-1 level (a fork and a join
    in the graph), the merge after both.  The merged curve of the replays is
    checked against the three levels run one after the other, eagerly."""
    levels = W.c3_levels()
    s = torch.cuda.Stream()
    s2 = torch.cuda.Stream()
    plans, hists, cells = [], [], []
    for wl in levels:
        p = ur.Plan(wl.n, wl.voxel, ur.UR_F32)
        p.set_bins(wl.edges)
        plans.append(p)
        hists.append(ur.Hist(wl.nbins))
        cells.append(ur.DeviceCell.from_host(wl.cell))
    edges = torch.as_tensor(levels[0].edges, device="cuda")
    ns, vox = [w.n for w in levels], [w.voxel for w in levels]
    nb = levels[0].nbins
    outs = (torch.empty(nb, dtype=torch.float64, device="cuda"), torch.empty(nb, dtype=torch.float64, device="cuda"),
            torch.empty(nb, dtype=torch.int32, device="cuda"))

    def run(concurrent):
        if not concurrent:
            for p, h, c, wl in zip(plans, hists, cells, levels):
                p.simulate(c, wl.mask, wl.zoom, h, stream=s)
            return ur.merge_zooms(hists, ns, vox, edges, ur.MERGE_FINEST, 32.0, stream=s, out=outs)
        fork = torch.cuda.Event(enable_timing=False)
        join = torch.cuda.Event(enable_timing=False)
        fork.record(s)
        s2.wait_event(fork)
        for p, h, c, wl in zip(plans[1:], hists[1:], cells[1:], levels[1:]):
            p.simulate(c, wl.mask, wl.zoom, h, stream=s2)
        plans[0].simulate(cells[0], levels[0].mask, levels[0].zoom, hists[0], stream=s)
        join.record(s2)
        s.wait_event(join)
        return ur.merge_zooms(hists, ns, vox, edges, ur.MERGE_FINEST, 32.0, stream=s, out=outs)

    with torch.cuda.stream(s):
        run(False)                                      # allocates workspaces
    torch.cuda.synchronize()
    want = outs[0].cpu().numpy().copy()
    g = ur.Graph(s)
    with torch.cuda.stream(s):
        with g:
            run(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    g.launch()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        g.launch()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    got = outs[0].cpu().numpy()
    import numpy as np
    fin = np.isfinite(want)
    same = bool(np.array_equal(fin, np.isfinite(got)) and
                np.allclose(got[fin], want[fin], rtol=1e-11, atol=0.0))
    vox_total = sum(w.n ** 3 for w in levels)
    out = {"ms_per_batch": round(ms, 3), "boxes": [f"{w.n}^3 f{w.zoom.factor}" for w in levels],
           "voxels_per_s": vox_total / (ms * 1e-3), "graph_launches": reps,
           "coarse_levels_on_second_stream": True, "curve_matches_sequential_eager": same}
    del g, plans, hists
    torch.cuda.empty_cache()
    return out


def radii_batch(ur, W, torch, reps, count=32, ensemble=False):
    """`count` particle radii (256^3 FP32 boxes, spheres R = 20..100) through
    one plan, recorded in one HIP graph and replayed; with `ensemble`, the
    polydisperse curve of the boxes (log-normal volume fractions) is formed
    in the same graph."""
    import math
    import numpy as np
    levels = W.b_radii(count=count)
    s = torch.cuda.Stream()
    plan = ur.Plan(levels[0].n, 1.0, ur.UR_F32)
    plan.set_bins(levels[0].edges)
    cell = ur.DeviceCell.from_host(levels[0].cell)
    batch = ur.HistBatch(len(levels), levels[0].nbins)
    hists = batch.hists
    radii = [math.sqrt(float(wl.mask.p0)) for wl in levels]
    phi = W.volume_fractions(radii, float(np.median(radii)), 0.4)
    wt = torch.as_tensor(phi / np.array([(4.0 / 3.0) * math.pi * r ** 3 for r in radii]), device="cuda")
    out = (torch.empty(batch.nbins, dtype=torch.float64, device="cuda"),
           torch.empty(batch.nbins, dtype=torch.float64, device="cuda"))

    def run():
        for wl, h in zip(levels, hists):
            plan.simulate(cell, wl.mask, wl.zoom, h, stream=s)
        if ensemble:
            ur.ensemble(batch, wt, out=out, stream=s)

    with torch.cuda.stream(s):
        run()
    torch.cuda.synchronize()
    g = ur.Graph(s)
    with torch.cuda.stream(s):
        with g:
            run()
    g.launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        g.launch()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out = {"ms_per_batch": round(ms, 3), "boxes": len(levels), "box": levels[0].n,
           "radii": [round(float(w.mask.p0) ** 0.5, 1) for w in (levels[0], levels[-1])],
           "voxels_per_s": len(levels) * levels[0].n ** 3 / (ms * 1e-3), "graph_launches": reps,
           "ensemble": ensemble}
    del g, plan, hists, batch
    torch.cuda.empty_cache()
    return out


def fill_host(ur, torch, plan, cell, wl, x_lo, x_hi, pinned, chunk=64):
    """Planes x_lo..x_hi of the density in host memory (exactly-sized pinned
    memory, or pageable memory when it exceeds what may be page-locked),
    generated on the device chunk by chunk (a 4096^3 box does not fit HBM).
    Returns (tensor, buffer to close or None)."""
    shape = (x_hi - x_lo + 1, wl.n, wl.n)
    hb = ur.HostBuffer(shape, torch.float32) if pinned else None
    host = hb.tensor if pinned else torch.empty(shape, dtype=torch.float32)
    for a in range(x_lo, x_hi + 1, chunk):
        b = min(a + chunk - 1, x_hi)
        host[a - x_lo:b - x_lo + 1].copy_(plan.rho_generate(cell, wl.mask, wl.zoom, x_lo=a, x_hi=b))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return host, hb


def mask_planes(W, wl):
    """Planes that can hold density: half-width of the mask (sphere: sqrt of
    the squared radius; cube and truncated octahedron: p0) about n/2."""
    import math
    r = math.isqrt(int(wl.mask.p0)) if wl.mask.kind == W.MASK_SPHERE else int(wl.mask.p0)
    return wl.n // 2 - r, wl.n // 2 + r


def pass_timing(plan, step, steps, torch):
    """Per-pass average duration (HIP events on the launch stream) and
    algorithmic bytes / GB/s of `steps` calls of `step` on `plan`."""
    plan.set_timing(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    passes = plan.read_timing()
    plan.set_timing(False)
    kernels = {}
    for name, d in passes.items():
        if d["launches"] == 0:
            continue
        avg = d["ms"] / d["launches"]
        kernels[name] = {"avg_ms": round(avg, 5), "alg_bytes": d["bytes"],
                         "alg_GBps": round(d["bytes"] / (avg * 1e-3) / 1e9, 1) if avg > 0 else None}
    return kernels


def other_configs(ur, W, torch, steps):
    """The forward path on the other single-box configurations: C1 (64^3
    FP64, full complex transform), C2 (512^3 FP32), C4 (256^3, FP32 and
    FP64); ms per box and voxels/s, inputs resident."""
    from dataclasses import replace
    out = {}
    for wl in (W.c1(), W.c2(), W.c4(), replace(W.c4(), name="C4_f64", prec=ur.UR_F64)):
        plan = ur.Plan(wl.n, wl.voxel, wl.prec, c2c=wl.transform == "c2c")
        plan.set_bins(wl.edges)
        cell = ur.DeviceCell.from_host(wl.cell)
        h = ur.Hist(wl.nbins)
        ms, _ = time_steps(lambda: plan.simulate(cell, wl.mask, wl.zoom, h), steps, 3, torch)
        out[wl.name] = {"ms_per_box": round(ms, 4), "voxels_per_s": wl.n ** 3 / (ms * 1e-3),
                        "prec": "f64" if wl.prec == ur.UR_F64 else "f32", "transform": wl.transform}
        del plan
    torch.cuda.empty_cache()
    return out


def mixed_radix(ur, W, torch, steps):
    """Boxes whose edge is not a power of two (the paper's 1000 / 2000 family):
    the mixed-radix forward path (one axis at a time; real plans pair two
    real pencils per z line and keep the half spectrum, complex plans the
    whole box) on the M1024 recipe scaled to the edge; ms per box, voxels/s
    and per-pass timing."""
    out = {}
    for n, prec, c2c in ((1000, ur.UR_F32, False), (1000, ur.UR_F64, False), (2000, ur.UR_F32, False),
                         (1000, ur.UR_F32, True), (1000, ur.UR_F64, True), (2000, ur.UR_F32, True)):
        wl = W.mixed(n, prec, nbins=512)
        plan = ur.Plan(wl.n, wl.voxel, prec, c2c=c2c)
        plan.set_bins(wl.edges)
        cell = ur.DeviceCell.from_host(wl.cell)
        h = ur.Hist(wl.nbins)
        step = lambda: plan.simulate(cell, wl.mask, wl.zoom, h)
        ms, _ = time_steps(step, steps, 2, torch)
        out[wl.name + ("_c2c" if c2c else "")] = {
            "ms_per_box": round(ms, 4), "voxels_per_s": wl.n ** 3 / (ms * 1e-3),
            "prec": "f64" if prec == ur.UR_F64 else "f32", "transform": "c2c" if c2c else "r2c",
            "kernels": pass_timing(plan, step, steps, torch)}
        del plan, step
        torch.cuda.empty_cache()
        note(f"mixed radix {wl.name} done")
    return out


def c4_fwd_adjoint(ur, W, torch, steps):
    """C4 (256^3 FP32, 40 atoms, sphere R = 100, 256 log bins): one forward
    call plus the adjoint to both the voxel density and the 40 amplitudes
    (recomputing the forward passes), and forward plus the amplitude
    adjoint from the held y-pass output; ms per step."""
    import numpy as np
    wl = W.c4()
    plan = ur.Plan(wl.n, wl.voxel, ur.UR_F32)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    d = h.numpy()
    g_bin = torch.as_tensor(np.where(d["count"] > 0, 1.0, 0.0), device="cuda")
    grho = torch.empty((wl.n,) * 3, dtype=torch.float32, device="cuda")
    gamp = torch.empty(wl.cell.n_atoms, dtype=torch.float64, device="cuda")

    def both():
        plan.simulate(cell, wl.mask, wl.zoom, h)
        plan.adjoint(h, g_bin, cell=cell, mask=wl.mask, grad_rho=grho, grad_amp=gamp)

    def keep():
        plan.simulate(cell, wl.mask, wl.zoom, h)
        plan.adjoint_reuse(h, g_bin, cell, wl.mask, gamp)

    ms_fwd, _ = time_steps(lambda: plan.simulate(cell, wl.mask, wl.zoom, h), steps, 3, torch)
    ms_both, _ = time_steps(both, steps, 3, torch)
    ms_keep, _ = time_steps(keep, steps, 3, torch)
    del plan, grho
    torch.cuda.empty_cache()
    return {"forward_ms": round(ms_fwd, 4), "fwd_adjoint_rho_and_amp_ms": round(ms_both, 4),
            "fwd_adjoint_amp_from_held_output_ms": round(ms_keep, 4)}


def rotated_lattices(ur, W, torch, plan, wl, hist, steps):
    """The M1024 box with its lattice rotated (trilinear and cubic B-spline
    periodic sampling of the cell) and as a polycrystal of 16 grains."""
    out = {}
    n = max(3, steps // 2)
    # the same box with its lattice rotated (trilinear periodic sampling of the cell)
    rcell = ur.DeviceCell.from_host(wl.cell.with_rot(W.rotation([1.0, 2.0, 3.0], 0.7)))
    msr, _ = time_steps(lambda: plan.simulate(rcell, wl.mask, wl.zoom, hist), n, 2, torch)
    out["rotated_lattice"] = {"ms_per_step": round(msr, 4), "voxels_per_s": wl.n ** 3 / (msr * 1e-3),
                              "pass_z_ms": pass_timing(plan, lambda: plan.simulate(rcell, wl.mask, wl.zoom, hist),
                                                       5, torch)["pass_z"]["avg_ms"]}
    # a polycrystalline particle: 16 grains of random orientation (trilinear)
    gs, gr = W.random_grains(16, 16, 0.35 * wl.n)
    gcell = ur.DeviceCell.from_host(wl.cell.with_grains(gs, gr, 1))
    msg, _ = time_steps(lambda: plan.simulate(gcell, wl.mask, wl.zoom, hist), n, 2, torch)
    out["polycrystal_16_grains"] = {"ms_per_step": round(msg, 4), "voxels_per_s": wl.n ** 3 / (msg * 1e-3)}
    # the same with the cell sampled by the cubic B-spline (64 coefficients per voxel)
    ccell = ur.DeviceCell.from_host(wl.cell.with_rot(W.rotation([1.0, 2.0, 3.0], 0.7), 3))
    msc, _ = time_steps(lambda: plan.simulate(ccell, wl.mask, wl.zoom, hist), n, 2, torch)
    out["rotated_lattice_cubic"] = {"ms_per_step": round(msc, 4), "voxels_per_s": wl.n ** 3 / (msc * 1e-3),
                                    "pass_z_ms": pass_timing(plan, lambda: plan.simulate(ccell, wl.mask, wl.zoom, hist),
                                                             5, torch)["pass_z"]["avg_ms"]}
    # forward + amplitude gradients (chi^2 bin weights of one) of the rotated
    # lattice and of the polycrystal: the adjoint recomputes passes Z and Y
    # and folds through the sampler's transpose
    import numpy as np
    plan.simulate(rcell, wl.mask, wl.zoom, hist)
    g_bin = torch.as_tensor(np.where(hist.numpy()["count"] > 0, 1.0, 0.0), device="cuda")
    gamp = torch.empty(wl.cell.n_atoms, dtype=torch.float64, device="cuda")
    for key, dc in (("rotated_fwd_adjoint_ms", rcell), ("polycrystal_fwd_adjoint_ms", gcell)):
        def fa(dc=dc):
            plan.simulate(dc, wl.mask, wl.zoom, hist)
            plan.adjoint(hist, g_bin, cell=dc, mask=wl.mask, grad_amp=gamp)
        ms, _ = time_steps(fa, n, 2, torch)
        out[key] = round(ms, 4)
    return out


def fwd_adjoint(ur, W, torch, plan, cell, wl, hist, steps):
    """Forward + adjoint (chi^2 gradient w.r.t. the atom amplitudes), FP32, at
    the headline box (recomputing passes Z and Y, and from the held y-pass
    output), then the 256^3 differentiable configuration."""
    import numpy as np
    out = {}
    plan.simulate(cell, wl.mask, wl.zoom, hist)
    d = hist.numpy()
    g_bin = torch.as_tensor(np.where(d["count"] > 0, 1.0, 0.0), device="cuda")
    gamp = torch.empty(wl.cell.n_atoms, dtype=torch.float64, device="cuda")

    def fwd_adj():
        plan.simulate(cell, wl.mask, wl.zoom, hist)
        plan.adjoint(hist, g_bin, cell=cell, mask=wl.mask, grad_amp=gamp)

    ms_fa, _ = time_steps(fwd_adj, max(3, steps // 2), 2, torch)
    out["fwd_adjoint_ms"] = round(ms_fa, 4)

    def fwd_adj_keep():
        plan.simulate(cell, wl.mask, wl.zoom, hist)
        plan.adjoint_reuse(hist, g_bin, cell, wl.mask, gamp)

    ms_fk, _ = time_steps(fwd_adj_keep, max(3, steps // 2), 2, torch)
    out["fwd_adjoint_keep_ms"] = round(ms_fk, 4)       # adjoint from the held y-pass output
    note("fwd_adjoint_keep_ms done")
    out["c4_fwd_adjoint"] = c4_fwd_adjoint(ur, W, torch, steps)
    return out


def note(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"# {msg}", file=sys.stderr, flush=True)


def out_of_core(ur, W, torch, wl, reps, pinned=True):
    """A box with its density in host memory: only the planes that hold
    density are copied, slab by slab, overlapped with the z and y passes
    (eq. 2 split); reports the PCIe-inclusive rate.  pinned=False keeps the
    density in pageable memory (the plan's pinned bounce slabs carry it)."""
    plan = ur.Plan(wl.n, wl.voxel, ur.UR_F32)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    x_lo, x_hi = mask_planes(W, wl)
    t_fill = time.perf_counter()
    host, hb = fill_host(ur, torch, plan, cell, wl, x_lo, x_hi, pinned)
    t_fill = time.perf_counter() - t_fill
    note(f"out-of-core {wl.name}: host density filled in {t_fill:.1f} s")
    h = ur.Hist(wl.nbins)
    nbytes = plan.simulate_host(host, x_lo, x_hi, h)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(reps):
        plan.simulate_host(host, x_lo, x_hi, h)
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    ms = e0.elapsed_time(e1) / reps
    out = {"ms_per_box": round(ms, 3), "h2d_bytes": nbytes, "pcie_GBps": round(nbytes / (ms * 1e-3) / 1e9, 2),
           "voxels_per_s_pcie_inclusive": wl.n ** 3 / (ms * 1e-3), "wall_ms": round(wall * 1e3, 3),
           "planes": [x_lo, x_hi], "host_fill_s": round(t_fill, 1), "host_memory": "pinned" if pinned else "pageable"}
    del host, plan
    if hb is not None:
        hb.close()
    torch.cuda.empty_cache()
    return out


def ooc4096_child(flag="--ooc4096-only"):
    """Run `bench.py --ooc4096-only` (or `--ooc4000-only`) as a child process
    (its progress notes go to this process's stderr) and return its result,
    or an error record."""
    import subprocess
    note(f"out-of-core {flag} in a child process")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), flag], stdout=subprocess.PIPE,
                           text=True, timeout=900)
    except subprocess.TimeoutExpired:
        return {"error": "timed out after 900 s"}
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"child exited with status {r.returncode}"}
    return json.loads(lines[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64 and adjoint measurements")
    ap.add_argument("--n", type=int, default=1024, help="box edge (1024 = the headline workload)")
    ap.add_argument("--no-ooc4096", action="store_true",
                    help="skip the 4096^3 out-of-core box (212 GiB of host memory, about 90 s, in a child process)")
    ap.add_argument("--ooc4000-only", action="store_true",
                    help="only stream the out-of-core recipe at the paper's ED-1 edge 4000 (real mixed-radix plan) "
                         "and print its result (the child of the full run)")
    ap.add_argument("--mixed-radix-only", action="store_true",
                    help="time only the mixed-radix boxes (1000^3, 2000^3) and print their JSON")
    ap.add_argument("--ooc4096-only", action="store_true",
                    help="only stream the 4096^3 out-of-core box and print its result (the child of the full run)")
    ap.add_argument("--only", choices=("adjoint", "c3", "rotated"),
                    help="time only one part and print its JSON: the forward + adjoint measurements "
                         "(1024^3 and 256^3), the multi-zoom batch (2048^3 + 1024^3 f4 + 512^3 f16) or the "
                         "rotated and polycrystalline lattices (1024^3)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              f"(the path runs on a single MI355X; sharding over several GPUs is described, not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")     # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "launches": 3}))
        return
    import paper_2303_13435_amd as ur
    import workloads as W
    if not os.path.exists(ur.LIBPATH):
        from paper_2303_13435_amd import build as _b
        _b.build()
    if args.ooc4096_only:
        # the out-of-core workload itself: 4096^3, 3399 planes (212 GiB, more
        # than a process may page-lock here: pageable memory through the
        # bounce slabs), 229 GB of spectrum in HBM
        print(json.dumps(out_of_core(ur, W, torch, W.c5(4096), 2, pinned=False)))
        return
    if args.ooc4000_only:
        # the out-of-core recipe at 4000^3 (2^5 5^3): truncated octahedron
        # R = 1855, pageable host memory, half spectrum of its planes in HBM
        print(json.dumps(out_of_core(ur, W, torch, W.c5(4000), 2, pinned=False)))
        return
    if args.mixed_radix_only:
        # the mixed-radix boxes alone (M1000 FP32/FP64, M2000 FP32)
        print(json.dumps(mixed_radix(ur, W, torch, max(2, args.steps // 4))))
        return

    if args.only == "c3":
        print(json.dumps(c3_batch(ur, W, torch, max(2, args.steps // 4))))
        return

    n = args.n
    wl = W.m1024() if n == 1024 else W.lattice_sphere(f"S{n}", n, 16, 40, 2, 400.0 * n / 1024, 512)
    plan = ur.Plan(wl.n, wl.voxel, ur.UR_F32)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    hist = ur.Hist(wl.nbins)
    step = lambda: plan.simulate(cell, wl.mask, wl.zoom, hist)
    if args.only == "adjoint":
        print(json.dumps(fwd_adjoint(ur, W, torch, plan, cell, wl, hist, args.steps)))
        return
    if args.only == "rotated":
        print(json.dumps(rotated_lattices(ur, W, torch, plan, wl, hist, args.steps)))
        return
    ms, wall = time_steps(step, args.steps, args.warmup, torch)
    value = wl.n ** 3 / (ms * 1e-3)
    got32, got64 = hist.numpy(), None

    # per-pass timing (HIP events on the launch stream) and algorithmic bytes
    kernels = pass_timing(plan, step, args.steps, torch)
    dom = max((k for k in kernels if k.startswith("pass_")), key=lambda k: kernels[k]["avg_ms"])
    dk = kernels[dom]
    achieved = dk["alg_GBps"]
    traffic = measured_traffic(dom, wl.name)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic}
    path_bytes = sum(kernels[k]["alg_bytes"] for k in kernels)
    path_ms = sum(kernels[k]["avg_ms"] for k in kernels)
    # the whole path: bytes summed over the passes / kernel time summed over
    # the passes (counter-measured bytes when every transform pass has a
    # summary taken from the current kernel sources)
    counted = {k: measured_traffic(k, wl.name) for k in ("pass_z", "pass_y", "pass_x")}
    roofline_path = {"kernel_ms": round(path_ms, 4), "step_ms": round(ms, 4),
                     "alg_bytes": path_bytes, "alg_GBps": round(path_bytes / (path_ms * 1e-3) / 1e9, 1),
                     "alg_frac": round(path_bytes / (path_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "counter_bytes": None, "counter_frac": None, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    if all(v is not None for v in counted.values()):
        cb = sum(counted.values()) + sum(kernels[k]["alg_bytes"] for k in kernels if k not in counted)
        roofline_path["counter_bytes"] = cb
        roofline_path["counter_frac"] = round(cb / (path_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)

    extras = {"kernels": kernels, "path_alg_bytes": path_bytes,
              "path_alg_GBps": round(path_bytes / (ms * 1e-3) / 1e9, 1),
              "sum_kernel_ms": round(path_ms, 4)}
    if not args.no_extras:
        # FP64 path on the same box
        p64 = ur.Plan(wl.n, wl.voxel, ur.UR_F64)
        p64.set_bins(wl.edges)
        h64 = ur.Hist(wl.nbins)
        ms64, _ = time_steps(lambda: p64.simulate(cell, wl.mask, wl.zoom, h64), max(3, args.steps // 2), 2, torch)
        got64 = h64.numpy()
        extras.update(rotated_lattices(ur, W, torch, plan, wl, hist, args.steps))
        extras["fp64"] = {"ms_per_step": round(ms64, 4), "voxels_per_s": wl.n ** 3 / (ms64 * 1e-3),
                          "kernels": pass_timing(p64, lambda: p64.simulate(cell, wl.mask, wl.zoom, h64), args.steps, torch)}
        note("fp64 done")
        del p64
        extras.update(fwd_adjoint(ur, W, torch, plan, cell, wl, hist, args.steps))
        note("c4 forward + adjoint done")
        torch.cuda.synchronize()
        # Ewald-sphere image of the same box: 1024 x 1024 pixels, 16
        # wavelength nodes (2 % spread), from the transform held in HBM
        spec = plan.fft3d(plan.rho_generate(cell, wl.mask, wl.zoom))
        geo = W.detector(W.rotation([0.0, 1.0, 0.0], 0.3), rel_spread=0.02, n_lambda=16, distance=1000.0,
                         pixel=0.05, nu=1024, nv=1024)
        img = torch.empty((geo.nv, geo.nu), dtype=torch.float64, device="cuda")
        ms_ew, _ = time_steps(lambda: plan.ewald_image(spec, geo, out=img), max(3, args.steps), 2, torch)
        extras["ewald_image"] = {"pixels": geo.nu * geo.nv, "n_lambda": geo.n_lambda, "ms": round(ms_ew, 4),
                                 "samples_per_s": geo.nu * geo.nv * geo.n_lambda / (ms_ew * 1e-3)}
        del spec, img
        torch.cuda.empty_cache()
        note("ewald_image done")
        # multi-zoom batch: ED-1 2048^3 + ED-2 1024^3 (f 4) + ED-3 512^3 (f 16)
        # and the merge, recorded in one HIP graph and replayed
        extras["c3_batch"] = c3_batch(ur, W, torch, max(2, args.steps // 4))
        note("c3_batch done")
        # many particle sizes: 32 radii of 256^3 boxes in one graph
        extras["radii_batch"] = radii_batch(ur, W, torch, max(2, args.steps // 4))
        # the paper's polydispersity estimate: 200 radii and their ensemble curve, one graph
        extras["ensemble_200"] = radii_batch(ur, W, torch, max(2, args.steps // 4), count=200, ensemble=True)
        # the other single-box configurations
        extras["configs"] = other_configs(ur, W, torch, args.steps)
        extras["mixed_radix"] = mixed_radix(ur, W, torch, max(2, args.steps // 4))
        note("configs done")
        note("radii_batch done")
        # out-of-core: the same box streamed from pinned host memory
        extras["out_of_core"] = out_of_core(ur, W, torch, wl, max(2, args.steps // 4))
        # the same from pageable host memory (pinned bounce slabs)
        extras["out_of_core_pageable"] = out_of_core(ur, W, torch, wl, 2, pinned=False)
        torch.cuda.empty_cache()
        # out-of-core at 2048^3 with the truncated-octahedron recipe of the
        # out-of-core workload
        extras["out_of_core_c5_2048"] = out_of_core(ur, W, torch, W.c5(2048), 2)
        if not args.no_ooc4096:
            # the out-of-core workload at its own size, in a child process: a
            # failure there (host memory refused) is reported, not fatal
            del plan
            torch.cuda.empty_cache()
            extras["out_of_core_c5_4096"] = ooc4096_child()
            # the same recipe at the paper's ED-1 edge, 4000 (mixed radix)
            extras["out_of_core_c5_4000_mixed"] = ooc4096_child("--ooc4000-only")

    cpu = None
    if not args.no_cpu_baseline:
        if n != 1024:
            note("the CPU baseline runs the 1024^3 box only")
        else:
            cpu = cpu_baseline(W.m1024(), got32, got64)

    line = {
        "metric": "voxels/s, FFT->|F|^2->Q-bin at 1024^3 FP32 (FP64 and fwd+adjoint ms in extras)",
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.n}^3 FP32 r2c, 16-voxel cell x 40 Gaussian atoms (seed 2), "
                               f"sphere R={int(round(400 * n / 1024))}, {wl.nbins} log |Q| bins",
                   "box": wl.n, "nbins": wl.nbins, "parallelism": "single GPU"},
        "roofline": roofline,
        "roofline_path": roofline_path,
        "cpu_baseline": cpu,
        "extras": extras,
        "wall_s": round(wall, 3),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
