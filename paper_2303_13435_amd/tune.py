"""Offline tuner of the compile-time choices of the transform passes.

The choices (macros of csrc/ur_tuned.hpp) fix register arrays, LDS layouts and
launch bounds, so they are compiled in, not picked at run time.  The tuner
builds one library per candidate (recompiling only the kernel parts the
candidate changes), times every candidate on the GPU on the 1024^3 box
(FP32 and FP64 forward paths, per-pass HIP events), checks that each
candidate's curve equals the default's, and writes the winners into
csrc/ur_tuned.hpp with the table of candidates and timings in
profiles/tuning_M1024.md.

    python -m paper_2303_13435_amd.tune build [MACRO ...]  # CPU: the candidate libraries (of those
                                                            # macros only, and the default)
    python -m paper_2303_13435_amd.tune run OUT.jsonl [MACRO ...]  # GPU: time them (one process per
                                                                    # library; only those macros' candidates)
    python -m paper_2303_13435_amd.tune pick OUT.jsonl [OUT2.jsonl ...]  # CPU: write ur_tuned.hpp and the table

A choice is judged on the passes it affects; choices of different passes
are picked independently (each candidate varies one macro from the default).
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
TUNED = os.path.join(CSRC, "ur_tuned.hpp")
LIBDIR = os.path.join(HERE, "tune_libs")
TABLE = os.path.join(ROOT, "profiles", "tuning_M1024.md")

# macro -> (candidate values, kernel parts of ur_kernels.hip it changes,
#           passes whose time decides it, precisions timed for it)
CHOICES = {
    "UR_X_THREADS": ((256, 128, 512), (0, 3, 4, 6), ("pass_x",), ("f32",)),
    "UR_X_THREADS_2K": ((256, 128), (3, 4), ("pass_x_2048",), ("f32",)),
    "UR_Y_HALF_2K": ((0, 1), (0, 5, 6), ("pass_y_2048", "pass_x_2048"), ("f32",)),
    "UR_X_MINW_F32": ((1, 3, 4), (3,), ("pass_x",), ("f32",)),
    "UR_X_MINW_F64": ((1, 2), (4,), ("pass_x",), ("f64",)),
    "UR_Z_PAIRS_F32": ((8, 4, 2), (0, 1, 5, 6, 7, 9), ("pass_z", "pass_y"), ("f32",)),
    "UR_ZI_PAIRS_F32": ((8, 4), (0, 5, 6), ("fwd_adjoint",), ("f32",)),
    "UR_Z_XCD": ((0, 1), (1, 7, 9), ("pass_z",), ("f32",)),
    "UR_ST_NT_A": ((1, 0), (1, 2), ("pass_z", "pass_y"), ("f32",)),
    "UR_ST_NT_B": ((1, 0), (5,), ("pass_y", "pass_x"), ("f32", "f64")),
    "UR_LD_NT": ((1, 0), (3, 4, 5), ("pass_y", "pass_x"), ("f32", "f64")),
    "UR_LD_SKIP_Y": ((1, 0), (5,), ("pass_y",), ("f32", "f64")),
    "UR_LD_SKIP_X": ((0, 1), (3, 4, 6), ("pass_x",), ("f32", "f64")),
    "UR_X_REFETCH": ((0, 1), (3, 4, 6), ("pass_x",), ("f32", "f64")),
    "UR_XADJ_REFETCH": ((1, 0), (6,), ("fwd_adjoint",), ("f32", "f64")),
}


def defaults() -> dict:
    """The values ur_tuned.hpp holds now."""
    text = open(TUNED).read()
    out = {}
    for m in CHOICES:
        v = re.search(r"#define %s (\d+)" % m, text)
        out[m] = int(v.group(1)) if v else CHOICES[m][0][0]
    return out


def candidates(macros=()):
    """(name, overrides): the default, then one macro changed at a time (of
    the named macros only, when given)."""
    base = defaults()
    out = [("default", {})]
    for m, (vals, _, _, _) in CHOICES.items():
        if macros and m not in macros:
            continue
        for v in vals:
            if v != base[m]:
                out.append((f"{m}={v}", {m: v}))
    return out


def _safe(name: str) -> str:
    return re.sub(r"[^A-Za-z0-9_.=-]", "_", name)


def build_all(macros=()) -> None:
    from . import build as B
    B.build()                                       # default objects of every source
    objdir = os.path.join(HERE, "_build")
    jobs = []
    for name, over in candidates(macros):
        if not over:
            continue
        parts = sorted({p for m in over for p in CHOICES[m][1]})
        defs = [f"-D{m}={v}" for m, v in over.items()]
        out = os.path.join(objdir, "tune", _safe(name))
        os.makedirs(out, exist_ok=True)
        for k in parts:
            jobs.append((name, "ur_kernels.hip", [f"-DUR_PART={k}"] + defs, os.path.join(out, f"ur_kernels.p{k}.o")))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        list(ex.map(lambda j: B._compile_one(j[1], j[3], j[2]), jobs))
    for name, over in candidates(macros):
        lib_dir = os.path.join(LIBDIR, _safe(name))
        os.makedirs(lib_dir, exist_ok=True)
        parts = {p for m in over for p in CHOICES[m][1]}
        objs = []
        for src in B.SOURCES:
            stem = os.path.splitext(src)[0]
            if src == "ur_kernels.hip":
                for k in range(B.KERNEL_PARTS):
                    d = os.path.join(objdir, "tune", _safe(name)) if k in parts else objdir
                    objs.append(os.path.join(d, f"{stem}.p{k}.o"))
            else:
                objs.append(os.path.join(objdir, stem + ".o"))
        lib = os.path.join(lib_dir, "libultima.so")
        r = subprocess.run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC"] + objs + ["-o", lib],
                           capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"link of {name} failed")
        with open(os.path.join(lib_dir, "candidate.json"), "w") as fh:
            json.dump({"name": name, "overrides": over}, fh)
    print(f"built {len(candidates(macros))} candidate libraries in {time.perf_counter() - t0:.0f} s under {LIBDIR}")


def measure(steps: int = 20) -> dict:
    """Per-pass timings of the M1024 forward path, FP32 and FP64, with the
    library named by UR_LIBPATH (run in a process of its own)."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import paper_2303_13435_amd as ur
    import workloads as W
    out = {}
    for tag, prec in (("f32", ur.UR_F32), ("f64", ur.UR_F64)):
        wl = W.m1024(prec)
        plan = ur.Plan(wl.n, wl.voxel, prec)
        plan.set_bins(wl.edges)
        cell = ur.DeviceCell.from_host(wl.cell)
        h = ur.Hist(wl.nbins)
        for _ in range(3):
            plan.simulate(cell, wl.mask, wl.zoom, h)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.simulate(cell, wl.mask, wl.zoom, h)
        e1.record()
        torch.cuda.synchronize()
        plan.set_timing(True)
        for _ in range(steps):
            plan.simulate(cell, wl.mask, wl.zoom, h)
        torch.cuda.synchronize()
        t = plan.read_timing()
        plan.set_timing(False)
        mean = h.mean.cpu().numpy()
        out[tag] = {"step_ms": e0.elapsed_time(e1) / steps,
                    "passes": dict({k: v["ms"] / v["launches"] for k, v in t.items() if v["launches"]},
                                   step=e0.elapsed_time(e1) / steps),
                    "mean": [float(x) for x in np.nan_to_num(mean, nan=-1.0)]}
        # forward + adjoint to the 40 amplitudes (recomputing the forward
        # passes): the inverse passes' choices are judged on it
        g_bin = torch.where(h.count > 0, torch.ones_like(h.count), torch.zeros_like(h.count))
        gamp = torch.empty(wl.cell.n_atoms, dtype=torch.float64, device="cuda")

        def fa():
            plan.simulate(cell, wl.mask, wl.zoom, h)
            plan.adjoint(h, g_bin, cell=cell, mask=wl.mask, grad_amp=gamp)
        for _ in range(2):
            fa()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps // 2):
            fa()
        e1.record()
        torch.cuda.synchronize()
        out[tag]["passes"]["fwd_adjoint"] = e0.elapsed_time(e1) / (steps // 2)
        out[tag]["grad_amp"] = [float(x) for x in gamp.cpu().numpy()]
        del plan
        torch.cuda.empty_cache()
    # the 2048^3 ED-1 level of the multi-zoom batch, FP32 (two-wavefront
    # columns): per-pass times, and its curve joins the comparison
    wl = W.c3_levels()[0]
    plan = ur.Plan(wl.n, wl.voxel, ur.UR_F32)
    plan.set_bins(wl.edges)
    cell = ur.DeviceCell.from_host(wl.cell)
    h = ur.Hist(wl.nbins)
    plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(max(3, steps // 4)):
        plan.simulate(cell, wl.mask, wl.zoom, h)
    e1.record()
    torch.cuda.synchronize()
    out["f32"]["passes"]["step_2048"] = e0.elapsed_time(e1) / max(3, steps // 4)
    plan.set_timing(True)
    for _ in range(max(3, steps // 4)):
        plan.simulate(cell, wl.mask, wl.zoom, h)
    torch.cuda.synchronize()
    t = plan.read_timing()
    plan.set_timing(False)
    for k, v in t.items():
        if v["launches"]:
            out["f32"]["passes"][k + "_2048"] = v["ms"] / v["launches"]
    out["f32"]["mean_2048"] = [float(x) for x in np.nan_to_num(h.mean.cpu().numpy(), nan=-1.0)]
    del plan
    torch.cuda.empty_cache()
    return out


def run_all(out_path: str, macros=()) -> None:
    """Times the built candidates (those of the named macros and the default
    when `macros` is given) and writes one JSON line per candidate."""
    names = sorted(os.listdir(LIBDIR)) if os.path.isdir(LIBDIR) else []
    with open(out_path, "w") as fh:
        for d in names:
            lib = os.path.join(LIBDIR, d, "libultima.so")
            meta = os.path.join(LIBDIR, d, "candidate.json")
            if not (os.path.exists(lib) and os.path.exists(meta)):
                continue
            cand = json.load(open(meta))
            if macros and cand["overrides"] and not any(m in cand["overrides"] for m in macros):
                continue
            env = dict(os.environ, UR_LIBPATH=lib)
            print(f"timing {cand['name']}", flush=True)
            r = subprocess.run([sys.executable, "-m", "paper_2303_13435_amd.tune", "measure"], cwd=ROOT, env=env,
                               capture_output=True, text=True, timeout=600)
            lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
            if r.returncode != 0 or not lines:
                rec = {"candidate": cand, "error": f"status {r.returncode}: {r.stderr[-400:]}"}
            else:
                rec = {"candidate": cand, "result": json.loads(lines[-1])}
            fh.write(json.dumps(rec) + "\n")
            fh.flush()
            msg = rec.get("error") or " ".join(f"{t}: {rec['result'][t]['step_ms']:.4f} ms" for t in ("f32", "f64"))
            print(f"  {msg}", flush=True)


def pick(results_paths) -> None:
    import numpy as np
    if isinstance(results_paths, str):
        results_paths = [results_paths]
    # one timing run per file, each with its own timing of the default: a
    # macro's candidates are judged against the default of their own run
    runs = []
    for path in results_paths:
        recs = [json.loads(ln) for ln in open(path) if ln.strip()]
        runs.append({r["candidate"]["name"]: r for r in recs if "result" in r})
    if not all("default" in run for run in runs):
        raise SystemExit("every timing run needs its timing of the default candidate")
    ref = runs[0]["default"]["result"]
    base = defaults()
    chosen = dict(base)
    rows = []
    for m, (vals, _, passes, precs) in CHOICES.items():
        best, best_t = base[m], None
        by_name = next((run for run in runs if any(k.startswith(m + "=") for k in run)), runs[0])
        ref = by_name["default"]["result"]
        for v in vals:
            name = "default" if v == base[m] else f"{m}={v}"
            r = by_name.get(name)
            if r is None:
                rows.append((m, v, None, "not timed"))
                continue
            res = r["result"]
            # the curve must be the default's (same arithmetic up to rounding order)
            ok = True
            for tg, key in (("f32", "mean"), ("f64", "mean"), ("f32", "mean_2048")):
                if key not in ref[tg] or key not in res[tg]:
                    continue
                a, b = np.array(res[tg][key]), np.array(ref[tg][key])
                pos = b > 0
                if not np.array_equal(a < 0, b < 0) or np.max(np.abs(a[pos] - b[pos]) / b[pos]) > 1e-6:
                    ok = False
                ga, gb = np.array(res[tg].get("grad_amp", [])), np.array(ref[tg].get("grad_amp", []))
                if ga.size and (ga.size != gb.size or np.max(np.abs(ga - gb)) > 1e-5 * np.max(np.abs(gb))):
                    ok = False
            t = sum(res[tg]["passes"].get(ps, 0.0) for tg in precs for ps in passes)
            rows.append((m, v, res, "" if ok else "curve differs: rejected"))
            if ok and (best_t is None or t < best_t * 0.99 or (v == base[m] and t <= best_t * 1.01)):
                best, best_t = v, t
        chosen[m] = best
    write_tuned(chosen)
    write_table(rows, chosen, ref)
    print("chosen:", chosen)


def write_tuned(chosen: dict) -> None:
    text = open(TUNED).read()
    for m, v in chosen.items():
        text = re.sub(r"#define %s \d+" % m, f"#define {m} {v}", text)
    open(TUNED, "w").write(text)


def write_table(rows, chosen, ref) -> None:
    lines = ["# Tuning of the compile-time choices: M1024 (1024^3, sphere R = 400, 512 log bins)", "",
             "Command: `python -m paper_2303_13435_amd.tune build` (CPU), then on the GPU",
             "`python -m paper_2303_13435_amd.tune run <out>.jsonl [MACRO ...]` (one or more runs, each timing the candidates of",
             "the macros it names and the default), then `python -m paper_2303_13435_amd.tune pick <out>.jsonl [<out2>.jsonl ...]`.",
             "Each candidate changes one macro of `csrc/ur_tuned.hpp` from the values it held; its library is timed in",
             "a process of its own (20 steps after 3 warm-up steps, per-pass HIP events).  A value is chosen on the",
             "passes it affects; a candidate whose curve differs from the default's by more than 1e-6 is rejected;",
             "a change must win by more than 1 %.  When the candidates were timed in several runs, each macro is",
             "judged against the default timed in its own run (its row of the current value shows that timing).", "",
             "The 2048^3 column is the ED-1 level of the multi-zoom batch (FP32, per-pass HIP events).", "",
             "| macro | value | FP32 step ms | FP32 pass Z / Y / X ms | FP32 fwd+adjoint ms | FP64 step ms | FP64 pass Z / Y / X ms | FP64 fwd+adjoint ms | 2048^3 FP32 pass Z / Y / X ms | note |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for m, v, res, note in rows:
        if res is None:
            lines.append(f"| {m} | {v} | | | | | | | | {note} |")
            continue
        cells = []
        for tg in ("f32", "f64"):
            ps = res[tg]["passes"]
            cells.append(f"{res[tg]['step_ms']:.4f}")
            cells.append(" / ".join(f"{ps.get(k, 0.0):.4f}" for k in ("pass_z", "pass_y", "pass_x")))
            cells.append(f"{ps['fwd_adjoint']:.4f}" if "fwd_adjoint" in ps else "")
        ps = res["f32"]["passes"]
        cells.append(" / ".join(f"{ps.get(k + '_2048', 0.0):.3f}" for k in ("pass_z", "pass_y", "pass_x")))
        mark = "**chosen**" if chosen[m] == v else ""
        lines.append(f"| {m} | {v} | {' | '.join(cells)} | {(mark + ' ' + note).strip()} |")
    lines += ["", "Chosen: " + ", ".join(f"`{m} = {v}`" for m, v in chosen.items())]
    os.makedirs(os.path.dirname(TABLE), exist_ok=True)
    open(TABLE, "w").write("\n".join(lines) + "\n")


def main(argv) -> None:
    if not argv:
        raise SystemExit(__doc__)
    cmd = argv[0]
    if cmd == "build":
        build_all(tuple(argv[1:]))
    elif cmd == "run":
        run_all(argv[1] if len(argv) > 1 else os.path.join(ROOT, "gpurun_out", "tune.jsonl"), tuple(argv[2:]))
    elif cmd == "measure":
        print(json.dumps(measure()))
    elif cmd == "pick":
        pick(argv[1:])
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
