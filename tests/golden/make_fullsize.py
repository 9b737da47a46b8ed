"""Per-bin statistics of the full-size workloads from the FP64 oracle.

Writes tests/golden/fullsize_<name>.npz for the boxes whose whole oracle run
takes minutes and tens of GB of host memory (M1024, the C3 zoom levels ED-2
1024^3 / f 4 and ED-3 512^3 / f 16, the mixed-radix M1000): count, sum,
sumsq, mean, sem, totals and the density moments, plus `sources`, a hash of
the oracle and workload sources they were computed from.  The GPU tests use
a file only when its hash matches the current sources and otherwise run the
oracle themselves, so a stale file can never stand in for the oracle.

Only oracle/ and workloads/ are called here.

    python tests/golden/make_fullsize.py [name ...]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

FIELDS = ("count", "sum", "sumsq", "mean", "sem", "totals")


def sources_hash() -> str:
    """Hash of every source the oracle's result depends on."""
    h = hashlib.sha256()
    for rel in ("oracle/ur_oracle.c", "oracle/__init__.py", "workloads/__init__.py"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:24]


def workload(name: str):
    if name == "M1024":
        return W.m1024(W.PREC_F64)
    if name in ("C3-ED2", "C3-ED3"):
        return {w.name: w for w in W.c3_levels()}[name]
    if name == "M1000":
        return W.mixed(1000, W.PREC_F64, nbins=512)
    raise KeyError(name)


NAMES = ("M1024", "C3-ED2", "C3-ED3", "M1000")


def path(name: str) -> str:
    return os.path.join(HERE, f"fullsize_{name}.npz")


def compute(name: str) -> dict:
    """The whole oracle path of one workload (density, eq. 1, binning)."""
    r = oracle.simulate(workload(name))
    out = {k: np.asarray(r[k], dtype=np.float64) for k in FIELDS}
    out["rho_sum"] = np.float64(r["rho_sum"])
    out["rho_sumsq"] = np.float64(r["rho_sumsq"])
    return out


def load(name: str):
    """The stored result when it was computed from the current sources, else None."""
    p = path(name)
    if not os.path.exists(p):
        return None
    with np.load(p, allow_pickle=False) as z:
        if str(z["sources"]) != sources_hash():
            return None
        return {k: z[k] for k in z.files if k != "sources"}


def main(names) -> None:
    oracle.lib()
    for name in names:
        t0 = time.perf_counter()
        res = compute(name)
        np.savez(path(name), sources=np.array(sources_hash()), **res)
        print(f"{name}: {time.perf_counter() - t0:.1f} s on {oracle.num_threads()} threads -> {path(name)}",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or NAMES)
