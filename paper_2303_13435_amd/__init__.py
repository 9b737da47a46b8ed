"""Python binding of the gfx950 wide-range scattering simulator.

Thin ctypes marshalling over ``include/ultima.h``: torch tensors supply
device memory and the current HIP stream; every step of the computation runs
in the HIP kernels of ``libultima.so``.  There is no CPU fallback: when the
library is missing, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree library; UR_LIBPATH names another build of it (the tuner's
# candidate libraries, each timed in a process of its own)
LIBPATH = os.environ.get("UR_LIBPATH") or os.path.join(HERE, "libultima.so")

UR_F32, UR_F64 = 0, 1
UR_R2C, UR_C2C = 0, 1
MERGE_FINEST, MERGE_POOLED, MERGE_IVW = 0, 1, 2
MAX_IN_CORE, MAX_OUT_OF_CORE = 2048, 4096     # box edges (include/ultima.h, ur_plan_create)

_c = ctypes
_vp = _c.c_void_p


class UrMask(_c.Structure):
    _fields_ = [("kind", _c.c_int32), ("p0", _c.c_int64), ("p1", _c.c_int64)]


class UrCell(_c.Structure):
    _fields_ = [("c", _c.c_int32), ("n_atoms", _c.c_int32), ("xyz", _vp), ("amp", _vp),
                ("sigma", _vp), ("background", _c.c_double), ("rot", _c.POINTER(_c.c_double)),
                ("interp", _c.c_int32), ("n_grains", _c.c_int32), ("grain_seed", _c.POINTER(_c.c_double)),
                ("grain_rot", _c.POINTER(_c.c_double))]


class UrZoom(_c.Structure):
    _fields_ = [("n1", _c.c_int32), ("factor", _c.c_int32)]


class UrHist(_c.Structure):
    _fields_ = [("sum", _vp), ("sumsq", _vp), ("count", _vp), ("totals", _vp), ("mean", _vp), ("sem", _vp)]


class UrEwald(_c.Structure):
    _fields_ = [("wavelength", _c.c_double), ("rel_spread", _c.c_double), ("n_lambda", _c.c_int32),
                ("beam", _c.c_double * 3), ("du", _c.c_double * 3), ("dv", _c.c_double * 3),
                ("distance", _c.c_double), ("pixel", _c.c_double), ("cu", _c.c_double), ("cv", _c.c_double),
                ("nu", _c.c_int32), ("nv", _c.c_int32)]

    @classmethod
    def from_geometry(cls, g) -> "UrEwald":
        return cls(float(g.wavelength), float(g.rel_spread), int(g.n_lambda), (_c.c_double * 3)(*g.beam),
                   (_c.c_double * 3)(*g.du), (_c.c_double * 3)(*g.dv), float(g.distance), float(g.pixel),
                   float(g.cu), float(g.cv), int(g.nu), int(g.nv))


_LIB = None

# (name, argtypes)
_SIGS = {
    "ur_plan_create": [_c.c_int32, _c.c_double, _c.c_int32, _c.c_uint32, _c.POINTER(_vp)],
    "ur_plan_destroy": [_vp],
    "ur_plan_workspace_size": [_vp, _c.c_int32, _c.POINTER(_c.c_size_t)],
    "ur_plan_workspace_size_host": [_vp, _c.c_int32, _c.c_int32, _c.c_int32, _c.POINTER(_c.c_size_t)],
    "ur_plan_set_workspace": [_vp, _vp, _c.c_size_t],
    "ur_plan_set_hbm_budget": [_vp, _c.c_size_t],
    "ur_plan_set_voxel_form": [_vp, _c.c_int32],
    "ur_plan_set_block_transfer": [_vp, _c.c_int32],
    "ur_plan_set_bins": [_vp, _c.c_int32, _c.POINTER(_c.c_double)],
    "ur_cell_synth": [_vp, _c.POINTER(UrCell), _vp, _vp],
    "ur_rho_generate": [_vp, _c.POINTER(UrCell), _c.POINTER(UrMask), _c.POINTER(UrZoom), _c.c_int32, _c.c_int32,
                        _vp, _vp],
    "ur_fft3d_exec": [_vp, _vp, _vp, _c.c_int32, _vp],
    "ur_intensity_bin": [_vp, _vp, _c.POINTER(UrHist), _vp],
    "ur_simulate": [_vp, _c.POINTER(UrCell), _c.POINTER(UrMask), _c.POINTER(UrZoom), _c.POINTER(UrHist), _vp],
    "ur_simulate_rho": [_vp, _vp, _c.POINTER(UrHist), _vp],
    "ur_simulate_noalloc": [_vp, _c.POINTER(UrCell), _c.POINTER(UrMask), _c.POINTER(UrZoom), _c.POINTER(UrHist), _vp],
    "ur_simulate_host": [_vp, _vp, _c.c_int32, _c.c_int32, _c.POINTER(UrHist), _vp, _c.POINTER(_c.c_size_t)],
    "ur_adjoint": [_vp, _vp, _c.POINTER(UrCell), _c.POINTER(UrMask), _c.POINTER(UrHist), _vp, _vp, _vp, _vp],
    "ur_adjoint_reuse": [_vp, _c.POINTER(UrCell), _c.POINTER(UrMask), _c.POINTER(UrHist), _vp, _vp, _vp],
    "ur_merge_zooms": [_c.c_int32, _c.POINTER(UrHist), _c.POINTER(_c.c_int32), _c.POINTER(_c.c_double),
                       _c.c_int32, _vp, _c.c_int32, _c.c_double, _vp, _vp, _vp, _vp],
    "ur_ewald_image": [_vp, _vp, _c.POINTER(UrEwald), _vp, _vp],
    "ur_peak_integrals": [_c.c_int32, _vp, _vp, _c.c_int32, _c.POINTER(_c.c_double), _vp, _vp],
    "ur_ensemble": [_c.c_int32, _c.c_int32, _vp, _vp, _vp, _vp, _vp, _vp],
    "ur_chi2": [_c.c_int32, _vp, _vp, _vp, _c.c_double, _vp, _vp, _vp],
    "ur_graph_begin": [_vp],
    "ur_graph_end": [_vp, _c.POINTER(_vp)],
    "ur_graph_launch": [_vp, _vp],
    "ur_graph_destroy": [_vp],
    "ur_host_alloc": [_c.c_size_t, _c.POINTER(_vp)],
    "ur_host_free": [_vp],
    "ur_plan_set_timing": [_vp, _c.c_int32],
    "ur_plan_read_timing": [_vp, _c.c_int32, _c.POINTER(_c.c_double), _c.POINTER(_c.c_double),
                            _c.POINTER(_c.c_int32)],
    "ur_last_error": [],
    "ur_version": [],
}

# every symbol include/ultima.h declares
EXPORTS = tuple(_SIGS.keys())


def lib():
    """Load libultima.so (built in-tree by ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = _c.CDLL(LIBPATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _c.c_int if name not in ("ur_plan_destroy", "ur_last_error", "ur_version") else None
        L.ur_last_error.restype = _c.c_char_p
        L.ur_version.restype = _c.c_char_p
        L.ur_plan_destroy.restype = None
        _LIB = L
    return _LIB


class UltimaError(RuntimeError):
    pass


def _check(st: int, what: str) -> None:
    if st != 0:
        raise UltimaError(f"{what}: status {st}: {lib().ur_last_error().decode()}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise UltimaError("no HIP device available: the scattering kernels run on the GPU only")
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _require(t, dtype, numel: Optional[int] = None, what: str = "tensor"):
    torch = _torch()
    if t.device.type != "cuda" or not t.is_contiguous() or t.dtype != dtype:
        raise UltimaError(f"{what} must be a contiguous {dtype} tensor on the GPU")
    if numel is not None and t.numel() != numel:
        raise UltimaError(f"{what} has {t.numel()} elements, expected {numel}")
    return t


# ---------------------------------------------------------------------------
# marshalled inputs
# ---------------------------------------------------------------------------

@dataclass
class DeviceCell:
    """Unit cell with its atom arrays in device memory (FP64); `rot` the
    optional 3x3 lattice orientation (host, row-major)."""
    c: int
    xyz: "object"
    amp: "object"
    sigma: "object"
    background: float
    rot: Optional[np.ndarray] = None
    interp: int = 1
    grain_seed: Optional[np.ndarray] = None     # host [G*3], integer voxel offsets
    grain_rot: Optional[np.ndarray] = None      # host [G*9]

    @staticmethod
    def from_host(cell) -> "DeviceCell":
        torch = _torch()
        dev = torch.device("cuda")
        n = int(cell.amp.shape[0])
        xyz = torch.as_tensor(np.ascontiguousarray(cell.xyz, dtype=np.float64).reshape(-1), device=dev)
        amp = torch.as_tensor(np.ascontiguousarray(cell.amp, dtype=np.float64), device=dev)
        sig = torch.as_tensor(np.ascontiguousarray(cell.sigma, dtype=np.float64), device=dev)
        if n == 0:
            xyz = torch.zeros(3, dtype=torch.float64, device=dev)
            amp = torch.zeros(1, dtype=torch.float64, device=dev)
            sig = torch.ones(1, dtype=torch.float64, device=dev)
        rot = getattr(cell, "rot", None)
        rot = None if rot is None else np.ascontiguousarray(rot, dtype=np.float64).reshape(9)
        gs = getattr(cell, "grain_seed", None)
        gr = getattr(cell, "grain_rot", None)
        gs = None if gs is None else np.ascontiguousarray(gs, dtype=np.float64).reshape(-1)
        gr = None if gr is None else np.ascontiguousarray(gr, dtype=np.float64).reshape(-1)
        return DeviceCell(int(cell.c), xyz, amp, sig, float(cell.background), rot, int(getattr(cell, "interp", 1)),
                          gs, gr)

    def struct(self, amp=None) -> UrCell:
        a = self.amp if amp is None else amp
        n = int(a.numel()) if self.xyz.numel() == 3 * a.numel() else 0
        rot = None if self.rot is None else self.rot.ctypes.data_as(_c.POINTER(_c.c_double))
        dp = lambda v: None if v is None else v.ctypes.data_as(_c.POINTER(_c.c_double))
        ng = 0 if self.grain_seed is None else int(self.grain_seed.size // 3)
        return UrCell(self.c, n, _ptr(self.xyz), _ptr(a), _ptr(self.sigma), self.background, rot, self.interp,
                      ng, dp(self.grain_seed), dp(self.grain_rot))


def mask_struct(mask) -> UrMask:
    return UrMask(int(mask.kind), int(mask.p0), int(mask.p1))


class Hist:
    """Per-bin statistics (device, FP64) written by the library: sums,
    voxel counts, mean and standard error of the mean, and the totals."""

    FIELDS = ("sum", "sumsq", "count", "totals", "mean", "sem")

    def __init__(self, nbins: int, mean=None, sem=None):
        """mean, sem: optional device views to write those two outputs into
        (rows of a HistBatch)."""
        torch = _torch()
        dev = torch.device("cuda")
        self.nbins = nbins
        self.sum = torch.zeros(nbins, dtype=torch.float64, device=dev)
        self.sumsq = torch.zeros(nbins, dtype=torch.float64, device=dev)
        self.count = torch.zeros(nbins, dtype=torch.float64, device=dev)
        self.totals = torch.zeros(4, dtype=torch.float64, device=dev)
        self.mean = torch.zeros(nbins, dtype=torch.float64, device=dev) if mean is None else mean
        self.sem = torch.zeros(nbins, dtype=torch.float64, device=dev) if sem is None else sem

    def struct(self) -> UrHist:
        return UrHist(*[_ptr(getattr(self, k)) for k in self.FIELDS])

    def numpy(self) -> dict:
        return {k: getattr(self, k).cpu().numpy() for k in self.FIELDS}


class HistBatch:
    """Histograms of several boxes sharing one bin set, whose means and SEMs
    are the rows of two [nboxes, nbins] device tensors (the layout
    ur_ensemble reads)."""

    def __init__(self, nboxes: int, nbins: int):
        torch = _torch()
        self.mean = torch.zeros((nboxes, nbins), dtype=torch.float64, device="cuda")
        self.sem = torch.zeros((nboxes, nbins), dtype=torch.float64, device="cuda")
        self.hists = [Hist(nbins, mean=self.mean[k], sem=self.sem[k]) for k in range(nboxes)]
        self.nboxes, self.nbins = nboxes, nbins


def peak_integrals(edges, mean, windows, out=None, stream=None):
    """Per q window [(q_lo, q_hi), ...]: (peak integral above the straight
    baseline through the window's end bins, total integral, bins used) of a
    binned curve; `edges` and `mean` device FP64 tensors, result (nwin, 3)."""
    torch = _torch()
    w = np.ascontiguousarray(windows, dtype=np.float64).reshape(-1, 2)
    nb = int(mean.numel())
    _require(edges, torch.float64, nb + 1, "edges")
    _require(mean, torch.float64, nb, "mean")
    if out is None:
        out = torch.empty((len(w), 3), dtype=torch.float64, device="cuda")
    _require(out, torch.float64, 3 * len(w), "out")
    _check(lib().ur_peak_integrals(nb, _ptr(edges), _ptr(mean), len(w), w.ctypes.data_as(_c.POINTER(_c.c_double)),
                                   _ptr(out), _stream(stream)), "ur_peak_integrals")
    return out


def ensemble(batch: HistBatch, weights, out=None, stream=None):
    """Weighted ensemble of the batch's curves (ur_ensemble): returns the
    (mean, sem) device tensors; pass `out` under graph capture."""
    torch = _torch()
    _require(weights, torch.float64, batch.nboxes, "weights")
    if out is None:
        out = (torch.empty(batch.nbins, dtype=torch.float64, device="cuda"),
               torch.empty(batch.nbins, dtype=torch.float64, device="cuda"))
    _check(lib().ur_ensemble(batch.nboxes, batch.nbins, _ptr(batch.mean), _ptr(batch.sem), _ptr(weights),
                             _ptr(out[0]), _ptr(out[1]), _stream(stream)), "ur_ensemble")
    return out


def chi2(mean, count, target, rel_sigma: float = 0.01, out=None, g_bin=None, stream=None):
    """chi^2 of a binned curve against a target (ur_chi2) and, into `g_bin`
    when given, its gradient per bin; device FP64 tensors.  Returns the
    1-element device tensor holding chi^2."""
    torch = _torch()
    nb = int(mean.numel())
    _require(mean, torch.float64, nb, "mean")
    _require(count, torch.float64, nb, "count")
    _require(target, torch.float64, nb, "target")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device="cuda")
    _require(out, torch.float64, 1, "out")
    if g_bin is not None:
        _require(g_bin, torch.float64, nb, "g_bin")
    _check(lib().ur_chi2(nb, _ptr(mean), _ptr(count), _ptr(target), float(rel_sigma), _ptr(out), _ptr(g_bin),
                         _stream(stream)), "ur_chi2")
    return out


class Plan:
    """An n^3 box plan (precision, transform kind, bins, workspace)."""

    def __init__(self, n: int, voxel: float = 1.0, prec: int = UR_F32, c2c: bool = False,
                 workspace: bool = True):
        _torch()
        h = _vp()
        _check(lib().ur_plan_create(int(n), float(voxel), int(prec), UR_C2C if c2c else UR_R2C, _c.byref(h)),
               "ur_plan_create")
        self.h = h
        self.calls = 0          # library calls that touch this plan's workspace
        self.n, self.voxel, self.prec, self.c2c = int(n), float(voxel), int(prec), bool(c2c)
        self.mixed = self.n & (self.n - 1) != 0      # mixed-radix edge: natural-order [kx][ky][kz] spectrum
        self.nbins = 0
        self._ws = None
        self._use_torch_ws = workspace
        self._budget = 0

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and _LIB is not None:
                _LIB.ur_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def real_dtype(self):
        torch = _torch()
        return torch.float32 if self.prec == UR_F32 else torch.float64

    @property
    def complex_dtype(self):
        torch = _torch()
        return torch.complex64 if self.prec == UR_F32 else torch.complex128

    def set_bins(self, edges: np.ndarray) -> None:
        e = np.ascontiguousarray(edges, dtype=np.float64)
        self.calls += 1
        _check(lib().ur_plan_set_bins(self.h, int(e.size - 1), e.ctypes.data_as(_c.POINTER(_c.c_double))),
               "ur_plan_set_bins")
        self.nbins = int(e.size - 1)
        # larger boxes, and plans given an HBM budget, size their (out-of-core)
        # workspace at the streaming call instead
        if self.n <= MAX_IN_CORE and not self._budget:
            self._attach(self.workspace_size())

    def workspace_size(self, nbins: Optional[int] = None) -> int:
        v = _c.c_size_t()
        _check(lib().ur_plan_workspace_size(self.h, int(nbins or max(self.nbins, 1)), _c.byref(v)),
               "ur_plan_workspace_size")
        return int(v.value)

    def set_voxel_form(self, enable: bool = True) -> None:
        """Weight binned intensities by the voxel form factor
        S(h) S(k) S(l), S(m) = sinc^2(pi m / n) (ur_plan_set_voxel_form)."""
        _check(lib().ur_plan_set_voxel_form(self.h, int(bool(enable))), "ur_plan_set_voxel_form")

    def set_block_transfer(self, factor: int) -> None:
        """Divide every binned intensity by the block transfer of a zoom
        level made by block sums of `factor` (0 or 1: off)
        (ur_plan_set_block_transfer)."""
        _check(lib().ur_plan_set_block_transfer(self.h, int(factor)), "ur_plan_set_block_transfer")

    def set_hbm_budget(self, nbytes: int) -> None:
        """Out-of-core workspace limit in bytes (0: none); above it the path
        runs in kz chunks, streaming the host planes once per chunk."""
        _check(lib().ur_plan_set_hbm_budget(self.h, int(nbytes)), "ur_plan_set_hbm_budget")
        self._budget = int(nbytes)

    def workspace_size_host(self, x_lo: int, x_hi: int) -> int:
        v = _c.c_size_t()
        _check(lib().ur_plan_workspace_size_host(self.h, int(max(self.nbins, 1)), int(x_lo), int(x_hi),
                                                 _c.byref(v)), "ur_plan_workspace_size_host")
        return int(v.value)

    def _attach(self, nbytes: int) -> None:
        """Workspace from torch's allocator (256-byte aligned)."""
        if not self._use_torch_ws:
            return
        torch = _torch()
        if self._ws is not None and self._ws.numel() >= nbytes:
            return
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = int(self._ws.data_ptr())
        aligned = (base + 255) & ~255
        self.calls += 1
        _check(lib().ur_plan_set_workspace(self.h, _vp(aligned), _c.c_size_t(nbytes)), "ur_plan_set_workspace")

    # -- timing -------------------------------------------------------------
    PASSES = ("cell", "pass_z", "pass_y", "pass_x", "finalize")

    def set_timing(self, on: bool) -> None:
        _check(lib().ur_plan_set_timing(self.h, 1 if on else 0), "ur_plan_set_timing")

    def read_timing(self) -> dict:
        """Per pass: summed ms, algorithmic bytes of one launch, launches."""
        k = len(self.PASSES)
        ms = (_c.c_double * k)()
        by = (_c.c_double * k)()
        nl = (_c.c_int32 * k)()
        _check(lib().ur_plan_read_timing(self.h, k, ms, by, nl), "ur_plan_read_timing")
        return {name: {"ms": ms[i], "bytes": by[i], "launches": nl[i]} for i, name in enumerate(self.PASSES)}

    # -- entry points -------------------------------------------------------
    def simulate(self, cell: DeviceCell, mask, zoom, hist: Hist, stream=None, amp=None) -> Hist:
        cs = cell.struct(amp)
        ms = mask_struct(mask)
        zs = UrZoom(int(zoom.n1), int(zoom.factor))
        hs = hist.struct()
        self.calls += 1
        _check(lib().ur_simulate(self.h, _c.byref(cs), _c.byref(ms), _c.byref(zs), _c.byref(hs), _stream(stream)),
               "ur_simulate")
        return hist

    def simulate_noalloc(self, cell: DeviceCell, mask, zoom, hist: Hist, stream=None, amp=None) -> Hist:
        """ur_simulate_noalloc: the fused forward path with its scratch in the
        library's static device array (nothing allocated by the call; boxes
        up to 256^3 FP32)."""
        cs = cell.struct(amp)
        ms = mask_struct(mask)
        zs = UrZoom(int(zoom.n1), int(zoom.factor))
        hs = hist.struct()
        _check(lib().ur_simulate_noalloc(self.h, _c.byref(cs), _c.byref(ms), _c.byref(zs), _c.byref(hs),
                                         _stream(stream)), "ur_simulate_noalloc")
        return hist

    def simulate_rho(self, rho, hist: Hist, stream=None) -> Hist:
        n = self.n
        _require(rho, self.complex_dtype if self.c2c else self.real_dtype, n ** 3, "rho")
        hs = hist.struct()
        self.calls += 1
        _check(lib().ur_simulate_rho(self.h, _ptr(rho), _c.byref(hs), _stream(stream)), "ur_simulate_rho")
        return hist

    def simulate_host(self, rho_host, x_lo: int, x_hi: int, hist: Hist, stream=None) -> int:
        """rho_host: pinned CPU tensor holding planes x_lo..x_hi of the density
        ((x_hi - x_lo + 1) n^2 reals). Returns the H2D byte count."""
        if rho_host.device.type != "cpu" or not rho_host.is_contiguous() or rho_host.dtype != self.real_dtype \
                or rho_host.numel() != (int(x_hi) - int(x_lo) + 1) * self.n ** 2:
            raise UltimaError("rho_host must be a contiguous CPU tensor of (x_hi - x_lo + 1) n^2 reals of the plan "
                              "precision")
        if self._use_torch_ws:
            self._attach(self.workspace_size_host(x_lo, x_hi))
        hs = hist.struct()
        nb = _c.c_size_t()
        self.calls += 1
        _check(lib().ur_simulate_host(self.h, _ptr(rho_host), int(x_lo), int(x_hi), _c.byref(hs), _stream(stream),
                                      _c.byref(nb)), "ur_simulate_host")
        return int(nb.value)

    def rho_generate(self, cell: DeviceCell, mask, zoom, out=None, stream=None, x_lo: int = 0, x_hi=None):
        """Planes x_lo..x_hi (default: the whole box) of the density, as a
        device tensor [x - x_lo][y][z]."""
        torch = _torch()
        x_hi = self.n - 1 if x_hi is None else int(x_hi)
        planes = x_hi - int(x_lo) + 1
        if out is None:
            out = torch.empty((max(planes, 0), self.n, self.n), dtype=self.real_dtype, device="cuda")
        _require(out, self.real_dtype, max(planes, 0) * self.n ** 2, "out")
        cs, ms, zs = cell.struct(), mask_struct(mask), UrZoom(int(zoom.n1), int(zoom.factor))
        self.calls += 1
        _check(lib().ur_rho_generate(self.h, _c.byref(cs), _c.byref(ms), _c.byref(zs), int(x_lo), x_hi, _ptr(out),
                                     _stream(stream)), "ur_rho_generate")
        return out

    def cell_synth(self, cell: DeviceCell, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty((cell.c,) * 3, dtype=torch.float64, device="cuda")
        cs = cell.struct()
        self.calls += 1
        _check(lib().ur_cell_synth(self.h, _c.byref(cs), _ptr(out), _stream(stream)), "ur_cell_synth")
        return out

    def nkz(self) -> int:
        return self.n if self.c2c else self.n // 2 + 1

    def fft3d(self, x, out=None, direction: int = -1, stream=None):
        """eq. 1 forward (1/n^3) into the [kz][ky][kx] layout ([kx][ky][kz] on a
        mixed-radix plan, which needs no workspace; kz in [0, n/2] for a real
        plan), or its inverse (not on real mixed-radix plans)."""
        torch = _torch()
        n = self.n
        if direction < 0:
            _require(x, self.complex_dtype if self.c2c else self.real_dtype, n ** 3, "input")
            if out is None:
                shape = (n, n, self.nkz()) if self.mixed else (self.nkz(), n, n)
                out = torch.empty(shape, dtype=self.complex_dtype, device="cuda")
            _require(out, self.complex_dtype, self.nkz() * n * n, "output")
        else:
            _require(x, self.complex_dtype, self.nkz() * n * n, "spectrum")
            if out is None:
                out = torch.empty((n, n, n), dtype=self.complex_dtype if self.c2c else self.real_dtype, device="cuda")
            _require(out, self.complex_dtype if self.c2c else self.real_dtype, n ** 3, "output")
        if self.nbins == 0 and not self.mixed:
            self._attach(self.workspace_size(1))
        self.calls += 1
        _check(lib().ur_fft3d_exec(self.h, _ptr(x), _ptr(out), int(direction), _stream(stream)), "ur_fft3d_exec")
        return out

    def ewald_image(self, spectrum, geometry, out=None, stream=None):
        """Detector image (nv, nu) in FP64 of the spectrum of ``fft3d`` on the
        Ewald sphere of a flat detector (``workloads.Ewald`` fields)."""
        torch = _torch()
        _require(spectrum, self.complex_dtype, self.nkz() * self.n * self.n, "spectrum")
        if out is None:
            out = torch.empty((int(geometry.nv), int(geometry.nu)), dtype=torch.float64, device="cuda")
        _require(out, torch.float64, int(geometry.nv) * int(geometry.nu), "image")
        g = UrEwald.from_geometry(geometry)
        _check(lib().ur_ewald_image(self.h, _ptr(spectrum), _c.byref(g), _ptr(out), _stream(stream)),
               "ur_ewald_image")
        return out

    def intensity_bin(self, spectrum, hist: Hist, stream=None) -> Hist:
        _require(spectrum, self.complex_dtype, self.nkz() * self.n ** 2, "spectrum")
        hs = hist.struct()
        self.calls += 1
        _check(lib().ur_intensity_bin(self.h, _ptr(spectrum), _c.byref(hs), _stream(stream)), "ur_intensity_bin")
        return hist

    def adjoint(self, fwd: Hist, g_bin, rho=None, cell: Optional[DeviceCell] = None, mask=None,
                grad_rho=None, grad_amp=None, stream=None, amp=None):
        _require(g_bin, _torch().float64, self.nbins, "g_bin")
        hs = fwd.struct()
        cs = cell.struct(amp) if cell is not None else None
        ms = mask_struct(mask) if mask is not None else None
        self.calls += 1
        _check(lib().ur_adjoint(self.h, _ptr(rho), _c.byref(cs) if cs is not None else None,
                                _c.byref(ms) if ms is not None else None, _c.byref(hs), _ptr(g_bin),
                                _ptr(grad_rho), _ptr(grad_amp), _stream(stream)), "ur_adjoint")
        return grad_rho, grad_amp

    def adjoint_reuse(self, fwd: Hist, g_bin, cell: DeviceCell, mask, grad_amp, stream=None, amp=None):
        """Amplitude gradient from the y-pass output held by the preceding
        simulate call on this plan (no recomputation); raises UltimaError
        when the plan holds none."""
        _require(g_bin, _torch().float64, self.nbins, "g_bin")
        hs, cs, ms = fwd.struct(), cell.struct(amp), mask_struct(mask)
        self.calls += 1
        _check(lib().ur_adjoint_reuse(self.h, _c.byref(cs), _c.byref(ms), _c.byref(hs), _ptr(g_bin), _ptr(grad_amp),
                                      _stream(stream)), "ur_adjoint_reuse")
        return grad_amp


def merge_zooms(hists: Sequence[Hist], ns: Sequence[int], voxels: Sequence[float], edges_dev, mode: int = MERGE_FINEST,
                n_min: float = 32.0, stream=None, out=None):
    """One curve from several zoom levels; `out` = (mean, sem, owner) device
    tensors to write (allocated here when None -- pass them under capture)."""
    torch = _torch()
    k = len(hists)
    nb = hists[0].nbins
    arr = (UrHist * k)(*[h.struct() for h in hists])
    n_arr = (_c.c_int32 * k)(*[int(v) for v in ns])
    v_arr = (_c.c_double * k)(*[float(v) for v in voxels])
    _require(edges_dev, torch.float64, nb + 1, "edges")
    if out is None:
        out = (torch.empty(nb, dtype=torch.float64, device="cuda"),
               torch.empty(nb, dtype=torch.float64, device="cuda"),
               torch.empty(nb, dtype=torch.int32, device="cuda"))
    mean, sem, owner = out
    _require(mean, torch.float64, nb, "mean")
    _require(sem, torch.float64, nb, "sem")
    _require(owner, torch.int32, nb, "owner")
    _check(lib().ur_merge_zooms(k, arr, n_arr, v_arr, nb, _ptr(edges_dev), int(mode), float(n_min), _ptr(mean),
                                _ptr(sem), _ptr(owner), _stream(stream)), "ur_merge_zooms")
    return mean, sem, owner


class Graph:
    """HIP graph recorded from the calls made between begin() and end()."""

    def __init__(self, stream):
        self.stream = stream
        self.h = None

    def __enter__(self):
        _check(lib().ur_graph_begin(int(self.stream.cuda_stream)), "ur_graph_begin")
        return self

    def __exit__(self, et, ev, tb):
        h = _vp()
        st = lib().ur_graph_end(int(self.stream.cuda_stream), _c.byref(h))
        if et is None:
            _check(st, "ur_graph_end")
            self.h = h
        return False

    def launch(self):
        _check(lib().ur_graph_launch(self.h, int(self.stream.cuda_stream)), "ur_graph_launch")

    def __del__(self):
        try:
            if self.h is not None and _LIB is not None:
                _LIB.ur_graph_destroy(self.h)
        except Exception:
            pass


class HostBuffer:
    """Page-locked host memory of exactly the requested size (ur_host_alloc;
    torch's pinned allocator rounds up to a power of two), exposed as the CPU
    tensor ``.tensor``.  Views of it must not outlive the buffer: ``close()``
    (or collection of the object) frees the memory."""

    def __init__(self, shape, dtype):
        torch = _torch()
        self.shape = tuple(int(d) for d in shape)
        count = int(np.prod(self.shape, dtype=np.int64))
        np_dtype = {torch.float32: np.float32, torch.float64: np.float64}[dtype]
        self.nbytes = count * np.dtype(np_dtype).itemsize
        p = _vp()
        _check(lib().ur_host_alloc(self.nbytes, _c.byref(p)), "ur_host_alloc")
        self.ptr = p.value
        raw = (_c.c_char * self.nbytes).from_address(self.ptr)
        self.tensor = torch.from_numpy(np.frombuffer(raw, dtype=np_dtype, count=count).reshape(self.shape))

    def close(self):
        if getattr(self, "ptr", None):
            self.tensor = None
            lib().ur_host_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return lib().ur_version().decode()
