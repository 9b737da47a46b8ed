"""FP64 CPU oracle for the wide-range scattering simulation (arXiv 2303.13435).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It is the plain, slow, obviously
correct statement of the computation, written from the paper:

* O1  unit-cell density (workflow step 1; "Electron density generation")
* O2  ED-1 = tiled cell x particle mask (workflow step 2); O2r with a rotated lattice
  (trilinear or cubic B-spline sampling of the cell); O2g polycrystalline grains
* O3  zoomed-out ED-2/ED-3 by block integration and zero padding (step 3),
  also of rotated and polycrystalline ED-1 boxes
* O4  3D transform, eq. 1 (axis by axis, as eq. 2 separates it)
* O5-O8  |Q| map, integer-threshold bins, per-bin mean and SEM (step 5)
* O9  merge of zoom levels into one curve (step 6; reading in ``merge``)
* O10 chi^2 misfit of a binned curve and its gradients (derived from eq. 1)
* O11 low-frequency Fourier coefficients by direct summation (eq. 1/eq. 2)
* O12 per-bin counts and two-voxel intensities of boxes too large for O4-O8
* O13 per-bin intensities of a uniform cube at any box size (eq. 1 factorised)
* O14 polydisperse ensemble of boxes (Results and Discussion; reading in ``ensemble``)
* O15 voxel form factor (the voxel-sized sinc; reading in ``voxel_form``)
* O16 Ewald-sphere detector image (Q-calculation and spherical averaging;
  reading in ``ewald_image``)
* O17 peak integrals for the degree of crystallinity (Results and
  Discussion; reading in ``peak_integrals``)
* O18 block transfer of a zoom level and its removal from the level's
  intensities (high-Q correction of coarse levels; reading in ``block_transfer``)

The heavy loops live in ``ur_oracle.c`` (plain C, FP64, OpenMP over
independent lines); this module marshals numpy arrays and holds the small
per-bin arithmetic (merge, chi^2) written out in numpy.

It shares no code with the HIP library; the only common import is the seeded
input generator package ``workloads``, which holds none of the arithmetic.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ur_oracle.c")
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_LIB = None

_D = ctypes.POINTER(ctypes.c_double)
_LL = ctypes.POINTER(ctypes.c_longlong)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIBPATH):
        tmp = _LIBPATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIBPATH)
    return _LIBPATH


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_LIBPATH):
            build(force=False)
        L = ctypes.CDLL(_LIBPATH)
        L.or_atom_profile.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
        L.or_cell_synth.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.c_double, _D]
        L.or_mask_inside.argtypes = [ctypes.c_int] + [ctypes.c_longlong] * 5
        L.or_mask_inside.restype = ctypes.c_int
        L.or_ed1.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_longlong,
                             ctypes.c_longlong, _D]
        L.or_ed1_rot.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_longlong,
                                 ctypes.c_longlong, _D, ctypes.c_int, _D]
        L.or_ed1_grains.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_longlong,
                                    ctypes.c_longlong, ctypes.c_int, _LL, _D, ctypes.c_int, _D]
        L.or_ed1_grains_points.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_longlong,
                                           ctypes.c_longlong, ctypes.c_int, _LL, _D, ctypes.c_int, ctypes.c_longlong,
                                           _LL, _D]
        L.or_zoom.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_longlong,
                              ctypes.c_longlong, ctypes.c_int, ctypes.c_int, _D]
        L.or_fft3d.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        L.or_fft1d_batch.argtypes = [ctypes.c_int, ctypes.c_longlong, ctypes.c_void_p, ctypes.c_int]
        L.or_thresholds.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, _D, _LL]
        L.or_bin.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_int, _D,
                             _D, _D, _D, _D, _D, _D]
        L.or_bin_counts.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, _D, _D]
        L.or_lowfreq_dft.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int, ctypes.c_longlong,
                                     ctypes.c_longlong, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p]
        L.or_density_moments.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int,
                                         ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int,
                                         ctypes.c_int, _D]
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        L.or_dft_points.argtypes = [ctypes.c_int, ctypes.c_longlong, _LL, _D, ctypes.c_longlong, _LL,
                                    ctypes.c_void_p]
        L.or_axis_pair_bins.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, _D, ctypes.c_longlong,
                                        ctypes.c_double, ctypes.c_double, _D, _D]
        L.or_cube_bins.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, _D, ctypes.c_longlong,
                                   ctypes.c_double, ctypes.c_int, _D, _D]
        _LIB = L
    return _LIB


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(t: int) -> None:
    lib().or_set_num_threads(int(t))


# ---------------------------------------------------------------------------
# O1  unit cell
# ---------------------------------------------------------------------------

def atom_profile(c: int, x: float, sigma: float) -> np.ndarray:
    """Voxel-integrated periodic Gaussian along one axis (sums to 1)."""
    p = np.zeros(c)
    lib().or_atom_profile(int(c), float(x), float(sigma), _dp(p))
    return p


def atom_profiles(cell) -> np.ndarray:
    """(n_atoms, 3, c) array of per-axis profiles."""
    out = np.zeros((cell.n_atoms, 3, cell.c))
    for a in range(cell.n_atoms):
        for d in range(3):
            out[a, d] = atom_profile(cell.c, cell.xyz[a, d], cell.sigma[a])
    return out


def cell_synth(cell) -> np.ndarray:
    c = int(cell.c)
    out = np.zeros((c, c, c))
    xyz = np.ascontiguousarray(cell.xyz, dtype=np.float64).reshape(-1)
    amp = np.ascontiguousarray(cell.amp, dtype=np.float64)
    sig = np.ascontiguousarray(cell.sigma, dtype=np.float64)
    if xyz.size == 0:
        xyz = np.zeros(3)
        amp = np.zeros(1)
        sig = np.ones(1)
        lib().or_cell_synth(c, 0, _dp(xyz), _dp(amp), _dp(sig), float(cell.background), _dp(out))
    else:
        lib().or_cell_synth(c, cell.n_atoms, _dp(xyz), _dp(amp), _dp(sig), float(cell.background),
                            _dp(out))
    return out


# ---------------------------------------------------------------------------
# O2/O3  densities
# ---------------------------------------------------------------------------

def mask_inside(mask, dx: int, dy: int, dz: int) -> bool:
    return bool(lib().or_mask_inside(int(mask.kind), int(mask.p0), int(mask.p1), int(dx), int(dy), int(dz)))


def ed1(n: int, cell_grid: np.ndarray, mask) -> np.ndarray:
    c = cell_grid.shape[0]
    cg = np.ascontiguousarray(cell_grid, dtype=np.float64)
    out = np.empty((n, n, n))
    lib().or_ed1(int(n), int(c), _dp(cg), int(mask.kind), int(mask.p0), int(mask.p1), _dp(out))
    return out


def bspline_coefficients(cell_grid: np.ndarray) -> np.ndarray:
    """Periodic cubic B-spline coefficients C of the cell (the spline through
    its values): sampled at the integers the spline is C filtered by
    (1, 4, 1)/6 along each axis, so in the DFT domain C = S / (b b b) with
    b(k) = (4 + 2 cos(2 pi k / c)) / 6."""
    c = cell_grid.shape[0]
    b = (4.0 + 2.0 * np.cos(2.0 * np.pi * np.arange(c) / c)) / 6.0
    B = b[:, None, None] * b[None, :, None] * b[None, None, :]
    return np.real(np.fft.ifftn(np.fft.fftn(np.asarray(cell_grid, dtype=np.float64)) / B))


def ed1_rot(n: int, cell_grid: np.ndarray, mask, rot: np.ndarray, interp: int = 1) -> np.ndarray:
    """O2r: ED-1 of a lattice oriented by the 3x3 matrix rot (cell sampled at
    u = rot d with periodic wrap): trilinear (interp 1) or the cubic
    B-spline through the cell values (interp 3, the order-3 spline of the
    interpolation routine the paper names)."""
    assert interp in (1, 3)
    c = cell_grid.shape[0]
    cg = np.ascontiguousarray(cell_grid if interp == 1 else bspline_coefficients(cell_grid), dtype=np.float64)
    R = np.ascontiguousarray(rot, dtype=np.float64).reshape(9)
    out = np.empty((n, n, n))
    lib().or_ed1_rot(int(n), int(c), _dp(cg), int(mask.kind), int(mask.p0), int(mask.p1), _dp(R), int(interp),
                     _dp(out))
    return out


def ed1_grains(n: int, cell_grid: np.ndarray, mask, seeds: np.ndarray, rots: np.ndarray, interp: int = 1) -> np.ndarray:
    """O2g: polycrystalline ED-1 (the rotated grid builds crystallites of
    random orientation; the outlook names polycrystalline grains): each
    inside voxel belongs to the grain of the nearest integer seed (ties to
    the lower index) and samples the cell at u = R_g d as ``ed1_rot``."""
    assert interp in (1, 3)
    c = cell_grid.shape[0]
    cg = np.ascontiguousarray(cell_grid if interp == 1 else bspline_coefficients(cell_grid), dtype=np.float64)
    S = np.ascontiguousarray(np.rint(seeds), dtype=np.int64).reshape(-1)
    R = np.ascontiguousarray(rots, dtype=np.float64).reshape(-1)
    g = S.size // 3
    assert R.size == 9 * g and g >= 1
    out = np.empty((n, n, n))
    lib().or_ed1_grains(int(n), int(c), _dp(cg), int(mask.kind), int(mask.p0), int(mask.p1), int(g),
                        S.ctypes.data_as(_LL), _dp(R), int(interp), _dp(out))
    return out


def oriented_points(n: int, cell_grid: np.ndarray, mask, xyz: np.ndarray, seeds: np.ndarray, rots: np.ndarray,
                    interp: int = 1) -> np.ndarray:
    """O2r / O2g at the voxels xyz[p] = (x, y, z) only (one orientation is
    one grain), for boxes too large to generate whole."""
    assert interp in (1, 3)
    c = cell_grid.shape[0]
    cg = np.ascontiguousarray(cell_grid if interp == 1 else bspline_coefficients(cell_grid), dtype=np.float64)
    S = np.ascontiguousarray(np.rint(seeds), dtype=np.int64).reshape(-1)
    R = np.ascontiguousarray(rots, dtype=np.float64).reshape(-1)
    P = np.ascontiguousarray(xyz, dtype=np.int64).reshape(-1)
    out = np.empty(P.size // 3)
    lib().or_ed1_grains_points(int(n), int(c), _dp(cg), int(mask.kind), int(mask.p0), int(mask.p1), int(S.size // 3),
                               S.ctypes.data_as(_LL), _dp(R), int(interp), int(out.size), P.ctypes.data_as(_LL),
                               _dp(out))
    return out


def zoomed(n1: int, cell_grid: np.ndarray, mask, f: int, nk: int) -> np.ndarray:
    c = cell_grid.shape[0]
    cg = np.ascontiguousarray(cell_grid, dtype=np.float64)
    out = np.empty((nk, nk, nk))
    lib().or_zoom(int(n1), int(c), _dp(cg), int(mask.kind), int(mask.p0), int(mask.p1), int(f),
                  int(nk), _dp(out))
    return out


def block_level(rho1: np.ndarray, f: int, nk: int) -> np.ndarray:
    """O3 from a given ED-1 box (workflow step 3): block sums of f^3 fine
    voxels, the reduced region centred in an nk^3 box at offset
    o = (nk - n1/f)/2, zero elsewhere."""
    n1 = rho1.shape[0]
    m = n1 // f
    assert m * f == n1 and m <= nk
    red = rho1.reshape(m, f, m, f, m, f).sum(axis=(1, 3, 5))
    out = np.zeros((nk, nk, nk))
    o = (nk - m) // 2
    out[o:o + m, o:o + m, o:o + m] = red
    return out


def density(wl, cell_grid: Optional[np.ndarray] = None) -> np.ndarray:
    """Real-space box of a workload: ED-1 (factor 1) or a zoomed level; a
    zoom level of a rotated or polycrystalline lattice is the block sum of
    that lattice's ED-1 (O2r / O2g, then O3)."""
    if cell_grid is None:
        cell_grid = cell_synth(wl.cell)
    seeds = getattr(wl.cell, "grain_seed", None)
    if seeds is not None:
        rho1 = ed1_grains(wl.zoom.n1, cell_grid, wl.mask, seeds, wl.cell.grain_rot, int(getattr(wl.cell, "interp", 1)))
        return rho1 if wl.zoom.factor == 1 and wl.zoom.n1 == wl.n else block_level(rho1, wl.zoom.factor, wl.n)
    rot = getattr(wl.cell, "rot", None)
    if rot is not None:
        rho1 = ed1_rot(wl.zoom.n1, cell_grid, wl.mask, rot, int(getattr(wl.cell, "interp", 1)))
        return rho1 if wl.zoom.factor == 1 and wl.zoom.n1 == wl.n else block_level(rho1, wl.zoom.factor, wl.n)
    if wl.zoom.factor == 1 and wl.zoom.n1 == wl.n:
        return ed1(wl.n, cell_grid, wl.mask)
    return zoomed(wl.zoom.n1, cell_grid, wl.mask, wl.zoom.factor, wl.n)


# ---------------------------------------------------------------------------
# O4  transform
# ---------------------------------------------------------------------------

def fft3d(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised 3D DFT (sign -1 forward, +1 inverse) of an n^3 array."""
    n = a.shape[0]
    assert a.shape == (n, n, n)
    z = np.ascontiguousarray(a, dtype=np.complex128).copy()
    lib().or_fft3d(int(n), z.ctypes.data_as(ctypes.c_void_p), int(sign))
    return z


def fft1d(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised 1D DFT along the last axis."""
    n = a.shape[-1]
    z = np.ascontiguousarray(a, dtype=np.complex128).copy()
    lib().or_fft1d_batch(int(n), int(z.size // n), z.ctypes.data_as(ctypes.c_void_p), int(sign))
    return z


def forward(rho: np.ndarray) -> np.ndarray:
    """F of eq. 1: the forward DFT scaled by 1/(M N L)."""
    n = rho.shape[0]
    return fft3d(rho, -1) / float(n) ** 3


# ---------------------------------------------------------------------------
# O5-O8  binning
# ---------------------------------------------------------------------------

def thresholds(n: int, voxel: float, edges: np.ndarray) -> np.ndarray:
    e = np.ascontiguousarray(edges, dtype=np.float64)
    U = np.zeros(e.size, dtype=np.int64)
    lib().or_thresholds(int(n), float(voxel), int(e.size - 1), _dp(e), U.ctypes.data_as(_LL))
    return U


def bin_spectrum(F: np.ndarray, voxel: float, edges: np.ndarray) -> Dict[str, np.ndarray]:
    """Per-bin count / sum / sumsq / mean / sem of I = |F|^2 over the full
    (n^3) spectrum F, plus totals = [sum of all I, Re F(0), Im F(0)]."""
    n = F.shape[0]
    Fc = np.ascontiguousarray(F, dtype=np.complex128)
    e = np.ascontiguousarray(edges, dtype=np.float64)
    nb = e.size - 1
    out = {k: np.zeros(nb) for k in ("count", "sum", "sumsq", "mean", "sem")}
    tot = np.zeros(3)
    lib().or_bin(int(n), Fc.ctypes.data_as(ctypes.c_void_p), float(voxel), int(nb), _dp(e),
                 _dp(out["count"]), _dp(out["sum"]), _dp(out["sumsq"]), _dp(out["mean"]),
                 _dp(out["sem"]), _dp(tot))
    out["totals"] = tot
    return out


def bin_counts(n: int, voxel: float, edges: np.ndarray) -> np.ndarray:
    e = np.ascontiguousarray(edges, dtype=np.float64)
    out = np.zeros(e.size - 1)
    lib().or_bin_counts(int(n), float(voxel), int(e.size - 1), _dp(e), _dp(out))
    return out


def voxel_form(n: int) -> np.ndarray:
    """O15: amplitude factor of a density uniform over each voxel instead of
    sampled at its centre (the voxel-sized sinc of Q-calculation and
    spherical averaging): sinc(pi h/n) sinc(pi k/n) sinc(pi l/n) on the
    [u][v][w] frequency grid, signed indices, sinc(x) = sin(x)/x."""
    u = np.arange(n)
    h = np.where(u < n // 2, u, u - n).astype(np.float64)
    x = np.pi * h / n
    s1 = np.ones(n)
    nz = h != 0
    s1[nz] = np.sin(x[nz]) / x[nz]
    return s1[:, None, None] * s1[None, :, None] * s1[None, None, :]


def block_transfer(n: int, f: int) -> np.ndarray:
    """O18: amplitude transfer of the block sum that makes a zoom level.

    A level's voxel X holds the sum of the f^3 fine voxels f X + j (j in
    [0, f)^3, step 3 of the workflow), so along one axis its absolute
    amplitude at coarse index m is sum_s T(m - s n) A1(m - s n) over the f
    aliases s, with A1 the fine box's amplitude on the f n grid and
        T(m) = (1/f) sum_{j<f} exp(+2 pi i m j / (f n)),
    written here as that sum (the identity is pinned against transforms of
    a box and of its block sums).  Returns T(h) T(k) T(l) on the level's
    [u][v][w] grid, signed indices.  Dividing a level's amplitudes by it
    undoes the attenuation of the block sum (|T|^2 = 0.81 per axis at half
    the level's Nyquist index, for large f); aliased fine frequencies are
    not removed.  Reading: the paper names the correction of coarse levels
    near their cut-off without a formula; this is the exact transfer of its
    own block integration, applied to the intensities before binning."""
    u = np.arange(n)
    h = np.where(u < n // 2, u, u - n).astype(np.float64)
    j = np.arange(f, dtype=np.float64)
    t1 = np.exp(2j * np.pi * np.outer(h, j) / (f * n)).sum(axis=1) / f
    return t1[:, None, None] * t1[None, :, None] * t1[None, None, :]


def simulate(wl, return_fields: bool = False, voxel_form_factor: bool = False,
             block_transfer_removed: bool = False):
    """Whole forward path of one box: density -> eq. 1 -> per-bin statistics
    (of the voxel-uniform density's intensities with voxel_form_factor; of
    intensities divided by the level's block transfer |T|^2 (O18) with
    block_transfer_removed, for a zoom level).  Also reports the density
    moments sum(rho) and sum(rho^2)."""
    cg = cell_synth(wl.cell)
    rho = density(wl, cg)
    F = forward(rho)
    G = F * voxel_form(wl.n) if voxel_form_factor else F
    if block_transfer_removed and wl.zoom.factor > 1:
        G = G / block_transfer(wl.n, wl.zoom.factor)
    res = bin_spectrum(G, wl.voxel, wl.edges)
    res["rho_sum"] = float(rho.sum(dtype=np.float64))
    res["rho_sumsq"] = float(np.sum(rho * rho))
    if return_fields:
        res["rho"] = rho
        res["F"] = F
        res["cell"] = cg
    return res


# ---------------------------------------------------------------------------
# O11  low-frequency coefficients by direct summation
# ---------------------------------------------------------------------------

def lowfreq_dft(wl, K: int, cell_grid: Optional[np.ndarray] = None) -> np.ndarray:
    """F(h, k, l) of eq. 1 for |h|,|k|,|l| <= K, array index [h+K][k+K][l+K]."""
    if cell_grid is None:
        cell_grid = cell_synth(wl.cell)
    cg = np.ascontiguousarray(cell_grid, dtype=np.float64)
    nf = 2 * K + 1
    out = np.zeros((nf, nf, nf), dtype=np.complex128)
    lib().or_lowfreq_dft(int(wl.zoom.n1), int(cg.shape[0]), _dp(cg), int(wl.mask.kind),
                         int(wl.mask.p0), int(wl.mask.p1), int(wl.zoom.factor), int(wl.n), int(K),
                         out.ctypes.data_as(ctypes.c_void_p))
    return out


def dft_points(n: int, xyz: np.ndarray, values: np.ndarray, uvw: np.ndarray) -> np.ndarray:
    """eq. 1 by direct summation over the nonzero voxels xyz[p] = (x, y, z)
    with densities values[p], at the frequencies uvw[q] = (u, v, w)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.int64)
    uvw = np.ascontiguousarray(uvw, dtype=np.int64)
    val = np.ascontiguousarray(values, dtype=np.float64)
    out = np.zeros(len(uvw), dtype=np.complex128)
    lib().or_dft_points(int(n), len(val), xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), _dp(val),
                        len(uvw), uvw.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                        out.ctypes.data_as(ctypes.c_void_p))
    return out


def axis_pair_bins(n: int, voxel: float, edges: np.ndarray, d: int, rho1: float, rho2: float):
    """O12: per-bin voxel count and sum of |F|^2 (eq. 1) over the n^3 box for
    the density of two voxels, rho1 and rho2, d apart along one axis; the
    count alone is the geometry of any density."""
    e = np.ascontiguousarray(edges, dtype=np.float64)
    nb = e.size - 1
    count, s = np.zeros(nb), np.zeros(nb)
    lib().or_axis_pair_bins(int(n), float(voxel), int(nb), _dp(e), int(d), float(rho1), float(rho2),
                            _dp(count), _dp(s))
    return count, s


def cube_bins(n: int, voxel: float, edges: np.ndarray, half_width: int, value: float = 1.0,
              voxel_form_factor: bool = False):
    """O13: per-bin voxel count and sum of |F|^2 (eq. 1) over the n^3 box for
    a uniform cube of the given value on max_i |x_i - n/2| <= half_width;
    with voxel_form_factor, each axis factor a(u) also carries sinc^2(pi u/n)
    (O15), which keeps the product form."""
    e = np.ascontiguousarray(edges, dtype=np.float64)
    nb = e.size - 1
    count, s = np.zeros(nb), np.zeros(nb)
    lib().or_cube_bins(int(n), float(voxel), int(nb), _dp(e), int(half_width), float(value),
                       int(bool(voxel_form_factor)), _dp(count), _dp(s))
    return count, s


def lattice_points_below(m: int) -> np.ndarray:
    """Every integer (h, k, l) with h^2 + k^2 + l^2 < m, as rows."""
    r = math.isqrt(max(m - 1, 0))
    a = np.arange(-r, r + 1, dtype=np.int64)
    h, k, l = np.meshgrid(a, a, a, indexing="ij")
    sel = h * h + k * k + l * l < m
    return np.stack([h[sel], k[sel], l[sel]], axis=1)


def sparse_low_bins(n: int, voxel: float, edges: np.ndarray, xyz: np.ndarray, values: np.ndarray, m: int):
    """Exact count / sum / mean of |F|^2 (eq. 1, by direct summation over the
    nonzero voxels) for every bin lying wholly below n2 = m, i.e. whose every
    lattice point has h^2 + k^2 + l^2 < m (m <= (n/2)^2 keeps them inside the
    box's frequency range).  Returns (bin indices, count, sum, mean)."""
    assert m <= (n // 2) ** 2
    U = thresholds(n, voxel, edges)
    pts = lattice_points_below(m)
    n2 = np.sum(pts * pts, axis=1)
    I = np.abs(dft_points(n, xyz, values, pts)) ** 2
    sel = [b for b in range(len(U) - 1) if U[b + 1] <= m and U[b + 1] > U[b]]
    cnt = np.array([np.count_nonzero((n2 >= U[b]) & (n2 < U[b + 1])) for b in sel], dtype=np.float64)
    s = np.array([I[(n2 >= U[b]) & (n2 < U[b + 1])].sum() for b in sel])
    mean = np.where(cnt > 0, s / np.maximum(cnt, 1), np.nan)
    return np.array(sel, dtype=np.int64), cnt, s, mean


def density_moments(wl, cell_grid: Optional[np.ndarray] = None):
    if cell_grid is None:
        cell_grid = cell_synth(wl.cell)
    cg = np.ascontiguousarray(cell_grid, dtype=np.float64)
    out = np.zeros(2)
    lib().or_density_moments(int(wl.zoom.n1), int(cg.shape[0]), _dp(cg), int(wl.mask.kind),
                             int(wl.mask.p0), int(wl.mask.p1), int(wl.zoom.factor), int(wl.n),
                             _dp(out))
    return float(out[0]), float(out[1])


def lowfreq_bins(wl, K: int, cell_grid: Optional[np.ndarray] = None):
    """Exact per-bin count/sum/mean for every bin whose voxels all satisfy
    |h|,|k|,|l| <= K (i.e. bins lying wholly below n2 = (K+1)^2).  Returns
    (bin indices, count, sum, mean)."""
    F = lowfreq_dft(wl, K, cell_grid)
    U = thresholds(wl.n, wl.voxel, wl.edges)
    nb = wl.nbins
    r = np.arange(-K, K + 1)
    h2 = r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2
    I = np.abs(F) ** 2
    limit = (K + 1) ** 2      # every voxel with n2 < limit lies inside the cube
    sel = [b for b in range(nb) if U[b + 1] <= limit and U[b + 1] > U[b]]
    cnt = np.zeros(len(sel))
    s = np.zeros(len(sel))
    for i, b in enumerate(sel):
        m = (h2 >= U[b]) & (h2 < U[b + 1])
        cnt[i] = m.sum()
        s[i] = I[m].sum()
    mean = np.where(cnt > 0, s / np.maximum(cnt, 1), np.nan)
    return np.array(sel, dtype=np.int64), cnt, s, mean


# ---------------------------------------------------------------------------
# O9  merge of zoom levels
# ---------------------------------------------------------------------------
MERGE_FINEST, MERGE_POOLED, MERGE_IVW = 0, 1, 2


def bin_centres(edges: np.ndarray) -> np.ndarray:
    lo, hi = edges[:-1], edges[1:]
    return np.where(lo > 0, np.sqrt(np.abs(lo * hi)), 0.5 * (lo + hi))


def sem_from_sums(count, s, s2):
    count = np.asarray(count, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        var = (np.asarray(s2) - np.asarray(s) ** 2 / count) / (count - 1.0)
        var = np.maximum(var, 0.0)
        return np.where(count > 1, np.sqrt(var / count), np.nan)


def merge(levels: Sequence[dict], edges: np.ndarray, mode: int = MERGE_FINEST, n_min: float = 32.0):
    """One curve from several zoom levels (workflow step 6).

    The paper merges with dataMerge, whose rule it does not give.  Reading
    taken here: each level's eq.-1 intensities are scaled back to absolute
    |sum rho e^{-iqx}|^2 by s_k = (n_k^3)^2; a level is *valid* for a bin when
    the bin centre lies in [dq_k, Q_cut,k], Q_cut,k = sqrt(3) pi / (2 voxel_k)
    (beyond half the corner frequency artefacts appear, Fig. 2 caption) and
    the bin holds at least ``n_min`` voxels at that level.

    * FINEST: the finest valid level owns the bin (mean and SEM scaled by s_k)
    * POOLED: pooled scaled sums and counts over the valid levels
    * IVW:    inverse-variance weighted mean of the valid levels' means

    ``levels``: dicts with n, voxel, count, sum, sumsq (per bin).  Returns
    (mean, sem, owner) with owner = -1 / NaN where no level is valid; for
    POOLED and IVW owner is the number of contributing levels.
    """
    nb = edges.size - 1
    qc = bin_centres(np.asarray(edges, dtype=np.float64))
    order = sorted(range(len(levels)), key=lambda k: levels[k]["voxel"])
    mean = np.full(nb, np.nan)
    sem = np.full(nb, np.nan)
    owner = np.full(nb, -1, dtype=np.int64)
    for b in range(nb):
        valid = []
        for k in order:
            L = levels[k]
            dq = 2.0 * math.pi / (L["n"] * L["voxel"])
            qcut = math.sqrt(3.0) * math.pi / (2.0 * L["voxel"])
            if dq <= qc[b] <= qcut and L["count"][b] >= n_min:
                valid.append(k)
        if not valid:
            continue
        if mode == MERGE_FINEST:
            k = valid[0]
            L = levels[k]
            s = float(L["n"]) ** 6
            cnt, sm, s2 = L["count"][b], L["sum"][b], L["sumsq"][b]
            mean[b] = s * sm / cnt
            sem[b] = s * float(sem_from_sums(np.array([cnt]), np.array([sm]), np.array([s2]))[0])
            owner[b] = k
        elif mode == MERGE_POOLED:
            C = S1 = S2 = 0.0
            for k in valid:
                L = levels[k]
                s = float(L["n"]) ** 6
                C += L["count"][b]
                S1 += s * L["sum"][b]
                S2 += s * s * L["sumsq"][b]
            mean[b] = S1 / C
            sem[b] = float(sem_from_sums(np.array([C]), np.array([S1]), np.array([S2]))[0])
            owner[b] = len(valid)
        else:
            W = WM = 0.0
            for k in valid:
                L = levels[k]
                s = float(L["n"]) ** 6
                cnt = L["count"][b]
                m = s * L["sum"][b] / cnt
                e = s * float(sem_from_sums(np.array([cnt]), np.array([L["sum"][b]]),
                                            np.array([L["sumsq"][b]]))[0])
                if not (e > 0.0 and np.isfinite(e)):
                    continue
                W += 1.0 / (e * e)
                WM += m / (e * e)
            if W > 0.0:
                mean[b] = WM / W
                sem[b] = 1.0 / math.sqrt(W)
                owner[b] = len(valid)
    return mean, sem, owner


# ---------------------------------------------------------------------------
# O10  chi^2 misfit and gradients (derived from eq. 1)
# ---------------------------------------------------------------------------

# ---------------------------------------------------------------------------
# O14  polydisperse ensemble
# ---------------------------------------------------------------------------

def ensemble(means: Sequence[np.ndarray], sems: Sequence[np.ndarray], weights: Sequence[float]):
    """Curve of a dilute polydisperse population (Results and Discussion:
    polydispersity as some 200 volume-weighted contributions, one
    simulation each).  Reading: particles scatter incoherently, so with
    number weights w_k the ensemble intensity of a bin is sum_k w_k I_k(b);
    the boxes are independent, so its SEM is sqrt(sum_k (w_k SEM_k(b))^2).
    Every box must share one bin set (same geometry, same counts)."""
    nb = len(means[0])
    mean = np.zeros(nb)
    var = np.zeros(nb)
    for m, e, w in zip(means, sems, weights):
        mean += w * np.asarray(m, dtype=np.float64)
        var += (w * np.asarray(e, dtype=np.float64)) ** 2
    return mean, np.sqrt(var)


# ---------------------------------------------------------------------------
# O16  Ewald-sphere image
# ---------------------------------------------------------------------------

def wavelength_nodes(rel_spread: float, n_lambda: int):
    """Reading of the shell thickness set by the wavelength distribution: a
    Gaussian of relative width rel_spread, truncated at three widths and
    taken at n_lambda evenly spaced points t_j of [-3, 3] with weights
    proportional to exp(-t_j^2 / 2), normalised to sum 1 (lambda_j =
    lambda (1 + rel_spread t_j)).  No spread, or one node: the single point
    t = 0."""
    if rel_spread == 0.0 or n_lambda == 1:
        return np.zeros(1), np.ones(1)
    t = np.linspace(-3.0, 3.0, n_lambda)
    w = np.exp(-0.5 * t * t)
    return t, w / w.sum()


def ewald_pixels(n: int, voxel: float, geo, iv: np.ndarray, iu: np.ndarray, intensity) -> np.ndarray:
    """Ewald-sphere intensities at detector pixels (iv[p], iu[p]) (Q-calculation
    and spherical averaging: intensity taken on the Ewald sphere, a shell
    whose thickness follows the wavelength distribution).

    The pixel (iu, iv) sits at P = distance e + (iu - cu) pixel du +
    (iv - cv) pixel dv from the sample and scatters along s = P / |P|; at
    the wavelength lambda_j the elastic momentum transfer is
    q = (2 pi / lambda_j)(s - e), at grid coordinate g = q / dq with
    dq = 2 pi / (n voxel) (the spacing of eq. 1's frequencies, u along the
    box's x axis).  I = |F|^2 is taken between the grid points by trilinear
    interpolation, the grid periodic (the DFT is), and the result is the
    node-weighted sum over the wavelengths (``wavelength_nodes``).
    ``intensity`` maps an (M, 3) array of frequencies in [0, n) to |F|^2."""
    e, du, dv = (np.asarray(v, dtype=np.float64) for v in (geo.beam, geo.du, geo.dv))
    iv = np.asarray(iv, dtype=np.float64)
    iu = np.asarray(iu, dtype=np.float64)
    P = (geo.distance * e[None, :] + ((iu - geo.cu) * geo.pixel)[:, None] * du[None, :]
         + ((iv - geo.cv) * geo.pixel)[:, None] * dv[None, :])
    s = P / np.linalg.norm(P, axis=-1, keepdims=True)
    dq = 2.0 * math.pi / (n * voxel)
    t, w = wavelength_nodes(geo.rel_spread, geo.n_lambda)
    out = np.zeros(len(iu))
    for tj, wj in zip(t, w):
        k = 2.0 * math.pi / (geo.wavelength * (1.0 + geo.rel_spread * tj))
        g = k * (s - e[None, :]) / dq
        g0 = np.floor(g)
        f = g - g0
        g0 = g0.astype(np.int64)
        val = np.zeros(len(iu))
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    wt = ((f[:, 0] if a else 1.0 - f[:, 0]) * (f[:, 1] if b else 1.0 - f[:, 1])
                          * (f[:, 2] if c else 1.0 - f[:, 2]))
                    val += wt * intensity(np.mod(g0 + np.array([a, b, c]), n))
        out += wj * val
    return out


def ewald_image(F: np.ndarray, voxel: float, geo) -> np.ndarray:
    """O16 over the whole detector from the full n^3 spectrum F[u][v][w] of
    eq. 1; returns image[iv][iu]."""
    n = F.shape[0]
    I = np.abs(np.asarray(F, dtype=np.complex128)) ** 2
    iv, iu = np.meshgrid(np.arange(geo.nv), np.arange(geo.nu), indexing="ij")
    img = ewald_pixels(n, voxel, geo, iv.reshape(-1), iu.reshape(-1), lambda q: I[q[:, 0], q[:, 1], q[:, 2]])
    return img.reshape(geo.nv, geo.nu)


def ewald_pixels_sparse(n: int, voxel: float, geo, iv, iu, xyz: np.ndarray, values: np.ndarray) -> np.ndarray:
    """O16 at chosen pixels of a box that is zero but at the voxels xyz, with
    every needed coefficient of eq. 1 summed directly (``dft_points``): for
    boxes whose transform the oracle cannot hold."""
    def intensity(q):
        uq, inv = np.unique(q, axis=0, return_inverse=True)
        F = dft_points(n, xyz, values, uq)
        return (np.abs(F) ** 2)[inv.reshape(-1)]
    return ewald_pixels(n, voxel, geo, iv, iu, intensity)


# ---------------------------------------------------------------------------
# O17  peak integrals (degree of crystallinity)
# ---------------------------------------------------------------------------

def peak_integrals(edges: np.ndarray, mean: np.ndarray, windows) -> np.ndarray:
    """Integral intensity under a diffraction peak (Results and Discussion:
    the simulated, perfectly crystalline peak integral stands for 100 %
    crystallinity).  Reading: per window [q_lo, q_hi], the populated bins
    whose centres lie in it; the background is the straight line through
    the (centre, mean) of the first and last of them; peak = sum over them
    of (mean - background) * width, total = sum of mean * width.  Rows
    (peak, total, bins used); NaN below two bins."""
    e = np.asarray(edges, dtype=np.float64)
    m = np.asarray(mean, dtype=np.float64)
    q = 0.5 * (e[:-1] + e[1:])
    width = e[1:] - e[:-1]
    out = []
    for lo, hi in np.asarray(windows, dtype=np.float64).reshape(-1, 2):
        idx = [b for b in range(len(m)) if lo <= q[b] <= hi and not np.isnan(m[b])]
        if len(idx) < 2:
            out.append((np.nan, np.nan, float(len(idx))))
            continue
        f, l = idx[0], idx[-1]
        base = lambda x: m[f] + (m[l] - m[f]) * (x - q[f]) / (q[l] - q[f])
        peak = sum((m[b] - base(q[b])) * width[b] for b in idx)
        total = sum(m[b] * width[b] for b in idx)
        out.append((peak, total, float(len(idx))))
    return np.array(out)


def chi2(mean: np.ndarray, count: np.ndarray, target: np.ndarray, rel_sigma: float = 0.01) -> float:
    """chi^2 = sum over populated bins of ((I_b - T_b) / (rel_sigma T_b))^2."""
    m = count > 0
    r = (mean[m] - target[m]) / (rel_sigma * target[m])
    return float(np.sum(r * r))


def chi2_bin_grad(mean, count, target, rel_sigma: float = 0.01) -> np.ndarray:
    """d chi^2 / d I_b = 2 (I_b - T_b) / (rel_sigma T_b)^2 (0 for empty bins)."""
    g = np.zeros_like(mean)
    m = count > 0
    g[m] = 2.0 * (mean[m] - target[m]) / (rel_sigma * target[m]) ** 2
    return g


def grad_rho(F: np.ndarray, voxel: float, edges: np.ndarray, count: np.ndarray,
             g_bin: np.ndarray, weight: np.ndarray | None = None) -> np.ndarray:
    """Gradient of L(I_b) with respect to every voxel density, given
    g_b = dL/dI_b.  With I_b = (1/count_b) sum_{q in b} |F(q)|^2 and eq. 1,
    dI_b/drho(x) = (2/count_b) sum_q Re(conj F(q) e^{-iqx}) / n^3, hence
    grad = 2 Re(IFFT(G * F)) with G(q) = g_{b(q)}/count_{b(q)} (0 for
    unbinned q) and IFFT carrying 1/n^3.  With an intensity weight w(q)
    (the binned values are w |F|^2: the voxel form factor, O15, makes w the
    square of voxel_form), the real weight enters the same way: G w F."""
    n = F.shape[0]
    U = thresholds(n, voxel, edges)
    nb = edges.size - 1
    idx = np.arange(n)
    h = np.where(idx < n // 2, idx, idx - n)
    n2 = h[:, None, None] ** 2 + h[None, :, None] ** 2 + h[None, None, :] ** 2
    b = np.searchsorted(U, n2, side="right") - 1
    ok = (n2 >= U[0]) & (n2 < U[nb])
    Gb = np.where(count > 0, g_bin / np.maximum(count, 1.0), 0.0)
    G = np.zeros(n2.shape)
    G[ok] = Gb[b[ok]]
    if weight is not None:
        G = G * weight
    H = fft3d(G * F, +1) / float(n) ** 3
    return 2.0 * H.real


def fold_to_cell(grad: np.ndarray, n1: int, c: int, mask) -> np.ndarray:
    """Sum of a per-voxel field over every inside voxel that maps to each
    cell voxel (the adjoint of tiling + masking, O2)."""
    n = grad.shape[0]
    assert n == n1
    h = n // 2
    inside = ed1(n, np.ones((c, c, c)), mask)       # mask as 0/1 field
    g = grad * inside
    out = np.zeros((c, c, c))
    idx = (np.arange(n) - h) % c
    for i in range(c):
        gi = g[idx == i]
        for j in range(c):
            gij = gi[:, idx == j]
            for k in range(c):
                out[i, j, k] = gij[:, :, idx == k].sum()
    return out


def grad_amp_oriented(grad_rho_field: np.ndarray, cell, mask) -> np.ndarray:
    """d L / d amp_a for a rotated or polycrystalline lattice (O10 with
    O2r / O2g): the ED-1 is linear in the cell grid (interpolation is a fixed
    linear map of the grid) and the grid is background + sum_a amp_a p_a
    (O1), so d L / d amp_a = sum_x grad_rho(x) rho_a(x), with rho_a the
    lattice's ED-1 of the grid of atom a alone (unit amplitude, no
    background)."""
    n = grad_rho_field.shape[0]
    P = atom_profiles(cell)
    interp = int(getattr(cell, "interp", 1))
    seeds = getattr(cell, "grain_seed", None)
    out = np.empty(P.shape[0])
    for a in range(P.shape[0]):
        grid = P[a, 0][:, None, None] * P[a, 1][None, :, None] * P[a, 2][None, None, :]
        if seeds is not None:
            rho_a = ed1_grains(n, grid, mask, seeds, cell.grain_rot, interp)
        else:
            rho_a = ed1_rot(n, grid, mask, cell.rot, interp)
        out[a] = float(np.sum(grad_rho_field * rho_a))
    return out


def grad_amp(grad_rho_field: np.ndarray, cell, mask) -> np.ndarray:
    """d L / d amp_a = sum over inside voxels of grad_rho(x) * p_a(cell(x)),
    p_a the atom's separable voxel profile (O1)."""
    n = grad_rho_field.shape[0]
    folded = fold_to_cell(grad_rho_field, n, cell.c, mask)
    P = atom_profiles(cell)
    return np.einsum("ijk,ai,aj,ak->a", folded, P[:, 0], P[:, 1], P[:, 2])
