"""Seeded synthetic inputs for the wide-range scattering simulation.

This package only *draws and lays out inputs*: unit-cell atom lists, particle
mask parameters, bin edges, zoom geometry and the named workload recipes.  It
holds none of the method's arithmetic (no density synthesis, no Fourier
transform, no binning, no merging), so both the FP64 oracle and the HIP path
can consume it without sharing any computation.

The paper's own inputs (a DFT electron density of a ZIF-8 unit cell, 630^3
voxels, block-reduced to 105^3; Methodology, "Electron density generation")
are not available.  They are stood in for by cubic unit cells filled with
isotropic Gaussian "atoms" whose positions, electron counts and widths are
drawn from a seeded ``numpy.random.default_rng``.

Random draws happen in a fixed order per recipe: positions U[0, c)^3,
amplitudes U[1, 30), widths U[0.3, 0.8).  The arrays are passed as data to
both sides, so no random number generator is reimplemented anywhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

# Mask kinds (integer codes shared by the C ABI header and the oracle API).
MASK_NONE = 0
MASK_SPHERE = 1
MASK_CUBE = 2
MASK_TRUNC_OCT = 3

PREC_F32 = 0
PREC_F64 = 1


@dataclass(frozen=True)
class Cell:
    """Unit cell of edge ``c`` voxels holding Gaussian atoms.

    ``xyz`` are atom centres in cell-voxel units in [0, c) (voxel i spans
    [i - 1/2, i + 1/2]); ``amp`` is the electron count carried by each atom;
    ``sigma`` the Gaussian width in voxels; ``background`` a uniform density
    added to every cell voxel.
    """

    c: int
    xyz: np.ndarray
    amp: np.ndarray
    sigma: np.ndarray
    background: float = 0.0
    rot: Optional[np.ndarray] = None   # 3x3 lattice orientation (None: aligned with the box)
    interp: int = 1                    # sampling of a rotated cell: 1 trilinear, 3 cubic B-spline
    grain_seed: Optional[np.ndarray] = None   # [G, 3] integer offsets of grain seeds from the particle centre
    grain_rot: Optional[np.ndarray] = None    # [G, 3, 3] grain orientations

    @property
    def n_atoms(self) -> int:
        return int(self.amp.shape[0])

    def with_amp(self, amp: np.ndarray) -> "Cell":
        return replace(self, amp=np.ascontiguousarray(amp, dtype=np.float64))

    def with_grains(self, seeds: np.ndarray, rots: np.ndarray, interp: int = 1) -> "Cell":
        return replace(self, rot=None, interp=int(interp),
                       grain_seed=np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3),
                       grain_rot=np.ascontiguousarray(rots, dtype=np.float64).reshape(-1, 3, 3))

    def with_rot(self, rot: Optional[np.ndarray], interp: int = 1) -> "Cell":
        return replace(self, rot=None if rot is None else np.ascontiguousarray(rot, dtype=np.float64).reshape(3, 3),
                       interp=int(interp))


@dataclass(frozen=True)
class Mask:
    """Particle shape, centred on voxel (N1/2, N1/2, N1/2) of the ED-1 grid.

    Integer parameters so that the inside test is exact integer arithmetic on
    the offset d = (x, y, z) - N1/2:

    * SPHERE:    d.d <= p0                       (p0 = floor(R^2))
    * CUBE:      max |d_i| <= p0                 (p0 = half-width)
    * TRUNC_OCT: max |d_i| <= p0 and sum |d_i| <= p1
                 (p0 = floor(2R/sqrt5), p1 = floor(3R/sqrt5): the truncated
                 octahedron inscribed in a sphere of radius R)
    * NONE:      every voxel inside (p0, p1 ignored)

    An empty particle is expressed with p0 < 0.
    """

    kind: int
    p0: int = 0
    p1: int = 0


@dataclass(frozen=True)
class Zoom:
    """Zoom level: the ED-1 grid of edge ``n1`` block-summed by ``factor``
    per axis and centred in the box of the level that uses it."""

    n1: int
    factor: int = 1


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # box edge (voxels)
    voxel: float           # voxel edge of this box, nm (or unit-less 1.0)
    prec: int              # PREC_F32 / PREC_F64
    transform: str         # "r2c" or "c2c"
    cell: Cell
    mask: Mask
    zoom: Zoom
    edges: np.ndarray      # nbins + 1 strictly increasing bin edges (nm^-1)
    notes: str = ""

    @property
    def nbins(self) -> int:
        return int(self.edges.shape[0] - 1)


# ----------------------------------------------------------------------------
# primitive draws / parameter helpers
# ----------------------------------------------------------------------------

def draw_atoms(seed: int, n_atoms: int, c: int, background: float = 0.0) -> Cell:
    """Gaussian atoms for a cubic cell of edge ``c``: positions U[0,c)^3,
    amplitudes U[1,30) electrons, widths U[0.3,0.8) voxel, in that order."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0.0, float(c), size=(n_atoms, 3))
    amp = rng.uniform(1.0, 30.0, size=n_atoms)
    sigma = rng.uniform(0.3, 0.8, size=n_atoms)
    return Cell(c=c, xyz=np.ascontiguousarray(xyz), amp=np.ascontiguousarray(amp),
                sigma=np.ascontiguousarray(sigma), background=float(background))


def single_atom_cell(c: int, amp: float, sigma: float, background: float,
                     pos=(0.0, 0.0, 0.0)) -> Cell:
    return Cell(c=c, xyz=np.array([pos], dtype=np.float64),
                amp=np.array([amp], dtype=np.float64),
                sigma=np.array([sigma], dtype=np.float64), background=float(background))


def empty_cell(c: int, background: float = 1.0) -> Cell:
    z = np.zeros((0,), dtype=np.float64)
    return Cell(c=c, xyz=np.zeros((0, 3)), amp=z, sigma=z.copy(), background=float(background))


def sphere(radius: float) -> Mask:
    return Mask(MASK_SPHERE, int(math.floor(radius * radius + 1e-9)), 0)


def cube(half_width: int) -> Mask:
    return Mask(MASK_CUBE, int(half_width), 0)


def trunc_oct(radius: float) -> Mask:
    return Mask(MASK_TRUNC_OCT, int(math.floor(2.0 * radius / math.sqrt(5.0))),
                int(math.floor(3.0 * radius / math.sqrt(5.0))))


def no_mask() -> Mask:
    return Mask(MASK_NONE, 0, 0)


def log_edges(lo: float, hi: float, nbins: int) -> np.ndarray:
    i = np.arange(nbins + 1, dtype=np.float64)
    e = lo * (hi / lo) ** (i / nbins)
    e[0], e[-1] = lo, hi
    return e


def lin_edges(lo: float, hi: float, nbins: int) -> np.ndarray:
    i = np.arange(nbins + 1, dtype=np.float64)
    return lo + (hi - lo) * i / nbins


def q_step(n: int, voxel: float) -> float:
    """Frequency spacing 2*pi/(n*voxel) of a box: the bin-range recipe uses it
    to choose edges (it is an input choice, not part of the computation)."""
    return 2.0 * math.pi / (n * voxel)


def default_log_edges(n: int, voxel: float, nbins: int) -> np.ndarray:
    """Log bins from the first shell to the box corner: [dq, sqrt(3)*pi/voxel]."""
    return log_edges(q_step(n, voxel), math.sqrt(3.0) * math.pi / voxel, nbins)


def random_voxels(seed: int, n: int, count: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, size=(count, 3), dtype=np.int64)


def perturbed_amplitudes(cell: Cell, seed: int, rel: float = 0.05) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return cell.amp * (1.0 + rel * rng.standard_normal(cell.n_atoms))


def random_density(seed: int, n: int, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n, n)).astype(dtype)


def sparse_voxels(seed: int, n: int, npts: int, dtype=np.float32):
    """A density that is zero except at npts distinct random voxels:
    (xyz int64 [npts, 3], values [npts] in [0.5, 2) rounded to dtype)."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n * n * n, size=npts, replace=False)
    xyz = np.stack([flat // (n * n), (flat // n) % n, flat % n], axis=1).astype(np.int64)
    val = rng.uniform(0.5, 2.0, npts).astype(dtype)
    return xyz, val


def sparse_slab(seed: int, n: int, x_lo: int, planes: int, npts: int, dtype=np.float32):
    """npts distinct random voxels of planes x_lo .. x_lo + planes - 1 of an
    n^3 box (any y, z), values in [0.5, 2) rounded to dtype."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(planes * n * n, size=npts, replace=False)
    xyz = np.stack([x_lo + flat // (n * n), (flat // n) % n, flat % n], axis=1).astype(np.int64)
    val = rng.uniform(0.5, 2.0, npts).astype(dtype)
    return xyz, val


def random_frequencies(seed: int, n: int, count: int, half_z: bool = True) -> np.ndarray:
    """count random frequency triples (u, v, w) of an n^3 box, w in [0, n/2]
    for a half spectrum, plus the corners (0,0,0) and (n/2, n/2, n/2)."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n, count)
    v = rng.integers(0, n, count)
    w = rng.integers(0, n // 2 + 1 if half_z else n, count)
    q = np.stack([u, v, w], axis=1).astype(np.int64)
    extra = np.array([[0, 0, 0], [n // 2, n // 2, n // 2], [n - 1, 1, n // 2], [1, n - 1, 0]], dtype=np.int64)
    return np.concatenate([extra, q], axis=0)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def c1() -> Workload:
    """64^3 FP64 box, voxel 0.5 nm: uniform sphere (R = 12 voxels, density
    1.0) with a simple-cubic lattice (period 4) of Gaussian blobs
    (sigma 0.6 voxel, 2.0 electrons) inside; 64 linear bins [0, pi/voxel]."""
    cell = single_atom_cell(4, 2.0, 0.6, 1.0)
    return Workload("C1", 64, 0.5, PREC_F64, "c2c", cell, sphere(12.0), Zoom(64, 1),
                    lin_edges(0.0, math.pi / 0.5, 64), "full complex transform")


def lattice_sphere(name: str, n: int, c: int, n_atoms: int, seed: int, radius: float,
                   nbins: int, prec: int = PREC_F32, voxel: float = 1.0) -> Workload:
    cell = draw_atoms(seed, n_atoms, c)
    return Workload(name, n, voxel, prec, "r2c", cell, sphere(radius), Zoom(n, 1),
                    default_log_edges(n, voxel, nbins))


def mixed(n: int, prec: int = PREC_F32, nbins: int = 256, c: int = 16) -> Workload:
    """A box whose edge is not a power of two (2^a 3^b 5^c: the paper's 250,
    500, 1000, 2000 family): the M1024 recipe (cell of c voxels, 16 as
    there, 40 atoms, seed 2) in a sphere of radius 0.39 n, complex
    transform, log bins.  c may be any edge (the paper's reduced cell is
    105^3)."""
    cell = draw_atoms(2, 40, c)
    return Workload(f"M{n}" + ("_f64" if prec == PREC_F64 else ""), n, 1.0, prec, "c2c", cell,
                    sphere(0.39 * n), Zoom(n, 1), default_log_edges(n, 1.0, nbins))


def mixed_zoom(n: int, n1: int, f: int, prec: int = PREC_F32, nbins: int = 64) -> Workload:
    """A zoom level on a box whose edge is not a power of two (the paper's
    ED-2 is its 4000^3 ED-1 block-summed by 16 into 250^3): the mixed()
    particle on an ED-1 grid of edge n1 (sphere of radius 0.39 n1), block
    factor f, voxel f, complex transform."""
    cell = draw_atoms(2, 40, 16)
    return Workload(f"M{n}_from{n1}f{f}", n, float(f), prec, "c2c", cell, sphere(0.39 * n1), Zoom(n1, f),
                    default_log_edges(n, float(f), nbins))


def c2() -> Workload:
    """512^3 FP32: 16-voxel cell with 40 atoms (seed 2), sphere R = 200,
    512 log bins."""
    return lattice_sphere("C2", 512, 16, 40, 2, 200.0, 512)


def m1024(prec: int = PREC_F32) -> Workload:
    """1024^3 headline box: the C2 recipe scaled by two (sphere R = 400),
    512 log bins."""
    return lattice_sphere("M1024" + ("_f64" if prec == PREC_F64 else ""), 1024, 16, 40, 2,
                          400.0, 512, prec)


def c4() -> Workload:
    """256^3 FP32 differentiable box: 40 atoms (seed 4), sphere R = 100,
    256 log bins."""
    return lattice_sphere("C4", 256, 16, 40, 4, 100.0, 256)


def c3_levels() -> List[Workload]:
    """Multi-zoom batch: ED-1 2048^3 (64-voxel cell, 40 atoms, seed 3, sphere
    R = 900), ED-2 1024^3 (block factor 4) and ED-3 512^3 (factor 16), all
    binned on one set of 1024 log edges spanning four decades that end at the
    ED-1 corner frequency sqrt(3)*pi/voxel1."""
    cell = draw_atoms(3, 40, 64)
    mask = sphere(900.0)
    hi = math.sqrt(3.0) * math.pi / 1.0
    edges = log_edges(hi * 1e-4, hi, 1024)
    out = []
    for name, n, f in (("C3-ED1", 2048, 1), ("C3-ED2", 1024, 4), ("C3-ED3", 512, 16)):
        out.append(Workload(name, n, float(f), PREC_F32, "r2c", cell, mask, Zoom(2048, f), edges))
    return out


def zoom_levels(n1: int, c: int, n_atoms: int, seed: int, radius: float, levels, nbins: int,
                decades: float = 4.0) -> List[Workload]:
    """Scaled-down multi-zoom family with the C3 structure: ``levels`` is a
    list of (box edge, block factor)."""
    cell = draw_atoms(seed, n_atoms, c)
    mask = sphere(radius)
    hi = math.sqrt(3.0) * math.pi
    edges = log_edges(hi * 10.0 ** (-decades), hi, nbins)
    return [Workload(f"Z{n}f{f}", n, float(f), PREC_F32, "r2c", cell, mask, Zoom(n1, f), edges)
            for (n, f) in levels]


def b_radii(n: int = 256, count: int = 32, r_lo: float = 20.0, r_hi: float = 100.0, nbins: int = 256,
            prec: int = PREC_F32) -> List[Workload]:
    """Many particle sizes in one batch: the 16-voxel cell with 40 atoms of
    seed 2 (the C2/M1024 cell) inside spheres of ``count`` radii log-spaced
    on [r_lo, r_hi], each an n^3 box with ``nbins`` log bins on [dq, sqrt(3) pi]."""
    cell = draw_atoms(2, 40, 16)
    edges = default_log_edges(n, 1.0, nbins)
    out = []
    for i in range(count):
        r = r_lo * (r_hi / r_lo) ** (i / max(count - 1, 1))
        out.append(Workload(f"B{n}_R{r:.1f}", n, 1.0, prec, "r2c", cell, sphere(r), Zoom(n, 1), edges))
    return out


def rotation(axis: Sequence[float], angle: float) -> np.ndarray:
    """3x3 rotation by `angle` (radians) about `axis` (Rodrigues' formula):
    an orientation for a lattice, input data."""
    k = np.asarray(axis, dtype=np.float64)
    k = k / np.linalg.norm(k)
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def random_grains(seed: int, count: int, radius: float):
    """count grain seeds (distinct integer points within `radius` of the
    particle centre) and orientations uniform over the rotations (unit
    quaternions from four normal deviates): input data for a polycrystalline
    particle."""
    rng = np.random.default_rng(seed)
    r = int(math.floor(radius))
    pts = []
    while len(pts) < count:
        p = tuple(int(v) for v in rng.integers(-r, r + 1, 3))
        if p[0] * p[0] + p[1] * p[1] + p[2] * p[2] <= radius * radius and p not in pts:
            pts.append(p)
    rots = []
    for _ in range(count):
        q = rng.standard_normal(4)
        w, x, y, z = q / np.linalg.norm(q)
        rots.append(np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                              [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                              [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]]))
    return np.array(pts, dtype=np.float64), np.array(rots)


def volume_fractions(radii: Sequence[float], r0: float, width: float) -> np.ndarray:
    """A log-normal volume-fraction distribution over the given radii
    (median r0, log-width `width`), normalised to sum 1: input data for a
    polydisperse ensemble."""
    r = np.asarray(radii, dtype=np.float64)
    phi = np.exp(-0.5 * (np.log(r / r0) / width) ** 2)
    return phi / phi.sum()


@dataclass(frozen=True)
class Ewald:
    """Geometry of a flat detector for an Ewald-sphere image: incident beam
    direction and the detector's row/column directions (orthonormal, box
    axes x, y, z), sample-detector distance and pixel pitch (same unit),
    beam centre in pixels, pixel counts, and the wavelength (nm) with the
    relative Gaussian spread of its distribution and the number of
    wavelength nodes used for it."""
    wavelength: float
    rel_spread: float
    n_lambda: int
    beam: tuple
    du: tuple
    dv: tuple
    distance: float
    pixel: float
    cu: float
    cv: float
    nu: int
    nv: int


def detector(R: np.ndarray, wavelength: float = 0.1, rel_spread: float = 0.0, n_lambda: int = 1,
             distance: float = 1000.0, pixel: float = 0.5, nu: int = 200, nv: int = 160,
             cu: Optional[float] = None, cv: Optional[float] = None) -> Ewald:
    """A detector whose frame (beam, du, dv) is the columns (z, x, y) of the
    rotation R: R = identity puts the beam along z, rows along x and columns
    along y.  Beam centre in the middle unless given."""
    R = np.asarray(R, dtype=np.float64)
    col = lambda i: tuple(float(v) for v in R[:, i])
    return Ewald(float(wavelength), float(rel_spread), int(n_lambda), col(2), col(0), col(1),
                 float(distance), float(pixel), (nu - 1) / 2.0 if cu is None else float(cu),
                 (nv - 1) / 2.0 if cv is None else float(cv), int(nu), int(nv))


def c5(n: int = 4096) -> Workload:
    """Out-of-core box: 128-voxel cell with 200 atoms (seed 5), truncated
    octahedron inscribed in R = 1900 (scaled with n), 2048 log bins."""
    cell = draw_atoms(5, 200, 128)
    r = 1900.0 * n / 4096
    return Workload(f"C5_{n}", n, 1.0, PREC_F32, "r2c", cell, trunc_oct(r), Zoom(n, 1),
                    default_log_edges(n, 1.0, 2048 if n >= 2048 else 512))


def uniform_cube(n: int, half_width: int, nbins: int, prec: int = PREC_F32, value: float = 1.0) -> Workload:
    """A cube of uniform density `value` (a cell without atoms, background
    `value`) on max_i |x_i - n/2| <= half_width; log bins over the box."""
    empty = np.zeros((0, 3))
    cell = Cell(16, empty, np.zeros(0), np.zeros(0), float(value))
    return Workload(f"cube{n}_{half_width}", n, 1.0, prec, "r2c", cell, cube(half_width), Zoom(n, 1),
                    default_log_edges(n, 1.0, nbins))


def small(n: int, c: int = 8, n_atoms: int = 10, seed: int = 7, radius: Optional[float] = None,
          nbins: int = 64, prec: int = PREC_F32, mask: Optional[Mask] = None,
          voxel: float = 1.0, transform: str = "r2c") -> Workload:
    """Small lattice-in-sphere box for parity tests."""
    cell = draw_atoms(seed, n_atoms, c)
    if mask is None:
        mask = sphere(radius if radius is not None else 0.39 * n)
    return Workload(f"S{n}", n, voxel, prec, transform, cell, mask, Zoom(n, 1),
                    default_log_edges(n, voxel, nbins))


CONFIGS = {"C1": c1, "C2": c2, "M1024": m1024, "C4": c4}
