"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, an off-by-one in a threshold)
breaks at least one of them.  None of them re-types the oracle's own code.
"""
import dataclasses
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_dft3(rho):
    """eq. 1 evaluated as a plain triple sum (with its 1/(MNL) factor),
    written as three explicit DFT-matrix contractions."""
    n = rho.shape[0]
    k = np.arange(n)
    Wm = np.exp(-2j * np.pi * np.outer(k, k) / n)
    return np.einsum("ux,vy,wz,xyz->uvw", Wm, Wm, Wm, rho.astype(np.complex128)) / n ** 3


def r3_table():
    vals = []
    with open(os.path.join(GOLDEN, "r3_sum_of_three_squares.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            vals += [int(t) for t in line.split()]
    return np.array(vals)


# ---------------------------------------------------------------------------
# O4  transform
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [6, 8, 10, 12, 15, 16])
def test_fft3d_matches_brute_force_dft(oracle_lib, n):
    rng = np.random.default_rng(n)
    rho = rng.standard_normal((n, n, n))
    F = oracle_lib.forward(rho)
    ref = brute_dft3(rho)
    assert np.max(np.abs(F - ref)) <= 1e-14 * np.max(np.abs(ref)) * n


@pytest.mark.parametrize("n", [2, 4, 8, 32, 256, 4096, 3, 5, 40, 48, 250, 1000, 1536, 2000])
def test_fft1d_matches_library_routine(oracle_lib, n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    ours = oracle_lib.fft1d(a, -1)
    lib = np.fft.fft(a, axis=-1)
    assert np.max(np.abs(ours - lib)) <= 1e-13 * np.max(np.abs(lib))
    back = oracle_lib.fft1d(ours, +1) / n
    assert np.max(np.abs(back - a)) <= 1e-14 * np.max(np.abs(a)) * math.log2(max(n, 2))


@pytest.mark.parametrize("n", [32, 64, 40, 48, 100])
def test_fft3d_matches_library_fftn(oracle_lib, n):
    rng = np.random.default_rng(100 + n)
    rho = rng.standard_normal((n, n, n))
    F = oracle_lib.fft3d(rho, -1)
    ref = np.fft.fftn(rho)
    assert np.max(np.abs(F - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_parseval_and_delta(oracle_lib):
    n = 32
    rng = np.random.default_rng(5)
    rho = rng.standard_normal((n, n, n))
    F = oracle_lib.forward(rho)
    # eq. 1 carries 1/n^3, so sum|F|^2 = sum rho^2 / n^3
    assert abs(np.sum(np.abs(F) ** 2) - np.sum(rho ** 2) / n ** 3) <= 1e-13 * np.sum(rho ** 2) / n ** 3
    d = np.zeros((n, n, n))
    d[3, 7, 11] = 1.0
    I = np.abs(oracle_lib.forward(d)) ** 2
    assert np.allclose(I, n ** -6.0, rtol=1e-13, atol=0)
    # a single delta has a pure phase: F(u,v,w) = exp(-2 pi i (3u+7v+11w)/n) / n^3
    Fd = oracle_lib.forward(d)
    assert abs(Fd[1, 0, 0] - np.exp(-2j * np.pi * 3 / n) / n ** 3) < 1e-18
    assert abs(Fd[0, 0, 1] - np.exp(-2j * np.pi * 11 / n) / n ** 3) < 1e-18


# ---------------------------------------------------------------------------
# O1  unit cell
# ---------------------------------------------------------------------------

def test_atom_profile_integrates_gaussian(oracle_lib):
    from scipy.integrate import quad
    c, x, s = 8, 6.7, 0.55
    p = oracle_lib.atom_profile(c, x, s)
    assert abs(p.sum() - 1.0) < 1e-14
    g = lambda t: math.exp(-0.5 * ((t - x) / s) ** 2) / (s * math.sqrt(2 * math.pi))
    for i in range(c):
        # periodic images: voxel i collects the Gaussian over i + m*c
        ref = sum(quad(g, i - 0.5 + m * c, i + 0.5 + m * c, epsabs=1e-15, epsrel=1e-13)[0]
                  for m in (-1, 0, 1))
        assert abs(p[i] - ref) < 1e-12


def test_cell_electron_count_and_symmetry(oracle_lib):
    cell = W.draw_atoms(11, 7, 16, background=0.25)
    g = oracle_lib.cell_synth(cell)
    assert abs(g.sum() - (0.25 * 16 ** 3 + cell.amp.sum())) < 1e-11
    # an atom at the cell centre gives a mirror-symmetric cell about that centre
    one = W.single_atom_cell(8, 3.0, 0.7, 0.0, pos=(4.0, 4.0, 4.0))
    h = oracle_lib.cell_synth(one)
    idx = (8 - np.arange(8)) % 8
    assert np.allclose(h, h[idx][:, idx][:, :, idx], rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# O2  tiling and masks
# ---------------------------------------------------------------------------

def test_unmasked_tiling_is_a_comb(oracle_lib):
    """Without a mask the box is the cell repeated n/c times per axis: the
    spectrum vanishes off the comb u = 0 mod n/c and on the comb equals the
    cell's own DFT / c^3 (Bragg peaks at Q = 2 pi h / (c voxel))."""
    n, c = 32, 8
    cell = W.draw_atoms(3, 5, c)
    g = oracle_lib.cell_synth(cell)
    rho = oracle_lib.ed1(n, g, W.no_mask())
    F = oracle_lib.forward(rho)
    step = n // c
    on = np.zeros((n, n, n), dtype=bool)
    on[::step, ::step, ::step] = True
    assert np.max(np.abs(F[~on])) < 1e-14 * np.max(np.abs(F))
    Fc = brute_dft3(g)     # = DFT_c(cell) / c^3
    sign = (-1.0) ** (np.add.outer(np.add.outer(np.arange(c), np.arange(c)), np.arange(c)) * step)
    assert np.max(np.abs(F[::step, ::step, ::step] - Fc * sign)) < 1e-13 * np.max(np.abs(Fc))


def test_mask_voxel_counts_are_lattice_point_counts(oracle_lib):
    n = 64
    ones = np.ones((4, 4, 4))
    for R2 in (0, 1, 2, 3, 50, 144, 300):
        rho = oracle_lib.ed1(n, ones, W.Mask(W.MASK_SPHERE, R2))
        # points of Z^3 in the ball |d|^2 <= R2: sum of r3 over shells
        r3 = r3_table()
        if R2 < len(r3):
            assert rho.sum() == r3[: R2 + 1].sum()
        # and a direct count over (dx, dy) with an integer root for dz
        cnt = 0
        R = int(math.isqrt(R2))
        for dx in range(-R, R + 1):
            for dy in range(-R, R + 1):
                rem = R2 - dx * dx - dy * dy
                if rem >= 0:
                    cnt += 2 * math.isqrt(rem) + 1
        assert rho.sum() == cnt
    # truncated octahedron: max|d| <= a and sum|d| <= b
    a, b = 5, 8
    rho = oracle_lib.ed1(n, ones, W.Mask(W.MASK_TRUNC_OCT, a, b))
    cnt = sum(1 for x in range(-a, a + 1) for y in range(-a, a + 1) for z in range(-a, a + 1)
              if abs(x) + abs(y) + abs(z) <= b)
    assert rho.sum() == cnt
    assert rho[n // 2 + a, n // 2, n // 2] == 1 and rho[n // 2 + a + 1, n // 2, n // 2] == 0
    assert oracle_lib.ed1(n, ones, W.Mask(W.MASK_SPHERE, -1)).sum() == 0


@pytest.mark.parametrize("R", [3.0, 5.3, 9.999999, 11.3, 12.0, 17.9, 25.0, 28.62])
def test_integer_mask_parameters_match_real_shapes(oracle_lib, R):
    """The masks cross the boundary as integers (inside test on the integer
    offset d of a voxel centre); the workload constructors derive them from
    a real radius R.  The integer masks must contain exactly the voxel
    centres of the real shapes: the ball |d| <= R, and the truncated
    octahedron inscribed in it, built here independently as the convex hull
    of its 24 vertices (permutations of (0, +-1, +-2) R / sqrt 5, all at
    distance R from the centre; square faces normal to the axes)."""
    from itertools import permutations
    from scipy.spatial import ConvexHull
    n = 64
    ones = np.ones((4, 4, 4))
    r = int(math.ceil(R)) + 1
    g = np.arange(-r, r + 1, dtype=np.float64)
    d = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    # ball: voxel centres within distance R (real arithmetic, tie within 1e-9)
    ball = int(np.count_nonzero(np.sqrt(np.sum(d * d, axis=1)) <= R + 1e-9))
    assert oracle_lib.ed1(n, ones, W.sphere(R)).sum() == ball
    # truncated octahedron as a hull of vertices, not of the face planes
    base = set()
    for p in permutations((0.0, 1.0, 2.0)):
        for sx in (-1, 1):
            for sy in (-1, 1):
                for sz in (-1, 1):
                    base.add((sx * p[0], sy * p[1], sz * p[2]))
    verts = np.array(sorted(base)) * (R / math.sqrt(5.0))
    assert len(verts) == 24 and np.allclose(np.linalg.norm(verts, axis=1), R)
    hull = ConvexHull(verts)
    side = d @ hull.equations[:, :3].T + hull.equations[:, 3]
    inside = int(np.count_nonzero(np.all(side <= 1e-9, axis=1)))
    assert oracle_lib.ed1(n, ones, W.trunc_oct(R)).sum() == inside


def test_cube_mask_dirichlet_closed_form(oracle_lib):
    """Uniform cube of half-width h: |F|^2 = prod_axes D(u)^2 with the Dirichlet
    kernel D(u) = sin(pi u (2h+1)/n) / (n sin(pi u / n)), D(0) = (2h+1)/n."""
    n, h = 32, 5
    rho = oracle_lib.ed1(n, np.ones((4, 4, 4)), W.cube(h))
    I = np.abs(oracle_lib.forward(rho)) ** 2
    u = np.arange(n)
    with np.errstate(invalid="ignore", divide="ignore"):
        D = np.sin(np.pi * u * (2 * h + 1) / n) / (n * np.sin(np.pi * u / n))
    D[0] = (2 * h + 1) / n
    ref = (D[:, None, None] * D[None, :, None] * D[None, None, :]) ** 2
    assert np.max(np.abs(I - ref)) < 1e-15


# ---------------------------------------------------------------------------
# O3  zoom
# ---------------------------------------------------------------------------

def test_zoom_block_sum(oracle_lib):
    n1, f, nk, c = 32, 4, 16, 8
    cell = W.draw_atoms(9, 6, c)
    g = oracle_lib.cell_synth(cell)
    mask = W.sphere(11.0)
    rho1 = oracle_lib.ed1(n1, g, mask)
    rk = oracle_lib.zoomed(n1, g, mask, f, nk)
    m = n1 // f
    o = (nk - m) // 2
    blocks = rho1.reshape(m, f, m, f, m, f).sum(axis=(1, 3, 5))
    ref = np.zeros((nk, nk, nk))
    ref[o:o + m, o:o + m, o:o + m] = blocks
    assert np.max(np.abs(rk - ref)) < 1e-12
    assert abs(rk.sum() - rho1.sum()) < 1e-10 * abs(rho1.sum())


@pytest.mark.parametrize("f", [2, 4])
def test_zoom_levels_of_rotated_lattices(oracle_lib, f):
    """O3 of an oriented ED-1: with the identity orientation the level equals
    the aligned level of the C route (block sums evaluated per level voxel);
    for a general orientation, cubic sampling and grains the level keeps the
    electrons of its ED-1 and is zero outside the reduced region."""
    from dataclasses import replace
    n1, nk, c = 32, 16, 8
    base = W.zoom_levels(n1, c, 6, 9, 11.0, [(nk, f)], 16)[0]
    g = oracle_lib.cell_synth(base.cell)
    ident = replace(base, cell=base.cell.with_rot(np.eye(3), 1))
    assert np.max(np.abs(oracle_lib.density(ident, g) - oracle_lib.zoomed(n1, g, base.mask, f, nk))) < 1e-12
    m, o = n1 // f, (nk - n1 // f) // 2
    R = W.rotation([1.0, 2.0, 3.0], 0.7)
    seeds, rots = W.random_grains(5, 4, 0.3 * n1)
    for cell, rho1 in ((base.cell.with_rot(R, 1), oracle_lib.ed1_rot(n1, g, base.mask, R, 1)),
                       (base.cell.with_rot(R, 3), oracle_lib.ed1_rot(n1, g, base.mask, R, 3)),
                       (base.cell.with_grains(seeds, rots, 1), oracle_lib.ed1_grains(n1, g, base.mask, seeds, rots, 1))):
        lvl = oracle_lib.density(replace(base, cell=cell), g)
        assert abs(lvl.sum() - rho1.sum()) <= 1e-10 * abs(rho1.sum())
        inner = np.zeros_like(lvl, dtype=bool)
        inner[o:o + m, o:o + m, o:o + m] = True
        assert np.all(lvl[~inner] == 0.0)
        assert abs(lvl[o, o, o] - rho1[:f, :f, :f].sum()) <= 1e-12 * max(1.0, abs(rho1).max())


# ---------------------------------------------------------------------------
# O5-O8  binning
# ---------------------------------------------------------------------------

def test_linear_bin_thresholds_closed_form(oracle_lib):
    """C1 bins: 64 linear bins on [0, pi/voxel] of a 64^3 box are half a
    frequency step wide, so edge b sits at n2 = b^2/4: U_b = ceil(b^2/4)."""
    wl = W.c1()
    U = oracle_lib.thresholds(wl.n, wl.voxel, wl.edges)
    b = np.arange(64)
    assert np.array_equal(U[:64], -((-(b * b)) // 4))
    assert U[64] == 32 * 32 + 1      # last edge inclusive: n2 = 1024 is in
    # log bins from dq to the corner: first threshold 1, last 3 n^2/4 inclusive
    wl2 = W.small(64, nbins=50)
    U2 = oracle_lib.thresholds(64, 1.0, wl2.edges)
    assert U2[0] == 1 and U2[-1] == 3 * 32 * 32 + 1


@pytest.mark.parametrize("n", [32, 40, 48])
def test_bin_counts_are_shell_counts(oracle_lib, n):
    edges = W.lin_edges(0.0, 16 * 2.0 * math.pi / n, 64)     # U_b = ceil(b^2/4) as above
    cnt = oracle_lib.bin_counts(n, 1.0, edges)
    U = oracle_lib.thresholds(n, 1.0, edges)
    r3 = r3_table()
    for b in range(64):
        if U[b + 1] - 1 < len(r3):
            assert cnt[b] == r3[U[b]:U[b + 1]].sum(), b
    # every voxel is binned once or left out: total = voxels with n2 <= 256
    h = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n)
    n2 = h[:, None, None] ** 2 + h[None, :, None] ** 2 + h[None, None, :] ** 2
    assert cnt.sum() == np.count_nonzero(n2 <= 256)


def test_bin_statistics_of_constructed_spectra(oracle_lib):
    n = 16
    edges = W.lin_edges(0.0, math.pi, 16)
    # constant |F|: every populated bin has mean |c|^2 and zero spread
    F = np.full((n, n, n), 0.3 - 0.4j)
    r = oracle_lib.bin_spectrum(F, 1.0, edges)
    pop = r["count"] > 0
    assert np.allclose(r["mean"][pop], 0.25, rtol=1e-15)
    assert np.all(r["sem"][r["count"] > 1] < 1e-16)
    assert np.all(np.isnan(r["mean"][~pop]))
    assert abs(r["totals"][0] - 0.25 * n ** 3) < 1e-10
    # |F|^2 = n2: the mean over a bin is the mean of n2 over its shells,
    # sum_m m r3(m) / sum_m r3(m)
    h = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n)
    n2 = (h[:, None, None] ** 2 + h[None, :, None] ** 2 + h[None, None, :] ** 2).astype(float)
    r = oracle_lib.bin_spectrum(np.sqrt(n2).astype(complex), 1.0, edges)
    U = oracle_lib.thresholds(n, 1.0, edges)
    r3 = r3_table()
    checked = 0
    for b in range(16):
        if U[b + 1] > len(r3):
            break
        m = np.arange(U[b], U[b + 1])
        w = r3[m]
        c = w.sum()
        if c > 0:
            mean = (m * w).sum() / c
            assert abs(r["mean"][b] - mean) < 1e-12
            assert r["count"][b] == c
            if c == 1:
                assert np.isnan(r["sem"][b])              # one voxel: no spread estimate
                continue
            # SEM from the shell table: the population variance of n2 over the
            # bin, sum m^2 r3 / sum r3 - mean^2, turned into the sample
            # variance (x c/(c-1)) and divided by the count
            var_pop = (m * m * w).sum() / c - mean * mean
            sem = math.sqrt(max(var_pop, 0.0) * c / (c - 1.0) / c)
            if np.count_nonzero(w) == 1:                  # one shell: every value equal
                assert r["sem"][b] <= 1e-12 * mean, (b, r["sem"][b])
                continue
            assert abs(r["sem"][b] - sem) <= 1e-12 * sem, (b, r["sem"][b], sem)
            checked += 1
    assert checked >= 8 and r["count"][0] == 1


def test_circular_shift_leaves_bins_unchanged(oracle_lib):
    wl = W.small(32, c=8, n_atoms=5, radius=9.0, nbins=40)
    g = oracle_lib.cell_synth(wl.cell)
    rho = oracle_lib.ed1(32, g, wl.mask)
    a = oracle_lib.bin_spectrum(oracle_lib.forward(rho), 1.0, wl.edges)
    b = oracle_lib.bin_spectrum(oracle_lib.forward(np.roll(rho, (3, -5, 7), axis=(0, 1, 2))),
                                1.0, wl.edges)
    pop = a["count"] > 0
    assert np.allclose(a["mean"][pop], b["mean"][pop], rtol=1e-12)


# ---------------------------------------------------------------------------
# whole forward path against physics
# ---------------------------------------------------------------------------

def test_uniform_sphere_form_factor(oracle_lib):
    """A uniform voxelised sphere follows the continuous form factor
    [3 (sin qR - qR cos qR)/(qR)^3]^2 at low q (R from the voxel volume)."""
    n, R = 128, 16.0
    wl = W.Workload("sph", n, 1.0, W.PREC_F64, "r2c", W.empty_cell(4, 1.0), W.sphere(R),
                    W.Zoom(n, 1), W.lin_edges(0.0, math.pi, 64))
    rho = oracle_lib.density(wl)
    F = oracle_lib.forward(rho)
    V = rho.sum()
    Reff = (3.0 * V / (4.0 * math.pi)) ** (1.0 / 3.0)
    I0 = (V / n ** 3) ** 2
    assert abs(abs(F[0, 0, 0]) ** 2 - I0) < 1e-12 * I0
    dq = 2 * math.pi / n
    for (u, v, w) in [(1, 0, 0), (0, 2, 0), (2, 2, 1), (3, 0, 0), (0, 4, 3)]:
        q = dq * math.sqrt(u * u + v * v + w * w)
        x = q * Reff
        ff = (3 * (math.sin(x) - x * math.cos(x)) / x ** 3) ** 2
        assert abs(abs(F[u, v, w]) ** 2 / I0 - ff) < 0.02 * max(ff, 0.05), (u, v, w)
    # the first zero of the form factor sits at qR = 4.493: deep minimum there
    u0 = 4.493 / Reff / dq
    near = np.abs(F[int(round(u0)), 0, 0]) ** 2 / I0
    assert near < 0.02


def test_lowfreq_direct_sum_matches_transform(oracle_lib):
    """O11 (direct summation in the order of eq. 2) against O4 (recursive
    FFT): two independent routes to the same coefficients."""
    wl = W.small(32, c=8, n_atoms=6, radius=10.0, nbins=30)
    g = oracle_lib.cell_synth(wl.cell)
    F = oracle_lib.forward(oracle_lib.density(wl, g))
    K = 3
    D = oracle_lib.lowfreq_dft(wl, K, g)
    r = np.arange(-K, K + 1) % 32
    ref = F[np.ix_(r, r, r)]
    assert np.max(np.abs(D - ref)) < 1e-14 * np.max(np.abs(ref)) * 10
    # zoomed level (factor 2 into a 32 box from a 32 ED-1)
    wz = W.Workload("z", 32, 2.0, W.PREC_F64, "r2c", wl.cell, wl.mask, W.Zoom(32, 2), wl.edges)
    Fz = oracle_lib.forward(oracle_lib.density(wz, g))
    Dz = oracle_lib.lowfreq_dft(wz, K, g)
    assert np.max(np.abs(Dz - Fz[np.ix_(r, r, r)])) < 1e-13 * np.max(np.abs(Fz))
    s1, s2 = oracle_lib.density_moments(wz, g)
    rz = oracle_lib.density(wz, g)
    assert abs(s1 - rz.sum()) < 1e-11 * abs(s1) and abs(s2 - (rz ** 2).sum()) < 1e-11 * s2


def test_lowfreq_bins_match_full_binning(oracle_lib):
    wl = W.small(32, c=8, n_atoms=6, radius=10.0, nbins=200)
    g = oracle_lib.cell_synth(wl.cell)
    full = oracle_lib.bin_spectrum(oracle_lib.forward(oracle_lib.density(wl, g)), wl.voxel, wl.edges)
    sel, cnt, s, mean = oracle_lib.lowfreq_bins(wl, 4, g)
    assert len(sel) > 10
    assert np.array_equal(cnt, full["count"][sel])
    assert np.allclose(mean, full["mean"][sel], rtol=1e-12, equal_nan=True)


# ---------------------------------------------------------------------------
# O9  merge
# ---------------------------------------------------------------------------

def _level(n, voxel, count, mean, spread):
    count = np.asarray(count, dtype=float)
    s = count * mean
    s2 = count * (mean ** 2 + spread ** 2)
    return {"n": n, "voxel": voxel, "count": count, "sum": s, "sumsq": s2}


def test_merge_rules_on_constructed_levels(oracle_lib):
    edges = np.array([0.002, 0.004, 0.02, 0.2, 1.0, 2.0, 4.0])
    nb = 6
    # fine level: n=64, voxel 1  -> dq = 0.098, qcut = 2.72
    # coarse level: n=64, voxel 8 -> dq = 0.0123, qcut = 0.34
    fine = _level(64, 1.0, [0, 0, 40, 100, 100, 100], np.full(nb, 2.0) / 64.0 ** 6, 0.5 / 64.0 ** 6)
    coarse = _level(64, 8.0, [0, 40, 40, 40, 40, 40], np.full(nb, 3.0) / 64.0 ** 6, 0.5 / 64.0 ** 6)
    mean, sem, owner = oracle_lib.merge([coarse, fine], edges, oracle_lib.MERGE_FINEST, 32)
    qc = oracle_lib.bin_centres(edges)
    # bin 0: centre 0.0028 below both dq -> no owner
    assert owner[0] == -1 and np.isnan(mean[0])
    # bin 1 (centre 0.0089 < dq_coarse 0.0123): no owner either
    assert owner[1] == -1
    # bin 2 (0.063): coarse valid (0.0123..0.34), fine not (below 0.098) -> coarse
    assert owner[2] == 0 and abs(mean[2] - 3.0) < 1e-12
    # bin 3 (0.447): beyond coarse qcut, fine valid -> fine
    assert owner[3] == 1 and abs(mean[3] - 2.0) < 1e-12
    # SEM of the owner: sqrt(var * c/(c-1) / c) with var = spread^2
    c = 100.0
    assert abs(sem[3] - math.sqrt(0.25 * c / (c - 1) / c)) < 1e-12
    # bin 5 (2.83) beyond the fine cut 2.72 -> no owner
    assert qc[5] > math.sqrt(3) * math.pi / 2 and owner[5] == -1
    # pooled with a single valid level equals that level; IVW likewise
    mp, sp, op = oracle_lib.merge([coarse, fine], edges, oracle_lib.MERGE_POOLED, 32)
    assert abs(mp[3] - 2.0) < 1e-12 and op[3] == 1
    # n_min above the available counts removes the owner
    m2, _, o2 = oracle_lib.merge([coarse, fine], edges, oracle_lib.MERGE_FINEST, 101)
    assert o2[3] == -1


def test_merge_pooled_and_ivw_two_levels(oracle_lib):
    """Two levels both valid for one bin (centre 0.141): a (n 256, voxel 0.2:
    dq 0.123, cut 13.6) and b (n 128, voxel 0.5: dq 0.098, cut 5.44)."""
    edges = np.array([0.1, 0.2])
    a = _level(256, 0.2, [50], np.array([4.0]) / 256.0 ** 6, 1.0 / 256.0 ** 6)
    b = _level(128, 0.5, [150], np.array([2.0]) / 128.0 ** 6, 2.0 / 128.0 ** 6)
    mp, sp, op = oracle_lib.merge([a, b], edges, oracle_lib.MERGE_POOLED, 32)
    assert op[0] == 2
    assert abs(mp[0] - (50 * 4.0 + 150 * 2.0) / 200.0) < 1e-12
    # pooled spread: (sum of count*(m^2+s^2) - C*mean^2) / (C-1), SEM = sqrt(var/C)
    var = (50 * 17.0 + 150 * 8.0 - 200 * 2.5 ** 2) / 199.0
    assert abs(sp[0] - math.sqrt(var / 200.0)) < 1e-12
    mi, si, oi = oracle_lib.merge([a, b], edges, oracle_lib.MERGE_IVW, 32)
    ea = 1.0 / math.sqrt(49.0)          # SEM = spread / sqrt(count - 1)
    eb = 2.0 / math.sqrt(149.0)
    wa, wb = 1 / ea ** 2, 1 / eb ** 2
    assert abs(mi[0] - (wa * 4.0 + wb * 2.0) / (wa + wb)) < 1e-10
    assert abs(si[0] - 1 / math.sqrt(wa + wb)) < 1e-10
    mf, _, of = oracle_lib.merge([a, b], edges, oracle_lib.MERGE_FINEST, 32)
    assert of[0] == 0 and abs(mf[0] - 4.0) < 1e-12    # a has the smaller voxel


# ---------------------------------------------------------------------------
# O10  chi^2 gradients against finite differences of the forward oracle
# ---------------------------------------------------------------------------

def _forward_curve(oracle_lib, rho, wl):
    F = oracle_lib.forward(rho)
    r = oracle_lib.bin_spectrum(F, wl.voxel, wl.edges)
    return F, r


def test_grad_rho_matches_central_differences(oracle_lib):
    wl = W.small(16, c=4, n_atoms=3, radius=5.0, nbins=12)
    g = oracle_lib.cell_synth(wl.cell)
    rho = oracle_lib.density(wl, g)
    rng = np.random.default_rng(1)
    target_rho = rho * (1 + 0.05 * rng.standard_normal(rho.shape))
    _, tr = _forward_curve(oracle_lib, target_rho, wl)
    T = np.where(tr["count"] > 0, tr["mean"], 1.0)
    F, r = _forward_curve(oracle_lib, rho, wl)
    gb = oracle_lib.chi2_bin_grad(r["mean"], r["count"], T)
    grad = oracle_lib.grad_rho(F, wl.voxel, wl.edges, r["count"], gb)
    h = 1e-4
    for (x, y, z) in [(8, 8, 8), (5, 9, 7), (0, 0, 0), (12, 3, 8)]:
        rp = rho.copy(); rp[x, y, z] += h
        rm = rho.copy(); rm[x, y, z] -= h
        _, a = _forward_curve(oracle_lib, rp, wl)
        _, b = _forward_curve(oracle_lib, rm, wl)
        fd = (oracle_lib.chi2(a["mean"], a["count"], T) - oracle_lib.chi2(b["mean"], b["count"], T)) / (2 * h)
        assert abs(fd - grad[x, y, z]) <= 1e-6 * max(1.0, abs(fd)), (x, y, z, fd, grad[x, y, z])


def test_grad_rho_with_voxel_form_factor_matches_central_differences(oracle_lib):
    """The voxel form factor (O15) weights every intensity by the square of
    voxel_form; the gradient takes that weight (O10), checked against central
    differences of chi^2 through the weighted forward curve.  The weight is
    far from 1 near the box's Nyquist frequencies at n = 16, so a dropped or
    unsquared weight fails."""
    wl = W.small(16, c=4, n_atoms=3, radius=5.0, nbins=12)
    g = oracle_lib.cell_synth(wl.cell)
    rho = oracle_lib.density(wl, g)
    S = oracle_lib.voxel_form(wl.n)

    def curve(r):
        F = oracle_lib.forward(r)
        return F, oracle_lib.bin_spectrum(F * S, wl.voxel, wl.edges)

    rng = np.random.default_rng(2)
    _, tr = curve(rho * (1 + 0.05 * rng.standard_normal(rho.shape)))
    T = np.where(tr["count"] > 0, tr["mean"], 1.0)
    F, r = curve(rho)
    gb = oracle_lib.chi2_bin_grad(r["mean"], r["count"], T)
    grad = oracle_lib.grad_rho(F, wl.voxel, wl.edges, r["count"], gb, weight=S * S)
    plain = oracle_lib.grad_rho(F, wl.voxel, wl.edges, r["count"], gb)
    assert np.max(np.abs(plain - grad)) > 1e-3 * np.max(np.abs(grad))
    h = 1e-4
    for (x, y, z) in [(8, 8, 8), (5, 9, 7), (0, 0, 0), (12, 3, 8)]:
        rp = rho.copy(); rp[x, y, z] += h
        rm = rho.copy(); rm[x, y, z] -= h
        _, a = curve(rp)
        _, b = curve(rm)
        fd = (oracle_lib.chi2(a["mean"], a["count"], T) - oracle_lib.chi2(b["mean"], b["count"], T)) / (2 * h)
        assert abs(fd - grad[x, y, z]) <= 1e-6 * max(1.0, abs(fd)), (x, y, z, fd, grad[x, y, z])


def test_grad_amp_matches_central_differences(oracle_lib):
    wl = W.small(16, c=4, n_atoms=3, radius=5.0, nbins=12)
    cell = wl.cell
    tgt = cell.with_amp(cell.amp * np.array([1.05, 0.97, 1.02]))
    wt = W.Workload("t", wl.n, wl.voxel, wl.prec, wl.transform, tgt, wl.mask, wl.zoom, wl.edges)
    tr = oracle_lib.simulate(wt)
    T = np.where(tr["count"] > 0, tr["mean"], 1.0)

    def loss(c):
        w2 = W.Workload("x", wl.n, wl.voxel, wl.prec, wl.transform, c, wl.mask, wl.zoom, wl.edges)
        r = oracle_lib.simulate(w2, return_fields=True)
        return oracle_lib.chi2(r["mean"], r["count"], T), r

    L0, r = loss(cell)
    gb = oracle_lib.chi2_bin_grad(r["mean"], r["count"], T)
    grho = oracle_lib.grad_rho(r["F"], wl.voxel, wl.edges, r["count"], gb)
    ga = oracle_lib.grad_amp(grho, cell, wl.mask)
    h = 1e-4
    for a in range(cell.n_atoms):
        up = cell.amp.copy(); up[a] += h
        dn = cell.amp.copy(); dn[a] -= h
        fd = (loss(cell.with_amp(up))[0] - loss(cell.with_amp(dn))[0]) / (2 * h)
        assert abs(fd - ga[a]) <= 1e-6 * max(1.0, abs(fd)), (a, fd, ga[a])


@pytest.mark.parametrize("kind", ["rotated", "grains"])
def test_grad_amp_oriented_matches_central_differences(oracle_lib, kind):
    """The amplitude gradient of a rotated lattice and of a polycrystal
    (trilinear sampling), by linearity, against central differences of chi^2
    through the whole oracle forward path."""
    wl = W.small(16, c=4, n_atoms=3, radius=5.0, nbins=12)
    if kind == "rotated":
        cell = wl.cell.with_rot(W.rotation([1.0, 2.0, 3.0], 0.7), 1)
    else:
        seeds, rots = W.random_grains(7, 3, 4.0)
        cell = wl.cell.with_grains(seeds, rots, 1)
    tgt = cell.with_amp(cell.amp * np.array([1.05, 0.97, 1.02]))
    wt = W.Workload("t", wl.n, wl.voxel, wl.prec, wl.transform, tgt, wl.mask, wl.zoom, wl.edges)
    tr = oracle_lib.simulate(wt)
    T = np.where(tr["count"] > 0, tr["mean"], 1.0)

    def loss(c):
        w2 = W.Workload("x", wl.n, wl.voxel, wl.prec, wl.transform, c, wl.mask, wl.zoom, wl.edges)
        r = oracle_lib.simulate(w2, return_fields=True)
        return oracle_lib.chi2(r["mean"], r["count"], T), r

    L0, r = loss(cell)
    gb = oracle_lib.chi2_bin_grad(r["mean"], r["count"], T)
    grho = oracle_lib.grad_rho(r["F"], wl.voxel, wl.edges, r["count"], gb)
    ga = oracle_lib.grad_amp_oriented(grho, cell, wl.mask)
    h = 1e-4
    for a in range(cell.n_atoms):
        up = cell.amp.copy(); up[a] += h
        dn = cell.amp.copy(); dn[a] -= h
        fd = (loss(cell.with_amp(up))[0] - loss(cell.with_amp(dn))[0]) / (2 * h)
        assert abs(fd - ga[a]) <= 1e-6 * max(1.0, abs(fd)), (a, fd, ga[a])


# ---------------------------------------------------------------------------
# eq. 1 at sampled frequencies for sparse densities (used to check boxes too
# large for the full oracle transform)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 32])
def test_dft_points_matches_numpy_fftn(oracle_lib, n):
    """Every frequency of a sparse box against numpy.fft.fftn / n^3 (pocketfft,
    a library routine independent of the oracle)."""
    import oracle
    xyz, val = W.sparse_voxels(5 + n, n, 17, dtype=np.float64)
    rho = np.zeros((n, n, n))
    rho[xyz[:, 0], xyz[:, 1], xyz[:, 2]] = val
    ref = np.fft.fftn(rho) / n ** 3
    u, v, w = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    uvw = np.stack([u.ravel(), v.ravel(), w.ravel()], axis=1)
    got = oracle.dft_points(n, xyz, val, uvw).reshape(n, n, n)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_dft_points_large_box_phase_reduction(oracle_lib):
    """At n = 2048 the integer phase reduction must agree with the same
    coefficients computed for the box embedded at 4x the resolution of a
    16-voxel lattice: a density on every 128th voxel of a 2048 box is a 16^3
    box, whose transform (numpy) repeats with period 16 in each frequency."""
    import oracle
    n, m = 2048, 16
    xyz_c, val = W.sparse_voxels(77, m, 9, dtype=np.float64)
    xyz = xyz_c * (n // m)
    rho_c = np.zeros((m, m, m))
    rho_c[xyz_c[:, 0], xyz_c[:, 1], xyz_c[:, 2]] = val
    ref_c = np.fft.fftn(rho_c) / float(n) ** 3          # same sums, box normalisation 1/n^3
    uvw = W.random_frequencies(78, n, 200, half_z=False)
    got = oracle.dft_points(n, xyz, val, uvw)
    ref = ref_c[uvw[:, 0] % m, uvw[:, 1] % m, uvw[:, 2] % m]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# O12: per-bin counts and two-voxel intensities without the n^3 loops (used
# at 4096^3, where neither the oracle transform nor its binning loop fits)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 32, 64])
def test_separable_counts_equal_voxel_loop(oracle_lib, n):
    """Counts taken axis by axis against the n^3 voxel loop, for log bins
    (last edge inclusive) and linear bins that end inside the box."""
    import oracle
    for edges in (W.default_log_edges(n, 1.0, 40), W.lin_edges(0.0, 0.8 * math.pi, 23)):
        cnt, _ = oracle.axis_pair_bins(n, 1.0, edges, 3, 1.0, 0.5)
        assert np.array_equal(cnt, oracle_lib.bin_counts(n, 1.0, edges))


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_two_voxel_bin_sums_match_library_transform(oracle_lib, n, axis):
    """Two voxels d apart along one axis: the closed form of O12 against
    numpy.fft.fftn / n^3 binned voxel by voxel, for a d coprime to n (every
    phase distinct) and d = n/2 (alternating signs)."""
    import oracle
    edges = W.default_log_edges(n, 1.0, 30)
    for d in (3, n // 2):
        p = np.array([5, 9, 2])
        q = p.copy()
        q[axis] = (q[axis] + d) % n
        rho = np.zeros((n, n, n))
        rho[tuple(p)] = 1.0
        rho[tuple(q)] = 0.6
        ref = oracle_lib.bin_spectrum(np.fft.fftn(rho) / float(n) ** 3, 1.0, edges)
        cnt, s = oracle.axis_pair_bins(n, 1.0, edges, d, 1.0, 0.6)
        assert np.array_equal(cnt, ref["count"])
        assert np.max(np.abs(s - ref["sum"])) <= 1e-12 * np.max(ref["sum"])


def test_sparse_low_bins_match_full_binning(oracle_lib):
    """Bins below n2 = m from direct summation over the nonzero voxels
    against numpy.fft.fftn / n^3 binned voxel by voxel."""
    import oracle
    n = 32
    xyz, val = W.sparse_voxels(91, n, 23, dtype=np.float64)
    rho = np.zeros((n, n, n))
    np.add.at(rho, (xyz[:, 0], xyz[:, 1], xyz[:, 2]), val)
    edges = W.default_log_edges(n, 1.0, 60)
    ref = oracle_lib.bin_spectrum(np.fft.fftn(rho) / float(n) ** 3, 1.0, edges)
    bins, cnt, s, mean = oracle.sparse_low_bins(n, 1.0, edges, xyz, val, (n // 2) ** 2)
    assert len(bins) > 20
    assert np.array_equal(cnt, ref["count"][bins])
    assert np.allclose(s, ref["sum"][bins], rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("n,hw", [(16, 0), (16, 3), (32, 5), (32, 15), (64, 20)])
def test_cube_bin_sums_match_library_transform(oracle_lib, n, hw):
    """O13 against numpy.fft.fftn / n^3 of the uniform cube binned voxel by
    voxel: a single voxel (flat |F|^2), small and box-filling cubes."""
    import oracle
    edges = W.default_log_edges(n, 1.0, 40)
    rho = np.zeros((n, n, n))
    c = n // 2
    rho[c - hw:c + hw + 1, c - hw:c + hw + 1, c - hw:c + hw + 1] = 1.5
    ref = oracle_lib.bin_spectrum(np.fft.fftn(rho) / float(n) ** 3, 1.0, edges)
    cnt, s = oracle.cube_bins(n, 1.0, edges, hw, 1.5)
    assert np.array_equal(cnt, ref["count"])
    assert np.max(np.abs(s - ref["sum"])) <= 1e-12 * np.max(ref["sum"])
    # Parseval over the binned plus unbinned voxels: only n2 = 0 is unbinned
    F0 = 1.5 * (2 * hw + 1) ** 3 / float(n) ** 3
    assert abs(s.sum() + F0 ** 2 - 1.5 ** 2 * (2 * hw + 1) ** 3 / float(n) ** 3) <= 1e-12 * F0 ** 2


def test_cube_bin_sums_per_bin_at_128(oracle_lib):
    """O13 bin by bin at 128^3 against numpy.fft.fftn: the sum over the l of
    one bin is a short range of a long running sum, so its relative accuracy
    is checked per bin (to the library transform's own rounding level),
    not against the largest bin."""
    import oracle
    n, hw = 128, 50
    edges = W.default_log_edges(n, 1.0, 120)
    rho = np.zeros((n, n, n))
    c = n // 2
    rho[c - hw:c + hw + 1, c - hw:c + hw + 1, c - hw:c + hw + 1] = 1.0
    ref = oracle_lib.bin_spectrum(np.fft.fftn(rho) / float(n) ** 3, 1.0, edges)
    cnt, s = oracle.cube_bins(n, 1.0, edges, hw, 1.0)
    assert np.array_equal(cnt, ref["count"])
    pop = cnt > 0
    ibar = (2 * hw + 1) ** 3 / float(n) ** 6
    mean = s[pop] / cnt[pop]
    bound = np.maximum(1e-13, 8 * 2.0 ** -53 * math.sqrt(21.0) * np.sqrt(ibar / mean))
    assert np.all(np.abs(mean - ref["mean"][pop]) / mean <= bound)


def test_ensemble_is_the_binned_sum_of_intensities(oracle_lib):
    """O14 against the binning of the summed intensity: for incoherent
    particles the ensemble curve is the bin mean of sum_k w_k |F_k|^2, a
    different route through the oracle (one binning of the summed field
    instead of a weighted sum of per-box means)."""
    import oracle
    levels = W.b_radii(32, 4, 5.0, 13.0, nbins=30)
    w = W.volume_fractions([math.isqrt(int(wl.mask.p0)) for wl in levels], 9.0, 0.4)
    w = w / np.array([(4.0 / 3.0) * math.pi * float(wl.mask.p0) ** 1.5 for wl in levels])
    outs = [oracle.simulate(wl, return_fields=True) for wl in levels]
    mean, sem = oracle.ensemble([o["mean"] for o in outs], [o["sem"] for o in outs], w)
    I = sum(wk * np.abs(o["F"]) ** 2 for wk, o in zip(w, outs))
    ref = oracle_lib.bin_spectrum(np.sqrt(I), levels[0].voxel, levels[0].edges)
    pop = ref["count"] > 0
    assert np.array_equal(np.isnan(mean), ~pop)
    assert np.allclose(mean[pop], ref["mean"][pop], rtol=1e-12, atol=0.0)
    # one box with weight 1 is that box; the SEM of two equal boxes is sqrt(2) w SEM
    m1, s1 = oracle.ensemble([outs[0]["mean"]], [outs[0]["sem"]], [1.0])
    assert np.array_equal(m1[pop], outs[0]["mean"][pop])
    m2, s2 = oracle.ensemble([outs[1]["mean"]] * 2, [outs[1]["sem"]] * 2, [0.5, 0.5])
    multi = ref["count"] > 1
    assert np.allclose(s2[multi], math.sqrt(0.5) * outs[1]["sem"][multi], rtol=1e-15)


# ---------------------------------------------------------------------------
# O2r: ED-1 of a rotated lattice
# ---------------------------------------------------------------------------

def _rot_case():
    cell = W.draw_atoms(17, 5, 8)
    mask = W.sphere(11.0)
    return cell, mask


def test_rotated_lattice_identity_and_quarter_turn(oracle_lib):
    """R = identity samples the cell at integer points: the aligned tiling
    exactly.  A quarter turn about z, u = (-dy, dx, dz), is the tiling with
    the cell's first two axes exchanged (modular indexing)."""
    import oracle
    n = 32
    cell, mask = _rot_case()
    cg = oracle.cell_synth(cell)
    assert np.array_equal(oracle.ed1_rot(n, cg, mask, np.eye(3)), oracle.ed1(n, cg, mask))
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    got = oracle.ed1_rot(n, cg, mask, R)
    d = np.arange(n) - n // 2
    dx, dy, dz = np.meshgrid(d, d, d, indexing="ij")
    inside = dx * dx + dy * dy + dz * dz <= int(mask.p0)
    c = cg.shape[0]
    want = np.where(inside, cg[(-dy) % c, dx % c, dz % c], 0.0)
    assert np.array_equal(got, want)


def test_rotated_lattice_matches_scipy_map_coordinates(oracle_lib):
    """A general orientation against scipy.ndimage.map_coordinates (order 1,
    periodic 'grid-wrap'), a library routine for the same interpolation, at
    every inside voxel of a 24^3 box."""
    import oracle
    from scipy.ndimage import map_coordinates
    n = 24
    cell, mask = _rot_case()
    cg = oracle.cell_synth(cell)
    R = W.rotation([1.0, 2.0, 3.0], 0.7)
    got = oracle.ed1_rot(n, cg, mask, R)
    d = np.arange(n) - n // 2
    dx, dy, dz = np.meshgrid(d, d, d, indexing="ij")
    inside = dx * dx + dy * dy + dz * dz <= int(mask.p0)
    D = np.stack([dx[inside], dy[inside], dz[inside]]).astype(np.float64)
    U = R @ D
    ref = map_coordinates(cg, U, order=1, mode="grid-wrap")
    assert np.max(np.abs(got[inside] - ref)) <= 1e-12 * np.max(np.abs(cg))
    assert np.all(got[~inside] == 0.0)


def test_cubic_spline_coefficients_match_scipy_spline_filter(oracle_lib):
    """The periodic cubic B-spline coefficients of a cell against
    scipy.ndimage.spline_filter (order 3, 'grid-wrap'), and the defining
    property: filtered by (1, 4, 1)/6 along each axis they give the cell."""
    import oracle
    from scipy.ndimage import spline_filter
    cell, _ = _rot_case()
    cg = oracle.cell_synth(cell)
    C = oracle.bspline_coefficients(cg)
    assert np.max(np.abs(C - spline_filter(cg, order=3, mode="grid-wrap"))) <= 1e-12 * np.max(np.abs(cg))
    back = C
    for ax in range(3):
        back = (np.roll(back, 1, axis=ax) + 4.0 * back + np.roll(back, -1, axis=ax)) / 6.0
    assert np.max(np.abs(back - cg)) <= 1e-12 * np.max(np.abs(cg))


def test_cubic_rotated_lattice(oracle_lib):
    """Cubic B-spline sampling: through the cell values at integer points
    (identity: the aligned tiling; quarter turn: the trilinear result, both
    exact up to rounding), and a general orientation against
    scipy.ndimage.map_coordinates (order 3, 'grid-wrap') at every inside voxel
    of a 24^3 box."""
    import oracle
    from scipy.ndimage import map_coordinates
    cell, mask = _rot_case()
    cg = oracle.cell_synth(cell)
    scale = np.max(np.abs(cg))
    n = 32
    assert np.max(np.abs(oracle.ed1_rot(n, cg, mask, np.eye(3), 3) - oracle.ed1(n, cg, mask))) <= 1e-12 * scale
    Rq = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    assert np.max(np.abs(oracle.ed1_rot(n, cg, mask, Rq, 3) - oracle.ed1_rot(n, cg, mask, Rq, 1))) <= 1e-12 * scale
    n = 24
    R = W.rotation([1.0, 2.0, 3.0], 0.7)
    got = oracle.ed1_rot(n, cg, mask, R, 3)
    d = np.arange(n) - n // 2
    dx, dy, dz = np.meshgrid(d, d, d, indexing="ij")
    inside = dx * dx + dy * dy + dz * dz <= int(mask.p0)
    U = R @ np.stack([dx[inside], dy[inside], dz[inside]]).astype(np.float64)
    ref = map_coordinates(cg, U, order=3, mode="grid-wrap")
    assert np.max(np.abs(got[inside] - ref)) <= 1e-12 * scale
    assert np.all(got[~inside] == 0.0)
    assert np.max(np.abs(got - oracle.ed1_rot(n, cg, mask, R, 1))) > 1e-3 * scale   # not the trilinear sampling


@pytest.mark.parametrize("interp", [1, 3])
def test_grains_are_voronoi_pieces_of_rotated_lattices(oracle_lib, interp):
    """O2g: the grain of every inside voxel against a brute-force nearest
    seed (numpy argmin over squared distances, ties to the lower index, with
    two seeds placed so that the plane between them is tied), and each
    grain's voxels equal to the single rotated lattice of its orientation;
    all grains aligned give the aligned tiling."""
    import oracle
    n = 32
    cell, mask = _rot_case()
    cg = oracle.cell_synth(cell)
    seeds = np.array([[-4, 0, 0], [4, 0, 0], [0, 7, -3], [2, -6, 5]], dtype=np.float64)
    rots = np.stack([W.rotation([1.0, 2.0, 3.0], 0.7), W.rotation([0.0, 1.0, 0.0], 1.3),
                     W.rotation([1.0, -1.0, 0.5], 2.1), W.rotation([0.3, 0.2, -1.0], 0.4)])
    got = oracle.ed1_grains(n, cg, mask, seeds, rots, interp)
    d = np.arange(n) - n // 2
    dx, dy, dz = np.meshgrid(d, d, d, indexing="ij")
    inside = dx * dx + dy * dy + dz * dz <= int(mask.p0)
    D2 = np.stack([(dx - s[0]) ** 2 + (dy - s[1]) ** 2 + (dz - s[2]) ** 2 for s in seeds.astype(np.int64)])
    owner = np.argmin(D2, axis=0)
    tied = (D2[0] == D2[1]) & (D2[0] <= D2.min(axis=0)) & inside
    assert tied.sum() > 50 and np.all(owner[tied] == 0)
    assert np.all(got[~inside] == 0.0)
    for g in range(len(seeds)):
        sel = inside & (owner == g)
        assert sel.sum() > 100
        single = oracle.ed1_rot(n, cg, mask, rots[g], interp)
        assert np.array_equal(got[sel], single[sel]), g
    eye = np.stack([np.eye(3)] * len(seeds))
    aligned = oracle.ed1_grains(n, cg, mask, seeds, eye, interp)
    assert np.max(np.abs(aligned - oracle.ed1(n, cg, mask))) <= 1e-12 * np.max(np.abs(cg))


# ---------------------------------------------------------------------------
# O17: peak integrals (degree of crystallinity)
# ---------------------------------------------------------------------------

def test_peak_integrals_closed_forms(oracle_lib):
    """A Gaussian peak of area A on a sloping straight background, sampled at
    the centres of fine bins: the peak integral is A (the midpoint rule of a
    Gaussian over +-6 widths, and the baseline through the window's ends is
    the background to exp(-18)); the background alone integrates to zero
    above its own baseline, and its total is the trapezoid of a line; a
    window of fewer than two populated bins gives NaN; an empty bin inside a
    window is skipped."""
    import oracle
    e = W.lin_edges(0.0, 10.0, 2000)
    q = 0.5 * (e[:-1] + e[1:])
    A, q0, s = 3.0, 4.0, 0.07
    bg = 2.0 - 0.1 * q
    m = bg + A / (s * math.sqrt(2.0 * math.pi)) * np.exp(-0.5 * ((q - q0) / s) ** 2)
    lo, hi = q0 - 6 * s, q0 + 6 * s
    r = oracle.peak_integrals(e, m, [(lo, hi), (1.0, 2.0), (5.0001, 5.0049)])
    assert abs(r[0, 0] - A) <= 1e-6 * A
    line = oracle.peak_integrals(e, bg, [(lo, hi), (1.0, 2.0)])
    assert np.all(np.abs(line[:, 0]) <= 1e-12 * line[:, 1])
    sel = (q >= 1.0) & (q <= 2.0)
    qa, qb = q[sel][0] - 0.0025, q[sel][-1] + 0.0025
    trap = (2.0 - 0.05 * (qa + qb)) * (qb - qa)
    assert abs(line[1, 1] - trap) <= 1e-12 * trap and line[1, 2] == sel.sum()
    assert np.isnan(r[2, 0]) and np.isnan(r[2, 1]) and r[2, 2] < 2
    m2 = m.copy()
    m2[np.argmin(np.abs(q - 1.5))] = np.nan
    r2 = oracle.peak_integrals(e, m2, [(1.0, 2.0)])
    assert r2[0, 2] == r[1, 2] - 1 and np.isfinite(r2[0, 0])


# ---------------------------------------------------------------------------
# O15: voxel form factor (a density uniform over each voxel)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("f", [2, 4])
def test_block_transfer_is_the_ratio_of_level_to_fine_amplitudes(oracle_lib, f):
    """O18 pinned by transforms: for a fine density whose spectrum lies
    inside the level's band (|u| < n_k/2 on every axis, so no alias reaches
    the level's grid), the level made of block sums has amplitude
    T(m) A1(m) at every shared frequency and zero at the level's Nyquist
    index. A1 and the level's amplitude are numpy transforms of the box and
    of its block sums; T is the oracle's sum."""
    n1 = 32
    nk = n1 // f
    rng = np.random.default_rng(18 + f)
    A = np.zeros((n1, n1, n1), dtype=complex)
    band = [u % n1 for u in range(-(nk // 2) + 1, nk // 2)]
    for u in band:
        for v in band:
            for w in band:
                A[u, v, w] = rng.normal() + 1j * rng.normal()
    rho1 = np.real(np.fft.ifftn(A))
    a1 = np.fft.fftn(rho1)
    level = rho1.reshape(nk, f, nk, f, nk, f).sum(axis=(1, 3, 5))
    ak = np.fft.fftn(level)
    T = oracle_lib.block_transfer(nk, f)
    scale = np.abs(a1).max()
    idx = [m % nk for m in range(-(nk // 2) + 1, nk // 2)]
    for u in idx:
        for v in idx:
            for w in idx:
                uf, vf, wf = [(m if m < nk // 2 else m - nk) % n1 for m in (u, v, w)]
                assert abs(ak[u, v, w] - T[u, v, w] * a1[uf, vf, wf]) <= 1e-12 * scale
    assert np.abs(ak[nk // 2, :, :]).max() <= 1e-12 * scale
    # the level keeps the electrons: T(0) = 1
    assert abs(T[0, 0, 0] - 1.0) < 1e-15 and abs(ak[0, 0, 0] - a1[0, 0, 0]) <= 1e-12 * scale


@pytest.mark.parametrize("n, f", [(16, 2), (16, 4), (64, 16), (250, 5)])
def test_block_transfer_power_is_the_dirichlet_kernel(oracle_lib, n, f):
    """|T(m)|^2 per axis against the closed form of a sum of f unit phasors,
    sin^2(pi m / n) / (f sin(pi m / (f n)))^2, and 0.81 at half the Nyquist
    index for large f."""
    T = oracle_lib.block_transfer(n, f)
    for m in range(1, n // 2 + 1):
        ref = (math.sin(math.pi * m / n) / (f * math.sin(math.pi * m / (f * n)))) ** 2
        assert abs(abs(T[m, 0, 0]) ** 2 - ref) <= 1e-13
    big = oracle_lib.block_transfer(64, 125)
    assert abs(abs(big[16, 0, 0]) ** 2 - 8.0 / math.pi ** 2) < 1e-4      # (sin(pi/4) / (pi/4))^2


@pytest.mark.parametrize("n,hw", [(32, 5), (32, 10), (16, 7)])
def test_voxel_form_of_a_cube_is_the_continuous_cube(oracle_lib, n, hw):
    """A cube of W = 2 hw + 1 voxels, each voxel uniform, is the continuous
    cube of edge W: per axis sin(pi h W/n)/sin(pi h/n) * sinc(pi h/n) =
    sin(pi h W/n)/(pi h/n).  O13 with the factor against that closed form
    binned voxel by voxel, and O15 applied to the transform of the voxel
    cube (oracle.simulate) against both."""
    import oracle
    W_ = 2 * hw + 1
    edges = W.default_log_edges(n, 1.0, 30)
    u = np.arange(n)
    h = np.where(u < n // 2, u, u - n).astype(np.float64)
    g = np.full(n, float(W_))
    nz = h != 0
    g[nz] = np.sin(np.pi * h[nz] * W_ / n) / (np.pi * h[nz] / n)
    Fc = g[:, None, None] * g[None, :, None] * g[None, None, :] / float(n) ** 3
    ref = oracle_lib.bin_spectrum(Fc.astype(np.complex128), 1.0, edges)
    cnt, s = oracle.cube_bins(n, 1.0, edges, hw, 1.0, voxel_form_factor=True)
    assert np.array_equal(cnt, ref["count"])
    assert np.max(np.abs(s - ref["sum"])) <= 1e-12 * np.max(ref["sum"])
    wl = W.uniform_cube(n, hw, 30, prec=1)
    sim = oracle.simulate(wl, voxel_form_factor=True)
    pop = cnt > 0
    assert np.allclose(sim["mean"][pop], ref["mean"][pop], rtol=1e-11, atol=1e-14 * np.nanmax(ref["mean"]))
    f = oracle.voxel_form(n)
    assert f[0, 0, 0] == 1.0 and abs(f[n // 2, 0, 0] - 2.0 / np.pi) <= 1e-15


# ---------------------------------------------------------------------------
# O16: Ewald-sphere detector image
# ---------------------------------------------------------------------------

def _affine_spectra(n, c0=None):
    """Three spectra with |F|^2 = c0 + g_axis on the signed frequencies
    (|g| < n/2): trilinear interpolation reproduces an affine field exactly
    away from the wrap, so an image of each returns the grid coordinate of
    every pixel along one axis."""
    c0 = float(n) if c0 is None else c0
    u = np.arange(n)
    h = np.where(u < n // 2, u, u - n).astype(np.float64)
    out = []
    for ax in range(3):
        shape = [1, 1, 1]
        shape[ax] = n
        I = c0 + np.broadcast_to(h.reshape(shape), (n, n, n))
        out.append(np.sqrt(I).astype(np.complex128))
    return c0, out


def _grid_coords(n, voxel, geo):
    import oracle
    c0, Fs = _affine_spectra(n)
    return np.stack([oracle.ewald_image(F, voxel, geo) - c0 for F in Fs], axis=-1)


GEOS = [
    ("identity", W.detector(np.eye(3), pixel=5.0, nu=41, nv=33, cu=20, cv=16)),
    ("tilted", W.detector(W.rotation([0.3, -0.5, 0.8], 1.1), pixel=5.0, nu=37, nv=29, cu=11.0, cv=20.0)),
]


@pytest.mark.parametrize("name,geo", GEOS)
def test_ewald_coordinates_lie_on_the_sphere(oracle_lib, name, geo):
    """The grid coordinates the image samples (read back through affine
    spectra) against the geometry of elastic scattering: q + k e has length
    k (the Ewald sphere), |q| = (4 pi / lambda) sin(theta) with
    tan(2 theta) = r / distance (Bragg), the component of q across the beam
    points along the pixel's offset on the detector, and the beam centre
    pixel samples q = 0."""
    n, voxel = 128, 0.25
    g = _grid_coords(n, voxel, geo)
    assert np.max(np.abs(g)) < n // 2 - 1
    dq = 2.0 * math.pi / (n * voxel)
    q = g * dq
    k = 2.0 * math.pi / geo.wavelength
    e, du, dv = (np.asarray(v) for v in (geo.beam, geo.du, geo.dv))
    assert np.max(np.abs(np.linalg.norm(q + k * e, axis=-1) - k)) <= 1e-9 * k
    iv, iu = np.meshgrid(np.arange(geo.nv), np.arange(geo.nu), indexing="ij")
    a, b = (iu - geo.cu) * geo.pixel, (iv - geo.cv) * geo.pixel
    r = np.hypot(a, b)
    theta = 0.5 * np.arctan2(r, geo.distance)
    qn = np.linalg.norm(q, axis=-1)
    assert np.max(np.abs(qn - 4.0 * math.pi * np.sin(theta) / geo.wavelength)) <= 1e-9 * qn.max()
    qa, qb = q @ du, q @ dv
    assert np.max(np.abs(qa * b - qb * a)) <= 1e-9 * qn.max() * r.max()
    assert np.all(qa * a + qb * b >= -1e-12)
    assert np.max(np.abs(q[int(geo.cv), int(geo.cu)])) <= 1e-12
    assert qn.max() > 5 * dq


@pytest.mark.parametrize("name,geo", GEOS)
def test_ewald_interpolation_is_scipy_map_coordinates(oracle_lib, name, geo):
    """The image of a random spectrum against scipy's order-1 spline (the
    trilinear interpolant) of |F|^2 with periodic wrap, sampled at the
    coordinates read back on a finer grid of the same frequency step: on the
    32-point grid they run past the Nyquist frequency, so the wrap is
    exercised in both directions."""
    import oracle
    from scipy.ndimage import map_coordinates
    g = _grid_coords(128, 0.25, geo)
    n = 32
    assert np.max(np.abs(g)) > n / 2 + 1
    rng = np.random.default_rng(16)
    F = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    img = oracle.ewald_image(F, 1.0, geo)
    ref = map_coordinates(np.abs(F) ** 2, g.reshape(-1, 3).T, order=1, mode="grid-wrap").reshape(img.shape)
    assert np.max(np.abs(img - ref)) <= 1e-12 * np.max(np.abs(F) ** 2)


def test_ewald_wavelength_spread_is_the_gaussian_average(oracle_lib):
    """With an affine |F|^2 the image is c0 + (g at lambda) E[lambda / lambda_j];
    the 64-node rule against the truncated Gaussian integral of that
    expectation (quadrature), which differs from 1 by about rel_spread^2.
    No spread, or one node, reproduce the single wavelength, and the beam
    centre gives |F(0)|^2 for any spread."""
    import oracle
    from scipy import integrate
    geo0 = GEOS[1][1]
    n, voxel, s = 128, 0.25, 0.05
    c0, Fs = _affine_spectra(n)
    geo = dataclasses.replace(geo0, rel_spread=s, n_lambda=64)
    phi = lambda t: math.exp(-0.5 * t * t)
    ek = (integrate.quad(lambda t: phi(t) / (1.0 + s * t), -3.0, 3.0, epsabs=0, epsrel=1e-12)[0]
          / integrate.quad(phi, -3.0, 3.0, epsabs=0, epsrel=1e-12)[0])
    assert ek - 1.0 > 2e-3
    for F in Fs:
        one = oracle.ewald_image(F, voxel, geo0) - c0
        spread = oracle.ewald_image(F, voxel, geo) - c0
        assert np.max(np.abs(spread - ek * one)) <= 3e-5 * np.max(np.abs(one))
        for g2 in (dataclasses.replace(geo0, n_lambda=16), dataclasses.replace(geo, n_lambda=1)):
            assert np.max(np.abs(oracle.ewald_image(F, voxel, g2) - c0 - one)) <= 1e-12 * np.max(np.abs(one))
    rng = np.random.default_rng(3)
    F = rng.standard_normal((16, 16, 16)) + 1j * rng.standard_normal((16, 16, 16))
    geo = W.detector(np.eye(3), rel_spread=0.1, n_lambda=9, nu=9, nv=7, cu=4, cv=3)
    img = oracle.ewald_image(F, 1.0, geo)
    assert abs(img[3, 4] - abs(F[0, 0, 0]) ** 2) <= 1e-14 * abs(F[0, 0, 0]) ** 2


def test_ewald_sparse_route_matches_full_spectrum(oracle_lib):
    """O16 at chosen pixels with every needed coefficient summed directly over
    the nonzero voxels (the route for boxes too large to transform) against
    the image of the full transform, on a 32^3 box of 20 voxels."""
    import oracle
    n = 32
    xyz, val = W.sparse_voxels(5, n, 20, dtype=np.float64)
    rho = np.zeros((n, n, n))
    rho[xyz[:, 0], xyz[:, 1], xyz[:, 2]] = val
    geo = W.detector(W.rotation([0.3, -0.5, 0.8], 1.1), rel_spread=0.05, n_lambda=5, pixel=5.0,
                     nu=21, nv=17, cu=7.0, cv=9.0)
    full = oracle.ewald_image(oracle.forward(rho), 1.0, geo)
    iv, iu = np.array([0, 5, 16, 8, 9]), np.array([0, 20, 3, 11, 7])
    sp = oracle.ewald_pixels_sparse(n, 1.0, geo, iv, iu, xyz, val)
    assert np.max(np.abs(sp - full[iv, iu])) <= 1e-13 * np.max(full)


@pytest.mark.parametrize("interp", [1, 3])
def test_oriented_points_match_the_whole_box(oracle_lib, interp):
    """O2r / O2g evaluated at chosen voxels (the route for boxes too large to
    generate) against the same voxels of the whole-box evaluation, for one
    orientation and for grains."""
    import oracle
    n = 32
    cell, mask = _rot_case()
    cg = oracle.cell_synth(cell)
    rng = np.random.default_rng(9)
    xyz = rng.integers(0, n, (300, 3))
    R = W.rotation([1.0, 2.0, 3.0], 0.7)
    whole = oracle.ed1_rot(n, cg, mask, R, interp)
    pts = oracle.oriented_points(n, cg, mask, xyz, np.zeros((1, 3)), R[None], interp)
    assert np.array_equal(pts, whole[xyz[:, 0], xyz[:, 1], xyz[:, 2]])
    seeds, rots = W.random_grains(4, 5, 12.0)
    whole = oracle.ed1_grains(n, cg, mask, seeds, rots, interp)
    pts = oracle.oriented_points(n, cg, mask, xyz, seeds, rots, interp)
    assert np.array_equal(pts, whole[xyz[:, 0], xyz[:, 1], xyz[:, 2]])


def test_constant_solvent_is_a_background_shift(oracle_lib):
    """A particle in a solvent of constant density rho_s (the outlook's
    surrounding matrix, without fluctuations) against the particle with its
    cell background lowered by rho_s: the two boxes differ by a uniform box,
    whose eq. 1 transform is zero away from q = 0, so every bin that holds
    no q = 0 voxel agrees (the first bin's lower edge is above zero here)."""
    import dataclasses
    import oracle
    wl = W.small(32, c=8, n_atoms=6, seed=11, radius=10.0, nbins=40, prec=1)
    rho_s = 0.7
    cg = oracle.cell_synth(wl.cell)
    inside = oracle.density(wl, cg) != 0.0
    solvent = np.where(inside, oracle.density(wl, cg), rho_s)
    shifted = dataclasses.replace(wl, cell=dataclasses.replace(wl.cell, background=wl.cell.background - rho_s))
    a = oracle.bin_spectrum(oracle.forward(solvent), wl.voxel, wl.edges)
    b = oracle.simulate(shifted)
    assert wl.edges[0] > 0.0
    pop = a["count"] > 0
    assert np.array_equal(a["count"], b["count"])
    assert np.max(np.abs(a["mean"][pop] - b["mean"][pop])) <= 1e-12 * np.max(a["mean"][pop])
