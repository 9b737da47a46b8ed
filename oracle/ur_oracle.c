/*
 * FP64 CPU oracle for the wide-range scattering simulation
 * (Pauw et al., "Ultima Ratio", arXiv 2303.13435).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU path computes.  It is called by the tests, by the
 * smoke check and by the CPU-baseline leg of the benchmark, never by the
 * product path, and it shares no code with the HIP library.
 *
 * Every function names the passage of the paper it follows.  Where the paper
 * is silent the reading taken is stated in the comment (the same readings are
 * listed in the design notes of the repository).
 *
 * Conventions
 *   box index layout  [x][y][z], z fastest, edge n
 *   particle centre   voxel (n1/2, n1/2, n1/2) of the ED-1 grid; the unit-cell
 *                     lattice is anchored there too
 *   signed frequency  h(u) = u for u < n/2, else u - n   (u = n/2 -> -n/2)
 *   forward transform F = (1/n^3) * sum rho exp(-2 pi i (ux+vy+wz)/n)   (eq. 1)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cdouble;

/* ------------------------------------------------------------------------ */
/* compensated (Neumaier) accumulator                                        */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } kahan_t;

static void kadd(kahan_t* k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else                       k->c += (v - t) + k->s;
    k->s = t;
}
static double kval(const kahan_t* k) { return k->s + k->c; }

/* ------------------------------------------------------------------------ */
/* O1  unit-cell density ("ED-Unit"; Methodology, general workflow step 1 and
 *     "Electron density generation").  The paper's ED-Unit comes from DFT;
 *     here it is a sum of voxel-integrated Gaussian atoms with periodic
 *     images, so each atom contributes exactly its electron count.           */
/* ------------------------------------------------------------------------ */

/* cumulative normal */
static double phi_cdf(double t) { return 0.5 * erfc(-t / sqrt(2.0)); }

/* p[i] = integral over voxel i (i-1/2 .. i+1/2) of a unit Gaussian centred at
 * x with width sigma, summed over periodic images x + m*c, |m| <= M. */
void or_atom_profile(int c, double x, double sigma, double* p)
{
    int M = (int)ceil(8.0 * sigma / c) + 1;
    for (int i = 0; i < c; ++i) {
        double acc = 0.0;
        for (int m = -M; m <= M; ++m) {
            double hi = (i + 0.5 - x + (double)m * c) / sigma;
            double lo = (i - 0.5 - x + (double)m * c) / sigma;
            acc += phi_cdf(hi) - phi_cdf(lo);
        }
        p[i] = acc;
    }
}

/* cell[i][j][k] = background + sum_a amp_a * px_a[i] * py_a[j] * pz_a[k] */
void or_cell_synth(int c, int n_atoms, const double* xyz, const double* amp,
                   const double* sigma, double background, double* cell)
{
    size_t c3 = (size_t)c * c * c;
    for (size_t v = 0; v < c3; ++v) cell[v] = background;
    double* px = (double*)malloc(sizeof(double) * 3 * (size_t)c);
    for (int a = 0; a < n_atoms; ++a) {
        or_atom_profile(c, xyz[3 * a + 0], sigma[a], px);
        or_atom_profile(c, xyz[3 * a + 1], sigma[a], px + c);
        or_atom_profile(c, xyz[3 * a + 2], sigma[a], px + 2 * c);
        for (int i = 0; i < c; ++i)
            for (int j = 0; j < c; ++j)
                for (int k = 0; k < c; ++k)
                    cell[((size_t)i * c + j) * c + k] += amp[a] * px[i] * px[c + j] * px[2 * c + k];
    }
    free(px);
}

/* ------------------------------------------------------------------------ */
/* O2  ED-1: the unit cell tiled over the box and multiplied by the particle
 *     mask (Methodology, "Electron density generation": tiling with periodic
 *     wrap, then a per-plane circular mask building up a sphere).  The
 *     paper's interpolation over a rotated grid is taken without rotation, so
 *     every interpolation order reproduces the grid values exactly and the
 *     tiling is plain modular indexing.                                      */
/* ------------------------------------------------------------------------ */

/* kinds: 0 none, 1 sphere (d.d <= p0), 2 cube (max|d| <= p0),
 *        3 truncated octahedron (max|d| <= p0 and sum|d| <= p1) */
int or_mask_inside(int kind, long long p0, long long p1, long long dx, long long dy, long long dz)
{
    long long ax = llabs(dx), ay = llabs(dy), az = llabs(dz);
    long long mx = ax > ay ? ax : ay;
    if (az > mx) mx = az;
    switch (kind) {
    case 0: return 1;
    case 1: return dx * dx + dy * dy + dz * dz <= p0;
    case 2: return mx <= p0;
    case 3: return mx <= p0 && ax + ay + az <= p1;
    default: return 0;
    }
}

static long long pmod(long long a, long long m) { long long r = a % m; return r < 0 ? r + m : r; }

/* value of ED-1 at voxel (x, y, z) of the n1 grid */
static double ed1_value(int n1, int c, const double* cell, int kind, long long p0, long long p1,
                        long long x, long long y, long long z)
{
    long long h = n1 / 2;
    if (!or_mask_inside(kind, p0, p1, x - h, y - h, z - h)) return 0.0;
    long long i = pmod(x - h, c), j = pmod(y - h, c), k = pmod(z - h, c);
    return cell[((size_t)i * c + j) * c + k];
}

/* half-width of the axis-aligned cube that contains every inside voxel */
static long long mask_halfwidth(int kind, long long p0, long long p1, int n1)
{
    (void)p1;
    switch (kind) {
    case 1: { if (p0 < 0) return -1; long long r = (long long)floor(sqrt((double)p0)); while ((r + 1) * (r + 1) <= p0) ++r; while (r * r > p0) --r; return r; }
    case 2: case 3: return p0;
    default: return n1;
    }
}

void or_ed1(int n, int c, const double* cell, int kind, long long p0, long long p1, double* rho)
{
#pragma omp parallel for schedule(static)
    for (long long x = 0; x < n; ++x)
        for (long long y = 0; y < n; ++y)
            for (long long z = 0; z < n; ++z)
                rho[((size_t)x * n + y) * n + z] = ed1_value(n, c, cell, kind, p0, p1, x, y, z);
}

/* ------------------------------------------------------------------------ */
/* O2r ED-1 of a rotated lattice ("Electron density generation": the cell is
 *     interpolated over a rotated grid and repeated beyond its bounds).  The
 *     voxel at offset d = (x, y, z) - n/2 from the particle centre takes the
 *     cell's value at u = R d, linearly interpolated between the cell voxels
 *     along each axis with periodic wrap (cell voxel i at coordinate i), the
 *     third axis first; zero outside the mask.  u_i = (R_i0 dx + R_i1 dy)
 *     + R_i2 dz, each operation rounded on its own.                          */
/* ------------------------------------------------------------------------ */
static double lerp(double a, double b, double t) { return a + t * (b - a); }

/* cubic B-spline B3(x): (2 - |x|)^3 / 6 for 1 <= |x| < 2, (4 - 6 x^2 + 3 |x|^3) / 6
 * for |x| < 1, zero beyond */
static double bspline3(double x)
{
    const double a = fabs(x);
    if (a >= 2.0) return 0.0;
    if (a >= 1.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
    return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
}

/* Polycrystalline ED-1: the inside voxel at offset d belongs to the grain g
 * whose integer seed s_g is nearest (squared distance, ties to the lower
 * index) and takes the cell at u = R_g d (R_g row-major, 9 per grain).
 * order 1: `cell` holds the cell values, trilinear; order 3: `cell` holds the
 * periodic cubic B-spline coefficients C, value = sum over the 4^3 nearest
 * coefficients of C[i] B3(u0 - i0) B3(u1 - i1) B3(u2 - i2).  One grain with
 * any seed is a single rotated lattice. */
/* one voxel of the polycrystalline ED-1 (see or_ed1_grains) */
static double grains_voxel(int n, int c, const double* cell, int kind, long long p0, long long p1, int ngrain,
                           const long long* seed, const double* Rg, int order, long long x, long long y, long long z)
{
    const long long h = n / 2;
    const long long dx = x - h, dy = y - h, dz = z - h;
    if (!or_mask_inside(kind, p0, p1, dx, dy, dz)) return 0.0;
    int g = 0;
    long long best = -1;
    for (int k = 0; k < ngrain; ++k) {
        const long long ex = dx - seed[3 * k], ey = dy - seed[3 * k + 1], ez = dz - seed[3 * k + 2];
        const long long d2 = ex * ex + ey * ey + ez * ez;
        if (best < 0 || d2 < best) { best = d2; g = k; }
    }
    const double* R = Rg + 9 * g;
    double u[3];
    for (int i = 0; i < 3; ++i)
        u[i] = (R[3 * i] * (double)dx + R[3 * i + 1] * (double)dy) + R[3 * i + 2] * (double)dz;
    long long i0[3];
    double t[3];
    for (int i = 0; i < 3; ++i) {
        const double f = floor(u[i]);
        i0[i] = (long long)f;
        t[i] = u[i] - f;
    }
    if (order == 3) {
        double s = 0.0;
        for (int a0 = -1; a0 <= 2; ++a0)
            for (int a1 = -1; a1 <= 2; ++a1)
                for (int a2 = -1; a2 <= 2; ++a2) {
                    const double w = bspline3(t[0] - a0) * bspline3(t[1] - a1) * bspline3(t[2] - a2);
                    s += w * cell[((size_t)pmod(i0[0] + a0, c) * c + pmod(i0[1] + a1, c)) * c + pmod(i0[2] + a2, c)];
                }
        return s;
    }
    double a[2][2];
    for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj) {
            const long long ci = pmod(i0[0] + di, c), cj = pmod(i0[1] + dj, c);
            const double* row = cell + ((size_t)ci * c + cj) * c;
            a[di][dj] = lerp(row[pmod(i0[2], c)], row[pmod(i0[2] + 1, c)], t[2]);
        }
    return lerp(lerp(a[0][0], a[0][1], t[1]), lerp(a[1][0], a[1][1], t[1]), t[0]);
}

void or_ed1_grains(int n, int c, const double* cell, int kind, long long p0, long long p1, int ngrain,
                   const long long* seed, const double* Rg, int order, double* rho)
{
#pragma omp parallel for schedule(static)
    for (long long x = 0; x < n; ++x)
        for (long long y = 0; y < n; ++y)
            for (long long z = 0; z < n; ++z)
                rho[((size_t)x * n + y) * n + z] = grains_voxel(n, c, cell, kind, p0, p1, ngrain, seed, Rg, order, x, y, z);
}

/* the same at npts voxels xyz[3p .. 3p+2] of the box (for boxes too large to
 * generate whole) */
void or_ed1_grains_points(int n, int c, const double* cell, int kind, long long p0, long long p1, int ngrain,
                          const long long* seed, const double* Rg, int order, long long npts, const long long* xyz,
                          double* out)
{
#pragma omp parallel for schedule(static)
    for (long long p = 0; p < npts; ++p)
        out[p] = grains_voxel(n, c, cell, kind, p0, p1, ngrain, seed, Rg, order, xyz[3 * p], xyz[3 * p + 1], xyz[3 * p + 2]);
}

void or_ed1_rot(int n, int c, const double* cell, int kind, long long p0, long long p1, const double* R,
                int order, double* rho)
{
    const long long origin[3] = {0, 0, 0};
    or_ed1_grains(n, c, cell, kind, p0, p1, 1, origin, R, order, rho);
}

/* ------------------------------------------------------------------------ */
/* O3  zoomed-out levels ED-2/ED-3 (Methodology, workflow step 3 and
 *     "Electron density generation": block integration of ED-1 by a linear
 *     factor, with the result zero-padded into a smaller box).  Block
 *     integration is read as a sum (electron conserving); the reduced
 *     particle is centred: offset o = (nk - n1/f)/2.                         */
/* ------------------------------------------------------------------------ */
static double edk_value(int n1, int c, const double* cell, int kind, long long p0, long long p1,
                        int f, int nk, long long X, long long Y, long long Z)
{
    long long m = n1 / f, o = (nk - m) / 2;
    if (X < o || X >= o + m || Y < o || Y >= o + m || Z < o || Z >= o + m) return 0.0;
    double s = 0.0;
    for (int a = 0; a < f; ++a)
        for (int b = 0; b < f; ++b)
            for (int d = 0; d < f; ++d)
                s += ed1_value(n1, c, cell, kind, p0, p1, f * (X - o) + a, f * (Y - o) + b, f * (Z - o) + d);
    return s;
}

void or_zoom(int n1, int c, const double* cell, int kind, long long p0, long long p1,
             int f, int nk, double* rho)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long long X = 0; X < nk; ++X)
        for (long long Y = 0; Y < nk; ++Y)
            for (long long Z = 0; Z < nk; ++Z)
                rho[((size_t)X * nk + Y) * nk + Z] = edk_value(n1, c, cell, kind, p0, p1, f, nk, X, Y, Z);
}

/* ------------------------------------------------------------------------ */
/* O4  3D discrete Fourier transform (eq. 1), evaluated axis by axis as the
 *     separation of eq. 2 allows: 1D transforms along z, then y, then x.
 *     Each 1D transform is the textbook recursive radix-2 decimation in time
 *     with every twiddle evaluated directly as exp(sign 2 pi i k / len).
 *     Unnormalised here; the caller applies 1/n^3 for eq. 1.                 */
/* ------------------------------------------------------------------------ */
static void fft_rec(const cdouble* in, int len, int stride, cdouble* out, int sign)
{
    if (len == 1) { out[0] = in[0]; return; }
    if (len % 2) {
        /* odd length (the 3^b 5^c part of a mixed-radix edge): the DFT sum
         * itself, X_k = sum_j x_j w^(j k), with w^m = exp(sign 2 pi i m / len) */
        cdouble* w = (cdouble*)malloc(sizeof(cdouble) * len);
        for (int m = 0; m < len; ++m) w[m] = cexp(sign * 2.0 * M_PI * I * (double)m / (double)len);
        for (int k = 0; k < len; ++k) {
            cdouble acc = 0.0;
            for (int j = 0; j < len; ++j) acc += in[(size_t)j * stride] * w[(long long)j * k % len];
            out[k] = acc;
        }
        free(w);
        return;
    }
    int h = len / 2;
    fft_rec(in, h, 2 * stride, out, sign);               /* even samples -> out[0, h)   */
    fft_rec(in + stride, h, 2 * stride, out + h, sign);  /* odd samples  -> out[h, len) */
    for (int k = 0; k < h; ++k) {
        cdouble w = cexp(sign * 2.0 * M_PI * I * (double)k / (double)len);
        cdouble e = out[k], o = out[k + h] * w;
        out[k] = e + o;
        out[k + h] = e - o;
    }
}

/* in-place 1D transforms of all lines of a [n][n][n] array along `axis` */
static void fft_axis(cdouble* a, int n, int axis, int sign)
{
    size_t st = axis == 2 ? 1 : (axis == 1 ? (size_t)n : (size_t)n * n);
#pragma omp parallel
    {
        cdouble* line = (cdouble*)malloc(sizeof(cdouble) * n);
        cdouble* res = (cdouble*)malloc(sizeof(cdouble) * n);
#pragma omp for schedule(static)
        for (long long l = 0; l < (long long)n * n; ++l) {
            long long p = l / n, q = l % n;
            size_t base;
            if (axis == 2)      base = ((size_t)p * n + q) * n;
            else if (axis == 1) base = (size_t)p * n * n + (size_t)q;
            else                base = (size_t)p * n + (size_t)q;
            for (int i = 0; i < n; ++i) line[i] = a[base + i * st];
            fft_rec(line, n, 1, res, sign);
            for (int i = 0; i < n; ++i) a[base + i * st] = res[i];
        }
        free(line);
        free(res);
    }
}

/* unnormalised 3D transform in place; sign -1 forward, +1 inverse */
void or_fft3d(int n, cdouble* a, int sign)
{
    fft_axis(a, n, 2, sign);
    fft_axis(a, n, 1, sign);
    fft_axis(a, n, 0, sign);
}

/* 1D transform of `count` contiguous lines of length n (used by pins) */
void or_fft1d_batch(int n, long long count, cdouble* a, int sign)
{
#pragma omp parallel
    {
        cdouble* res = (cdouble*)malloc(sizeof(cdouble) * n);
#pragma omp for schedule(static)
        for (long long l = 0; l < count; ++l) {
            fft_rec(a + (size_t)l * n, n, 1, res, sign);
            memcpy(a + (size_t)l * n, res, sizeof(cdouble) * n);
        }
        free(res);
    }
}

/* ------------------------------------------------------------------------ */
/* O5/O6  |Q| of a voxel and its bin (Methodology, "Q-calculation and
 *     spherical averaging": a Q map from box length, voxels per side and the
 *     distance from the centre).  Q = dq * sqrt(n2), dq = 2 pi/(n voxel),
 *     n2 = h^2 + k^2 + l^2 in integers.  A bin edge e is turned into the
 *     integer threshold t = (e/dq)^2, snapped to the nearest integer when
 *     within 1e-9 relative; bin b holds ceil(t_b) <= n2 < ceil(t_b+1), and
 *     the last bin also holds n2 == floor(t_B) (upper edge inclusive).        */
/* ------------------------------------------------------------------------ */
static double snap_threshold(double e, double dq)
{
    double r = e / dq;
    double t = r * r;
    double rt = nearbyint(t);
    if (fabs(t - rt) <= 1e-9 * fmax(1.0, t)) t = rt;
    return t;
}

/* U[0..nbins]: bin b holds U[b] <= n2 < U[b+1] */
void or_thresholds(int n, double voxel, int nbins, const double* edges, long long* U)
{
    double dq = 2.0 * M_PI / ((double)n * voxel);
    for (int b = 0; b < nbins; ++b) {
        double t = snap_threshold(edges[b], dq);
        U[b] = t <= 0.0 ? 0 : (long long)ceil(t);
    }
    double tl = snap_threshold(edges[nbins], dq);
    U[nbins] = tl < 0.0 ? 0 : (long long)floor(tl) + 1;
}

static int find_bin(long long n2, int nbins, const long long* U)
{
    if (n2 < U[0] || n2 >= U[nbins]) return -1;
    int lo = 0, hi = nbins;          /* U[lo] <= n2 < U[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (U[mid] <= n2) lo = mid; else hi = mid;
    }
    return lo;
}

static long long sgn_index(long long u, long long n) { return u < n / 2 ? u : u - n; }

/* ------------------------------------------------------------------------ */
/* O7/O8  per-bin statistics: count, mean and standard error of the mean of
 *     the intensity I = |F|^2 over every voxel whose |Q| falls in the bin
 *     (Methodology, dataMerge binning).  Pooling the per-slice sums and
 *     counts, as the per-slice-then-combine procedure does, gives exactly the
 *     same numbers, so the oracle bins the whole box at once.  Outputs:
 *     count, sum, sumsq (compensated sums), mean, sem (two-pass), and
 *     totals = { sum of I over every voxel, Re F(0), Im F(0) }.              */
/* ------------------------------------------------------------------------ */
void or_bin(int n, const cdouble* F, double voxel, int nbins, const double* edges,
            double* count, double* sum, double* sumsq, double* mean, double* sem, double* totals)
{
    long long* U = (long long*)malloc(sizeof(long long) * (nbins + 1));
    or_thresholds(n, voxel, nbins, edges, U);
    kahan_t* ks = (kahan_t*)calloc((size_t)nbins, sizeof(kahan_t));
    kahan_t* kq = (kahan_t*)calloc((size_t)nbins, sizeof(kahan_t));
    kahan_t* kv = (kahan_t*)calloc((size_t)nbins, sizeof(kahan_t));
    long long* cnt = (long long*)calloc((size_t)nbins, sizeof(long long));
    kahan_t tot = {0, 0};
    for (long long u = 0; u < n; ++u) {
        long long h = sgn_index(u, n);
        for (long long v = 0; v < n; ++v) {
            long long k = sgn_index(v, n);
            for (long long w = 0; w < n; ++w) {
                long long l = sgn_index(w, n);
                cdouble f = F[((size_t)u * n + v) * n + w];
                double inten = creal(f) * creal(f) + cimag(f) * cimag(f);
                kadd(&tot, inten);
                int b = find_bin(h * h + k * k + l * l, nbins, U);
                if (b < 0) continue;
                cnt[b] += 1;
                kadd(&ks[b], inten);
                kadd(&kq[b], inten * inten);
            }
        }
    }
    for (int b = 0; b < nbins; ++b) {
        count[b] = (double)cnt[b];
        sum[b] = kval(&ks[b]);
        sumsq[b] = kval(&kq[b]);
        mean[b] = cnt[b] > 0 ? sum[b] / count[b] : NAN;
    }
    /* second pass: spread about the mean */
    for (long long u = 0; u < n; ++u) {
        long long h = sgn_index(u, n);
        for (long long v = 0; v < n; ++v) {
            long long k = sgn_index(v, n);
            for (long long w = 0; w < n; ++w) {
                long long l = sgn_index(w, n);
                int b = find_bin(h * h + k * k + l * l, nbins, U);
                if (b < 0) continue;
                cdouble f = F[((size_t)u * n + v) * n + w];
                double inten = creal(f) * creal(f) + cimag(f) * cimag(f);
                double d = inten - mean[b];
                kadd(&kv[b], d * d);
            }
        }
    }
    for (int b = 0; b < nbins; ++b)
        sem[b] = cnt[b] > 1 ? sqrt(kval(&kv[b]) / (double)(cnt[b] - 1) / (double)cnt[b]) : NAN;
    totals[0] = kval(&tot);
    totals[1] = creal(F[0]);
    totals[2] = cimag(F[0]);
    free(U); free(ks); free(kq); free(kv); free(cnt);
}

/* number of voxels of an n^3 box whose n2 falls in each bin (geometry only);
 * integer counts, so the per-plane split over threads is exact */
void or_bin_counts(int n, double voxel, int nbins, const double* edges, double* count)
{
    long long* U = (long long*)malloc(sizeof(long long) * (nbins + 1));
    or_thresholds(n, voxel, nbins, edges, U);
    long long* cnt = (long long*)calloc((size_t)nbins, sizeof(long long));
#pragma omp parallel
    {
        long long* mine = (long long*)calloc((size_t)nbins, sizeof(long long));
#pragma omp for schedule(static)
        for (long long u = 0; u < n; ++u) {
            long long h = sgn_index(u, n);
            for (long long v = 0; v < n; ++v) {
                long long k = sgn_index(v, n);
                for (long long w = 0; w < n; ++w) {
                    long long l = sgn_index(w, n);
                    int b = find_bin(h * h + k * k + l * l, nbins, U);
                    if (b >= 0) mine[b] += 1;
                }
            }
        }
#pragma omp critical
        for (int b = 0; b < nbins; ++b) cnt[b] += mine[b];
        free(mine);
    }
    for (int b = 0; b < nbins; ++b) count[b] = (double)cnt[b];
    free(U); free(cnt);
}

/* ------------------------------------------------------------------------ */
/* O12  per-bin sums of boxes too large for the n^3 loops of O7.
 *  (a) The voxel count of bin b is the number of lattice points (t, u, v),
 *      each in [-n/2, n/2), with U_b <= t^2 + u^2 + v^2 < U_b+1.  Taking t
 *      outermost: count_b = sum over t of P(U_b+1 - t^2) - P(U_b - t^2), with
 *      P(m) the number of (u, v) with u^2 + v^2 < m, tabulated once.
 *  (b) For a density of two voxels, rho1 at p and rho2 at p + d e_a (d along
 *      one axis a), eq. 1 gives n^6 |F(q)|^2 = rho1^2 + rho2^2
 *      + 2 rho1 rho2 cos(2 pi q_a d / n): the intensity depends on q only
 *      through its a-component t, so the bin sum of |F|^2 is the same sum
 *      over t, each term weighted by its intensity.  The phase t d is reduced
 *      mod n in integers.  Outputs count[b] and sum[b] = sum of |F|^2.       */
/* ------------------------------------------------------------------------ */
void or_axis_pair_bins(int n, double voxel, int nbins, const double* edges, long long d,
                       double rho1, double rho2, double* count, double* sum)
{
    long long* U = (long long*)malloc(sizeof(long long) * (nbins + 1));
    or_thresholds(n, voxel, nbins, edges, U);
    const long long h = n / 2;
    const long long mtop = 2 * h * h + 1;            /* u^2 + v^2 < mtop for every (u, v) */
    /* P[m] = #{(u, v) : u^2 + v^2 < m}, m in [0, mtop] */
    long long* P = (long long*)calloc((size_t)mtop + 1, sizeof(long long));
    for (long long u = -h; u < h; ++u)
        for (long long v = -h; v < h; ++v) P[u * u + v * v + 1] += 1;
    for (long long m = 1; m <= mtop; ++m) P[m] += P[m - 1];
    const double norm = 1.0 / ((double)n * n * n) / ((double)n * n * n);
#pragma omp parallel for schedule(dynamic, 8)
    for (int b = 0; b < nbins; ++b) {
        long long cnt = 0;
        kahan_t acc = {0.0, 0.0};
        for (long long t = -h; t < h; ++t) {
            long long lo = U[b] - t * t, hi = U[b + 1] - t * t;
            long long plo = lo <= 0 ? 0 : P[lo > mtop ? mtop : lo];
            long long phi = hi <= 0 ? 0 : P[hi > mtop ? mtop : hi];
            long long c = phi - plo;
            if (c == 0) continue;
            cnt += c;
            long long e = pmod(t * d, n);
            double inten = rho1 * rho1 + rho2 * rho2 + 2.0 * rho1 * rho2 * cos(2.0 * M_PI * (double)e / (double)n);
            kadd(&acc, (double)c * inten);
        }
        count[b] = (double)cnt;
        sum[b] = kval(&acc) * norm;
    }
    free(P);
    free(U);
}

/* ------------------------------------------------------------------------ */
/* O13  per-bin sums of a uniform cube (value v on every voxel with
 *      max_i |x_i - n/2| <= hw, zero elsewhere) at any n.  The density is a
 *      product of one indicator per axis, so eq. 1 factorises:
 *      F(h, k, l) = v S(h) S(k) S(l) / n^3 with S(u) the sum of
 *      exp(-2 pi i u x / n) over the 2 hw + 1 voxels of one axis, evaluated
 *      here by direct summation (integer phase reduced mod n).  With
 *      a(u) = |S(u)|^2, the sum of |F|^2 over bin b is
 *      v^2 / n^6 * sum over (h, k) of a(h) a(k) * (sum of a(l) over the l with
 *      U_b <= h^2 + k^2 + l^2 < U_b+1); the inner sum is a difference of the
 *      running sums of a(l) over |l| <= r.  Outputs count[b] and sum[b].
 *      voxel_form != 0 multiplies a(u) by sinc^2(pi u / n) (O15, the form
 *      factor of a voxel-uniform density), which keeps the product form.     */
/* ------------------------------------------------------------------------ */
static long long isqrt_floor(long long v)
{
    if (v <= 0) return 0;
    long long r = (long long)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

void or_cube_bins(int n, double voxel, int nbins, const double* edges, long long hw, double v,
                  int voxel_form, double* count, double* sum)
{
    long long* U = (long long*)malloc(sizeof(long long) * (nbins + 1));
    or_thresholds(n, voxel, nbins, edges, U);
    const long long h2 = n / 2;
    /* a[u + n/2] = |S(u)|^2 for u in [-n/2, n/2) */
    double* a = (double*)malloc(sizeof(double) * n);
#pragma omp parallel for schedule(static)
    for (long long u = -h2; u < h2; ++u) {
        cdouble s = 0;
        for (long long x = h2 - hw; x <= h2 + hw; ++x) {
            long long e = pmod(u * x, n);
            s += cexp(-2.0 * M_PI * I * (double)e / (double)n);
        }
        a[u + h2] = creal(s) * creal(s) + cimag(s) * cimag(s);
        if (voxel_form && u != 0) {             /* O15: times sinc^2(pi u / n) */
            const double x = M_PI * (double)u / (double)n;
            a[u + h2] *= (sin(x) / x) * (sin(x) / x);
        }
    }
    /* P[r] = sum of a(l) over l in [-n/2, n/2) with |l| <= r, kept as an
     * unevaluated pair Ph + Pl (exact two-sum accumulation): a bin's range
     * sum P[r1] - P[r0] can be many orders below P itself, and a single
     * rounded prefix would lose those digits.  Q[r] = number of such l.    */
    double* Ph = (double*)malloc(sizeof(double) * (h2 + 1));
    double* Pl = (double*)malloc(sizeof(double) * (h2 + 1));
    long long* Q = (long long*)malloc(sizeof(long long) * (h2 + 1));
    {
        double hi = 0.0, lo = 0.0;
#define OR_TWO_SUM_ADD(x) do { double t_ = hi + (x); double bp_ = t_ - hi; \
        lo += (hi - (t_ - bp_)) + ((x) - bp_); hi = t_; } while (0)
        OR_TWO_SUM_ADD(a[h2]);
        Ph[0] = hi; Pl[0] = lo;
        Q[0] = 1;
        for (long long r = 1; r <= h2; ++r) {
            if (r < h2) OR_TWO_SUM_ADD(a[h2 + r]);      /* l = +r exists only below n/2 */
            OR_TWO_SUM_ADD(a[h2 - r]);
            Ph[r] = hi; Pl[r] = lo;
            Q[r] = Q[r - 1] + (r < h2 ? 2 : 1);
        }
#undef OR_TWO_SUM_ADD
    }
    const int nt = omp_get_max_threads();
    long long* cnt_t = (long long*)calloc((size_t)nt * nbins, sizeof(long long));
    kahan_t* sum_t = (kahan_t*)calloc((size_t)nt * nbins, sizeof(kahan_t));
#pragma omp parallel
    {
        const int t = omp_get_thread_num();
        long long* mc = cnt_t + (size_t)t * nbins;
        kahan_t* ms = sum_t + (size_t)t * nbins;
#pragma omp for schedule(dynamic, 16)
        for (long long hh = -h2; hh < h2; ++hh)
            for (long long kk = -h2; kk < h2; ++kk) {
                const long long s2 = hh * hh + kk * kk;
                const double w = a[hh + h2] * a[kk + h2];
                /* first bin whose upper threshold exceeds s2 */
                int lo = 0, hi = nbins;
                while (lo < hi) { int mid = (lo + hi) / 2; if (U[mid + 1] <= s2) lo = mid + 1; else hi = mid; }
                for (int b = lo; b < nbins && U[b] <= s2 + h2 * h2; ++b) {
                    const long long m0 = U[b] - s2, m1 = U[b + 1] - s2;   /* l^2 in [m0, m1) */
                    const long long r0 = m0 <= 0 ? -1 : (isqrt_floor(m0 - 1) < h2 ? isqrt_floor(m0 - 1) : h2);
                    const long long r1 = m1 <= 0 ? -1 : (isqrt_floor(m1 - 1) < h2 ? isqrt_floor(m1 - 1) : h2);
                    if (r1 <= r0) continue;
                    mc[b] += Q[r1] - (r0 >= 0 ? Q[r0] : 0);
                    const double d = r0 >= 0 ? (Ph[r1] - Ph[r0]) + (Pl[r1] - Pl[r0]) : Ph[r1] + Pl[r1];
                    kadd(&ms[b], w * d);
                }
            }
    }
    const double norm = v * v / ((double)n * n * n) / ((double)n * n * n);
    for (int b = 0; b < nbins; ++b) {
        long long c = 0;
        kahan_t k = {0, 0};
        for (int t = 0; t < nt; ++t) {
            c += cnt_t[(size_t)t * nbins + b];
            kadd(&k, kval(&sum_t[(size_t)t * nbins + b]));
        }
        count[b] = (double)c;
        sum[b] = kval(&k) * norm;
    }
    free(cnt_t); free(sum_t); free(Ph); free(Pl); free(Q); free(a); free(U);
}

/* ------------------------------------------------------------------------ */
/* O11  Fourier coefficients on a small cube of low frequencies
 *     |h|, |k|, |l| <= K of the box of level (n1, f, nk), straight from eq. 1
 *     summed in the order of eq. 2 (z, then y, then x), with the density
 *     evaluated voxel by voxel from its definition (O2/O3).  Only voxels
 *     inside the cube that bounds the particle are visited (the density is
 *     zero elsewhere by definition).  out[(h+K)][(k+K)][(l+K)], normalised
 *     by 1/nk^3.  Phases use the exact integer product reduced mod nk.       */
/* ------------------------------------------------------------------------ */
void or_lowfreq_dft(int n1, int c, const double* cell, int kind, long long p0, long long p1,
                    int f, int nk, int K, cdouble* out)
{
    int nf = 2 * K + 1;
    long long m = n1 / f, o = (nk - m) / 2;
    long long hw = mask_halfwidth(kind, p0, p1, n1);
    /* coarse index range that can hold density */
    long long lo, hi;
    if (hw < 0) { for (int i = 0; i < nf * nf * nf; ++i) out[i] = 0; return; }
    {
        long long flo = n1 / 2 - hw, fhi = n1 / 2 + hw;
        if (flo < 0) flo = 0;
        if (fhi > n1 - 1) fhi = n1 - 1;
        lo = flo / f + o;
        hi = fhi / f + o;
    }
    long long span = hi - lo + 1;
    cdouble* ph = (cdouble*)malloc(sizeof(cdouble) * (size_t)nf * nk);   /* ph[j][x] = exp(-2 pi i (j-K) x / nk) */
    for (int j = 0; j < nf; ++j)
        for (long long x = 0; x < nk; ++x) {
            long long e = pmod((long long)(j - K) * x, nk);
            ph[(size_t)j * nk + x] = cexp(-2.0 * M_PI * I * (double)e / (double)nk);
        }
    /* G1[x][y][l] = sum_z rho e(l z) ; G2[x][k][l] = sum_y G1 e(k y) */
    cdouble* G2 = (cdouble*)calloc((size_t)span * nf * nf, sizeof(cdouble));
#pragma omp parallel
    {
        cdouble* g1 = (cdouble*)malloc(sizeof(cdouble) * nf);
        double* col = (double*)malloc(sizeof(double) * (size_t)span);
#pragma omp for schedule(dynamic, 1)
        for (long long xi = 0; xi < span; ++xi) {
            long long X = lo + xi;
            for (long long yi = 0; yi < span; ++yi) {
                long long Y = lo + yi;
                int any = 0;
                for (long long zi = 0; zi < span; ++zi) {
                    col[zi] = f == 1 ? ed1_value(n1, c, cell, kind, p0, p1, X, Y, lo + zi)
                                     : edk_value(n1, c, cell, kind, p0, p1, f, nk, X, Y, lo + zi);
                    any |= col[zi] != 0.0;
                }
                if (!any) continue;
                for (int l = 0; l < nf; ++l) {
                    cdouble s = 0;
                    for (long long zi = 0; zi < span; ++zi) s += col[zi] * ph[(size_t)l * nk + lo + zi];
                    g1[l] = s;
                }
                for (int k = 0; k < nf; ++k) {
                    cdouble e = ph[(size_t)k * nk + Y];
                    for (int l = 0; l < nf; ++l) G2[((size_t)xi * nf + k) * nf + l] += g1[l] * e;
                }
            }
        }
        free(g1);
        free(col);
    }
    double norm = 1.0 / ((double)nk * nk * nk);
    for (int h = 0; h < nf; ++h)
        for (int k = 0; k < nf; ++k)
            for (int l = 0; l < nf; ++l) {
                cdouble s = 0;
                for (long long xi = 0; xi < span; ++xi) s += G2[((size_t)xi * nf + k) * nf + l] * ph[(size_t)h * nk + lo + xi];
                out[((size_t)h * nf + k) * nf + l] = s * norm;
            }
    free(ph);
    free(G2);
}

/* eq. 1 at chosen frequencies for a density given by its nonzero voxels:
 *     F(u, v, w) = (1/n^3) sum_p rho_p exp(-2 pi i (u x_p + v y_p + w z_p) / n)
 * with the phase from the exact integer product reduced mod n.  Used to
 * sample transforms of boxes too large for or_fft3d.                        */
void or_dft_points(int n, long long npts, const long long* xyz, const double* val,
                   long long nq, const long long* uvw, cdouble* out)
{
    const double norm = 1.0 / ((double)n * n * n);
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < nq; ++q) {
        const long long u = uvw[3 * q], v = uvw[3 * q + 1], w = uvw[3 * q + 2];
        cdouble s = 0;
        for (long long p = 0; p < npts; ++p) {
            long long e = pmod(u * xyz[3 * p] + v * xyz[3 * p + 1] + w * xyz[3 * p + 2], n);
            s += val[p] * cexp(-2.0 * M_PI * I * (double)e / (double)n);
        }
        out[q] = s * norm;
    }
}

/* sum of rho and of rho^2 over the box of level (n1, f, nk), from the
 * definition (used for F(0) and for the Parseval check at sizes where the
 * full transform is not run) */
void or_density_moments(int n1, int c, const double* cell, int kind, long long p0, long long p1,
                        int f, int nk, double* out2)
{
    long long m = n1 / f, o = (nk - m) / 2;
    long long hw = mask_halfwidth(kind, p0, p1, n1);
    if (hw < 0) { out2[0] = out2[1] = 0.0; return; }
    long long flo = n1 / 2 - hw, fhi = n1 / 2 + hw;
    if (flo < 0) flo = 0;
    if (fhi > n1 - 1) fhi = n1 - 1;
    long long lo = flo / f + o, hi = fhi / f + o, span = hi - lo + 1;
    double s1 = 0.0, s2 = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : s1, s2)
    for (long long xi = 0; xi < span; ++xi) {
        kahan_t a = {0, 0}, b = {0, 0};
        for (long long yi = 0; yi < span; ++yi)
            for (long long zi = 0; zi < span; ++zi) {
                double r = f == 1 ? ed1_value(n1, c, cell, kind, p0, p1, lo + xi, lo + yi, lo + zi)
                                  : edk_value(n1, c, cell, kind, p0, p1, f, nk, lo + xi, lo + yi, lo + zi);
                kadd(&a, r);
                kadd(&b, r * r);
            }
        s1 += kval(&a);
        s2 += kval(&b);
    }
    out2[0] = s1;
    out2[1] = s2;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
