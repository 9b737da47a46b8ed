// gfx950 kernels of the scattering-simulation hot path (arXiv 2303.13435):
//   pass Z  : ED generation (tiled cell x mask, zoom block sums) fused with
//             the first 1D transform (r2c, two real pencils per complex FFT),
//             written transposed as [x][kz][y] in 128-byte row segments;
//   pass Y  : contiguous column FFTs along y, written transposed as
//             [kz][ky][x] in 128-byte segments;
//   pass X  : contiguous column FFTs along x with |F|^2 and integer-threshold
//             |Q| binning fused (persistent blocks, LDS histograms);
//   finalize: fixed-order compensated reduction of the block histograms;
//   merge   : zoom-level merge per bin;
//   inverse passes and the adjoint column pass for the gradients.
// eq. 1 defines the transform; eq. 2 is the axis-by-axis separation used.
#include <hip/hip_runtime.h>

#include "ur_device.hpp"
#include "ur_geom.hpp"
#include "ur_kernels.hpp"

// The file is compiled once per part (-DUR_PART=k, k in [0, UR_NPARTS)) so
// that the large template instantiations build in parallel: part 0 holds the
// small kernels and the dispatchers, the others one group of transform passes
// each.  Without UR_PART it is a single translation unit holding everything.
#ifndef UR_PART
#define UR_PART -1
#endif
#define UR_IN(k) (UR_PART < 0 || UR_PART == (k))

// compile-time choices picked by the tuner (paper_2303_13435_amd/tune.py)
#include "ur_tuned.hpp"

namespace ur {

// ---------------------------------------------------------------------------
// block configuration
// ---------------------------------------------------------------------------
// Stores of the first intermediate (pass Z) and of the second (pass Y): with
// the streaming policy or plain (tuned)
template <typename T> __device__ __forceinline__ void st_a2(cx2<T>* p, cx2<T> v) {
  if constexpr (UR_ST_NT_A) st_nt2(p, v); else *p = v;
}
template <typename T> __device__ __forceinline__ void st_b(cx<T>* p, cx<T> v) {
  if constexpr (UR_ST_NT_B) st_nt(p, v); else *p = v;
}
template <typename T> struct Seg { static constexpr int cols = 128 / (int)sizeof(cx<T>); };  // 16 f32, 8 f64

// z pass: groups per block (each group = one complex FFT = two real pencils
// in r2c); PAIRS is the pencil-pair count of real FP32 columns up to 1024
// points (the forward pass and the inverse passes are tuned apart)
template <typename T, int N, bool C2C, int PAIRS = UR_Z_PAIRS_F32> struct ZCfg {
  static constexpr int G = Geo<N>::G;
  // 2048-point columns span two wavefronts and sync with the workgroup
  // barrier: half-width tiles keep two blocks per CU (measured faster than
  // one block of full 128-byte rows); 4096-point columns (four wavefronts)
  // take quarter-width tiles for the same LDS budget
  // (real FP32 columns up to 1024 points: UR_Z_PAIRS_F32 pencil pairs, tuned)
  static constexpr int want = N >= 4096 ? (C2C ? Seg<T>::cols / 4 : Seg<T>::cols / 8)
                            : N == 2048 ? (C2C ? Seg<T>::cols / 2 : Seg<T>::cols / 4)
                            : C2C       ? Seg<T>::cols
                                        : (sizeof(T) == 4 ? PAIRS : Seg<T>::cols / 2);
  static constexpr int fill = 256 / G > 0 ? 256 / G : 1;
  static constexpr int ng0 = want > fill ? want : fill;
  static constexpr int cap = C2C ? N : N / 2;
  static constexpr int NG = ng0 < cap ? ng0 : cap;
  static constexpr int TY = C2C ? NG : 2 * NG;
  static constexpr int threads = NG * G;
};
// y pass: x planes per block (two per group)
template <typename T, int N> struct YCfg {
  static constexpr int G = Geo<N>::G;
  // 4096-point columns: half-width tiles (1024 threads, 150 KB of LDS);
  // 2048-point FP32 columns: half-width tiles when UR_Y_HALF_2K (two blocks of
  // 75 KB per CU instead of one of 150 KB; 64-byte instead of 128-byte
  // segments of B; tuned)
  static constexpr bool HALF = N >= 4096 || (N == 2048 && UR_Y_HALF_2K && sizeof(T) == 4);
  static constexpr int TX = HALF ? Seg<T>::cols / 2 : (Seg<T>::cols < N ? Seg<T>::cols : N);
  static constexpr int NS = TX / 2;
  static constexpr int threads = NS * G;
};
// inverse y pass: every plane of the tile has its own LDS column
template <typename T, int N> struct YICfg {
  static constexpr int G = Geo<N>::G;
  static constexpr int TX = YCfg<T, N>::TX;
  static constexpr int threads = TX * G;
};
// x pass: columns per block
template <int N> struct XCfg {
  static constexpr int G = Geo<N>::G;
  // 4096-point columns: two per block, so that a CU holds eight wavefronts;
  // one-wavefront columns (1024 points): UR_X_THREADS threads' worth, and
  // two-wavefront columns (2048 points) UR_X_THREADS_2K (tuned; a block of
  // one such column syncs only its own two wavefronts); shorter columns:
  // 256 threads' worth
  static constexpr int T0 = G == 64 ? UR_X_THREADS : (G == 128 ? UR_X_THREADS_2K : 256);
  static constexpr int want = T0 / G > 0 ? T0 / G : 1;
  static constexpr int NG = G > 128 ? 2 : (want < 64 ? want : 64);
  static constexpr int threads = NG * G;
};
// minimum resident waves per SIMD the binning x pass is compiled for (a VGPR
// cap; 1 = none), per precision (tuned)
template <typename T> struct XMinW { static constexpr int v = sizeof(T) == 4 ? UR_X_MINW_F32 : UR_X_MINW_F64; };
// LDS column stride: a multiple of 32 elements plus 4, so that reading the
// same few consecutive rows from 8 neighbouring columns (the transposed
// write-outs) touches 32 distinct 8-byte bank pairs
template <int N> struct CS {
  static constexpr int v = ((Padded<N>::size + 31) / 32) * 32 + 4;
};
// minimum resident waves per SIMD the streaming passes are compiled for
// (caps VGPRs at 128 for FP32 and 256 for FP64)
template <typename T> struct MinW { static constexpr int v = sizeof(T) == 4 ? 4 : 2; };

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
template <int W = 64>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// ---------------------------------------------------------------------------
// cell synthesis: voxel-integrated Gaussians with periodic images
// ---------------------------------------------------------------------------
__device__ __forceinline__ double phi_cdf(double t) { return 0.5 * erfc(-t * 0.70710678118654752440); }

#if UR_IN(0)
__global__ void k_cell_profiles(int c, int n_atoms, const double* __restrict__ xyz,
                                const double* __restrict__ sigma, double* __restrict__ prof) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long total = (long long)n_atoms * 3 * c;
  if (t >= total) return;
  int i = (int)(t % c);
  long long ad = t / c;
  int d = (int)(ad % 3);
  long long a = ad / 3;
  double x = xyz[3 * a + d], s = sigma[a];
  double acc = 0.0;
  if (s > 0.0) {
    int M = (int)ceil(8.0 * s / c) + 1;
    if (M > 64) M = 64;
    for (int m = -M; m <= M; ++m) {
      double base = (double)i - x + (double)m * c;
      acc += phi_cdf((base + 0.5) / s) - phi_cdf((base - 0.5) / s);
    }
  }
  prof[t] = acc;
}

// cell = background + sum over atoms of A_a p_x p_y p_z; the profiles (and
// amplitudes) are staged in LDS when they fit (dynamic LDS of the launch),
// else read from global memory; with cellT the working-precision copy is
// written too (the only table of a level of factor 1)
template <typename T>
__global__ void __launch_bounds__(256) k_cell_sum(int c, int n_atoms, const double* __restrict__ amp,
                                                  const double* __restrict__ prof, double bg, double* __restrict__ cell,
                                                  T* __restrict__ cellT, int staged) {
  extern __shared__ double lp[];                       // staged: 3 c n_atoms profiles, then n_atoms amplitudes
  const long long c3 = (long long)c * c * c;
  const double* P = prof;
  const double* Am = amp;
  if (staged) {
    const int np = 3 * c * n_atoms;
    for (int i = threadIdx.x; i < np; i += 256) lp[i] = prof[i];
    for (int i = threadIdx.x; i < n_atoms; i += 256) lp[np + i] = amp[i];
    __syncthreads();
    P = lp;
    Am = lp + np;
  }
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c3) return;
  const int k = (int)(v % c), j = (int)((v / c) % c), i = (int)(v / ((long long)c * c));
  double acc = bg;
  for (int a = 0; a < n_atoms; ++a) {
    const double* p = P + (size_t)a * 3 * c;
    acc += Am[a] * p[i] * p[c + j] * p[2 * c + k];
  }
  cell[v] = acc;
  if (cellT) cellT[v] = (T)acc;
}

#endif
template <typename T>
__global__ void k_cell_tables(int c, int f, const double* __restrict__ cell, T* __restrict__ cellT,
                              double* __restrict__ pre, T* __restrict__ cb, int cbn) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long c3 = (long long)c * c * c;
  if (t < c3) cellT[t] = (T)cell[t];
  if (f > 1) {
    // row prefix sums: pre[(i c + j)(c+1) + k] = sum_{k' < k} cell[i][j][k']
    if (t < (long long)c * c) {
      const double* row = cell + t * c;
      double* pr = pre + t * (c + 1);
      double s = 0.0;
      pr[0] = 0.0;
      for (int k = 0; k < c; ++k) { s += row[k]; pr[k + 1] = s; }
    }
  }
}

// Block table of a zoomed level: cb[I][J][K] = sum of the cell over the
// fe^3 voxels from (I fe, J fe, K fe), fe = min(f, c), times (f/fe)^3 (a block
// larger than the cell holds (f/c)^3 whole cells).  One workgroup per entry,
// fixed-order tree reduction.
template <typename T>
__global__ void __launch_bounds__(256) k_cell_blocks(int c, int f, const double* __restrict__ cell, T* __restrict__ cb, int cbn) {
  __shared__ double red[256];
  const int t = blockIdx.x;
  const int K = t % cbn, J = (t / cbn) % cbn, I = t / (cbn * cbn);
  const int fe = f < c ? f : c;
  const int ne = fe * fe * fe;
  double s = 0.0;
  for (int e = threadIdx.x; e < ne; e += 256) {
    const int d = e % fe, b = (e / fe) % fe, aa = e / (fe * fe);
    s += cell[((size_t)(I * fe + aa) * c + (J * fe + b)) * c + (K * fe + d)];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = (double)(f / fe);
    cb[t] = (T)(red[0] * (m * m * m));
  }
}

// ---------------------------------------------------------------------------
// density of one pencil (x, y) along z: tiled cell x mask, block-summed for
// zoomed levels.  Exact integer geometry; values from the cell tables.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pmodi(long long a, int m) { long long r = a % m; return (int)(r < 0 ? r + m : r); }

// cubic B-spline weights of the four coefficients around a point at
// fractional offset t in [0, 1): B3(t + 1), B3(t), B3(t - 1), B3(t - 2)
template <typename T>
__device__ __forceinline__ void bspline_weights(T t, T* w) {
  const T t2 = t * t, t3 = t2 * t, s = (T)1 - t;
  const T k = (T)1 / (T)6;
  w[0] = k * s * s * s;
  w[1] = k * ((T)3 * t3 - (T)6 * t2 + (T)4);
  w[2] = k * ((T)-3 * t3 + (T)3 * t2 + (T)3 * t + (T)1);
  w[3] = k * t3;
}

template <typename T>
struct Pencil {
  int zlo, zhi;             // coarse z range that can hold density (zlo > zhi: empty)
  // f == 1: value(z) = row[(z + zoff) & cmask] inside [zlo, zhi]
  const T* row;
  int zoff, cmask;
  // f > 1
  long long rin;            // blocks with max|dz| <= rin are fully inside
  int I, J;                 // block-table indices of this pencil
  long long fx0, fy0;       // first fine x, y of the pencil's block column
  int zin_lo, zin_hi;       // coarse z of the blocks wholly inside the mask
  // rotated lattice (f == 1): u = rot (dx, dy, dz), dz = z + zoff; (ux, uy, uz) = rot (dx, dy, 0)
  double ux, uy, uz;
  int pdx, pdy;             // pencil offset from the particle centre (grains)
  const double* GR;         // grain orientations [g][9] (the arguments, or a copy in LDS)
  int A[kMaxGrains];        // grains: squared in-plane distance of the pencil to each seed

  // grains: |(dx, dy) - seed_g (x, y)|^2 for every grain (int32: offsets
  // stay below 4096 and seeds below 8192 in magnitude, so squared distances
  // stay below 2^30)
  __device__ __forceinline__ void init_grains(const ZArgs& a) {
#pragma unroll
    for (int g = 0; g < kMaxGrains; ++g) {
      const int ex = pdx - a.gseed[g][0], ey = pdy - a.gseed[g][1];
      A[g] = g < a.ngrain ? ex * ex + ey * ey : 0x7fffffff;
    }
  }

  __device__ __forceinline__ void init(const ZArgs& a, long long X, long long Y) { init_at(a, a.L, X, Y); }

  // the pencil (X, Y) of level L (the arguments' own level, or the ED-1
  // grid beneath a zoom level)
  __device__ __forceinline__ void init_at(const ZArgs& a, const Level& L, long long X, long long Y) {
    long long lo, hi;
    col_range(L, a.m, X, Y, lo, hi);
    zlo = (int)lo;
    zhi = (int)hi;
    if (lo > hi) { zlo = 1; zhi = 0; }
    cmask = L.c - 1;                                   // c is a power of two
    if (L.f == 1) {
      const int i = (int)(X - L.o - L.h) & cmask, j = (int)(Y - L.o - L.h) & cmask;
      row = (const T*)a.cellT + ((size_t)i * L.c + j) * L.c;
      zoff = -(L.o + L.h);
      if (a.rotated) {
        // each product and sum rounded on its own (no contraction), in the
        // order the reference evaluation uses
        const double dx = (double)(X - L.o - L.h), dy = (double)(Y - L.o - L.h);
        ux = __dadd_rn(__dmul_rn(a.rot[0], dx), __dmul_rn(a.rot[1], dy));
        uy = __dadd_rn(__dmul_rn(a.rot[3], dx), __dmul_rn(a.rot[4], dy));
        uz = __dadd_rn(__dmul_rn(a.rot[6], dx), __dmul_rn(a.rot[7], dy));
        pdx = (int)(X - L.o - L.h);
        pdy = (int)(Y - L.o - L.h);
        GR = &a.grot[0][0];
      }
    } else {
      long long ax, bx, ay, by;
      block_dist(L, X, ax, bx);
      block_dist(L, Y, ay, by);
      // a factor that is not a power of two (mixed-radix levels) has blocks
      // that are not aligned to cell periods: no whole-block table, every
      // block summed pencil by pencil (value_zoom's exact route)
      rin = (L.f & (L.f - 1)) ? -1 : mask_reach(a.m, bx, by);
      fx0 = (long long)L.f * (X - L.o);
      fy0 = (long long)L.f * (Y - L.o);
      if (L.f <= L.c) {
        I = pmodi(fx0 - L.h, L.c) / L.f;
        J = pmodi(fy0 - L.h, L.c) / L.f;
      } else {
        I = J = 0;
      }
      // block Z is wholly inside iff its fine z range [f(Z-o), f(Z-o)+f-1]
      // lies in [h - rin, h + rin]; f is a power of two (floor division by
      // an arithmetic shift)
      zin_lo = 1; zin_hi = 0;
      if (rin >= 0 && zlo <= zhi) {
        const int lf = __builtin_ctz(L.f);
        const long long lo2 = -((-(L.h - rin)) >> lf) + L.o;       // ceil((h - rin) / f) + o
        const long long hi2 = ((L.h + rin - L.f + 1) >> lf) + L.o;  // floor((h + rin - f + 1) / f) + o
        zin_lo = (int)(lo2 > zlo ? lo2 : zlo);
        zin_hi = (int)(hi2 < zhi ? hi2 : zhi);
      }
    }
  }

  // zoomed level, all but the boundary blocks: the block table for blocks
  // wholly inside, zero outside [zlo, zhi]; *bnd flags a block that is
  // partly inside (its value is left to the caller)
  __device__ __forceinline__ T zoom_fast(const ZArgs& a, int Z, bool& bnd) const {
    bnd = false;
    if (Z < zlo || Z > zhi) return (T)0;
    if (Z >= zin_lo && Z <= zin_hi) {
      const Level& L = a.L;
      const int K = L.f <= L.c ? (((L.f * (Z - L.o) - L.h) & (L.c - 1)) >> __builtin_ctz(L.f)) : 0;
      return ((const T*)a.cb)[((size_t)I * a.cbn + J) * a.cbn + K];
    }
    bnd = true;
    return (T)0;
  }

  // ED-1 voxel of a rotated lattice: the cell at u = rot d, trilinear
  // between its voxels with periodic wrap (interpolated along the cell's
  // third index, then the second, then the first); zero outside the mask
  // cell coordinate u = R d of inside voxel z: R the lattice's orientation,
  // or with grains that of the seed nearest to d (squared integer distance,
  // ties to the lower index); products and sums rounded one by one
  template <bool GRAINS>
  __device__ __forceinline__ void coords(const ZArgs& a, int z, double& u, double& v, double& w) const {
    const double dz = (double)(z + zoff);
    if constexpr (!GRAINS) {
      u = __dadd_rn(ux, __dmul_rn(a.rot[2], dz));
      v = __dadd_rn(uy, __dmul_rn(a.rot[5], dz));
      w = __dadd_rn(uz, __dmul_rn(a.rot[8], dz));
      return;
    }
    const int iz = z + zoff;
    int best = 0, bd = 0x7fffffff;
#pragma unroll
    for (int g = 0; g < kMaxGrains; ++g) {               // A[g] is 2^31 - 1 beyond the grains
      const int ez = iz - a.gseed[g][2];
      const int d2 = A[g] == 0x7fffffff ? 0x7fffffff : A[g] + ez * ez;
      if (d2 < bd) { bd = d2; best = g; }
    }
    const double* R = GR + 9 * best;
    const double dx = (double)pdx, dy = (double)pdy;
    u = __dadd_rn(__dadd_rn(__dmul_rn(R[0], dx), __dmul_rn(R[1], dy)), __dmul_rn(R[2], dz));
    v = __dadd_rn(__dadd_rn(__dmul_rn(R[3], dx), __dmul_rn(R[4], dy)), __dmul_rn(R[5], dz));
    w = __dadd_rn(__dadd_rn(__dmul_rn(R[6], dx), __dmul_rn(R[7], dy)), __dmul_rn(R[8], dz));
  }

  template <bool GRAINS>
  __device__ __forceinline__ T value_rot(const ZArgs& a, int z, const T* C) const {
    if (z < zlo || z > zhi) return (T)0;
    double u, v, w;
    coords<GRAINS>(a, z, u, v, w);
    const double fu = floor(u), fv = floor(v), fw = floor(w);
    const T tu = (T)(u - fu), tv = (T)(v - fv), tw = (T)(w - fw);
    const int c = cmask + 1;
    const int i0 = (int)(long long)fu & cmask, i1 = (i0 + 1) & cmask;
    const int j0 = (int)(long long)fv & cmask, j1 = (j0 + 1) & cmask;
    const int k0 = (int)(long long)fw & cmask, k1 = (k0 + 1) & cmask;
    const T* r00 = C + ((size_t)i0 * c + j0) * c;
    const T* r01 = C + ((size_t)i0 * c + j1) * c;
    const T* r10 = C + ((size_t)i1 * c + j0) * c;
    const T* r11 = C + ((size_t)i1 * c + j1) * c;
    const T a00 = r00[k0] + tw * (r00[k1] - r00[k0]);
    const T a01 = r01[k0] + tw * (r01[k1] - r01[k0]);
    const T a10 = r10[k0] + tw * (r10[k1] - r10[k0]);
    const T a11 = r11[k0] + tw * (r11[k1] - r11[k0]);
    const T b0 = a00 + tv * (a01 - a00);
    const T b1 = a10 + tv * (a11 - a10);
    return b0 + tu * (b1 - b0);
  }

  // ED-1 voxel of a rotated lattice, cubic B-spline: cellT holds the
  // periodic spline coefficients C; the value at u is the sum over the
  // 4 x 4 x 4 coefficients around floor(u) with the cubic B-spline weights
  // of the fractional offsets (third index innermost)
  template <bool GRAINS>
  __device__ __forceinline__ T value_rot3(const ZArgs& a, int z, const T* C) const {
    if (z < zlo || z > zhi) return (T)0;
    double u, v, w;
    coords<GRAINS>(a, z, u, v, w);
    const double fu = floor(u), fv = floor(v), fw = floor(w);
    T wu[4], wv[4], ww[4];
    bspline_weights<T>((T)(u - fu), wu);
    bspline_weights<T>((T)(v - fv), wv);
    bspline_weights<T>((T)(w - fw), ww);
    const int c = cmask + 1;
    const int i0 = (int)(long long)fu - 1, j0 = (int)(long long)fv - 1, k0 = (int)(long long)fw - 1;
    T acc = (T)0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      T sp = (T)0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T* r = C + ((size_t)((i0 + p) & cmask) * c + ((j0 + q) & cmask)) * c;
        T sq = (T)0;
#pragma unroll
        for (int m = 0; m < 4; ++m) sq += ww[m] * r[(k0 + m) & cmask];
        sp += wv[q] * sq;
      }
      acc += wu[p] * sp;
    }
    return acc;
  }

  // the sampler chosen at compile time (pass Z modes), or at run time from
  // the arguments (density generation)
  template <int INTERP, bool GRAINS>
  __device__ __forceinline__ T value_rotated(const ZArgs& a, int z, const T* C) const {
    if constexpr (INTERP == 3) return value_rot3<GRAINS>(a, z, C);
    else return value_rot<GRAINS>(a, z, C);
  }
  __device__ __forceinline__ T value_rotated_rt(const ZArgs& a, int z) const {
    const T* C = (const T*)a.cellT;
    if (a.cubic) return a.ngrain ? value_rot3<true>(a, z, C) : value_rot3<false>(a, z, C);
    return a.ngrain ? value_rot<true>(a, z, C) : value_rot<false>(a, z, C);   // init_grains first
  }

  // ED-1 voxel (factor 1): tiled cell inside the mask, exact integer test
  __device__ __forceinline__ T value1(int z) const {
    return (z >= zlo && z <= zhi) ? row[(z + zoff) & cmask] : (T)0;
  }

  // sum of the periodic cell row (i, j) over fine z in [za, zb]
  __device__ __forceinline__ double rowsum(const ZArgs& a, int i, int j, long long za, long long zb) const {
    const Level& L = a.L;
    const int c = L.c;
    const double* P = a.pre + ((size_t)i * c + j) * (c + 1);
    int ka = pmodi(za - L.h, c);
    long long len = zb - za + 1;
    long long q = len / c;
    int rem = (int)(len - q * c);
    double s = (double)q * P[c];
    if (ka + rem <= c) s += P[ka + rem] - P[ka];
    else s += (P[c] - P[ka]) + P[ka + rem - c];
    return s;
  }

  // zoomed level (factor f > 1): block sum of ED-1 over the f^3 fine voxels
  __device__ __noinline__ T value_zoom(const ZArgs& a, long long Z) const {
    if (Z < zlo || Z > zhi) return (T)0;
    const Level& L = a.L;
    long long cz, dz;
    block_dist(L, Z, cz, dz);
    if (rin >= 0 && dz <= rin) {            // whole block inside: block table
      int K = L.f <= L.c ? pmodi((long long)L.f * (Z - L.o) - L.h, L.c) / L.f : 0;
      return ((const T*)a.cb)[((size_t)I * a.cbn + J) * a.cbn + K];
    }
    // boundary block: sum the inside part of every fine pencil of the block
    const long long fz0 = (long long)L.f * (Z - L.o);
    double s = 0.0;
    for (int u = 0; u < L.f; ++u) {
      long long fx = fx0 + u, dxa = fx - L.h < 0 ? L.h - fx : fx - L.h;
      int i = pmodi(fx - L.h, L.c);
      for (int w = 0; w < L.f; ++w) {
        long long fy = fy0 + w, dya = fy - L.h < 0 ? L.h - fy : fy - L.h;
        long long r = mask_reach(a.m, dxa, dya);
        if (r < 0) continue;
        long long za = fz0 > L.h - r ? fz0 : L.h - r;
        long long zb = fz0 + L.f - 1 < L.h + r ? fz0 + L.f - 1 : L.h + r;
        if (za > zb) continue;
        s += rowsum(a, i, pmodi(fy - L.h, L.c), za, zb);
      }
    }
    return (T)s;
  }

  __device__ __forceinline__ T value(const ZArgs& a, long long Z) const {
    return a.L.f == 1 ? value1((int)Z) : value_zoom(a, Z);
  }
};

// Sum of ED-1 over the inside fine voxels of one zoom block whose fine
// corner is (fx0, fy0, fz0), evaluated by all 64 lanes of the wavefront
// together: lane l takes the fine pencils k = l, l + 64, ... of the f^2 in the
// block, each an O(1) prefix-sum difference over its inside z segment; the
// result is returned to every lane.  Cell edge c and factor f are powers of two.
__device__ __forceinline__ double zoom_block_sum(const ZArgs& a, int fx0, int fy0, int fz0) {
  const Level& L = a.L;
  const int f = L.f, c = L.c, h = L.h, lf = __builtin_ctz(f), lc = __builtin_ctz(c);
  double s = 0.0;
  for (int k = __lane_id(); k < f * f; k += 64) {
    const int fx = fx0 + (k >> lf), fy = fy0 + (k & (f - 1));
    const long long r = mask_reach(a.m, fx < h ? h - fx : fx - h, fy < h ? h - fy : fy - h);
    if (r < 0) continue;
    const long long za = fz0 > h - r ? fz0 : h - r;
    const long long zb = fz0 + f - 1 < h + r ? fz0 + f - 1 : h + r;
    if (za > zb) continue;
    const double* P = a.pre + ((size_t)((fx - h) & (c - 1)) * c + ((fy - h) & (c - 1))) * (c + 1);
    const int ka = (int)((za - h) & (c - 1));
    const long long len = zb - za + 1;
    const int rem = (int)(len & (c - 1));
    double t = (double)(len >> lc) * P[c];
    if (ka + rem <= c) t += P[ka + rem] - P[ka];
    else t += (P[c] - P[ka]) + P[ka + rem - c];
    s += t;
  }
  return wave_sum<64>(s);
}

// ---------------------------------------------------------------------------
// pass Z: density -> 1D transform along z -> A[x][kz][y]
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ void __launch_bounds__((ZCfg<T, N, (MODE == Z_GEN_C2C || MODE == Z_LOAD_C2C || MODE == Z_ZOOM_C2C)>::threads), MinW<T>::v)
k_pass_z(ZArgs a) {
  constexpr bool C2C = MODE == Z_GEN_C2C || MODE == Z_LOAD_C2C || MODE == Z_ZOOM_C2C;
  constexpr bool ZOOM = MODE == Z_ZOOM_R2C || MODE == Z_ZOOM_C2C;
  constexpr bool ROT = MODE == Z_ROT_R2C || MODE == Z_ROT3_R2C || MODE == Z_ROTG_R2C || MODE == Z_ROT3G_R2C;
  constexpr int RI = (MODE == Z_ROT3_R2C || MODE == Z_ROT3G_R2C) ? 3 : 1;     // sampler of a rotated cell
  constexpr bool RG = MODE == Z_ROTG_R2C || MODE == Z_ROT3G_R2C;              // grains
  constexpr bool GEN = MODE == Z_GEN_R2C || MODE == Z_GEN_C2C || ZOOM || ROT;
  using C = ZCfg<T, N, C2C>;
  constexpr int G = C::G, NG = C::NG, TY = C::TY, E = Geo<N>::E;
  constexpr int R0 = Radix<N, 1>::r, NB0 = E / R0, PS = CS<N>::v;
  __shared__ cx<T> sm[NG * PS];
  __shared__ double red[C::threads];                   // per-lane sums of rho^2
  constexpr int CL = ROT ? 4096 : 1;                   // rotated: cells up to 16^3 staged in LDS
  __shared__ T cl[CL];
  __shared__ double grl[RG ? kMaxGrains * 9 : 1];      // grain orientations (per-voxel choice)

  // Tiles narrower than a 128-byte line of A (UR_Z_XCD): workgroups are
  // dealt to the 8 XCDs in turn, so blocks b and b + 8 run on the same XCD
  // at about the same time; within every 16 blocks the two tiles that share
  // each line go to such a pair, and both halves of the line meet in one L2.
  unsigned bid = blockIdx.x;
  if constexpr (UR_Z_XCD && TY * sizeof(cx<T>) < 128) {
    const unsigned j = bid & 15u;
    if ((bid | 15u) < gridDim.x && a.ntiles % 16 == 0) bid = (bid & ~15u) + 2 * (j & 7u) + (j >> 3);
  }
  const int tile = bid % a.ntiles;
  const long long X = a.x0 + bid / a.ntiles;
  const int y0 = tile * TY;
  const cx<T>* tw = (const cx<T>*)a.tw;
  cx<T>* A = (cx<T>*)a.A;

  if (GEN) {
    long long ylo, yhi;
    row_range(a.L, a.m, X, ylo, yhi);
    if (ylo > yhi || y0 + TY - 1 < ylo || y0 > yhi) {   // no density in this tile
      if (a.mom && threadIdx.x == 0) { a.mom[2 * blockIdx.x] = 0.0; a.mom[2 * blockIdx.x + 1] = 0.0; }
      return;
    }
  }
  // with G >= 64 every wavefront lies inside one group, so the pencil index
  // is wave-uniform: the pencil set-up (integer geometry) runs on the scalar unit
  const int q = G >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / G) : threadIdx.x / G;
  const int g = threadIdx.x % G;
  cx<T>* s = sm + q * PS;
  cx<T> v[E];
  double m2 = 0.0;                                       // sum of rho^2 (the finalize uses it)

  if (!C2C) {
    const long long yA = y0 + 2 * q, yB = yA + 1;
    if (GEN) {
      Pencil<T> pa, pb;
      pa.init(a, X, yA);
      pb.init(a, X, yB);
      if constexpr (ROT) {
        // the cell's samples are gathers at arbitrary positions: from LDS
        // when the cell fits (block-uniform test), else through the caches
        const int c3 = a.L.c * a.L.c * a.L.c;
        if constexpr (RG) {
          for (int i = threadIdx.x; i < 9 * a.ngrain; i += C::threads) grl[i] = (&a.grot[0][0])[i];
          pa.GR = grl;
          pb.GR = grl;
          pa.init_grains(a);
          pb.init_grains(a);
        }
        if (c3 <= CL) {
          for (int i = threadIdx.x; i < c3; i += C::threads) cl[i] = ((const T*)a.cellT)[i];
          __syncthreads();
#pragma unroll
          for (int i = 0; i < NB0; ++i)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              const int z = first_index<N>(g, i, r);
              v[i * R0 + r] = mk(pa.template value_rotated<RI, RG>(a, z, cl), pb.template value_rotated<RI, RG>(a, z, cl));
            }
        } else {
          if constexpr (RG) __syncthreads();             // the grain table
          const T* cg = (const T*)a.cellT;
#pragma unroll
          for (int i = 0; i < NB0; ++i)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              const int z = first_index<N>(g, i, r);
              v[i * R0 + r] = mk(pa.template value_rotated<RI, RG>(a, z, cg), pb.template value_rotated<RI, RG>(a, z, cg));
            }
        }
      } else if (!ZOOM) {
        // the cell residue of z = b + r N/R0 does not depend on r when the
        // cell edge divides N/R0: one cell load per pencil and butterfly
        const bool one_load = ((N / R0) & pa.cmask) == 0;
        if (one_load) {
#pragma unroll
          for (int i = 0; i < NB0; ++i) {
            const int b = g + Geo<N>::G * i;
            const T ca = pa.row[(b + pa.zoff) & pa.cmask], cb = pb.row[(b + pb.zoff) & pb.cmask];
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              const int z = b + r * (N / R0);
              v[i * R0 + r] = mk((z >= pa.zlo && z <= pa.zhi) ? ca : (T)0, (z >= pb.zlo && z <= pb.zhi) ? cb : (T)0);
            }
          }
        } else {
#pragma unroll
          for (int i = 0; i < NB0; ++i) {
            const int b = g + Geo<N>::G * i;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              const int z = b + r * (N / R0);
              v[i * R0 + r] = mk(pa.value1(z), pb.value1(z));
            }
          }
        }
      } else if constexpr (C::threads % 64 == 0) {
        // table lookups per lane; each block that is only partly inside is
        // summed by the whole wavefront (ballot, then one block at a time)
        const int lane = __lane_id();
#pragma unroll
        for (int i = 0; i < NB0; ++i)
#pragma unroll
          for (int r = 0; r < R0; ++r) {
            const int z = first_index<N>(g, i, r);
            bool ba, bb;
            T va = pa.zoom_fast(a, z, ba), vb = pb.zoom_fast(a, z, bb);
            for (unsigned long long m = __ballot(ba); m; m &= m - 1) {
              const int l = __builtin_ctzll(m);
              const double t = zoom_block_sum(a, __builtin_amdgcn_readlane((int)pa.fx0, l), __builtin_amdgcn_readlane((int)pa.fy0, l),
                                              a.L.f * (__builtin_amdgcn_readlane(z, l) - a.L.o));
              if (lane == l) va = (T)t;
            }
            for (unsigned long long m = __ballot(bb); m; m &= m - 1) {
              const int l = __builtin_ctzll(m);
              const double t = zoom_block_sum(a, __builtin_amdgcn_readlane((int)pb.fx0, l), __builtin_amdgcn_readlane((int)pb.fy0, l),
                                              a.L.f * (__builtin_amdgcn_readlane(z, l) - a.L.o));
              if (lane == l) vb = (T)t;
            }
            v[i * R0 + r] = mk(va, vb);
          }
      } else {
#pragma unroll
        for (int i = 0; i < NB0; ++i)
#pragma unroll
          for (int r = 0; r < R0; ++r) {
            const int z = first_index<N>(g, i, r);
            v[i * R0 + r] = mk(pa.value_zoom(a, z), pb.value_zoom(a, z));
          }
      }
      // sum of rho^2 of the two pencils (per pencil in the working precision)
      T qa = (T)0, qb = (T)0;
#pragma unroll
      for (int e = 0; e < E; ++e) { qa += v[e].x * v[e].x; qb += v[e].y * v[e].y; }
      m2 += (double)qa + (double)qb;
    } else {
      const T* rho = (const T*)a.rho + ((size_t)(X - a.rho_x0) * N) * N;
#pragma unroll
      for (int i = 0; i < NB0; ++i)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          int z = first_index<N>(g, i, r);
          T ra = rho[(size_t)yA * N + z], rb = rho[(size_t)yB * N + z];
          v[i * R0 + r] = mk(ra, rb);
          m2 += (double)ra * ra + (double)rb * rb;
        }
    }
  } else {
    const long long y = y0 + q;
    if (GEN) {
      Pencil<T> p;
      p.init(a, X, y);
#pragma unroll
      for (int i = 0; i < NB0; ++i)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          const int z = first_index<N>(g, i, r);
          T ra;
          if constexpr (ZOOM && C::threads % 64 == 0) {
            bool bd;
            ra = p.zoom_fast(a, z, bd);
            const int lane = __lane_id();
            for (unsigned long long m = __ballot(bd); m; m &= m - 1) {
              const int l = __builtin_ctzll(m);
              const double t = zoom_block_sum(a, __builtin_amdgcn_readlane((int)p.fx0, l), __builtin_amdgcn_readlane((int)p.fy0, l),
                                              a.L.f * (__builtin_amdgcn_readlane(z, l) - a.L.o));
              if (lane == l) ra = (T)t;
            }
          } else {
            ra = ZOOM ? p.value_zoom(a, z) : p.value1(z);
          }
          v[i * R0 + r] = mk(ra, (T)0);
          m2 += (double)ra * ra;
        }
    } else {
      const cx<T>* rho = (const cx<T>*)a.rho + ((size_t)(X - a.rho_x0) * N) * N;
#pragma unroll
      for (int i = 0; i < NB0; ++i)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          int z = first_index<N>(g, i, r);
          cx<T> e = rho[(size_t)y * N + z];
          v[i * R0 + r] = e;
          m2 += (double)e.x * e.x + (double)e.y * e.y;
        }
    }
  }

  fft_column<T, N, -1>(s, g, tw, v);

  // block sum of rho^2: lane partials through LDS (the barrier is needed by
  // the write-out anyway), then one wavefront sums them in a fixed order
  if (a.mom) red[threadIdx.x] = m2;
  __syncthreads();
  if (a.mom && threadIdx.x < 64) {
    constexpr int W = C::threads < 64 ? C::threads : 64;
    double t = 0.0;
    for (int i = threadIdx.x; i < C::threads; i += 64) t += red[i];
    t = wave_sum<W>(t);
    if (threadIdx.x == 0) {
      a.mom[2 * blockIdx.x] = 0.0;
      a.mom[2 * blockIdx.x + 1] = t;
    }
  }

  cx<T>* Ap = A + ((size_t)(X - a.ax0) * a.nkz) * N + y0;
  // each thread keeps one tile column j and walks kz with a fixed stride
  // (needs at least one thread per column: KS >= 1)
  constexpr int KS = C::threads / TY;
  const int j = threadIdx.x % TY;
  if constexpr (KS < 1 || C::threads % TY != 0) {
    constexpr int NK = C2C ? N : N / 2 + 1;
    for (int idx = threadIdx.x; idx < TY * NK; idx += C::threads) {
      const int jj = idx % TY, kz = idx / TY;
      if (!C2C) {
        const cx<T>* col = sm + (jj >> 1) * PS;
        const cx<T> zk = col[pad(kz)], zm = col[pad((N - kz) & (N - 1))];
        Ap[(size_t)kz * N + jj] = (jj & 1) ? mk((zk.y + zm.y) * (T)0.5, (zm.x - zk.x) * (T)0.5)
                                           : mk((zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5);
      } else {
        Ap[(size_t)kz * N + jj] = sm[jj * PS + pad(kz)];
      }
    }
  } else if (!C2C) {
    // unpack the two real transforms of column p: A_k = (Z_k + conj Z_{N-k}) / 2
    // to tile column 2p, B_k = (Z_k - conj Z_{N-k}) / (2i) to column 2p + 1,
    // k in [0, N/2]; one thread writes both (adjacent) outputs
    constexpr int KP = C::threads / NG;                 // kz stride (>= 1: threads = NG G)
    const int p = threadIdx.x % NG, kz0 = threadIdx.x / NG;
    const cx<T>* col = sm + p * PS;
    cx2<T>* dst = (cx2<T>*)(Ap + (size_t)kz0 * N + 2 * p);
    auto unpack = [](cx<T> zk, cx<T> zm) {
      cx2<T> o;
      o.a = mk((zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5);
      o.b = mk((zk.y + zm.y) * (T)0.5, (zm.x - zk.x) * (T)0.5);
      return o;
    };
    if constexpr (KP % 16 == 0) {
      // kz = kz0 + KP m and N - kz step by multiples of 16: both LDS reads
      // are one padded base plus a compile-time offset
      constexpr int M = (N / 2) / KP, DK = KP + KP / 16;
      const cx<T>* zkb = col + pad(kz0);
      const cx<T>* zmb = col + pad(N - kz0);             // kz0 = 0, m = 0 wraps to Z_0 (below)
#pragma unroll
      for (int m = 0; m < M; ++m, dst += (size_t)KP * N / 2) {
        const cx<T> zk = zkb[m * DK];
        const cx<T> zm = (m == 0 && kz0 == 0) ? col[0] : zmb[-m * DK];
        st_a2(dst, unpack(zk, zm));
      }
      if (kz0 == 0) {                                      // kz = N/2 (self-conjugate)
        const cx<T> zh = col[pad(N / 2)];
        st_a2(dst, unpack(zh, zh));
      }
    } else {
      for (int kz = kz0; kz <= N / 2; kz += KP, dst += (size_t)KP * N / 2)
        st_a2(dst, unpack(col[pad(kz)], col[pad((N - kz) & (N - 1))]));
    }
  } else {
    const cx<T>* col = sm + j * PS;
    cx<T>* dst = Ap + (size_t)(threadIdx.x / TY) * N + j;
    for (int kz = threadIdx.x / TY; kz < N; kz += KS, dst += (size_t)KS * N) *dst = col[pad(kz)];
  }
}

// ED materialisation (tile + mask + zoom) of planes x0, x0 + 1, ... into a
// real [x - x0][y][z] array: one block per pencil, same generator as the z pass.
template <typename T>
__global__ void __launch_bounds__(256) k_rho_generate(ZArgs a, int n, int x0, T* __restrict__ rho) {
  const long long t = blockIdx.x;                 // one block per pencil
  const long long X = x0 + t / n, Y = t % n;
  Pencil<T> p;
  p.init(a, X, Y);
  if (a.ngrain) p.init_grains(a);
  T* row = rho + t * n;
  for (int z = threadIdx.x; z < n; z += 256) row[z] = a.rotated ? p.value_rotated_rt(a, z) : p.value(a, z);
}

// Zoom level of a rotated or polycrystalline lattice (real [x - x0][y][z]
// planes): each level voxel is the sum of the f^3 ED-1 voxels of its block,
// every one generated as the ED-1 generator does (the inside test of the
// fine voxel, then the cell at u = R d with the chosen interpolation),
// summed in FP64 and rounded once.  One block per level pencil (X, Y): the
// f^2 fine pencils of its block column are the same for the whole block, so
// their set-up (inside range, rotated base coordinates) is wave-uniform; the
// threads take the level's z.  Level boxes up to kZoomRotMaxBox.

template <typename T, int INTERP, bool GRAINS>
__global__ void __launch_bounds__(256) k_zoom_rot(ZArgs a, int n, int x0, T* __restrict__ rho) {
  constexpr int KZ = kZoomRotMaxBox / 256;
  __shared__ T cl[4096];                               // the cell, when c^3 <= 4096
  __shared__ double grl[GRAINS ? kMaxGrains * 9 : 1];
  const long long t = blockIdx.x;
  const long long X = x0 + t / n, Y = t % n;
  const Level& Lk = a.L;
  const int f = Lk.f;
  T* row = rho + (size_t)t * n;
  long long clo, chi;
  col_range(Lk, a.m, X, Y, clo, chi);                 // level voxels whose block can hold density
  if (clo > chi) {
    for (int z = threadIdx.x; z < n; z += 256) row[z] = (T)0;
    return;
  }
  const int c3 = Lk.c * Lk.c * Lk.c;
  const bool in_lds = c3 <= 4096;
  if (in_lds)
    for (int i = threadIdx.x; i < c3; i += 256) cl[i] = ((const T*)a.cellT)[i];
  if constexpr (GRAINS)
    for (int i = threadIdx.x; i < 9 * a.ngrain; i += 256) grl[i] = (&a.grot[0][0])[i];
  __syncthreads();
  const T* C = in_lds ? cl : (const T*)a.cellT;
  const Level L1 = make_level(Lk.n1, Lk.n1, 1, Lk.c);
  const long long fx0 = (long long)f * (X - Lk.o), fy0 = (long long)f * (Y - Lk.o);
  double acc[KZ];
#pragma unroll
  for (int k = 0; k < KZ; ++k) acc[k] = 0.0;
  for (int u = 0; u < f; ++u)
    for (int v = 0; v < f; ++v) {
      Pencil<T> p;
      p.init_at(a, L1, fx0 + u, fy0 + v);
      if (p.zlo > p.zhi) continue;                     // block-uniform
      if constexpr (GRAINS) { p.GR = grl; p.init_grains(a); }
#pragma unroll
      for (int k = 0; k < KZ; ++k) {
        const int Z = (int)threadIdx.x + 256 * k;
        if (Z >= n || Z < clo || Z > chi) continue;
        const long long fz0 = (long long)f * (Z - Lk.o);
        if (fz0 + f - 1 < p.zlo || fz0 > p.zhi) continue;
        for (int w = 0; w < f; ++w) {
          const int fz = (int)(fz0 + w);
          if (fz >= p.zlo && fz <= p.zhi) acc[k] += (double)p.template value_rotated<INTERP, GRAINS>(a, fz, C);
        }
      }
    }
#pragma unroll
  for (int k = 0; k < KZ; ++k) {
    const int Z = (int)threadIdx.x + 256 * k;
    if (Z < n) row[Z] = (T)acc[k];
  }
}

// ---------------------------------------------------------------------------
// pass Y: A[x][kz][y] columns -> transform along y -> B[kz][ky][x]
// Each group transforms two x planes of the block's TX-plane tile one after
// the other (results of the first kept in registers), so only TX/2 LDS
// columns are needed and two blocks fit a CU; the transposed write leaves in
// chunks of G rows, every row a TX-element (128-byte) segment.
// ---------------------------------------------------------------------------
// Zero-extended column loads when every wavefront lies in one column (G >= 64), where
// the column address is wave-uniform: a raw buffer resource whose size ends
// at the last valid element makes the hardware return zero beyond it.  No
// branch per element, no masked load.  Two forms (SKIP; tuned per pass:
// UR_LD_SKIP_Y for the y passes, UR_LD_SKIP_X for the x passes):
//  1: the resource starts at element 0; lanes below the first valid element
//     use offset 2^31, which is always out of range, and chunks of G
//     elements wholly outside the range are skipped by a scalar branch (the
//     registers zeroed instead).  Offsets are never negative, so a constant
//     part folded into the instruction offset cannot wrap.
//  0: the resource starts at the first valid element and every chunk is
//     loaded: a lane below it has a negative offset, which as an unsigned
//     number lies far beyond the resource's size; the whole offset is kept
//     in the register (no constant folded into the instruction offset,
//     where the 32-bit sum could wrap back into range).  One integer add per
//     element, no select, no zeroing, no branch.
constexpr unsigned kOutOfRange = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t column_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

// The columns are read once per pass: non-temporal cache policy (aux bit 1).
template <typename T>
__device__ __forceinline__ cx<T> column_ld(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  constexpr int aux = UR_LD_NT ? 2 : 0;                 // non-temporal policy (tuned)
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, aux));
  else return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, aux));
}

// v[i R0 + r] = col[p] for p = g + G i + r N/R0 inside [lo, hi], zero elsewhere
// (col points at element 0; lo, hi and col are wave-uniform; 0 <= lo)
template <typename T, int N, bool SKIP>
__device__ __forceinline__ void load_column_u(const cx<T>* col, int lo, int hi, int g, cx<T>* v) {
  constexpr int G = Geo<N>::G, E = Geo<N>::E, R0 = Radix<N, 1>::r, NB0 = E / R0;
  constexpr unsigned SZ = sizeof(cx<T>);
  if constexpr (SKIP) {
    const __amdgpu_buffer_rsrc_t rs = column_rsrc(col, lo <= hi ? (hi + 1) * (int)SZ : 0);
    const unsigned gb = (unsigned)g * SZ;
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int c = G * i + r * (N / R0);              // compile-time displacement
        if (c + G - 1 < lo || c > hi) {                    // wave-uniform: no load at all
          v[i * R0 + r] = mk((T)0, (T)0);
        } else {
          unsigned o = g >= lo - c ? gb : kOutOfRange;
          asm("" : "+v"(o));   // keeps the constant out of the select: it becomes the instruction offset
          v[i * R0 + r] = column_ld<T>(rs, o + (unsigned)c * SZ);
        }
      }
  } else {
    const __amdgpu_buffer_rsrc_t rs = column_rsrc(col + lo, lo <= hi ? (hi - lo + 1) * (int)SZ : 0);
    const unsigned gb = (unsigned)(g - lo) * SZ;       // wraps below lo
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        unsigned o = gb + (unsigned)(G * i + r * (N / R0)) * SZ;
        asm("" : "+v"(o));                                 // the whole offset stays in the register
        v[i * R0 + r] = column_ld<T>(rs, o);
      }
  }
}

template <typename T, int N>
__device__ __forceinline__ void y_load_column(const YArgs& a, long long X, int kz, int g, cx<T>* v) {
  constexpr int G = Geo<N>::G, E = Geo<N>::E, R0 = Radix<N, 1>::r, NB0 = E / R0;
  long long ylo = 0, yhi = N - 1;
  if (X < a.xlo || X > a.xhi) { ylo = 1; yhi = 0; }
  else if (a.gen) {
    row_range(a.L, a.m, X, ylo, yhi);
    // widen to whole z-pass tiles (the tile height is a power of two)
    if (ylo <= yhi) { ylo &= ~(long long)(a.ty - 1); yhi |= (long long)(a.ty - 1); }
  }
  const cx<T>* col = (const cx<T>*)a.A + ((size_t)(X - a.ax0) * a.nkz + kz) * N;
  if constexpr (G >= 64) {
    load_column_u<T, N, UR_LD_SKIP_Y>(col, (int)ylo, (int)yhi, g, v);
  } else {
    const int lo = (int)ylo, hi = (int)yhi;
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int y = first_index<N>(g, i, r);
        v[i * R0 + r] = (y >= lo && y <= hi) ? col[y] : mk((T)0, (T)0);
      }
  }
}

template <typename T, int N>
__global__ void __launch_bounds__((YCfg<T, N>::threads), MinW<T>::v)
k_pass_y(YArgs a) {
  using C = YCfg<T, N>;
  constexpr int G = C::G, TX = C::TX, NS = C::NS, E = Geo<N>::E, PS = CS<N>::v;
  constexpr int SS = NS + 1;                               // staging row stride
  __shared__ cx<T> sm[NS * PS + G * SS];
  cx<T>* stg = sm + NS * PS;

  // x tile fastest: the blocks resident at one time cover whole B rows
  // (one kz, all x tiles), so their 128-byte row segments are contiguous
  const int xt = a.xt0 + blockIdx.x % a.nxt;
  const int kz = a.kz0 + blockIdx.x / a.nxt;
  const int xbase = xt * TX;
  // G >= 64: every wavefront lies in one group, the plane index is
  // wave-uniform and the row range of the plane is computed on the scalar unit
  const int q = G >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / G) : threadIdx.x / G;
  const int g = threadIdx.x % G;
  const cx<T>* tw = (const cx<T>*)a.tw;
  cx<T>* s = sm + q * PS;
  cx<T> keep[E];
  {
    cx<T> v[E];
    y_load_column<T, N>(a, xbase + q, kz, g, v);
    fft_column<T, N, -1>(s, g, tw, v);
    // component-wise copies: a whole-struct copy between LDS and the register
    // array becomes a memory copy that keeps the FP64 array out of registers
    if constexpr (G % 16 == 0) {
      const cx<T>* kp = s + pad(g);
#pragma unroll
      for (int t = 0; t < E; ++t) keep[t] = mk(kp[t * (G + G / 16)].x, kp[t * (G + G / 16)].y);   // rows g + G t
    } else {
#pragma unroll
      for (int t = 0; t < E; ++t) keep[t] = mk(s[pad(g + G * t)].x, s[pad(g + G * t)].y);
    }
    col_sync<G>();
    y_load_column<T, N>(a, xbase + NS + q, kz, g, v);
    fft_column<T, N, -1>(s, g, tw, v);
  }
  __syncthreads();
  cx<T>* Bp = (cx<T>*)a.B + ((size_t)(kz - a.kz0) * N) * a.bs + (xbase - a.bx0);
  constexpr int RS = C::threads / TX;                      // rows per pass of the block
  if constexpr (G % 16 == 0 && RS % 16 == 0 && (G * TX) % C::threads == 0) {
    // thread = (plane j, row r0 + k RS of the chunk): one LDS base and one
    // global base per thread, compile-time offsets per (chunk, k)
    const int j = threadIdx.x % TX, r0 = threadIdx.x / TX;
    const bool from_stg = j < NS;
    const cx<T>* src = from_stg ? stg + r0 * SS + j : sm + (j - NS) * PS + pad(r0);
    // rows G t + k RS are visited in increasing order: one running pointer
    cx<T>* dst = Bp + (size_t)r0 * a.bs + j;
    const size_t rstep = (size_t)RS * a.bs;
    static_for<0, E>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      stg[g * SS + q].x = keep[t].x;                       // row ky = g + G t, plane q
      stg[g * SS + q].y = keep[t].y;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < G / RS; ++k, dst += rstep) {
        const int off = from_stg ? k * RS * SS : t * (G + G / 16) + k * (RS + RS / 16);
        st_b(dst, src[off]);
      }
      __syncthreads();
    });
  } else {
    static_for<0, E>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      stg[g * SS + q].x = keep[t].x;                       // row ky = g + G t, plane q
      stg[g * SS + q].y = keep[t].y;
      __syncthreads();
      for (int idx = threadIdx.x; idx < G * TX; idx += C::threads) {
        const int j = idx % TX, r = idx / TX, ky = G * t + r;
        Bp[(size_t)ky * a.bs + j] = j < NS ? stg[r * SS + j] : sm[(j - NS) * PS + pad(ky)];
      }
      __syncthreads();
    });
  }
}

// ---------------------------------------------------------------------------
// binning helpers: thresholds U[0..nbins] in LDS; bin b holds U[b] <= n2 < U[b+1]
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bin_search(const int* U, int nbins, long long n2) {
  if (n2 < U[0]) return -1;
  if (n2 >= U[nbins]) return nbins;
  int lo = 0, hi = nbins;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if ((long long)U[mid] <= n2) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int bin_advance(const int* U, int nbins, int b, long long n2) {
  while (b < nbins && n2 >= (long long)U[b + 1]) ++b;
  return b;
}

// ---------------------------------------------------------------------------
// pass X: B columns -> transform along x -> |F|^2 -> bins (or store)
// Persistent blocks sized to the resident count; after each column FFT a
// group issues the loads of its next column, which stay in flight while it
// bins the current one.  The LDS
// histogram holds sum w I and sum w I^2 per bin (the voxel counts are pure
// geometry, computed once per bin set).
// ---------------------------------------------------------------------------
template <typename T, int N>
__device__ __forceinline__ void x_load_column(const XArgs& a, long long col, int g, cx<T>* v) {
  constexpr int G = Geo<N>::G, E = Geo<N>::E, R0 = Radix<N, 1>::r, NB0 = E / R0;
  const cx<T>* src = (const cx<T>*)a.B + (size_t)col * a.bs - a.bx0;   // element x = 0
  if constexpr (G >= 64) {
    load_column_u<T, N, UR_LD_SKIP_X>(src, a.xa, a.xb, g, v);
  } else {
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int x = first_index<N>(g, i, r);
        v[i * R0 + r] = (x >= a.xa && x <= a.xb) ? src[x] : mk((T)0, (T)0);
      }
  }
}

template <typename T, int N, int MODE, int DIR>
__global__ void __launch_bounds__((XCfg<N>::threads), XMinW<T>::v)
k_pass_x(XArgs a) {
  using C = XCfg<N>;
  // every wavefront reads only its own column: no bank skew between columns
  // is needed, the column stride is the padded length itself (this keeps
  // the FP64 block within the LDS of two blocks per CU)
  constexpr int G = C::G, NG = C::NG, E = Geo<N>::E, PS = Padded<N>::size;
  constexpr bool SINC = MODE == X_FFT_BIN_SINC || MODE == X_BIN_ONLY_SINC;
  constexpr bool BINONLY = MODE == X_BIN_ONLY || MODE == X_BIN_ONLY_SINC;
  __shared__ cx<T> sm[NG * PS];
  extern __shared__ double dyn[];
  // hist[2 b], hist[2 b + 1] for b in [-1, nbins]: the two outer slots take
  // the runs below the first and above the last threshold (discarded)
  double* hist = dyn + 2;
  double* tot_s = dyn + 2 * ((size_t)a.nbins + 2);
  int* U = (int*)(tot_s + 1);                          // nbins + 3 (last two: sentinels)
  short* Ls = (short*)(U + a.nbins + 3);               // nlut: bin of n2 = s^2
  // SINC: voxel form factor S(|m|) for |m| in [0, N/2], 16-byte aligned after Ls
  T* St = (T*)((char*)dyn + ((((char*)(Ls + a.nlut) - (char*)dyn) + 15) & ~(size_t)15));

  // G >= 64: every wavefront lies in one column, wave-uniform column index.
  // For G > 64 the column syncs are workgroup barriers: the launcher makes
  // the number of columns a multiple of NG, so every group of a block runs
  // the same iterations.
  const int q = G >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / G) : threadIdx.x / G;
  const int g0 = threadIdx.x % G;
  cx<T>* s = sm + q * PS;
  const cx<T>* tw = (const cx<T>*)a.tw;
  constexpr bool BIN = MODE != X_FFT_STORE;

  if (BIN) {
    for (int i = threadIdx.x; i < 2 * (a.nbins + 2) + 1; i += C::threads) dyn[i] = 0.0;
    for (int i = threadIdx.x; i <= a.nbins; i += C::threads) U[i] = a.U[i];
    for (int i = threadIdx.x; i < a.nlut; i += C::threads) Ls[i] = a.lut[i];
    if constexpr (SINC)
      for (int i = threadIdx.x; i <= N / 2; i += C::threads) St[i] = ((const T*)a.sinc)[i];
    if (threadIdx.x == 0) { U[a.nbins + 1] = 0x7fffffff; U[a.nbins + 2] = 0x7fffffff; }
    __syncthreads();
  }
  const long long stride = (long long)gridDim.x * NG;
  long long col = (long long)blockIdx.x * NG + q;
  cx<T> v[E];
  if (!BINONLY && col < a.ncols) x_load_column<T, N>(a, col, g0, v);
  for (; col < a.ncols; col += stride) {
    // UR_X_REFETCH: the lane index is opaque in every column, so that the
    // lane's twiddles and LDS offsets are reloaded and recomputed per column
    // instead of held in registers across the loop
    int g = g0;
    if constexpr (UR_X_REFETCH) asm volatile("" : "+v"(g));
    const int kz = a.kz0 + (int)(col / N), ky = (int)(col % N);
    if (BINONLY) {
      const cx<T>* src = (const cx<T>*)a.B + (size_t)col * a.bs - a.bx0;
      for (int i = g; i < N; i += G) s[pad(i)] = (i >= a.xa && i <= a.xb) ? src[i] : mk((T)0, (T)0);
      col_sync<G>();
    } else {
      fft_column<T, N, DIR>(s, g, tw, v);
      if (col + stride < a.ncols) x_load_column<T, N>(a, col + stride, g, v);   // in flight during the binning
    }
    if (!BIN) {
      cx<T>* dst = (cx<T>*)a.out + (size_t)col * N;
      for (int i = g; i < N; i += G) dst[i] = scale(s[pad(i)], (T)a.oscale);
      col_sync<G>();
      continue;
    }
    // |F|^2 and bins. Lane g walks |h| over its own range in increasing
    // order, so n2 and the bin index never decrease along the walk.
    const int k = sidx(ky, N);
    const int l = a.r2c ? kz : sidx(kz, N);
    const int base = k * k + l * l;
    // lane g owns |h| in [hlo, hlo + NH) (both signs), the last lane also
    // |h| = N/2; NH consecutive |h| stay inside one 16-element LDS block.
    // Within a run of equal bins, |X|^2 and |X|^4 of the working-precision
    // values are both summed in FP64, so that a bin's sum and sum of squares
    // describe the same numbers (the one-pass variance of the finalize
    // subtracts them; a bin whose intensities barely vary would lose its SEM
    // to the rounding of a working-precision run sum).  The LDS histogram
    // holds the sums relative to the common column weight wref (2 for a real
    // transform: the conjugate half counted twice), so most columns flush
    // their runs unscaled; wref and the scale 1/n^6 of eq. 1 are applied once
    // per block when the partials are written.
    constexpr int NH = G == 1 ? N / 2 : E / 2;
    const int hlo = G == 1 ? 0 : g * NH;
    // starting bin: the table entry of s = isqrt(n2) (the bin of s^2 <= n2),
    // then forward over the few thresholds between s^2 and n2
    const int n20 = hlo * hlo + base;
    int sq = (int)sqrtf((float)n20);
    if (sq * sq > n20) --sq;
    else if ((sq + 1) * (sq + 1) <= n20) ++sq;
    int b = Ls[sq];
    int nextU = U[b + 1];
    while (n20 >= nextU) { ++b; nextU = U[b + 1]; }
    int nextU2 = U[b + 2];                               // one threshold ahead, off the critical path
    int cb = b;
    double cs = 0.0, cs2 = 0.0;
    // this column's weight relative to wref: 1/2 at kz = 0 and N/2 of a real
    // transform; SINC: times S(|k|) S(|l|) (S(|h|) is applied per voxel)
    const double wcol = SINC ? (double)St[k < 0 ? -k : k] * (double)St[l < 0 ? -l : l] : 1.0;
    const double wr = (a.r2c && (kz == 0 || kz == N / 2)) ? 0.5 : 1.0;
    const double ws = wr * wcol, ws2 = wr * wcol * wcol;
    const bool unit = !SINC && wr == 1.0;
    const cx<T>* sp = s + pad(hlo);
    // the lane's intensities first, in one batch of LDS reads: |F|^2 at +|h|
    // and -|h| for its NH values of |h| (nothing at -0), so the walk below
    // runs on registers
    T qp[NH], qm[NH];
#pragma unroll
    for (int t = 0; t < NH; ++t) {
      const int ha = hlo + t;
      const cx<T> f1 = (NH <= 16 || G == 1) ? sp[t + (G == 1 ? (t >> 4) : 0)] : s[pad(ha)];
      const cx<T> f2 = s[pad((N - ha) & (N - 1))];       // ha = 0 reads F(0) again; weighted out below
      qp[t] = f1.x * f1.x + f1.y * f1.y;
      qm[t] = ha != 0 ? f2.x * f2.x + f2.y * f2.y : (T)0;
    }
    auto flush = [&]() {
      if (unit) {
        atomicAdd(&hist[2 * cb + 0], cs);
        atomicAdd(&hist[2 * cb + 1], cs2);
      } else {
        atomicAdd(&hist[2 * cb + 0], cs * ws);
        atomicAdd(&hist[2 * cb + 1], cs2 * ws2);
      }
    };
    auto take = [&](int ha, T q1, T q2) {
      if constexpr (SINC) { const T sh = St[ha]; q1 *= sh; q2 *= sh; }
      const int n2 = ha * ha + base;
      if (n2 >= nextU) {
        flush();
        cs = 0.0;
        cs2 = 0.0;
        ++b;
        nextU = nextU2;
        while (n2 >= nextU) { ++b; nextU = U[b + 1]; }     // several thresholds at once (rare)
        nextU2 = U[b + 2];
        cb = b;
      }
      // the squares of working-precision values are exact in FP64
      const double d1 = (double)q1, d2 = (double)q2;
      cs += d1 + d2;
      cs2 = fma(d1, d1, cs2);
      cs2 = fma(d2, d2, cs2);
    };
#pragma unroll
    for (int t = 0; t < NH; ++t) take(hlo + t, qp[t], qm[t]);
    if (g == G - 1) {                                      // |h| = N/2 (kx = N/2 only)
      const cx<T> f1 = s[pad(N / 2)];
      take(N / 2, f1.x * f1.x + f1.y * f1.y, (T)0);
    }
    flush();
    if (kz == 0 && ky == 0 && g == 0 && a.f0) {
      const cx<T> f = s[pad(0)];
      a.f0[0] = (double)f.x * sqrt(a.iscale);
      a.f0[1] = (double)f.y * sqrt(a.iscale);
    }
    col_sync<G>();
  }
  if (!BIN) return;
  __syncthreads();
  // every run went to one slot (the two outer slots included): the block's
  // total is the sum of the slots, taken in a fixed order by one wavefront
  const double wref = a.r2c ? 2.0 : 1.0, s1 = wref * a.iscale, s2 = wref * a.iscale * a.iscale;
  if (threadIdx.x < 64) {
    double t = 0.0;
    for (int i = (int)threadIdx.x - 1; i <= a.nbins; i += 64) t += hist[2 * i];
    t = wave_sum(t);
    if (threadIdx.x == 0) *tot_s = t;
  }
  __syncthreads();
  double* out = a.part + (size_t)blockIdx.x * (2 * (size_t)a.nbins + 1);
  for (int i = threadIdx.x; i < 2 * a.nbins + 1; i += C::threads) {
    const double v = i < 2 * a.nbins ? hist[i] * ((i & 1) ? s2 : s1) : *tot_s * s1;
    out[i] = a.accum ? out[i] + v : v;
  }
}

#if UR_IN(0)
// voxel count per bin (geometry only): one thread per (ky, kz) column walks
// |h| upward; integer LDS histogram, integer global totals
__global__ void __launch_bounds__(256) k_bin_counts(int n, int nkz, int r2c, int nbins, const int* __restrict__ Ug,
                                                    unsigned long long* __restrict__ out) {
  extern __shared__ unsigned long long hc[];
  int* U = (int*)(hc + nbins);
  for (int i = threadIdx.x; i < nbins; i += 256) hc[i] = 0ull;
  for (int i = threadIdx.x; i <= nbins; i += 256) U[i] = Ug[i];
  if (threadIdx.x == 0) U[nbins + 1] = 0x7fffffff;
  __syncthreads();
  const long long col = (long long)blockIdx.x * 256 + threadIdx.x;
  if (col < (long long)nkz * n) {
    const int kz = (int)(col / n), ky = (int)(col % n);
    const int k = sidx(ky, n), l = r2c ? kz : sidx(kz, n);
    const unsigned long long w = (r2c && kz != 0 && kz != n / 2) ? 2ull : 1ull;
    const int base = k * k + l * l;
    int b = bin_search(U, nbins, base);
    int nextU = U[b + 1];
    unsigned long long acc = 0ull;
    for (int ha = 0; ha <= n / 2; ++ha) {
      const int n2 = ha * ha + base;
      if (n2 >= nextU) {
        if (b >= 0 && b < nbins && acc) atomicAdd(&hc[b], acc);
        acc = 0ull;
        do { ++b; nextU = U[b + 1]; } while (n2 >= nextU);
      }
      acc += w * ((ha == 0 || ha == n / 2) ? 1ull : 2ull);
    }
    if (b >= 0 && b < nbins && acc) atomicAdd(&hc[b], acc);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbins; i += 256)
    if (hc[i]) atomicAdd(&out[i], hc[i]);
}

__global__ void k_counts_to_double(int nbins, const unsigned long long* __restrict__ c, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbins) out[i] = (double)c[i];
}

#endif
// ---------------------------------------------------------------------------
// finalize: fixed-order compensated sums over the block partials
// ---------------------------------------------------------------------------
struct Kahan {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v; else c += (v - t) + s;
    s = t;
  }
  __device__ __forceinline__ double val() const { return s + c; }
};

#if UR_IN(0)
// block b < nvb: 8 values x 32 phases; the last block reduces the z-pass
// moments and copies the (geometric) bin counts
__global__ void __launch_bounds__(256) k_finalize(FinArgs a) {
  __shared__ double ls[256], lc[256], fin[8];
  const int nv = 2 * a.nbins + 1;
  const int nvb = (nv + 7) / 8;
  const int t = threadIdx.x;
  if ((int)blockIdx.x < nvb) {
    const int vv = t % 8, p = t / 8;
    const int v = blockIdx.x * 8 + vv;
    Kahan k;
    if (v < nv) {
      int w = p;
      for (; w + 3 * 32 < a.nblk; w += 4 * 32) {
        double x0 = a.part[(size_t)w * nv + v];
        double x1 = a.part[(size_t)(w + 32) * nv + v];
        double x2 = a.part[(size_t)(w + 64) * nv + v];
        double x3 = a.part[(size_t)(w + 96) * nv + v];
        k.add(x0); k.add(x1); k.add(x2); k.add(x3);
      }
      for (; w < a.nblk; w += 32) k.add(a.part[(size_t)w * nv + v]);
    }
    ls[t] = k.s;
    lc[t] = k.c;
    __syncthreads();
    if (p == 0 && v < nv) {
      Kahan r;
      for (int pp = 0; pp < 32; ++pp) { r.add(ls[pp * 8 + vv]); r.add(lc[pp * 8 + vv]); }
      double val = r.val();
      fin[vv] = val;
      if (v == nv - 1) {
        a.totals[0] = val;
        a.totals[1] = a.f0 ? a.f0[0] : 0.0;
        a.totals[2] = a.f0 ? a.f0[1] : 0.0;
      } else {
        (v % 2 == 0 ? a.sum : a.sumsq)[v / 2] = val;
      }
    }
    // mean and standard error of the mean of bin v/2: its sum and sum of
    // squares (v, v + 1) were reduced by this block (8 values per block)
    __syncthreads();
    if ((a.mean || a.sem) && p == 0 && vv % 2 == 0 && v + 1 < nv) {
      const int b = v / 2;
      const double c = a.cnt[b], S = fin[vv], S2 = fin[vv + 1];
      const double m = c > 0.0 ? S / c : __builtin_nan("");
      double se = __builtin_nan("");
      if (c > 1.0) {
        const double ss = S2 - S * m;                    // sum of (I - mean)^2
        se = sqrt((ss > 0.0 ? ss : 0.0) / (c - 1.0) / c);
      }
      if (a.mean) a.mean[b] = m;
      if (a.sem) a.sem[b] = se;
    }
  } else {
    for (int i = t; i < a.nbins; i += 256) a.count[i] = a.cnt[i];
    // sum of rho^2 over the z-pass blocks, beside the blocks reducing the
    // bins: up to kFoldMoments blocks thread t takes blocks t, t + 256, ...
    // (eight compensated sums, eight loads in flight), above that the 256
    // first-level partials of k_moments; then thread 0 adds the 256 partials
    // in order
    Kahan k;
    if (a.mom && a.nzb > kFoldMoments) {
      k.add(a.mpart[t]);
    } else if (a.mom) {
      Kahan kk[8];
      int i = t;
      for (; i + 7 * 256 < a.nzb; i += 8 * 256) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = a.mom[2 * (size_t)(i + u * 256) + 1];
#pragma unroll
        for (int u = 0; u < 8; ++u) kk[u].add(x[u]);
      }
      for (; i < a.nzb; i += 256) kk[0].add(a.mom[2 * (size_t)i + 1]);
#pragma unroll
      for (int u = 0; u < 8; ++u) { k.add(kk[u].s); k.add(kk[u].c); }
    }
    ls[t] = k.s;
    lc[t] = k.c;
    __syncthreads();
    if (t == 0) {
      Kahan r;
      for (int i = 0; i < 256; ++i) { r.add(ls[i]); r.add(lc[i]); }
      a.totals[3] = a.mom ? r.val() : 0.0;
    }
  }
}

// first level of the sum of rho^2 over many z-pass blocks: block b reduces a
// contiguous chunk of the per-block moments in a fixed order
__global__ void __launch_bounds__(256) k_moments(const double* __restrict__ mom, int nzb, double* __restrict__ mpart) {
  __shared__ double ls[256], lc[256];
  const int chunk = (nzb + gridDim.x - 1) / gridDim.x;
  const int lo = blockIdx.x * chunk, hi = min(nzb, lo + chunk);
  Kahan k;
  for (int i = lo + threadIdx.x; i < hi; i += 256) k.add(mom[2 * (size_t)i + 1]);
  ls[threadIdx.x] = k.s;
  lc[threadIdx.x] = k.c;
  __syncthreads();
  if (threadIdx.x == 0) {
    Kahan r;
    for (int i = 0; i < 256; ++i) { r.add(ls[i]); r.add(lc[i]); }
    mpart[blockIdx.x] = r.val();
  }
}

#endif
// ---------------------------------------------------------------------------
// merge of zoom levels, one thread per bin
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sem_from_sums(double cnt, double s, double s2) {
  if (!(cnt > 1.0)) return NAN;
  double var = (s2 - s * s / cnt) / (cnt - 1.0);
  if (var < 0.0) var = 0.0;
  return sqrt(var / cnt);
}

#if UR_IN(0)
__global__ void k_merge(MergeArgs a) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.nbins) return;
  double lo = a.edges[b], hi = a.edges[b + 1];
  double qc = lo > 0.0 ? sqrt(fabs(lo * hi)) : 0.5 * (lo + hi);
  int valid[8];
  int nv = 0;
  for (int i = 0; i < a.nlevels; ++i) {
    int k = a.order[i];
    if (a.dq[k] <= qc && qc <= a.qcut[k] && a.count[k][b] >= a.n_min) valid[nv++] = k;
  }
  double mean = NAN, sem = NAN;
  int owner = -1;
  if (nv > 0) {
    if (a.mode == 0) {
      int k = valid[0];
      double s = a.scale[k], cnt = a.count[k][b];
      mean = s * a.sum[k][b] / cnt;
      sem = s * sem_from_sums(cnt, a.sum[k][b], a.sumsq[k][b]);
      owner = k;
    } else if (a.mode == 1) {
      double Cn = 0.0, S1 = 0.0, S2 = 0.0;
      for (int i = 0; i < nv; ++i) {
        int k = valid[i];
        double s = a.scale[k];
        Cn += a.count[k][b];
        S1 += s * a.sum[k][b];
        S2 += s * s * a.sumsq[k][b];
      }
      mean = S1 / Cn;
      sem = sem_from_sums(Cn, S1, S2);
      owner = nv;
    } else {
      double W = 0.0, WM = 0.0;
      for (int i = 0; i < nv; ++i) {
        int k = valid[i];
        double s = a.scale[k], cnt = a.count[k][b];
        double m = s * a.sum[k][b] / cnt;
        double e = s * sem_from_sums(cnt, a.sum[k][b], a.sumsq[k][b]);
        if (!(e > 0.0) || !isfinite(e)) continue;
        W += 1.0 / (e * e);
        WM += m / (e * e);
      }
      if (W > 0.0) { mean = WM / W; sem = 1.0 / sqrt(W); owner = nv; }
    }
  }
  a.mean[b] = mean;
  a.sem[b] = sem;
  a.owner[b] = owner;
}

// Ensemble of boxes that share a bin set (one particle each, incoherent sum
// with number weights w): per bin, mean = sum_k w_k mean_k and
// sem = sqrt(sum_k (w_k sem_k)^2), compensated sums in box order.  One
// thread per bin; mean and sem are [box][bin].
__global__ void __launch_bounds__(256) k_ensemble(int nboxes, int nbins, const double* __restrict__ mean,
                                                   const double* __restrict__ sem, const double* __restrict__ w,
                                                   double* __restrict__ out_mean, double* __restrict__ out_sem) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  Kahan m, v;
  for (int k = 0; k < nboxes; ++k) {
    const double wk = w[k];
    m.add(wk * mean[(size_t)k * nbins + b]);
    const double e = wk * sem[(size_t)k * nbins + b];
    v.add(e * e);
  }
  out_mean[b] = m.val();                   // NaN where the bin is empty (every box)
  out_sem[b] = sqrt(v.val());              // NaN for one-voxel bins
}

// chi^2 of a binned curve against a target and its gradient per bin, one
// block: thread t takes bins t, t + 256, ... in order (compensated), then a
// fixed-order tree over the 256 partials, so the sum does not depend on
// timing.  Empty bins (count 0) take no part and get a zero gradient.
__global__ void __launch_bounds__(256) k_chi2(int nbins, const double* __restrict__ mean,
                                              const double* __restrict__ count, const double* __restrict__ target,
                                              double rel_sigma, double* __restrict__ out, double* __restrict__ g) {
  __shared__ double ps[256], pc[256];
  Kahan k;
  for (int b = threadIdx.x; b < nbins; b += 256) {
    double gb = 0.0;
    if (count[b] > 0.0) {
      const double sg = rel_sigma * target[b];
      const double r = (mean[b] - target[b]) / sg;
      k.add(r * r);
      gb = 2.0 * r / sg;                     // d (r^2) / d mean_b
    }
    if (g) g[b] = gb;
  }
  ps[threadIdx.x] = k.s;
  pc[threadIdx.x] = k.c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      Kahan m;
      m.s = ps[threadIdx.x];
      m.c = pc[threadIdx.x];
      m.add(ps[threadIdx.x + w]);
      m.c += pc[threadIdx.x + w];
      ps[threadIdx.x] = m.s;
      pc[threadIdx.x] = m.c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = ps[0] + pc[0];
}

#endif
// ---------------------------------------------------------------------------
// adjoint column pass along x: FFT_x, multiply by G(|q|) * gscale, IFFT_x
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__((XCfg<N>::threads))
k_pass_x_adj(XAdjArgs a) {
  using C = XCfg<N>;
  constexpr int G = C::G, NG = C::NG, E = Geo<N>::E;
  constexpr int R0 = Radix<N, 1>::r, NB0 = E / R0, PS = CS<N>::v;
  __shared__ cx<T> sm[NG * PS];
  extern __shared__ double dyn[];
  // G(b) for b in [-1, nbins] (the two outer slots are zero), thresholds with
  // a sentinel, and the start-of-walk table of the bins (as in the x pass)
  double* Gb = dyn + 1;
  int* U = (int*)(dyn + a.nbins + 2);                 // nbins + 2
  short* Ls = (short*)(U + a.nbins + 2);              // nlut
  for (int i = threadIdx.x; i < a.nbins + 2; i += C::threads) {
    const int b = i - 1;
    dyn[i] = (b >= 0 && b < a.nbins && a.count[b] > 0.0) ? a.g_bin[b] / a.count[b] * a.gscale : 0.0;
  }
  for (int i = threadIdx.x; i <= a.nbins; i += C::threads) U[i] = a.U[i];
  for (int i = threadIdx.x; i < a.nlut; i += C::threads) Ls[i] = a.lut[i];
  if (threadIdx.x == 0) U[a.nbins + 1] = 0x7fffffff;
  __syncthreads();
  const int q = G >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / G) : threadIdx.x / G;
  const int g0 = threadIdx.x % G;
  cx<T>* s = sm + q * PS;
  const cx<T>* tw = (const cx<T>*)a.tw;

  // After its forward transform a group issues the loads of its next column,
  // which stay in flight during the weighting, the inverse transform and
  // the write-back of the current one.
  auto load = [&](long long c, cx<T>* v, int g) {
    const cx<T>* src = (const cx<T>*)a.B + (size_t)c * a.bs - a.bx0;
    if constexpr (G >= 64) {
      load_column_u<T, N, UR_LD_SKIP_X>(src, a.xa, a.xb, g, v);
    } else {
#pragma unroll
      for (int i = 0; i < NB0; ++i)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          int x = first_index<N>(g, i, r);
          v[i * R0 + r] = (x >= a.xa && x <= a.xb) ? src[x] : mk((T)0, (T)0);
        }
    }
  };
  const long long stride = (long long)gridDim.x * NG;
  long long col = (long long)blockIdx.x * NG + q;
  cx<T> v[E];
  if (col < a.ncols) load(col, v, g0);
  for (; col < a.ncols; col += stride) {
    // UR_XADJ_REFETCH: the lane index is opaque in every column, so the
    // twiddles of both transforms and the LDS offsets are reloaded and
    // recomputed per column instead of held in registers across the loop
    // (1024 points FP32: 126 VGPRs instead of 153, four blocks per CU)
    int g = g0;
    if constexpr (UR_XADJ_REFETCH) asm volatile("" : "+v"(g));
    const int kz = (int)(col / N), ky = (int)(col % N);
    cx<T>* src = (cx<T>*)a.B + (size_t)col * a.bs - a.bx0;
    fft_column<T, N, -1>(s, g, tw, v);
    if (col + stride < a.ncols) load(col + stride, v, g);
    const int k = sidx(ky, N);
    const int l = a.r2c ? kz : sidx(kz, N);
    const int base = k * k + l * l;
    // lane g owns |h| in [hlo, hlo + NH) (both signs), the last lane also
    // |h| = N/2; the bin walk starts from the table entry of isqrt(n2)
    constexpr int NH = G == 1 ? N / 2 : E / 2;
    const int hlo = G == 1 ? 0 : g * NH;
    const int n20 = hlo * hlo + base;
    int sq = (int)sqrtf((float)n20);
    if (sq * sq > n20) --sq;
    else if ((sq + 1) * (sq + 1) <= n20) ++sq;
    int b = Ls[sq];
    int nextU = U[b + 1];
    while (n20 >= nextU) { ++b; nextU = U[b + 1]; }
    // the weight is rounded to the working precision once per bin
    T gv = (T)Gb[b];
    cx<T>* sp = s + pad(hlo);
    // intensity weight of the forward binning (voxel form factor): the
    // gradient of w |F|^2 is w times that of |F|^2, so each element's factor
    // is G(b) S(|k|) S(|l|) S(|h|); the column part is taken in FP64 as in
    // the forward pass, once per column
    const T* Sw = (const T*)a.sinc;
    const T wc = Sw ? (T)((double)Sw[k < 0 ? -k : k] * (double)Sw[l < 0 ? -l : l]) : (T)1;
    auto weigh = [&](auto wt) {
      constexpr bool WT = decltype(wt)::value;
#pragma unroll
      for (int t = 0; t < NH; ++t) {
        const int ha = hlo + t;
        const int n2 = ha * ha + base;
        while (n2 >= nextU) { ++b; nextU = U[b + 1]; gv = (T)Gb[b]; }
        const T ge = WT ? gv * wc * Sw[ha] : gv;
        cx<T>* p1 = (NH <= 16 || G == 1) ? sp + t + (G == 1 ? (t >> 4) : 0) : s + pad(ha);
        const cx<T> f = *p1;
        *p1 = mk(f.x * ge, f.y * ge);
        if (ha != 0) {
          const cx<T> f2 = s[pad(N - ha)];
          s[pad(N - ha)] = mk(f2.x * ge, f2.y * ge);
        }
      }
      if (g == G - 1) {                                    // |h| = N/2 (kx = N/2 only)
        const int n2 = (N / 2) * (N / 2) + base;
        while (n2 >= nextU) { ++b; nextU = U[b + 1]; gv = (T)Gb[b]; }
        const T ge = WT ? gv * wc * Sw[N / 2] : gv;
        const cx<T> f = s[pad(N / 2)];
        s[pad(N / 2)] = mk(f.x * ge, f.y * ge);
      }
    };
    if (Sw) weigh(std::integral_constant<bool, true>{});
    else weigh(std::integral_constant<bool, false>{});
    col_sync<G>();
    stages_from<T, N, 1, +1>(s, g, tw);
    for (int i = a.oa + g; i <= a.ob; i += G) src[i] = s[pad(i)];
    col_sync<G>();
  }
}

// ---------------------------------------------------------------------------
// inverse pass Y: B[kz][ky][x] -> inverse transform along y -> A[x][kz][y]
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__((YICfg<T, N>::threads))
k_pass_y_inv(YInvArgs a) {
  using C = YICfg<T, N>;
  constexpr int G = C::G, TX = C::TX, PS = CS<N>::v;
  __shared__ cx<T> sm[TX * PS];
  // x tile fastest: the blocks resident together read whole B rows
  const int xt = a.xt0 + blockIdx.x % a.nxt;
  const int kz = blockIdx.x / a.nxt;
  const int xbase = xt * TX;
  const cx<T>* Bp = (const cx<T>*)a.B + ((size_t)kz * N) * a.bs + (xbase - a.bx0);
  // transposed read of the tile: all loads of a thread are issued before
  // its LDS stores (a load-store loop would wait on every load in turn)
  {
    constexpr int IT = TX * N / C::threads;
    static_assert(IT * C::threads == TX * N, "the tile is a whole number of block sweeps");
    T rx[IT], ry[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int idx = threadIdx.x + k * C::threads, j = idx % TX, ky = idx / TX;
      const cx<T> e = Bp[(size_t)ky * a.bs + j];
      rx[k] = e.x;
      ry[k] = e.y;
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int idx = threadIdx.x + k * C::threads, j = idx % TX, ky = idx / TX;
      sm[j * PS + pad(ky)].x = rx[k];
      sm[j * PS + pad(ky)].y = ry[k];
    }
  }
  __syncthreads();
  const int q = threadIdx.x / G, g = threadIdx.x % G;
  cx<T>* s = sm + q * PS;
  stages_from<T, N, 1, +1>(s, g, (const cx<T>*)a.tw);
  cx<T>* col = (cx<T>*)a.A + ((size_t)(xbase + q) * a.nkz + kz) * N;
  int ylo = 0, yhi = N - 1;
  if (a.rows) {
    long long lo, hi;
    row_range(a.L, a.m, xbase + q, lo, hi);
    ylo = lo <= hi ? (int)(lo & ~(long long)(a.ty - 1)) : 1;
    yhi = lo <= hi ? (int)(hi | (long long)(a.ty - 1)) : 0;
  }
  for (int i = ylo + g; i <= yhi; i += G) col[i] = s[pad(i)];
}

// ---------------------------------------------------------------------------
// inverse pass Z: A[x][kz][y] -> inverse transform along z -> real (c2r) or
// complex box [x][y][z], times `scale`; optionally only a plane range and,
// within each plane, the y tiles that meet the particle's rows (the pencils
// an amplitude fold reads; the others are left unwritten)
// ---------------------------------------------------------------------------
template <typename T, int N, bool C2C>
struct ZICfg {
  static constexpr int G = Geo<N>::G;
  static constexpr int TY = ZCfg<T, N, C2C, UR_ZI_PAIRS_F32>::TY;
  static constexpr int NG = ZCfg<T, N, C2C, UR_ZI_PAIRS_F32>::NG;
  static constexpr int threads = NG * G;
  static constexpr int HS = C2C ? N : N / 2 + 1;       // staged rows per pencil
};

template <typename T, int N, bool C2C>
__global__ void __launch_bounds__((ZICfg<T, N, C2C>::threads))
k_pass_z_inv(ZInvArgs a) {
  using C = ZICfg<T, N, C2C>;
  constexpr int G = C::G, NG = C::NG, TY = C::TY, HS = C::HS, E = Geo<N>::E;
  constexpr int R0 = Radix<N, 1>::r, NB0 = E / R0, PS = CS<N>::v;
  constexpr int HP = HS + 1;                            // staged pencil stride (r2c)
  // r2c: staged half spectra of TY pencils, then NG separate FFT columns;
  // c2c: every staged pencil is its own group's FFT column (padded layout)
  constexpr int LDS_ELEMS = C2C ? TY * PS : TY * HP + NG * PS;
  __shared__ cx<T> lds[LDS_ELEMS];
  const int tile = blockIdx.x % a.ntiles;
  const long long X = a.x0 + blockIdx.x / a.ntiles;
  const int y0 = tile * TY;
  if (a.prune) {                                        // block-uniform
    long long lo, hi;
    row_range(a.L, a.m, X, lo, hi);
    if (y0 + TY - 1 < lo || y0 > hi) return;
  }
  const cx<T>* Ap = (const cx<T>*)a.A + ((size_t)X * a.nkz) * N + y0;
  for (int idx = threadIdx.x; idx < TY * HS; idx += C::threads) {
    const int j = idx % TY, kz = idx / TY;
    if (C2C) lds[j * PS + pad(kz)] = Ap[(size_t)kz * N + j];
    else lds[j * HP + kz] = Ap[(size_t)kz * N + j];
  }
  __syncthreads();
  const int q = threadIdx.x / G, g = threadIdx.x % G;
  cx<T>* s = C2C ? lds + q * PS : lds + TY * HP + q * PS;
  cx<T> v[E];
  if (!C2C) {
    const cx<T>* ha = lds + (2 * q) * HP;
    const cx<T>* hb = lds + (2 * q + 1) * HP;
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        int k = first_index<N>(g, i, r);
        cx<T> A_, B_;
        if (k <= N / 2) {
          A_ = ha[k]; B_ = hb[k];
          if (k == 0 || k == N / 2) { A_.y = (T)0; B_.y = (T)0; }   // self-conjugate bins are real
        } else {
          A_ = conjg(ha[N - k]); B_ = conjg(hb[N - k]);
        }
        v[i * R0 + r] = mk(A_.x - B_.y, A_.y + B_.x);                  // A + i B
      }
  } else {
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) v[i * R0 + r] = s[pad(first_index<N>(g, i, r))];
    col_sync<G>();
  }
  fft_column<T, N, +1>(s, g, (const cx<T>*)a.tw, v);
  const T sc = (T)a.scale;
  if (!C2C) {
    T* outA = (T*)a.out + ((size_t)X * N + (y0 + 2 * q)) * N;
    T* outB = outA + N;
    for (int i = g; i < N; i += G) {
      cx<T> z = s[pad(i)];
      outA[i] = z.x * sc;
      outB[i] = z.y * sc;
    }
  } else {
    cx<T>* o = (cx<T>*)a.out + ((size_t)X * N + (y0 + q)) * N;
    for (int i = g; i < N; i += G) o[i] = scale(s[pad(i)], sc);
  }
}

// ---------------------------------------------------------------------------
// inverse z pass fused with the fold onto the unit cell: for every pencil of
// the particle's rows, the c2r transform along z of the weighted spectrum
// gives grad rho(x, y, :); its inside voxels are summed into the cell voxel
// they tile from (adjoint of tiling + masking), in LDS per block.  Persistent
// blocks walk the (plane, y tile) list; the r2c half spectra of a tile are
// staged, then the same LDS holds the transform columns.
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__((ZICfg<T, N, false>::threads), MinW<T>::v)
k_pass_z_fold(ZFoldArgs a) {
  using C = ZICfg<T, N, false>;
  constexpr int G = C::G, NG = C::NG, TY = C::TY, HS = C::HS, E = Geo<N>::E;
  constexpr int R0 = Radix<N, 1>::r, NB0 = E / R0, PS = CS<N>::v;
  constexpr int HP = HS + 1;
  constexpr int STG = TY * HP > NG * PS ? TY * HP : NG * PS;
  __shared__ cx<T> lds[STG];
  extern __shared__ double acc[];                      // c^2 (c <= 16): [cj][k] of this block's ci
  const int c = a.L.c, cm = c - 1;
  const bool use_lds = c <= 16;
  if (use_lds) for (int i = threadIdx.x; i < c * c; i += C::threads) acc[i] = 0.0;
  __syncthreads();
  const int q = threadIdx.x / G, g = threadIdx.x % G;
  // c <= 16: block b takes only the planes whose cell index is ci = b mod c
  // (the grid is a multiple of c), so its accumulator is one c x c slice;
  // otherwise every block strides over all tiles (global accumulation)
  const int ci_b = use_lds ? (int)(blockIdx.x % c) : 0;
  const long long X0 = use_lds ? a.xlo + ((ci_b - (a.xlo - a.L.o - a.L.h)) & cm) : a.xlo;
  const long long xstep = use_lds ? c : 1;
  const long long np = X0 <= a.xhi ? (a.xhi - X0) / xstep + 1 : 0;
  const long long ntile = np * a.ntiles;
  const long long t0 = use_lds ? blockIdx.x / c : blockIdx.x;
  const long long tstep = use_lds ? gridDim.x / c : gridDim.x;
  for (long long t = t0; t < ntile; t += tstep) {
    const long long X = X0 + (t / a.ntiles) * xstep;
    const int y0 = (int)(t % a.ntiles) * TY;
    long long ylo, yhi;
    row_range(a.L, a.m, X, ylo, yhi);
    if (ylo > yhi || y0 + TY - 1 < ylo || y0 > yhi) continue;   // uniform per block
    const cx<T>* Ap = (const cx<T>*)a.A + ((size_t)X * a.nkz) * N + y0;
    {
      // all loads of a thread before its LDS stores
      constexpr int NST = TY * HS, IT = (NST + C::threads - 1) / C::threads;
      T rx[IT], ry[IT];
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        const int idx = threadIdx.x + k * C::threads;
        if (idx < NST) {
          const cx<T> e = Ap[(size_t)(idx / TY) * N + idx % TY];
          rx[k] = e.x;
          ry[k] = e.y;
        }
      }
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        const int idx = threadIdx.x + k * C::threads;
        if (idx < NST) {
          lds[(idx % TY) * HP + idx / TY].x = rx[k];
          lds[(idx % TY) * HP + idx / TY].y = ry[k];
        }
      }
    }
    __syncthreads();
    cx<T> v[E];
    {
      const cx<T>* ha = lds + (2 * q) * HP;
      const cx<T>* hb = lds + (2 * q + 1) * HP;
#pragma unroll
      for (int i = 0; i < NB0; ++i)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          const int k = first_index<N>(g, i, r);
          cx<T> A_, B_;
          if (k <= N / 2) {
            A_ = ha[k]; B_ = hb[k];
            if (k == 0 || k == N / 2) { A_.y = (T)0; B_.y = (T)0; }
          } else {
            A_ = conjg(ha[N - k]); B_ = conjg(hb[N - k]);
          }
          v[i * R0 + r] = mk(A_.x - B_.y, A_.y + B_.x);
        }
    }
    __syncthreads();                                   // staging consumed: reuse it for the columns
    cx<T>* s = lds + q * PS;
    fft_column<T, N, +1>(s, g, (const cx<T>*)a.tw, v);
    // fold the two pencils' inside voxels
    const long long yA = y0 + 2 * q;
#pragma unroll
    for (int p2 = 0; p2 < 2; ++p2) {
      const long long Y = yA + p2;
      long long zlo, zhi;
      col_range(a.L, a.m, X, Y, zlo, zhi);
      const int ci = (int)(X - a.L.o - a.L.h) & cm, cj = (int)(Y - a.L.o - a.L.h) & cm;
      const int zoff = -(a.L.o + a.L.h);
      if (use_lds && G % c == 0) {
        // the voxels of a lane (z = zlo + g + G m) share one cell residue:
        // sum them in a register, one LDS atomic per lane and pencil
        double sum = 0.0;
        for (int z = (int)zlo + g; z <= (int)zhi; z += G) {
          const cx<T> f = s[pad(z)];
          sum += (double)(p2 == 0 ? f.x : f.y);
        }
        if ((int)zlo + g <= (int)zhi) atomicAdd(&acc[cj * c + (((int)zlo + g + zoff) & cm)], sum * a.scale);
      } else {
        for (int z = (int)zlo + g; z <= (int)zhi; z += G) {
          const cx<T> f = s[pad(z)];
          const double val = (double)(p2 == 0 ? f.x : f.y) * a.scale;
          if (use_lds) atomicAdd(&acc[cj * c + ((z + zoff) & cm)], val);
          else atomicAdd(&a.gcell[(ci * c + cj) * c + ((z + zoff) & cm)], val);
        }
      }
    }
    __syncthreads();                                   // columns done before the next staging
  }
  if (use_lds) {
    __syncthreads();
    double* out = a.part + (size_t)blockIdx.x * c * c;
    for (int i = threadIdx.x; i < c * c; i += C::threads) out[i] = acc[i];
  }
}

// ---------------------------------------------------------------------------
// fold of a voxel field over the inside voxels onto the cell (adjoint of
// tiling + masking), ED-1 geometry (factor 1)
// ---------------------------------------------------------------------------
template <typename T, bool LDS>
__global__ void __launch_bounds__(256) k_fold(FoldArgs a, int n) {
  extern __shared__ double acc[];
  const int c = a.L.c, c3 = c * c * c;
  if (LDS) {
    for (int i = threadIdx.x; i < c3; i += 256) acc[i] = 0.0;
    __syncthreads();
  }
  if constexpr (LDS) {
    // cell edges up to 16 (powers of two): 16 threads per pencil, 16 pencils
    // per block at a time; thread r of a pencil takes z = zlo + r, zlo + r +
    // 16, ..., all of one cell residue (16 is a multiple of the edge), sums
    // them in a register and adds the sum to the cell once
    const int r = threadIdx.x & 15;
    for (long long pc = (long long)blockIdx.x * 16 + (threadIdx.x >> 4); pc < a.npencils; pc += (long long)gridDim.x * 16) {
      const long long X = pc / n, Y = pc % n;
      long long zlo, zhi;
      col_range(a.L, a.m, X, Y, zlo, zhi);
      if (zlo > zhi) continue;
      const int i = pmodi(X - a.L.o - a.L.h, c), j = pmodi(Y - a.L.o - a.L.h, c);
      const T* gp = (const T*)a.g + (size_t)pc * n;
      double sum = 0.0;
      long long z = zlo + r;
      for (; z + 48 <= zhi; z += 64) {
        const double v0 = (double)gp[z], v1 = (double)gp[z + 16], v2 = (double)gp[z + 32], v3 = (double)gp[z + 48];
        sum += v0;
        sum += v1;
        sum += v2;
        sum += v3;
      }
      for (; z <= zhi; z += 16) sum += (double)gp[z];
      if (zlo + r <= zhi) atomicAdd(&acc[(i * c + j) * c + pmodi(zlo + r - a.L.o - a.L.h, c)], sum);
    }
  } else {
    for (long long pc = blockIdx.x; pc < a.npencils; pc += gridDim.x) {
      const long long X = pc / n, Y = pc % n;
      long long zlo, zhi;
      col_range(a.L, a.m, X, Y, zlo, zhi);
      if (zlo > zhi) continue;
      const int i = pmodi(X - a.L.o - a.L.h, c), j = pmodi(Y - a.L.o - a.L.h, c);
      const T* gp = (const T*)a.g + (size_t)pc * n;
      for (long long z = zlo + threadIdx.x; z <= zhi; z += 256) {
        const int k = pmodi(z - a.L.o - a.L.h, c);
        atomicAdd(&a.gcell[(i * c + j) * c + k], (double)gp[z]);
      }
    }
  }
  if (LDS) {
    __syncthreads();
    double* out = a.part + (size_t)blockIdx.x * c3;
    for (int i = threadIdx.x; i < c3; i += 256) out[i] = acc[i];
  }
}

// Adjoint of the rotated and polycrystalline ED-1 sampler (factor 1): the
// gradient at every inside voxel is spread back onto the cell values its
// interpolation read, with the weights it read them with (trilinear: the
// eight cell voxels around floor(u), (1 - t) or t per axis; cubic B-spline:
// the 4 x 4 x 4 coefficients, the product of the three weight sets).  One
// wavefront per pencil, lanes along z; every block adds into its own FP64
// c^3 accumulator in LDS (c <= 16) and writes it out as its partial.
// Blocks of 16 wavefronts: the partial buffer fixes the grid (one partial
// per block), so the block size sets how many waves each SIMD runs.
constexpr int kFoldRotThreads = 1024;
template <typename T, int INTERP, bool GRAINS>
__global__ void __launch_bounds__(kFoldRotThreads) k_fold_rot(ZArgs a, const void* __restrict__ gfield, double* __restrict__ part, int n) {
  extern __shared__ double acc[];
  __shared__ double grl[GRAINS ? kMaxGrains * 9 : 1];
  const int c = a.L.c, c3 = c * c * c, cm = c - 1;
  for (int i = threadIdx.x; i < c3; i += kFoldRotThreads) acc[i] = 0.0;
  if constexpr (GRAINS)
    for (int i = threadIdx.x; i < 9 * a.ngrain; i += kFoldRotThreads) grl[i] = (&a.grot[0][0])[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const long long np = (long long)n * n;
  constexpr int WPB = kFoldRotThreads / 64;
  for (long long pc = (long long)blockIdx.x * WPB + (threadIdx.x >> 6); pc < np; pc += (long long)gridDim.x * WPB) {
    const long long X = pc / n, Y = pc % n;
    Pencil<T> p;
    p.init(a, X, Y);
    if (p.zlo > p.zhi) continue;                       // wave-uniform
    if constexpr (GRAINS) { p.GR = grl; p.init_grains(a); }
    const T* gp = (const T*)gfield + (size_t)pc * n;
    for (int z = p.zlo + lane; z <= p.zhi; z += 64) {
      const double gv = (double)gp[z];
      double u, v, w;
      p.template coords<GRAINS>(a, z, u, v, w);
      const double fu = floor(u), fv = floor(v), fw = floor(w);
      if constexpr (INTERP == 3) {
        T wu[4], wv[4], ww[4];
        bspline_weights<T>((T)(u - fu), wu);
        bspline_weights<T>((T)(v - fv), wv);
        bspline_weights<T>((T)(w - fw), ww);
        const int i0 = (int)(long long)fu - 1, j0 = (int)(long long)fv - 1, k0 = (int)(long long)fw - 1;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double gqr = gv * (double)wu[q] * (double)wv[r];
            double* row = acc + (((i0 + q) & cm) * c + ((j0 + r) & cm)) * c;
#pragma unroll
            for (int m = 0; m < 4; ++m) atomicAdd(&row[(k0 + m) & cm], gqr * (double)ww[m]);
          }
      } else {
        const double tu = (double)(T)(u - fu), tv = (double)(T)(v - fv), tw = (double)(T)(w - fw);
        const int i0 = (int)(long long)fu & cm, i1 = (i0 + 1) & cm;
        const int j0 = (int)(long long)fv & cm, j1 = (j0 + 1) & cm;
        const int k0 = (int)(long long)fw & cm, k1 = (k0 + 1) & cm;
        const double g0 = gv * (1.0 - tu), g1 = gv * tu;
        const double g00 = g0 * (1.0 - tv), g01 = g0 * tv, g10 = g1 * (1.0 - tv), g11 = g1 * tv;
        double* r00 = acc + (i0 * c + j0) * c;
        double* r01 = acc + (i0 * c + j1) * c;
        double* r10 = acc + (i1 * c + j0) * c;
        double* r11 = acc + (i1 * c + j1) * c;
        atomicAdd(&r00[k0], g00 * (1.0 - tw));
        atomicAdd(&r00[k1], g00 * tw);
        atomicAdd(&r01[k0], g01 * (1.0 - tw));
        atomicAdd(&r01[k1], g01 * tw);
        atomicAdd(&r10[k0], g10 * (1.0 - tw));
        atomicAdd(&r10[k1], g10 * tw);
        atomicAdd(&r11[k0], g11 * (1.0 - tw));
        atomicAdd(&r11[k1], g11 * tw);
      }
    }
  }
  __syncthreads();
  double* out = part + (size_t)blockIdx.x * c3;
  for (int i = threadIdx.x; i < c3; i += kFoldRotThreads) out[i] = acc[i];
}

#if UR_IN(0)
__global__ void __launch_bounds__(256) k_fold_reduce(int c3, const double* __restrict__ part, int nblk, double* __restrict__ gcell) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c3) return;
  // eight compensated sums (block b to sum b mod 8), eight loads in flight,
  // then added in order
  Kahan kk[8];
  int b = 0;
  for (; b + 8 <= nblk; b += 8) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = part[(size_t)(b + u) * c3 + v];
#pragma unroll
    for (int u = 0; u < 8; ++u) kk[u].add(x[u]);
  }
#pragma unroll
  for (int u = 0; u < 8; ++u)                        // the last nblk mod 8 blocks (compile-time indices)
    if (b + u < nblk) kk[u].add(part[(size_t)(b + u) * c3 + v]);
  Kahan k;
#pragma unroll
  for (int u = 0; u < 8; ++u) { k.add(kk[u].s); k.add(kk[u].c); }
  gcell[v] = k.val();
}

// grad_amp[a] = sum_j gcell[j] p_a,x[jx] p_a,y[jy] p_a,z[jz]; one block per atom
__global__ void __launch_bounds__(256) k_grad_amp(int c, const double* __restrict__ prof,
                                                  const double* __restrict__ gcell, double* __restrict__ ga) {
  __shared__ double red[4];
  const int at = blockIdx.x;
  const double* p = prof + (size_t)at * 3 * c;
  const int c3 = c * c * c;
  double s = 0.0;
  for (int v = threadIdx.x; v < c3; v += 256) {
    int k = v % c, j = (v / c) % c, i = v / (c * c);
    s += gcell[v] * p[i] * p[c + j] * p[2 * c + k];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) ga[at] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_zero(double* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

#endif
// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
#define UR_DISPATCH_N(n, MACRO)                  \
  switch (n) {                                   \
    case 16: MACRO(16); break;                   \
    case 32: MACRO(32); break;                   \
    case 64: MACRO(64); break;                   \
    case 128: MACRO(128); break;                 \
    case 256: MACRO(256); break;                 \
    case 512: MACRO(512); break;                 \
    case 1024: MACRO(1024); break;               \
    case 2048: MACRO(2048); break;               \
    default: return hipErrorInvalidValue;        \
  }

// LDS budget of one block (gfx950: 160 KB per CU); kernels whose
// configuration would exceed it are not instantiated for that size
constexpr size_t kLdsBytes = 160 * 1024;
template <typename T, int N, bool C2C> constexpr bool z_fits() {
  return (size_t)ZCfg<T, N, C2C>::NG * CS<N>::v * sizeof(cx<T>) + 1024 <= kLdsBytes;
}
template <typename T, int N> constexpr bool inv_fits() {      // inverse y / z passes
  return (size_t)YCfg<T, N>::TX * CS<N>::v * sizeof(cx<T>) <= kLdsBytes && N <= 1024;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
static unsigned nblk_of(long long total, int threads) { return (unsigned)((total + threads - 1) / threads); }

#if UR_IN(0)
hipError_t launch_cell_profiles(int c, int n_atoms, const double* xyz, const double* sigma, double* prof, hipStream_t s) {
  long long total = (long long)n_atoms * 3 * c;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cell_profiles, dim3(nblk_of(total, 256)), dim3(256), 0, s, c, n_atoms, xyz, sigma, prof);
  return hipGetLastError();
}

hipError_t launch_cell_sum(int c, int n_atoms, const double* amp, const double* prof, double bg, double* cell, hipStream_t s,
                           int prec, void* cellT) {
  const long long c3 = (long long)c * c * c;
  const size_t lds = ((size_t)3 * c * n_atoms + n_atoms) * sizeof(double);
  const int staged = lds <= kCellStageBytes ? 1 : 0;
  const size_t shm = staged ? lds : 0;
  if (prec == 1 && cellT)
    hipLaunchKernelGGL(k_cell_sum<double>, dim3(nblk_of(c3, 256)), dim3(256), shm, s, c, n_atoms, amp, prof, bg, cell, (double*)cellT, staged);
  else
    hipLaunchKernelGGL(k_cell_sum<float>, dim3(nblk_of(c3, 256)), dim3(256), shm, s, c, n_atoms, amp, prof, bg, cell, (float*)cellT, staged);
  return hipGetLastError();
}

hipError_t launch_cell_tables(int prec, int c, int f, const double* cell, void* cellT, double* pre, void* cb, int cbn, hipStream_t s) {
  const long long c3 = (long long)c * c * c;
  const long long nb = (long long)cbn * cbn * cbn;
  if (prec == 0)
    hipLaunchKernelGGL(k_cell_tables<float>, dim3(nblk_of(c3, 256)), dim3(256), 0, s, c, f, cell, (float*)cellT, pre, (float*)cb, cbn);
  else
    hipLaunchKernelGGL(k_cell_tables<double>, dim3(nblk_of(c3, 256)), dim3(256), 0, s, c, f, cell, (double*)cellT, pre, (double*)cb, cbn);
  if (f > 1) {
    if (prec == 0)
      hipLaunchKernelGGL(k_cell_blocks<float>, dim3((unsigned)nb), dim3(256), 0, s, c, f, cell, (float*)cb, cbn);
    else
      hipLaunchKernelGGL(k_cell_blocks<double>, dim3((unsigned)nb), dim3(256), 0, s, c, f, cell, (double*)cb, cbn);
  }
  return hipGetLastError();
}
#endif

// SAMP: the rotated-lattice modes of one sampler (1 trilinear, 3 cubic;
// instantiated in their own parts), or 0 for the aligned modes
template <typename T, int N, int SAMP>
static hipError_t pass_z_t(int mode, const ZArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid(nblocks), real_blk(ZCfg<T, N, false>::threads);
#define UR_ZK(M) hipLaunchKernelGGL((k_pass_z<T, N, M>), grid, real_blk, 0, s, a)
  if constexpr (SAMP == 1) {
    switch (mode) {
      case Z_ROT_R2C: UR_ZK(Z_ROT_R2C); break;
      case Z_ROTG_R2C: UR_ZK(Z_ROTG_R2C); break;
      default: return hipErrorInvalidValue;
    }
  } else if constexpr (SAMP == 3) {
    switch (mode) {
      case Z_ROT3_R2C: UR_ZK(Z_ROT3_R2C); break;
      case Z_ROT3G_R2C: UR_ZK(Z_ROT3G_R2C); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (mode) {
      case Z_GEN_R2C: UR_ZK(Z_GEN_R2C); break;
      case Z_LOAD_R2C: UR_ZK(Z_LOAD_R2C); break;
      case Z_ZOOM_R2C: UR_ZK(Z_ZOOM_R2C); break;
      case Z_GEN_C2C: case Z_LOAD_C2C: case Z_ZOOM_C2C:
        if constexpr (!z_fits<T, N, true>()) {
          return hipErrorNotSupported;
        } else {
          const dim3 cblk(ZCfg<T, N, true>::threads);
          if (mode == Z_GEN_C2C) hipLaunchKernelGGL((k_pass_z<T, N, Z_GEN_C2C>), grid, cblk, 0, s, a);
          else if (mode == Z_LOAD_C2C) hipLaunchKernelGGL((k_pass_z<T, N, Z_LOAD_C2C>), grid, cblk, 0, s, a);
          else hipLaunchKernelGGL((k_pass_z<T, N, Z_ZOOM_C2C>), grid, cblk, 0, s, a);
        }
        break;
      default: return hipErrorInvalidValue;
    }
  }
#undef UR_ZK
  return hipGetLastError();
}

// 4096^3 boxes run only the out-of-core forward path in FP32: the z pass
// from staged planes, the forward y pass and the binning x pass
constexpr int kBig = kMaxOutOfCore;
static_assert(kMaxInCore == 2048, "the in-HBM dispatch below instantiates sizes up to 2048");

template <typename T, int SAMP>
static hipError_t pass_z_any(int n, int mode, const ZArgs& a, int nblocks, hipStream_t s) {
  if (n == kBig) {
    if constexpr (sizeof(T) != 4 || SAMP != 0) {
      return hipErrorNotSupported;
    } else {
      if (mode != Z_LOAD_R2C) return hipErrorNotSupported;
      if (nblocks <= 0) return hipSuccess;
      hipLaunchKernelGGL((k_pass_z<float, kBig, Z_LOAD_R2C>), dim3(nblocks), dim3(ZCfg<float, kBig, false>::threads), 0, s, a);
      return hipGetLastError();
    }
  }
#define UR_Z(NN) return pass_z_t<T, NN, SAMP>(mode, a, nblocks, s)
  UR_DISPATCH_N(n, UR_Z);
#undef UR_Z
}

// per-precision and per-sampler entry points, each in its own part
hipError_t launch_pass_z_f32(int n, int mode, const ZArgs& a, int nblocks, hipStream_t s);
hipError_t launch_pass_z_f64(int n, int mode, const ZArgs& a, int nblocks, hipStream_t s);
hipError_t launch_pass_z_rot_f32(int n, int mode, const ZArgs& a, int nblocks, hipStream_t s);
hipError_t launch_pass_z_rot_f64(int n, int mode, const ZArgs& a, int nblocks, hipStream_t s);
hipError_t launch_pass_z_rot3_f32(int n, int mode, const ZArgs& a, int nblocks, hipStream_t s);
hipError_t launch_pass_z_rot3_f64(int n, int mode, const ZArgs& a, int nblocks, hipStream_t s);
#define UR_ZENTRY(PART, NAME, T, SAMP)                                                   \
  hipError_t NAME(int n, int mode, const ZArgs& a, int nblocks, hipStream_t s) { \
    return pass_z_any<T, SAMP>(n, mode, a, nblocks, s);                          \
  }
#if UR_IN(1)
UR_ZENTRY(1, launch_pass_z_f32, float, 0)
#endif
#if UR_IN(2)
UR_ZENTRY(2, launch_pass_z_f64, double, 0)
#endif
#if UR_IN(7)
UR_ZENTRY(7, launch_pass_z_rot_f32, float, 1)
#endif
#if UR_IN(8)
UR_ZENTRY(8, launch_pass_z_rot_f64, double, 1)
#endif
#if UR_IN(9)
UR_ZENTRY(9, launch_pass_z_rot3_f32, float, 3)
#endif
#if UR_IN(10)
UR_ZENTRY(10, launch_pass_z_rot3_f64, double, 3)
#endif
#undef UR_ZENTRY
#if UR_IN(0)
hipError_t launch_pass_z(int prec, int n, int mode, const ZArgs& a, int nblocks, hipStream_t s) {
  if (mode == Z_ROT_R2C || mode == Z_ROTG_R2C)
    return prec == 0 ? launch_pass_z_rot_f32(n, mode, a, nblocks, s) : launch_pass_z_rot_f64(n, mode, a, nblocks, s);
  if (mode == Z_ROT3_R2C || mode == Z_ROT3G_R2C)
    return prec == 0 ? launch_pass_z_rot3_f32(n, mode, a, nblocks, s) : launch_pass_z_rot3_f64(n, mode, a, nblocks, s);
  return prec == 0 ? launch_pass_z_f32(n, mode, a, nblocks, s) : launch_pass_z_f64(n, mode, a, nblocks, s);
}
#endif

template <typename T, int N>
static hipError_t pass_y_t(const YArgs& a, hipStream_t s) {
  long long nb = (long long)(a.nkzc > 0 ? a.nkzc : a.nkz) * a.nxt;
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_pass_y<T, N>), dim3((unsigned)nb), dim3(YCfg<T, N>::threads), 0, s, a);
  return hipGetLastError();
}

#if UR_IN(5)
hipError_t launch_pass_y(int prec, int n, const YArgs& a, hipStream_t s) {
  if (n == kBig) return prec == 0 ? pass_y_t<float, kBig>(a, s) : hipErrorNotSupported;
#define UR_Y(NN) return prec == 0 ? pass_y_t<float, NN>(a, s) : pass_y_t<double, NN>(a, s)
  UR_DISPATCH_N(n, UR_Y);
#undef UR_Y
}
#endif

static size_t x_shm(int mode, int nbins, int n, size_t ts = 8) {
  if (mode == X_FFT_BIN_SINC || mode == X_BIN_ONLY_SINC)
    return x_shm(mode == X_FFT_BIN_SINC ? X_FFT_BIN : X_BIN_ONLY, nbins, n) + 16 + ((size_t)n / 2 + 1) * ts;
  if (mode == X_ADJ)
    return ((size_t)nbins + 2) * sizeof(double) + ((size_t)nbins + 2) * sizeof(int) + (size_t)lut_len(n) * sizeof(short);
  return mode == X_FFT_STORE ? 0 : (2 * (size_t)nbins + 5) * sizeof(double) + ((size_t)nbins + 3) * sizeof(int)
                                    + (size_t)lut_len(n) * sizeof(short);
}

template <typename T, int N>
static int x_resident_t(int mode, int dir, int nbins) {
  int nb = 0;
  hipError_t e;
  size_t shm = x_shm(mode, nbins, N);
  if (mode == X_FFT_BIN) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pass_x<T, N, X_FFT_BIN, -1>, XCfg<N>::threads, shm);
  else if (mode == X_FFT_BIN_SINC || mode == X_BIN_ONLY_SINC) return x_resident_t<T, N>(mode == X_FFT_BIN_SINC ? X_FFT_BIN : X_BIN_ONLY, dir, nbins);
  else if constexpr (N == kBig) return 1;
  else if (mode == X_ADJ) return 1;                  // x_resident_adj_t
  else if (mode == X_BIN_ONLY) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pass_x<T, N, X_BIN_ONLY, -1>, XCfg<N>::threads, shm);
  else if (dir < 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pass_x<T, N, X_FFT_STORE, -1>, XCfg<N>::threads, shm);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pass_x<T, N, X_FFT_STORE, +1>, XCfg<N>::threads, shm);
  if (e != hipSuccess) { (void)hipGetLastError(); return 1; }
  return nb > 0 ? nb : 1;
}

template <typename T, int N>
static int x_resident_adj_t(int nbins) {
  if constexpr (!inv_fits<T, N>()) {
    return 1;
  } else {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pass_x_adj<T, N>, XCfg<N>::threads, x_shm(X_ADJ, nbins, N)) !=
        hipSuccess) {
      (void)hipGetLastError();
      return 1;
    }
    return nb > 0 ? nb : 1;
  }
}

template <typename T>
static int x_resident_any(int n, int mode, int dir, int nbins) {
  if (n == kBig) {
    if constexpr (sizeof(T) == 4) return mode == X_FFT_BIN ? x_resident_t<float, kBig>(mode, dir, nbins) : 1;
    else return 1;
  }
#define UR_XR(NN) return x_resident_t<T, NN>(mode, dir, nbins)
  switch (n) {
    case 16: UR_XR(16); case 32: UR_XR(32); case 64: UR_XR(64); case 128: UR_XR(128);
    case 256: UR_XR(256); case 512: UR_XR(512); case 1024: UR_XR(1024); case 2048: UR_XR(2048);
    default: return 1;
  }
#undef UR_XR
}

template <typename T>
static int x_resident_adj_any(int n, int nbins) {
#define UR_XR(NN) return x_resident_adj_t<T, NN>(nbins)
  switch (n) {
    case 16: UR_XR(16); case 32: UR_XR(32); case 64: UR_XR(64); case 128: UR_XR(128);
    case 256: UR_XR(256); case 512: UR_XR(512); case 1024: UR_XR(1024); case 2048: UR_XR(2048);
    default: return 1;
  }
#undef UR_XR
}

int x_resident_f32(int n, int mode, int dir, int nbins);
int x_resident_f64(int n, int mode, int dir, int nbins);
int x_resident_adj(int prec, int n, int nbins);
#if UR_IN(3)
int x_resident_f32(int n, int mode, int dir, int nbins) { return x_resident_any<float>(n, mode, dir, nbins); }
#endif
#if UR_IN(4)
int x_resident_f64(int n, int mode, int dir, int nbins) { return x_resident_any<double>(n, mode, dir, nbins); }
#endif
#if UR_IN(6)
int x_resident_adj(int prec, int n, int nbins) {
  return prec == 0 ? x_resident_adj_any<float>(n, nbins) : x_resident_adj_any<double>(n, nbins);
}
#endif
#if UR_IN(0)
int x_resident(int prec, int n, int mode, int dir, int nbins) {
  if (mode == X_ADJ) return x_resident_adj(prec, n, nbins);
  return prec == 0 ? x_resident_f32(n, mode, dir, nbins) : x_resident_f64(n, mode, dir, nbins);
}
#endif

#if UR_IN(0)
hipError_t launch_bin_counts(int n, int nkz, int r2c, int nbins, const int* U, unsigned long long* tmp, double* out, hipStream_t s) {
  long long ncols = (long long)nkz * n;
  size_t shm = (size_t)nbins * sizeof(unsigned long long) + ((size_t)nbins + 2) * sizeof(int);
  hipError_t e = launch_zero(tmp, (size_t)nbins * sizeof(unsigned long long), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_counts, dim3((unsigned)((ncols + 255) / 256)), dim3(256), shm, s, n, nkz, r2c, nbins, U, tmp);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_counts_to_double, dim3((nbins + 255) / 256), dim3(256), 0, s, nbins, tmp, out);
  return hipGetLastError();
}
#endif

template <typename T, int N>
static hipError_t pass_x_t(int mode, int dir, const XArgs& a, int nblocks, hipStream_t s) {
  if (a.sinc && mode == X_FFT_BIN) mode = X_FFT_BIN_SINC;        // voxel form factor requested
  if (a.sinc && mode == X_BIN_ONLY) mode = X_BIN_ONLY_SINC;
  size_t shm = x_shm(mode, a.nbins, N, sizeof(T));
  // columns spanning several wavefronts sync with workgroup barriers: every
  // group of a block must run the same number of iterations
  if (XCfg<N>::G > 64 && a.ncols % XCfg<N>::NG != 0) return hipErrorInvalidValue;
  dim3 grid(nblocks), blk(XCfg<N>::threads);
  if (mode == X_FFT_BIN) hipLaunchKernelGGL((k_pass_x<T, N, X_FFT_BIN, -1>), grid, blk, shm, s, a);
  else if (mode == X_FFT_BIN_SINC) hipLaunchKernelGGL((k_pass_x<T, N, X_FFT_BIN_SINC, -1>), grid, blk, shm, s, a);
  else if constexpr (N == kBig) return hipErrorNotSupported;
  else if (mode == X_BIN_ONLY_SINC) hipLaunchKernelGGL((k_pass_x<T, N, X_BIN_ONLY_SINC, -1>), grid, blk, shm, s, a);
  else if (mode == X_BIN_ONLY) hipLaunchKernelGGL((k_pass_x<T, N, X_BIN_ONLY, -1>), grid, blk, shm, s, a);
  else if (dir < 0) hipLaunchKernelGGL((k_pass_x<T, N, X_FFT_STORE, -1>), grid, blk, shm, s, a);
  else hipLaunchKernelGGL((k_pass_x<T, N, X_FFT_STORE, +1>), grid, blk, shm, s, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t pass_x_any(int n, int mode, int dir, const XArgs& a, int nblocks, hipStream_t s) {
  if (n == kBig) {
    if constexpr (sizeof(T) != 4) {
      return hipErrorNotSupported;
    } else {
      if (mode != X_FFT_BIN) return hipErrorNotSupported;
      return pass_x_t<float, kBig>(mode, dir, a, nblocks, s);
    }
  }
#define UR_X(NN) return pass_x_t<T, NN>(mode, dir, a, nblocks, s)
  UR_DISPATCH_N(n, UR_X);
#undef UR_X
}

hipError_t launch_pass_x_f32(int n, int mode, int dir, const XArgs& a, int nblocks, hipStream_t s);
hipError_t launch_pass_x_f64(int n, int mode, int dir, const XArgs& a, int nblocks, hipStream_t s);
#if UR_IN(3)
hipError_t launch_pass_x_f32(int n, int mode, int dir, const XArgs& a, int nblocks, hipStream_t s) {
  return pass_x_any<float>(n, mode, dir, a, nblocks, s);
}
#endif
#if UR_IN(4)
hipError_t launch_pass_x_f64(int n, int mode, int dir, const XArgs& a, int nblocks, hipStream_t s) {
  return pass_x_any<double>(n, mode, dir, a, nblocks, s);
}
#endif
#if UR_IN(0)
hipError_t launch_pass_x(int prec, int n, int mode, int dir, const XArgs& a, int nblocks, hipStream_t s) {
  return prec == 0 ? launch_pass_x_f32(n, mode, dir, a, nblocks, s) : launch_pass_x_f64(n, mode, dir, a, nblocks, s);
}
#endif

#if UR_IN(0)
hipError_t launch_finalize(const FinArgs& a, hipStream_t s) {
  int nv = 2 * a.nbins + 1;
  int nvb = (nv + 7) / 8;
  if (a.mom && a.nzb > kFoldMoments) {
    hipLaunchKernelGGL(k_moments, dim3(256), dim3(256), 0, s, a.mom, a.nzb, a.mpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_finalize, dim3(nvb + 1), dim3(256), 0, s, a);
  return hipGetLastError();
}

// |F|^2 at the integer frequency (h, k, l) (signed, any range: the DFT is
// periodic); a real transform keeps kz in [0, n/2], the rest by F(-q) = F(q)*
template <typename T>
__device__ __forceinline__ double ewald_intensity(const EwaldArgs& a, long long h, long long k, long long l) {
  const long long n = a.n;
  long long lz = ((l % n) + n) % n;
  if (!a.c2c && lz > n / 2) { h = -h; k = -k; lz = (((-l) % n) + n) % n; }
  const long long kx = ((h % n) + n) % n, ky = ((k % n) + n) % n;
  const size_t at = a.natural ? ((size_t)kx * n + ky) * a.nkz + lz : ((size_t)lz * n + ky) * n + kx;
  const cx<T> f = ((const cx<T>*)a.spec)[at];
  return (double)f.x * (double)f.x + (double)f.y * (double)f.y;
}

// One thread per pixel: flat detector normal to the beam e at distance
// dist, pixel (iu, iv) at dist e + (iu - cu) pixel du + (iv - cv) pixel dv;
// scattered direction s; for each wavelength node q = k_j (s - e), grid
// coordinates q / dq, trilinear interpolation of |F|^2 (the third axis
// first), weighted sum over the nodes.
template <typename T>
__global__ void __launch_bounds__(256) k_ewald(EwaldArgs a) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)a.nu * a.nv) return;
  const int iu = (int)(t % a.nu), iv = (int)(t / a.nu);
  double P[3];
  for (int i = 0; i < 3; ++i)
    P[i] = a.dist * a.e[i] + ((double)iu - a.cu) * a.pixel * a.du[i] + ((double)iv - a.cv) * a.pixel * a.dv[i];
  const double r = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
  double acc = 0.0;
  for (int j = 0; j < a.nl; ++j) {
    double g[3], tt[3];
    long long f[3];
    for (int i = 0; i < 3; ++i) {
      g[i] = a.k[j] * (P[i] / r - a.e[i]) / a.dq;
      const double fl = floor(g[i]);
      f[i] = (long long)fl;
      tt[i] = g[i] - fl;
    }
    double cz[2][2];
    for (int di = 0; di < 2; ++di)
      for (int dj = 0; dj < 2; ++dj) {
        const double i0 = ewald_intensity<T>(a, f[0] + di, f[1] + dj, f[2]);
        const double i1 = ewald_intensity<T>(a, f[0] + di, f[1] + dj, f[2] + 1);
        cz[di][dj] = i0 + tt[2] * (i1 - i0);
      }
    const double c0 = cz[0][0] + tt[1] * (cz[0][1] - cz[0][0]);
    const double c1 = cz[1][0] + tt[1] * (cz[1][1] - cz[1][0]);
    acc += a.w[j] * (c0 + tt[0] * (c1 - c0));
  }
  a.image[t] = acc;
}

hipError_t launch_ewald(int prec, const EwaldArgs& a, hipStream_t s) {
  const long long np = (long long)a.nu * a.nv;
  if (prec == 0) hipLaunchKernelGGL(k_ewald<float>, dim3(nblk_of(np, 256)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_ewald<double>, dim3(nblk_of(np, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
#endif

// Window w: the populated bins whose centres lie in [lo, hi]; a first scan
// finds the first and last of them (the baseline's ends), a second adds
// (mean - baseline) * width and mean * width in bin order.
#if UR_IN(0)
__global__ void k_peaks(PeakArgs a) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= a.nwin) return;
  const double lo = a.lo[w], hi = a.hi[w];
  int first = -1, last = -1, cnt = 0;
  for (int b = 0; b < a.nbins; ++b) {
    const double q = 0.5 * (a.edges[b] + a.edges[b + 1]);
    if (q < lo || q > hi || isnan(a.mean[b])) continue;
    if (first < 0) first = b;
    last = b;
    ++cnt;
  }
  double peak = NAN, total = NAN;
  if (cnt >= 2) {
    const double q0 = 0.5 * (a.edges[first] + a.edges[first + 1]), q1 = 0.5 * (a.edges[last] + a.edges[last + 1]);
    const double m0 = a.mean[first], slope = (a.mean[last] - m0) / (q1 - q0);
    peak = 0.0;
    total = 0.0;
    for (int b = first; b <= last; ++b) {
      if (isnan(a.mean[b])) continue;
      const double q = 0.5 * (a.edges[b] + a.edges[b + 1]), d = a.edges[b + 1] - a.edges[b];
      peak += (a.mean[b] - (m0 + slope * (q - q0))) * d;
      total += a.mean[b] * d;
    }
  }
  a.out[3 * w] = peak;
  a.out[3 * w + 1] = total;
  a.out[3 * w + 2] = (double)cnt;
}

hipError_t launch_peaks(const PeakArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_peaks, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ensemble(int nboxes, int nbins, const double* mean, const double* sem, const double* w,
                           double* out_mean, double* out_sem, hipStream_t s) {
  hipLaunchKernelGGL(k_ensemble, dim3(nblk_of(nbins, 256)), dim3(256), 0, s, nboxes, nbins, mean, sem, w, out_mean, out_sem);
  return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_merge, dim3(nblk_of(a.nbins, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_chi2(int nbins, const double* mean, const double* count, const double* target, double rel_sigma,
                       double* out, double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_chi2, dim3(1), dim3(256), 0, s, nbins, mean, count, target, rel_sigma, out, g);
  return hipGetLastError();
}

#endif
template <typename T, int N>
static hipError_t pass_x_adj_t(const XAdjArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if constexpr (!inv_fits<T, N>()) { return hipErrorNotSupported; } else {
  size_t shm = ((size_t)a.nbins + 2) * sizeof(double) + ((size_t)a.nbins + 2) * sizeof(int) + (size_t)a.nlut * sizeof(short);
  hipLaunchKernelGGL((k_pass_x_adj<T, N>), dim3(nblocks), dim3(XCfg<N>::threads), shm, s, a);
  return hipGetLastError();
  }
}

#if UR_IN(6)
hipError_t launch_pass_x_adj(int prec, int n, const XAdjArgs& a, int nblocks, hipStream_t s) {
#define UR_XA(NN) return prec == 0 ? pass_x_adj_t<float, NN>(a, nblocks, s) : pass_x_adj_t<double, NN>(a, nblocks, s)
  UR_DISPATCH_N(n, UR_XA);
#undef UR_XA
}
#endif

template <typename T, int N>
static hipError_t pass_y_inv_t(const YInvArgs& a, hipStream_t s) {
  if constexpr (!inv_fits<T, N>()) { return hipErrorNotSupported; } else {
  long long nb = (long long)a.nkz * a.nxt;
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_pass_y_inv<T, N>), dim3((unsigned)nb), dim3(YICfg<T, N>::threads), 0, s, a);
  return hipGetLastError();
  }
}

#if UR_IN(5)
hipError_t launch_pass_y_inv(int prec, int n, const YInvArgs& a, hipStream_t s) {
#define UR_YI(NN) return prec == 0 ? pass_y_inv_t<float, NN>(a, s) : pass_y_inv_t<double, NN>(a, s)
  UR_DISPATCH_N(n, UR_YI);
#undef UR_YI
}
#endif

template <typename T, int N>
static hipError_t pass_z_inv_t(int c2c, const ZInvArgs& a, hipStream_t s) {
  if constexpr (!inv_fits<T, N>()) { return hipErrorNotSupported; } else {
  if (a.x0 < 0 || a.nx < 0 || a.x0 + a.nx > N) return hipErrorInvalidValue;
  unsigned nb = (unsigned)((long long)(a.nx > 0 ? a.nx : N) * a.ntiles);
  if (c2c) hipLaunchKernelGGL((k_pass_z_inv<T, N, true>), dim3(nb), dim3(ZICfg<T, N, true>::threads), 0, s, a);
  else hipLaunchKernelGGL((k_pass_z_inv<T, N, false>), dim3(nb), dim3(ZICfg<T, N, false>::threads), 0, s, a);
  return hipGetLastError();
  }
}

#if UR_IN(5)
hipError_t launch_pass_z_inv(int prec, int n, int c2c, const ZInvArgs& a, hipStream_t s) {
#define UR_ZI(NN) return prec == 0 ? pass_z_inv_t<float, NN>(c2c, a, s) : pass_z_inv_t<double, NN>(c2c, a, s)
  UR_DISPATCH_N(n, UR_ZI);
#undef UR_ZI
}
#endif

#if UR_IN(0)
hipError_t launch_fold(int prec, int n, const FoldArgs& a, int nblocks, hipStream_t s) {
  const int c3 = a.L.c * a.L.c * a.L.c;
  const bool lds = a.L.c <= 16;
  size_t shm = lds ? (size_t)c3 * sizeof(double) : 0;
  if (prec == 0) {
    if (lds) hipLaunchKernelGGL((k_fold<float, true>), dim3(nblocks), dim3(256), shm, s, a, n);
    else hipLaunchKernelGGL((k_fold<float, false>), dim3(nblocks), dim3(256), shm, s, a, n);
  } else {
    if (lds) hipLaunchKernelGGL((k_fold<double, true>), dim3(nblocks), dim3(256), shm, s, a, n);
    else hipLaunchKernelGGL((k_fold<double, false>), dim3(nblocks), dim3(256), shm, s, a, n);
  }
  return hipGetLastError();
}
#endif

#if UR_IN(0)
hipError_t launch_fold_rot(int prec, int n, const ZArgs& a, const void* g, double* part, int nblocks, hipStream_t s) {
  const int c = a.L.c;
  if (c > 16 || a.L.f != 1 || !a.rotated) return hipErrorInvalidValue;
  const size_t shm = (size_t)c * c * c * sizeof(double);
#define UR_FR(TT, I, G) hipLaunchKernelGGL((k_fold_rot<TT, I, G>), dim3(nblocks), dim3(kFoldRotThreads), shm, s, a, g, part, n)
#define UR_FRT(TT)                                        \
  if (a.cubic) {                                          \
    if (a.ngrain) UR_FR(TT, 3, true); else UR_FR(TT, 3, false); \
  } else {                                                \
    if (a.ngrain) UR_FR(TT, 1, true); else UR_FR(TT, 1, false); \
  }
  if (prec == 0) { UR_FRT(float) } else { UR_FRT(double) }
#undef UR_FRT
#undef UR_FR
  return hipGetLastError();
}
#endif

template <typename T, int N>
static hipError_t pass_z_fold_t(const ZFoldArgs& a, int nblocks, hipStream_t s) {
  if constexpr (!inv_fits<T, N>()) { return hipErrorNotSupported; } else {
    if (a.L.c <= 16 && nblocks % a.L.c != 0) return hipErrorInvalidValue;   // blocks per cell class
    size_t shm = a.L.c <= 16 ? (size_t)a.L.c * a.L.c * sizeof(double) : 0;
    hipLaunchKernelGGL((k_pass_z_fold<T, N>), dim3(nblocks), dim3(ZICfg<T, N, false>::threads), shm, s, a);
    return hipGetLastError();
  }
}

#if UR_IN(6)
hipError_t launch_pass_z_fold(int prec, int n, const ZFoldArgs& a, int nblocks, hipStream_t s) {
#define UR_ZF(NN) return prec == 0 ? pass_z_fold_t<float, NN>(a, nblocks, s) : pass_z_fold_t<double, NN>(a, nblocks, s)
  UR_DISPATCH_N(n, UR_ZF);
#undef UR_ZF
}
#endif

#if UR_IN(0)
// gcell[(ci c + cj) c + k] = sum over the blocks of class ci (b = r c + ci)
// of their slice partial [cj][k], in a fixed order
__global__ void k_fold_reduce_classes(int c, const double* __restrict__ part, int nblk, double* __restrict__ gcell) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int c2 = c * c;
  if (v >= c2 * c) return;
  const int ci = v / c2, rest = v % c2;
  Kahan k;
  for (int b = ci; b < nblk; b += c) k.add(part[(size_t)b * c2 + rest]);
  gcell[v] = k.val();
}

hipError_t launch_fold_reduce_classes(int c, const double* part, int nblk, double* gcell, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_reduce_classes, dim3(nblk_of((long long)c * c * c, 256)), dim3(256), 0, s, c, part, nblk, gcell);
  return hipGetLastError();
}

hipError_t launch_fold_reduce(int c3, const double* part, int nblk, double* gcell, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_reduce, dim3(nblk_of(c3, 256)), dim3(256), 0, s, c3, part, nblk, gcell);
  return hipGetLastError();
}

hipError_t launch_grad_amp(int c, int n_atoms, const double* prof, const double* gcell, double* grad_amp, hipStream_t s) {
  if (n_atoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_amp, dim3(n_atoms), dim3(256), 0, s, c, prof, gcell, grad_amp);
  return hipGetLastError();
}

// Periodic cubic B-spline coefficients along one axis of the c^3 cell, in
// place, one thread per line.  The cell values s and coefficients C satisfy
// (C[k-1] + 4 C[k] + C[k+1]) / 6 = s[k] (indices mod c).  With z = sqrt(3) - 2
// (z + 1/z = -4) the operator factors as -(1/z)(1 - z E^-1)(1 - z E), so
// C = -6 z w with y[k] = s[k] + z y[k-1] (causal) and w[k] = y[k] + z w[k+1]
// (anticausal); the periodic starts are the geometric sums
// y[0] = sum_m z^m s[-m] / (1 - z^c) and w[c-1] = sum_m z^m y[c-1+m] / (1 - z^c).
__global__ void __launch_bounds__(256) k_bspline_axis(double* __restrict__ cell, int c, int axis) {
  const int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= c * c) return;
  const size_t st = axis == 2 ? 1 : (axis == 1 ? (size_t)c : (size_t)c * c);
  const size_t base = axis == 2 ? (size_t)line * c
                    : (axis == 1 ? (size_t)(line / c) * c * c + line % c : (size_t)line);
  double* x = cell + base;
  const double z = 1.7320508075688772935 - 2.0;
  double zc = 1.0, y0 = 0.0;
  for (int m = 0; m < c; ++m) {
    y0 += zc * x[(size_t)((c - m) % c) * st];
    zc *= z;
  }
  y0 /= 1.0 - zc;
  x[0] = y0;
  for (int k = 1; k < c; ++k) x[(size_t)k * st] += z * x[(size_t)(k - 1) * st];
  double zm = 1.0, wl = 0.0;
  for (int m = 0; m < c; ++m) {
    wl += zm * x[(size_t)((c - 1 + m) % c) * st];
    zm *= z;
  }
  wl /= 1.0 - zc;
  x[(size_t)(c - 1) * st] = wl;
  for (int k = c - 2; k >= 0; --k) x[(size_t)k * st] += z * x[(size_t)(k + 1) * st];
  for (int k = 0; k < c; ++k) x[(size_t)k * st] *= -6.0 * z;
}

hipError_t launch_bspline_cell(int c, double* cell, hipStream_t s) {
  const int lines = c * c;
  for (int axis = 0; axis < 3; ++axis) {
    hipLaunchKernelGGL(k_bspline_axis, dim3((lines + 255) / 256), dim3(256), 0, s, cell, c, axis);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

#endif
// A level's density as complex values (rho, 0) for the mixed-radix passes
// (zoom levels there: block sums of ED-1), one block per (x, y) pencil, with
// the pencil's [sum rho, sum rho^2] (fixed-order block sum) in mom.
template <typename T>
__global__ void __launch_bounds__(256) k_level_complex(ZArgs a, int n, cx<T>* __restrict__ S, double* __restrict__ mom) {
  __shared__ double r1[256], r2[256];
  const long long t = blockIdx.x;
  Pencil<T> p;
  p.init(a, t / n, t % n);
  cx<T>* row = S + t * n;
  double s1 = 0.0, s2 = 0.0;
  for (int z = threadIdx.x; z < n; z += 256) {
    const T v = p.value(a, z);
    row[z] = mk(v, (T)0);
    s1 += (double)v;
    s2 += (double)v * (double)v;
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u1 = 0.0, u2 = 0.0;
    for (int i = 0; i < 256; ++i) { u1 += r1[i]; u2 += r2[i]; }
    mom[2 * t] = u1;
    mom[2 * t + 1] = u2;
  }
}

#if UR_IN(0)
hipError_t launch_level_complex(int prec, int n, const ZArgs& a, void* S, double* mom, hipStream_t s) {
  const unsigned nn = (unsigned)((long long)n * n);
  if (prec == 0) hipLaunchKernelGGL(k_level_complex<float>, dim3(nn), dim3(256), 0, s, a, n, (cx<float>*)S, mom);
  else hipLaunchKernelGGL(k_level_complex<double>, dim3(nn), dim3(256), 0, s, a, n, (cx<double>*)S, mom);
  return hipGetLastError();
}

template <typename T>
static void zoom_rot_launch(unsigned nn, const ZArgs& a, int n, int x_lo, void* rho, hipStream_t s) {
  if (a.cubic) {
    if (a.ngrain) hipLaunchKernelGGL((k_zoom_rot<T, 3, true>), dim3(nn), dim3(256), 0, s, a, n, x_lo, (T*)rho);
    else hipLaunchKernelGGL((k_zoom_rot<T, 3, false>), dim3(nn), dim3(256), 0, s, a, n, x_lo, (T*)rho);
  } else {
    if (a.ngrain) hipLaunchKernelGGL((k_zoom_rot<T, 1, true>), dim3(nn), dim3(256), 0, s, a, n, x_lo, (T*)rho);
    else hipLaunchKernelGGL((k_zoom_rot<T, 1, false>), dim3(nn), dim3(256), 0, s, a, n, x_lo, (T*)rho);
  }
}

hipError_t launch_rho_generate(int prec, int n, int x_lo, int x_hi, const ZArgs& a, void* rho, hipStream_t s) {
  const unsigned nn = (unsigned)((long long)(x_hi - x_lo + 1) * n);
  if (a.rotated && a.L.f > 1) {                        // zoom level of an oriented lattice
    if (n > kZoomRotMaxBox) return hipErrorNotSupported;
    if (prec == 0) zoom_rot_launch<float>(nn, a, n, x_lo, rho, s);
    else zoom_rot_launch<double>(nn, a, n, x_lo, rho, s);
    return hipGetLastError();
  }
  if (prec == 0) hipLaunchKernelGGL(k_rho_generate<float>, dim3(nn), dim3(256), 0, s, a, n, x_lo, (float*)rho);
  else hipLaunchKernelGGL(k_rho_generate<double>, dim3(nn), dim3(256), 0, s, a, n, x_lo, (double*)rho);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  size_t n = bytes / sizeof(double);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (double*)p, n);
  return hipGetLastError();
}

// Stockham stage sequence (L, R) of a length-n column, as the kernels run it
template <int N>
static int stages_t(int* Ls, int* Rs) {
  int k = 0;
  for (int l = 1; l < N; l *= radix_at<N>(l)) { Ls[k] = l; Rs[k] = radix_at<N>(l); ++k; }
  return k;
}
int fft_stages(int n, int* Ls, int* Rs) {
  switch (n) {
    case 16: return stages_t<16>(Ls, Rs); case 32: return stages_t<32>(Ls, Rs);
    case 64: return stages_t<64>(Ls, Rs); case 128: return stages_t<128>(Ls, Rs);
    case 256: return stages_t<256>(Ls, Rs); case 512: return stages_t<512>(Ls, Rs);
    case 1024: return stages_t<1024>(Ls, Rs); case 2048: return stages_t<2048>(Ls, Rs);
    case kBig: return stages_t<kBig>(Ls, Rs);
#define UR_MR_CASE(NN) case NN: return stages_t<NN>(Ls, Rs);
    UR_MR_SIZES(UR_MR_CASE)
#undef UR_MR_CASE
    default: return 0;
  }
}

// tile geometry for the planner
#define UR_TILE(NN) { if (prec == 0) return c2c ? ZCfg<float, NN, true>::TY : ZCfg<float, NN, false>::TY; \
                      return c2c ? ZCfg<double, NN, true>::TY : ZCfg<double, NN, false>::TY; }
int z_tile(int prec, int n, int c2c) {
  if (n == kBig) return prec == 0 && !c2c ? ZCfg<float, kBig, false>::TY : 0;
  switch (n) {
    case 16: UR_TILE(16) case 32: UR_TILE(32) case 64: UR_TILE(64) case 128: UR_TILE(128)
    case 256: UR_TILE(256) case 512: UR_TILE(512) case 1024: UR_TILE(1024) case 2048: UR_TILE(2048)
    default: return 0;
  }
}
#undef UR_TILE
#define UR_ZITILE(NN) { if (prec == 0) return c2c ? ZICfg<float, NN, true>::TY : ZICfg<float, NN, false>::TY; \
                        return c2c ? ZICfg<double, NN, true>::TY : ZICfg<double, NN, false>::TY; }
int zinv_tile(int prec, int n, int c2c) {
  switch (n) {
    case 16: UR_ZITILE(16) case 32: UR_ZITILE(32) case 64: UR_ZITILE(64) case 128: UR_ZITILE(128)
    case 256: UR_ZITILE(256) case 512: UR_ZITILE(512) case 1024: UR_ZITILE(1024) case 2048: UR_ZITILE(2048)
    default: return 0;
  }
}
#undef UR_ZITILE

#define UR_YT(NN) return prec == 0 ? YCfg<float, NN>::TX : YCfg<double, NN>::TX
int y_tile(int prec, int n) {
  if (n == kBig) return prec == 0 ? YCfg<float, kBig>::TX : 0;
  switch (n) {
    case 16: UR_YT(16); case 32: UR_YT(32); case 64: UR_YT(64); case 128: UR_YT(128);
    case 256: UR_YT(256); case 512: UR_YT(512); case 1024: UR_YT(1024); case 2048: UR_YT(2048);
    default: return 0;
  }
}
#undef UR_YT

#define UR_XG(NN) return XCfg<NN>::NG
int x_groups(int n) {
  switch (n) {
    case 16: UR_XG(16); case 32: UR_XG(32); case 64: UR_XG(64); case 128: UR_XG(128);
    case 256: UR_XG(256); case 512: UR_XG(512); case 1024: UR_XG(1024); case 2048: UR_XG(2048);
    case kBig: UR_XG(kBig);
    default: return 0;
  }
}
#undef UR_XG

#endif

}  // namespace ur
