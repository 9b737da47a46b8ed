// Mixed-radix boxes (edges 2^a 3^b 5^c that are not powers of two): the
// in-place axis passes with the density generated in the first and |F|^2
// binned in the last, and the binning of a given spectrum.
#include <hip/hip_runtime.h>

#include "ur_device.hpp"
#include "ur_geom.hpp"
#include "ur_kernels.hpp"

namespace ur {

// ---------------------------------------------------------------------------
// mixed-radix boxes (n = 2^a 3^b 5^c, not a power of two)
// A block holds TL whole lines of one axis in LDS (padded columns), every
// line transformed by G lanes in a slot of GP = 2^ceil(log2 G) lanes (so a
// line never straddles two wavefronts), then written back in place.  Lines
// along z are contiguous, so a tile is TL n consecutive elements; lines
// along y and x are taken TL consecutive z at a time, so every load and
// store is a TL-element contiguous segment.
// Real boxes (R2C): the z pass packs two real pencils into one complex line
// (the first as real, the second as imaginary part), transforms it and
// unpacks the two half spectra, A_k = (Z_k + conj Z_{N-k}) / 2 and
// B_k = (Z_k - conj Z_{N-k}) / 2i for k in [0, N/2], into a box of
// N x N x (N/2 + 1) elements ([x][y][kz], then [kx][ky][kz] after the x
// pass); the y and x passes take lines of that box, and the binning counts
// kz in (0, N/2) twice (the conjugate half).
// ---------------------------------------------------------------------------
#ifndef UR_MR_CAP
#define UR_MR_CAP 0
#endif
// LDS of a tile outside the binning pass (72 KB: two blocks per CU; 144 KB,
// one block of 16 lines and 128-byte segments along y and x: 1000^3 8.50 ms
// per box against 7.65, the y pass 3 % faster and the z pass 53 % slower)
#ifndef UR_MR_TILE_KB
#define UR_MR_TILE_KB 72
#endif
constexpr int floor_pow2(int v) { int p = 1; while (2 * p <= v) p *= 2; return p; }
constexpr int ceil_pow2(int v) { int p = 1; while (p < v) p *= 2; return p; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Lines per tile: at most 64 (and 1024 threads), within 72 KB of LDS so that
// two blocks share a CU, but at least 8 (64-byte segments along y and x)
// when 144 KB allow it; the binning x pass keeps 76 KB for the tile so the
// histogram and its thresholds (up to 4096 bins: 82 KB) fit beside it.
template <typename T, int N, bool BIN> struct MrCfg {
  static constexpr int G = Geo<N>::G, GP = ceil_pow2(G);
  static constexpr int PS = Padded<N>::size, LB = PS * (int)sizeof(cx<T>);
  static constexpr int TL0 = cmin(64, 1024 / GP);
  static constexpr int TLa = floor_pow2(cmin(TL0, (BIN ? 76 * 1024 : UR_MR_TILE_KB * 1024) / LB > 0 ? (BIN ? 76 * 1024 : UR_MR_TILE_KB * 1024) / LB : 1));
  static constexpr int TLb = floor_pow2(cmin(cmin(TL0, 8), (144 * 1024) / LB > 0 ? (144 * 1024) / LB : 1));
  static constexpr int TL = (BIN || TLa >= 8) ? TLa : (TLb > TLa ? TLb : TLa);
  static constexpr int threads = TL * GP < 64 ? 64 : TL * GP;
  // UR_MR_CAP: FP32 lines of up to 24 elements per lane get registers for
  // two blocks per CU (the LDS holds two tiles; unbounded, the compiler
  // takes up to 256 VGPRs and leaves one block per CU).  Off: at 1000
  // points the cap spills 400-500 bytes per lane and the y pass of a
  // 1000^3 box takes 9.1 ms instead of 5.0.
  static constexpr int minw = (UR_MR_CAP && sizeof(T) == 4 && Geo<N>::E <= 24) ? cmin(4, threads / 128 > 0 ? threads / 128 : 1) : 1;
  // twiddles of a stage loaded ahead of it (more registers, more overlap),
  // except where the blocks the LDS holds per CU need 128 VGPRs or fewer
  // (16 waves): FP32 tiles load them at each butterfly there (1000^3: 11.0 ms
  // per box against 14.4 with the hoist; 2000^3, one block of 8 waves or two
  // of 4: 112 ms against 129 without it)
  static constexpr int BPC = (160 * 1024) / (TL * LB) > 0 ? (160 * 1024) / (TL * LB) : 1;
  static constexpr bool twh = sizeof(T) != 4 || BPC * threads < 1024;
  static_assert(G <= 64, "mixed-radix lines lie in one wavefront");
  static_assert(threads % 64 == 0 && TL * LB <= 144 * 1024, "tile exceeds the LDS");
};

template <typename T, int N, int AXIS, int MODE, bool R2C>
__host__ __device__ constexpr long long mr_tiles() {
  constexpr int TL = MrCfg<T, N, MODE == MR_BIN>::TL;
  constexpr long long LINES2 = R2C ? (long long)N * N / 2 : (long long)N * N;   // z lines (pencil pairs)
  constexpr int NZ = R2C ? N / 2 + 1 : N;                                        // extent of the third index
  return AXIS == 2 ? (LINES2 + TL - 1) / TL : (long long)N * ((NZ + TL - 1) / TL);
}

template <typename T, int N, int DIR, int AXIS, int MODE, bool R2C>
__global__ void __launch_bounds__((MrCfg<T, N, MODE == MR_BIN>::threads), (MrCfg<T, N, MODE == MR_BIN>::minw)) k_mr_axis(MrArgs a) {
  using C = MrCfg<T, N, MODE == MR_BIN>;
  constexpr int G = C::G, GP = C::GP, TL = C::TL, PS = C::PS, NT = C::threads;
  constexpr int E = Geo<N>::E, R0 = Radix<N, 1>::r, NB0 = E / R0;
  // loads in flight per thread: 16 FP32 elements outside the binning pass
  // (32 VGPRs), else 8
  constexpr int U = cmin(sizeof(T) == 4 && MODE != MR_BIN ? 16 : 8, (TL * N + NT - 1) / NT);
  constexpr int NZ = R2C ? N / 2 + 1 : N;              // extent of the third index of the box
  constexpr int NZT = (NZ + TL - 1) / TL;
  const int NZP = R2C && a.nzp > 0 ? a.nzp : NZ;       // its row pitch
  // tiles of this launch: the whole box, or the lines / planes given
  const long long NTILE = AXIS == 2 ? (a.lines > 0 ? (a.lines + TL - 1) / TL : mr_tiles<T, N, AXIS, MODE, R2C>())
                        : AXIS == 1 ? (long long)(a.planes > 0 ? a.planes : N) * NZT
                                    : mr_tiles<T, N, AXIS, MODE, R2C>();
  const long long LINES = a.lines > 0 ? a.lines : (R2C ? (long long)N * N / 2 : (long long)N * N);
  const int XA = a.xn > 0 ? a.xa : 0, XN = a.xn > 0 ? a.xn : N;   // stored x planes (x pass)
  static_assert(MODE != MR_GEN || AXIS == 2, "generation feeds the z pass");
  static_assert(MODE != MR_BIN || (AXIS == 0 && DIR < 0), "binning follows the forward x pass");
  static_assert(!R2C || DIR < 0, "real boxes run the forward transform");
  __shared__ cx<T> lds[TL * PS];
  // MR_BIN: 2 nbins + 1 sums, then the thresholds Us[b + 1] = U[b] for b in
  // [0, nbins] between two sentinels (Us[0] below every n2, Us[nbins + 2]
  // above), so the bin walk reads LDS and needs no range tests
  extern __shared__ double hist[];
  const cx<T>* __restrict__ src = (const cx<T>*)a.src;
  cx<T>* __restrict__ dst = (cx<T>*)a.dst;
  const int t = threadIdx.x;
  const int nv = 2 * a.nbins + 1;
  int* Us = (int*)(hist + nv);
  if constexpr (MODE == MR_BIN) {
    for (int i = t; i < nv; i += NT) hist[i] = 0.0;
    for (int i = t; i <= a.nbins; i += NT) Us[i + 1] = a.U[i];
    if (t == 0) { Us[0] = -1; Us[a.nbins + 2] = 0x7fffffff; }
  }
  double s1 = 0.0, s2 = 0.0, tot = 0.0;
  for (long long tile = blockIdx.x; tile < NTILE; tile += gridDim.x) {
    // the thread index is made opaque in every tile, so that the index
    // arithmetic of the loads, stores and transform stages (which depends on
    // the lane only) is not hoisted out of the tile loop into live registers
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    size_t base, es;
    int nl, o = 0, z0 = 0;
    if constexpr (AXIS == 2) {
      // complex: lines l0 .. l0 + nl - 1; real: pencil pairs, line l holding
      // pencils 2 (l0 + l) and 2 (l0 + l) + 1 (same x, adjacent y: N is even)
      const long long l0 = tile * TL;
      const long long left = LINES - l0;
      nl = left < TL ? (int)left : TL;
      base = (size_t)l0 * N * (R2C ? 2 : 1);
      es = 1;
    } else {
      constexpr int nzt = NZT;
      o = (AXIS == 1 ? a.px0 : 0) + (int)(tile / nzt);
      z0 = (int)(tile % nzt) * TL;
      nl = NZ - z0 < TL ? NZ - z0 : TL;
      base = AXIS == 1 ? (size_t)o * N * NZP + z0 : (size_t)o * NZP + z0;
      es = AXIS == 1 ? (size_t)NZP : (size_t)N * NZP;
    }
    if constexpr (AXIS == 2) {
      // pruned box: a tile none of whose pencils can hold density is skipped
      // (block-uniform: the barrier's OR), its lines left unwritten
      if (a.prune) {
        bool has = false;
        if (t < nl) {
          const long long line = tile * TL + t;
          const long long X = R2C ? (2 * line) / N : line / N, Y = R2C ? (2 * line) % N : line % N;
          long long lo, hi;
          row_range(a.z.L, a.z.m, X, lo, hi);
          has = Y + (R2C ? 1 : 0) >= lo && Y <= hi;
        }
        if (!__syncthreads_or(has)) continue;
      }
    }
    // pruned y pass: rows of plane o outside its row range read as zero
    int ylo = 0, yhi = N - 1;
    if (AXIS == 1 && a.prune) {
      long long lo, hi;
      row_range(a.z.L, a.z.m, o, lo, hi);
      ylo = (int)lo;
      yhi = (int)hi;
    }
    if constexpr (MODE == MR_GEN) {
      // every lane of a line's slot generates elements g, g + GP, ... of it
      const int l = t / GP, g = t % GP;
      if (l < nl) {
        // aligned lattice (rotated lattices refused), level factor 1: the
        // cell row of the pencil, inside the mask's z range
        const long long line = tile * TL + l;
        const Level& L = a.z.L;
        // periodic cell index by a true modulo: any cell edge
        const int c = L.c;
        auto wrap = [c](long long v) { const long long r = v % c; return (int)(r < 0 ? r + c : r); };
        const int zoff = -(int)(L.o + L.h);
        cx<T>* col = lds + l * PS;
        // cell index of element e: wrap(e + zoff), advanced by GP mod c per
        // step (32-bit adds instead of a 64-bit remainder per element)
        const int cstep = GP % c;
        int ci = wrap(g + zoff);
        if constexpr (R2C) {
          const long long X = (2 * line) / N, Y = (2 * line) % N;
          long long lo, hi, lo1, hi1;
          col_range(L, a.z.m, X, Y, lo, hi);
          col_range(L, a.z.m, X, Y + 1, lo1, hi1);
          const T* row = (const T*)a.z.cellT + ((size_t)wrap(X - L.o - L.h) * c + wrap(Y - L.o - L.h)) * c;
          const T* row1 = (const T*)a.z.cellT + ((size_t)wrap(X - L.o - L.h) * c + wrap(Y + 1 - L.o - L.h)) * c;
          const int ilo = (int)lo, ihi = (int)hi, ilo1 = (int)lo1, ihi1 = (int)hi1;
          if (cstep == 0) {
            // the cell edge divides the slot width: every element of this lane
            // takes the same cell value of each pencil
            const T cv = row[ci], cv1 = row1[ci];
            for (int e = g; e < N; e += GP) {
              const T v = (e >= ilo && e <= ihi) ? cv : (T)0;
              const T v1 = (e >= ilo1 && e <= ihi1) ? cv1 : (T)0;
              col[pad(e)] = mk(v, v1);
              s1 += (double)v + (double)v1;
              s2 += (double)v * (double)v + (double)v1 * (double)v1;
            }
          } else {
            for (int e = g; e < N; e += GP) {
              const T v = (e >= ilo && e <= ihi) ? row[ci] : (T)0;
              const T v1 = (e >= ilo1 && e <= ihi1) ? row1[ci] : (T)0;
              col[pad(e)] = mk(v, v1);
              s1 += (double)v + (double)v1;
              s2 += (double)v * (double)v + (double)v1 * (double)v1;
              ci += cstep;
              if (ci >= c) ci -= c;
            }
          }
        } else {
          const long long X = line / N, Y = line % N;
          long long lo, hi;
          col_range(L, a.z.m, X, Y, lo, hi);
          const T* row = (const T*)a.z.cellT + ((size_t)wrap(X - L.o - L.h) * c + wrap(Y - L.o - L.h)) * c;
          const int ilo = (int)lo, ihi = (int)hi;
          if (cstep == 0) {
            const T cv = row[ci];
            for (int e = g; e < N; e += GP) {
              const T v = (e >= ilo && e <= ihi) ? cv : (T)0;
              col[pad(e)] = mk(v, (T)0);
              s1 += (double)v;
              s2 += (double)v * (double)v;
            }
          } else {
            for (int e = g; e < N; e += GP) {
              const T v = (e >= ilo && e <= ihi) ? row[ci] : (T)0;
              col[pad(e)] = mk(v, (T)0);
              s1 += (double)v;
              s2 += (double)v * (double)v;
              ci += cstep;
              if (ci >= c) ci -= c;
            }
          }
        }
      }
    } else if constexpr (AXIS == 2 && R2C) {
      // two real pencils per line: 2 nl N consecutive reals
      const T* __restrict__ rs = (const T*)a.src;
      constexpr int TOT = 2 * TL * N;
      for (int i0 = 0; i0 < TOT; i0 += NT * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * NT + t;
          if (i < 2 * nl * N) v[u] = rs[base + i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * NT + t;
          if (i < 2 * nl * N) {
            const int j = i / N, e = i % N;
            cx<T>& d = lds[(j >> 1) * PS + pad(e)];
            if (j & 1) d.y = v[u]; else d.x = v[u];
            if (a.mom) { s1 += (double)v[u]; s2 += (double)v[u] * v[u]; }
          }
        }
      }
    } else if constexpr (AXIS == 2) {
      constexpr int TOT = TL * N;
      for (int i0 = 0; i0 < TOT; i0 += NT * U) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * NT + t;
          if (i < nl * N) v[u] = src[base + i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * NT + t;
          if (i < nl * N) {
            lds[(i / N) * PS + pad(i % N)] = v[u];
            if (a.mom) { s1 += (double)v[u].x; s2 += (double)v[u].x * v[u].x + (double)v[u].y * v[u].y; }
          }
        }
      }
    } else {
      constexpr int TOT = TL * N;
      for (int i0 = 0; i0 < TOT; i0 += NT * U) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * NT + t;
          if (i < TOT && i % TL < nl) {
            if constexpr (AXIS == 0) {
              // element e of the x line: stored planes [XA, XA + XN) only
              const int e = i / TL;
              v[u] = (e >= XA && e < XA + XN) ? src[base + (size_t)(e - XA) * es + i % TL] : mk((T)0, (T)0);
            } else {
              const int e = i / TL;
              v[u] = (e >= ylo && e <= yhi) ? src[base + (size_t)e * es + i % TL] : mk((T)0, (T)0);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * NT + t;
          if (i < TOT && i % TL < nl) {
            lds[(i % TL) * PS + pad(i / TL)] = v[u];
            if (a.mom) { s1 += (double)v[u].x; s2 += (double)v[u].x * v[u].x + (double)v[u].y * v[u].y; }
          }
        }
      }
    }
    __syncthreads();
    {
      const int l = t / GP, g = t % GP;
      if (l < nl && g < G) {
        cx<T>* col = lds + l * PS;
        cx<T> v[E];
#pragma unroll
        for (int i = 0; i < NB0; ++i)
#pragma unroll
          for (int r = 0; r < R0; ++r) v[i * R0 + r] = col[pad(first_index<N>(g, i, r))];
        wave_sync();
        fft_column<T, N, DIR, C::twh>(col, g, (const cx<T>*)a.tw, v);
      }
    }
    __syncthreads();
    if constexpr (MODE == MR_BIN) {
      // element (kx, ky = o, kz = z0 + l) of the spectrum, scaled by 1/n^3.
      // Lane g of line l's slot takes |h| in [g CH, (g + 1) CH), both signs
      // (kx = |h| and n - |h|), walking |h| upward so that n2 and the bin
      // index never decrease: runs of equal bin are summed in registers,
      // one LDS atomic pair per run, the next threshold held in a register.
      constexpr int CH = (N / 2 + GP) / GP;              // |h| in [0, N/2] over GP lanes
      const int l = t / GP, g = t % GP;
      if (l < nl) {
        const int k = sidx(o, N), lz = sidx(z0 + l, N);
        const int base2 = k * k + lz * lz;
        // real boxes: kz in (0, N/2) stands for its conjugate too
        const double wz = (R2C && z0 + l != 0 && 2 * (z0 + l) != N) ? 2.0 : 1.0;
        const T sc = (T)a.scale;
        const cx<T>* col = lds + l * PS;
        const int h0 = g * CH, h1 = h0 + CH < N / 2 + 1 ? h0 + CH : N / 2 + 1;
        if (h0 < h1) {
          // bin of the first |h| from the start-of-walk table, then forward
          const int n20 = h0 * h0 + base2;
          int b = a.lut[isqrt_ll(n20)];
          while (n20 >= Us[b + 2]) ++b;
          int nextU = Us[b + 2];
          int cur = b;
          double rs = 0.0, rs2 = 0.0;
          for (int ha = h0; ha < h1; ++ha) {
            const int n2 = ha * ha + base2;
            if (n2 >= nextU) {
              if (cur >= 0 && cur < a.nbins) { atomicAdd(&hist[2 * cur], wz * rs); atomicAdd(&hist[2 * cur + 1], wz * rs2); }
              rs = 0.0;
              rs2 = 0.0;
              ++b;
              while (n2 >= Us[b + 2]) ++b;
              nextU = Us[b + 2];
              cur = b;
            }
            const cx<T> f1 = scale(col[pad(ha)], sc);
            const double i1 = ((double)f1.x * f1.x + (double)f1.y * f1.y) * a.iscale;
            double i2 = 0.0;
            if (ha != 0 && 2 * ha != N) {                 // kx = n - |h| (the same voxel at 0 and n/2)
              const cx<T> f2 = scale(col[pad(N - ha)], sc);
              i2 = ((double)f2.x * f2.x + (double)f2.y * f2.y) * a.iscale;
            } else if (ha == 0 && base2 == 0 && o == 0 && z0 + l == 0) {
              a.f0[0] = (double)f1.x;
              a.f0[1] = (double)f1.y;
            }
            tot += wz * (i1 + i2);
            rs += i1 + i2;
            rs2 = fma(i1, i1, rs2);
            rs2 = fma(i2, i2, rs2);
          }
          if (cur >= 0 && cur < a.nbins) { atomicAdd(&hist[2 * cur], wz * rs); atomicAdd(&hist[2 * cur + 1], wz * rs2); }
        }
      }
    } else {
      const T sc = (T)a.scale;
      if constexpr (AXIS == 2 && R2C) {
        // unpack each line into its two pencils' half spectra: 2 nl rows of
        // N/2 + 1 elements, row pitch NZP
        const size_t ob = (size_t)(tile * TL) * 2 * NZP;
        for (int i = t; i < 2 * nl * NZ; i += NT) {
          const int j = i / NZ, k = i % NZ;
          const cx<T>* col = lds + (j >> 1) * PS;
          const cx<T> zk = col[pad(k)], zm = col[pad(k == 0 ? 0 : N - k)];
          const cx<T> r = (j & 1) ? mk((zk.y + zm.y) * (T)0.5, (zm.x - zk.x) * (T)0.5)
                                  : mk((zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5);
          dst[ob + (size_t)j * NZP + k] = scale(r, sc);
        }
      } else if constexpr (AXIS == 2) {
        for (int i = t; i < nl * N; i += NT) dst[base + i] = scale(lds[(i / N) * PS + pad(i % N)], sc);
      } else {
        for (int i = t; i < N * TL; i += NT) {
          const int e = i / TL, l2 = i % TL;
          if (l2 < nl) dst[base + e * es + l2] = scale(lds[l2 * PS + pad(e)], sc);
        }
      }
    }
    __syncthreads();
  }
  if (a.mom) {                                       // fixed-order block sum of the input values
    __shared__ double w1[NT / 64], w2[NT / 64];
    for (int o = 32; o > 0; o >>= 1) { s1 += __shfl_down(s1, o, 64); s2 += __shfl_down(s2, o, 64); }
    if (t % 64 == 0) { w1[t / 64] = s1; w2[t / 64] = s2; }
    __syncthreads();
    if (t == 0) {
      double u1 = 0.0, u2 = 0.0;
      for (int i = 0; i < NT / 64; ++i) { u1 += w1[i]; u2 += w2[i]; }
      a.mom[2 * (size_t)blockIdx.x] = u1;
      a.mom[2 * (size_t)blockIdx.x + 1] = u2;
    }
  }
  if constexpr (MODE == MR_BIN) {
    atomicAdd(&hist[nv - 1], tot);
    __syncthreads();
    for (int i = t; i < nv; i += NT) a.part[(size_t)blockIdx.x * nv + i] = hist[i];
  }
}

// blocks of a pass: one tile per block, except the binning pass, whose
// persistent blocks (at most kMrBinBlocks) each own one set of partials
constexpr int kMrBinBlocks = 1024;
template <typename T, int N, bool R2C> static long long mr_tiles_rt(int axis, int mode) {
  return axis == 2 ? mr_tiles<T, N, 2, 0, R2C>() : (mode == MR_BIN ? mr_tiles<T, N, 0, MR_BIN, R2C>() : mr_tiles<T, N, 1, 0, R2C>());
}
template <int N> static int mr_blocks_t(int prec, int axis, int mode, bool r2c) {
  long long nt;
  if (prec == 0) nt = r2c ? mr_tiles_rt<float, N, true>(axis, mode) : mr_tiles_rt<float, N, false>(axis, mode);
  else nt = r2c ? mr_tiles_rt<double, N, true>(axis, mode) : mr_tiles_rt<double, N, false>(axis, mode);
  return (int)(mode == MR_BIN ? (nt < kMrBinBlocks ? nt : kMrBinBlocks) : nt);
}

template <typename T, int N, int DIR, int AXIS, int MODE, bool R2C>
static hipError_t mr_launch(const MrArgs& a, int nblk, hipStream_t s) {
  const size_t shm = MODE == MR_BIN ? (2 * (size_t)a.nbins + 1) * sizeof(double) + ((size_t)a.nbins + 3) * sizeof(int) : 0;
  hipLaunchKernelGGL((k_mr_axis<T, N, DIR, AXIS, MODE, R2C>), dim3(nblk), dim3(MrCfg<T, N, MODE == MR_BIN>::threads), shm, s, a);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t mr_axis_t(int axis, int dir, int mode, bool r2c, const MrArgs& a, hipStream_t s) {
  if constexpr (N > 2048 && sizeof(T) != 4) {
    return hipErrorNotSupported;                     // edges above 2048: FP32 real plans only
  } else {
  int nblk = mr_blocks_t<N>(sizeof(T) == 4 ? 0 : 1, axis, mode, r2c);
  {
    // part of a box: one tile per block over the lines / planes given
    constexpr int TL = MrCfg<T, N, false>::TL, NZ1 = N / 2 + 1;
    if (axis == 2 && a.lines > 0 && mode != MR_BIN) nblk = (int)((a.lines + TL - 1) / TL);
    if (axis == 1 && a.planes > 0) nblk = a.planes * (((r2c ? NZ1 : N) + TL - 1) / TL);
  }
  if (nblk <= 0) return hipSuccess;
  if (r2c) {                                         // real boxes: forward only
    if (dir >= 0) return hipErrorInvalidValue;
    if (mode == MR_GEN) return axis == 2 ? mr_launch<T, N, -1, 2, MR_GEN, true>(a, nblk, s) : hipErrorInvalidValue;
    if (mode == MR_BIN) return axis == 0 ? mr_launch<T, N, -1, 0, MR_BIN, true>(a, nblk, s) : hipErrorInvalidValue;
    if (axis == 0) return mr_launch<T, N, -1, 0, MR_LOAD, true>(a, nblk, s);
    if (axis == 1) return mr_launch<T, N, -1, 1, MR_LOAD, true>(a, nblk, s);
    return mr_launch<T, N, -1, 2, MR_LOAD, true>(a, nblk, s);
  }
  if constexpr (N > 2048) {
    return hipErrorNotSupported;                     // complex plans run edges up to 2048
  } else {
    if (mode == MR_GEN) return axis == 2 && dir < 0 ? mr_launch<T, N, -1, 2, MR_GEN, false>(a, nblk, s) : hipErrorInvalidValue;
    if (mode == MR_BIN) return axis == 0 && dir < 0 ? mr_launch<T, N, -1, 0, MR_BIN, false>(a, nblk, s) : hipErrorInvalidValue;
    if (dir < 0) {
      if (axis == 0) return mr_launch<T, N, -1, 0, MR_LOAD, false>(a, nblk, s);
      if (axis == 1) return mr_launch<T, N, -1, 1, MR_LOAD, false>(a, nblk, s);
      return mr_launch<T, N, -1, 2, MR_LOAD, false>(a, nblk, s);
    }
    if (axis == 0) return mr_launch<T, N, 1, 0, MR_LOAD, false>(a, nblk, s);
    if (axis == 1) return mr_launch<T, N, 1, 1, MR_LOAD, false>(a, nblk, s);
    return mr_launch<T, N, 1, 2, MR_LOAD, false>(a, nblk, s);
  }
  }
}

bool mr_size(int n) {
  switch (n) {
#define UR_MR_CASE(NN) case NN:
    UR_MR_SIZES(UR_MR_CASE) return true;
#undef UR_MR_CASE
    default: return false;
  }
}

// z lines per tile of the loading and generating passes (the block count of
// a partial z pass is ceil(lines / that))
int mr_tile_lines(int prec, int n) {
  switch (n) {
#define UR_MR_CASE(NN) case NN: return prec == 0 ? MrCfg<float, NN, false>::TL : MrCfg<double, NN, false>::TL;
    UR_MR_SIZES(UR_MR_CASE)
#undef UR_MR_CASE
    default: return 0;
  }
}

int mr_axis_blocks(int prec, int n, int axis, int mode, bool r2c) {
  switch (n) {
#define UR_MR_CASE(NN) case NN: return mr_blocks_t<NN>(prec, axis, mode, r2c);
    UR_MR_SIZES(UR_MR_CASE)
#undef UR_MR_CASE
    default: return 0;
  }
}

hipError_t launch_mr_axis(int prec, int n, int axis, int dir, int mode, bool r2c, const MrArgs& a, hipStream_t s) {
  switch (n) {
#define UR_MR_CASE(NN) case NN: return prec == 0 ? mr_axis_t<float, NN>(axis, dir, mode, r2c, a, s) : mr_axis_t<double, NN>(axis, dir, mode, r2c, a, s);
    UR_MR_SIZES(UR_MR_CASE)
#undef UR_MR_CASE
    default: return hipErrorNotSupported;
  }
}

// |F|^2 of a full complex spectrum into integer-threshold |Q| bins: blocks
// stride over (kx, ky) rows, threads over kz; per-block partials of the
// sums and sums of squares (LDS FP64 atomics) and of the total intensity.
template <typename T>
__global__ void __launch_bounds__(256) k_mr_bin(MrBinArgs a) {
  extern __shared__ double hist[];                 // 2 nbins + 1
  const int nv = 2 * a.nbins + 1;
  for (int i = threadIdx.x; i < nv; i += 256) hist[i] = 0.0;
  __syncthreads();
  const cx<T>* __restrict__ S = (const cx<T>*)a.S;
  const int n = a.n;
  const int nz = a.r2c ? n / 2 + 1 : n;            // half spectrum: kz in [0, n/2], the rest conjugate
  double tot = 0.0;
  for (long long r = blockIdx.x; r < (long long)n * n; r += gridDim.x) {
    const int h = sidx((int)(r / n), n), k = sidx((int)(r % n), n);
    const int base = h * h + k * k;
    for (int z = threadIdx.x; z < nz; z += 256) {
      const cx<T> f = S[r * nz + z];
      if (r == 0 && z == 0) { a.f0[0] = (double)f.x; a.f0[1] = (double)f.y; }
      const int l = sidx(z, n);
      const int n2 = base + l * l;
      const double w = (a.r2c && z != 0 && 2 * z != n) ? 2.0 : 1.0;
      const double I = ((double)f.x * f.x + (double)f.y * f.y) * a.iscale;
      tot += w * I;
      int b = a.lut[isqrt_ll(n2)];
      while (b < a.nbins && n2 >= a.U[b + 1]) ++b;
      if (b >= 0 && b < a.nbins) {
        atomicAdd(&hist[2 * b], w * I);
        atomicAdd(&hist[2 * b + 1], w * I * I);
      }
    }
  }
  atomicAdd(&hist[nv - 1], tot);
  __syncthreads();
  for (int i = threadIdx.x; i < nv; i += 256) a.part[(size_t)blockIdx.x * nv + i] = hist[i];
}

hipError_t launch_mr_bin(int prec, const MrBinArgs& a, int nblocks, hipStream_t s) {
  const size_t shm = (2 * (size_t)a.nbins + 1) * sizeof(double);
  if (prec == 0) hipLaunchKernelGGL(k_mr_bin<float>, dim3(nblocks), dim3(256), shm, s, a);
  else hipLaunchKernelGGL(k_mr_bin<double>, dim3(nblocks), dim3(256), shm, s, a);
  return hipGetLastError();
}

}  // namespace ur
