// Particle geometry shared by the host planner and the device kernels:
// exact integer mask tests and the index ranges a zoom level can occupy.
// (Methodology, "Electron density generation": a mask per plane that builds
// up the particle; block integration into zoomed-out levels.)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ur {

struct MaskP {
  int kind;          // 0 none, 1 sphere, 2 cube, 3 truncated octahedron
  long long p0, p1;
};

constexpr long long kUnbounded = (1ll << 40);

__host__ __device__ inline long long isqrt_geom(long long v) {
  if (v <= 0) return 0;
  long long r = (long long)sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Largest |d3| such that a voxel with |d1| = a, |d2| = b, |d3| is inside;
// -1 when no such voxel exists.  Every supported shape is convex and
// symmetric under sign flips and axis permutations, so the inside set is
// monotone in each |d_i| and this one function answers every range query.
__host__ __device__ inline long long mask_reach(const MaskP& m, long long a, long long b) {
  switch (m.kind) {
    case 0: return kUnbounded;
    case 1: {
      if (m.p0 < 0) return -1;
      long long rem = m.p0 - a * a - b * b;
      return rem < 0 ? -1 : isqrt_geom(rem);
    }
    case 2: return (m.p0 >= 0 && a <= m.p0 && b <= m.p0) ? m.p0 : -1;
    case 3: {
      if (m.p0 < 0 || a > m.p0 || b > m.p0) return -1;
      long long r = m.p1 - a - b;
      if (r < 0) return -1;
      return r < m.p0 ? r : m.p0;
    }
    default: return -1;
  }
}

// Geometry of one box: ED-1 grid of edge n1 block-summed by f into a box of
// edge n, the reduced particle region [o, o + n1/f) per axis.
struct Level {
  int n;        // this box
  int n1;       // ED-1 edge
  int f;        // block factor
  int o;        // offset of the reduced region
  int h;        // particle centre on the ED-1 grid (n1/2)
  int c;        // cell edge
};

__host__ __device__ inline Level make_level(int n, int n1, int f, int c) {
  Level L;
  L.n = n; L.n1 = n1; L.f = f; L.o = (n - n1 / f) / 2; L.h = n1 / 2; L.c = c;
  return L;
}

// min and max of |d| = |x - h| over the fine block of coarse index X.
__host__ __device__ inline void block_dist(const Level& L, long long X, long long& dmin, long long& dmax) {
  long long lo = (long long)L.f * (X - L.o) - L.h;
  long long hi = lo + L.f - 1;
  long long alo = lo < 0 ? -lo : lo, ahi = hi < 0 ? -hi : hi;
  dmax = alo > ahi ? alo : ahi;
  dmin = (lo <= 0 && hi >= 0) ? 0 : (alo < ahi ? alo : ahi);
}

__host__ __device__ inline bool in_region(const Level& L, long long X) {
  return X >= L.o && X < L.o + (L.f == 1 ? L.n1 : L.n1 / L.f);
}

// coarse index range [*lo, *hi] of the fine interval [h - r, h + r]
__host__ __device__ inline void coarse_range(const Level& L, long long r, long long& lo, long long& hi) {
  if (r < 0) { lo = 1; hi = 0; return; }
  long long a = L.h - r, b = L.h + r;
  if (a < 0) a = 0;
  if (b > L.n1 - 1) b = L.n1 - 1;
  if (L.f == 1) {                          // ED-1: no division
    lo = a + L.o;
    hi = b + L.o;
  } else {
    lo = a / L.f + L.o;
    hi = b / L.f + L.o;
  }
}

// planes X that can hold density
__host__ __device__ inline void plane_range(const Level& L, const MaskP& m, long long& lo, long long& hi) {
  coarse_range(L, mask_reach(m, 0, 0), lo, hi);
}

// rows Y of plane X that can hold density (empty range when lo > hi)
__host__ __device__ inline void row_range(const Level& L, const MaskP& m, long long X, long long& lo, long long& hi) {
  if (!in_region(L, X)) { lo = 1; hi = 0; return; }
  long long dmin, dmax;
  block_dist(L, X, dmin, dmax);
  coarse_range(L, mask_reach(m, dmin, 0), lo, hi);
}

// voxels Z of pencil (X, Y) that can hold density
__host__ __device__ inline void col_range(const Level& L, const MaskP& m, long long X, long long Y, long long& lo, long long& hi) {
  if (!in_region(L, X) || !in_region(L, Y)) { lo = 1; hi = 0; return; }
  long long ax, bx, ay, by;
  block_dist(L, X, ax, bx);
  block_dist(L, Y, ay, by);
  coarse_range(L, mask_reach(m, ax, ay), lo, hi);
}

}  // namespace ur
