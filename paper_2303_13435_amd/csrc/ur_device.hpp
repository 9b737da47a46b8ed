// Device building blocks for the gfx950 scattering-simulation kernels:
// complex arithmetic, in-register radix-2/4/8/16 DFTs, and a Stockham
// (self-sorting) FFT of length N executed by a group of G = N/E lanes of one
// wavefront, with the data exchanged through LDS between radix stages.
//
// The transform computed is the discrete Fourier transform of eq. 1 along one
// axis (unnormalised; the caller applies the 1/(MNL) factor where needed), and
// its inverse (DIR = +1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace ur {

template <typename T> struct cx { T x, y; };
// two adjacent complex values, aligned for one wide store
template <typename T> struct alignas(4 * sizeof(T)) cx2 { cx<T> a, b; };

template <typename T> __device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// a * conj(b)
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) { return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
template <typename T> __device__ __forceinline__ cx<T> conjg(cx<T> a) { return mk(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }

// Streaming (non-temporal) stores of complex values: for intermediates that
// are written once and read back only by the next pass, long after any cache
// could hold them.
template <typename T> __device__ __forceinline__ void st_nt(cx<T>* p, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 t;
  t.x = v.x;
  t.y = v.y;
  __builtin_nontemporal_store(t, (v2*)p);
}
template <typename T> __device__ __forceinline__ void st_nt2(cx2<T>* p, cx2<T> v) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  v4 t;
  t.x = v.a.x;
  t.y = v.a.y;
  t.z = v.b.x;
  t.w = v.b.y;
  __builtin_nontemporal_store(t, (v4*)p);
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [I0, I1).
// Guarantees constant indices into register arrays whatever the unroller
// decides for a large body.
template <int I0, int I1, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I0 < I1) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, I1>(f);
  }
}

// LDS ordering between the lanes of one wavefront: the fences keep the
// compiler (and the memory model) from moving LDS accesses across the point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// multiply by exp(DIR * 2 pi i m / 16), m in [0, 8)
template <typename T, int DIR>
__device__ __forceinline__ cx<T> rot16(cx<T> a, int m) {
  const T c1 = (T)0.92387953251128675613;   // cos(pi/8)
  const T s1 = (T)0.38268343236508977173;   // sin(pi/8)
  const T s2 = (T)0.70710678118654752440;   // cos(pi/4)
  const T D = (T)DIR;
  switch (m) {
    case 0: return a;
    case 4: return mk(-D * a.y, D * a.x);                                 // * (D i)
    case 2: return mk(s2 * (a.x - D * a.y), s2 * (a.y + D * a.x));        // * (1 + D i)/sqrt2
    case 6: return mk(-s2 * (a.x + D * a.y), s2 * (D * a.x - a.y));       // * (-1 + D i)/sqrt2
    case 1: return mk(a.x * c1 - a.y * (D * s1), a.x * (D * s1) + a.y * c1);
    case 3: return mk(a.x * s1 - a.y * (D * c1), a.x * (D * c1) + a.y * s1);
    case 5: return mk(-a.x * s1 - a.y * (D * c1), a.x * (D * c1) - a.y * s1);
    default: return mk(-a.x * c1 - a.y * (D * s1), a.x * (D * s1) - a.y * c1);  // m == 7
  }
}

// In-register DFT of size R (power of two <= 16), natural order in and out:
// X_k = sum_r v_r exp(DIR 2 pi i r k / R). Radix-2 decimation in time.
template <typename T, int R, int DIR> struct DFT {
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
    DFT<T, R / 2, DIR>::run(e);
    DFT<T, R / 2, DIR>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      cx<T> t = rot16<T, DIR>(o[k], k * (16 / R));
      v[k] = e[k] + t;
      v[k + R / 2] = e[k] - t;
    }
  }
};
template <typename T, int DIR> struct DFT<T, 1, DIR> {
  static __device__ __forceinline__ void run(cx<T>*) {}
};

// i * a
template <typename T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return mk(-a.y, a.x); }

// DFT of size 3 from its definition: with w = exp(DIR 2 pi i / 3),
// X_1,2 = v0 - (v1 + v2)/2 +- DIR i sin(2 pi/3) (v1 - v2).
template <typename T, int DIR> struct DFT<T, 3, DIR> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const T s = (T)0.86602540378443864676 * (T)DIR;      // DIR sin(2 pi / 3)
    const cx<T> a = v[1] + v[2], b = v[1] - v[2];
    const cx<T> m = v[0] - scale(a, (T)0.5);
    const cx<T> t = mul_i(scale(b, s));
    v[0] = v[0] + a;
    v[1] = m + t;
    v[2] = m - t;
  }
};

// DFT of size 5 from its definition, pairing r with 5 - r: with
// a_j = v_j + v_{5-j}, b_j = v_j - v_{5-j} and theta = 2 pi / 5,
// X_1,4 = v0 + cos(theta) a1 + cos(2 theta) a2 +- DIR i (sin(theta) b1 + sin(2 theta) b2),
// X_2,3 = v0 + cos(2 theta) a1 + cos(theta) a2 +- DIR i (sin(2 theta) b1 - sin(theta) b2).
template <typename T, int DIR> struct DFT<T, 5, DIR> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212 * (T)DIR, s2 = (T)0.58778525229247312917 * (T)DIR;
    const cx<T> a1 = v[1] + v[4], b1 = v[1] - v[4], a2 = v[2] + v[3], b2 = v[2] - v[3];
    const cx<T> m1 = v[0] + scale(a1, c1) + scale(a2, c2);
    const cx<T> m2 = v[0] + scale(a1, c2) + scale(a2, c1);
    const cx<T> t1 = mul_i(scale(b1, s1) + scale(b2, s2));
    const cx<T> t2 = mul_i(scale(b1, s2) - scale(b2, s1));
    v[0] = v[0] + a1 + a2;
    v[1] = m1 + t1;
    v[4] = m1 - t1;
    v[2] = m2 + t2;
    v[3] = m2 - t2;
  }
};

// Padded LDS index: one spare element every 16 breaks the power-of-two
// strides of the Stockham write pattern across LDS banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }
template <int N> struct Padded { static constexpr int size = N + N / 16; };

// Elements per lane for a length-N column; G = N / E lanes per column.  Up to
// N = 1024 a column sits in one wavefront (G <= 64); N = 2048 and 4096 take
// two and four whole wavefronts (G = 128, 256), with 16 elements per lane as
// at 1024.
//
// Lengths N = 2^a 3^b 5^c that are not powers of two (mixed radix) take
// power-of-two radices of at most P, then radix 3, then radix 5;
// E = P (x 3 if b > 0) (x 5 if c > 0) so that every radix divides it; P is
// the smallest power of two (at most 8 and 2^a) that puts the column in one
// wavefront (G = N / E <= 64, not necessarily a power of two).
template <int N> struct Pow2 { static constexpr bool v = (N & (N - 1)) == 0; };
constexpr int pow2_part(int n) { return n & -n; }
template <int N> struct Mixed {
  static_assert(N % 2 == 0, "mixed-radix edges are even");
  static constexpr int odd = (N % 3 == 0 ? 3 : 1) * (N % 5 == 0 ? 5 : 1);
  // the smallest power-of-two cap (at most 16) that keeps a line in one
  // wavefront: fewer elements per lane, fewer registers
  static constexpr int pick() {
    int p = 2;                                     // every compiled edge is even
    while (p < 16 && p < pow2_part(N) && N / (p * odd) > 64) p *= 2;
    return p < pow2_part(N) ? p : pow2_part(N);
  }
  static constexpr int P = pick();
  static constexpr int E = P * odd;
};
template <int N> struct Geo {
  static constexpr int E = Pow2<N>::v ? (N <= 16 ? N : (N == 512 ? 8 : 16)) : Mixed<N>::E;
  static constexpr int G = N / E;
  static_assert(G * E == N && G >= 1 && (G <= 64 || G == 128 || G == 256), "column group: part of one wavefront or whole ones");
};

// Ordering of the LDS accesses of the lanes that share a column: the
// wavefront-level fence when the column lies in one wavefront, otherwise the
// workgroup barrier (every thread of the block must then reach it).
template <int G>
__device__ __forceinline__ void col_sync() {
  if constexpr (G <= 64) wave_sync();
  else __syncthreads();
}

// radix of the stage with sub-transform length L: at most 16 and at most the
// per-lane element count, so each lane runs whole butterflies
template <int N> constexpr int radix_at(int L) {
  if constexpr (Pow2<N>::v) {
    constexpr int cap = Geo<N>::E < 16 ? Geo<N>::E : 16;
    return (N / L) < cap ? (N / L) : cap;
  } else {
    const int m = N / L, p2 = pow2_part(m);
    if (p2 > 1) return p2 < Mixed<N>::P ? p2 : Mixed<N>::P;
    return m % 3 == 0 ? 3 : 5;
  }
}
template <int N, int L> struct Radix { static constexpr int r = radix_at<N>(L); };

// Twiddle tables: stage (L, R) owns L*(R-1) entries exp(-2 pi i r j/(L R)),
// laid out [j][r-1], after the tables of the earlier stages.
template <int N> constexpr int tw_off(int L) {
  int off = 0, l = 1;
  while (l < L) { const int r = radix_at<N>(l); off += l * (r - 1); l *= r; }
  return off;
}

// Padded offset of a compile-time displacement k from a padded base whose
// low four index bits plus those of k stay below 16 (true for every access
// pattern below: the displacements are multiples of 16, or the base is
// aligned to the span of the displacements).
template <int K> struct PadOff { static constexpr int v = K + (K >> 4); };

// One Stockham radix-R stage with sub-transform length L (inputs read from
// the LDS column s, outputs written back to s, in place through registers).
// Lane g of the group performs butterflies b = g + G*i, i < E/R: inputs
// x[b + r N/R], twiddles exp(DIR 2 pi i r j/(L R)) with j = b mod L, outputs
// y[(b/L) L R + j + r L].  Every LDS address is one padded base per
// butterfly plus a compile-time offset.
// TWH: the stage's twiddles are loaded ahead of its LDS reads (their
// latency overlaps the reads and the fence; E R-1 values held at once) or
// else at each butterfly (fewer live registers).
template <typename T, int N, int L, int DIR, bool TWH = true>
__device__ __forceinline__ void stage_lds(cx<T>* s, int g, const cx<T>* __restrict__ tw) {
  constexpr int E = Geo<N>::E, G = Geo<N>::G, R = Radix<N, L>::r, NB = E / R;
  constexpr int NR = N / R;
  static_assert(NB * R == E, "radix must divide the per-lane count");
  cx<T> w[NB][R > 1 ? R - 1 : 1];
  if (L > 1 && TWH) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const cx<T>* wp = tw + (tw_off<N>(L) + ((g + G * i) % L) * (R - 1));
#pragma unroll
      for (int r = 1; r < R; ++r) w[i][r - 1] = wp[r - 1];     // exp(-2 pi i r j / (L R))
    }
  }
  cx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if constexpr (NR % 16 == 0) {                        // displacements are multiples of 16
      const cx<T>* base = s + pad(g + G * i);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = base[r * (NR + NR / 16)];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = s[pad(g + G * i + r * NR)];
    }
  }
  col_sync<G>();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = g + G * i;
    const int j = b % L;
    if (L > 1) {
      if constexpr (!TWH) {
        const cx<T>* wp = tw + (tw_off<N>(L) + j * (R - 1));
#pragma unroll
        for (int r = 1; r < R; ++r) w[i][r - 1] = wp[r - 1];
      }
#pragma unroll
      for (int r = 1; r < R; ++r) v[i][r] = DIR < 0 ? cmul(v[i][r], w[i][r - 1]) : cmulc(v[i][r], w[i][r - 1]);
    }
    DFT<T, R, DIR>::run(v[i]);
    if constexpr (Pow2<N>::v) {
      cx<T>* out = s + pad((b / L) * L * R + j);
#pragma unroll
      for (int r = 0; r < R; ++r) out[(r * L) + ((r * L) >> 4)] = v[i][r];
    } else {                                       // offsets r L may carry into the next 16-block
      const int o = (b / L) * L * R + j;
#pragma unroll
      for (int r = 0; r < R; ++r) s[pad(o + r * L)] = v[i][r];
    }
  }
  col_sync<G>();
}

template <typename T, int N, int L, int DIR, bool TWH = true>
__device__ __forceinline__ void stages_from(cx<T>* s, int g, const cx<T>* __restrict__ tw) {
  if constexpr (L < N) {
    stage_lds<T, N, L, DIR, TWH>(s, g, tw);
    stages_from<T, N, L * Radix<N, L>::r, DIR, TWH>(s, g, tw);
  }
}

// First stage fed from registers. The caller provides, for lane g, the E
// inputs in the order v[i*R0 + r] = x[b + r*(N/R0)], b = g + G*i, with R0 the
// first radix. Results of the whole transform are left in natural order in
// the LDS column s (padded indexing).
template <typename T, int N, int DIR, bool TWH = true>
__device__ __forceinline__ void fft_column(cx<T>* s, int g, const cx<T>* __restrict__ tw, cx<T>* v) {
  constexpr int E = Geo<N>::E, G = Geo<N>::G, R = Radix<N, 1>::r, NB = E / R;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = g + G * i;
    DFT<T, R, DIR>::run(v + i * R);
    if constexpr (Pow2<N>::v) {
      cx<T>* out = s + pad(b * R);                     // R | 16: the R outputs share one 16-block
#pragma unroll
      for (int r = 0; r < R; ++r) out[r] = v[i * R + r];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) s[pad(b * R + r)] = v[i * R + r];
    }
  }
  col_sync<G>();
  stages_from<T, N, R, DIR, TWH>(s, g, tw);
}

// Index of the r-th input of lane g's i-th first-stage butterfly.
template <int N>
__device__ __forceinline__ int first_index(int g, int i, int r) {
  constexpr int G = Geo<N>::G, R = Radix<N, 1>::r;
  return (g + G * i) + r * (N / R);
}

// signed frequency index of u in [0, n)
__device__ __forceinline__ int sidx(int u, int n) { return u < n / 2 ? u : u - n; }

// exact integer square root (largest r with r*r <= v), v >= 0
__device__ __host__ __forceinline__ long long isqrt_ll(long long v) {
  if (v <= 0) return 0;
  long long r = (long long)sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

}  // namespace ur
