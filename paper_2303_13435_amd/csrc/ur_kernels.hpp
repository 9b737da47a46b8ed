// Kernel argument blocks and host launchers of the gfx950 hot path.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ur_geom.hpp"

namespace ur {

// Box edges: every path up to kMaxInCore; FP32 real boxes up to
// kMaxOutOfCore through the out-of-core forward path only.
constexpr int kMaxInCore = 2048;
constexpr int kMaxOutOfCore = 4096;
// z-pass blocks up to which the finalize sums their rho^2 in one block (above:
// a first-level kernel of 256 blocks, one CU cannot read them fast enough)
constexpr int kFoldMoments = 32768;
// atom profiles and amplitudes up to this size are staged in LDS by the cell sum
constexpr size_t kCellStageBytes = 48 * 1024;

// Density source of the first (z) pass.
// GEN: ED-1 voxels (block factor 1); ZOOM: block-summed zoom levels.
// ROT: ED-1 of a rotated lattice (periodic interpolation of the cell):
// trilinear or cubic B-spline (ROT3), one orientation or grains (G).
enum ZMode { Z_GEN_R2C = 0, Z_LOAD_R2C = 1, Z_GEN_C2C = 2, Z_LOAD_C2C = 3, Z_ZOOM_R2C = 4, Z_ZOOM_C2C = 5,
             Z_ROT_R2C = 6, Z_ROT3_R2C = 7, Z_ROTG_R2C = 8, Z_ROT3G_R2C = 9 };
// What the last (x) pass does with each transformed column.
// X_ADJ: the adjoint column pass; the _SINC variants (chosen by the launcher
// when XArgs::sinc is set) weight every intensity by the voxel form factor.
enum XMode { X_FFT_BIN = 0, X_BIN_ONLY = 1, X_FFT_STORE = 2, X_ADJ = 3, X_FFT_BIN_SINC = 4, X_BIN_ONLY_SINC = 5 };

constexpr int kMaxGrains = 16;
// largest box of a zoom level of a rotated lattice (the generator keeps
// kZoomRotMaxBox / 256 level voxels per thread)
constexpr int kZoomRotMaxBox = 2048;

struct ZArgs {
  void* A;                  // out: [x - ax0][kz][y] complex
  long long ax0;            // first plane held by A
  const void* rho;          // LOAD: real (r2c) or complex (c2c) [x][y][z], planes from rho_x0
  long long rho_x0;
  const void* cellT;        // GEN: c^3 cell in the working precision
  const void* cb;           // GEN, f > 1: block-summed cell, cbn^3
  const double* pre;        // GEN, f > 1: per-row prefix sums of the FP64 cell, c^2 (c+1)
  const void* tw;           // n twiddles exp(-2 pi i k / n)
  double* mom;              // per block: sum rho, sum rho^2 (may be null)
  Level L;
  MaskP m;
  int nkz;                  // rows per plane of A
  int x0;                   // first plane of this launch
  int ntiles;               // y tiles per plane
  int cbn;                  // edge of the block table
  int rotated;              // ROT generation: the cell is sampled at u = rot d
  double rot[9];            // row-major
  int cubic;                // ROT: cellT holds cubic B-spline coefficients (64-tap sampling)
  int ngrain;               // ROT with grains: voxel d takes the orientation of its nearest seed
  int gseed[kMaxGrains][3]; // seed offsets from the particle centre (voxels)
  double grot[kMaxGrains][9];
};

struct YArgs {
  const void* A;            // [x - ax0][kz][y]
  long long ax0;
  void* B;                  // out: [kz][ky][x - bx0], column stride bs
  long long bx0;
  long long bs;
  const void* tw;
  Level L;
  MaskP m;
  int gen;                  // rows of A hold density only inside the particle's row range
  int nkz;
  int xlo, xhi;             // planes written by the z pass
  int xt0;                  // first x tile of the launch
  int nxt;                  // number of x tiles
  int ty;                   // y tile height of the z pass
  int kz0, nkzc;            // rows kz0 .. kz0 + nkzc - 1 of A go to B rows 0 .. nkzc - 1 (nkzc 0: all)
};

// entries of the start-of-walk bin table of an n^3 box: s = 0 .. isqrt(3 (n/2)^2) + 1
inline int lut_len(int n) {
  const long long n2max = 3ll * (n / 2) * (n / 2);
  long long s = 0;
  while ((s + 1) * (s + 1) <= n2max) ++s;
  return (int)s + 2;
}

struct XArgs {
  const void* B;            // [kz][ky][x - bx0] columns of stride bs
  long long bx0;
  long long bs;
  void* out;                // X_FFT_STORE: out columns [kz][ky][kx], stride n
  const void* tw;
  int nkz;
  int r2c;                  // half spectrum (weights 1/2) or full
  int xa, xb;               // rows of each column that hold data (others are zero)
  double iscale;            // intensity scale: I = |v|^2 * iscale
  double oscale;            // store scale
  int nbins;
  const int* U;             // nbins + 1 integer thresholds on n2
  const short* lut;         // bin of n2 = s^2 for s in [0, nlut): start of the bin walk
  int nlut;
  double* part;             // per block: 2*nbins (sum, sumsq) + 1 total
  double* f0;               // F(0) (2 doubles), written by the block holding it
  int ncols;
  int kz0;                  // kz of column 0 (B holds rows kz0 .. kz0 + ncols / n - 1)
  int accum;                // add to the block partials instead of writing them (later kz chunks)
  const void* sinc;         // null, or S(m) = sinc^2(pi m / n) for m in [0, n/2] (working precision)
};

struct FinArgs {
  const double* part;       // nblk x (2 nbins + 1)
  int nblk;
  int nbins;
  const double* mom;        // nzb x 2 (may be null)
  int nzb;
  double* mpart;            // 256 first-level partial sums of rho^2 (workspace), used above kFoldMoments blocks
  const double* f0;
  const double* cnt;        // per-bin voxel counts (geometry, computed with the bins)
  double* sum;
  double* sumsq;
  double* count;
  double* totals;
  double* mean;             // per-bin mean and SEM (may be null)
  double* sem;
};

struct MergeArgs {
  int nlevels;
  const double* sum[8];
  const double* sumsq[8];
  const double* count[8];
  double scale[8];
  double dq[8];
  double qcut[8];
  int order[8];             // level indices, finest voxel first
  int mode;
  double n_min;
  int nbins;
  const double* edges;      // device, nbins + 1
  double* mean;
  double* sem;
  int* owner;
};

// adjoint, inverse passes
struct XAdjArgs {
  void* B;                  // columns [kz][ky][x - bx0] of stride bs, transformed in place
  long long bx0, bs;
  const void* tw;
  int nkz;
  int r2c;
  int xa, xb;               // rows holding the forward data (others zero)
  int oa, ob;               // rows written back
  int nbins;
  const int* U;
  const short* lut;         // start-of-walk bin table (as in XArgs)
  int nlut;
  const double* g_bin;      // dL/dI_b
  const double* count;      // forward bin counts
  double gscale;            // 2 / n^6
  int ncols;
  const void* sinc;         // per-axis intensity weight S(|m|), m in [0, N/2], working precision, or null
};

struct YInvArgs {
  const void* B;            // [kz][ky][x - bx0], column stride bs
  long long bx0, bs;
  void* A;                  // out [x][kz][y]
  const void* tw;
  int nkz;
  int xt0, nxt;
  // rows != 0: write only the rows of plane x inside the particle's row
  // range, widened to whole tiles of ty rows (all a fold onto the cell reads)
  int rows, ty;
  Level L;
  MaskP m;
};

// inverse z pass fused with the fold onto the unit cell (amplitude gradients)
struct ZFoldArgs {
  const void* A;            // [x][kz][y] (r2c half spectra)
  const void* tw;
  Level L;
  MaskP m;
  int nkz;
  int xlo, xhi;             // planes holding particle voxels
  int ntiles;               // y tiles per plane
  double scale;
  double* part;             // per block c^3 partial folds (c <= 16)
  double* gcell;            // c^3 global accumulators (c > 16)
};

struct ZInvArgs {
  const void* A;            // [x][kz][y]
  void* out;                // real [x][y][z] (r2c) or complex (c2c)
  const void* tw;
  int nkz;
  int ntiles;
  double scale;
  int x0, nx;               // planes x0 .. x0 + nx - 1 (nx = 0: the whole box)
  int prune;                // 1: only the y tiles that meet the particle's rows (L, m)
  Level L;
  MaskP m;
};

struct FoldArgs {
  const void* g;            // real [x][y][z], n^3
  Level L;
  MaskP m;
  double* gcell;            // c^3 accumulators (global atomics when c > 16)
  double* part;             // per block c^3 (LDS path)
  int npencils;
};

// host launchers (return hipError_t of the launch)
hipError_t launch_cell_profiles(int c, int n_atoms, const double* xyz, const double* sigma, double* prof, hipStream_t s);
hipError_t launch_cell_sum(int c, int n_atoms, const double* amp, const double* prof, double bg, double* cell, hipStream_t s,
                           int prec = 0, void* cellT = nullptr);
hipError_t launch_cell_tables(int prec, int c, int f, const double* cell, void* cellT, double* pre, void* cb, int cbn, hipStream_t s);
hipError_t launch_pass_z(int prec, int n, int mode, const ZArgs& a, int nblocks, hipStream_t s);
hipError_t launch_pass_y(int prec, int n, const YArgs& a, hipStream_t s);
hipError_t launch_pass_x(int prec, int n, int mode, int dir, const XArgs& a, int nblocks, hipStream_t s);
hipError_t launch_finalize(const FinArgs& a, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
// Mixed-radix boxes: edges n = 2^a 3^b 5^c that are not powers of two, complex
// [x][y][z] arrays transformed in place one axis at a time; the spectrum
// stays in natural order [kx][ky][kz].
// the compiled mixed-radix edges: the 2^a 5^3 family of the paper's boxes and
// zoom levels (250 ... 2000) with smaller members for tests, and 2^a 3
#define UR_MR_SIZES(X) X(40) X(80) X(100) X(160) X(200) X(250) X(400) X(500) X(1000) X(2000) \
                       X(48) X(96) X(384) X(768) X(1536) X(4000)

bool mr_size(int n);
struct MrArgs {
  const void* src;          // this pass's input (may equal dst)
  void* dst;
  const void* tw;
  double scale;             // applied to the outputs
  double* mom;              // per-block [sum rho, sum |rho|^2] of the input (may be null)
  ZArgs z;                  // MR_GEN: the density generator of the level
  int nbins;                // MR_BIN: |F|^2 * iscale into the bins, no store
  const int* U;
  const short* lut;
  double iscale;
  double* part;             // nblk x (2 nbins + 1)
  double* f0;
  // part of a box (out-of-core): z pass over `lines` z lines (real boxes:
  // pencil pairs) from src, y pass over `planes` x planes of dst, x pass
  // over a box that stores only planes [xa, xa + xn) (the rest read as zero);
  // 0: the whole box
  long long lines;
  int planes;
  int xa, xn;
  // pruning of an in-HBM box whose density lies in the region of the level
  // in z (L and m): the z pass skips tiles of lines that hold no density
  // (leaving them unwritten), the y pass runs planes [px0, px0 + planes) and
  // reads the rows outside each plane's row range as zero
  int prune;
  int px0;
  // real boxes in the plan's workspace: row pitch of the kz index (0: the
  // natural n/2 + 1), rounded up so that every row starts on a 128-byte line
  int nzp;
};
// axis 0 = x (stride n^2), 1 = y (stride n), 2 = z (contiguous);
// mode MR_LOAD: src -> dst, MR_GEN (axis 2): generated density -> dst,
// MR_BIN (axis 0, forward): src -> bins
enum MrMode { MR_LOAD = 0, MR_GEN = 1, MR_BIN = 2 };
// r2c: a real box (two real pencils per z line, half spectrum [..][..][kz <= n/2]; forward only)
hipError_t launch_mr_axis(int prec, int n, int axis, int dir, int mode, bool r2c, const MrArgs& a, hipStream_t s);
int mr_axis_blocks(int prec, int n, int axis, int mode, bool r2c);
int mr_tile_lines(int prec, int n);
struct MrBinArgs {
  const void* S;            // complex [kx][ky][kz] (r2c: kz in [0, n/2])
  int n, nbins;
  int r2c;                  // half spectrum of a real box: kz in (0, n/2) counted twice
  const int* U;
  const short* lut;
  int nlut;
  double iscale;
  double* part;             // nblk x (2 nbins + 1)
  double* f0;
};
hipError_t launch_mr_bin(int prec, const MrBinArgs& a, int nblocks, hipStream_t s);

// Ewald-sphere image: per detector pixel, |F|^2 trilinear on the reciprocal
// grid at q = k_j (s - e), averaged over wavelength nodes j
struct EwaldArgs {
  const void* spec;         // [kz][ky][kx], kz in [0, nkz)
  int n, nkz, c2c;
  int natural;              // spectrum in [kx][ky][kz] order (mixed-radix plans)
  double dq;                // 2 pi / (n voxel)
  double e[3], du[3], dv[3];
  double dist, pixel, cu, cv;
  int nu, nv, nl;
  double k[64], w[64];      // 2 pi / lambda_j and the node weights
  double* image;            // [nv][nu]
};
hipError_t launch_ewald(int prec, const EwaldArgs& a, hipStream_t s);

// peak integrals over q windows of a binned curve, one thread per window
constexpr int kMaxWindows = 64;
struct PeakArgs {
  int nbins, nwin;
  const double* edges;
  const double* mean;
  double lo[kMaxWindows], hi[kMaxWindows];
  double* out;              // [nwin][3]: peak, total, bins
};
hipError_t launch_peaks(const PeakArgs& a, hipStream_t s);

hipError_t launch_chi2(int nbins, const double* mean, const double* count, const double* target, double rel_sigma,
                       double* out, double* g, hipStream_t s);
hipError_t launch_ensemble(int nboxes, int nbins, const double* mean, const double* sem, const double* w,
                           double* out_mean, double* out_sem, hipStream_t s);
hipError_t launch_pass_x_adj(int prec, int n, const XAdjArgs& a, int nblocks, hipStream_t s);
hipError_t launch_pass_y_inv(int prec, int n, const YInvArgs& a, hipStream_t s);
hipError_t launch_pass_z_inv(int prec, int n, int c2c, const ZInvArgs& a, hipStream_t s);
hipError_t launch_fold(int prec, int n, const FoldArgs& a, int nblocks, hipStream_t s);
hipError_t launch_fold_rot(int prec, int n, const ZArgs& a, const void* g, double* part, int nblocks, hipStream_t s);
hipError_t launch_pass_z_fold(int prec, int n, const ZFoldArgs& a, int nblocks, hipStream_t s);
hipError_t launch_fold_reduce_classes(int c, const double* part, int nblk, double* gcell, hipStream_t s);
hipError_t launch_fold_reduce(int c3, const double* part, int nblk, double* gcell, hipStream_t s);
hipError_t launch_grad_amp(int c, int n_atoms, const double* prof, const double* gcell, double* grad_amp, hipStream_t s);
// periodic cubic B-spline coefficients of a c^3 FP64 cell, in place
hipError_t launch_bspline_cell(int c, double* cell, hipStream_t s);
// a level's density as complex (rho, 0) with per-pencil moments (mixed-radix zoom levels)
hipError_t launch_level_complex(int prec, int n, const ZArgs& a, void* S, double* mom, hipStream_t s);
hipError_t launch_rho_generate(int prec, int n, int x_lo, int x_hi, const ZArgs& a, void* rho, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_bin_counts(int n, int nkz, int r2c, int nbins, const int* U, unsigned long long* tmp, double* out, hipStream_t s);
int x_resident(int prec, int n, int mode, int dir, int nbins);   // resident x-pass blocks per CU

// Allocation-free forward entry: bytes of its static device scratch (a
// 256^3 FP32 real box with its block partials and cell tables fits), and the
// scratch's address on the current device (resolved once per device).
constexpr size_t kNoAllocScratchBytes = (size_t)160 << 20;
hipError_t noalloc_scratch(void** ptr);

// Stockham stages (L, R) the kernels run for a length-n column; returns the
// count (the twiddle table of stage (L, R) holds exp(-2 pi i r j/(L R)) for
// j < L, 1 <= r < R, laid out [j][r-1], stages back to back)
int fft_stages(int n, int* Ls, int* Rs);

// tile geometry used by the host planner (must match the kernels)
int z_tile(int prec, int n, int c2c);     // y pencils per z-pass block
int y_tile(int prec, int n);              // x planes per y-pass block
int zinv_tile(int prec, int n, int c2c);  // y pencils per inverse z-pass block
int x_groups(int n);                      // columns per x-pass block

}  // namespace ur
