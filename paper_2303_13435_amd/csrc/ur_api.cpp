// C ABI of the gfx950 scattering simulator: plans, validation, integer bin
// thresholds, workspace, and the orchestration of the transform passes.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ultima.h"
#include "ur_geom.hpp"
#include "ur_kernels.hpp"

using namespace ur;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static ur_status fail(ur_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define UR_HIP(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(UR_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define UR_TRY(expr)                 \
  do {                               \
    ur_status s_ = (expr);           \
    if (s_ != UR_OK) return s_;      \
  } while (0)

static bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct ur_plan {
  int n = 0;
  double voxel = 0.0;
  int prec = 0;
  unsigned flags = 0;
  int nkz = 0;
  bool mixed = false;        // edge 2^a 3^b 5^c, not a power of two (complex, natural-order spectrum)
  size_t cs = 0;             // bytes per complex element
  size_t rs = 0;             // bytes per real element
  int device = 0;

  void* tw = nullptr;        // n twiddles (device)

  int ncu = 256;             // compute units of the device
  int nbins = 0;
  int* dU = nullptr;         // nbins + 1 thresholds (device)
  short* dLut = nullptr;     // bin of n2 = s^2, s in [0, nlut) (device)
  int nlut = 0;
  // y-pass output of the last ur_simulate still held in the workspace (ED-1,
  // real transform): its mask and cell edge; cleared by every other call
  bool keep_valid = false;
  MaskP keep_m{};
  int keep_c = 0;
  double* dCount = nullptr;  // per-bin voxel counts (device), computed with the bins
  unsigned long long* dCountTmp = nullptr;
  std::vector<long long> U;

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;

  // cell scratch (library owned, grown on demand)
  char* cs_buf = nullptr;
  size_t cs_bytes = 0;
  char* lvl_buf = nullptr;   // density of a zoom level of an oriented lattice (n^3 reals), owned
  size_t lvl_bytes = 0;

  // out-of-core staging: kStage slab buffers on the device, each filled on
  // its own copy stream (several host-to-device copies in flight keep PCIe
  // busy); pageable input first goes through kStage pinned bounce slabs
  static constexpr int kStage = 4;
  hipStream_t copy_stream[kStage] = {};
  hipEvent_t ev_copied[kStage] = {}, ev_free[kStage] = {};
  void* stage = nullptr;
  size_t stage_bytes = 0;
  void* bounce = nullptr;    // pinned host memory
  size_t bounce_bytes = 0;
  size_t hbm_budget = 0;     // out-of-core workspace bytes allowed (0: no limit)
  void* dSinc = nullptr;     // per-axis intensity weight W(m), m in [0, n/2], or null when off:
                             // the voxel form factor S(m) and/or the removed block transfer 1/|T(m)|^2
  bool vox = false;          // voxel form factor on
  int bt_f = 0;              // block-sum factor whose transfer is removed (0: none)

  // live HIP graphs recorded from this plan's calls (ur_graph_begin/end):
  // they hold raw pointers into the workspace and tables, so nothing may be
  // reallocated or rewritten while any exists; graph_external marks a call
  // recorded under a capture this library did not start (its graph's
  // lifetime is unknown, so the plan stays bound)
  int graphs = 0;
  bool graph_external = false;

  // per-pass timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;
  double pass_bytes[5] = {0, 0, 0, 0, 0};
  int xres[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};   // resident x-pass blocks per CU, by mode and direction
  int xres_nbins = -1;
};

enum { P_CELL = 0, P_Z = 1, P_Y = 2, P_X = 3, P_FIN = 4 };

// event pair around one pass launch (no-op unless timing is on)
struct PassTimer {
  ur_plan* p;
  int pass;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  PassTimer(ur_plan* p_, int pass_, hipStream_t s_) : p(p_), pass(pass_), s(s_) {
    if (!p->timing) return;
    a = take();
    b = take();
    if (a) (void)hipEventRecord(a, s);
  }
  hipEvent_t take() {
    if (!p->ev_pool.empty()) { hipEvent_t e = p->ev_pool.back(); p->ev_pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~PassTimer() {
    if (!p->timing || !a || !b) return;
    (void)hipEventRecord(b, s);
    try {
      p->ev_open.push_back({pass, {a, b}});
    } catch (...) {                      // no room to keep the pair: drop this sample
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  }
};

// x pass: persistent blocks = resident blocks per CU x CUs (at most kMaxXBlocks)
static const int kMaxXBlocks = 1024;
static int x_blocks_for(int) { return kMaxXBlocks; }
static int x_blocks(ur_plan* p, int mode = X_FFT_BIN, int dir = -1) {
  if (p->xres_nbins != p->nbins) {
    for (auto& m : p->xres) m[0] = m[1] = 0;
    p->xres_nbins = p->nbins;
  }
  int& r = p->xres[mode][dir < 0 ? 0 : 1];
  if (r == 0) r = x_resident(p->prec, p->n, mode, dir, std::max(p->nbins, 1));
  return std::max(1, std::min(r * p->ncu, kMaxXBlocks));
}

// largest ZMode tile over the modes the plan can run
static int zt(const ur_plan* p) { return z_tile(p->prec, p->n, p->flags & UR_C2C); }
static int ntiles(const ur_plan* p) { return p->n / zt(p); }

struct Layout {
  size_t A, B, part, mom, f0, total;
};

static Layout layout_incore(const ur_plan* p, int nbins) {
  Layout L;
  size_t n = p->n;
  size_t plane = (size_t)p->nkz * n * p->cs;
  L.A = 0;
  L.B = align256(L.A + n * plane);
  L.part = align256(L.B + (size_t)p->nkz * n * n * p->cs);
  L.mom = align256(L.part + (size_t)x_blocks_for(nbins) * (2 * (size_t)std::max(nbins, 1) + 1) * 8);
  L.f0 = align256(L.mom + n * (size_t)ntiles(p) * 16);
  L.total = align256(L.f0 + 64 + 256 * 8);
  return L;
}

// mixed-radix layout: the complex box (transformed in place), block
// partials, F(0) and the per-pencil moments
// the out-of-core box of a real mixed-radix plan: only planes [x_lo, x_hi]
// (nx of them) of the half spectrum
static Layout layout_mixed_ooc(const ur_plan* p, int nbins, size_t nx) {
  Layout L;
  const size_t n = p->n;
  L.A = 0;
  L.B = 0;
  L.part = align256(nx * n * (size_t)p->nkz * p->cs);
  L.mom = align256(L.part + (size_t)kMaxXBlocks * (2 * (size_t)std::max(nbins, 1) + 1) * 8);
  L.f0 = align256(L.mom + n * n * 16);
  L.total = align256(L.f0 + 64 + 256 * 8);
  return L;
}

// row pitch of the kz index of a real mixed-radix box in the workspace: n/2 + 1
// rounded up to whole 128-byte lines, so that the y and x passes' segments of
// consecutive kz start on line boundaries (complex boxes: n)
static int mixed_pitch(const ur_plan* p) {
  if (p->flags & UR_C2C) return p->nkz;
  const int q = (int)(128 / p->cs);
  return (p->nkz + q - 1) / q * q;
}

static Layout layout_mixed(const ur_plan* p, int nbins) {
  Layout L;
  const size_t n = p->n;
  L.A = 0;
  L.B = 0;
  L.part = align256(n * n * (size_t)mixed_pitch(p) * p->cs);  // the box (real plans: the half spectrum)
  L.mom = align256(L.part + (size_t)kMaxXBlocks * (2 * (size_t)std::max(nbins, 1) + 1) * 8);
  L.f0 = align256(L.mom + n * n * 16);
  L.total = align256(L.f0 + 64 + 256 * 8);
  return L;
}

// out-of-core layout: one slab of the first intermediate, rows kz of B over
// [xlo, xhi] for kzc values of kz at a time (the x passes of all kz chunks
// add into one set of block partials)
static Layout layout_host(const ur_plan* p, int nbins, int xlo, int xhi, int kzc) {
  Layout L;
  size_t n = p->n;
  int tx = y_tile(p->prec, p->n);
  size_t plane = (size_t)p->nkz * n * p->cs;
  long long xt0 = xlo / tx, xt1 = xhi / tx;
  size_t bs = (size_t)(xt1 - xt0 + 1) * tx;
  L.A = 0;
  L.B = align256(L.A + (size_t)tx * plane);
  L.part = align256(L.B + (size_t)kzc * n * bs * p->cs);
  L.mom = align256(L.part + (size_t)x_blocks_for(nbins) * (2 * (size_t)std::max(nbins, 1) + 1) * 8);
  L.f0 = align256(L.mom + n * (size_t)ntiles(p) * 16);
  L.total = align256(L.f0 + 64 + 256 * 8);
  return L;
}

// Split of the kz rows of the out-of-core spectrum into passes whose
// workspace fits the plan's HBM budget; every pass streams the host planes
// again (eq. 2's second stage then runs kz chunk by kz chunk).
struct OocSplit {
  int kzc = 0, nchunks = 0;
  Layout lay{};
};
static ur_status ooc_split(const ur_plan* p, int nbins, int xlo, int xhi, OocSplit& o) {
  for (int nc = 1; nc <= p->nkz; ++nc) {
    const int kzc = (p->nkz + nc - 1) / nc;
    if (nc > 1 && (p->nkz + kzc - 1) / kzc != nc) continue;       // same split as a smaller count
    Layout L = layout_host(p, nbins, xlo, xhi, kzc);
    if (p->hbm_budget == 0 || L.total <= p->hbm_budget) {
      o.kzc = kzc;
      o.nchunks = nc;
      o.lay = L;
      return UR_OK;
    }
    if (p->hbm_budget == 0) break;
  }
  return fail(UR_ERR_OOM, "HBM budget of %zu bytes is below the out-of-core workspace of one kz row", p->hbm_budget);
}

// ---------------------------------------------------------------------------
// graphs: which plans a live graph was recorded from
// ---------------------------------------------------------------------------
static std::mutex g_graph_mu;
static std::map<void*, std::vector<ur_plan*>> g_graph_plans;   // graph exec -> plans it uses
static thread_local bool tl_capturing = false;                // between ur_graph_begin and ur_graph_end
static thread_local std::vector<ur_plan*> tl_captured;

static bool graph_bound(const ur_plan* p) { return p->graphs > 0 || p->graph_external; }

// Entry of every call that enqueues work of the plan on `s`: under capture,
// note the plan as used by the graph being recorded.
static void note_stream(ur_plan* p, hipStream_t s) {
  hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
  if (!s || hipStreamIsCapturing(s, &cst) != hipSuccess) { (void)hipGetLastError(); return; }
  if (cst == hipStreamCaptureStatusNone) return;
  if (!tl_capturing) { p->graph_external = true; return; }
  if (std::find(tl_captured.begin(), tl_captured.end(), p) == tl_captured.end()) {
    try {
      tl_captured.push_back(p);
    } catch (...) {
      p->graph_external = true;                 // cannot track it: keep the plan bound
    }
  }
}

static ur_status refuse_bound(const ur_plan* p, const char* what) {
  return fail(UR_ERR_STATE, "%s: the plan is recorded in a live graph (destroy the graph with ur_graph_destroy first)%s",
              what, p->graph_external ? "; it was recorded under a capture not started by ur_graph_begin" : "");
}

static ur_status ensure_ws(ur_plan* p, size_t need, hipStream_t s) {
  if (p->ws && p->ws_bytes >= need) return UR_OK;
  if (graph_bound(p)) return refuse_bound(p, "workspace reallocation");
  if (p->ws && !p->ws_owned)
    return fail(UR_ERR_STATE, "attached workspace holds %zu bytes, this call needs %zu", p->ws_bytes, need);
  hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
  if (s) (void)hipStreamIsCapturing(s, &cst);
  if (cst != hipStreamCaptureStatusNone)
    return fail(UR_ERR_STATE, "workspace must be allocated (first call) before graph capture");
  if (p->ws) { UR_HIP(hipDeviceSynchronize()); UR_HIP(hipFree(p->ws)); p->ws = nullptr; p->ws_bytes = 0; }
  void* ptr = nullptr;
  if (hipMalloc(&ptr, need) != hipSuccess) { (void)hipGetLastError(); return fail(UR_ERR_OOM, "hipMalloc(%zu) failed", need); }
  p->ws = (char*)ptr;
  p->ws_bytes = need;
  p->ws_owned = true;
  return UR_OK;
}

static ur_status ensure_cell_scratch(ur_plan* p, size_t need, hipStream_t s) {
  if (p->cs_buf && p->cs_bytes >= need) return UR_OK;
  if (graph_bound(p)) return refuse_bound(p, "cell scratch reallocation");
  hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
  if (s) (void)hipStreamIsCapturing(s, &cst);
  if (cst != hipStreamCaptureStatusNone)
    return fail(UR_ERR_STATE, "cell scratch must be allocated (first call) before graph capture");
  if (p->cs_buf) { UR_HIP(hipDeviceSynchronize()); UR_HIP(hipFree(p->cs_buf)); p->cs_buf = nullptr; }
  void* ptr = nullptr;
  if (hipMalloc(&ptr, need) != hipSuccess) { (void)hipGetLastError(); return fail(UR_ERR_OOM, "hipMalloc(%zu) failed", need); }
  p->cs_buf = (char*)ptr;
  p->cs_bytes = need;
  return UR_OK;
}

// the density buffer of oriented zoom levels: the library's own, not the
// attached workspace (whose size query covers the transform passes only)
static ur_status ensure_level_buf(ur_plan* p, size_t need, hipStream_t s) {
  if (p->lvl_buf && p->lvl_bytes >= need) return UR_OK;
  if (graph_bound(p)) return refuse_bound(p, "level density reallocation");
  hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
  if (s) (void)hipStreamIsCapturing(s, &cst);
  if (cst != hipStreamCaptureStatusNone)
    return fail(UR_ERR_STATE, "the level density buffer must be allocated (first call) before graph capture");
  if (p->lvl_buf) { UR_HIP(hipDeviceSynchronize()); UR_HIP(hipFree(p->lvl_buf)); p->lvl_buf = nullptr; p->lvl_bytes = 0; }
  void* ptr = nullptr;
  if (hipMalloc(&ptr, need) != hipSuccess) { (void)hipGetLastError(); return fail(UR_ERR_OOM, "hipMalloc(%zu) failed", need); }
  p->lvl_buf = (char*)ptr;
  p->lvl_bytes = need;
  return UR_OK;
}

// per-stage twiddle tables exp(-2 pi i r j / (L R)), evaluated in long double
// and rounded once to the working precision
static ur_status make_twiddles(ur_plan* p) {
  const long double PI = 3.14159265358979323846264338327950288L;
  int Ls[32], Rs[32];
  const int ns = fft_stages(p->n, Ls, Rs);
  if (ns <= 0) return fail(UR_ERR_UNSUPPORTED, "no transform stages for n = %d", p->n);
  std::vector<long double> re, im;
  for (int k = 0; k < ns; ++k)
    for (int j = 0; j < Ls[k]; ++j)
      for (int r = 1; r < Rs[k]; ++r) {
        long double a = 2.0L * PI * (long double)(r * j) / (long double)(Ls[k] * Rs[k]);
        re.push_back(cosl(a));
        im.push_back(-sinl(a));
      }
  const size_t m = re.size() ? re.size() : 1;
  if (p->prec == UR_F32) {
    std::vector<float> h(2 * m, 0.f);
    for (size_t i = 0; i < re.size(); ++i) { h[2 * i] = (float)re[i]; h[2 * i + 1] = (float)im[i]; }
    UR_HIP(hipMalloc(&p->tw, 2 * m * sizeof(float)));
    UR_HIP(hipMemcpy(p->tw, h.data(), 2 * m * sizeof(float), hipMemcpyHostToDevice));
  } else {
    std::vector<double> h(2 * m, 0.0);
    for (size_t i = 0; i < re.size(); ++i) { h[2 * i] = (double)re[i]; h[2 * i + 1] = (double)im[i]; }
    UR_HIP(hipMalloc(&p->tw, 2 * m * sizeof(double)));
    UR_HIP(hipMemcpy(p->tw, h.data(), 2 * m * sizeof(double), hipMemcpyHostToDevice));
  }
  return UR_OK;
}

// Integer threshold of a bin edge: t = (e/dq)^2 snapped to the nearest
// integer when within 1e-9 relative.  Evaluated without fused multiply-add
// so that every implementation of the rule gets the same bits.
#pragma clang fp contract(off)
static double snap_threshold(double e, double dq) {
  double r = e / dq;
  double t = r * r;
  double rt = nearbyint(t);
  if (fabs(t - rt) <= 1e-9 * fmax(1.0, t)) t = rt;
  return t;
}
static void thresholds(int n, double voxel, int nbins, const double* edges, std::vector<long long>& U) {
  double dq = 2.0 * M_PI / ((double)n * voxel);
  U.assign(nbins + 1, 0);
  for (int b = 0; b < nbins; ++b) {
    double t = snap_threshold(edges[b], dq);
    U[b] = t <= 0.0 ? 0 : (long long)ceil(t);
  }
  double tl = snap_threshold(edges[nbins], dq);
  U[nbins] = tl < 0.0 ? 0 : (long long)floor(tl) + 1;
}
#pragma clang fp contract(on)

// Kind of a host-side input pointer: page-locked host memory known to HIP
// (the device reads it directly), ordinary pageable (or managed) memory, or
// device memory, which the host cannot read.
enum HostKind { HOST_PAGEABLE, HOST_PINNED, HOST_DEVICE };
static HostKind host_kind(const void* ptr) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return HOST_PAGEABLE;
  }
  if (a.type == hipMemoryTypeHost) return HOST_PINNED;
  if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeArray) return HOST_DEVICE;
  return HOST_PAGEABLE;
}

// Host copy of `bytes` split over up to 16 threads (memory bandwidth, not
// one core, then bounds the pageable-to-pinned step).  Parts whose thread
// cannot be started are copied by the calling thread (no exception leaves).
static void parallel_copy(char* dst, const char* src, size_t bytes) {
  const unsigned hc = std::thread::hardware_concurrency();
  const size_t nt = std::max<size_t>(1, std::min<size_t>({16, hc ? hc : 1, bytes >> 22}));
  if (nt == 1) { memcpy(dst, src, bytes); return; }
  std::vector<std::thread> th;
  const size_t part = (bytes / nt + 4095) & ~(size_t)4095;
  for (size_t t = 0; t < nt; ++t) {
    const size_t a = t * part;
    if (a >= bytes) break;
    const size_t len = std::min(part, bytes - a);
    try {
      th.emplace_back([=] { memcpy(dst + a, src + a, len); });
    } catch (...) {
      memcpy(dst + a, src + a, len);
    }
  }
  for (auto& t : th) t.join();
}

// Boxes up to kMaxInCore^3 run every path; larger ones (kMaxOutOfCore^3,
// FP32 real) run only the out-of-core forward path, whose spectrum in HBM
// covers just the particle's planes.
static ur_status need_in_core(const ur_plan* p) {
  if (p->n > kMaxInCore)
    return fail(UR_ERR_UNSUPPORTED, "n = %d runs only out of core (ur_simulate_host); in-HBM paths run up to %d^3",
                p->n, kMaxInCore);
  return UR_OK;
}

extern "C" {

const char* ur_last_error(void) { return g_err.c_str(); }
const char* ur_version(void) { return "ultima-gfx950 0.1"; }

ur_status ur_plan_create(int32_t n, double voxel, int32_t prec, uint32_t flags, ur_plan** out) {
  if (!out) return fail(UR_ERR_INVALID, "out is null");
  *out = nullptr;
  const bool mixed = !is_pow2(n) && mr_size(n);
  if (!mixed && (!is_pow2(n) || n < 16))
    return fail(UR_ERR_INVALID, "n = %d must be a power of two >= 16 or one of the mixed-radix edges", n);
  if (n > kMaxOutOfCore) return fail(UR_ERR_UNSUPPORTED, "n = %d: boxes run up to %d^3", n, kMaxOutOfCore);
  if (n > kMaxInCore && (prec != UR_F32 || (flags & UR_C2C)))
    return fail(UR_ERR_UNSUPPORTED, "n = %d: boxes above %d^3 are FP32 real (UR_F32, no UR_C2C)", n, kMaxInCore);
  if (n > 1024 && (flags & UR_C2C) && !mixed) return fail(UR_ERR_UNSUPPORTED, "complex transforms run up to 1024^3");
  if (!(voxel > 0.0) || !isfinite(voxel)) return fail(UR_ERR_INVALID, "voxel must be positive");
  if (prec != UR_F32 && prec != UR_F64) return fail(UR_ERR_INVALID, "prec must be UR_F32 or UR_F64");
  if (flags & ~1u) return fail(UR_ERR_INVALID, "unknown flags 0x%x", flags);
  ur_plan* p = new (std::nothrow) ur_plan();
  if (!p) return fail(UR_ERR_HOST, "plan allocation failed");
  p->n = n;
  p->voxel = voxel;
  p->prec = prec;
  p->flags = flags;
  p->nkz = (flags & UR_C2C) ? n : n / 2 + 1;
  p->mixed = mixed;
  p->rs = prec == UR_F32 ? 4 : 8;
  p->cs = 2 * p->rs;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return fail(UR_ERR_HIP, "hipGetDevice failed"); }
  if (hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || p->ncu < 1) p->ncu = 256;
  ur_status st;
  try {
    st = make_twiddles(p);
  } catch (...) {
    st = fail(UR_ERR_HOST, "host allocation failed while building the twiddle tables");
  }
  if (st != UR_OK) { ur_plan_destroy(p); return st; }
  *out = p;
  return UR_OK;
}

void ur_plan_destroy(ur_plan* p) {
  if (!p) return;
  if (p->graphs > 0) {                   // graphs that still name it forget it (replaying them is invalid)
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& e : g_graph_plans) e.second.erase(std::remove(e.second.begin(), e.second.end(), p), e.second.end());
  }
  (void)hipDeviceSynchronize();
  if (p->tw) (void)hipFree(p->tw);
  if (p->dU) (void)hipFree(p->dU);
  if (p->dLut) (void)hipFree(p->dLut);
  if (p->dSinc) (void)hipFree(p->dSinc);
  if (p->dCount) (void)hipFree(p->dCount);
  if (p->dCountTmp) (void)hipFree(p->dCountTmp);
  if (p->ws && p->ws_owned) (void)hipFree(p->ws);
  if (p->cs_buf) (void)hipFree(p->cs_buf);
  if (p->lvl_buf) (void)hipFree(p->lvl_buf);
  if (p->stage) (void)hipFree(p->stage);
  if (p->bounce) (void)hipHostFree(p->bounce);
  for (auto& e : p->ev_copied) if (e) (void)hipEventDestroy(e);
  for (auto& e : p->ev_free) if (e) (void)hipEventDestroy(e);
  for (auto& c : p->copy_stream) if (c) (void)hipStreamDestroy(c);
  for (auto& e : p->ev_open) { (void)hipEventDestroy(e.second.first); (void)hipEventDestroy(e.second.second); }
  for (auto& e : p->ev_pool) (void)hipEventDestroy(e);
  delete p;
}

ur_status ur_plan_workspace_size(const ur_plan* p, int32_t nbins, size_t* bytes) {
  if (!p || !bytes) return fail(UR_ERR_INVALID, "null argument");
  if (nbins < 1) return fail(UR_ERR_INVALID, "nbins must be >= 1");
  UR_TRY(need_in_core(p));
  *bytes = p->mixed ? layout_mixed(p, nbins).total : layout_incore(p, nbins).total;
  return UR_OK;
}

ur_status ur_plan_workspace_size_host(const ur_plan* p, int32_t nbins, int32_t x_lo, int32_t x_hi, size_t* bytes) {
  if (!p || !bytes) return fail(UR_ERR_INVALID, "null argument");
  if (nbins < 1) return fail(UR_ERR_INVALID, "nbins must be >= 1");
  if (x_lo < 0 || x_hi >= p->n || x_lo > x_hi) return fail(UR_ERR_INVALID, "plane range [%d, %d] outside the box", x_lo, x_hi);
  if (p->mixed) {
    *bytes = layout_mixed_ooc(p, nbins, (size_t)(x_hi - x_lo + 1)).total;
    return UR_OK;
  }
  OocSplit o;
  UR_TRY(ooc_split(p, nbins, x_lo, x_hi, o));
  *bytes = o.lay.total;
  return UR_OK;
}

// Per-axis weight table of the binned intensities, W(m) for m in [0, n/2]
// (signed index |m|), the product of the factors that are on:
//  * voxel form factor: S(m) = (sin(pi m / n) / (pi m / n))^2;
//  * removed block transfer of a zoom level made by block sums of f:
//    1/|T(m)|^2 = (f sin(pi m / (f n)) / sin(pi m / n))^2, the inverse of the
//    power of (1/f) sum_{j<f} exp(2 pi i m j / (f n)) (a sum of f phasors).
// Evaluated in long double and rounded once to the working precision.
static ur_status rebuild_weights(ur_plan* p, bool vox, int bt_f) {
  const bool on = vox || bt_f > 1;
  const bool same = on == (p->dSinc != nullptr) && (!on || (vox == p->vox && bt_f == p->bt_f));
  if (same) return UR_OK;
  if (graph_bound(p)) return refuse_bound(p, "a change of the intensity weights (voxel form factor, block transfer)");
  std::vector<double> v64;
  std::vector<float> v32;
  const int h = p->n / 2;
  if (on) {
    const long double PI = 3.14159265358979323846264338327950288L;
    try {
      v64.resize(h + 1);
      for (int m = 0; m <= h; ++m) {
        long double w = 1.0L;
        if (m > 0) {
          const long double x = PI * (long double)m / (long double)p->n;
          if (vox) { const long double sc = sinl(x) / x; w *= sc * sc; }
          if (bt_f > 1) {
            const long double r = (long double)bt_f * sinl(x / (long double)bt_f) / sinl(x);
            w *= r * r;
          }
        }
        v64[m] = (double)w;
      }
      if (p->prec == UR_F32) v32.assign(v64.begin(), v64.end());
    } catch (...) {
      return fail(UR_ERR_HOST, "host allocation failed for the intensity weight table");
    }
  }
  if (p->dSinc) { UR_HIP(hipDeviceSynchronize()); UR_HIP(hipFree(p->dSinc)); p->dSinc = nullptr; }
  p->vox = vox;
  p->bt_f = bt_f > 1 ? bt_f : 0;
  if (!on) return UR_OK;
  const size_t bytes = (size_t)(h + 1) * p->rs;
  UR_HIP(hipMalloc(&p->dSinc, bytes));
  UR_HIP(hipMemcpy(p->dSinc, p->prec == UR_F32 ? (const void*)v32.data() : (const void*)v64.data(), bytes,
                   hipMemcpyHostToDevice));
  return UR_OK;
}

ur_status ur_plan_set_voxel_form(ur_plan* p, int32_t enable) {
  if (!p) return fail(UR_ERR_INVALID, "plan is null");
  return rebuild_weights(p, enable != 0, p->bt_f);
}

ur_status ur_plan_set_block_transfer(ur_plan* p, int32_t factor) {
  if (!p) return fail(UR_ERR_INVALID, "plan is null");
  if (factor < 0) return fail(UR_ERR_INVALID, "block factor %d is negative", factor);
  if (p->mixed && factor > 1) return fail(UR_ERR_UNSUPPORTED, "mixed-radix boxes run without the block-transfer correction");
  return rebuild_weights(p, p->vox, factor);
}

// a plan that removes the block transfer of factor f bins only levels made
// with that factor
static ur_status check_block_transfer(const ur_plan* p, const ur_zoom* z) {
  if (p->bt_f > 1 && z->factor != p->bt_f)
    return fail(UR_ERR_INVALID, "the plan removes the block transfer of factor %d, the level has factor %d", p->bt_f, z->factor);
  return UR_OK;
}

ur_status ur_plan_set_hbm_budget(ur_plan* p, size_t bytes) {
  if (!p) return fail(UR_ERR_INVALID, "plan is null");
  p->hbm_budget = bytes;
  return UR_OK;
}

ur_status ur_plan_set_workspace(ur_plan* p, void* dev_ptr, size_t bytes) {
  if (p) p->keep_valid = false;
  if (!p || !dev_ptr) return fail(UR_ERR_INVALID, "null argument");
  if (((uintptr_t)dev_ptr) & 255) return fail(UR_ERR_INVALID, "workspace must be 256-byte aligned");
  if (graph_bound(p) && dev_ptr != (void*)p->ws) return refuse_bound(p, "ur_plan_set_workspace");
  if (p->ws && p->ws_owned) { UR_HIP(hipDeviceSynchronize()); UR_HIP(hipFree(p->ws)); }
  p->ws = (char*)dev_ptr;
  p->ws_bytes = bytes;
  p->ws_owned = false;
  return UR_OK;
}

ur_status ur_plan_set_timing(ur_plan* p, int32_t enable) {
  if (!p) return fail(UR_ERR_INVALID, "plan is null");
  p->timing = enable != 0;
  return UR_OK;
}

ur_status ur_plan_read_timing(ur_plan* p, int32_t npass, double* ms, double* bytes, int32_t* launches) {
  if (!p || !ms || !bytes || !launches) return fail(UR_ERR_INVALID, "null argument");
  if (npass < 1 || npass > 5) return fail(UR_ERR_INVALID, "npass must be in [1, 5]");
  for (int i = 0; i < npass; ++i) { ms[i] = 0.0; bytes[i] = p->pass_bytes[i]; launches[i] = 0; }
  for (auto& e : p->ev_open) {
    UR_HIP(hipEventSynchronize(e.second.second));
    float t = 0.f;
    UR_HIP(hipEventElapsedTime(&t, e.second.first, e.second.second));
    if (e.first < npass) { ms[e.first] += t; launches[e.first] += 1; }
  }
  for (auto& e : p->ev_open) {                 // back to the pool, or destroyed when it cannot grow
    for (hipEvent_t ev : {e.second.first, e.second.second}) {
      try {
        p->ev_pool.push_back(ev);
      } catch (...) {
        (void)hipEventDestroy(ev);
      }
    }
  }
  p->ev_open.clear();
  return UR_OK;
}

static ur_status set_bins_impl(ur_plan* p, int32_t nbins, const double* edges);

ur_status ur_plan_set_bins(ur_plan* p, int32_t nbins, const double* edges) {
  try {
    return set_bins_impl(p, nbins, edges);
  } catch (...) {
    return fail(UR_ERR_HOST, "host allocation failed while setting the bins");
  }
}

static ur_status set_bins_impl(ur_plan* p, int32_t nbins, const double* edges) {
  if (p) p->keep_valid = false;
  if (!p || !edges) return fail(UR_ERR_INVALID, "null argument");
  if (nbins < 1 || nbins > 4096) return fail(UR_ERR_INVALID, "nbins = %d outside [1, 4096]", nbins);
  if (graph_bound(p)) return refuse_bound(p, "ur_plan_set_bins");
  for (int b = 0; b <= nbins; ++b)
    if (!isfinite(edges[b]) || (b > 0 && !(edges[b] > edges[b - 1])))
      return fail(UR_ERR_INVALID, "bin edges must be finite and strictly increasing (edge %d)", b);
  std::vector<long long> U;
  thresholds(p->n, p->voxel, nbins, edges, U);
  long long n2max = 3ll * (p->n / 2) * (p->n / 2);
  std::vector<int> Ui(nbins + 1);
  for (int b = 0; b <= nbins; ++b) Ui[b] = (int)std::min<long long>(U[b], n2max + 1);
  if (p->dU && p->nbins < nbins) {
    UR_HIP(hipFree(p->dU)); p->dU = nullptr;
    UR_HIP(hipFree(p->dCount)); p->dCount = nullptr;
    UR_HIP(hipFree(p->dCountTmp)); p->dCountTmp = nullptr;
  }
  if (!p->dU) {
    UR_HIP(hipMalloc(&p->dU, (nbins + 1) * sizeof(int)));
    UR_HIP(hipMalloc(&p->dCount, nbins * sizeof(double)));
    UR_HIP(hipMalloc(&p->dCountTmp, nbins * sizeof(unsigned long long)));
  }
  UR_HIP(hipMemcpy(p->dU, Ui.data(), (nbins + 1) * sizeof(int), hipMemcpyHostToDevice));
  // start-of-walk table for the binning: the bin of n2 = s^2 for every
  // s <= isqrt(n2max) (-1 below the first threshold, nbins above the last)
  {
    const int nl = lut_len(p->n);
    std::vector<short> lut(nl);
    int b = -1;
    for (int sq = 0; sq < nl; ++sq) {
      const long long v = (long long)sq * sq;
      while (b < nbins && v >= (long long)Ui[b + 1]) ++b;
      lut[sq] = (short)b;
    }
    if (p->dLut && p->nlut < nl) { UR_HIP(hipFree(p->dLut)); p->dLut = nullptr; }
    if (!p->dLut) UR_HIP(hipMalloc(&p->dLut, nl * sizeof(short)));
    UR_HIP(hipMemcpy(p->dLut, lut.data(), nl * sizeof(short), hipMemcpyHostToDevice));
    p->nlut = nl;
  }
  // voxel counts per bin: pure geometry of the box and the thresholds
  UR_HIP(launch_bin_counts(p->n, p->nkz, !(p->flags & UR_C2C), nbins, p->dU, p->dCountTmp, p->dCount, nullptr));
  UR_HIP(hipDeviceSynchronize());
  p->nbins = nbins;
  p->U = U;
  return UR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// shared pieces of the forward path
// ---------------------------------------------------------------------------
static ur_status check_hist(const ur_hist* h) {
  if (!h || !h->sum || !h->sumsq || !h->count || !h->totals) return fail(UR_ERR_INVALID, "histogram pointers must be non-null");
  return UR_OK;
}

// any_edge: the call takes cell edges that are not powers of two (cell
// synthesis, and aligned ED-1 of mixed-radix plans, whose generator wraps by a
// modulo); every other generator wraps with a bit mask
static ur_status check_cell(const ur_cell* c, bool any_edge = false) {
  if (!c) return fail(UR_ERR_INVALID, "cell is null");
  if (c->c < 1 || c->c > 256 || (!any_edge && !is_pow2(c->c)))
    return fail(UR_ERR_INVALID, "cell edge %d must be a power of two <= 256 (any edge <= 256 on mixed-radix plans)", c->c);
  if (c->n_atoms < 0 || c->n_atoms > (1 << 20)) return fail(UR_ERR_INVALID, "n_atoms = %d out of range", c->n_atoms);
  if (c->n_atoms > 0 && (!c->xyz || !c->amp || !c->sigma)) return fail(UR_ERR_INVALID, "atom arrays must be non-null");
  if (!isfinite(c->background)) return fail(UR_ERR_INVALID, "background must be finite");
  if (c->rot)
    for (int i = 0; i < 9; ++i)
      if (!isfinite(c->rot[i])) return fail(UR_ERR_INVALID, "lattice rotation entry %d is not finite", i);
  if (c->interp != 0 && c->interp != 1 && c->interp != 3)
    return fail(UR_ERR_INVALID, "interp = %d: 1 (trilinear) or 3 (cubic B-spline)", c->interp);
  if (c->n_grains < 0 || c->n_grains > kMaxGrains)
    return fail(UR_ERR_INVALID, "n_grains = %d outside [0, %d]", c->n_grains, kMaxGrains);
  if (c->n_grains > 0) {
    if (c->rot) return fail(UR_ERR_INVALID, "give either rot or grains, not both");
    if (!c->grain_seed || !c->grain_rot) return fail(UR_ERR_INVALID, "grain arrays must be non-null");
    for (int i = 0; i < 3 * c->n_grains; ++i) {
      const double v = c->grain_seed[i];
      if (!isfinite(v) || v != floor(v) || fabs(v) > 8192.0)
        return fail(UR_ERR_INVALID, "grain seed entry %d must be an integer of magnitude <= 8192", i);
    }
    for (int i = 0; i < 9 * c->n_grains; ++i)
      if (!isfinite(c->grain_rot[i])) return fail(UR_ERR_INVALID, "grain orientation entry %d is not finite", i);
  }
  return UR_OK;
}

// a lattice that is not aligned with the box: one orientation or grains
static bool oriented(const ur_cell* c) { return c->rot || c->n_grains > 0; }

// A rotated lattice runs the ED-1 generator of real plans only; copies its
// matrix into the z-pass arguments.
// zoom levels of oriented lattices are generated as a density first
// (ur_simulate, ur_rho_generate: allow_zoom), the other entries take ED-1
static ur_status set_rotation(const ur_plan* p, const ur_cell* cell, const ur_zoom* zoom, ZArgs& za,
                              bool allow_zoom = false) {
  if (!oriented(cell)) return UR_OK;
  if (zoom->factor != 1 && !allow_zoom)
    return fail(UR_ERR_UNSUPPORTED, "this entry runs rotated lattices at zoom factor 1");
  if (p->flags & UR_C2C) return fail(UR_ERR_UNSUPPORTED, "rotated lattices run on real (UR_R2C) plans");
  za.rotated = 1;
  za.cubic = cell->interp == 3 ? 1 : 0;
  za.ngrain = cell->n_grains;
  if (cell->rot)
    for (int i = 0; i < 9; ++i) za.rot[i] = cell->rot[i];
  for (int g = 0; g < cell->n_grains; ++g) {
    for (int i = 0; i < 3; ++i) za.gseed[g][i] = (int)cell->grain_seed[3 * g + i];
    for (int i = 0; i < 9; ++i) za.grot[g][i] = cell->grain_rot[9 * g + i];
  }
  return UR_OK;
}

static ur_status check_level(const ur_plan* p, const ur_cell* cell, const ur_mask* m, const ur_zoom* z, Level& L, MaskP& mp) {
  if (!m || !z) return fail(UR_ERR_INVALID, "mask and zoom must be non-null");
  if (m->kind < 0 || m->kind > 3) return fail(UR_ERR_INVALID, "mask kind %d unknown", m->kind);
  if (m->p0 > (1ll << 40) || m->p1 > (1ll << 40)) return fail(UR_ERR_INVALID, "mask parameters too large");
  if (z->factor < 1 || z->n1 < 1) return fail(UR_ERR_INVALID, "zoom factor %d and n1 %d must be positive", z->factor, z->n1);
  if (p->mixed) {
    // ED-1 (n1 = n, factor 1) or a zoom level of any even ED-1 edge by any
    // factor dividing it (the prefix-sum tables need power-of-two cells)
    if (z->factor == 1 && z->n1 != p->n) return fail(UR_ERR_UNSUPPORTED, "mixed-radix ED-1 levels have n1 = n");
    if (z->factor > 1 && (!is_pow2(cell->c) || z->n1 % z->factor || z->n1 % 2 || z->n1 < 2))
      return fail(UR_ERR_UNSUPPORTED, "mixed-radix zoom levels take power-of-two cells and an even n1 divisible by the factor");
  } else if (!is_pow2(z->n1) || !is_pow2(z->factor)) {
    return fail(UR_ERR_INVALID, "zoom n1 and factor must be powers of two");
  }
  if (z->factor > 1 && z->factor > z->n1 / 2) return fail(UR_ERR_INVALID, "zoom factor %d too large for n1 = %d", z->factor, z->n1);
  if (z->n1 / z->factor > p->n) return fail(UR_ERR_INVALID, "reduced particle region %d exceeds the box %d", z->n1 / z->factor, p->n);
  if (z->factor > 1 && cell->c > z->n1) return fail(UR_ERR_INVALID, "cell larger than the ED-1 grid");
  L = make_level(p->n, z->n1, z->factor, cell->c);
  mp.kind = m->kind;
  mp.p0 = m->p0;
  mp.p1 = m->p1;
  return UR_OK;
}

struct CellTables {
  double* prof;
  double* cell64;
  void* cellT;
  double* pre;
  void* cb;
  double* gcell;
  double* fold_part;
  int cbn;
};

static const int kFoldBlocks = 512;

// Byte offsets of the cell tables; `fold` adds the adjoint's fold buffers.
struct CellLayout {
  size_t prof, cell, cellT, pre, cb, g, fp, total;
};
static CellLayout cell_layout(const ur_plan* p, const ur_cell* cell, int f, bool fold) {
  const size_t c = cell->c, c3 = c * c * c;
  const int cbn = f <= (int)c ? (int)c / f : 1;
  const size_t nb = (size_t)cbn * cbn * cbn;
  CellLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.prof = take(std::max<size_t>(1, (size_t)cell->n_atoms * 3 * c) * 8);
  L.cell = take(c3 * 8);
  L.cellT = take(c3 * p->rs);
  L.pre = take(c * c * (c + 1) * 8);
  L.cb = take(nb * p->rs);
  L.g = fold ? take(c3 * 8) : 0;
  L.fp = fold ? take((c <= 16 ? (size_t)kFoldBlocks * c3 : 1) * 8) : 0;
  L.total = off;
  return L;
}

// cell synthesis + tables for the generator (a1 of the path), in the plan's
// cell scratch, or at `base` (the static scratch of the allocation-free entry)
static ur_status prepare_cell(ur_plan* p, const ur_cell* cell, int f, CellTables& t, hipStream_t s,
                              char* base = nullptr) {
  const CellLayout CL = cell_layout(p, cell, f, base == nullptr);
  t.cbn = f <= (int)cell->c ? (int)cell->c / f : 1;
  const size_t o_prof = CL.prof, o_cell = CL.cell, o_cellT = CL.cellT, o_pre = CL.pre, o_cb = CL.cb, o_g = CL.g,
               o_fp = CL.fp;
  if (!base) UR_TRY(ensure_cell_scratch(p, CL.total, s));
  char* b = base ? base : p->cs_buf;
  t.prof = (double*)(b + o_prof);
  t.cell64 = (double*)(b + o_cell);
  t.cellT = b + o_cellT;
  t.pre = (double*)(b + o_pre);
  t.cb = b + o_cb;
  t.gcell = base ? nullptr : (double*)(b + o_g);
  t.fold_part = base ? nullptr : (double*)(b + o_fp);
  const bool spline = oriented(cell) && cell->interp == 3;
  UR_HIP(launch_cell_profiles(cell->c, cell->n_atoms, cell->xyz, cell->sigma, t.prof, s));
  if (f == 1 && !spline) {
    // a level of factor 1 needs only the working-precision copy: the sum writes it
    UR_HIP(launch_cell_sum(cell->c, cell->n_atoms, cell->amp, t.prof, cell->background, t.cell64, s, p->prec, t.cellT));
    return UR_OK;
  }
  UR_HIP(launch_cell_sum(cell->c, cell->n_atoms, cell->amp, t.prof, cell->background, t.cell64, s));
  if (spline) UR_HIP(launch_bspline_cell(cell->c, t.cell64, s));   // spline coefficients
  UR_HIP(launch_cell_tables(p->prec, cell->c, f, t.cell64, t.cellT, t.pre, t.cb, t.cbn, s));
  return UR_OK;
}

// passes Y and X + finalize, given A written for planes [xlo, xhi]
struct FwdGeom {
  int xlo, xhi;          // planes of A that hold data
  long long ax0;         // first plane held by A
  int gen;               // A rows limited to the particle row range
  Level L;
  MaskP m;
};

// rows of the first intermediate that hold data, summed over planes
static double live_rows(const ur_plan* p, const FwdGeom& g) {
  if (g.xlo > g.xhi) return 0.0;
  if (!g.gen) return (double)(g.xhi - g.xlo + 1) * p->n;
  const int ty = zt(p);
  double rows = 0.0;
  for (long long x = g.xlo; x <= g.xhi; ++x) {
    long long lo, hi;
    row_range(g.L, g.m, x, lo, hi);
    if (lo <= hi) rows += (double)((hi / ty - lo / ty + 1) * ty);
  }
  return rows;
}

static ur_status run_y_x(ur_plan* p, const FwdGeom& g, char* A, char* B, const Layout& lay,
                         const ur_hist* h, int nzb, hipStream_t s, char* ws) {
  const int n = p->n, tx = y_tile(p->prec, n);
  const double rows = live_rows(p, g);
  long long xt0 = 0, xt1 = -1, bx0 = 0, bs = tx;
  if (g.xlo <= g.xhi) {
    xt0 = g.xlo / tx;
    xt1 = g.xhi / tx;
    bx0 = xt0 * tx;
    bs = (xt1 - xt0 + 1) * tx;
    YArgs ya{};
    ya.A = A; ya.ax0 = g.ax0; ya.B = B; ya.bx0 = bx0; ya.bs = bs; ya.tw = p->tw;
    ya.L = g.L; ya.m = g.m; ya.gen = g.gen; ya.nkz = p->nkz; ya.xlo = g.xlo; ya.xhi = g.xhi;
    ya.xt0 = (int)xt0; ya.nxt = (int)(xt1 - xt0 + 1); ya.ty = zt(p);
    PassTimer tm(p, P_Y, s);
    UR_HIP(launch_pass_y(p->prec, n, ya, s));
  }
  const double spec_x = (double)p->nkz * n * (double)bs * p->cs;      // B over the live x range
  const int nxb = x_blocks(p);
  const double part_bytes = (double)nxb * (2.0 * p->nbins + 1.0) * 8.0;
  p->pass_bytes[P_Y] = g.xlo <= g.xhi ? rows * p->nkz * p->cs + spec_x : 0.0;
  p->pass_bytes[P_X] = (g.xlo <= g.xhi ? spec_x : 0.0) + part_bytes;
  p->pass_bytes[P_FIN] = part_bytes + 16.0 * nzb + 24.0 * p->nbins;
  XArgs xa{};
  xa.B = B; xa.bx0 = bx0; xa.bs = bs; xa.out = nullptr; xa.tw = p->tw;
  xa.nkz = p->nkz; xa.r2c = !(p->flags & UR_C2C);
  xa.xa = (int)bx0; xa.xb = g.xlo <= g.xhi ? (int)(bx0 + bs - 1) : -1;
  xa.iscale = 1.0 / ((double)n * n * n) / ((double)n * n * n);
  xa.oscale = 1.0; xa.nbins = p->nbins; xa.U = p->dU; xa.lut = p->dLut; xa.nlut = p->nlut; xa.sinc = p->dSinc;
  xa.part = (double*)(ws + lay.part); xa.f0 = (double*)(ws + lay.f0);
  xa.ncols = p->nkz * n;
  {
    PassTimer tm(p, P_X, s);
    UR_HIP(launch_pass_x(p->prec, n, X_FFT_BIN, -1, xa, nxb, s));
  }
  FinArgs fa{};
  fa.part = xa.part; fa.nblk = nxb; fa.nbins = p->nbins;
  fa.mom = nzb > 0 ? (const double*)(ws + lay.mom) : nullptr; fa.nzb = nzb;
  fa.mpart = (double*)(ws + lay.f0 + 64); fa.f0 = xa.f0; fa.cnt = p->dCount; fa.sum = h->sum; fa.sumsq = h->sumsq; fa.count = h->count; fa.totals = h->totals; fa.mean = h->mean; fa.sem = h->sem;
  {
    PassTimer tm(p, P_FIN, s);
    UR_HIP(launch_finalize(fa, s));
  }
  return UR_OK;
}

// mixed-radix passes in place on S: z (from `src`, or generated from `gen`,
// with per-block moments into `mom` when given), y, then x (scaled by 1/n^3
// forward); with `lay` the forward x pass bins |F|^2 instead of storing it
// (block partials and F(0) at their places in the workspace).  With `region`
// (the level whose density src holds or gen generates) the binning path is
// pruned as the power-of-two passes are: the z pass leaves the lines of
// pencils outside the region unwritten, the y pass runs the region's planes
// only and reads rows outside each plane's row range as zero, and the x pass
// reads those planes and takes the others as zero.
static ur_status mr_transform(ur_plan* p, const void* src, void* S, int dir, double* mom, const ZArgs* gen,
                              const Layout* lay, hipStream_t s, const ZArgs* region = nullptr) {
  const int n = p->n;
  const bool r2c = !(p->flags & UR_C2C);
  if (r2c && dir > 0) return fail(UR_ERR_UNSUPPORTED, "real mixed-radix plans run the forward transform only");
  MrArgs a{};
  a.tw = p->tw; a.dst = S; a.mom = mom; a.src = src; a.scale = 1.0;
  if (gen) a.z = *gen;
  // the binning path's box lives in the workspace: padded rows (a spectrum
  // written for the caller keeps the natural layout)
  if (lay && r2c) a.nzp = mixed_pitch(p);
  long long xlo = 0, xhi = n - 1;
  double rows = (double)n * n;                       // (x, y) lines that hold data
  if (region && lay && dir < 0) {
    plane_range(region->L, region->m, xlo, xhi);
    if (xlo <= xhi) {
      a.z.L = region->L;
      a.z.m = region->m;
      a.prune = 1;
      rows = 0.0;
      for (long long x = xlo; x <= xhi; ++x) {
        long long lo, hi;
        row_range(region->L, region->m, x, lo, hi);
        if (lo <= hi) rows += (double)(hi - lo + 1);
      }
    } else {
      xlo = 0;
      xhi = n - 1;
    }
  }
  const size_t plane = (size_t)n * (a.nzp > 0 ? a.nzp : p->nkz) * p->cs;   // one x plane of the box
  {
    PassTimer tm(p, P_Z, s);
    UR_HIP(launch_mr_axis(p->prec, n, 2, dir, gen ? MR_GEN : MR_LOAD, r2c, a, s));
  }
  a.src = S; a.mom = nullptr;
  if (a.prune) { a.px0 = (int)xlo; a.planes = (int)(xhi - xlo + 1); }
  {
    PassTimer tm(p, P_Y, s);
    UR_HIP(launch_mr_axis(p->prec, n, 1, dir, MR_LOAD, r2c, a, s));
  }
  a.px0 = 0; a.planes = 0;
  a.scale = dir < 0 ? 1.0 / ((double)n * n * n) : 1.0;
  if (lay) {
    a.nbins = p->nbins; a.U = p->dU; a.lut = p->dLut; a.iscale = 1.0;
    a.part = (double*)(p->ws + lay->part); a.f0 = (double*)(p->ws + lay->f0);
  }
  if (a.prune) { a.src = (const char*)S + (size_t)xlo * plane; a.xa = (int)xlo; a.xn = (int)(xhi - xlo + 1); }
  {
    PassTimer tm(p, P_X, s);
    UR_HIP(launch_mr_axis(p->prec, n, 0, dir, lay ? MR_BIN : MR_LOAD, r2c, a, s));
  }
  // algorithmic bytes: nkz complex elements per (x, y) line that holds data
  // (z pass writes, y pass reads), per line of the planes run (y pass
  // writes, x pass reads); a real input of n reals per line
  const double nx = (double)(xhi - xlo + 1);
  const double line = (double)p->nkz * p->cs;
  const double in = r2c ? rows * n * p->rs : rows * line;
  p->pass_bytes[P_Z] = (gen ? 0.0 : in) + rows * line;
  p->pass_bytes[P_Y] = rows * line + nx * n * line;
  p->pass_bytes[P_X] = (lay ? 1.0 : 2.0) * nx * n * line;
  return UR_OK;
}

// finalize of the block partials written by the binning x pass (or k_mr_bin)
static ur_status mr_finalize(ur_plan* p, const Layout& lay, int nblk, const ur_hist* h, int nzb, hipStream_t s) {
  FinArgs fa{};
  fa.part = (const double*)(p->ws + lay.part); fa.nblk = nblk; fa.nbins = p->nbins;
  fa.mom = nzb > 0 ? (const double*)(p->ws + lay.mom) : nullptr; fa.nzb = nzb;
  fa.mpart = (double*)(p->ws + lay.f0 + 64); fa.f0 = (const double*)(p->ws + lay.f0); fa.cnt = p->dCount;
  fa.sum = h->sum; fa.sumsq = h->sumsq; fa.count = h->count; fa.totals = h->totals; fa.mean = h->mean; fa.sem = h->sem;
  PassTimer tm(p, P_FIN, s);
  UR_HIP(launch_finalize(fa, s));
  p->pass_bytes[P_FIN] = (double)nblk * (2.0 * p->nbins + 1.0) * 8.0 + 16.0 * nzb;
  return UR_OK;
}

// |F|^2 binning of a given spectrum and the finalize
static ur_status mr_bin(ur_plan* p, const void* S, const Layout& lay, const ur_hist* h, hipStream_t s) {
  MrBinArgs b{};
  b.S = S; b.n = p->n; b.nbins = p->nbins; b.U = p->dU; b.lut = p->dLut; b.nlut = p->nlut; b.iscale = 1.0;
  b.r2c = (p->flags & UR_C2C) ? 0 : 1;
  b.part = (double*)(p->ws + lay.part); b.f0 = (double*)(p->ws + lay.f0);
  const int nblk = (int)std::min<long long>((long long)p->n * p->n, kMaxXBlocks);
  {
    PassTimer tm(p, P_X, s);
    UR_HIP(launch_mr_bin(p->prec, b, nblk, s));
  }
  p->pass_bytes[P_X] = (double)p->n * p->n * p->nkz * p->cs;
  return mr_finalize(p, lay, nblk, h, 0, s);
}

extern "C" {

ur_status ur_cell_synth(ur_plan* p, const ur_cell* cell, double* cell_out, void* stream) {
  if (p) p->keep_valid = false;
  if (!p || !cell_out) return fail(UR_ERR_INVALID, "null argument");
  UR_TRY(check_cell(cell, true));
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  size_t need = align256(std::max<size_t>(1, (size_t)cell->n_atoms * 3 * cell->c) * 8);
  UR_TRY(ensure_cell_scratch(p, std::max(need, p->cs_bytes), s));
  double* prof = (double*)p->cs_buf;
  UR_HIP(launch_cell_profiles(cell->c, cell->n_atoms, cell->xyz, cell->sigma, prof, s));
  UR_HIP(launch_cell_sum(cell->c, cell->n_atoms, cell->amp, prof, cell->background, cell_out, s));
  return UR_OK;
}

ur_status ur_rho_generate(ur_plan* p, const ur_cell* cell, const ur_mask* mask, const ur_zoom* zoom, int32_t x_lo,
                          int32_t x_hi, void* rho, void* stream) {
  if (p) p->keep_valid = false;
  if (!p || !rho) return fail(UR_ERR_INVALID, "null argument");
  if (x_lo < 0 || x_hi >= p->n || x_lo > x_hi) return fail(UR_ERR_INVALID, "plane range [%d, %d] outside the box", x_lo, x_hi);
  UR_TRY(check_cell(cell));
  Level L;
  MaskP m;
  UR_TRY(check_level(p, cell, mask, zoom, L, m));
  if (p->mixed && oriented(cell)) return fail(UR_ERR_UNSUPPORTED, "mixed-radix boxes run lattices aligned with the box");
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  CellTables t;
  UR_TRY(prepare_cell(p, cell, zoom->factor, t, s));
  ZArgs za{};
  za.cellT = t.cellT; za.cb = t.cb; za.pre = t.pre; za.L = L; za.m = m; za.cbn = t.cbn;
  UR_TRY(set_rotation(p, cell, zoom, za, true));
  if (za.rotated && zoom->factor > 1 && p->n > kZoomRotMaxBox)
    return fail(UR_ERR_UNSUPPORTED, "zoom levels of rotated lattices run in boxes up to %d", kZoomRotMaxBox);
  UR_HIP(launch_rho_generate(p->prec, p->n, x_lo, x_hi, za, rho, s));
  return UR_OK;
}

}  // extern "C"
static ur_status simulate_pow2(ur_plan* p, const ur_cell* cell, const ur_zoom* zoom, const ur_hist* h, hipStream_t s,
                               FwdGeom g, const ZArgs& rot_args, const CellTables& t, const Layout& lay, char* ws);
static ur_status simulate_rho_pow2(ur_plan* p, const void* rho, const ur_hist* h, const Layout& lay, hipStream_t s);
extern "C" {

ur_status ur_simulate(ur_plan* p, const ur_cell* cell, const ur_mask* mask, const ur_zoom* zoom, const ur_hist* h, void* stream) {
  if (p) p->keep_valid = false;
  if (!p) return fail(UR_ERR_INVALID, "plan is null");
  UR_TRY(need_in_core(p));
  if (p->nbins < 1) return fail(UR_ERR_STATE, "no bins set on the plan");
  UR_TRY(check_hist(h));
  UR_TRY(check_cell(cell, p->mixed));
  FwdGeom g;
  UR_TRY(check_level(p, cell, mask, zoom, g.L, g.m));
  UR_TRY(check_block_transfer(p, zoom));
  if (p->mixed && oriented(cell)) return fail(UR_ERR_UNSUPPORTED, "mixed-radix boxes run lattices aligned with the box");
  ZArgs rot_args{};
  UR_TRY(set_rotation(p, cell, zoom, rot_args, !p->mixed));
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  if (p->mixed) {
    if (p->dSinc) return fail(UR_ERR_UNSUPPORTED, "mixed-radix boxes run without the voxel form factor and block-transfer correction");
    Layout lay = layout_mixed(p, p->nbins);
    UR_TRY(ensure_ws(p, lay.total, s));
    CellTables t;
    {
      PassTimer tm(p, P_CELL, s);
      UR_TRY(prepare_cell(p, cell, zoom->factor, t, s));
    }
    {
      const double c = cell->c;
      p->pass_bytes[P_CELL] = 8.0 * (3.0 * c * cell->n_atoms) * 2.0 + c * c * c * (16.0 + p->rs);
    }
    ZArgs za = rot_args;
    za.cellT = t.cellT; za.cb = t.cb; za.pre = t.pre; za.L = g.L; za.m = g.m; za.cbn = t.cbn;
    double* mom = (double*)(p->ws + lay.mom);
    if (zoom->factor > 1) {
      if (!(p->flags & UR_C2C)) {
        // real box: the level's density into the plan's level buffer, then
        // the three passes from it (the z pass pairs its real pencils)
        UR_TRY(ensure_level_buf(p, (size_t)p->n * p->n * p->n * p->rs, s));
        UR_HIP(launch_rho_generate(p->prec, p->n, 0, p->n - 1, za, p->lvl_buf, s));
        UR_TRY(mr_transform(p, p->lvl_buf, p->ws + lay.A, -1, mom, nullptr, &lay, s, &za));
        return mr_finalize(p, lay, mr_axis_blocks(p->prec, p->n, 0, MR_BIN, true), h,
                           mr_axis_blocks(p->prec, p->n, 2, MR_LOAD, true), s);
      }
      // zoom level: block sums of ED-1 written as a complex box first, then
      // the three passes from it (the generating z pass serves ED-1 only)
      UR_HIP(launch_level_complex(p->prec, p->n, za, p->ws + lay.A, mom, s));
      UR_TRY(mr_transform(p, p->ws + lay.A, p->ws + lay.A, -1, nullptr, nullptr, &lay, s, &za));
      return mr_finalize(p, lay, mr_axis_blocks(p->prec, p->n, 0, MR_BIN, false), h, p->n * p->n, s);
    }
    UR_TRY(mr_transform(p, nullptr, p->ws + lay.A, -1, mom, &za, &lay, s, &za));
    return mr_finalize(p, lay, mr_axis_blocks(p->prec, p->n, 0, MR_BIN, !(p->flags & UR_C2C)), h, mr_axis_blocks(p->prec, p->n, 2, MR_GEN, !(p->flags & UR_C2C)), s);
  }
  Layout lay = layout_incore(p, p->nbins);
  if (rot_args.rotated && zoom->factor > 1) {
    // zoom level of an oriented lattice: the level's density (block sums of
    // the oriented ED-1) is generated into the plan's level buffer first,
    // then transformed and binned as a given density
    if (p->n > kZoomRotMaxBox)
      return fail(UR_ERR_UNSUPPORTED, "zoom levels of rotated lattices run in boxes up to %d", kZoomRotMaxBox);
    UR_TRY(ensure_ws(p, lay.total, s));
    UR_TRY(ensure_level_buf(p, (size_t)p->n * p->n * p->n * p->rs, s));
    CellTables t;
    ZArgs za = rot_args;
    {
      PassTimer tm(p, P_CELL, s);
      UR_TRY(prepare_cell(p, cell, 1, t, s));
      za.cellT = t.cellT; za.cb = t.cb; za.pre = t.pre; za.L = g.L; za.m = g.m; za.cbn = t.cbn;
      UR_HIP(launch_rho_generate(p->prec, p->n, 0, p->n - 1, za, p->lvl_buf, s));
    }
    {
      const double c = cell->c;
      p->pass_bytes[P_CELL] = 8.0 * (3.0 * c * cell->n_atoms) * 2.0 + c * c * c * (16.0 + p->rs) +
                              (double)p->n * p->n * p->n * p->rs;
    }
    return simulate_rho_pow2(p, p->lvl_buf, h, lay, s);
  }
  UR_TRY(ensure_ws(p, lay.total, s));
  CellTables t;
  {
    PassTimer tm(p, P_CELL, s);
    UR_TRY(prepare_cell(p, cell, zoom->factor, t, s));
  }
  return simulate_pow2(p, cell, zoom, h, s, g, rot_args, t, lay, p->ws);
}

}  // extern "C"

// passes Z, Y, X and the finalize of a power-of-two box, with the transform
// intermediates and partials at `ws` (layout `lay`) and the cell tables `t`
static ur_status simulate_pow2(ur_plan* p, const ur_cell* cell, const ur_zoom* zoom, const ur_hist* h, hipStream_t s,
                               FwdGeom g, const ZArgs& rot_args, const CellTables& t, const Layout& lay, char* ws) {
  {
    const double c = cell->c;
    p->pass_bytes[P_CELL] = 8.0 * (3.0 * c * cell->n_atoms) * 2.0 + c * c * c * (16.0 + p->rs);
  }

  long long xlo, xhi;
  plane_range(g.L, g.m, xlo, xhi);
  if (xlo < 0) xlo = 0;
  if (xhi > p->n - 1) xhi = p->n - 1;
  g.xlo = (int)xlo; g.xhi = (int)xhi; g.ax0 = xlo; g.gen = 1;
  int nzb = 0;
  if (xlo <= xhi) {
    ZArgs za = rot_args;
    za.A = ws + lay.A; za.ax0 = xlo; za.cellT = t.cellT; za.cb = t.cb; za.pre = t.pre; za.tw = p->tw;
    za.mom = (double*)(ws + lay.mom); za.L = g.L; za.m = g.m; za.nkz = p->nkz; za.x0 = (int)xlo;
    za.ntiles = ntiles(p); za.cbn = t.cbn;
    nzb = (int)((xhi - xlo + 1) * za.ntiles);
    PassTimer tm(p, P_Z, s);
    const int zm = za.rotated ? (za.cubic ? (za.ngrain ? Z_ROT3G_R2C : Z_ROT3_R2C) : (za.ngrain ? Z_ROTG_R2C : Z_ROT_R2C))
                 : zoom->factor > 1 ? ((p->flags & UR_C2C) ? Z_ZOOM_C2C : Z_ZOOM_R2C) : ((p->flags & UR_C2C) ? Z_GEN_C2C : Z_GEN_R2C);
    UR_HIP(launch_pass_z(p->prec, p->n, zm, za, nzb, s));
  }
  p->pass_bytes[P_Z] = live_rows(p, g) * p->nkz * p->cs + 16.0 * nzb;
  const ur_status st = run_y_x(p, g, ws + lay.A, ws + lay.B, lay, h, nzb, s, ws);
  if (st == UR_OK && ws == p->ws && zoom->factor == 1 && zoom->n1 == p->n && !(p->flags & UR_C2C) && !oriented(cell)) {
    p->keep_valid = true;
    p->keep_m = g.m;
    p->keep_c = cell->c;
  }
  return st;
}

extern "C" {

ur_status ur_simulate_noalloc(ur_plan* p, const ur_cell* cell, const ur_mask* mask, const ur_zoom* zoom,
                              const ur_hist* h, void* stream) {
  if (p) p->keep_valid = false;
  if (!p) return fail(UR_ERR_INVALID, "plan is null");
  UR_TRY(need_in_core(p));
  if (p->mixed) return fail(UR_ERR_UNSUPPORTED, "the allocation-free entry runs power-of-two boxes");
  if (p->nbins < 1) return fail(UR_ERR_STATE, "no bins set on the plan");
  UR_TRY(check_hist(h));
  UR_TRY(check_cell(cell));
  FwdGeom g;
  UR_TRY(check_level(p, cell, mask, zoom, g.L, g.m));
  UR_TRY(check_block_transfer(p, zoom));
  ZArgs rot_args{};
  UR_TRY(set_rotation(p, cell, zoom, rot_args));
  const Layout lay = layout_incore(p, p->nbins);
  const size_t cell_off = align256(lay.total);
  const size_t need = cell_off + cell_layout(p, cell, zoom->factor, false).total;
  if (need > kNoAllocScratchBytes)
    return fail(UR_ERR_UNSUPPORTED,
                "this box needs %zu bytes of scratch; the allocation-free entry holds %zu (a %d^3 %s box with %d bins "
                "does not fit; at most a 256^3 FP32 real box)",
                need, kNoAllocScratchBytes, p->n, p->prec == UR_F32 ? "FP32" : "FP64", p->nbins);
  void* base = nullptr;
  UR_HIP(noalloc_scratch(&base));
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  char* ws = (char*)base;
  const bool timing = p->timing;
  p->timing = false;                  // per-pass timing would create event objects
  CellTables t;
  ur_status st = prepare_cell(p, cell, zoom->factor, t, s, ws + cell_off);
  if (st == UR_OK) st = simulate_pow2(p, cell, zoom, h, s, g, rot_args, t, lay, ws);
  p->timing = timing;
  return st;
}

ur_status ur_simulate_rho(ur_plan* p, const void* rho, const ur_hist* h, void* stream) {
  if (p) p->keep_valid = false;
  if (!p || !rho) return fail(UR_ERR_INVALID, "null argument");
  UR_TRY(need_in_core(p));
  if (p->nbins < 1) return fail(UR_ERR_STATE, "no bins set on the plan");
  UR_TRY(check_hist(h));
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  if (p->mixed) {
    if (p->dSinc) return fail(UR_ERR_UNSUPPORTED, "mixed-radix boxes run without the voxel form factor and block-transfer correction");
    Layout lay = layout_mixed(p, p->nbins);
    UR_TRY(ensure_ws(p, lay.total, s));
    UR_TRY(mr_transform(p, rho, p->ws + lay.A, -1, (double*)(p->ws + lay.mom), nullptr, &lay, s));
    return mr_finalize(p, lay, mr_axis_blocks(p->prec, p->n, 0, MR_BIN, !(p->flags & UR_C2C)), h, mr_axis_blocks(p->prec, p->n, 2, MR_LOAD, !(p->flags & UR_C2C)), s);
  }
  Layout lay = layout_incore(p, p->nbins);
  UR_TRY(ensure_ws(p, lay.total, s));
  p->pass_bytes[P_CELL] = 0.0;
  return simulate_rho_pow2(p, rho, h, lay, s);
}

}  // extern "C"

// passes Z (from a given real or complex density), Y, X and the finalize of
// a power-of-two box; the workspace holds at least `lay`
static ur_status simulate_rho_pow2(ur_plan* p, const void* rho, const ur_hist* h, const Layout& lay, hipStream_t s) {
  FwdGeom g{};
  g.xlo = 0; g.xhi = p->n - 1; g.ax0 = 0; g.gen = 0;
  g.L = make_level(p->n, p->n, 1, 1);
  ZArgs za{};
  za.A = p->ws + lay.A; za.ax0 = 0; za.rho = rho; za.rho_x0 = 0; za.tw = p->tw;
  za.mom = (double*)(p->ws + lay.mom); za.L = g.L; za.nkz = p->nkz; za.x0 = 0; za.ntiles = ntiles(p);
  int nzb = p->n * za.ntiles;
  {
    PassTimer tm(p, P_Z, s);
    UR_HIP(launch_pass_z(p->prec, p->n, (p->flags & UR_C2C) ? Z_LOAD_C2C : Z_LOAD_R2C, za, nzb, s));
  }
  p->pass_bytes[P_Z] = (double)p->n * p->n * p->n * ((p->flags & UR_C2C) ? p->cs : p->rs) +
                       (double)p->n * p->nkz * p->n * p->cs + 16.0 * nzb;
  return run_y_x(p, g, p->ws + lay.A, p->ws + lay.B, lay, h, nzb, s, p->ws);
}

extern "C" {

ur_status ur_fft3d_exec(ur_plan* p, const void* in, void* out, int32_t dir, void* stream) {
  if (p) p->keep_valid = false;
  if (!p || !in || !out) return fail(UR_ERR_INVALID, "null argument");
  UR_TRY(need_in_core(p));
  if (dir != -1 && dir != 1) return fail(UR_ERR_INVALID, "dir must be -1 or +1");
  if (dir > 0 && p->n > 1024) return fail(UR_ERR_UNSUPPORTED, "inverse transforms run up to 1024^3");
  if (in == out) return fail(UR_ERR_INVALID, "in and out must differ");
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  if (p->mixed) return mr_transform(p, in, out, dir, nullptr, nullptr, nullptr, s);
  Layout lay = layout_incore(p, std::max(p->nbins, 1));
  UR_TRY(ensure_ws(p, lay.total, s));
  const int n = p->n, c2c = (p->flags & UR_C2C) ? 1 : 0;
  char* A = p->ws + lay.A;
  char* B = p->ws + lay.B;
  const int tx = y_tile(p->prec, n);
  if (dir < 0) {
    ZArgs za{};
    za.A = A; za.ax0 = 0; za.rho = in; za.rho_x0 = 0; za.tw = p->tw; za.mom = nullptr;
    za.L = make_level(n, n, 1, 1); za.nkz = p->nkz; za.x0 = 0; za.ntiles = ntiles(p);
    UR_HIP(launch_pass_z(p->prec, n, c2c ? Z_LOAD_C2C : Z_LOAD_R2C, za, n * za.ntiles, s));
    YArgs ya{};
    ya.A = A; ya.ax0 = 0; ya.B = B; ya.bx0 = 0; ya.bs = n; ya.tw = p->tw; ya.L = za.L; ya.gen = 0;
    ya.nkz = p->nkz; ya.xlo = 0; ya.xhi = n - 1; ya.xt0 = 0; ya.nxt = n / tx; ya.ty = zt(p);
    UR_HIP(launch_pass_y(p->prec, n, ya, s));
    XArgs xa{};
    xa.B = B; xa.bx0 = 0; xa.bs = n; xa.out = out; xa.tw = p->tw; xa.nkz = p->nkz; xa.r2c = !c2c;
    xa.xa = 0; xa.xb = n - 1; xa.oscale = 1.0 / ((double)n * n * n); xa.ncols = p->nkz * n;
    UR_HIP(launch_pass_x(p->prec, n, X_FFT_STORE, -1, xa, x_blocks(p, X_FFT_STORE, -1), s));
  } else {
    XArgs xa{};
    xa.B = in; xa.bx0 = 0; xa.bs = n; xa.out = B; xa.tw = p->tw; xa.nkz = p->nkz; xa.r2c = !c2c;
    xa.xa = 0; xa.xb = n - 1; xa.oscale = 1.0; xa.ncols = p->nkz * n;
    UR_HIP(launch_pass_x(p->prec, n, X_FFT_STORE, +1, xa, x_blocks(p, X_FFT_STORE, +1), s));
    YInvArgs yi{};
    yi.B = B; yi.bx0 = 0; yi.bs = n; yi.A = A; yi.tw = p->tw; yi.nkz = p->nkz; yi.xt0 = 0; yi.nxt = n / tx;
    UR_HIP(launch_pass_y_inv(p->prec, n, yi, s));
    ZInvArgs zi{};
    zi.A = A; zi.out = out; zi.tw = p->tw; zi.nkz = p->nkz; zi.ntiles = n / zinv_tile(p->prec, n, c2c); zi.scale = 1.0;
    UR_HIP(launch_pass_z_inv(p->prec, n, c2c, zi, s));
  }
  return UR_OK;
}

ur_status ur_intensity_bin(ur_plan* p, const void* spectrum, const ur_hist* h, void* stream) {
  if (p) p->keep_valid = false;
  if (!p || !spectrum) return fail(UR_ERR_INVALID, "null argument");
  UR_TRY(need_in_core(p));
  if (p->nbins < 1) return fail(UR_ERR_STATE, "no bins set on the plan");
  UR_TRY(check_hist(h));
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  if (p->mixed) {
    if (p->dSinc) return fail(UR_ERR_UNSUPPORTED, "mixed-radix boxes run without the voxel form factor and block-transfer correction");
    Layout lay = layout_mixed(p, p->nbins);
    UR_TRY(ensure_ws(p, lay.total, s));
    return mr_bin(p, spectrum, lay, h, s);
  }
  Layout lay = layout_incore(p, p->nbins);
  UR_TRY(ensure_ws(p, lay.total, s));
  const int n = p->n;
  XArgs xa{};
  xa.B = spectrum; xa.bx0 = 0; xa.bs = n; xa.tw = p->tw; xa.nkz = p->nkz; xa.r2c = !(p->flags & UR_C2C);
  xa.xa = 0; xa.xb = n - 1; xa.iscale = 1.0; xa.nbins = p->nbins; xa.U = p->dU; xa.lut = p->dLut; xa.nlut = p->nlut;
  xa.sinc = p->dSinc;
  xa.part = (double*)(p->ws + lay.part); xa.f0 = (double*)(p->ws + lay.f0); xa.ncols = p->nkz * n;
  const int nxb = x_blocks(p, X_BIN_ONLY);
  UR_HIP(launch_pass_x(p->prec, n, X_BIN_ONLY, -1, xa, nxb, s));
  FinArgs fa{};
  fa.part = xa.part; fa.nblk = nxb; fa.nbins = p->nbins; fa.mom = nullptr; fa.nzb = 0;
  fa.f0 = xa.f0; fa.cnt = p->dCount; fa.sum = h->sum; fa.sumsq = h->sumsq; fa.count = h->count; fa.totals = h->totals; fa.mean = h->mean; fa.sem = h->sem;
  UR_HIP(launch_finalize(fa, s));
  return UR_OK;
}

}  // extern "C"

// Staging of the out-of-core paths: K slabs of `slab_bytes` on the device
// and, for pageable input, as many page-locked bounce slabs; the copy
// streams and their events
static ur_status ensure_staging(ur_plan* p, size_t slab_bytes, bool pinned) {
  constexpr int K = ur_plan::kStage;
  if (!p->stage || p->stage_bytes < K * slab_bytes) {
    UR_HIP(hipDeviceSynchronize());
    if (p->stage) UR_HIP(hipFree(p->stage));
    p->stage = nullptr;
    if (hipMalloc(&p->stage, K * slab_bytes) != hipSuccess) { (void)hipGetLastError(); return fail(UR_ERR_OOM, "staging allocation failed"); }
    p->stage_bytes = K * slab_bytes;
  }
  if (!pinned && (!p->bounce || p->bounce_bytes < K * slab_bytes)) {
    UR_HIP(hipDeviceSynchronize());
    if (p->bounce) UR_HIP(hipHostFree(p->bounce));
    p->bounce = nullptr;
    if (hipHostMalloc(&p->bounce, K * slab_bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p->bounce = nullptr;
      return fail(UR_ERR_HOST, "pinned bounce allocation failed");
    }
    p->bounce_bytes = K * slab_bytes;
  }
  for (auto& c : p->copy_stream) if (!c) UR_HIP(hipStreamCreateWithFlags(&c, hipStreamNonBlocking));
  for (auto& e : p->ev_copied) if (!e) UR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& e : p->ev_free) if (!e) UR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return UR_OK;
}

// Out-of-core forward path of a real mixed-radix box (eq. 2 with the second
// stage in HBM): slabs of planes [x_lo, x_hi] stream from host memory into
// the staging buffers; each slab is transformed along z (two real pencils
// per complex line, half spectra) and along y right away, into a box that
// holds only the planes of [x_lo, x_hi]; the x pass then takes every (ky,
// kz) line of that box with the other planes read as zero, and bins.
static ur_status simulate_host_mixed(ur_plan* p, const void* rho_host, int x_lo, int x_hi, const ur_hist* h,
                                     hipStream_t s, size_t* h2d_bytes, bool pinned) {
  const int n = p->n;
  const size_t nx = (size_t)(x_hi - x_lo + 1);
  const Layout lay = layout_mixed_ooc(p, p->nbins, nx);
  UR_TRY(ensure_ws(p, lay.total, s));
  const size_t plane_bytes = (size_t)n * n * p->rs;
  const int ts = 8;                                       // planes per slab
  const size_t slab_bytes = (size_t)ts * plane_bytes;
  UR_TRY(ensure_staging(p, slab_bytes, pinned));
  constexpr int K = ur_plan::kStage;
  char* box = p->ws;
  const size_t box_plane = (size_t)n * p->nkz * p->cs;    // bytes of one x plane of the box
  double* mom = (double*)(p->ws + lay.mom);
  const int tl = mr_tile_lines(p->prec, n);
  for (int b = 0; b < K; ++b) {
    UR_HIP(hipEventRecord(p->ev_free[b], s));
    UR_HIP(hipEventRecord(p->ev_copied[b], p->copy_stream[b]));
  }
  size_t copied = 0;
  long long zb = 0;
  long long slab = 0;
  for (long long lo = x_lo; lo <= x_hi; lo += ts, ++slab) {
    const long long hi = std::min<long long>(lo + ts - 1, x_hi);
    const int buf = (int)(slab % K);
    hipStream_t cs = p->copy_stream[buf];
    char* st = (char*)p->stage + buf * slab_bytes;
    const char* src = (const char*)rho_host + (size_t)(lo - x_lo) * plane_bytes;
    const size_t len = (size_t)(hi - lo + 1) * plane_bytes;
    if (!pinned) {
      char* bb = (char*)p->bounce + buf * slab_bytes;
      UR_HIP(hipEventSynchronize(p->ev_copied[buf]));
      parallel_copy(bb, src, len);
      src = bb;
    }
    UR_HIP(hipStreamWaitEvent(cs, p->ev_free[buf], 0));
    UR_HIP(hipMemcpyAsync(st, src, len, hipMemcpyHostToDevice, cs));
    copied += len;
    UR_HIP(hipEventRecord(p->ev_copied[buf], cs));
    UR_HIP(hipStreamWaitEvent(s, p->ev_copied[buf], 0));
    char* dst = box + (size_t)(lo - x_lo) * box_plane;
    MrArgs a{};
    a.tw = p->tw; a.src = st; a.dst = dst; a.scale = 1.0;
    a.lines = (long long)(hi - lo + 1) * n / 2;           // pencil pairs of the slab
    a.mom = mom + 2 * (size_t)zb;
    {
      PassTimer tm(p, P_Z, s);
      UR_HIP(launch_mr_axis(p->prec, n, 2, -1, MR_LOAD, true, a, s));
    }
    zb += (a.lines + tl - 1) / tl;
    UR_HIP(hipEventRecord(p->ev_free[buf], s));
    MrArgs y{};
    y.tw = p->tw; y.src = dst; y.dst = dst; y.scale = 1.0;
    y.planes = (int)(hi - lo + 1);
    {
      PassTimer tm(p, P_Y, s);
      UR_HIP(launch_mr_axis(p->prec, n, 1, -1, MR_LOAD, true, y, s));
    }
  }
  MrArgs x{};
  x.tw = p->tw; x.src = box; x.dst = box; x.xa = x_lo; x.xn = (int)nx;
  x.scale = 1.0 / ((double)n * n * n);
  x.nbins = p->nbins; x.U = p->dU; x.lut = p->dLut; x.iscale = 1.0;
  x.part = (double*)(p->ws + lay.part); x.f0 = (double*)(p->ws + lay.f0);
  {
    PassTimer tm(p, P_X, s);
    UR_HIP(launch_mr_axis(p->prec, n, 0, -1, MR_BIN, true, x, s));
  }
  const double boxb = (double)nx * n * p->nkz * p->cs;
  p->pass_bytes[P_CELL] = 0.0;
  p->pass_bytes[P_Z] = (double)nx * n * n * p->rs + boxb;
  p->pass_bytes[P_Y] = 2.0 * boxb;
  p->pass_bytes[P_X] = boxb;
  if (h2d_bytes) *h2d_bytes = copied;
  return mr_finalize(p, lay, mr_axis_blocks(p->prec, n, 0, MR_BIN, true), h, (int)zb, s);
}

extern "C" {

ur_status ur_simulate_host(ur_plan* p, const void* rho_host, int32_t x_lo, int32_t x_hi, const ur_hist* h,
                           void* stream, size_t* h2d_bytes) {
  if (p) p->keep_valid = false;
  if (!p || !rho_host) return fail(UR_ERR_INVALID, "null argument");
  if (p->nbins < 1) return fail(UR_ERR_STATE, "no bins set on the plan");
  if (p->flags & UR_C2C) return fail(UR_ERR_UNSUPPORTED, "the out-of-core path takes real densities (UR_R2C plans)");
  if (x_lo < 0 || x_hi >= p->n || x_lo > x_hi) return fail(UR_ERR_INVALID, "plane range [%d, %d] outside the box", x_lo, x_hi);
  UR_TRY(check_hist(h));
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
  if (s) (void)hipStreamIsCapturing(s, &cst);
  if (cst != hipStreamCaptureStatusNone) return fail(UR_ERR_STATE, "the out-of-core path is a host-driven pipeline and cannot be captured");
  const HostKind hk = host_kind(rho_host);
  if (hk == HOST_DEVICE) return fail(UR_ERR_INVALID, "rho_host is device memory (ur_simulate_rho takes device densities)");
  if (p->mixed) {
    if (p->dSinc) return fail(UR_ERR_UNSUPPORTED, "mixed-radix boxes run without the voxel form factor and block-transfer correction");
    return simulate_host_mixed(p, rho_host, x_lo, x_hi, h, s, h2d_bytes, hk == HOST_PINNED);
  }
  const int n = p->n, tx = y_tile(p->prec, n);
  OocSplit split;
  UR_TRY(ooc_split(p, p->nbins, x_lo, x_hi, split));
  const Layout lay = split.lay;
  UR_TRY(ensure_ws(p, lay.total, s));
  const size_t plane_bytes = (size_t)n * n * p->rs;
  const size_t slab_bytes = (size_t)tx * plane_bytes;
  constexpr int K = ur_plan::kStage;
  if (!p->stage || p->stage_bytes < K * slab_bytes) {
    UR_HIP(hipDeviceSynchronize());
    if (p->stage) UR_HIP(hipFree(p->stage));
    p->stage = nullptr;
    if (hipMalloc(&p->stage, K * slab_bytes) != hipSuccess) { (void)hipGetLastError(); return fail(UR_ERR_OOM, "staging allocation failed"); }
    p->stage_bytes = K * slab_bytes;
  }
  const bool pinned = hk == HOST_PINNED;
  if (!pinned && (!p->bounce || p->bounce_bytes < K * slab_bytes)) {
    UR_HIP(hipDeviceSynchronize());
    if (p->bounce) UR_HIP(hipHostFree(p->bounce));
    p->bounce = nullptr;
    if (hipHostMalloc(&p->bounce, K * slab_bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p->bounce = nullptr;
      return fail(UR_ERR_HOST, "pinned bounce allocation failed");
    }
    p->bounce_bytes = K * slab_bytes;
  }
  for (auto& c : p->copy_stream) if (!c) UR_HIP(hipStreamCreateWithFlags(&c, hipStreamNonBlocking));
  for (auto& e : p->ev_copied) if (!e) UR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& e : p->ev_free) if (!e) UR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));

  FwdGeom g{};
  g.xlo = x_lo; g.xhi = x_hi; g.gen = 0; g.L = make_level(n, n, 1, 1);
  const long long xt0 = x_lo / tx, xt1 = x_hi / tx;
  const long long bx0 = xt0 * tx, bs = (xt1 - xt0 + 1) * tx;
  char* A = p->ws + lay.A;
  char* B = p->ws + lay.B;
  size_t copied = 0;
  // slab k goes to staging buffer k mod K on copy stream k mod K;
  // ev_copied[b]: buffer b filled, ev_free[b]: buffer b consumed by the z pass
  for (int b = 0; b < K; ++b) {
    UR_HIP(hipEventRecord(p->ev_free[b], s));
    UR_HIP(hipEventRecord(p->ev_copied[b], p->copy_stream[b]));   // after any earlier copy on that stream
  }
  const int ntl = ntiles(p);
  const int nxb = x_blocks(p);
  int zb = 0;
  long long slab = 0;                                     // slabs streamed so far (staging buffer = slab mod K)
  // each pass streams every slab and keeps rows kz0 .. kz0 + nk - 1 of the
  // spectrum; a single pass when the whole x range fits the budget
  for (int chunk = 0; chunk < split.nchunks; ++chunk) {
    const int kz0 = chunk * split.kzc, nk = std::min(split.kzc, p->nkz - kz0);
    for (long long xt = xt0; xt <= xt1; ++xt, ++slab) {
      const int buf = (int)(slab % K);
      hipStream_t cs = p->copy_stream[buf];
      char* st = (char*)p->stage + buf * slab_bytes;
      const long long sx0 = xt * tx;
      const long long lo = std::max<long long>(sx0, x_lo), hi = std::min<long long>(sx0 + tx - 1, x_hi);
      const char* src = (const char*)rho_host + (size_t)(lo - x_lo) * plane_bytes;
      const size_t len = (size_t)(hi - lo + 1) * plane_bytes;
      if (!pinned) {
        // pageable input: once the previous copy out of this bounce slab has
        // finished, the host copies the planes into it (the copies of the
        // slabs before it and the z / y passes keep running meanwhile)
        char* bb = (char*)p->bounce + buf * slab_bytes;
        UR_HIP(hipEventSynchronize(p->ev_copied[buf]));
        parallel_copy(bb, src, len);
        src = bb;
      }
      // wait until the previous user of this staging buffer is done, then copy
      UR_HIP(hipStreamWaitEvent(cs, p->ev_free[buf], 0));
      UR_HIP(hipMemcpyAsync(st + (lo - sx0) * plane_bytes, src, len, hipMemcpyHostToDevice, cs));
      copied += len;
      UR_HIP(hipEventRecord(p->ev_copied[buf], cs));
      UR_HIP(hipStreamWaitEvent(s, p->ev_copied[buf], 0));
      // z pass over the planes of this slab (its rho^2 sums taken in the
      // first pass only), then y pass of this x tile for the pass's kz rows
      ZArgs za{};
      za.A = A; za.ax0 = sx0; za.rho = st; za.rho_x0 = sx0; za.tw = p->tw;
      za.mom = chunk == 0 ? (double*)(p->ws + lay.mom) + 2 * (size_t)zb : nullptr;
      za.L = g.L; za.nkz = p->nkz; za.x0 = (int)lo; za.ntiles = ntl;
      const int nb = (int)((hi - lo + 1) * ntl);
      UR_HIP(launch_pass_z(p->prec, n, Z_LOAD_R2C, za, nb, s));
      if (chunk == 0) zb += nb;
      UR_HIP(hipEventRecord(p->ev_free[buf], s));
      YArgs ya{};
      ya.A = A; ya.ax0 = sx0; ya.B = B; ya.bx0 = bx0; ya.bs = bs; ya.tw = p->tw; ya.L = g.L; ya.gen = 0;
      ya.nkz = p->nkz; ya.xlo = (int)lo; ya.xhi = (int)hi; ya.xt0 = (int)xt; ya.nxt = 1; ya.ty = zt(p);
      ya.kz0 = kz0; ya.nkzc = nk;
      UR_HIP(launch_pass_y(p->prec, n, ya, s));
    }
    // x pass over this pass's rows of the spectrum, added to the block partials
    // of the earlier passes (a fixed order: chunk after chunk)
    XArgs xa{};
    xa.B = B; xa.bx0 = bx0; xa.bs = bs; xa.tw = p->tw; xa.nkz = p->nkz; xa.r2c = 1;
    xa.xa = (int)bx0; xa.xb = (int)(bx0 + bs - 1);
    xa.iscale = 1.0 / ((double)n * n * n) / ((double)n * n * n);
    xa.nbins = p->nbins; xa.U = p->dU; xa.lut = p->dLut; xa.nlut = p->nlut; xa.sinc = p->dSinc;
    xa.part = (double*)(p->ws + lay.part); xa.f0 = (double*)(p->ws + lay.f0);
    xa.ncols = nk * n; xa.kz0 = kz0; xa.accum = chunk > 0;
    UR_HIP(launch_pass_x(p->prec, n, X_FFT_BIN, -1, xa, nxb, s));
  }
  if (h2d_bytes) *h2d_bytes = copied;
  FinArgs fa{};
  fa.part = (const double*)(p->ws + lay.part); fa.nblk = nxb; fa.nbins = p->nbins;
  fa.mom = (const double*)(p->ws + lay.mom); fa.nzb = zb;
  fa.mpart = (double*)(p->ws + lay.f0 + 64); fa.f0 = (const double*)(p->ws + lay.f0); fa.cnt = p->dCount;
  fa.sum = h->sum; fa.sumsq = h->sumsq; fa.count = h->count; fa.totals = h->totals; fa.mean = h->mean; fa.sem = h->sem;
  UR_HIP(launch_finalize(fa, s));
  return UR_OK;
}

// The adjoint from the plan's state: with `reuse`, the y-pass output left by
// the preceding ur_simulate (same density) stands in for the recomputed
// z and y passes.
static ur_status adjoint_run(ur_plan* p, const void* rho, const ur_cell* cell, const ur_mask* mask, const ur_hist* fwd,
                             const double* g_bin, void* grad_rho, double* grad_amp, void* stream, bool reuse);

ur_status ur_host_alloc(size_t bytes, void** out) {
  if (!out) return fail(UR_ERR_INVALID, "out is null");
  *out = nullptr;
  if (bytes == 0) return fail(UR_ERR_INVALID, "bytes must be > 0");
  if (hipHostMalloc(out, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(UR_ERR_HOST, "pinned host allocation of %zu bytes failed", bytes);
  }
  return UR_OK;
}

ur_status ur_host_free(void* ptr) {
  if (!ptr) return UR_OK;
  UR_HIP(hipHostFree(ptr));
  return UR_OK;
}

ur_status ur_adjoint(ur_plan* p, const void* rho, const ur_cell* cell, const ur_mask* mask, const ur_hist* fwd,
                     const double* g_bin, void* grad_rho, double* grad_amp, void* stream) {
  if (p) p->keep_valid = false;
  return adjoint_run(p, rho, cell, mask, fwd, g_bin, grad_rho, grad_amp, stream, false);
}

ur_status ur_adjoint_reuse(ur_plan* p, const ur_cell* cell, const ur_mask* mask, const ur_hist* fwd,
                           const double* g_bin, double* grad_amp, void* stream) {
  if (!p || !cell || !mask || !fwd || !g_bin || !grad_amp) return fail(UR_ERR_INVALID, "null argument");
  const bool held = p->keep_valid;
  p->keep_valid = false;                               // the x pass below overwrites the held output
  if (!held) return fail(UR_ERR_STATE, "no forward output held: the last call on this plan was not ur_simulate");
  MaskP m{};
  m.kind = mask->kind; m.p0 = mask->p0; m.p1 = mask->p1;
  if (m.kind != p->keep_m.kind || m.p0 != p->keep_m.p0 || m.p1 != p->keep_m.p1 || cell->c != p->keep_c)
    return fail(UR_ERR_STATE, "mask or cell edge differ from those of the held forward output");
  return adjoint_run(p, nullptr, cell, mask, fwd, g_bin, nullptr, grad_amp, stream, true);
}

static ur_status adjoint_run(ur_plan* p, const void* rho, const ur_cell* cell, const ur_mask* mask, const ur_hist* fwd,
                             const double* g_bin, void* grad_rho, double* grad_amp, void* stream, bool reuse) {
  if (!p || !fwd || !fwd->count || !g_bin) return fail(UR_ERR_INVALID, "null argument");
  if (p->nbins < 1) return fail(UR_ERR_STATE, "no bins set on the plan");
  if ((rho != nullptr) == (cell != nullptr)) return fail(UR_ERR_INVALID, "give exactly one of rho and cell");
  if (grad_amp && !cell) return fail(UR_ERR_INVALID, "grad_amp needs the cell description");
  const bool orient = cell && oriented(cell);
  if (orient && reuse) return fail(UR_ERR_UNSUPPORTED, "the held forward output is of a lattice aligned with the box");
  if (orient && grad_amp && cell->c > 16)
    return fail(UR_ERR_UNSUPPORTED, "amplitude gradients of rotated lattices and grains take cell edges up to 16");
  if (p->bt_f > 1) return fail(UR_ERR_UNSUPPORTED, "the adjoint runs without the block-transfer correction");
  if (p->mixed) return fail(UR_ERR_UNSUPPORTED, "the adjoint runs on power-of-two boxes");
  if (!grad_rho && !grad_amp) return UR_OK;
  if (p->n > 1024) return fail(UR_ERR_UNSUPPORTED, "the adjoint runs up to 1024^3");
  hipStream_t s = (hipStream_t)stream;
  note_stream(p, s);
  Layout lay = layout_incore(p, p->nbins);
  UR_TRY(ensure_ws(p, lay.total, s));
  const int n = p->n, c2c = (p->flags & UR_C2C) ? 1 : 0, tx = y_tile(p->prec, n);
  char* A = p->ws + lay.A;
  char* B = p->ws + lay.B;
  FwdGeom g{};
  CellTables t{};
  ZArgs za{};
  int zmode;
  if (cell) {
    UR_TRY(check_cell(cell));
    ur_zoom z1{n, 1};
    UR_TRY(check_level(p, cell, mask, &z1, g.L, g.m));
    UR_TRY(set_rotation(p, cell, &z1, za));
    UR_TRY(prepare_cell(p, cell, 1, t, s));
    long long xlo, xhi;
    plane_range(g.L, g.m, xlo, xhi);
    if (xlo < 0) xlo = 0;
    if (xhi > n - 1) xhi = n - 1;
    g.xlo = (int)xlo; g.xhi = (int)xhi; g.gen = 1;
    za.cellT = t.cellT; za.cb = t.cb; za.pre = t.pre; za.cbn = t.cbn;
    zmode = orient ? (za.cubic ? (za.ngrain ? Z_ROT3G_R2C : Z_ROT3_R2C) : (za.ngrain ? Z_ROTG_R2C : Z_ROT_R2C))
                   : c2c ? Z_GEN_C2C : Z_GEN_R2C;
  } else {
    g.xlo = 0; g.xhi = n - 1; g.gen = 0; g.L = make_level(n, n, 1, 1);
    za.rho = rho; za.rho_x0 = 0;
    zmode = c2c ? Z_LOAD_C2C : Z_LOAD_R2C;
  }
  g.ax0 = 0;
  // Only the amplitude gradient wanted: every inverse pass is pruned to the
  // particle exactly like the forward ones, and the inverse z pass folds
  // straight onto the cell (the n^3 gradient box is never written).
  const bool amp_fold = cell && grad_amp && !grad_rho && !c2c;
  const bool amp_only = amp_fold && !orient;        // fused inverse z pass + fold
  long long bx0 = 0, bs = n, xt0 = 0, xt1 = n / tx - 1;
  if (amp_fold && g.xlo <= g.xhi) {
    xt0 = g.xlo / tx;
    xt1 = g.xhi / tx;
    bx0 = xt0 * tx;
    bs = (xt1 - xt0 + 1) * tx;
  }
  // forward transform along z and y: recomputed, or held from the forward call
  if (!reuse && g.xlo <= g.xhi) {
    za.A = A; za.ax0 = 0; za.tw = p->tw; za.mom = nullptr; za.L = g.L; za.m = g.m; za.nkz = p->nkz;
    za.x0 = g.xlo; za.ntiles = ntiles(p);
    UR_HIP(launch_pass_z(p->prec, n, zmode, za, (g.xhi - g.xlo + 1) * za.ntiles, s));
    YArgs ya{};
    ya.A = A; ya.ax0 = 0; ya.B = B; ya.bx0 = bx0; ya.bs = bs; ya.tw = p->tw; ya.L = g.L; ya.m = g.m; ya.gen = g.gen;
    ya.nkz = p->nkz; ya.xlo = g.xlo; ya.xhi = g.xhi; ya.xt0 = g.xlo / tx; ya.nxt = g.xhi / tx - g.xlo / tx + 1; ya.ty = zt(p);
    UR_HIP(launch_pass_y(p->prec, n, ya, s));
  }
  // x: transform, weight by G(|q|) 2/n^6, inverse transform
  XAdjArgs xj{};
  xj.B = B; xj.bx0 = bx0; xj.bs = bs; xj.tw = p->tw; xj.nkz = p->nkz; xj.r2c = !c2c;
  const long long fx0 = (long long)(g.xlo / tx) * tx;
  xj.xa = (int)fx0; xj.xb = g.xlo <= g.xhi ? (int)((g.xhi / tx) * tx + tx - 1) : -1;
  xj.oa = amp_fold ? (int)bx0 : 0;
  xj.ob = amp_fold ? (int)(bx0 + bs - 1) : n - 1;
  xj.nbins = p->nbins; xj.U = p->dU; xj.lut = p->dLut; xj.nlut = p->nlut; xj.g_bin = g_bin; xj.count = fwd->count;
  xj.gscale = 2.0 / ((double)n * n * n) / ((double)n * n * n); xj.ncols = p->nkz * n; xj.sinc = p->dSinc;
  UR_HIP(launch_pass_x_adj(p->prec, n, xj, x_blocks(p, X_ADJ), s));
  YInvArgs yi{};
  yi.B = B; yi.bx0 = bx0; yi.bs = bs; yi.A = A; yi.tw = p->tw; yi.nkz = p->nkz;
  yi.xt0 = (int)xt0; yi.nxt = (int)(xt1 - xt0 + 1);
  if (amp_fold) {          // the fold reads only the particle's row tiles
    yi.rows = 1; yi.ty = zinv_tile(p->prec, n, 0); yi.L = g.L; yi.m = g.m;
  }
  if (!amp_fold || g.xlo <= g.xhi) UR_HIP(launch_pass_y_inv(p->prec, n, yi, s));
  const int c = cell ? cell->c : 1, c3 = c * c * c;
  if (amp_only) {
    if (c > 16) UR_HIP(launch_zero(t.gcell, (size_t)c3 * 8, s));
    if (g.xlo <= g.xhi) {
      ZFoldArgs zf{};
      zf.A = A; zf.tw = p->tw; zf.L = g.L; zf.m = g.m; zf.nkz = p->nkz; zf.xlo = g.xlo; zf.xhi = g.xhi;
      zf.ntiles = n / zinv_tile(p->prec, n, 0); zf.scale = 1.0; zf.part = t.fold_part; zf.gcell = t.gcell;
      UR_HIP(launch_pass_z_fold(p->prec, n, zf, kFoldBlocks, s));
      if (c <= 16) UR_HIP(launch_fold_reduce_classes(c, t.fold_part, kFoldBlocks, t.gcell, s));
    } else if (c <= 16) {
      UR_HIP(launch_zero(t.gcell, (size_t)c3 * 8, s));
    }
    UR_HIP(launch_grad_amp(c, cell->n_atoms, t.prof, t.gcell, grad_amp, s));
    return UR_OK;
  }
  // the inverse z pass writes grad_rho, or the free B buffer when only grad_amp is wanted
  void* gr = grad_rho ? grad_rho : (void*)B;
  ZInvArgs zi{};
  zi.A = A; zi.out = gr; zi.tw = p->tw; zi.nkz = p->nkz; zi.ntiles = n / zinv_tile(p->prec, n, c2c); zi.scale = 1.0;
  if (amp_fold) {          // oriented lattices: only the particle's pencils, for the fold
    zi.x0 = g.xlo; zi.nx = g.xhi - g.xlo + 1; zi.prune = 1; zi.L = g.L; zi.m = g.m;
  }
  if (!amp_fold || g.xlo <= g.xhi) UR_HIP(launch_pass_z_inv(p->prec, n, c2c, zi, s));
  if (grad_amp) {
    if (c2c) return fail(UR_ERR_UNSUPPORTED, "amplitude gradients need an UR_R2C plan");
    FoldArgs fo{};
    fo.g = gr; fo.L = g.L; fo.m = g.m; fo.gcell = t.gcell; fo.part = t.fold_part; fo.npencils = n * n;
    if (orient) {
      // the sampler's adjoint onto the cell (or its spline coefficients,
      // then through the spline solve, a symmetric linear map)
      ZArgs zr = za;
      zr.L = g.L; zr.m = g.m;
      UR_HIP(launch_fold_rot(p->prec, n, zr, gr, t.fold_part, kFoldBlocks, s));
      UR_HIP(launch_fold_reduce(c3, t.fold_part, kFoldBlocks, t.gcell, s));
      if (za.cubic) UR_HIP(launch_bspline_cell(c, t.gcell, s));
    } else if (c <= 16) {
      UR_HIP(launch_fold(p->prec, n, fo, kFoldBlocks, s));
      UR_HIP(launch_fold_reduce(c3, t.fold_part, kFoldBlocks, t.gcell, s));
    } else {
      UR_HIP(launch_zero(t.gcell, (size_t)c3 * 8, s));
      UR_HIP(launch_fold(p->prec, n, fo, kFoldBlocks, s));
    }
    UR_HIP(launch_grad_amp(c, cell->n_atoms, t.prof, t.gcell, grad_amp, s));
  }
  return UR_OK;
}

ur_status ur_ewald_image(ur_plan* p, const void* spectrum, const ur_ewald* geo, double* image, void* stream) {
  if (!p || !spectrum || !geo || !image) return fail(UR_ERR_INVALID, "null argument");
  UR_TRY(need_in_core(p));
  if (!(geo->wavelength > 0.0) || !isfinite(geo->wavelength)) return fail(UR_ERR_INVALID, "wavelength must be positive");
  if (!(geo->rel_spread >= 0.0) || !isfinite(geo->rel_spread) || geo->rel_spread >= 0.3)
    return fail(UR_ERR_INVALID, "rel_spread must be in [0, 0.3)");
  if (geo->n_lambda < 1 || geo->n_lambda > 64) return fail(UR_ERR_INVALID, "n_lambda = %d outside [1, 64]", geo->n_lambda);
  if (!(geo->distance > 0.0) || !(geo->pixel > 0.0) || !isfinite(geo->distance) || !isfinite(geo->pixel))
    return fail(UR_ERR_INVALID, "distance and pixel must be positive");
  if (geo->nu < 1 || geo->nv < 1 || (long long)geo->nu * geo->nv > (1ll << 28))
    return fail(UR_ERR_INVALID, "detector of %d x %d pixels", geo->nu, geo->nv);
  if (!isfinite(geo->cu) || !isfinite(geo->cv)) return fail(UR_ERR_INVALID, "beam centre must be finite");
  auto dot = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  const double* vs[3] = {geo->beam, geo->du, geo->dv};
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j)
      if (fabs(dot(vs[i], vs[j]) - (i == j ? 1.0 : 0.0)) > 1e-9)
        return fail(UR_ERR_INVALID, "beam, du and dv must be orthonormal");
  EwaldArgs a{};
  a.spec = spectrum; a.n = p->n; a.nkz = p->nkz; a.c2c = (p->flags & UR_C2C) ? 1 : 0; a.natural = p->mixed ? 1 : 0;
  a.dq = 2.0 * M_PI / ((double)p->n * p->voxel);
  for (int i = 0; i < 3; ++i) { a.e[i] = geo->beam[i]; a.du[i] = geo->du[i]; a.dv[i] = geo->dv[i]; }
  a.dist = geo->distance; a.pixel = geo->pixel; a.cu = geo->cu; a.cv = geo->cv;
  a.nu = geo->nu; a.nv = geo->nv; a.nl = geo->rel_spread > 0.0 ? geo->n_lambda : 1;
  // wavelength nodes lambda (1 + sigma t_j), t_j evenly spaced on [-3, 3],
  // weights exp(-t_j^2 / 2) normalised
  double wsum = 0.0;
  for (int j = 0; j < a.nl; ++j) {
    const double t = a.nl == 1 ? 0.0 : -3.0 + 6.0 * j / (a.nl - 1);
    a.k[j] = 2.0 * M_PI / (geo->wavelength * (1.0 + geo->rel_spread * t));
    a.w[j] = exp(-0.5 * t * t);
    wsum += a.w[j];
  }
  for (int j = 0; j < a.nl; ++j) a.w[j] /= wsum;
  a.image = image;
  UR_HIP(launch_ewald(p->prec, a, (hipStream_t)stream));
  return UR_OK;
}

ur_status ur_peak_integrals(int32_t nbins, const double* edges, const double* mean, int32_t nwin,
                            const double* windows, double* out, void* stream) {
  if (!edges || !mean || !windows || !out) return fail(UR_ERR_INVALID, "null argument");
  if (nbins < 1 || nbins > 4096) return fail(UR_ERR_INVALID, "nbins = %d outside [1, 4096]", nbins);
  if (nwin < 1 || nwin > kMaxWindows) return fail(UR_ERR_INVALID, "nwin = %d outside [1, %d]", nwin, kMaxWindows);
  PeakArgs a{};
  a.nbins = nbins; a.nwin = nwin; a.edges = edges; a.mean = mean; a.out = out;
  for (int w = 0; w < nwin; ++w) {
    const double lo = windows[2 * w], hi = windows[2 * w + 1];
    if (!isfinite(lo) || !isfinite(hi) || !(lo < hi)) return fail(UR_ERR_INVALID, "window %d must have finite q_lo < q_hi", w);
    a.lo[w] = lo;
    a.hi[w] = hi;
  }
  UR_HIP(launch_peaks(a, (hipStream_t)stream));
  return UR_OK;
}

ur_status ur_chi2(int32_t nbins, const double* mean, const double* count, const double* target, double rel_sigma,
                  double* out_chi2, double* g_bin, void* stream) {
  if (nbins < 1 || nbins > 4096) return fail(UR_ERR_INVALID, "nbins = %d outside [1, 4096]", nbins);
  if (!mean || !count || !target || !out_chi2) return fail(UR_ERR_INVALID, "null argument");
  if (!(rel_sigma > 0.0) || !isfinite(rel_sigma)) return fail(UR_ERR_INVALID, "rel_sigma must be positive and finite");
  UR_HIP(launch_chi2(nbins, mean, count, target, rel_sigma, out_chi2, g_bin, (hipStream_t)stream));
  return UR_OK;
}

ur_status ur_ensemble(int32_t nboxes, int32_t nbins, const double* mean, const double* sem, const double* weights,
                      double* out_mean, double* out_sem, void* stream) {
  if (nboxes < 1) return fail(UR_ERR_INVALID, "nboxes = %d must be >= 1", nboxes);
  if (nbins < 1 || nbins > 4096) return fail(UR_ERR_INVALID, "nbins = %d outside [1, 4096]", nbins);
  if (!mean || !sem || !weights || !out_mean || !out_sem) return fail(UR_ERR_INVALID, "null argument");
  UR_HIP(launch_ensemble(nboxes, nbins, mean, sem, weights, out_mean, out_sem, (hipStream_t)stream));
  return UR_OK;
}

ur_status ur_merge_zooms(int32_t nlevels, const ur_hist* levels, const int32_t* n, const double* voxel, int32_t nbins,
                         const double* edges, int32_t mode, double n_min, double* mean, double* sem, int32_t* owner,
                         void* stream) {
  if (nlevels < 1 || nlevels > 8) return fail(UR_ERR_INVALID, "nlevels = %d outside [1, 8]", nlevels);
  if (!levels || !n || !voxel || !edges || !mean || !sem || !owner) return fail(UR_ERR_INVALID, "null argument");
  if (nbins < 1) return fail(UR_ERR_INVALID, "nbins must be >= 1");
  if (mode < 0 || mode > 2) return fail(UR_ERR_INVALID, "unknown merge mode %d", mode);
  MergeArgs a{};
  a.nlevels = nlevels;
  int ord[8];                                          // nlevels <= 8 (checked above)
  for (int k = 0; k < nlevels; ++k) {
    if (!levels[k].sum || !levels[k].sumsq || !levels[k].count) return fail(UR_ERR_INVALID, "level %d histogram is null", k);
    if (n[k] < 1 || !(voxel[k] > 0.0)) return fail(UR_ERR_INVALID, "level %d geometry invalid", k);
    a.sum[k] = levels[k].sum;
    a.sumsq[k] = levels[k].sumsq;
    a.count[k] = levels[k].count;
    double n3 = (double)n[k] * n[k] * n[k];
    a.scale[k] = n3 * n3;
    a.dq[k] = 2.0 * M_PI / ((double)n[k] * voxel[k]);
    a.qcut[k] = sqrt(3.0) * M_PI / (2.0 * voxel[k]);
    ord[k] = k;
  }
  std::stable_sort(ord, ord + nlevels, [&](int x, int y) { return voxel[x] < voxel[y]; });
  for (int k = 0; k < nlevels; ++k) a.order[k] = ord[k];
  a.mode = mode; a.n_min = n_min; a.nbins = nbins; a.edges = edges; a.mean = mean; a.sem = sem; a.owner = owner;
  UR_HIP(launch_merge(a, (hipStream_t)stream));
  return UR_OK;
}

ur_status ur_graph_begin(void* stream) {
  if (!stream) return fail(UR_ERR_INVALID, "capture needs a non-null stream");
  if (tl_capturing) return fail(UR_ERR_STATE, "a capture started by ur_graph_begin is already open on this thread");
  UR_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
  tl_capturing = true;
  tl_captured.clear();
  return UR_OK;
}

ur_status ur_graph_end(void* stream, void** graph_exec) {
  if (!stream || !graph_exec) return fail(UR_ERR_INVALID, "null argument");
  std::vector<ur_plan*> used;
  used.swap(tl_captured);
  tl_capturing = false;
  hipGraph_t g = nullptr;
  UR_HIP(hipStreamEndCapture((hipStream_t)stream, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(UR_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  try {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    g_graph_plans[(void*)ex] = used;
    for (ur_plan* p : used) p->graphs += 1;
  } catch (...) {
    for (ur_plan* p : used) p->graph_external = true;          // untracked: bound for good
  }
  *graph_exec = (void*)ex;
  return UR_OK;
}

ur_status ur_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return fail(UR_ERR_INVALID, "null graph");
  UR_HIP(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
  return UR_OK;
}

ur_status ur_graph_destroy(void* graph_exec) {
  if (!graph_exec) return UR_OK;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graph_plans.find(graph_exec);
    if (it != g_graph_plans.end()) {
      for (ur_plan* p : it->second) p->graphs -= 1;
      g_graph_plans.erase(it);
    }
  }
  UR_HIP(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
  return UR_OK;
}

}  // extern "C"
