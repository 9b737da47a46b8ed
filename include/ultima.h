/*
 * ultima.h -- C ABI of the MI355X (gfx950) wide-range scattering simulator.
 *
 * The library computes, on one GPU, the hot path of the "Ultima Ratio"
 * method (Pauw et al., arXiv 2303.13435):
 *
 *   1. electron density (ED) of a particle: a unit-cell density tiled over a
 *      box and multiplied by a particle mask (Methodology, general workflow
 *      steps 1-2, "Electron density generation"), optionally block-summed
 *      into a zoomed-out level ED-2/ED-3 (step 3);
 *   2. its 3D Fourier transform, eq. 1, evaluated as 1D transforms along z,
 *      y and x (the separation of eq. 2);
 *   3. the intensity |F|^2 averaged into |Q| bins (step 5, "Q-calculation and
 *      spherical averaging");
 *   4. the merge of several zoom levels into one curve (step 6);
 *   5. the adjoint of 1-3: gradients of a loss on the binned curve with
 *      respect to voxel densities and atom amplitudes (derived from eq. 1).
 *
 * General conventions
 *   - Every call returns ur_status (UR_OK = 0).  On failure nothing has been
 *     enqueued, and ur_last_error() describes the problem (thread-local text,
 *     valid until the next call on the same thread).  No C++ exception and no
 *     abort crosses this boundary.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it asynchronously; outputs are valid after
 *     the stream is synchronised.  A plan must not run on two streams at once.
 *   - Pointers documented as DEVICE point to memory of the current HIP
 *     device, owned by the caller; HOST pointers are read during the call
 *     only (the out-of-core density: until the stream is synchronised).
 *     The library never frees caller memory.
 *   - Box layout: real densities are [x][y][z] row-major, z fastest, edge n
 *     (a power of two, 16 <= n <= 2048; FP32 real boxes of n = 4096 through
 *     the out-of-core path only; complex transforms, inverse transforms and
 *     the adjoint: n <= 1024).  The particle and the lattice are
 *     centred on voxel (n1/2, n1/2, n1/2) of the ED-1 grid.
 *   - Spectra exchanged through ur_fft3d_exec / ur_intensity_bin use the
 *     transposed layout [kz][ky][kx] (kx fastest, complex interleaved), with
 *     kz in [0, n/2] for real transforms and [0, n) for complex ones.  This is
 *     the order in which the last transform pass produces them.
 *   - Frequencies: u in [0, n) stands for the signed index h = u (u < n/2) or
 *     u - n; |Q| = dq * sqrt(h^2 + k^2 + l^2) with dq = 2 pi / (n voxel).
 */
#ifndef ULTIMA_H
#define ULTIMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  UR_OK = 0,
  UR_ERR_INVALID = 1,      /* bad argument (null pointer, size, range)        */
  UR_ERR_UNSUPPORTED = 2,  /* valid request the library does not implement  */
  UR_ERR_OOM = 3,          /* device allocation failed                        */
  UR_ERR_HIP = 4,          /* a HIP runtime call failed                       */
  UR_ERR_HOST = 5,         /* host memory (pageable or page-locked) unavailable */
  UR_ERR_STATE = 6         /* call out of order (e.g. no bins set on the plan) */
} ur_status;

typedef enum { UR_F32 = 0, UR_F64 = 1 } ur_prec;

/* plan flags */
#define UR_R2C 0u         /* real input, half spectrum (default)              */
#define UR_C2C 1u         /* full complex transform of a real or complex box  */

/* mask kinds (integer parameters make the inside test exact):
 *   UR_MASK_SPHERE     d.d <= p0
 *   UR_MASK_CUBE       max|d_i| <= p0
 *   UR_MASK_TRUNC_OCT  max|d_i| <= p0 and |d_x|+|d_y|+|d_z| <= p1
 * with d the voxel offset from the particle centre.  p0 < 0 gives an empty
 * particle.  (Methodology, "Electron density generation": the per-plane
 * circular mask that builds up a spherical particle.) */
#define UR_MASK_NONE 0
#define UR_MASK_SPHERE 1
#define UR_MASK_CUBE 2
#define UR_MASK_TRUNC_OCT 3

typedef struct { int32_t kind; int64_t p0; int64_t p1; } ur_mask;

/* Unit cell ("ED-Unit", workflow step 1).  Edge c voxels (power of two
 * dividing n1/2; any edge up to 256, such as the paper's reduced 105^3
 * cell, for ur_cell_synth and for ur_simulate on mixed-radix plans, whose
 * generator wraps the cell index by a modulo); n_atoms Gaussian atoms.  DEVICE arrays, FP64:
 * xyz[3*n_atoms] centres in cell-voxel units, amp[n_atoms] electrons per atom,
 * sigma[n_atoms] widths in voxels.  Each voxel holds the Gaussian integrated
 * over it, with periodic images, plus `background`.
 * rot: NULL for the lattice aligned with the box, or HOST 9 doubles R
 * (row-major, finite) orienting it ("Electron density generation": the
 * cell interpolated over a rotated grid, repeated outside its bounds): the
 * ED-1 voxel at offset d = (x, y, z) - n1/2 from the particle centre takes
 * the cell's value at u = R d, interpolated between the cell voxels with
 * periodic wrap (R = identity gives the aligned lattice exactly).
 * interp selects the interpolation: 0 or 1 trilinear; 3 the cubic B-spline
 * through the cell values (periodic spline coefficients, then the sum over
 * the 4 x 4 x 4 neighbouring coefficients with the cubic B-spline weights
 * of the fractional offsets: the order-3 spline of the interpolation
 * routine the paper names); other values fail with UR_ERR_INVALID.
 * n_grains (0 .. 16) > 0 makes a polycrystalline particle (the rotated
 * grid serves to build crystallites of random orientations; the outlook
 * names polycrystalline grains): HOST grain_seed[3*n_grains] integer voxel
 * offsets from the particle centre and grain_rot[9*n_grains] orientations
 * (row-major, finite); the inside voxel at offset d belongs to the grain
 * whose seed is nearest (squared integer distance, ties to the lower grain
 * index) and takes the cell at u = R_g d, sampled as chosen by interp; rot
 * must then be NULL.  Seeds that are not integers or exceed 8192 in
 * magnitude fail with UR_ERR_INVALID.
 * Rotated lattices and grains run the forward paths at zoom factor 1 on
 * real (UR_R2C) plans; the adjoint refuses them (UR_ERR_UNSUPPORTED). */
typedef struct {
  int32_t c;
  int32_t n_atoms;
  const double* xyz;
  const double* amp;
  const double* sigma;
  double background;
  const double* rot;
  int32_t interp;
  int32_t n_grains;
  const double* grain_seed;
  const double* grain_rot;
} ur_cell;

/* Zoom level (workflow step 3): the ED-1 grid of edge n1 is block-summed by
 * `factor` per axis and centred in this plan's box (offset
 * (n - n1/factor)/2).  factor = 1 and n1 = n is ED-1 itself. */
typedef struct { int32_t n1; int32_t factor; } ur_zoom;

/* Per-bin statistics, DEVICE arrays of nbins doubles each, written by the
 * library: sum of w*I, sum of w*I^2 and sum of w over the voxels of the bin
 * (w counts a voxel of the half spectrum twice when it stands for its
 * conjugate partner too, so every statistic is that of the full n^3 box).
 * totals (DEVICE, 4 doubles): [0] sum of I over every voxel (binned or not),
 * [1] Re F(0), [2] Im F(0), [3] sum of rho^2 over the box (0 when the density
 * was not generated or loaded by the call).  I = |F|^2 with F of eq. 1.
 * mean, sem (DEVICE, nbins each, or NULL to skip): the per-bin mean sum/count
 * and standard error of the mean sqrt((sumsq - sum^2/count)/(count-1)/count)
 * of I (section "Q-calculation and spherical averaging"); NaN for an empty
 * bin, and SEM NaN for a bin of one voxel. */
typedef struct { double* sum; double* sumsq; double* count; double* totals; double* mean; double* sem; } ur_hist;

typedef struct ur_plan ur_plan;

/* Create a plan for an n^3 box of voxel edge `voxel` (nm, > 0) in precision
 * `prec`.  flags: UR_R2C or UR_C2C.  Allocates the plan's device tables
 * (twiddles) with hipMalloc; the large work buffers are either attached with
 * ur_plan_set_workspace or allocated lazily on first use.  Errors:
 * UR_ERR_INVALID for n neither a power of two nor a mixed-radix edge (below), a voxel that is not positive and
 * finite, or an unknown precision; UR_ERR_UNSUPPORTED for n above 4096, for
 * n above 2048 in FP64 or complex, or for a complex (UR_C2C) power-of-two
 * plan above 1024.  A plan above 2048 (4096, or the mixed-radix 4000) runs
 * only ur_plan_set_bins, ur_rho_generate, ur_cell_synth and the out-of-core
 * path (ur_simulate_host and its workspace query); its other calls fail
 * with UR_ERR_UNSUPPORTED.
 * Mixed-radix edges (boxes of the paper's 4000 family, Methodology,
 * "Electron density generation"): n = 40, 80, 100, 160, 200, 250, 400, 500,
 * 1000, 2000, 4000, 48, 96, 384, 768 or 1536 make a plan whose transform
 * runs one axis at a time, in place, through radix 2/4/8/16, 3 and 5
 * stages; its spectrum (ur_fft3d_exec, and the input of ur_intensity_bin
 * and ur_ewald_image) is in natural order [kx][ky][kz], kz in [0, n/2] on a
 * real plan (two real z pencils per complex line, unpacked into their half
 * spectra; forward transform only) and in [0, n) on a complex one.  Such
 * plans run ED-1 levels (zoom n1 = n, factor 1, any cell edge up to 256)
 * and zoom levels (any factor dividing an even n1, such as the paper's 125;
 * power-of-two cells) through ur_simulate, ur_simulate_rho (a real density
 * on real plans, complex on complex ones), ur_simulate_host (real plans),
 * ur_rho_generate, ur_fft3d_exec, ur_intensity_bin and ur_ewald_image; the
 * adjoint, oriented lattices, the voxel form factor and the block-transfer
 * correction fail with UR_ERR_UNSUPPORTED.  Other edges that are not powers
 * of two fail with UR_ERR_INVALID. */
ur_status ur_plan_create(int32_t n, double voxel, int32_t prec, uint32_t flags, ur_plan** out);
void ur_plan_destroy(ur_plan* plan);

/* Bytes of device workspace the plan needs for `nbins` bins (transform
 * buffers, partial histograms, cell tables) on the in-HBM paths. */
ur_status ur_plan_workspace_size(const ur_plan* plan, int32_t nbins, size_t* bytes);
/* Attach caller-owned device workspace (>= the size above, 256-B aligned). */
ur_status ur_plan_set_workspace(ur_plan* plan, void* dev_ptr, size_t bytes);

/* Set the |Q| bins: nbins >= 1 strictly increasing edges (HOST, nm^-1).  The
 * edges become integer thresholds on n2 = h^2+k^2+l^2: t = (e/dq)^2 snapped
 * to the nearest integer within 1e-9 relative; bin b holds
 * ceil(t_b) <= n2 < ceil(t_b+1); the last upper edge is inclusive.  Copies a
 * small table to the device synchronously; call before capture. */
ur_status ur_plan_set_bins(ur_plan* plan, int32_t nbins, const double* edges);

/* Unit-cell density: writes the c^3 values (DEVICE, FP64, [i][j][k]) of the
 * cell, using the plan's scratch for the per-atom profiles. */
ur_status ur_cell_synth(ur_plan* plan, const ur_cell* cell, double* cell_out, void* stream);

/* Materialise planes x_lo..x_hi of the ED of this plan's box (tiled cell x
 * mask, optionally zoomed; section "Electron density generation") as
 * (x_hi - x_lo + 1) n^2 reals of the plan precision at `rho` (DEVICE,
 * [x - x_lo][y][z]); [0, n - 1] gives the whole box; zoom levels of oriented
 * lattices as block sums of the oriented ED-1 (boxes up to 2048^3).
 * UR_ERR_INVALID for a range outside [0, n - 1]. */
ur_status ur_rho_generate(ur_plan* plan, const ur_cell* cell, const ur_mask* mask,
                          const ur_zoom* zoom, int32_t x_lo, int32_t x_hi, void* rho, void* stream);

/* 3D transform of eq. 1.  dir = -1: forward, scaled by 1/n^3; input `in`
 * real [x][y][z] (UR_R2C) or complex [x][y][z] (UR_C2C); output `out`
 * spectrum [kz][ky][kx] (mixed-radix plans: natural order [kx][ky][kz], see
 * ur_plan_create).  dir = +1: inverse, unscaled; input spectrum, output
 * real (UR_R2C, the half spectrum is taken as Hermitian) or complex box.
 * in and out must not overlap. */
ur_status ur_fft3d_exec(ur_plan* plan, const void* in, void* out, int32_t dir, void* stream);

/* Spherical averaging of a given spectrum (workflow step 5; section
 * "Q-calculation and spherical averaging"): bin I = |F|^2 of a spectrum
 * already in this plan's layout (DEVICE: [kz][ky][kx] on power-of-two plans,
 * the natural order [kx][ky][kz] on mixed-radix plans, as ur_fft3d_exec
 * writes it) into the plan's |Q| bins; outputs as for ur_hist. */
ur_status ur_intensity_bin(ur_plan* plan, const void* spectrum, const ur_hist* hist, void* stream);

/* Fused forward path from the unit cell (workflow steps 1-5): generate the
 * ED (tile + mask + zoom; section "Electron density generation") inside the
 * first transform pass, transform it (eq. 1, axis by axis as eq. 2
 * separates it), and bin |F|^2 into the plan's |Q| bins inside the last pass
 * (section "Q-calculation and spherical averaging"); planes, pencils and
 * rows that lie outside the particle are skipped (the paper's skipping of
 * slices without density, extended to rows and pencils).  The cell is
 * synthesised on the device from its atoms in the same call.  A zoom level
 * (factor > 1) of an oriented lattice (rot or grains) is the block sum of the
 * oriented ED-1 (workflow step 3 on the rotated-plane density): its density
 * is generated first into an n^3 buffer the plan allocates at the first such
 * call (outside any attached workspace; boxes up to 2048^3), then
 * transformed and binned.  Outputs as for ur_hist. */
ur_status ur_simulate(ur_plan* plan, const ur_cell* cell, const ur_mask* mask,
                      const ur_zoom* zoom, const ur_hist* hist, void* stream);

/* Fused forward path from a given density (workflow steps 4-5: eq. 1 axis by
 * axis as eq. 2 separates it, then the spherical averaging of section
 * "Q-calculation and spherical averaging"): rho DEVICE, n^3 reals of the plan
 * precision [x][y][z] (complex values on complex plans, UR_C2C). */
ur_status ur_simulate_rho(ur_plan* plan, const void* rho, const ur_hist* hist, void* stream);

/* Allocation-free variant of ur_simulate, for callers that cannot allocate
 * device memory: code under HIP graph capture (no eager call is needed
 * first), tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, computation and outputs as ur_simulate, but the transform
 * intermediates, block partials and cell tables live in one static device
 * array of the library (160 MiB, held by every device the library runs on
 * until the process ends) instead of the plan's workspace and cell scratch;
 * the call makes no hipMalloc / hipFree and no allocating library call.  The
 * plan's own small tables (twiddles, bin thresholds) come from
 * ur_plan_create and ur_plan_set_bins as before.
 * Limit: power-of-two plans whose workspace plus cell tables fit the array,
 * at most a 256^3 FP32 real box (with up to about 2000 bins); larger boxes
 * fail with UR_ERR_UNSUPPORTED before anything is enqueued.
 * Every call on one device shares the array, which keeps the last call's
 * contents: calls that overlap on one device (on different streams, or from
 * different threads) race and give wrong results; serialise them.  No scratch
 * word is read before the same call has written it, so nothing needs
 * clearing between calls.  Per-pass timing is not recorded for this call,
 * and ur_adjoint_reuse cannot start from it (the held forward output is that
 * of the plan's workspace). */
ur_status ur_simulate_noalloc(ur_plan* plan, const ur_cell* cell, const ur_mask* mask, const ur_zoom* zoom,
                              const ur_hist* hist, void* stream);

/* Out-of-core forward path (the 2D + 1D separation of eq. 2).
 *
 * rho_host: HOST memory holding planes x_lo..x_hi of the density,
 * [x - x_lo][y][z], (x_hi - x_lo + 1) n^2 reals of the plan precision.
 * Planes outside [x_lo, x_hi] are taken as zero and never copied (the
 * slices without density need no 2D transform).
 *   - Page-locked memory (ur_host_alloc, or any hipHostMalloc buffer) is
 *     copied to the device directly.
 *   - Ordinary pageable memory goes through four pinned bounce slabs of the
 *     plan, refilled by up to 16 host threads while the slabs ahead are in
 *     flight; the call then returns once the last slab has been handed to
 *     the copy engine.
 *   - Device memory is refused with UR_ERR_INVALID (use ur_simulate_rho).
 * Slabs of planes go to four device staging buffers, each filled on its own
 * copy stream, while earlier slabs run through the z and y passes on
 * `stream`; the x pass with binning follows.  HBM holds the staging slabs,
 * one slab of the first intermediate and the x range of the spectrum (or,
 * under an HBM budget, a kz chunk of it per pass: ur_plan_set_hbm_budget).
 * The staging and bounce buffers are allocated by the plan on first use.
 * Real mixed-radix plans: slabs of 8 planes are transformed along z (two
 * real pencils per complex line) and y as they arrive, into a half spectrum
 * that holds only planes x_lo..x_hi; the x pass reads the other planes as
 * zero (no HBM budget: the planes' half spectrum must fit).  Complex plans
 * are refused (UR_ERR_UNSUPPORTED).
 * The host buffer must stay valid until the stream is synchronised.
 * *h2d_bytes (when non-null) receives the bytes copied host to device. */
ur_status ur_simulate_host(ur_plan* plan, const void* rho_host, int32_t x_lo, int32_t x_hi,
                           const ur_hist* hist, void* stream, size_t* h2d_bytes);
/* Device workspace of the out-of-core path for planes [x_lo, x_hi] under
 * the plan's HBM budget (the four staging slabs are extra: 4 y-tiles of
 * planes).  UR_ERR_OOM when the budget cannot hold one kz row. */
ur_status ur_plan_workspace_size_host(const ur_plan* plan, int32_t nbins, int32_t x_lo, int32_t x_hi,
                                      size_t* bytes);

/* Voxel form factor (Q-calculation and spherical averaging: the earlier
 * voxel-sized sinc step, left out for tiny voxels and suggested for
 * precision near the upper Q limit).  With enable != 0 every binned
 * intensity of this plan is that of the density taken as uniform over each
 * voxel rather than sampled at its centre:
 *     I'(h, k, l) = I(h, k, l) S(h) S(k) S(l),  S(m) = sinc^2(pi m / n),
 * sinc(x) = sin(x)/x, for the fused forward paths and ur_intensity_bin
 * (totals[0] then sums I').  A zoom level applies its own voxel.  Allocates
 * a small table (call before capture); enable = 0 frees it.  The adjoint
 * (ur_adjoint, ur_adjoint_reuse) then differentiates the weighted curve:
 * each element of the weighted spectrum takes S(h) S(k) S(l) as well. */
ur_status ur_plan_set_voxel_form(ur_plan* plan, int32_t enable);

/* Block-transfer correction of a zoom level (Q-calculation and spherical
 * averaging: corrections of the coarse levels near their cut-off before the
 * merge; workflow step 3 makes a level by block integration).  A level
 * voxel sums f^3 fine voxels, which multiplies the amplitude at level index
 * m by T(m) = (1/f) sum_{j<f} exp(2 pi i m j / (f n)) per axis (fine
 * frequencies beyond the level's band alias onto it as well).  With
 * factor f >= 2 every binned intensity of this plan is divided by it:
 *     I'(h, k, l) = I(h, k, l) W(h) W(k) W(l),
 *     W(m) = (f sin(pi m / (f n)) / sin(pi m / n))^2,  W(0) = 1,
 * for the fused forward paths and ur_intensity_bin (totals[0] then sums
 * I'), times the voxel form factor when that is on too.  ur_simulate and
 * ur_simulate_noalloc then take only levels whose zoom factor is f
 * (UR_ERR_INVALID otherwise).  factor 0 or 1 turns it off.  Allocates a
 * small table (call before capture; UR_ERR_STATE while the plan is bound to
 * a live graph).  Mixed-radix plans and the adjoint refuse it
 * (UR_ERR_UNSUPPORTED). */
ur_status ur_plan_set_block_transfer(ur_plan* plan, int32_t factor);

/* Limit the out-of-core workspace to `bytes` (0: no limit).  When the x
 * range of the spectrum does not fit, ur_simulate_host runs the second stage
 * of eq. 2 kz chunk by kz chunk: every pass streams the host planes again
 * (the z pass is repeated, the y pass keeps that pass's kz rows, the x pass
 * adds their bins to the block partials of the earlier passes), so
 * host-to-device traffic grows with the number of passes while the results
 * stay those of one pass up to the order of the FP64 sums.  Sizes below one
 * kz row make ur_simulate_host fail with UR_ERR_OOM. */
ur_status ur_plan_set_hbm_budget(ur_plan* plan, size_t bytes);

/* Page-locked HOST memory for the out-of-core input, allocated with
 * hipHostMalloc at exactly `bytes` (no rounding up, so a box that takes most
 * of the host memory still fits); *out receives the pointer.  UR_ERR_OOM
 * when the allocation fails.  Free with ur_host_free (NULL is accepted). */
ur_status ur_host_alloc(size_t bytes, void** out);
ur_status ur_host_free(void* ptr);

/* Adjoint of the binned forward path (derived from eq. 1).  Given
 * g_bin[b] = dL/dI_b (DEVICE, nbins doubles) with I_b = sum/count of the
 * forward histogram `fwd`, computes
 *     grad_rho(x) = 2 Re( IFFT( G(q) F(q) ) ),  G(q) = g_bin[b(q)] / count_b,
 * (IFFT carrying 1/n^3, F of eq. 1; with the plan's voxel form factor on,
 * G(q) also carries that factor's weight S(h) S(k) S(l), and a plan that
 * removes a block transfer fails with UR_ERR_UNSUPPORTED) and, when a cell
 * is given,
 *     grad_amp[a] = sum over inside voxels of grad_rho(x) p_a(cell(x)),
 * p_a the atom's voxel-integrated profile.  For a rotated lattice or grains
 * (real plans) p_a(cell(x)) is the atom's cell grid read with the lattice's
 * interpolation at the voxel's cell coordinate (the transpose of the
 * sampler: trilinear weights, or cubic B-spline weights followed by the
 * spline solve, which is symmetric); their amplitude gradients take cell
 * edges up to 16 (larger: UR_ERR_UNSUPPORTED).  The forward transform is
 * recomputed, not stored.  Exactly one of rho (DEVICE density) and cell
 * (with mask and zoom factor 1) describes the density.  grad_rho (DEVICE, n^3
 * reals of the plan precision) and grad_amp (DEVICE, n_atoms doubles) may
 * each be NULL when not wanted. */
ur_status ur_adjoint(ur_plan* plan, const void* rho, const ur_cell* cell, const ur_mask* mask,
                     const ur_hist* fwd, const double* g_bin, void* grad_rho, double* grad_amp,
                     void* stream);

/* The amplitude gradient of ur_adjoint, starting from the y-pass output that
 * the preceding ur_simulate call on this plan left in the workspace instead
 * of recomputing the z and y passes (the forward intermediate is kept rather
 * than recomputed).  Valid when the last call on the plan was ur_simulate of
 * an ED-1 box (zoom factor 1) of a lattice aligned with the box (an oriented
 * cell: UR_ERR_UNSUPPORTED) with a real transform, with the same mask and
 * cell edge (checked: UR_ERR_STATE otherwise) and the same cell contents and
 * amplitudes (the caller's guarantee: device memory is not inspected).  The
 * held output is consumed: a second call needs a new ur_simulate.  Arguments
 * as for ur_adjoint; grad_amp (DEVICE, n_atoms doubles) is required. */
ur_status ur_adjoint_reuse(ur_plan* plan, const ur_cell* cell, const ur_mask* mask, const ur_hist* fwd,
                           const double* g_bin, double* grad_amp, void* stream);

/* Merge modes (workflow step 6; dataMerge's rule is not given in the paper,
 * the rule below is this library's reading):
 *   each level's eq.-1 intensities are scaled back to absolute units by
 *   s_k = (n_k^3)^2; a level is valid for a bin when the bin centre lies in
 *   [dq_k, sqrt(3) pi / (2 voxel_k)] and its count >= n_min.
 *   UR_MERGE_FINEST  the valid level with the smallest voxel owns the bin
 *   UR_MERGE_POOLED  pooled scaled sums over the valid levels
 *   UR_MERGE_IVW     inverse-variance weighted mean of the valid levels */
#define UR_MERGE_FINEST 0
#define UR_MERGE_POOLED 1
#define UR_MERGE_IVW 2

/* levels: HOST array of nlevels (<= 8) histograms (their arrays DEVICE),
 * with box edges n[] and voxel sizes voxel[] (HOST).  edges: DEVICE, nbins+1
 * values shared by every level.  Outputs DEVICE: mean[nbins], sem[nbins],
 * owner[nbins] (level index for FINEST, number of contributing levels
 * otherwise, -1 with NaN mean/sem when no level is valid). */
ur_status ur_merge_zooms(int32_t nlevels, const ur_hist* levels, const int32_t* n,
                         const double* voxel, int32_t nbins, const double* edges, int32_t mode,
                         double n_min, double* mean, double* sem, int32_t* owner, void* stream);

/* Ewald-sphere detector image (Q-calculation and spherical averaging: 2D
 * data of an anisotropic sample taken on a spherical shell whose thickness
 * follows the wavelength distribution).  Flat detector normal to the beam:
 * pixel (iu, iv) sits at distance * beam + (iu - cu) pixel du
 * + (iv - cv) pixel dv from the sample (box axes x, y, z; beam, du, dv
 * orthonormal); s is its unit direction.  For each wavelength node
 * lambda_j = wavelength (1 + rel_spread t_j), t_j evenly spaced on [-3, 3]
 * with weights exp(-t_j^2/2) normalised (one node at t = 0 when
 * rel_spread = 0), q = (2 pi / lambda_j)(s - beam) (nm^-1) is located on
 * the reciprocal grid (step 2 pi / (n voxel)) and I = |F|^2 is
 * interpolated trilinearly between the grid points (the DFT taken as
 * periodic; a real transform's missing half from F(-q) = F(q)*).
 * image[iv][iu] (DEVICE, nv x nu doubles) receives the node-weighted mean.
 * spectrum: DEVICE, this plan's [kz][ky][kx] layout (ur_fft3d_exec).
 * UR_ERR_INVALID for non-positive lengths, rel_spread outside [0, 0.3),
 * n_lambda outside [1, 64], or axes that are not orthonormal. */
typedef struct {
  double wavelength;   /* nm */
  double rel_spread;   /* Gaussian sigma of the wavelength, relative */
  int32_t n_lambda;    /* wavelength nodes when rel_spread > 0 */
  double beam[3];      /* unit vector of the incident beam */
  double du[3];        /* unit vector along detector rows (iu) */
  double dv[3];        /* unit vector along detector columns (iv) */
  double distance;     /* sample to detector, along the beam */
  double pixel;        /* pixel pitch, same unit as distance */
  double cu, cv;       /* beam centre on the detector, pixels */
  int32_t nu, nv;      /* pixels per row, rows */
} ur_ewald;
ur_status ur_ewald_image(ur_plan* plan, const void* spectrum, const ur_ewald* geom, double* image, void* stream);

/* Peak integrals for the degree of crystallinity (Results and Discussion: the
 * simulation assumes perfect crystallinity, so the integral intensity under
 * a simulated diffraction peak stands for 100 % crystallinity, in absolute
 * units or relative to the small-angle signal; a measured peak integral
 * divided by it gives the degree of crystallinity).  For each window
 * w = [q_lo, q_hi] (HOST windows[2*nwin], nm^-1, q_lo < q_hi) the bins of
 * the curve whose centres (e_b + e_b+1)/2 lie in the window and whose mean
 * is not NaN (empty bins are skipped) give, with widths d_b = e_b+1 - e_b:
 *   out[3w+0] peak  = sum_b (mean_b - base(q_b)) d_b, base the straight line
 *             through the (centre, mean) of the window's first and last bins,
 *   out[3w+1] total = sum_b mean_b d_b,
 *   out[3w+2] the number of bins used;
 * fewer than two bins give NaN peak and total.  edges: DEVICE nbins+1
 * (strictly increasing), mean: DEVICE nbins, out: DEVICE 3*nwin doubles.
 * No allocation (capturable).  UR_ERR_INVALID for nbins outside [1, 4096],
 * nwin outside [1, 64], a window with q_lo >= q_hi or non-finite ends, or a
 * null pointer. */
ur_status ur_peak_integrals(int32_t nbins, const double* edges, const double* mean, int32_t nwin,
                            const double* windows, double* out, void* stream);

/* chi^2 misfit of a simulated curve against a target curve, and its
 * gradient per bin, the g_bin that ur_adjoint takes (Results and Discussion:
 * the polydispersity estimate from some 200 volume-weighted simulations is a
 * fit of simulated to measured curves; the relative uncertainty
 * sigma_b = rel_sigma target_b is this library's reading, the paper gives
 * none):
 *     chi2     = sum over bins with count_b > 0 of ((mean_b - target_b) / sigma_b)^2,
 *     g_bin[b] = d chi2 / d mean_b = 2 (mean_b - target_b) / sigma_b^2  (0 for empty bins).
 * mean, count (the ur_hist fields of the simulated curve), target: DEVICE,
 * nbins doubles; out_chi2: DEVICE, 1 double; g_bin: DEVICE nbins doubles, or
 * NULL.  The sum is compensated and taken in a fixed order (the same bits on
 * every call).  No allocation (capturable).  UR_ERR_INVALID for nbins outside
 * [1, 4096], rel_sigma not positive and finite, or a null pointer. */
ur_status ur_chi2(int32_t nbins, const double* mean, const double* count, const double* target, double rel_sigma,
                  double* out_chi2, double* g_bin, void* stream);

/* Polydisperse ensemble (Results and Discussion: polydispersity described by
 * some 200 volume-weighted contributions, one simulation each).  For nboxes
 * boxes that share one bin set (one particle each, summed incoherently),
 * per bin:
 *     out_mean[b] = sum_k w[k] mean[k][b],
 *     out_sem[b]  = sqrt( sum_k (w[k] sem[k][b])^2 )   (independent boxes).
 * mean, sem: DEVICE [nboxes][nbins] (the per-box outputs of ur_simulate);
 * weights: DEVICE nboxes number weights (a volume fraction phi_k gives
 * w_k = phi_k / V_k with V_k the particle volume); outputs DEVICE nbins.
 * Empty bins give NaN means, one-voxel bins NaN SEMs.  No allocation: the
 * call can sit in a captured graph after the boxes.  UR_ERR_INVALID for
 * nboxes < 1, nbins outside [1, 4096] or a null pointer. */
ur_status ur_ensemble(int32_t nboxes, int32_t nbins, const double* mean, const double* sem,
                      const double* weights, double* out_mean, double* out_sem, void* stream);

/* Record the work enqueued on `stream` between begin and end into a HIP
 * graph, instantiate it, and return the executable graph (as void*); replay
 * it with ur_graph_launch and release it with ur_graph_destroy.  Every entry
 * point above except ur_plan_create / set_bins / set_workspace and the
 * out-of-core ur_simulate_host may be recorded; the plans' workspaces must
 * already be large enough (make the same calls once eagerly first), since
 * nothing is allocated under capture.
 * Lifetime: a graph holds raw device pointers into the workspaces and tables
 * of the plans whose calls it recorded.  From ur_graph_end until
 * ur_graph_destroy of every such graph, a plan refuses (UR_ERR_STATE, before
 * anything is freed) every call that would reallocate or rewrite them:
 * ur_plan_set_bins, ur_plan_set_workspace with another pointer, switching
 * ur_plan_set_voxel_form, and calls needing a larger workspace or cell
 * scratch (more bins, larger cells or more atoms, a larger out-of-core
 * range).  A plan recorded under a capture that ur_graph_begin did not start
 * stays bound for its whole life.  Destroying a plan invalidates the graphs
 * recorded from it (replaying them is undefined).  One open capture per
 * thread. */
ur_status ur_graph_begin(void* stream);
ur_status ur_graph_end(void* stream, void** graph_exec);
ur_status ur_graph_launch(void* graph_exec, void* stream);
ur_status ur_graph_destroy(void* graph_exec);

/* Per-pass timing of the plan's own launches: when enabled, the forward path
 * records a HIP event pair on the call's stream around each of its passes
 * (0 cell tables, 1 z pass, 2 y pass, 3 x pass, 4 finalize).
 * ur_plan_read_timing waits for those events and returns, per pass, the
 * summed elapsed ms, the algorithmic HBM bytes of one launch (the bytes the
 * pruned pass must read and write: spectrum elements moved x element size,
 * plus partial histograms) and the number of timed launches since the last
 * read.  Arrays hold npass (<= 5) entries. */
ur_status ur_plan_set_timing(ur_plan* plan, int32_t enable);
ur_status ur_plan_read_timing(ur_plan* plan, int32_t npass, double* ms, double* bytes, int32_t* launches);

/* Thread-local description of the last failure on this thread. */
const char* ur_last_error(void);

/* Library version string. */
const char* ur_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ULTIMA_H */
