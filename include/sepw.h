/*
 * sepw.h -- separable W-projection gridding and degridding on MI355X (gfx950).
 *
 * C ABI of the hot path of Merry (2015), "Approximating W projection as a
 * separable kernel" (arXiv:1511.07152):
 *
 *   sepw_make_kernels  oversampled 1D GCF tables per w-plane (Section 3, the
 *                      separable screen g1_w and g~_w = g1_w(l) g1_w(m);
 *                      Section 2, oversampled lookup tables and the
 *                      anti-aliasing taper c; Section 4.1, facet tables)
 *   sepw_plan_create   uv -> grid cell and 1/O sub-cell offset, w -> plane,
 *                      counting sort of visibilities into grid tiles
 *                      (sepw_plan_create_channels: uvw in metres per row,
 *                      scaled per channel)
 *   sepw_grid          visibilities -> uv grid -> dirty image (Section 2,
 *                      dirty-image equation and its W-projection form;
 *                      Section 5, separable update with the row product reused)
 *   sepw_degrid        model image -> uv grid -> visibilities (Section 2,
 *                      prediction equation; Section 6, prediction for major
 *                      cycles)
 *   sepw_grid_batched  many facet/snapshot jobs in one persistent launch
 *                      (sepw_autotune_batched picks its launch shape)
 *                      (Section 4.1 faceting, Section 4.2 snapshots)
 *   sepw_wstack_*      W-stacking hybrid: w-slices corrected in image space,
 *                      residual w by separable W projection (Section 4.3)
 *   sepw_wsnap_*       W snapshots: per-snapshot plane fit, residual w by
 *                      separable W projection, image reprojection (Section 4.2)
 *   sepw_kernels_set_correction
 *                      the 2D correction table F_w - F~_w applied beside the
 *                      separable GCF by grid and degrid (Section 6)
 *
 * Conventions (the paper leaves these open; the library fixes them):
 *   N     grid and image size, even.           fov  full image width in
 *   S     GCF support in cells, odd, 1..31 and       direction cosines [rad].
 *         at most N - 1.  Up to 15 the footprints are gridded as tiles on the
 *         matrix cores (all precisions); 17..31 take a per-visibility FP32 path
 *         on the vector unit (FP16/BF16 and the correction table are
 *         SEPW_ERR_UNSUPPORTED there).
 *   O     oversampling factor, power of two, 1..128.
 *   P     number of w-planes, 1..65535, uniform on [w_lo, w_hi]; plane k
 *         stands for w_k = w_lo + (k + 1/2)(w_hi - w_lo)/P; a visibility goes
 *         to plane clamp(floor((w - w_lo) P / (w_hi - w_lo)), 0, P-1).
 *   Pixel p is at l_p = (p - N/2) fov / N; grid cell j is at u_j = (j - N/2)/fov.
 *   Images and grids are N*N row-major complex64, rows along m (v).
 *   Grid -> image is the centred, unnormalised DFT with sign +, matching the
 *   dirty-image equation; image -> grid is its conjugate transpose.
 *   uv rounding: nearest 1/O cell, ties upwards; a visibility whose S x S
 *   footprint leaves the grid, or whose u, v or w is not finite, is skipped and
 *   counted as dropped (never wrapped).
 *
 * Memory and streams: every vis / weight / image / grid pointer is a DEVICE
 * pointer owned by the caller; tables, plans and scratch are owned by the
 * library.  Every call is asynchronous on the given HIP stream (NULL = the
 * default stream) unless stated; a kernel failure surfaces as SEPW_ERR_HIP at
 * a later call.  A plan or kernels object must not be used by two calls that
 * overlap in time (its scratch and FFT plan are shared).  A batched call
 * (sepw_grid_batched, sepw_autotune_batched) keeps its job table, work
 * counter and launch width in its first plan, and the W-stacking and
 * W-snapshot calls in their first plan: there is no process-wide batch state,
 * so batched calls whose plans and kernels objects are distinct may overlap
 * on different streams.
 *
 * Errors: every call returns SEPW_OK or a negative code; no exception crosses
 * the ABI.  Arguments are validated on the host before any device work, so a
 * rejected call has no side effect.
 */
#ifndef SEPW_H
#define SEPW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } sepw_c64;
typedef struct sepw_kernels_s* sepw_kernels;   /* tables + taper + FFT plan   */
typedef struct sepw_plan_s*    sepw_plan;       /* binned uvw for one kernels  */
typedef struct sepw_wstack_s*  sepw_wstack;     /* W-stacking slices + plans   */
typedef struct sepw_wsnap_s*   sepw_wsnap;      /* W-snapshot planes + plans   */

enum {
  SEPW_OK = 0,
  SEPW_ERR_ARG = -1,          /* invalid argument (checked before device work) */
  SEPW_ERR_NO_DEVICE = -2,    /* no HIP device visible                         */
  SEPW_ERR_HIP = -3,          /* a HIP runtime or kernel error                 */
  SEPW_ERR_OOM = -4,          /* device allocation failed                      */
  SEPW_ERR_UNSUPPORTED = -5,  /* valid but not implemented (e.g. S > 31)       */
  SEPW_ERR_FFT = -6           /* hipFFT failure                                */
};

enum { SEPW_TAPER_PSWF = 0, SEPW_TAPER_NONE = 1, SEPW_TAPER_USER = 2 };
enum { SEPW_FP32 = 0, SEPW_FP16 = 1, SEPW_BF16 = 2 };

/* Flags for sepw_grid / sepw_degrid / sepw_grid_batched. */
#define SEPW_GRID_ONLY 0x1u  /* grid: output the uv grid (no FFT, no correction).
                                degrid: the input is a uv grid.                  */
#define SEPW_MUL_N     0x2u  /* grid: dirty image I_D = n F+[G] / (c1 c1).       */
#define SEPW_DIV_N     0x4u  /* grid: F+[G] / (n c1 c1), the exact adjoint of
                                degrid with SEPW_DIV_N.
                                degrid: X = image / n before the FFT, i.e. the
                                prediction equation for a model image I.        */
/* The same flags under the names of the problem statement: the dirty image
   (x n), the adjoint pair (/ n on both sides) and the model (/ n).  Footprints
   that leave the grid are always dropped, never wrapped. */
#define SEPW_DIRTY     SEPW_MUL_N
#define SEPW_ADJOINT   SEPW_DIV_N
#define SEPW_MODEL     SEPW_DIV_N
#define SEPW_WRAP_FORBIDDEN 0x0u
#define SEPW_REAL      0x8u  /* sepw_grid / sepw_degrid only, not with GRID_ONLY:
                                the image is real, DEVICE float32[N*N]: degrid
                                reads a real model image; grid writes the real
                                part of the image (the adjoint of predicting
                                from a real model).  Gridding then transforms
                                in the kernels' work array, shared by the
                                kernels' plans, so such calls on one kernels
                                object do not overlap across streams.        */

/* Kernel (GCF table) parameters.  Fill with sepw_default_params first. */
typedef struct {
  int32_t grid_size;       /* N                                                  */
  int32_t support;         /* S                                                  */
  int32_t oversample;      /* O                                                  */
  int32_t n_planes;        /* P                                                  */
  double  fov;             /* field of view [rad]                                */
  double  w_lo, w_hi;      /* w-plane range [wavelengths], w_lo < w_hi           */
  int32_t taper;           /* SEPW_TAPER_*                                       */
  int32_t precision;       /* SEPW_FP32 (FP16/BF16 select the MFMA form)         */
  double  taper_width;     /* PSWF: width W in cells, c = pi W / 2; <= 0 means S */
  const double* taper_samples; /* SEPW_TAPER_USER: N host doubles c1(l_p) > 0    */
  double  a_u, b_u;        /* u-axis screen exp(-2 pi i w (a l^2 + b l^4))        */
  double  a_v, b_v;        /* v-axis screen; defaults 1/2 and gamma = 5/24       */
  int32_t facet;           /* nonzero: image-plane facet at (l0, m0), Section 4.1;
                              a_u, a_v, b_u, b_v are then derived and ignored    */
  int32_t reserved;
  double  l0, m0;          /* facet centre (direction cosines)                   */
} sepw_kernel_params;

/* Defaults: taper PSWF of width S, a = 1/2, b = 5/24 (Section 3's minimax
   gamma), FP32, no facet.  Geometry fields are zeroed and must be set. */
void sepw_default_params(sepw_kernel_params* p);

/* Build the GCF tables on the device (FP64 phase and sums, stored complex64):
 *   T[k][fi][s] = (1/N) sum_{p<N} c1(l_p) exp(-2 pi i w_k (a l_p^2 + b l_p^4))
 *                       * exp(-2 pi i (s - S/2 - (fi - O/2)/O)(p - N/2)/N)
 * for the u axis (a_u, b_u) and, if different, the v axis (a_v, b_v).  With
 * facet != 0 the axis coefficients are 1/2 (1/n0 + l0^2/n0^3) and
 * 1/2 (1/n0 + m0^2/n0^3) with b = 0 (Section 4.1).  c1 is the zeroth prolate
 * spheroidal wave function psi_0(pi W / 2, 2 l / fov), normalised to c1(0) = 1.
 * Besides the tables the object holds an N x N complex64 work grid, a hipFFT
 * plan and, for FP16 / BF16 kernels with S <= 15, the degridding operand grid
 * ((N + 32)^2 dwords, two such planes for BF16; 68 MB at N = 4096).
 * Synchronises the stream once (host set-up of the taper coefficients).
 * Errors: SEPW_ERR_ARG for any out-of-range field, SEPW_ERR_NO_DEVICE,
 * SEPW_ERR_OOM, SEPW_ERR_HIP, SEPW_ERR_FFT.  *out is NULL on error. */
int sepw_make_kernels(const sepw_kernel_params* params, void* hip_stream, sepw_kernels* out);

/* Copy a table (axis 0 = u, 1 = v) into a device buffer of P*O*S complex64,
   layout [k][fi][s]; or the taper c1(l_p) into a device buffer of N doubles. */
int sepw_kernels_table(sepw_kernels k, int32_t axis, sepw_c64* out, void* hip_stream);
int sepw_kernels_taper(sepw_kernels k, double* out, void* hip_stream);

/* Section 6 (the correction F_w - F~_w stored as a small full 2D table):
 * attach to k a correction table with odd support Sc = support and
 * oversampling Oc = oversample, or remove it (support = 0).  While attached,
 * sepw_grid, sepw_degrid, sepw_grid_batched and the W-stacking calls on plans
 * of k add, beside every separable footprint, the 2D footprint
 *   y_i C[k_i][fu][fv][sv][su] at cell (cv_c - Sc/2 + sv, cu_c - Sc/2 + su)
 * (degridding: its adjoint, the sum of G conj(C) over the same cells), where
 *   C[k][fu][fv][su][sv] = (1/N^2) sum_{q,p} c1(l_p) c1(m_q)
 *       [exp(2 pi i w_k (n - 1)) - exp(-2 pi i w_k (phi_u(l_p) + phi_v(m_q)))]
 *       exp(-2 pi i [Du (p - N/2) + Dv (q - N/2)] / N),
 *   phi(l) = a l^2 + b l^4 per axis, Du = su - Sc/2 - (fu - Oc/2)/Oc (Dv alike),
 * i.e. the exact 2D table minus the outer product of the separable ones,
 * sampled at the correction's own support and rate; and (cu_c, fu) is the
 * point of the 1/Oc lattice nearest to the visibility's quantised position
 * cu + (fi_u - O/2)/O, ties upwards (cu_c is cu or cu + 1).  With Sc = S and
 * Oc = O gridding is then exactly gridding with the exact 2D GCF.  The table
 * is generated now (FP64, stored complex64) and again by
 * sepw_kernels_set_wrange; existing plans stay valid.  For FP32 kernels the
 * table is then also factored, per plane, into at most 8 separable terms
 * sum_r a_r[fu][su] b_r[fv][sv] with every entry of the difference within
 * 1e-6 of the table's largest entry (cross approximation with complete
 * pivoting; the table's exponent gap is a short polynomial in l^2 and m^2, so
 * few terms suffice: 3 at 3 degrees), and grid / degrid run the separable
 * matrix-core kernels once per term instead of walking the table; otherwise
 * (16-bit kernels, more terms needed, or a table above 2^24 entries) the
 * correction passes walk the table.  Both give the same footprint sums.
 * Synchronises the stream (taper check; the factoring, here and in
 * sepw_kernels_set_wrange, copies the table to the host).
 * Errors: SEPW_ERR_ARG (null k; support even, negative or above S; oversample
 * not a power of two or above O; support above S - 2 when 1 < oversample < O,
 * where the coarse cell can be the next one), SEPW_ERR_UNSUPPORTED (facet
 * kernels; kernels with S above 15; a taper not symmetric about the image
 * centre; (Sc/2) Oc + Oc/2 above 63), SEPW_ERR_OOM, SEPW_ERR_HIP. */
int sepw_kernels_set_correction(sepw_kernels k, int32_t support, int32_t oversample,
                                void* hip_stream);
/* Copy the attached correction table into a device buffer of P*Oc*Oc*Sc*Sc
 * complex64, layout [k][fu][fv][sv][su] (su fastest).
 * Errors: SEPW_ERR_ARG (null pointers, no correction attached), SEPW_ERR_HIP. */
int sepw_kernels_correction_table(sepw_kernels k, sepw_c64* out, void* hip_stream);
/* Choose how corrections of k run: enable = 1 (the default) factors the
 * table into separable terms where it can (see sepw_kernels_set_correction),
 * 0 makes grid / degrid walk the table itself.  Applies to the attached table
 * (factoring it now synchronises the stream) and to later ones.
 * Errors: SEPW_ERR_ARG (null k, enable not 0 or 1), SEPW_ERR_OOM, SEPW_ERR_HIP. */
int sepw_kernels_correction_terms(sepw_kernels k, int32_t enable, void* hip_stream);
/* Number of separable terms the attached correction runs as (*rank >= 0; 0
 * for an all-zero table), or -1 when the correction passes walk the table.
 * Errors: SEPW_ERR_ARG (null pointers, no correction attached). */
int sepw_kernels_correction_rank(sepw_kernels k, int32_t* rank);

/* Quantise and bin nvis visibilities (u, v, w: DEVICE float64 arrays in
 * wavelengths, caller order).  In facet mode u, v are shifted by -w l0/n0,
 * -w m0/n0 (Section 4.1) and the per-visibility phase rotation
 * exp(+2 pi i (u l0 + v m0 + w (n0 - 1))) is stored in the plan.
 * The plan keeps its own binned copy; u, v, w may be freed afterwards.
 * n_dropped: optional pointer to the number of skipped visibilities: a HOST
 * pointer makes the call synchronise the stream and store it; a DEVICE pointer
 * (device memory, told apart with hipPointerGetAttributes) gets it written on
 * the stream, without a synchronisation.  nvis may be 0.
 * Errors: SEPW_ERR_ARG (null kernels, nvis < 0 or > 2^31-2, null arrays with
 * nvis > 0), SEPW_ERR_UNSUPPORTED (more tiles than the in-LDS tile sort
 * handles: N > 16384 at S = 15, N > 32768 at S <= 13), SEPW_ERR_OOM,
 * SEPW_ERR_HIP. */
int sepw_plan_create(sepw_kernels k, int64_t nvis, const double* u, const double* v,
                     const double* w, int64_t* n_dropped, void* hip_stream, sepw_plan* out);

/* Re-bin a new batch of nvis <= (nvis at creation) visibilities into an
 * existing plan without any allocation (the per-batch form of plan creation;
 * also required after sepw_kernels_set_wrange).  Same inputs and n_dropped
 * semantics as sepw_plan_create.  Errors: SEPW_ERR_ARG (null plan, nvis out of
 * range, null arrays with nvis > 0), SEPW_ERR_HIP. */
int sepw_plan_rebin(sepw_plan p, int64_t nvis, const double* u, const double* v, const double* w,
                    int64_t* n_dropped, void* hip_stream);

/* Channel-shared coordinates: the plan of nrows * nchan visibilities whose
 * u, v, w are given once per (baseline, time) row in metres and scaled per
 * channel, visibility i = row * nchan + ch (caller order of vis, weight and
 * results) at
 *   u_i = uvw[row][0] * (freq[ch] / c),   c = 299,792,458 m/s,
 * (likewise v, w) -- one IEEE division, then one IEEE multiplication, so the
 * bins equal those of sepw_plan_create on u, v, w formed that way.  Section 2
 * works in wavelengths; this layout reads 24 / nchan bytes of coordinates per
 * visibility instead of 24.  uvw: DEVICE float64 [nrows][3]; freq: DEVICE
 * float64 [nchan] in Hz.  Everything else as sepw_plan_create /
 * sepw_plan_rebin (facet mode included).
 * Errors: SEPW_ERR_ARG (null pointers, nrows < 0, nchan < 1, nrows * nchan
 * above 2^31 - 2 or, for rebin, above the plan's capacity), and those of
 * sepw_plan_create. */
int sepw_plan_create_channels(sepw_kernels k, int64_t nrows, int32_t nchan, const double* uvw,
                              const double* freq, int64_t* n_dropped, void* hip_stream,
                              sepw_plan* out);
int sepw_plan_rebin_channels(sepw_plan p, int64_t nrows, int32_t nchan, const double* uvw,
                             const double* freq, int64_t* n_dropped, void* hip_stream);

/* Per-visibility bins in caller order, for verification: out is a DEVICE
   int32 array [nvis][7] = (cell_u, fi_u, cell_v, fi_v, plane, tile, dropped);
   tile = (cell_v / c) * ceil(N / c) + cell_u / c with c = sepw_plan_tile_size;
   dropped rows are (0, 0, 0, 0, 0, -1, 1). */
int sepw_plan_bins(sepw_plan p, int32_t* out, void* hip_stream);
int32_t sepw_plan_tile_size(sepw_plan p);

/* Grid weighted visibilities: G = sum_i W_i V_i Tu[k_i][fi_u][.] (x) Tv[k_i][fi_v][.]
 * placed at cells cell - S/2 .. cell + S/2 (Section 5's separable update).
 * vis: DEVICE complex64[nvis]; weight: DEVICE float[nvis] or NULL (all 1);
 * out: DEVICE complex64[N*N], overwritten.  Without SEPW_GRID_ONLY the output is
 * the image F+[G] / (c1 c1), times n (SEPW_MUL_N) or over n (SEPW_DIV_N).
 * Errors: SEPW_ERR_ARG (null pointers, both MUL_N and DIV_N, REAL with
 * GRID_ONLY), SEPW_ERR_HIP, SEPW_ERR_FFT. */
int sepw_grid(sepw_plan p, const sepw_c64* vis, const float* weight, sepw_c64* out,
              uint32_t flags, void* hip_stream);

/* Non-finite values.  For S <= 15 the sums run over 16 x 16 cell regions
 * (tile core plus footprint, zero taps outside the footprint), and 0 times
 * NaN or Inf is NaN: a NaN or Inf in W V makes the whole region of its tile
 * non-finite (cells within 16 of its own cell, a superset of its footprint),
 * and a NaN or Inf grid cell makes non-finite every degridded visibility
 * whose tile region holds it (cells past the grid edge read the edge cell
 * times 0).  Other cells and visibilities are unaffected; the FP16 form's
 * power-of-two scales are taken over finite values only.  For S = 17..31
 * (per-visibility path) a non-finite value reaches its own footprint only.
 * The images and predictions of the FFT passes spread it over the plane. */

/* Degrid: V_i = sum_t conj(Tv[..][t]) sum_s conj(Tu[..][s]) Ghat[cv-S/2+t][cu-S/2+s],
 * the adjoint of sepw_grid.  Without SEPW_GRID_ONLY, Ghat = F-[X / (c1 c1)] with
 * X = image (or image / n with SEPW_DIV_N).  in: DEVICE complex64[N*N] (not
 * modified); vis_out: DEVICE complex64[nvis], dropped visibilities get 0.
 * Errors: as sepw_grid (SEPW_MUL_N is rejected). */
int sepw_degrid(sepw_plan p, const sepw_c64* in, sepw_c64* vis_out, uint32_t flags,
                void* hip_stream);

/* Grid njobs independent jobs (facets or snapshots, each with its own kernels
 * and plan, all with the same N, S and precision) in ONE persistent launch
 * that walks a combined work list ordered by descending cost; then one
 * batched FFT and correction.  Arrays are host arrays of njobs entries
 * holding device pointers; weights may be NULL (or hold NULLs).  Same flags
 * and output as sepw_grid, per job.
 * Errors: SEPW_ERR_ARG (njobs < 1, mismatched N/S/precision, nulls),
 * SEPW_ERR_OOM, SEPW_ERR_HIP, SEPW_ERR_FFT. */
int sepw_grid_batched(int32_t njobs, const sepw_plan* plans, const sepw_c64* const* vis,
                      const float* const* weight, sepw_c64* const* out, uint32_t flags,
                      void* hip_stream);

/* sepw_grid_batched for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same jobs, flags, output and errors, but the job tables, the per-job work
 * prefix and the work counters live in one static device array of the library
 * (about 51 KB; each GPU the library runs on holds its own copy until the
 * process ends), written by a small kernel from kernel arguments, so the call
 * makes no hipMalloc, hipFree, pinned-host or other allocating call.  At most
 * 256 jobs: njobs > 256 returns SEPW_ERR_UNSUPPORTED with no device work.
 * The plans and the caller's outputs must already exist.  Every call on one
 * GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap in time on one GPU (different streams or threads) race. */
int sepw_grid_batched_noalloc(int32_t njobs, const sepw_plan* plans, const sepw_c64* const* vis,
                              const float* const* weight, sepw_c64* const* out, uint32_t flags,
                              void* hip_stream);

/* W-stacking hybrid (Section 4.3): the visibilities are partitioned into
 * n_slices uniform w-slices on [w_lo, w_hi] (slice s = clamp(floor((w - w_lo)
 * n_slices / (w_hi - w_lo)), 0, n_slices - 1), centre w_s = w_lo + (s + 1/2)
 * (w_hi - w_lo) / n_slices); slice s is imaged with the separable W-projection
 * path on its residual w - w_s, and its image is multiplied by the exact
 * phase exp(2 pi i w_s (n - 1)) before the slice images are summed.  k holds
 * the residual tables: plain (non-facet) kernels whose planes span exactly
 * [-h, h], h = (w_hi - w_lo) / (2 n_slices).  u, v, w: DEVICE float64[nvis],
 * read during the call only.  *n_dropped (host, may be NULL) counts
 * visibilities whose footprint leaves the grid or whose w is not finite.
 * Synchronises the stream (the slice sizes come to the host).  The object
 * holds, besides a plan per slice, as many N x N complex64 slice images as fit
 * in 4 GiB (at least one, at most n_slices): the slices are gridded that many
 * at a time in one batched launch (sepw_grid_batched) and, in FP32, degridded
 * likewise.
 * Errors: SEPW_ERR_ARG (null k or out, facet kernels, n_slices outside
 * [1, 4096], w_lo >= w_hi, kernels' w range not [-h, h], nvis out of range),
 * SEPW_ERR_OOM, SEPW_ERR_HIP. */
int sepw_wstack_create(sepw_kernels k, int32_t n_slices, double w_lo, double w_hi, int64_t nvis,
                       const double* u, const double* v, const double* w, int64_t* n_dropped,
                       void* hip_stream, sepw_wstack* out);

/* W-stacking with non-uniform slices (Section 4.3 suggests many narrow
 * slices near w = 0 and wider ones at large |w|, adapted to the visibility
 * density).  edges: HOST float64[n_slices + 1], finite and strictly
 * increasing; slice s holds e_s <= w < e_{s+1} (w below e_0 in slice 0, w at
 * or above e_ns in the last slice, non-finite w in slice 0 and dropped),
 * centre w_s = (e_s + e_{s+1}) / 2.  Each non-empty slice gets tables of its
 * own: k's parameters (N, fov, S, O, P, taper, precision) with the w range
 * [-h_s, h_s], h_s = (e_{s+1} - e_s) / 2, so a narrow slice has finely spaced
 * planes; k's own w range is not used.  The object holds those slices'
 * tables (with k's taper, FFT plan and work array) besides the plans; in
 * FP32 the slices are degridded in one batched launch that reads each slice's
 * tables through the caches.  Everything else as sepw_wstack_create; the object is
 * used with sepw_wstack_grid / _degrid / sepw_free_wstack.
 * Errors: SEPW_ERR_ARG (null k, edges or out, facet kernels, n_slices outside
 * [1, 4096], edges not finite and increasing, nvis out of range),
 * SEPW_ERR_UNSUPPORTED (k carries a correction table), SEPW_ERR_OOM,
 * SEPW_ERR_HIP, SEPW_ERR_FFT. */
int sepw_wstack_create_edges(sepw_kernels k, int32_t n_slices, const double* edges, int64_t nvis,
                             const double* u, const double* v, const double* w,
                             int64_t* n_dropped, void* hip_stream, sepw_wstack* out);

/* Density-adapted slice edges (Section 4.3's adaptation of slice width to the
 * visibility density): the finite w (DEVICE float64[nvis]) are counted in
 * 16384 uniform bins of [w_lo, w_hi] (bin floor((w - w_lo) 16384 / (w_hi -
 * w_lo)), clamped); edge k, 0 < k < n_slices, is w_lo + j d (d = (w_hi - w_lo)
 * / 16384) for the first bin boundary j below which at least k n / n_slices of
 * the n finite visibilities lie, raised to keep the edges increasing and
 * lowered to leave one bin for each later slice; e_0 = w_lo,
 * e_ns = w_hi.  Slices then hold about n / n_slices visibilities each.
 * edges: HOST float64[n_slices + 1], written.  Synchronises the stream.
 * Errors: SEPW_ERR_ARG (null edges, n_slices outside [1, 4096], w_lo >= w_hi
 * or not finite, nvis out of range, null w with nvis > 0),
 * SEPW_ERR_NO_DEVICE, SEPW_ERR_OOM, SEPW_ERR_HIP. */
int sepw_wstack_density_edges(int64_t nvis, const double* w, int32_t n_slices, double w_lo,
                              double w_hi, double* edges, void* hip_stream);

/* Dirty image of the W-stacking hybrid: sum over slices of
 * exp(2 pi i w_s (n - 1)) times the slice's image (sepw_grid without
 * SEPW_GRID_ONLY, same flags SEPW_MUL_N / SEPW_DIV_N).  vis, weight: DEVICE,
 * caller order (weight may be NULL); image_out: DEVICE complex64[N*N].
 * Errors: SEPW_ERR_ARG (null pointers, SEPW_GRID_ONLY or both n flags), and
 * those of sepw_grid. */
int sepw_wstack_grid(sepw_wstack ws, const sepw_c64* vis, const float* weight, sepw_c64* image_out,
                     uint32_t flags, void* hip_stream);

/* Prediction, the adjoint of sepw_wstack_grid: slice s degrids
 * image exp(-2 pi i w_s (n - 1)) (with SEPW_DIV_N: image / n) on its residual
 * w.  image: DEVICE complex64[N*N]; vis_out: DEVICE complex64[nvis], caller
 * order, 0 for dropped visibilities.
 * Errors: SEPW_ERR_ARG (null pointers, flags other than SEPW_DIV_N), and those
 * of sepw_degrid. */
int sepw_wstack_degrid(sepw_wstack ws, const sepw_c64* image, sepw_c64* vis_out, uint32_t flags,
                       void* hip_stream);

/* Length of the plan's gridding work items: the number of tile slots
 * (visibilities, each tile padded to whole groups of 4) of one row of tiles
 * that one wave processes in order.  Default 1024; must be a multiple of 4 in
 * [64, 8192].  Rebuilds the plan's gridding work list asynchronously on the
 * stream (it waits for the stream once when the list has to grow); later
 * rebins keep the length.  Used by sepw_grid and sepw_grid_batched.
 * Errors: SEPW_ERR_ARG (null p, invalid slots), SEPW_ERR_OOM, SEPW_ERR_HIP. */
int sepw_plan_set_item_slots(sepw_plan p, int32_t slots, void* hip_stream);

/* The same for the degridding work list (sepw_degrid).  Default 224: shorter
 * items keep fewer rows of scattered results in flight per L2.  Same range,
 * behaviour and errors as sepw_plan_set_item_slots. */
int sepw_plan_set_degrid_item_slots(sepw_plan p, int32_t slots, void* hip_stream);

/* Autotuner of the batching form's launch shape: times sepw_grid_batched with
 * SEPW_GRID_ONLY on these jobs (HIP events, one warm-up and two timed runs per
 * candidate) for every work-item length in {256, 512, 1024, 2048} and every
 * persistent launch width in {2, 4, 8} workgroups per compute unit, and keeps
 * the fastest pair: the plans keep that item length and that width (used by
 * later batched calls that they lead).  The pair is returned in *item_slots and
 * *blocks_per_cu (either may be NULL).  Results are cached per process by
 * (device, N, S, O, precision, job count, total visibilities rounded down to a
 * power of two): a later call with the same key applies the cached pair without
 * timing (out[] is then not written).  The grid-tile edge is not a search
 * dimension: 17 - S is the largest tile whose footprints fit one 16-cell MFMA
 * region, and smaller tiles only add padding for the same matrix work.
 * Synchronous.  Errors: as sepw_grid_batched, and those of
 * sepw_plan_set_item_slots. */
int sepw_autotune_batched(int32_t njobs, const sepw_plan* plans, const sepw_c64* const* vis,
                          const float* const* weight, sepw_c64* const* out, void* hip_stream,
                          int32_t* item_slots, int32_t* blocks_per_cu);

/* Regenerate the tables of k for a new w range (same P), asynchronously on
 * the stream: the per-batch form of table generation when the w-planes span
 * the batch's own +/- max|w|.  Plans created for the old range become invalid:
 * sepw_grid / sepw_degrid on them return SEPW_ERR_ARG.  With a correction
 * table attached to FP32 kernels, factoring it into separable terms
 * synchronises the stream.
 * Errors: SEPW_ERR_ARG (null k, non-finite or empty range), SEPW_ERR_OOM,
 * SEPW_ERR_HIP. */
int sepw_kernels_set_wrange(sepw_kernels k, double w_lo, double w_hi, void* hip_stream);

/* Optional per-stage timing for benchmarking: while enabled, every kernel the
 * library launches is bracketed by HIP events recorded on its launch stream.
 * sepw_timing_collect waits for the recorded events, adds their durations per
 * stage into ms[SEPW_NSTAGES] and launch counts into n[SEPW_NSTAGES] (both
 * host arrays, zeroed first), and forgets them. */
enum {
  SEPW_STAGE_TABLES = 0,   /* GCF table generation                  */
  SEPW_STAGE_QUANTISE,     /* quantise + histogram                  */
  SEPW_STAGE_SORT,         /* scans + scatter + work items          */
  SEPW_STAGE_GATHER,       /* W V (and facet rotation) to bin order */
  SEPW_STAGE_GRID,         /* gridding kernel                       */
  SEPW_STAGE_FFT,          /* hipFFT (both directions)              */
  SEPW_STAGE_CORRECT,      /* taper / n correction, both directions */
  SEPW_STAGE_DEGRID,       /* degridding kernel                     */
  SEPW_STAGE_FILL,         /* zero fills of outputs                 */
  SEPW_STAGE_CORR_TABLE,   /* correction table generation           */
  SEPW_STAGE_CORR_APPLY,   /* correction passes of grid / degrid    */
  SEPW_NSTAGES
};
int sepw_timing_enable(int32_t on);
int sepw_timing_collect(double* ms, int64_t* n);

int sepw_free_kernels(sepw_kernels k);
int sepw_free_plan(sepw_plan p);
int sepw_free_wstack(sepw_wstack ws);

/* W snapshots (Section 4.2).  The caller's visibilities form n_snap snapshots,
 * contiguous in caller order: snapshot s is [offsets[s], offsets[s + 1])
 * (offsets: HOST int64 [n_snap + 1], offsets[0] = 0, non-decreasing; empty
 * snapshots allowed; u, v, w: DEVICE float64 [offsets[n_snap]] in
 * wavelengths).  Per snapshot the plane w ~ d_u u + d_v v is fitted by least
 * squares through the origin over its visibilities with finite u, v, w (by
 * Cramer's rule on Suu, Suv, Svv, Suw, Svw; d0 = 0 unless det > 1e-12 Suu Svv),
 * and the snapshot is binned on its residual w' = w - (d_u u + d_v v) into the
 * P planes of k, whose w range create sets to [-h, h], h = max |w'| (1 + 2^-20)
 * (1 if every w' is 0; k's tables are regenerated, so plans made earlier from
 * k become invalid).  Synchronises the stream.  The object holds, besides a
 * plan per snapshot, as many N x N complex64 snapshot images as fit in 4 GiB
 * (at least one, at most n_snap): sepw_wsnap_grid grids that many snapshots
 * in one batched launch (sepw_grid_batched) and, in FP32, degrids them
 * likewise.
 * sepw_wsnap_grid: image_out (DEVICE complex64 [N N]) = sum over snapshots of
 *   R_s[F+[G_s] / (c1 c1)], times n (SEPW_MUL_N) or over n (SEPW_DIV_N), where
 *   G_s is the snapshot's separable gridding on w' and R_s the reprojection:
 *   output pixel l takes the snapshot image at l^s = l + d0 (n(l) - 1),
 *   sampled at pixel x = l^s N / fov + N/2 (y alike) by separable cubic
 *   convolution (Keys, a = -1/2) over the 4 x 4 nearest pixels, pixels off the
 *   image counting 0.
 * sepw_wsnap_degrid: its adjoint: per snapshot the transposed reprojection of
 *   image (times 1/n with SEPW_DIV_N), then separable degridding on w' into
 *   vis_out (DEVICE complex64 [nvis], caller order).
 * sepw_wsnap_plane: d0 (host double[2]) of a snapshot and h (host, may be NULL).
 * Errors: SEPW_ERR_ARG (null pointers, n_snap outside [1, 2^20], offsets not
 * starting at 0 or decreasing, more than 2^31 - 2 visibilities, flags other
 * than the n flags (grid) or SEPW_DIV_N (degrid)), SEPW_ERR_UNSUPPORTED (facet
 * kernels), SEPW_ERR_NO_DEVICE, SEPW_ERR_OOM, SEPW_ERR_HIP, SEPW_ERR_FFT. */
int sepw_wsnap_create(sepw_kernels k, int32_t n_snap, const int64_t* offsets, const double* u,
                      const double* v, const double* w, int64_t* n_dropped, void* hip_stream,
                      sepw_wsnap* out);
int sepw_wsnap_grid(sepw_wsnap ws, const sepw_c64* vis, const float* weight, sepw_c64* image_out,
                    uint32_t flags, void* hip_stream);
int sepw_wsnap_degrid(sepw_wsnap ws, const sepw_c64* image, sepw_c64* vis_out, uint32_t flags,
                      void* hip_stream);
int sepw_wsnap_plane(sepw_wsnap ws, int32_t snapshot, double* d0, double* h);
int sepw_free_wsnap(sepw_wsnap ws);
const char* sepw_strerror(int code);
int32_t sepw_device_count(void);   /* 0 when no HIP device is visible */

#ifdef __cplusplus
}
#endif
#endif /* SEPW_H */
