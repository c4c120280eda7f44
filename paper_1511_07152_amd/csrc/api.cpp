// C ABI of the separable W-projection library (include/sepw.h).
//
// Host-side orchestration only: argument validation (always before any device
// work), allocation of tables and plans, and the launch sequence of the
// kernels in tables.hip, binning.hip, grid.hip, degrid.hip and correct.hip.
// The FFT between grid and image is a hipFFT library call.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

using namespace sepw;

struct sepw_kernels_s : Kernels {};
struct sepw_plan_s : Plan {};

// W-stacking hybrid (Section 4.3): one plan per non-empty w-slice over the
// slice's residual w, the visibilities in slice order, and one image buffer.
struct sepw_wstack_s {
  Kernels* K = nullptr;
  int ns = 0;
  int64_t nvis = 0;
  std::vector<double> centre;    // slice centres w_s
  std::vector<int64_t> off;      // [ns + 1] slice offsets in slice order
  std::vector<Plan*> plans;      // [ns], null for empty slices
  std::vector<Kernels*> kern;    // non-uniform slices: tables per slice on its own residual range
  uint32_t* order = nullptr;     // [nvis] slice-ordered position -> caller index
  float2* vis = nullptr;         // [nvis] slice-ordered W V (gridding) or results (degridding)
  float2* img = nullptr;         // [nimg N N] slice images (gridded or degridded nimg at a time)
  int nimg = 1;
};

// W snapshots (Section 4.2): per snapshot (a contiguous range of the caller's
// visibilities) its fitted plane d0 and a plan over its residual w.
struct sepw_wsnap_s {
  Kernels* K = nullptr;
  int ns = 0;
  int64_t nvis = 0;
  std::vector<int64_t> off;      // [ns + 1]
  std::vector<double> d0;        // [2 ns]
  std::vector<Plan*> plans;      // [ns], null for empty snapshots
  double h = 0.0;                // residual w range [-h, h]
  float2* img = nullptr;         // [nimg N N] snapshot images (gridded nimg at a time)
  int nimg = 1;
};

namespace {

void release_batch(BatchScratch& b);

// Error code for a failed runtime call.  Also clears the thread's last-error
// state, which a failed call (an allocation, say) leaves set: the next kernel
// launch checks it and would otherwise report this failure again.
int map_hip(hipError_t e) {
  if (e == hipSuccess) return SEPW_OK;
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SEPW_ERR_OOM;
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return SEPW_ERR_NO_DEVICE;
  return SEPW_ERR_HIP;
}

#define SEPW_TRY(expr)                  \
  do {                                  \
    hipError_t e_ = (expr);             \
    if (e_ != hipSuccess) return map_hip(e_); \
  } while (0)

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// ---- optional per-stage timing (benchmarking aid) ----
struct TimingRec {
  int stage;
  hipEvent_t a, b;
};
std::mutex g_tmx;
bool g_timing = false;
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t pool_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one stage's launches on stream s with HIP events when timing is on.
class Stage {
 public:
  Stage(int stage, hipStream_t s) : stage_(stage), s_(s) {
    std::lock_guard<std::mutex> lk(g_tmx);
    if (!g_timing) return;
    a_ = pool_event();
    b_ = pool_event();
    if (a_ && b_) (void)hipEventRecord(a_, s_);
  }
  ~Stage() {
    std::lock_guard<std::mutex> lk(g_tmx);
    if (!a_ || !b_) return;
    (void)hipEventRecord(b_, s_);
    g_recs.push_back({stage_, a_, b_});
  }

 private:
  int stage_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

int device_count() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

template <typename T>
hipError_t dalloc(T** p, int64_t n) {
  if (n < 1) n = 1;
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)n);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

int validate_params(const sepw_kernel_params* p) {
  if (!p) return SEPW_ERR_ARG;
  if (p->grid_size < 2 || p->grid_size % 2 != 0 || p->grid_size > 32768) return SEPW_ERR_ARG;
  if (p->support < 1 || p->support % 2 == 0 || p->support > p->grid_size - 1) return SEPW_ERR_ARG;
  if (!is_pow2(p->oversample) || p->oversample > 128) return SEPW_ERR_ARG;
  if (p->n_planes < 1 || p->n_planes > 65535) return SEPW_ERR_ARG;
  if (!std::isfinite(p->fov) || p->fov <= 0.0 || p->fov >= std::sqrt(2.0)) return SEPW_ERR_ARG;
  if (!std::isfinite(p->w_lo) || !std::isfinite(p->w_hi) || !(p->w_lo < p->w_hi)) return SEPW_ERR_ARG;
  if (p->taper < SEPW_TAPER_PSWF || p->taper > SEPW_TAPER_USER) return SEPW_ERR_ARG;
  if (p->taper == SEPW_TAPER_PSWF && !std::isfinite(p->taper_width)) return SEPW_ERR_ARG;
  if (p->taper == SEPW_TAPER_USER) {
    if (!p->taper_samples) return SEPW_ERR_ARG;
    for (int i = 0; i < p->grid_size; ++i)
      if (!std::isfinite(p->taper_samples[i]) || p->taper_samples[i] <= 0.0) return SEPW_ERR_ARG;
  }
  if (p->precision < SEPW_FP32 || p->precision > SEPW_BF16) return SEPW_ERR_ARG;
  if (p->facet) {
    if (!std::isfinite(p->l0) || !std::isfinite(p->m0)) return SEPW_ERR_ARG;
    if (p->l0 * p->l0 + p->m0 * p->m0 >= 1.0) return SEPW_ERR_ARG;
  } else {
    if (!std::isfinite(p->a_u) || !std::isfinite(p->b_u) || !std::isfinite(p->a_v) ||
        !std::isfinite(p->b_v))
      return SEPW_ERR_ARG;
  }
  // above the MFMA region only the FP32 per-visibility path exists
  if (p->support > kMaxWideSupport) return SEPW_ERR_UNSUPPORTED;
  if (wide_support(p->support) && p->precision != SEPW_FP32) return SEPW_ERR_UNSUPPORTED;
  return SEPW_OK;
}

void free_corr_terms(Kernels* K);

void destroy_kernels(Kernels* k) {
  if (!k) return;
  if (k->tab_v && k->tab_v != k->tab_u) dfree(k->tab_v);
  k->tab_v = nullptr;
  dfree(k->tab_u);
  dfree(k->c1);
  if (!k->borrowed) {
    dfree(k->scratch);
    dfree(k->g16);
  }
  if (k->pad_v && k->pad_v != k->pad_u) dfree(k->pad_v);
  k->pad_v = nullptr;
  dfree(k->pad_u);
  if (k->pad_sv && k->pad_sv != k->pad_su) dfree(k->pad_sv);
  k->pad_sv = nullptr;
  dfree(k->pad_su);
  if (k->lp_v && k->lp_v != k->lp_u) dfree(k->lp_v);
  k->lp_v = nullptr;
  dfree(k->lp_u);
  dfree(k->corr);
  dfree(k->corr_tmp);
  free_corr_terms(k);
  if (k->fft_ok && !k->borrowed) hipfftDestroy(k->fft);
  delete static_cast<sepw_kernels_s*>(k);
}

void destroy_plan(Plan* p) {
  if (!p) return;
  dfree(p->rbin);
  dfree(p->qrec);
  dfree(p->rowcount);
  dfree(p->rowoff);
  dfree(p->chist);
  dfree(p->gsum);
  dfree(p->delta);
  dfree(p->ckept);
  dfree(p->rowpad);
  dfree(p->prowoff);
  dfree(p->binperm);
  dfree(p->rrec);
  dfree(p->place);
  dfree(p->yrow);
  dfree(p->krec);
  dfree(p->tdesc);
  dfree(p->rot);
  for (WorkList* l : {&p->gl, &p->dl}) {
    dfree(l->nit);
    dfree(l->itoff);
    dfree(l->items);
  }
  dfree(p->qctr);
  dfree(p->lp_max);
  dfree(p->scan_tmp);
  if (p->batch) {
    release_batch(*p->batch);
    delete p->batch;
  }
  delete static_cast<sepw_plan_s*>(p);
}

QuantGeom make_geom(const Kernels* K, int tile_c, int ntx) {
  QuantGeom g;
  g.fov = K->fov;
  g.half_n = (double)(K->N / 2);
  g.over = (double)K->O;
  g.w_lo = K->w_lo;
  g.inv_dw = K->inv_dw;
  g.N = K->N;
  g.S = K->S;
  g.O = K->O;
  g.lo = 0;
  while ((1 << g.lo) < K->O) ++g.lo;
  g.P = K->P;
  g.tile_c = tile_c;
  g.ntx = ntx;
  g.facet = K->facet ? 1 : 0;
  g.l0 = K->l0;
  g.m0 = K->m0;
  g.n0 = K->n0;
  return g;
}

int fft_exec(Kernels* K, float2* data, int direction, hipStream_t s) {
  if (hipfftSetStream(K->fft, s) != HIPFFT_SUCCESS) return SEPW_ERR_FFT;
  if (hipfftExecC2C(K->fft, reinterpret_cast<hipfftComplex*>(data),
                    reinterpret_cast<hipfftComplex*>(data), direction) != HIPFFT_SUCCESS)
    return SEPW_ERR_FFT;
  return SEPW_OK;
}

hipError_t make_separable_tables(Kernels* K, hipStream_t s) {
  Stage st(SEPW_STAGE_TABLES, s);
  hipError_t e = launch_tables(K->c1, K->N, K->fov, K->P, K->O, K->S, K->w_lo, K->w_hi, K->a_u,
                               K->b_u, K->tab_u, s);
  if (e == hipSuccess && K->tab_v != K->tab_u)
    e = launch_tables(K->c1, K->N, K->fov, K->P, K->O, K->S, K->w_lo, K->w_hi, K->a_v, K->b_v,
                      K->tab_v, s);
  // kernel-side layouts of the tiled path: zero-padded rows (and the
  // precision form's 16-bit tables); the per-visibility path reads the raw tables
  if (wide_support(K->S)) return e;
  if (e == hipSuccess) e = launch_pad_table(K->tab_u, nullptr, K->P, K->O, K->S, K->pad_u, s);
  if (e == hipSuccess && K->pad_v != K->pad_u)
    e = launch_pad_table(K->tab_v, nullptr, K->P, K->O, K->S, K->pad_v, s);
  if (e == hipSuccess) e = launch_pad_table(K->tab_u, nullptr, K->P, K->O, K->S, K->pad_su, s, true);
  if (e == hipSuccess && K->pad_sv != K->pad_su)
    e = launch_pad_table(K->tab_v, nullptr, K->P, K->O, K->S, K->pad_sv, s, true);
  if (e == hipSuccess && K->lp_u) {
    const int bf16 = K->prm.precision == SEPW_BF16 ? 1 : 0;
    e = launch_lp_table(K->tab_u, K->P, K->O, K->S, bf16, K->tab_len, K->lp_u, s);
    if (e == hipSuccess && K->lp_v != K->lp_u)
      e = launch_lp_table(K->tab_v, K->P, K->O, K->S, bf16, K->tab_len, K->lp_v, s);
  }
  return e;
}

void free_corr_terms(Kernels* K) {
  for (int r = 0; r < kMaxCorrRank; ++r) {
    if (K->ck_v[r] == K->ck_u[r]) K->ck_v[r] = nullptr;
    if (K->ck_sv[r] == K->ck_su[r]) K->ck_sv[r] = nullptr;
    dfree(K->ck_u[r]);
    dfree(K->ck_v[r]);
    dfree(K->ck_su[r]);
    dfree(K->ck_sv[r]);
  }
  K->corr_rank = -1;
  K->ck_lds = 0;
}

// Correction tables of the FP32 tiled path as separable terms (at most
// kMaxCorrRank, every residual entry within 1e-6 of the table's largest): the
// table comes to the host (the stream is synchronised), and the terms' padded
// tables go back.  Otherwise corr_rank stays -1 and the correction passes
// walk the table.
hipError_t factor_corr(Kernels* K, hipStream_t s) {
  K->corr_rank = -1;
  if (!K->corr_terms || K->prm.precision != SEPW_FP32 || wide_support(K->S)) return hipSuccess;
  const int64_t nC = (int64_t)K->P * K->corr_O * K->corr_O * K->corr_S * K->corr_S;
  if (nC > ((int64_t)1 << 24)) return hipSuccess;   // host copy above 128 MiB: keep the passes
  std::vector<float2> C((size_t)nC);
  hipError_t e = hipMemcpyAsync(C.data(), K->corr, sizeof(float2) * nC, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  std::vector<float2> tu, tv;
  bool shared = false;
  const int rank = factor_corr_table(C.data(), K->P, K->O, K->S, K->corr_O, K->corr_S,
                                     kMaxCorrRank, 1e-6, &tu, &tv, &shared);
  if (rank < 0) return hipSuccess;
  // the tables of earlier terms are rewritten in place (stream order); a
  // shared u / v table and a separate pair are not interchangeable
  for (int r = 0; r < kMaxCorrRank; ++r)
    if (K->ck_u[r] && (K->ck_v[r] == K->ck_u[r]) != shared) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      free_corr_terms(K);
      break;
    }
  const int64_t one = (int64_t)K->P * K->O * K->S;
  float2* dev = nullptr;
  if (rank > 0) e = dalloc(&dev, 2 * rank * one);
  for (int r = 0; r < rank && e == hipSuccess; ++r) {
    float2* du = dev + (int64_t)r * one;
    float2* dv = dev + (int64_t)(rank + r) * one;
    e = hipMemcpyAsync(du, tu.data() + (size_t)r * one, sizeof(float2) * one, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !shared)
      e = hipMemcpyAsync(dv, tv.data() + (size_t)r * one, sizeof(float2) * one, hipMemcpyHostToDevice, s);
    float2** dst[4] = {&K->ck_u[r], &K->ck_su[r], &K->ck_v[r], &K->ck_sv[r]};
    for (int t = 0; t < (shared ? 2 : 4) && e == hipSuccess; ++t)
      if (!*dst[t]) e = dalloc(dst[t], (int64_t)K->tab_len);
    if (shared) {
      K->ck_v[r] = K->ck_u[r];
      K->ck_sv[r] = K->ck_su[r];
    }
    if (e == hipSuccess) e = launch_pad_table(du, nullptr, K->P, K->O, K->S, K->ck_u[r], s);
    if (e == hipSuccess) e = launch_pad_table(du, nullptr, K->P, K->O, K->S, K->ck_su[r], s, true);
    if (e == hipSuccess && !shared) e = launch_pad_table(dv, nullptr, K->P, K->O, K->S, K->ck_v[r], s);
    if (e == hipSuccess && !shared)
      e = launch_pad_table(dv, nullptr, K->P, K->O, K->S, K->ck_sv[r], s, true);
  }
  // the host tables must outlive the copies
  if (dev) {
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    dfree(dev);
  }
  if (e != hipSuccess) return e;
  const int64_t bytes = (int64_t)sizeof(float2) * (shared ? 1 : 2) * K->tab_len;
  K->ck_lds = bytes <= (int64_t)K->lds_max ? (int)bytes : 0;
  K->corr_rank = rank;
  return hipSuccess;
}

hipError_t make_corr_table(Kernels* K, hipStream_t s) {
  if (!K->corr) return hipSuccess;
  Stage st(SEPW_STAGE_CORR_TABLE, s);
  hipError_t e = launch_corr_tables(K->c1, K->N, K->fov, K->P, K->w_lo, K->w_hi, K->a_u, K->b_u,
                                    K->a_v, K->b_v, K->corr_S, K->corr_O, K->corr_nkb,
                                    K->corr_tmp, K->corr, s);
  if (e == hipSuccess) e = factor_corr(K, s);
  return e;
}

// every table of the kernel set for its current w range
hipError_t make_tables(Kernels* K, hipStream_t s) {
  hipError_t e = make_separable_tables(K, s);
  if (e == hipSuccess) e = make_corr_table(K, s);
  return e;
}

int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

// Correction pass over one plan's work list (the correction table must exist).
CorrArgs corr_args(const Plan* p, const WorkList& l, float2* grid, int checker) {
  const Kernels* K = p->K;
  CorrArgs a;
  a.items = l.items;
  a.nitems = l.itoff + 8 * p->r8;
  a.tdesc = p->tdesc;
  a.krec = p->krec;
  a.yrow = p->yrow;
  a.tab = K->corr;
  a.g.O = K->O;
  a.g.lo = ilog2(K->O);
  a.g.Oc = K->corr_O;
  a.g.lr = ilog2(K->O / K->corr_O);
  a.g.Sc = K->corr_S;
  a.g.hc = K->corr_S / 2;
  a.g.T2 = K->corr_S * K->corr_S;
  // footprints about cell or (1 < Oc < O) cell + 1 of the tile's C cells
  const bool may_move = K->corr_O != K->O && K->corr_O != 1;
  a.g.win = (kRegion + 1 - K->S) + K->corr_S - (may_move ? 0 : 1);
  a.N = K->N;
  a.ntx = p->ntx;
  a.checker = checker;
  a.grid = grid;
  return a;
}

// The correction beside a plan's separable pass (nothing without a table):
// factored, the separable kernels once per term with the term's tables
// (gridding adds into the grid; degridding adds into the results the
// separable pass left in row-bin order); otherwise the passes that walk the
// table itself.
int corr_grid_pass(Plan* p, float2* grid, int checker, hipStream_t s) {
  const Kernels* K = p->K;
  if (!K->corr) return SEPW_OK;
  Stage st(SEPW_STAGE_CORR_APPLY, s);
  if (K->corr_rank < 0) {
    SEPW_TRY(launch_corr_grid(K->S, corr_args(p, p->gl, grid, checker), p->gl.max_items, s));
    return SEPW_OK;
  }
  for (int r = 0; r < K->corr_rank; ++r) {
    GridArgs a{p->gl.items, p->gl.itoff + 8 * p->r8, p->gl.itoff, p->r8, p->qctr, p->tdesc, p->krec,
               p->yrow, K->ck_u[r], K->ck_v[r], K->tab_len, K->N, p->ntx, checker, grid};
    if (K->ck_lds > 0) {
      SEPW_TRY(launch_fill_u32(p->qctr, 0u, 8 * kCtrStride, s));
      SEPW_TRY(launch_grid_fp32_lds(K->S, a, K->ck_lds, K->n_cu, s));
    } else {
      SEPW_TRY(launch_grid_fp32(K->S, a, p->gl.max_items, s));
    }
  }
  return SEPW_OK;
}

int corr_degrid_pass(Plan* p, const float2* grid, int checker, hipStream_t s) {
  const Kernels* K = p->K;
  if (!K->corr) return SEPW_OK;
  Stage st(SEPW_STAGE_CORR_APPLY, s);
  if (K->corr_rank < 0) {
    SEPW_TRY(launch_corr_degrid(K->S, corr_args(p, p->dl, const_cast<float2*>(grid), checker),
                                p->dl.max_items, s));
    return SEPW_OK;
  }
  for (int r = 0; r < K->corr_rank; ++r) {
    DegridArgs a{p->dl.items, p->dl.itoff + 8 * p->r8, p->dl.itoff, p->r8, p->qctr, p->tdesc, p->krec,
                 grid, checker ? K->ck_su[r] : K->ck_u[r], checker ? K->ck_sv[r] : K->ck_v[r],
                 K->tab_len, K->N, p->ntx, checker, p->yrow, 1};
    SEPW_TRY(launch_fill_u32(p->qctr, 0u, 8 * kCtrStride, s));
    SEPW_TRY(launch_degrid_fp32(K->S, a, p->dl.max_items, K->ck_lds, K->n_cu, s));
  }
  return SEPW_OK;
}

// share: null, or a kernels object with the same N, fov and taper whose taper
// samples are copied and whose FFT plan and work grid are used, not made (the
// tables of W-stacking slices; share outlives K).
int build_kernels(const sepw_kernel_params* p, hipStream_t s, Kernels* K,
                  const Kernels* share = nullptr) {
  K->prm = *p;
  K->prm.taper_samples = nullptr;
  K->N = p->grid_size;
  K->S = p->support;
  K->O = p->oversample;
  K->P = p->n_planes;
  K->fov = p->fov;
  K->w_lo = p->w_lo;
  K->w_hi = p->w_hi;
  K->inv_dw = (double)p->n_planes / (p->w_hi - p->w_lo);
  K->facet = p->facet != 0;
  K->l0 = K->facet ? p->l0 : 0.0;
  K->m0 = K->facet ? p->m0 : 0.0;
  K->n0 = std::sqrt(1.0 - K->l0 * K->l0 - K->m0 * K->m0);
  if (K->facet) {
    // Section 4.1: second-order Taylor terms of h(l0 + l) about the facet centre
    const double n0 = K->n0, n03 = n0 * n0 * n0;
    K->a_u = 0.5 * (1.0 / n0 + K->l0 * K->l0 / n03);
    K->a_v = 0.5 * (1.0 / n0 + K->m0 * K->m0 / n03);
    K->b_u = K->b_v = 0.0;
  } else {
    K->a_u = p->a_u;
    K->b_u = p->b_u;
    K->a_v = p->a_v;
    K->b_v = p->b_v;
  }
  K->taper_width = p->taper_width > 0.0 ? p->taper_width : (double)p->support;

  const int N = K->N;
  SEPW_TRY(dalloc(&K->c1, N));
  if (share) {
    SEPW_TRY(hipMemcpyAsync(K->c1, share->c1, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  } else if (p->taper == SEPW_TAPER_NONE) {
    SEPW_TRY(launch_ones(K->c1, N, s));
  } else if (p->taper == SEPW_TAPER_USER) {
    SEPW_TRY(hipMemcpyAsync(K->c1, p->taper_samples, sizeof(double) * N, hipMemcpyHostToDevice, s));
    SEPW_TRY(hipStreamSynchronize(s));
  } else {
    const int max_terms = 4096;
    std::vector<double> coef(max_terms);
    double psi0 = 0.0;
    const double c = M_PI * K->taper_width / 2.0;
    int m = pswf_coefficients(c, coef.data(), max_terms, &psi0);
    double* dcoef = nullptr;
    SEPW_TRY(dalloc(&dcoef, m));
    hipError_t e = hipMemcpyAsync(dcoef, coef.data(), sizeof(double) * m, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_taper(dcoef, m, psi0, N, K->c1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dcoef);
    SEPW_TRY(e);
  }
  const int64_t ntab = (int64_t)K->P * K->O * K->S;
  SEPW_TRY(dalloc(&K->tab_u, ntab));
  const bool shared_axes = K->a_v == K->a_u && K->b_v == K->b_u;
  if (shared_axes) {
    K->tab_v = K->tab_u;
  } else {
    SEPW_TRY(dalloc(&K->tab_v, ntab));
  }
  const int64_t npad = (int64_t)K->P * K->O * padded_len(K->S);
  SEPW_TRY(dalloc(&K->pad_u, npad));
  SEPW_TRY(dalloc(&K->pad_su, npad));
  if (shared_axes) {
    K->pad_v = K->pad_u;
    K->pad_sv = K->pad_su;
  } else {
    SEPW_TRY(dalloc(&K->pad_v, npad));
    SEPW_TRY(dalloc(&K->pad_sv, npad));
  }
  // the 16-bit tables: (Re, Im) dwords, BF16 high then low parts
  const int64_t nlp = npad * (p->precision == SEPW_BF16 ? 2 : 1);
  K->tab_len = (int)npad;
  if (p->precision != SEPW_FP32) {
    SEPW_TRY(dalloc(&K->lp_u, nlp));
    if (shared_axes) {
      K->lp_v = K->lp_u;
    } else {
      SEPW_TRY(dalloc(&K->lp_v, nlp));
    }
  }
  SEPW_TRY(make_tables(K, s));
  if (share) {
    K->scratch = share->scratch;
    K->g16 = share->g16;
    K->borrowed = true;
  } else {
    SEPW_TRY(dalloc(&K->scratch, (int64_t)N * N));
    if (p->precision != SEPW_FP32 && !wide_support(K->S)) {
      // the 16-bit degridding operand grid (BF16: two planes); its border stays zero
      const int64_t pitch = N + 2 * kG16Border;
      const int64_t n = pitch * pitch * (p->precision == SEPW_BF16 ? 2 : 1);
      SEPW_TRY(dalloc(&K->g16, n));
      SEPW_TRY(launch_fill_u32(K->g16, 0u, n, s));
    }
  }
  // stage the FP32 tables in LDS when both fit in one workgroup's share
  {
    int dev = 0, max_lds = 0, ncu = 0;
    SEPW_TRY(hipGetDevice(&dev));
    SEPW_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    SEPW_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t bytes = (int64_t)sizeof(float2) * npad * (shared_axes ? 1 : 2);
    K->n_cu = ncu > 0 ? ncu : 1;
    K->lds_max = max_lds;
    K->lds_bytes = bytes <= (int64_t)max_lds ? (int)bytes : 0;
    const int64_t lp_bytes = (int64_t)sizeof(uint32_t) * nlp * (shared_axes ? 1 : 2);
    K->lds_bytes_lp = lp_bytes <= (int64_t)max_lds ? (int)lp_bytes : 0;
  }
  if (share) {
    K->fft = share->fft;
  } else if (hipfftPlan2d(&K->fft, N, N, HIPFFT_C2C) != HIPFFT_SUCCESS) {
    return SEPW_ERR_FFT;
  }
  K->fft_ok = true;
  return SEPW_OK;
}

int alloc_plan(Kernels* K, int64_t capacity, Plan* P) {
  P->K = K;
  P->capacity = capacity;
  P->tile_c = (wide_support(K->S) ? kWideRegion : kRegion) + 1 - K->S;
  P->ntx = (K->N + P->tile_c - 1) / P->tile_c;
  P->nty = P->ntx;
  P->ntiles = (int64_t)P->ntx * P->nty;
  const int64_t nt = P->ntiles;
  // level-1 row bins: group 2^rshift tile rows so that there are at most
  // kMaxRowBins bins and each bin's tiles fit the level-2 LDS histogram
  // (about 512 bins keeps the level-1 placement runs long enough to coalesce)
  auto bins_for = [&](int r) { return (P->nty + (1 << r) - 1) >> r; };
  P->rshift = 0;
  while (bins_for(P->rshift) > kTargetRowBins) P->rshift += 1;
  while (P->rshift > 0 && ((int64_t)P->ntx << P->rshift) > kMaxRowTiles) P->rshift -= 1;
  P->nbins = bins_for(P->rshift);
  if (P->nbins > kMaxRowBins || ((int64_t)P->ntx << P->rshift) > kMaxRowTiles)
    return SEPW_ERR_UNSUPPORTED;
  // tile slots: every visibility plus room to pad each non-empty tile to a
  // multiple of 4, each row bin's range rounded to 4
  P->pcap = capacity + 3 * std::min<int64_t>(nt, capacity) + 4 * (int64_t)P->nbins;
  if (P->pcap > 2147483647LL - 64) return SEPW_ERR_UNSUPPORTED;
  P->gl.slots = kItemMaxVis;
  P->dl.slots = kDegridItemSlots;
  P->r8 = (P->nty + 7) / 8;
  P->scan_tmp_len = scan_tmp_size(std::max<int64_t>(P->nbins, 8 * (int64_t)P->r8) + 1);
  SEPW_TRY(dalloc(&P->rbin, capacity));
  SEPW_TRY(dalloc(&P->qrec, capacity));
  SEPW_TRY(dalloc(&P->rowcount, P->nbins + 1));
  SEPW_TRY(dalloc(&P->rowoff, P->nbins + 1));
  const int64_t nch = (capacity + kL1Chunk - 1) / kL1Chunk;
  const int64_t ngroups = (nch + kGroupChunks - 1) / kGroupChunks;
  SEPW_TRY(dalloc(&P->chist, std::max<int64_t>(nch, 1) * P->nbins));
  SEPW_TRY(dalloc(&P->gsum, std::max<int64_t>(ngroups, 1) * P->nbins));
  SEPW_TRY(dalloc(&P->delta, std::max<int64_t>(nch, 1) * P->nbins));
  SEPW_TRY(dalloc(&P->ckept, std::max<int64_t>(nch, 1)));
  SEPW_TRY(dalloc(&P->rowpad, P->nbins + 1));
  SEPW_TRY(dalloc(&P->prowoff, P->nbins + 1));
  SEPW_TRY(dalloc(&P->binperm, P->nbins));
  SEPW_TRY(dalloc(&P->rrec, capacity));
  SEPW_TRY(dalloc(&P->place, capacity));
  SEPW_TRY(dalloc(&P->yrow, capacity + 1));
  SEPW_TRY(dalloc(&P->krec, P->pcap));
  SEPW_TRY(dalloc(&P->tdesc, nt));
  for (WorkList* l : {&P->gl, &P->dl}) {
    l->max_items = P->nty + P->pcap / l->slots + 1;
    SEPW_TRY(dalloc(&l->nit, 8 * (int64_t)P->r8 + 1));
    SEPW_TRY(dalloc(&l->itoff, 8 * (int64_t)P->r8 + 1));
    SEPW_TRY(dalloc(&l->items, l->max_items));
  }
  SEPW_TRY(dalloc(&P->qctr, 8 * kCtrStride));
  SEPW_TRY(dalloc(&P->lp_max, 2));
  SEPW_TRY(dalloc(&P->scan_tmp, P->scan_tmp_len));
  if (K->facet) SEPW_TRY(dalloc(&P->rot, capacity));
  return SEPW_OK;
}

WideArgs wide_args(const Plan* p, int checker) {
  const Kernels* K = p->K;
  return WideArgs{p->qrec, p->rbin, K->tab_u, K->tab_v, p->rot, p->nvis, K->N, K->S, K->O, checker};
}

MoveArgs move_args(const Plan* p, const sepw_c64* vis, const float* weight) {
  MoveArgs m;
  m.vis = reinterpret_cast<const float2*>(vis);
  m.weight = weight;
  m.rot = p->rot;
  m.place = p->place;
  m.delta = p->delta;
  m.ckept = p->ckept;
  m.yrow = p->yrow;
  m.nvis = p->nvis;
  m.nbins = p->nbins;
  m.vmax = nullptr;
  return m;
}

// Work list: items of l.slots slots per row of tiles, in 8 lists by row % 8.
hipError_t build_list(Plan* P, WorkList& l, hipStream_t s) {
  hipError_t e = launch_item_counts(P->tdesc, P->ntx, P->nty, P->r8, l.slots, l.nit, s);
  if (e == hipSuccess) e = launch_scan(l.nit, l.itoff, 8 * (int64_t)P->r8 + 1, P->scan_tmp, s);
  if (e == hipSuccess)
    e = launch_items(P->tdesc, l.itoff, P->ntx, P->nty, P->r8, l.slots, l.items, s);
  return e;
}

hipError_t build_items(Plan* P, hipStream_t s) {
  hipError_t e = build_list(P, P->gl, s);
  if (e == hipSuccess) e = build_list(P, P->dl, s);
  return e;
}

// New length of one work list (the list grows when needed).
int set_list_slots(Plan* p, WorkList& l, int32_t slots, hipStream_t s) {
  if (slots < kItemMinSlots || slots > kItemMaxSlots || (slots & 3) != 0) return SEPW_ERR_ARG;
  const int64_t need = p->nty + p->pcap / slots + 1;
  if (need > l.max_items) {
    // the old list may still be read by queued launches on this stream
    SEPW_TRY(hipStreamSynchronize(s));
    int4* items = nullptr;
    SEPW_TRY(dalloc(&items, need));
    dfree(l.items);
    l.items = items;
    l.max_items = need;
  }
  l.slots = slots;
  if (!wide_support(p->K->S)) SEPW_TRY(build_list(p, l, s));   // no tiles on the per-visibility path
  return SEPW_OK;
}

// Quantise, sort and build the work list for nvis <= capacity visibilities.
Coords plain_coords(const double* u, const double* v, const double* w) {
  Coords c;
  c.u = u;
  c.v = v;
  c.w = w;
  return c;
}

int bin_plan(Plan* P, int64_t nvis, const Coords& src, hipStream_t s) {
  Kernels* K = P->K;
  P->nvis = nvis;
  const QuantGeom g = make_geom(K, P->tile_c, P->ntx);
  P->generation = K->generation;
  {
    Stage st(SEPW_STAGE_QUANTISE, s);
    SEPW_TRY(launch_quantise_rows(src, nvis, g, P->rshift, P->nbins, P->rbin, P->qrec, P->chist, s));
  }
  {
    Stage st(SEPW_STAGE_SORT, s);
    SEPW_TRY(launch_level1_counts(P->chist, nvis, P->nbins, P->gsum, P->rowcount, s));
    SEPW_TRY(launch_scan(P->rowcount, P->rowoff, P->nbins + 1, P->scan_tmp, s));
    SEPW_TRY(launch_chunk_deltas(P->chist, P->gsum, P->rowoff, nvis, P->nbins, P->delta, P->ckept,
                                 s));
    SEPW_TRY(launch_pad_sizes(P->rowcount, P->nbins, P->rshift, P->ntx, P->nty, P->rowpad, s));
    SEPW_TRY(launch_scan(P->rowpad, P->prowoff, P->nbins + 1, P->scan_tmp, s));
    SEPW_TRY(launch_row_scatter(P->rbin, P->qrec, nvis, P->nbins, P->chist, P->delta, P->rrec,
                                P->place, s));
    if (wide_support(K->S)) {
      // the per-visibility path reads the packed bins in caller order
      if (K->facet) SEPW_TRY(launch_rotation(src, nvis, g, P->rot, s));
      return SEPW_OK;
    }
    // padding slots point at yrow[capacity], which nothing writes: keep it 0
    SEPW_TRY(launch_zero_c64(P->yrow + P->capacity, 1, s));
    SEPW_TRY(launch_row_sort(P->rowcount, P->rowoff, P->prowoff, P->rrec, P->rshift, P->nbins,
                             P->ntx, P->nty, P->tile_c, K->O, K->S, (uint32_t)P->capacity,
                             P->binperm, P->tdesc, P->krec, s));
    SEPW_TRY(build_items(P, s));
    if (K->facet) SEPW_TRY(launch_rotation(src, nvis, g, P->rot, s));
  }
  return SEPW_OK;
}

int read_dropped(Plan* P, int64_t* n_dropped, hipStream_t s) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, n_dropped) == hipSuccess && at.type == hipMemoryTypeDevice) {
    // device memory: written on the stream, no synchronisation
    SEPW_TRY(launch_dropped(P->rowoff + P->nbins, P->nvis, n_dropped, s));
    return SEPW_OK;
  }
  (void)hipGetLastError();   // a host pointer unknown to the runtime reports an error
  uint32_t kept = 0;
  hipError_t e = hipMemcpyAsync(&kept, P->rowoff + P->nbins, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return map_hip(e);
  *n_dropped = P->nvis - (int64_t)kept;
  return SEPW_OK;
}

}  // namespace

namespace sepw {
// Library-owned scratch of the batched launches: the job tables (pinned host
// copies and device copies), the per-job item prefix and the work counter.
// Each plan owns one, used by the batched calls it leads (as plans[0]), grown
// on demand; a new call waits until the previous call's job table has reached
// the device before overwriting it.  Calls led by different plans share
// nothing, so they may overlap on different streams.
struct BatchScratch {
  int cap = 0;
  int device = -1;
  int blocks = 0;
  GridArgs* host = nullptr;     // pinned
  GridArgs* jobs = nullptr;     // device
  MoveArgs* mhost = nullptr;    // pinned movement-pass job table
  MoveArgs* mjobs = nullptr;    // device
  uint32_t* mfirst_host = nullptr;  // pinned [cap + 1] first workgroup per job
  uint32_t* mfirst = nullptr;       // device
  DegridArgs* dhost = nullptr;  // pinned degridding job table
  DegridArgs* djobs = nullptr;  // device
  uint32_t* first = nullptr;    // device [cap + 1]
  uint32_t* counter = nullptr;  // device [8 kCtrStride]: the launch's work counters
  hipEvent_t copied = nullptr;
  int n_cu = 0;
};
}  // namespace sepw

namespace {

void release_batch(BatchScratch& b) {
  if (b.copied) (void)hipEventSynchronize(b.copied);
  if (b.host) (void)hipHostFree(b.host);
  if (b.mhost) (void)hipHostFree(b.mhost);
  if (b.mfirst_host) (void)hipHostFree(b.mfirst_host);
  if (b.dhost) (void)hipHostFree(b.dhost);
  dfree(b.djobs);
  dfree(b.jobs);
  dfree(b.mjobs);
  dfree(b.mfirst);
  dfree(b.first);
  dfree(b.counter);
  if (b.copied) (void)hipEventDestroy(b.copied);
  b = BatchScratch();
}

int batch_scratch(Plan* lead, int njobs, hipStream_t s, BatchScratch** out) {
  if (!lead->batch) lead->batch = new BatchScratch();
  BatchScratch& b = *lead->batch;
  int dev = 0;
  SEPW_TRY(hipGetDevice(&dev));
  if (b.copied) SEPW_TRY(hipEventSynchronize(b.copied));
  if (b.cap < njobs || b.device != dev) {
    release_batch(b);
    const int cap = njobs < 64 ? 64 : njobs;
    SEPW_TRY(hipHostMalloc(reinterpret_cast<void**>(&b.host), sizeof(GridArgs) * (size_t)cap));
    SEPW_TRY(hipHostMalloc(reinterpret_cast<void**>(&b.mhost), sizeof(MoveArgs) * (size_t)cap));
    SEPW_TRY(hipHostMalloc(reinterpret_cast<void**>(&b.mfirst_host),
                           sizeof(uint32_t) * (size_t)(cap + 1)));
    SEPW_TRY(hipHostMalloc(reinterpret_cast<void**>(&b.dhost), sizeof(DegridArgs) * (size_t)cap));
    SEPW_TRY(dalloc(&b.djobs, cap));
    SEPW_TRY(dalloc(&b.jobs, cap));
    SEPW_TRY(dalloc(&b.mjobs, cap));
    SEPW_TRY(dalloc(&b.mfirst, cap + 1));
    SEPW_TRY(dalloc(&b.first, cap + 1));
    SEPW_TRY(dalloc(&b.counter, 8 * kCtrStride));
    SEPW_TRY(hipEventCreateWithFlags(&b.copied, hipEventDisableTiming));
    hipDeviceProp_t prop;
    SEPW_TRY(hipGetDeviceProperties(&prop, dev));
    b.n_cu = prop.multiProcessorCount;
    b.cap = cap;
    b.device = dev;
  }
  (void)s;
  b.blocks = b.n_cu * lead->blocks_per_cu;
  *out = &b;
  return SEPW_OK;
}

// Degridding of nj FP32 plans (on kernels K, or on kernels of their own with
// K's N, S, taper and no correction table) from images held in
// grids (N x N each, consecutive): per plan the correction (times n^npow;
// skipped when the images come corrected) and the FFT in place, then the
// degridding launch(es) over the plans' items, then per plan the
// correction-table pass and the move of its results into vis[j] (its caller
// order).
int degrid_images_batched(Kernels* K, Plan* const* plans, int nj, float2* grids, int npow,
                          float2* const* vis, hipStream_t s, bool corrected = false) {
  const int N = K->N;
  for (int j = 0; j < nj; ++j) {
    float2* g = grids + (int64_t)j * N * N;
    if (!corrected) {
      Stage st(SEPW_STAGE_CORRECT, s);
      SEPW_TRY(launch_correct(g, g, K->c1, N, K->fov, K->l0, K->m0, npow, s));
    }
    Stage st(SEPW_STAGE_FFT, s);
    int rc = fft_exec(K, g, HIPFFT_FORWARD, s);
    if (rc != SEPW_OK) return rc;
  }
  bool shared = true;
  for (int j = 0; j < nj; ++j) shared = shared && plans[j]->K == K;
  if (!shared && K->lds_bytes > 0) {
    // jobs with tables of their own (non-uniform W-stacking slices): one
    // launch per job, each with its tables in LDS (measured faster than one
    // persistent launch reading every job's tables through the caches)
    Stage st(SEPW_STAGE_DEGRID, s);
    for (int j = 0; j < nj; ++j) {
      const Plan* p = plans[j];
      const DegridArgs a{p->dl.items, p->dl.itoff + 8 * p->r8, p->dl.itoff, p->r8, p->qctr,
                         p->tdesc, p->krec, grids + (int64_t)j * N * N, p->K->pad_su,
                         p->K->pad_sv, p->K->tab_len, N, p->ntx, 1, p->yrow};
      SEPW_TRY(launch_fill_u32(p->qctr, 0u, 8 * kCtrStride, s));
      SEPW_TRY(launch_degrid_fp32(K->S, a, p->dl.max_items, p->K->lds_bytes, K->n_cu, s));
    }
  } else {
  BatchScratch* bs = nullptr;
  int rc = batch_scratch(plans[0], nj, s, &bs);
  if (rc != SEPW_OK) return rc;
  // the tables stay in LDS when every job uses K's; otherwise (tables too
  // large for LDS) the jobs read them through the caches
  for (int j = 0; j < nj; ++j) {
    const Plan* p = plans[j];
    bs->dhost[j] = DegridArgs{p->dl.items, p->dl.itoff + 8 * p->r8, p->dl.itoff, p->r8, p->qctr,
                              p->tdesc, p->krec, grids + (int64_t)j * N * N, p->K->pad_su,
                              p->K->pad_sv, p->K->tab_len, N, p->ntx, 1, p->yrow};
  }
  SEPW_TRY(hipMemcpyAsync(bs->djobs, bs->dhost, sizeof(DegridArgs) * (size_t)nj,
                          hipMemcpyHostToDevice, s));
  SEPW_TRY(hipEventRecord(bs->copied, s));
  {
    Stage st(SEPW_STAGE_DEGRID, s);
    SEPW_TRY(launch_job_prefix(bs->djobs, nj, bs->first, bs->counter, s));
    SEPW_TRY(launch_degrid_fp32_batched(K->S, bs->djobs, bs->first, nj, bs->counter,
                                        shared ? K->lds_bytes : 0, K->n_cu, s));
  }
  }
  for (int j = 0; j < nj; ++j) {
    Plan* p = plans[j];
    int rc2 = corr_degrid_pass(p, grids + (int64_t)j * N * N, 1, s);
    if (rc2 != SEPW_OK) return rc2;
    Stage st(SEPW_STAGE_GATHER, s);
    SEPW_TRY(launch_vis_from_rows(p->yrow, p->rot, p->place, p->delta, p->ckept, p->nvis,
                                  p->nbins, vis[j], s));
  }
  return SEPW_OK;
}

// Images gridded or degridded in one batch by the multi-plan hybrids: as many
// N x N complex64 images as fit in kBatchImageBytes (at least 1, at most n).
constexpr int64_t kBatchImageBytes = 4ll << 30;
int batch_images(int N, int n) {
  const int64_t img_bytes = (int64_t)sizeof(float2) * N * N;
  return (int)std::max<int64_t>(1, std::min<int64_t>(n, kBatchImageBytes / img_bytes));
}

void destroy_wstack(sepw_wstack_s* W) {
  if (!W) return;
  for (Plan* p : W->plans) destroy_plan(p);
  for (Kernels* k : W->kern) destroy_kernels(k);
  dfree(W->order);
  dfree(W->vis);
  dfree(W->img);
  delete W;
}

// Partition into slices (count, offsets, scatter with residual w), one plan
// per non-empty slice.  Synchronises the stream (slice sizes come to the host).
// edges: null for uniform slices on [w_lo, w_hi], else ns + 1 increasing
// host values (slice s = [e_s, e_{s+1}), centre (e_s + e_{s+1}) / 2).
int wstack_build(sepw_wstack_s* W, Kernels* K, int ns, double w_lo, double w_hi,
                 const double* edges, int64_t nvis, const double* u, const double* v,
                 const double* w, int64_t* n_dropped, hipStream_t s) {
  W->K = K;
  W->ns = ns;
  W->nvis = nvis;
  W->centre.resize(ns);
  for (int j = 0; j < ns; ++j)
    W->centre[j] = edges ? (edges[j] + edges[j + 1]) * 0.5 : w_lo + ((j + 0.5) * (w_hi - w_lo)) / ns;
  const double inv_ds = (double)ns / (w_hi - w_lo);
  W->off.assign(ns + 1, 0);
  W->plans.assign(ns, nullptr);
  SEPW_TRY(dalloc(&W->order, std::max<int64_t>(nvis, 1)));
  SEPW_TRY(dalloc(&W->vis, std::max<int64_t>(nvis, 1)));
  W->nimg = batch_images(K->N, ns);
  SEPW_TRY(dalloc(&W->img, (int64_t)W->nimg * K->N * K->N));
  uint32_t* count = nullptr;
  double *cdev = nullptr, *edev = nullptr, *us = nullptr, *vs = nullptr, *wsr = nullptr;
  auto cleanup = [&]() {
    dfree(count);
    dfree(cdev);
    dfree(edev);
    dfree(us);
    dfree(vs);
    dfree(wsr);
  };
  auto run = [&]() -> int {
    SEPW_TRY(dalloc(&count, ns));
    SEPW_TRY(dalloc(&cdev, ns));
    SEPW_TRY(dalloc(&us, std::max<int64_t>(nvis, 1)));
    SEPW_TRY(dalloc(&vs, std::max<int64_t>(nvis, 1)));
    SEPW_TRY(dalloc(&wsr, std::max<int64_t>(nvis, 1)));
    if (edges) {
      SEPW_TRY(dalloc(&edev, ns + 1));
      SEPW_TRY(hipMemcpyAsync(edev, edges, sizeof(double) * (ns + 1), hipMemcpyHostToDevice, s));
    }
    SEPW_TRY(launch_fill_u32(count, 0u, ns, s));
    SEPW_TRY(launch_slice_count(w, nvis, w_lo, inv_ds, ns, edev, count, s));
    std::vector<uint32_t> hc(ns);
    SEPW_TRY(hipMemcpyAsync(hc.data(), count, sizeof(uint32_t) * ns, hipMemcpyDeviceToHost, s));
    SEPW_TRY(hipStreamSynchronize(s));
    std::vector<uint32_t> cur(ns);
    for (int j = 0; j < ns; ++j) {
      cur[j] = (uint32_t)W->off[j];
      W->off[j + 1] = W->off[j] + hc[j];
    }
    SEPW_TRY(hipMemcpyAsync(count, cur.data(), sizeof(uint32_t) * ns, hipMemcpyHostToDevice, s));
    SEPW_TRY(hipMemcpyAsync(cdev, W->centre.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
    SEPW_TRY(launch_slice_scatter(u, v, w, nvis, w_lo, inv_ds, ns, edev, cdev, count, W->order,
                                  us, vs, wsr, s));
    int64_t dropped = 0;
    for (int j = 0; j < ns; ++j) {
      const int64_t n = W->off[j + 1] - W->off[j];
      if (n == 0) continue;
      Kernels* KS = K;
      if (edges) {
        // the slice's own residual range [-h_s, h_s]: k's parameters with that w range
        sepw_kernels_s* k2 = new (std::nothrow) sepw_kernels_s();
        if (!k2) return SEPW_ERR_OOM;
        W->kern.push_back(k2);
        // (K's taper samples, FFT plan and work grid)
        sepw_kernel_params prm = K->prm;
        const double hs = (edges[j + 1] - edges[j]) * 0.5;
        prm.w_lo = -hs;
        prm.w_hi = hs;
        int rk = build_kernels(&prm, s, k2, K);
        if (rk != SEPW_OK) return rk;
        KS = k2;
      }
      sepw_plan_s* P = new (std::nothrow) sepw_plan_s();
      if (!P) return SEPW_ERR_OOM;
      W->plans[j] = P;
      int rc = alloc_plan(KS, n, P);
      if (rc == SEPW_OK) rc = bin_plan(P, n, plain_coords(us + W->off[j], vs + W->off[j], wsr + W->off[j]), s);
      if (rc == SEPW_OK && n_dropped) {
        int64_t d = 0;
        rc = read_dropped(P, &d, s);
        dropped += d;
      }
      if (rc != SEPW_OK) return rc;
    }
    if (n_dropped) *n_dropped = dropped;
    // the plans hold their own bins: the slice-ordered coordinates can go
    SEPW_TRY(hipStreamSynchronize(s));
    return SEPW_OK;
  };
  const int rc = run();
  cleanup();
  return rc;
}

void destroy_wsnap(sepw_wsnap_s* ws) {
  if (!ws) return;
  for (Plan* p : ws->plans) destroy_plan(p);
  dfree(ws->img);
  delete ws;
}

constexpr int64_t kSnapBlock = 65536;   // visibilities per block of the plane fit

// Fit the planes, form the residual w, set the kernels' range to it and bin
// each snapshot.
int wsnap_build(sepw_wsnap_s* W, const double* u, const double* v, const double* w, hipStream_t s) {
  Kernels* K = W->K;
  const int ns = W->ns;
  std::vector<int64_t> range;
  std::vector<int> snap, first(ns + 1, 0);
  for (int i = 0; i < ns; ++i) {
    first[i] = (int)snap.size();
    for (int64_t a = W->off[i]; a < W->off[i + 1]; a += kSnapBlock) {
      range.push_back(a);
      range.push_back(std::min(a + kSnapBlock, W->off[i + 1]));
      snap.push_back(i);
    }
  }
  first[ns] = (int)snap.size();
  const int nb = (int)snap.size();
  int64_t* d_range = nullptr;
  int *d_snap = nullptr, *d_first = nullptr;
  double *d_part = nullptr, *d_wr = nullptr;
  double2* d_d0 = nullptr;
  uint32_t* d_max = nullptr;
  auto cleanup = [&]() {
    dfree(d_range);
    dfree(d_snap);
    dfree(d_first);
    dfree(d_part);
    dfree(d_wr);
    dfree(d_d0);
    dfree(d_max);
  };
  hipError_t e = dalloc(&d_range, 2 * (int64_t)nb);
  if (e == hipSuccess) e = dalloc(&d_snap, nb);
  if (e == hipSuccess) e = dalloc(&d_first, ns + 1);
  if (e == hipSuccess) e = dalloc(&d_part, 5 * (int64_t)nb);
  if (e == hipSuccess) e = dalloc(&d_wr, W->nvis);
  if (e == hipSuccess) e = dalloc(&d_d0, ns);
  if (e == hipSuccess) e = dalloc(&d_max, 2);
  if (e == hipSuccess && nb > 0)
    e = hipMemcpyAsync(d_range, range.data(), sizeof(int64_t) * range.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && nb > 0)
    e = hipMemcpyAsync(d_snap, snap.data(), sizeof(int) * snap.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_fill_u32(d_max, 0u, 2, s);
  if (e == hipSuccess)
    e = launch_snap_fit(u, v, w, d_range, d_snap, d_first, nb, ns, d_part, d_d0, d_wr,
                        reinterpret_cast<unsigned long long*>(d_max), s);
  uint64_t maxbits = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(W->d0.data(), d_d0, sizeof(double2) * ns, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&maxbits, d_max, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return map_hip(e);
  }
  double m = 0.0;
  std::memcpy(&m, &maxbits, sizeof(m));
  W->h = m > 0.0 ? m * (1.0 + 0x1p-20) : 1.0;
  // the kernels' planes span the residual range
  K->w_lo = -W->h;
  K->w_hi = W->h;
  K->prm.w_lo = -W->h;
  K->prm.w_hi = W->h;
  K->inv_dw = (double)K->P / (K->w_hi - K->w_lo);
  K->generation += 1;
  int rc = map_hip(make_tables(K, s));
  for (int i = 0; i < ns && rc == SEPW_OK; ++i) {
    const int64_t n = W->off[i + 1] - W->off[i];
    if (n == 0) continue;
    Plan* P = new (std::nothrow) sepw_plan_s();
    if (!P) {
      rc = SEPW_ERR_OOM;
      break;
    }
    W->plans[i] = P;
    rc = alloc_plan(K, n, P);
    if (rc == SEPW_OK)
      rc = bin_plan(P, n, plain_coords(u + W->off[i], v + W->off[i], d_wr + W->off[i]), s);
  }
  if (rc == SEPW_OK) rc = map_hip(hipStreamSynchronize(s));
  cleanup();
  return rc;
}

// ---- batched gridding that allocates nothing ----
// The job tables of sepw_grid_batched_noalloc live in one static device array
// (each GPU the library runs on holds its own copy until the process ends);
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device, never through the array's name.
constexpr int kNoAllocMaxJobs = 256;
struct NoAllocArea {
  GridArgs jobs[kNoAllocMaxJobs];      // gridding jobs, largest first
  MoveArgs mjobs[kNoAllocMaxJobs];     // movement jobs, caller order
  uint32_t first[kNoAllocMaxJobs + 1];   // prefix of work items per job
  uint32_t mfirst[kNoAllocMaxJobs + 1];  // first movement workgroup per job
  alignas(256) uint32_t counter[8 * kCtrStride];   // work counters of the persistent launch
                                                   // (eight, each in a cache line of its own)
};

}  // namespace

static __device__ __align__(256) unsigned char scratch[sizeof(NoAllocArea)];

namespace {

// Up to kStoreJobs entries of the job tables, passed by value as a kernel
// argument and written into the area by one small kernel (no host copy).
constexpr int kStoreJobs = 8;
struct JobBlock {
  GridArgs g[kStoreJobs];
  MoveArgs m[kStoreJobs];
  uint32_t mfirst[kStoreJobs + 1];
  int base, n;
  int last;                            // write mfirst[base + n] too
};

__global__ void store_jobs_kernel(JobBlock b, NoAllocArea* area) {
  const int t = threadIdx.x;
  if (t < b.n) {
    area->jobs[b.base + t] = b.g[t];
    area->mjobs[b.base + t] = b.m[t];
    area->mfirst[b.base + t] = b.mfirst[t];
  }
  if (b.last && t == b.n) area->mfirst[b.base + b.n] = b.mfirst[b.n];
}

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_namx;
NoAllocArea* g_na_ptr[kNoAllocMaxDevices] = {};

// The area of the current device: its address is looked up once per device,
// with that device current.
int noalloc_area(NoAllocArea** out) {
  int dev = 0;
  SEPW_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return SEPW_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_namx);
  if (!g_na_ptr[dev]) {
    void* ptr = nullptr;
    SEPW_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return SEPW_ERR_HIP;
    g_na_ptr[dev] = static_cast<NoAllocArea*>(ptr);
  }
  *out = g_na_ptr[dev];
  return SEPW_OK;
}

int store_job_tables(NoAllocArea* area, int njobs, const GridArgs* g, const MoveArgs* m,
                     const uint32_t* mfirst, hipStream_t s) {
  for (int b0 = 0; b0 < njobs; b0 += kStoreJobs) {
    JobBlock b;
    b.base = b0;
    b.n = std::min(kStoreJobs, njobs - b0);
    b.last = b0 + b.n == njobs ? 1 : 0;
    for (int t = 0; t < b.n; ++t) {
      b.g[t] = g[b0 + t];
      b.m[t] = m[b0 + t];
      b.mfirst[t] = mfirst[b0 + t];
    }
    b.mfirst[b.n] = mfirst[b0 + b.n];
    hipLaunchKernelGGL(store_jobs_kernel, dim3(1), dim3(64), 0, s, b, area);
    SEPW_TRY(hipGetLastError());
  }
  return SEPW_OK;
}

}  // namespace


extern "C" {

void sepw_default_params(sepw_kernel_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->taper = SEPW_TAPER_PSWF;
  p->precision = SEPW_FP32;
  p->taper_width = 0.0;
  p->a_u = p->a_v = 0.5;
  p->b_u = p->b_v = 5.0 / 24.0;
}

int32_t sepw_device_count(void) { return device_count(); }

const char* sepw_strerror(int code) {
  switch (code) {
    case SEPW_OK: return "success";
    case SEPW_ERR_ARG: return "invalid argument";
    case SEPW_ERR_NO_DEVICE: return "no HIP device";
    case SEPW_ERR_HIP: return "HIP runtime or kernel error";
    case SEPW_ERR_OOM: return "device out of memory";
    case SEPW_ERR_UNSUPPORTED: return "unsupported parameter combination";
    case SEPW_ERR_FFT: return "hipFFT error";
    default: return "unknown error";
  }
}

int sepw_make_kernels(const sepw_kernel_params* params, void* hip_stream, sepw_kernels* out) {
  if (!out) return SEPW_ERR_ARG;
  *out = nullptr;
  int rc = validate_params(params);
  if (rc != SEPW_OK) return rc;
  if (device_count() < 1) return SEPW_ERR_NO_DEVICE;
  sepw_kernels_s* K = new (std::nothrow) sepw_kernels_s();
  if (!K) return SEPW_ERR_OOM;
  rc = build_kernels(params, static_cast<hipStream_t>(hip_stream), K);
  if (rc != SEPW_OK) {
    destroy_kernels(K);
    return rc;
  }
  *out = K;
  return SEPW_OK;
}

int sepw_kernels_table(sepw_kernels k, int32_t axis, sepw_c64* out, void* hip_stream) {
  if (!k || !out || (axis != 0 && axis != 1)) return SEPW_ERR_ARG;
  const size_t n = (size_t)k->P * k->O * k->S;
  SEPW_TRY(hipMemcpyAsync(out, axis == 0 ? k->tab_u : k->tab_v, sizeof(float2) * n,
                          hipMemcpyDeviceToDevice, static_cast<hipStream_t>(hip_stream)));
  return SEPW_OK;
}

int sepw_kernels_taper(sepw_kernels k, double* out, void* hip_stream) {
  if (!k || !out) return SEPW_ERR_ARG;
  SEPW_TRY(hipMemcpyAsync(out, k->c1, sizeof(double) * (size_t)k->N, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(hip_stream)));
  return SEPW_OK;
}

int sepw_kernels_set_correction(sepw_kernels k, int32_t support, int32_t oversample,
                                void* hip_stream) {
  if (!k) return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (support == 0) {
    if (k->corr) SEPW_TRY(hipStreamSynchronize(s));
    dfree(k->corr);
    dfree(k->corr_tmp);
    free_corr_terms(k);
    k->corr_S = k->corr_O = k->corr_nkb = 0;
    return SEPW_OK;
  }
  if (support < 1 || support % 2 == 0 || support > k->S) return SEPW_ERR_ARG;
  if (!is_pow2(oversample) || oversample > k->O) return SEPW_ERR_ARG;
  // the footprint about the coarse cell (possibly the next cell) stays inside the separable one
  if (oversample != k->O && oversample != 1 && support > k->S - 2) return SEPW_ERR_ARG;
  if (corr_dmax(support, oversample) + 1 > kCorrMaxD) return SEPW_ERR_UNSUPPORTED;
  // the correction passes run on the tiled path only
  if (k->facet || wide_support(k->S)) return SEPW_ERR_UNSUPPORTED;
  // the generation folds the screen about the image centre: the taper must be symmetric
  const int N = k->N;
  std::vector<double> c1(N);
  SEPW_TRY(hipMemcpyAsync(c1.data(), k->c1, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  SEPW_TRY(hipStreamSynchronize(s));
  for (int c = 1; c < N / 2; ++c)
    if (c1[N / 2 + c] != c1[N / 2 - c]) return SEPW_ERR_UNSUPPORTED;
  SEPW_TRY(hipStreamSynchronize(s));
  dfree(k->corr);
  dfree(k->corr_tmp);
  free_corr_terms(k);
  k->corr_S = k->corr_O = k->corr_nkb = 0;
  // planes per generation batch: FP64 work space of at most 2^25 doubles beyond the weights
  const int64_t one = corr_tmp_doubles(N, support, oversample, 1) - corr_tmp_doubles(N, support, oversample, 0);
  int64_t nkb = ((int64_t)1 << 25) / std::max<int64_t>(one, 1);
  nkb = std::max<int64_t>(1, std::min<int64_t>(nkb, k->P));
  SEPW_TRY(dalloc(&k->corr, (int64_t)k->P * oversample * oversample * support * support));
  hipError_t e = dalloc(&k->corr_tmp, corr_tmp_doubles(N, support, oversample, (int)nkb));
  if (e != hipSuccess) {
    dfree(k->corr);
    return map_hip(e);
  }
  k->corr_S = support;
  k->corr_O = oversample;
  k->corr_nkb = (int)nkb;
  SEPW_TRY(make_corr_table(k, s));
  return SEPW_OK;
}

int sepw_kernels_correction_table(sepw_kernels k, sepw_c64* out, void* hip_stream) {
  if (!k || !out || !k->corr) return SEPW_ERR_ARG;
  const size_t n = (size_t)k->P * k->corr_O * k->corr_O * k->corr_S * k->corr_S;
  SEPW_TRY(hipMemcpyAsync(out, k->corr, sizeof(float2) * n, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(hip_stream)));
  return SEPW_OK;
}

int sepw_kernels_correction_terms(sepw_kernels k, int32_t enable, void* hip_stream) {
  if (!k || (enable != 0 && enable != 1)) return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  k->corr_terms = enable != 0;
  if (!k->corr) return SEPW_OK;
  if (enable) {
    if (k->corr_rank < 0) SEPW_TRY(factor_corr(k, s));
  } else {
    SEPW_TRY(hipStreamSynchronize(s));   // calls in flight may still read the term tables
    free_corr_terms(k);
  }
  return SEPW_OK;
}

int sepw_kernels_correction_rank(sepw_kernels k, int32_t* rank) {
  if (!k || !rank || !k->corr) return SEPW_ERR_ARG;
  *rank = k->corr_rank;
  return SEPW_OK;
}

int sepw_plan_create(sepw_kernels k, int64_t nvis, const double* u, const double* v,
                     const double* w, int64_t* n_dropped, void* hip_stream, sepw_plan* out) {
  if (!out) return SEPW_ERR_ARG;
  *out = nullptr;
  if (!k || nvis < 0 || nvis > 2147483646LL) return SEPW_ERR_ARG;
  if (nvis > 0 && (!u || !v || !w)) return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  sepw_plan_s* P = new (std::nothrow) sepw_plan_s();
  if (!P) return SEPW_ERR_OOM;
  int rc = alloc_plan(k, nvis, P);
  if (rc == SEPW_OK) rc = bin_plan(P, nvis, plain_coords(u, v, w), s);
  if (rc == SEPW_OK && n_dropped) rc = read_dropped(P, n_dropped, s);
  if (rc != SEPW_OK) {
    destroy_plan(P);
    return rc;
  }
  *out = P;
  return SEPW_OK;
}

int sepw_plan_rebin(sepw_plan p, int64_t nvis, const double* u, const double* v, const double* w,
                    int64_t* n_dropped, void* hip_stream) {
  if (!p || nvis < 0 || nvis > p->capacity) return SEPW_ERR_ARG;
  if (nvis > 0 && (!u || !v || !w)) return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int rc = bin_plan(p, nvis, plain_coords(u, v, w), s);
  if (rc == SEPW_OK && n_dropped) rc = read_dropped(p, n_dropped, s);
  return rc;
}

int sepw_plan_create_channels(sepw_kernels k, int64_t nrows, int32_t nchan, const double* uvw,
                              const double* freq, int64_t* n_dropped, void* hip_stream,
                              sepw_plan* out) {
  if (!out) return SEPW_ERR_ARG;
  *out = nullptr;
  if (!k || nrows < 0 || nrows > 2147483646LL || nchan < 1 || nrows * (int64_t)nchan > 2147483646LL)
    return SEPW_ERR_ARG;
  if (nrows > 0 && (!uvw || !freq)) return SEPW_ERR_ARG;
  const int64_t nvis = nrows * (int64_t)nchan;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  sepw_plan_s* P = new (std::nothrow) sepw_plan_s();
  if (!P) return SEPW_ERR_OOM;
  Coords c;
  c.uvw = uvw;
  c.freq = freq;
  c.nchan = nchan;
  int rc = alloc_plan(k, nvis, P);
  if (rc == SEPW_OK) rc = bin_plan(P, nvis, c, s);
  if (rc == SEPW_OK && n_dropped) rc = read_dropped(P, n_dropped, s);
  if (rc != SEPW_OK) {
    destroy_plan(P);
    return rc;
  }
  *out = P;
  return SEPW_OK;
}

int sepw_plan_rebin_channels(sepw_plan p, int64_t nrows, int32_t nchan, const double* uvw,
                             const double* freq, int64_t* n_dropped, void* hip_stream) {
  if (!p || nrows < 0 || nrows > 2147483646LL || nchan < 1 || nrows * (int64_t)nchan > p->capacity)
    return SEPW_ERR_ARG;
  if (nrows > 0 && (!uvw || !freq)) return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Coords c;
  c.uvw = uvw;
  c.freq = freq;
  c.nchan = nchan;
  int rc = bin_plan(p, nrows * (int64_t)nchan, c, s);
  if (rc == SEPW_OK && n_dropped) rc = read_dropped(p, n_dropped, s);
  return rc;
}

int32_t sepw_plan_tile_size(sepw_plan p) { return p ? p->tile_c : 0; }

int sepw_plan_bins(sepw_plan p, int32_t* out, void* hip_stream) {
  if (!p || (!out && p->nvis > 0)) return SEPW_ERR_ARG;
  SEPW_TRY(launch_bins_export(p->rrec, p->place, p->delta, p->nbins, p->nvis, p->tile_c, p->ntx,
                              out, static_cast<hipStream_t>(hip_stream)));
  return SEPW_OK;
}

int sepw_grid(sepw_plan p, const sepw_c64* vis, const float* weight, sepw_c64* out,
              uint32_t flags, void* hip_stream) {
  if (!p || !out || (!vis && p->nvis > 0)) return SEPW_ERR_ARG;
  if ((flags & ~(SEPW_GRID_ONLY | SEPW_MUL_N | SEPW_DIV_N | SEPW_REAL)) != 0) return SEPW_ERR_ARG;
  if ((flags & SEPW_MUL_N) && (flags & SEPW_DIV_N)) return SEPW_ERR_ARG;
  if ((flags & SEPW_REAL) && (flags & SEPW_GRID_ONLY)) return SEPW_ERR_ARG;
  Kernels* K = p->K;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // a real output image: the grid and its transform go through the kernels'
  // complex work array, and only the real part reaches out
  const bool real_out = flags & SEPW_REAL;
  float2* img = real_out ? K->scratch : reinterpret_cast<float2*>(out);
  const int N = K->N;
  const bool grid_only = flags & SEPW_GRID_ONLY;
  if (p->generation != K->generation) return SEPW_ERR_ARG;
  if (wide_support(K->S)) {
    if (K->corr) return SEPW_ERR_UNSUPPORTED;
    {
      Stage st(SEPW_STAGE_FILL, s);
      SEPW_TRY(launch_zero_c64(img, (int64_t)N * N, s));
    }
    {
      Stage st(SEPW_STAGE_GRID, s);
      SEPW_TRY(launch_grid_wide(wide_args(p, grid_only ? 0 : 1), reinterpret_cast<const float2*>(vis),
                                weight, img, s));
    }
  } else {
  {
    Stage st(SEPW_STAGE_GATHER, s);
    MoveArgs m = move_args(p, vis, weight);
    if (K->prm.precision == SEPW_FP16) {
      SEPW_TRY(launch_fill_u32(p->lp_max, 0u, 1, s));
      m.vmax = p->lp_max;
    }
    SEPW_TRY(launch_vis_to_rows(m, s));
  }
  {
    Stage st(SEPW_STAGE_FILL, s);
    SEPW_TRY(launch_zero_c64(img, (int64_t)N * N, s));
  }
  {
    Stage st(SEPW_STAGE_GRID, s);
    if (K->prm.precision == SEPW_FP32) {
      GridArgs a{p->gl.items, p->gl.itoff + 8 * p->r8, p->gl.itoff, p->r8, p->qctr, p->tdesc, p->krec,
                 p->yrow, K->pad_u, K->pad_v,
                 K->tab_len, N, p->ntx, grid_only ? 0 : 1, img};
      if (K->lds_bytes > 0) {
        SEPW_TRY(launch_fill_u32(p->qctr, 0u, 8 * kCtrStride, s));
        SEPW_TRY(launch_grid_fp32_lds(K->S, a, K->lds_bytes, K->n_cu, s));
      } else {
        SEPW_TRY(launch_grid_fp32(K->S, a, p->gl.max_items, s));
      }
    } else {
      GridArgsLp a{p->gl.items, p->gl.itoff + 8 * p->r8, p->tdesc, p->krec, p->yrow, K->pad_u,
                   K->pad_v, K->tab_len, p->lp_max, p->qctr, N, p->ntx, grid_only ? 0 : 1, img};
      SEPW_TRY(launch_fill_u32(p->qctr, 0u, 8 * kCtrStride, s));
      SEPW_TRY(launch_grid_lp(K->S, K->prm.precision == SEPW_BF16, a, K->lds_bytes, K->n_cu, s));
    }
  }
  {
    int rc = corr_grid_pass(p, img, grid_only ? 0 : 1, s);
    if (rc != SEPW_OK) return rc;
  }
  }
  if (grid_only) return SEPW_OK;
  {
    Stage st(SEPW_STAGE_FFT, s);
    int rc = fft_exec(K, img, HIPFFT_BACKWARD, s);
    if (rc != SEPW_OK) return rc;
  }
  const int npow = (flags & SEPW_MUL_N) ? 1 : ((flags & SEPW_DIV_N) ? -1 : 0);
  {
    Stage st(SEPW_STAGE_CORRECT, s);
    if (real_out)
      SEPW_TRY(launch_correct_real_out(img, reinterpret_cast<float*>(out), K->c1, N, K->fov, K->l0,
                                       K->m0, npow, s));
    else
      SEPW_TRY(launch_correct(img, img, K->c1, N, K->fov, K->l0, K->m0, npow, s));
  }
  return SEPW_OK;
}

int sepw_degrid(sepw_plan p, const sepw_c64* in, sepw_c64* vis_out, uint32_t flags,
                void* hip_stream) {
  if (!p || !in || (!vis_out && p->nvis > 0)) return SEPW_ERR_ARG;
  if ((flags & ~(SEPW_GRID_ONLY | SEPW_DIV_N | SEPW_REAL)) != 0) return SEPW_ERR_ARG;
  if ((flags & SEPW_REAL) && (flags & SEPW_GRID_ONLY)) return SEPW_ERR_ARG;
  Kernels* K = p->K;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int N = K->N;
  if (p->generation != K->generation) return SEPW_ERR_ARG;
  const float2* src = reinterpret_cast<const float2*>(in);
  int checker = 0;
  if (!(flags & SEPW_GRID_ONLY)) {
    const int npow = (flags & SEPW_DIV_N) ? -1 : 0;
    {
      Stage st(SEPW_STAGE_CORRECT, s);
      if (flags & SEPW_REAL)
        SEPW_TRY(launch_correct_real_in(reinterpret_cast<const float*>(in), K->scratch, K->c1, N,
                                        K->fov, K->l0, K->m0, npow, s));
      else
        SEPW_TRY(launch_correct(src, K->scratch, K->c1, N, K->fov, K->l0, K->m0, npow, s));
    }
    {
      Stage st(SEPW_STAGE_FFT, s);
      int rc = fft_exec(K, K->scratch, HIPFFT_FORWARD, s);
      if (rc != SEPW_OK) return rc;
    }
    src = K->scratch;
    checker = 1;
  }
  if (p->nvis == 0) return SEPW_OK;
  float2* vo = reinterpret_cast<float2*>(vis_out);
  if (wide_support(K->S)) {
    if (K->corr) return SEPW_ERR_UNSUPPORTED;
    Stage st(SEPW_STAGE_DEGRID, s);
    SEPW_TRY(launch_degrid_wide(wide_args(p, checker), src, vo, s));
    return SEPW_OK;
  }
  {
    Stage st(SEPW_STAGE_DEGRID, s);
    SEPW_TRY(launch_fill_u32(p->qctr, 0u, 8 * kCtrStride, s));
    if (K->prm.precision == SEPW_FP32) {
      DegridArgs a{p->dl.items, p->dl.itoff + 8 * p->r8, p->dl.itoff, p->r8, p->qctr, p->tdesc, p->krec,
                   src, checker ? K->pad_su : K->pad_u, checker ? K->pad_sv : K->pad_v,
                   K->tab_len, N, p->ntx, checker, p->yrow};
      SEPW_TRY(launch_degrid_fp32(K->S, a, p->dl.max_items, K->lds_bytes, K->n_cu, s));
    } else {
      const bool bf16 = K->prm.precision == SEPW_BF16;
      // the 16-bit degridding kernel addresses records and results through
      // 32-bit buffer offsets
      if (p->pcap * (int64_t)sizeof(SlotRec) > 0x7FFFFFFFLL ||
          (p->capacity + 1) * (int64_t)sizeof(float2) > 0x7FFFFFFFLL)
        return SEPW_ERR_UNSUPPORTED;
      if (!bf16) {
        SEPW_TRY(launch_fill_u32(p->lp_max + 1, 0u, 1, s));
        SEPW_TRY(launch_absmax(src, (int64_t)N * N, p->lp_max + 1, s));
      }
      DegridArgsLp a{p->dl.items, p->dl.itoff, p->r8, p->qctr, p->tdesc, p->krec, src, K->lp_u,
                     K->lp_v, K->tab_len, p->lp_max + 1, N, p->ntx, checker, p->yrow,
                     p->pcap, p->capacity + 1};
      if (!K->g16) return SEPW_ERR_UNSUPPORTED;   // 16-bit kernels always hold it
      SEPW_TRY(launch_lp_grid(src, N, bf16, p->lp_max + 1, checker, K->g16, s));
      a.g16 = K->g16;
      SEPW_TRY(launch_degrid_lp(K->S, bf16, a, K->lds_bytes_lp, K->n_cu, s));
    }
  }
  {
    int rc = corr_degrid_pass(p, src, checker, s);
    if (rc != SEPW_OK) return rc;
  }
  {
    Stage st(SEPW_STAGE_GATHER, s);
    SEPW_TRY(launch_vis_from_rows(p->yrow, p->rot, p->place, p->delta, p->ckept, p->nvis,
                                  p->nbins, vo, s));
  }
  return SEPW_OK;
}

// Internal flag of grid_batched: grids as for a transform (the centred FFT's
// checkerboard included) but no FFT and no correction (FP32 tiled jobs only).
constexpr uint32_t kGridNoTransform = 0x40000000u;

int grid_batched(int32_t njobs, const sepw_plan* plans, const sepw_c64* const* vis,
                 const float* const* weight, sepw_c64* const* out, uint32_t flags, hipStream_t s);

int sepw_grid_batched(int32_t njobs, const sepw_plan* plans, const sepw_c64* const* vis,
                      const float* const* weight, sepw_c64* const* out, uint32_t flags,
                      void* hip_stream) {
  if (njobs < 1 || !plans || !vis || !out) return SEPW_ERR_ARG;
  if ((flags & ~(SEPW_GRID_ONLY | SEPW_MUL_N | SEPW_DIV_N)) != 0) return SEPW_ERR_ARG;
  if ((flags & SEPW_MUL_N) && (flags & SEPW_DIV_N)) return SEPW_ERR_ARG;
  for (int j = 0; j < njobs; ++j) {
    if (!plans[j] || !out[j] || (!vis[j] && plans[j]->nvis > 0)) return SEPW_ERR_ARG;
    const Kernels* K = plans[j]->K;
    const Kernels* K0 = plans[0]->K;
    if (K->N != K0->N || K->S != K0->S || K->prm.precision != K0->prm.precision) return SEPW_ERR_ARG;
    if (plans[j]->generation != K->generation) return SEPW_ERR_ARG;
  }
  return grid_batched(njobs, plans, vis, weight, out, flags, static_cast<hipStream_t>(hip_stream));
}

// sepw_grid_batched after argument checks (flags may add kGridNoTransform)
int grid_batched(int32_t njobs, const sepw_plan* plans, const sepw_c64* const* vis,
                 const float* const* weight, sepw_c64* const* out, uint32_t flags, hipStream_t s) {
  void* hip_stream = s;
  if (plans[0]->K->prm.precision != SEPW_FP32 || wide_support(plans[0]->K->S)) {
    if (flags & kGridNoTransform) return SEPW_ERR_UNSUPPORTED;
    // the persistent launch is built for the FP32 path; other precisions go job by job
    for (int j = 0; j < njobs; ++j) {
      int rc = sepw_grid(plans[j], vis[j], weight ? weight[j] : nullptr, out[j], flags, hip_stream);
      if (rc != SEPW_OK) return rc;
    }
    return SEPW_OK;
  }
  const bool grid_only = flags & SEPW_GRID_ONLY;
  const int N = plans[0]->K->N, S = plans[0]->K->S;
  // jobs in decreasing size, so the largest start first
  std::vector<int> order(njobs);
  for (int j = 0; j < njobs; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return plans[a]->nvis > plans[b]->nvis; });
  BatchScratch* bs = nullptr;
  int rc = batch_scratch(plans[0], njobs, s, &bs);
  if (rc != SEPW_OK) return rc;
  // one movement launch for all jobs (job table and workgroup prefix on the host)
  int64_t mtotal = 0;
  bs->mfirst_host[0] = 0;
  for (int j = 0; j < njobs; ++j) {
    bs->mhost[j] = move_args(plans[j], vis[j], weight ? weight[j] : nullptr);
    mtotal += move_blocks(plans[j]->nvis);
    if (mtotal > 0xFFFFFFFFLL) return SEPW_ERR_UNSUPPORTED;
    bs->mfirst_host[j + 1] = (uint32_t)mtotal;
  }
  SEPW_TRY(hipMemcpyAsync(bs->mjobs, bs->mhost, sizeof(MoveArgs) * (size_t)njobs,
                          hipMemcpyHostToDevice, s));
  SEPW_TRY(hipMemcpyAsync(bs->mfirst, bs->mfirst_host, sizeof(uint32_t) * (size_t)(njobs + 1),
                          hipMemcpyHostToDevice, s));
  {
    Stage st(SEPW_STAGE_GATHER, s);
    SEPW_TRY(launch_vis_to_rows_batched(bs->mjobs, bs->mfirst, njobs, mtotal, s));
  }
  {
    Stage st(SEPW_STAGE_FILL, s);
    for (int j = 0; j < njobs; ++j)
      SEPW_TRY(launch_zero_c64(reinterpret_cast<float2*>(out[j]), (int64_t)N * N, s));
  }
  for (int r = 0; r < njobs; ++r) {
    Plan* p = plans[order[r]];
    Kernels* K = p->K;
    bs->host[r] = GridArgs{p->gl.items, p->gl.itoff + 8 * p->r8, p->gl.itoff, p->r8, p->qctr, p->tdesc,
                           p->krec, p->yrow, K->pad_u,
                           K->pad_v, K->tab_len, N, p->ntx, grid_only ? 0 : 1,
                           reinterpret_cast<float2*>(out[order[r]])};
  }
  SEPW_TRY(hipMemcpyAsync(bs->jobs, bs->host, sizeof(GridArgs) * (size_t)njobs,
                          hipMemcpyHostToDevice, s));
  SEPW_TRY(hipEventRecord(bs->copied, s));
  {
    Stage st(SEPW_STAGE_GRID, s);
    SEPW_TRY(launch_job_prefix(bs->jobs, njobs, bs->first, bs->counter, s));
    SEPW_TRY(launch_grid_fp32_batched(S, bs->jobs, bs->first, njobs, bs->counter, bs->blocks, s));
  }
  for (int j = 0; j < njobs; ++j) {
    rc = corr_grid_pass(plans[j], reinterpret_cast<float2*>(out[j]), grid_only ? 0 : 1, s);
    if (rc != SEPW_OK) return rc;
  }
  if (grid_only || (flags & kGridNoTransform)) return SEPW_OK;
  const int npow = (flags & SEPW_MUL_N) ? 1 : ((flags & SEPW_DIV_N) ? -1 : 0);
  for (int j = 0; j < njobs; ++j) {
    Kernels* K = plans[j]->K;
    float2* img = reinterpret_cast<float2*>(out[j]);
    {
      Stage st(SEPW_STAGE_FFT, s);
      rc = fft_exec(K, img, HIPFFT_BACKWARD, s);
      if (rc != SEPW_OK) return rc;
    }
    Stage st(SEPW_STAGE_CORRECT, s);
    SEPW_TRY(launch_correct(img, img, K->c1, N, K->fov, K->l0, K->m0, npow, s));
  }
  return SEPW_OK;
}

int sepw_grid_batched_noalloc(int32_t njobs, const sepw_plan* plans, const sepw_c64* const* vis,
                              const float* const* weight, sepw_c64* const* out, uint32_t flags,
                              void* hip_stream) {
  if (njobs < 1 || !plans || !vis || !out) return SEPW_ERR_ARG;
  if (njobs > kNoAllocMaxJobs) return SEPW_ERR_UNSUPPORTED;   // the static job tables' size
  if ((flags & ~(SEPW_GRID_ONLY | SEPW_MUL_N | SEPW_DIV_N)) != 0) return SEPW_ERR_ARG;
  if ((flags & SEPW_MUL_N) && (flags & SEPW_DIV_N)) return SEPW_ERR_ARG;
  for (int j = 0; j < njobs; ++j) {
    if (!plans[j] || !out[j] || (!vis[j] && plans[j]->nvis > 0)) return SEPW_ERR_ARG;
    const Kernels* K = plans[j]->K;
    const Kernels* K0 = plans[0]->K;
    if (K->N != K0->N || K->S != K0->S || K->prm.precision != K0->prm.precision) return SEPW_ERR_ARG;
    if (plans[j]->generation != K->generation) return SEPW_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (plans[0]->K->prm.precision != SEPW_FP32 || wide_support(plans[0]->K->S)) {
    // job by job, as sepw_grid_batched does (sepw_grid allocates nothing)
    for (int j = 0; j < njobs; ++j) {
      int rc = sepw_grid(plans[j], vis[j], weight ? weight[j] : nullptr, out[j], flags, hip_stream);
      if (rc != SEPW_OK) return rc;
    }
    return SEPW_OK;
  }
  NoAllocArea* area = nullptr;
  int rc = noalloc_area(&area);
  if (rc != SEPW_OK) return rc;
  const bool grid_only = flags & SEPW_GRID_ONLY;
  const int N = plans[0]->K->N, S = plans[0]->K->S;
  // jobs in decreasing size (stable), so the largest start first
  int order[kNoAllocMaxJobs];
  for (int j = 0; j < njobs; ++j) {
    int i = j;
    while (i > 0 && plans[order[i - 1]]->nvis < plans[j]->nvis) {
      order[i] = order[i - 1];
      --i;
    }
    order[i] = j;
  }
  GridArgs g[kNoAllocMaxJobs];
  MoveArgs m[kNoAllocMaxJobs];
  uint32_t mfirst[kNoAllocMaxJobs + 1];
  int64_t mtotal = 0;
  mfirst[0] = 0;
  for (int j = 0; j < njobs; ++j) {
    m[j] = move_args(plans[j], vis[j], weight ? weight[j] : nullptr);
    mtotal += move_blocks(plans[j]->nvis);
    if (mtotal > 0xFFFFFFFFLL) return SEPW_ERR_UNSUPPORTED;
    mfirst[j + 1] = (uint32_t)mtotal;
  }
  for (int r = 0; r < njobs; ++r) {
    Plan* p = plans[order[r]];
    Kernels* K = p->K;
    g[r] = GridArgs{p->gl.items, p->gl.itoff + 8 * p->r8, p->gl.itoff, p->r8, p->qctr, p->tdesc,
                    p->krec, p->yrow, K->pad_u, K->pad_v, K->tab_len, N, p->ntx,
                    grid_only ? 0 : 1, reinterpret_cast<float2*>(out[order[r]])};
  }
  rc = store_job_tables(area, njobs, g, m, mfirst, s);
  if (rc != SEPW_OK) return rc;
  SEPW_TRY(launch_vis_to_rows_batched(area->mjobs, area->mfirst, njobs, mtotal, s));
  for (int j = 0; j < njobs; ++j)
    SEPW_TRY(launch_zero_c64(reinterpret_cast<float2*>(out[j]), (int64_t)N * N, s));
  SEPW_TRY(launch_job_prefix(area->jobs, njobs, area->first, area->counter, s));
  SEPW_TRY(launch_grid_fp32_batched(S, area->jobs, area->first, njobs, area->counter,
                                    plans[0]->K->n_cu * plans[0]->blocks_per_cu, s));
  for (int j = 0; j < njobs; ++j) {
    rc = corr_grid_pass(plans[j], reinterpret_cast<float2*>(out[j]), grid_only ? 0 : 1, s);
    if (rc != SEPW_OK) return rc;
  }
  if (grid_only) return SEPW_OK;
  const int npow = (flags & SEPW_MUL_N) ? 1 : ((flags & SEPW_DIV_N) ? -1 : 0);
  for (int j = 0; j < njobs; ++j) {
    Kernels* K = plans[j]->K;
    float2* img = reinterpret_cast<float2*>(out[j]);
    rc = fft_exec(K, img, HIPFFT_BACKWARD, s);
    if (rc != SEPW_OK) return rc;
    SEPW_TRY(launch_correct(img, img, K->c1, N, K->fov, K->l0, K->m0, npow, s));
  }
  return SEPW_OK;
}

int sepw_plan_set_item_slots(sepw_plan p, int32_t slots, void* hip_stream) {
  if (!p) return SEPW_ERR_ARG;
  return set_list_slots(p, p->gl, slots, static_cast<hipStream_t>(hip_stream));
}

int sepw_plan_set_degrid_item_slots(sepw_plan p, int32_t slots, void* hip_stream) {
  if (!p) return SEPW_ERR_ARG;
  return set_list_slots(p, p->dl, slots, static_cast<hipStream_t>(hip_stream));
}

namespace {
// Autotuner results by (device, N, S, O, precision, jobs, floor(log2 total vis)).
std::mutex g_tune_mx;
std::map<std::array<int64_t, 7>, std::pair<int, int>> g_tune;
}  // namespace

int sepw_autotune_batched(int32_t njobs, const sepw_plan* plans, const sepw_c64* const* vis,
                          const float* const* weight, sepw_c64* const* out, void* hip_stream,
                          int32_t* item_slots, int32_t* blocks_per_cu) {
  if (njobs < 1 || !plans) return SEPW_ERR_ARG;
  for (int j = 0; j < njobs; ++j)
    if (!plans[j]) return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int64_t total = 0;
  for (int j = 0; j < njobs; ++j) total += plans[j]->nvis;
  int bucket = 0;
  while (bucket < 62 && (int64_t(2) << bucket) <= total) ++bucket;
  int dev = 0;
  SEPW_TRY(hipGetDevice(&dev));
  const Kernels* K0 = plans[0]->K;
  const std::array<int64_t, 7> key{dev, K0->N, K0->S, K0->O, K0->prm.precision, njobs, bucket};
  {
    std::unique_lock<std::mutex> lk(g_tune_mx);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      const std::pair<int, int> best = it->second;
      lk.unlock();
      int rc = SEPW_OK;
      for (int j = 0; j < njobs; ++j) plans[j]->blocks_per_cu = best.second;
      for (int j = 0; j < njobs && rc == SEPW_OK; ++j)
        rc = sepw_plan_set_item_slots(plans[j], best.first, hip_stream);
      if (rc != SEPW_OK) return rc;
      if (item_slots) *item_slots = best.first;
      if (blocks_per_cu) *blocks_per_cu = best.second;
      return SEPW_OK;
    }
  }
  const int kSlots[] = {256, 512, 1024, 2048};
  const int kWidth[] = {2, 4, 8};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SEPW_TRY(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return map_hip(he);
  }
  float best = 0.f;
  int best_slots = kItemMaxVis, best_width = 8, rc = SEPW_OK;
  for (int si = 0; si < 4 && rc == SEPW_OK; ++si) {
    for (int j = 0; j < njobs && rc == SEPW_OK; ++j)
      rc = sepw_plan_set_item_slots(plans[j], kSlots[si], hip_stream);
    for (int wi = 0; wi < 3 && rc == SEPW_OK; ++wi) {
      for (int j = 0; j < njobs; ++j) plans[j]->blocks_per_cu = kWidth[wi];
      rc = sepw_grid_batched(njobs, plans, vis, weight, out, SEPW_GRID_ONLY, hip_stream);
      if (rc != SEPW_OK) break;
      he = hipEventRecord(e0, s);
      for (int r = 0; r < 2 && rc == SEPW_OK; ++r)
        rc = sepw_grid_batched(njobs, plans, vis, weight, out, SEPW_GRID_ONLY, hip_stream);
      if (he == hipSuccess) he = hipEventRecord(e1, s);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) rc = map_hip(he);
      if (rc == SEPW_OK && (best == 0.f || ms < best)) {
        best = ms;
        best_slots = kSlots[si];
        best_width = kWidth[wi];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int j = 0; j < njobs; ++j) plans[j]->blocks_per_cu = best_width;
  for (int j = 0; j < njobs && rc == SEPW_OK; ++j)
    rc = sepw_plan_set_item_slots(plans[j], best_slots, hip_stream);
  if (rc != SEPW_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mx);
    g_tune[key] = std::make_pair(best_slots, best_width);
  }
  if (item_slots) *item_slots = best_slots;
  if (blocks_per_cu) *blocks_per_cu = best_width;
  return SEPW_OK;
}

int sepw_kernels_set_wrange(sepw_kernels k, double w_lo, double w_hi, void* hip_stream) {
  if (!k || !std::isfinite(w_lo) || !std::isfinite(w_hi) || !(w_lo < w_hi)) return SEPW_ERR_ARG;
  k->w_lo = w_lo;
  k->w_hi = w_hi;
  k->prm.w_lo = w_lo;
  k->prm.w_hi = w_hi;
  k->inv_dw = (double)k->P / (w_hi - w_lo);
  k->generation += 1;
  SEPW_TRY(make_tables(k, static_cast<hipStream_t>(hip_stream)));
  return SEPW_OK;
}

int sepw_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_tmx);
  g_timing = on != 0;
  return SEPW_OK;
}

int sepw_timing_collect(double* ms, int64_t* n) {
  if (!ms || !n) return SEPW_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_tmx);
  for (int i = 0; i < SEPW_NSTAGES; ++i) {
    ms[i] = 0.0;
    n[i] = 0;
  }
  int rc = SEPW_OK;
  for (const TimingRec& r : g_recs) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) {
      rc = map_hip(e);
    } else {
      ms[r.stage] += t;
      n[r.stage] += 1;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return rc;
}

int sepw_free_kernels(sepw_kernels k) {
  if (!k) return SEPW_ERR_ARG;
  destroy_kernels(k);
  return SEPW_OK;
}

int sepw_free_plan(sepw_plan p) {
  if (!p) return SEPW_ERR_ARG;
  destroy_plan(p);
  return SEPW_OK;
}

int sepw_free_wstack(sepw_wstack ws) {
  if (!ws) return SEPW_ERR_ARG;
  destroy_wstack(ws);
  return SEPW_OK;
}

int sepw_wstack_create(sepw_kernels k, int32_t n_slices, double w_lo, double w_hi, int64_t nvis,
                       const double* u, const double* v, const double* w, int64_t* n_dropped,
                       void* hip_stream, sepw_wstack* out) {
  if (!out) return SEPW_ERR_ARG;
  *out = nullptr;
  if (!k || k->facet || n_slices < 1 || n_slices > kMaxSlices) return SEPW_ERR_ARG;
  if (!std::isfinite(w_lo) || !std::isfinite(w_hi) || !(w_lo < w_hi)) return SEPW_ERR_ARG;
  if (nvis < 0 || nvis > 2147483646LL) return SEPW_ERR_ARG;
  if (nvis > 0 && (!u || !v || !w)) return SEPW_ERR_ARG;
  // the kernels' planes must span the residual range [-h, h] of one slice
  const double h = (w_hi - w_lo) / (2.0 * n_slices);
  if (std::fabs(k->w_lo + h) > 1e-12 * h || std::fabs(k->w_hi - h) > 1e-12 * h)
    return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  sepw_wstack_s* W = new (std::nothrow) sepw_wstack_s();
  if (!W) return SEPW_ERR_OOM;
  int rc = wstack_build(W, k, n_slices, w_lo, w_hi, nullptr, nvis, u, v, w, n_dropped, s);
  if (rc != SEPW_OK) {
    destroy_wstack(W);
    return rc;
  }
  *out = W;
  return SEPW_OK;
}

int sepw_wstack_create_edges(sepw_kernels k, int32_t n_slices, const double* edges, int64_t nvis,
                             const double* u, const double* v, const double* w,
                             int64_t* n_dropped, void* hip_stream, sepw_wstack* out) {
  if (!out) return SEPW_ERR_ARG;
  *out = nullptr;
  if (!k || k->facet || n_slices < 1 || n_slices > kMaxSlices || !edges) return SEPW_ERR_ARG;
  if (nvis < 0 || nvis > 2147483646LL) return SEPW_ERR_ARG;
  if (nvis > 0 && (!u || !v || !w)) return SEPW_ERR_ARG;
  for (int j = 0; j <= n_slices; ++j)
    if (!std::isfinite(edges[j])) return SEPW_ERR_ARG;
  for (int j = 0; j < n_slices; ++j)
    if (!(edges[j] < edges[j + 1])) return SEPW_ERR_ARG;
  // every slice gets tables of its own (k's parameters, the slice's w range)
  if (k->corr) return SEPW_ERR_UNSUPPORTED;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  sepw_wstack_s* W = new (std::nothrow) sepw_wstack_s();
  if (!W) return SEPW_ERR_OOM;
  int rc = wstack_build(W, k, n_slices, edges[0], edges[n_slices], edges, nvis, u, v, w, n_dropped,
                        s);
  if (rc != SEPW_OK) {
    destroy_wstack(W);
    return rc;
  }
  *out = W;
  return SEPW_OK;
}

int sepw_wstack_density_edges(int64_t nvis, const double* w, int32_t n_slices, double w_lo,
                              double w_hi, double* edges, void* hip_stream) {
  if (!edges || n_slices < 1 || n_slices > kMaxSlices) return SEPW_ERR_ARG;
  if (!std::isfinite(w_lo) || !std::isfinite(w_hi) || !(w_lo < w_hi)) return SEPW_ERR_ARG;
  if (nvis < 0 || nvis > 2147483646LL || (nvis > 0 && !w)) return SEPW_ERR_ARG;
  if (device_count() < 1) return SEPW_ERR_NO_DEVICE;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int nfine = kDensityBins;
  std::vector<uint32_t> hc(nfine);
  uint32_t* counts = nullptr;
  SEPW_TRY(dalloc(&counts, nfine));
  auto run = [&]() -> int {
    SEPW_TRY(launch_fill_u32(counts, 0u, nfine, s));
    SEPW_TRY(launch_w_hist(w, nvis, w_lo, (double)nfine / (w_hi - w_lo), nfine, counts, s));
    SEPW_TRY(hipMemcpyAsync(hc.data(), counts, sizeof(uint32_t) * nfine, hipMemcpyDeviceToHost, s));
    SEPW_TRY(hipStreamSynchronize(s));
    return SEPW_OK;
  };
  const int rc = run();
  dfree(counts);
  if (rc != SEPW_OK) return rc;
  // below[j] = finite visibilities in bins < j; edge k at the first j with
  // below[j] ns >= k n, kept increasing with one bin left for each later slice
  std::vector<int64_t> below(nfine + 1, 0);
  for (int j = 0; j < nfine; ++j) below[j + 1] = below[j] + hc[j];
  const int64_t n = below[nfine];
  const double d = (w_hi - w_lo) / nfine;
  edges[0] = w_lo;
  edges[n_slices] = w_hi;
  int search = 0, prev = 0;
  for (int k = 1; k < n_slices; ++k) {
    while (search < nfine && below[search] * n_slices < (int64_t)k * n) ++search;
    const int jk = std::min(std::max(search, prev + 1), nfine - (n_slices - k));
    const double t = (double)jk * d;
    edges[k] = w_lo + t;
    prev = jk;
  }
  return SEPW_OK;
}

int sepw_wstack_grid(sepw_wstack ws, const sepw_c64* vis, const float* weight, sepw_c64* image_out,
                     uint32_t flags, void* hip_stream) {
  if (!ws || !image_out || (!vis && ws->nvis > 0)) return SEPW_ERR_ARG;
  if ((flags & ~(SEPW_MUL_N | SEPW_DIV_N)) != 0) return SEPW_ERR_ARG;
  if ((flags & SEPW_MUL_N) && (flags & SEPW_DIV_N)) return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Kernels* K = ws->K;
  float2* out = reinterpret_cast<float2*>(image_out);
  if (ws->nvis > 0) {
    Stage st(SEPW_STAGE_GATHER, s);
    SEPW_TRY(launch_slice_gather(reinterpret_cast<const float2*>(vis), weight, ws->order, ws->nvis,
                                 ws->vis, s));
  }
  // the slices' images, up to nimg of them in one batched gridding launch,
  // each then phase-corrected into out
  bool first = true;
  const int64_t nn = (int64_t)K->N * K->N;
  std::vector<sepw_plan> plans;
  std::vector<const sepw_c64*> vs;
  std::vector<const float*> wts;
  std::vector<sepw_c64*> imgs;
  std::vector<int> idx;
  for (int j0 = 0; j0 < ws->ns;) {
    plans.clear();
    vs.clear();
    wts.clear();
    imgs.clear();
    idx.clear();
    for (; j0 < ws->ns && (int)idx.size() < ws->nimg; ++j0) {
      if (!ws->plans[j0]) continue;
      plans.push_back(static_cast<sepw_plan>(ws->plans[j0]));
      vs.push_back(reinterpret_cast<const sepw_c64*>(ws->vis + ws->off[j0]));
      wts.push_back(nullptr);
      imgs.push_back(reinterpret_cast<sepw_c64*>(ws->img + (int64_t)idx.size() * nn));
      idx.push_back(j0);
    }
    if (idx.empty()) break;
    // FP32 tiled: grids only, then per slice the FFT and one pass for the
    // correction and the slice phase; otherwise images, then the phase
    const bool fused = K->prm.precision == SEPW_FP32 && !wide_support(K->S);
    const int npow = (flags & SEPW_MUL_N) ? 1 : ((flags & SEPW_DIV_N) ? -1 : 0);
    int rc = fused ? grid_batched((int32_t)idx.size(), plans.data(), vs.data(), wts.data(),
                                  imgs.data(), kGridNoTransform, s)
                   : sepw_grid_batched((int32_t)idx.size(), plans.data(), vs.data(), wts.data(),
                                       imgs.data(), flags, hip_stream);
    if (rc != SEPW_OK) return rc;
    for (size_t k = 0; k < idx.size(); ++k) {
      float2* img = reinterpret_cast<float2*>(imgs[k]);
      if (fused) {
        Stage st(SEPW_STAGE_FFT, s);
        rc = fft_exec(static_cast<Plan*>(plans[k])->K, img, HIPFFT_BACKWARD, s);
        if (rc != SEPW_OK) return rc;
      }
      Stage st(SEPW_STAGE_CORRECT, s);
      SEPW_TRY(launch_slice_phase(img, out, K->N, K->fov, ws->centre[idx[k]], +1, !first,
                                  fused ? K->c1 : nullptr, npow, s));
      first = false;
    }
  }
  if (first) SEPW_TRY(launch_zero_c64(out, (int64_t)K->N * K->N, s));
  return SEPW_OK;
}

int sepw_wstack_degrid(sepw_wstack ws, const sepw_c64* image, sepw_c64* vis_out, uint32_t flags,
                       void* hip_stream) {
  if (!ws || !image || (!vis_out && ws->nvis > 0)) return SEPW_ERR_ARG;
  if ((flags & ~SEPW_DIV_N) != 0) return SEPW_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Kernels* K = ws->K;
  if (K->prm.precision != SEPW_FP32 || ws->nimg < 2 || wide_support(K->S)) {
    for (int j = 0; j < ws->ns; ++j) {
      if (!ws->plans[j]) continue;
      {
        Stage st(SEPW_STAGE_CORRECT, s);
        SEPW_TRY(launch_slice_phase(reinterpret_cast<const float2*>(image), ws->img, K->N, K->fov,
                                    ws->centre[j], -1, false, nullptr, 0, s));
      }
      int rc = sepw_degrid(static_cast<sepw_plan_s*>(ws->plans[j]),
                           reinterpret_cast<const sepw_c64*>(ws->img),
                           reinterpret_cast<sepw_c64*>(ws->vis + ws->off[j]), flags, hip_stream);
      if (rc != SEPW_OK) return rc;
    }
  } else {
    // FP32: per slice one pass for the slice phase and the correction into
    // its own image, then the slices' degridding in batches of up to nimg
    const int64_t nn = (int64_t)K->N * K->N;
    const int npow = (flags & SEPW_DIV_N) ? -1 : 0;
    std::vector<Plan*> plans;
    std::vector<float2*> outs;
    for (int j0 = 0; j0 < ws->ns;) {
      plans.clear();
      outs.clear();
      for (; j0 < ws->ns && (int)plans.size() < ws->nimg; ++j0) {
        if (!ws->plans[j0]) continue;
        Stage st(SEPW_STAGE_CORRECT, s);
        SEPW_TRY(launch_slice_phase(reinterpret_cast<const float2*>(image),
                                    ws->img + (int64_t)plans.size() * nn, K->N, K->fov,
                                    ws->centre[j0], -1, false, K->c1, npow, s));
        plans.push_back(ws->plans[j0]);
        outs.push_back(ws->vis + ws->off[j0]);
      }
      if (plans.empty()) break;
      int rc = degrid_images_batched(K, plans.data(), (int)plans.size(), ws->img, npow,
                                     outs.data(), s, true);
      if (rc != SEPW_OK) return rc;
    }
  }
  if (ws->nvis > 0) {
    Stage st(SEPW_STAGE_GATHER, s);
    SEPW_TRY(launch_slice_return(ws->vis, ws->order, ws->nvis, reinterpret_cast<float2*>(vis_out),
                                 s));
  }
  return SEPW_OK;
}

int sepw_free_wsnap(sepw_wsnap ws) {
  if (!ws) return SEPW_ERR_ARG;
  destroy_wsnap(ws);
  return SEPW_OK;
}

int sepw_wsnap_create(sepw_kernels k, int32_t n_snap, const int64_t* offsets, const double* u,
                      const double* v, const double* w, int64_t* n_dropped, void* hip_stream,
                      sepw_wsnap* out) {
  if (!out) return SEPW_ERR_ARG;
  *out = nullptr;
  if (!k || n_snap < 1 || n_snap > (1 << 20) || !offsets) return SEPW_ERR_ARG;
  if (offsets[0] != 0) return SEPW_ERR_ARG;
  for (int i = 0; i < n_snap; ++i)
    if (offsets[i + 1] < offsets[i]) return SEPW_ERR_ARG;
  const int64_t nvis = offsets[n_snap];
  if (nvis > 2147483646LL) return SEPW_ERR_ARG;
  if (nvis > 0 && (!u || !v || !w)) return SEPW_ERR_ARG;
  if (k->facet) return SEPW_ERR_UNSUPPORTED;
  if (device_count() < 1) return SEPW_ERR_NO_DEVICE;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  sepw_wsnap_s* W = new (std::nothrow) sepw_wsnap_s();
  if (!W) return SEPW_ERR_OOM;
  W->K = k;
  W->ns = n_snap;
  W->nvis = nvis;
  W->off.assign(offsets, offsets + n_snap + 1);
  W->d0.assign(2 * (size_t)n_snap, 0.0);
  W->plans.assign(n_snap, nullptr);
  W->nimg = batch_images(k->N, n_snap);
  int rc = map_hip(dalloc(&W->img, (int64_t)W->nimg * k->N * k->N));
  if (rc == SEPW_OK) rc = wsnap_build(W, u, v, w, s);
  int64_t dropped = 0;
  for (int i = 0; i < n_snap && rc == SEPW_OK && n_dropped; ++i) {
    if (!W->plans[i]) continue;
    int64_t d = 0;
    rc = read_dropped(W->plans[i], &d, s);
    dropped += d;
  }
  if (rc != SEPW_OK) {
    destroy_wsnap(W);
    return rc;
  }
  if (n_dropped) *n_dropped = dropped;
  *out = W;
  return SEPW_OK;
}

int sepw_wsnap_plane(sepw_wsnap ws, int32_t snapshot, double* d0, double* h) {
  if (!ws || snapshot < 0 || snapshot >= ws->ns || !d0) return SEPW_ERR_ARG;
  d0[0] = ws->d0[2 * (size_t)snapshot];
  d0[1] = ws->d0[2 * (size_t)snapshot + 1];
  if (h) *h = ws->h;
  return SEPW_OK;
}

int sepw_wsnap_grid(sepw_wsnap ws, const sepw_c64* vis, const float* weight, sepw_c64* image_out,
                    uint32_t flags, void* hip_stream) {
  if (!ws || !image_out || (!vis && ws->nvis > 0)) return SEPW_ERR_ARG;
  if ((flags & ~(SEPW_MUL_N | SEPW_DIV_N)) != 0) return SEPW_ERR_ARG;
  if ((flags & SEPW_MUL_N) && (flags & SEPW_DIV_N)) return SEPW_ERR_ARG;
  Kernels* K = ws->K;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int N = K->N;
  float2* out = reinterpret_cast<float2*>(image_out);
  {
    Stage st(SEPW_STAGE_FILL, s);
    SEPW_TRY(launch_zero_c64(out, (int64_t)N * N, s));
  }
  // the snapshots' images, up to nimg of them in one batched gridding launch
  // (independent jobs on the same tables), each then reprojected into out
  std::vector<sepw_plan> plans;
  std::vector<const sepw_c64*> vs;
  std::vector<const float*> ws_;
  std::vector<sepw_c64*> imgs;
  std::vector<int> idx;
  for (int i0 = 0; i0 < ws->ns;) {
    plans.clear();
    vs.clear();
    ws_.clear();
    imgs.clear();
    idx.clear();
    for (; i0 < ws->ns && (int)idx.size() < ws->nimg; ++i0) {
      if (!ws->plans[i0]) continue;
      const int64_t o = ws->off[i0];
      plans.push_back(static_cast<sepw_plan>(ws->plans[i0]));
      vs.push_back(vis + o);
      ws_.push_back(weight ? weight + o : nullptr);
      imgs.push_back(reinterpret_cast<sepw_c64*>(ws->img + (int64_t)idx.size() * N * N));
      idx.push_back(i0);
    }
    if (idx.empty()) break;
    int rc = sepw_grid_batched((int32_t)idx.size(), plans.data(), vs.data(), ws_.data(),
                               imgs.data(), 0u, hip_stream);
    if (rc != SEPW_OK) return rc;
    Stage st(SEPW_STAGE_CORRECT, s);
    for (size_t j = 0; j < idx.size(); ++j)
      SEPW_TRY(launch_snap_reproject(reinterpret_cast<const float2*>(imgs[j]), out, N, K->fov,
                                     ws->d0[2 * (size_t)idx[j]], ws->d0[2 * (size_t)idx[j] + 1],
                                     true, s));
  }
  const int npow = (flags & SEPW_MUL_N) ? 1 : ((flags & SEPW_DIV_N) ? -1 : 0);
  if (npow) {
    Stage st(SEPW_STAGE_CORRECT, s);
    SEPW_TRY(launch_snap_npow(out, N, K->fov, npow, s));
  }
  return SEPW_OK;
}

int sepw_wsnap_degrid(sepw_wsnap ws, const sepw_c64* image, sepw_c64* vis_out, uint32_t flags,
                      void* hip_stream) {
  if (!ws || !image || (!vis_out && ws->nvis > 0)) return SEPW_ERR_ARG;
  if ((flags & ~SEPW_DIV_N) != 0) return SEPW_ERR_ARG;
  Kernels* K = ws->K;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int N = K->N;
  const int npow = (flags & SEPW_DIV_N) ? -1 : 0;
  if (K->prm.precision != SEPW_FP32 || ws->nimg < 2 || wide_support(K->S)) {
    for (int i = 0; i < ws->ns; ++i) {
      Plan* p = ws->plans[i];
      if (!p) continue;
      {
        Stage st(SEPW_STAGE_CORRECT, s);
        SEPW_TRY(launch_snap_reproject_adjoint(reinterpret_cast<const float2*>(image), ws->img, N,
                                               K->fov, ws->d0[2 * (size_t)i],
                                               ws->d0[2 * (size_t)i + 1], npow, nullptr, s));
      }
      int rc = sepw_degrid(static_cast<sepw_plan>(p), reinterpret_cast<const sepw_c64*>(ws->img),
                           vis_out + ws->off[i], 0u, hip_stream);
      if (rc != SEPW_OK) return rc;
    }
    return SEPW_OK;
  }
  // FP32: per snapshot the transposed reprojection into its own image (with
  // the image correction in the same pass), then the snapshots' degridding in
  // batches of up to nimg
  std::vector<int> idx;
  std::vector<Plan*> plans;
  std::vector<float2*> outs;
  for (int i0 = 0; i0 < ws->ns;) {
    idx.clear();
    for (; i0 < ws->ns && (int)idx.size() < ws->nimg; ++i0)
      if (ws->plans[i0]) idx.push_back(i0);
    if (idx.empty()) break;
    plans.clear();
    outs.clear();
    for (size_t j = 0; j < idx.size(); ++j) {
      const int i = idx[j];
      Stage st(SEPW_STAGE_CORRECT, s);
      SEPW_TRY(launch_snap_reproject_adjoint(reinterpret_cast<const float2*>(image),
                                             ws->img + (int64_t)j * N * N, N, K->fov,
                                             ws->d0[2 * (size_t)i], ws->d0[2 * (size_t)i + 1],
                                             npow, K->c1, s));
      plans.push_back(ws->plans[i]);
      outs.push_back(reinterpret_cast<float2*>(vis_out + ws->off[i]));
    }
    int rc = degrid_images_batched(K, plans.data(), (int)idx.size(), ws->img, 0, outs.data(), s,
                                   true);
    if (rc != SEPW_OK) return rc;
  }
  return SEPW_OK;
}

}  // extern "C"
