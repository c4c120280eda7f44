// Kernel-table generation: taper samples and the oversampled 1D GCF tables.
//
// Section 3 approximates the W screen g_w(l, m) = exp(2 pi i w (n - 1)) by the
// separable g1_w(l) g1_w(m) with g1_w(l) = exp(2 pi i w [-l^2/2 - gamma l^4]);
// Section 4.1's facet screens have the same form with coefficient a_l (a_m) on
// l^2 and none on l^4.  Combined with the separable taper c1 (Section 2's
// anti-aliasing function, Section 3's separability assumption) each axis needs
// one oversampled 1D table per w-plane (Section 2: oversampled lookup tables).
//
// Entry (k, fi, s) is the GCF at offset Delta = s - S/2 - f/O cells, f = fi - O/2,
// sampled as the inverse of the centred image <- grid transform over the N
// pixels:
//   T = (1/N) sum_p c1(l_p) exp(-2 pi i w_k (a l_p^2 + b l_p^4)) exp(-2 pi i Delta (p - N/2)/N)
// Everything is FP64 (phase, argument reduction, sincos, sum); the result is
// stored complex64.  One workgroup per (plane, sub-cell row); threads stride
// over pixels and the S partial sums are reduced across the workgroup.
#include "internal.h"

namespace sepw {

namespace {

constexpr int kTabThreads = 256;

__global__ void taper_kernel(const double* __restrict__ coef, int ncoef, double inv_norm, int N,
                             double* __restrict__ c1) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  double x = 2.0 * (double)(p - N / 2) / (double)N;
  // sum_j coef_j sqrt(2j + 1/2) P_{2j}(x), Legendre recurrence in FP64
  double pm1 = 1.0, pc = x;
  double acc = coef[0] * sqrt(0.5);
  int nmax = 2 * (ncoef - 1);
  for (int n = 1; n < nmax; ++n) {
    double pn = ((2 * n + 1) * x * pc - n * pm1) / (n + 1);
    pm1 = pc;
    pc = pn;
    int deg = n + 1;
    if ((deg & 1) == 0) acc += coef[deg / 2] * sqrt(deg + 0.5) * pc;
  }
  c1[p] = acc * inv_norm;
}

__global__ void ones_kernel(double* c1, int N) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < N) c1[p] = 1.0;
}

__device__ inline double block_sum(double v, double* sh) {
  // wave64 reduction, then across the workgroup's waves through LDS
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < kTabThreads / 64; ++i) t += sh[i];
  return t;
}

// SMAX: taps held per thread (16 for the tiled path, 32 above it)
template <int SMAX>
__global__ __launch_bounds__(kTabThreads) void table_kernel(
    const double* __restrict__ c1, int N, double fov, int P, int O, int S, double w_lo,
    double w_hi, double a, double b, float2* __restrict__ out) {
  __shared__ double sh[kTabThreads / 64];
  const int k = blockIdx.x / O;
  const int fi = blockIdx.x % O;
  const int f = fi - O / 2;
  const int h = S / 2;
  const double wk = w_lo + ((double)k + 0.5) * (w_hi - w_lo) / (double)P;
  const int64_t period = (int64_t)O * N;
  double acc_re[SMAX], acc_im[SMAX];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) acc_re[s] = acc_im[s] = 0.0;

  for (int p = threadIdx.x; p < N; p += kTabThreads) {
    const double l = (double)(p - N / 2) * fov / (double)N;
    const double l2 = l * l;
    const double cyc = wk * (a * l2 + b * l2 * l2);     // phase in cycles
    const double frac = cyc - rint(cyc);
    double sp, cp;
    sincospi(-2.0 * frac, &sp, &cp);
    const double are = c1[p] * cp, aim = c1[p] * sp;
    const int64_t dp = p - N / 2;
    // Twiddle of tap s: exp(-2 pi i m_s / (O N)) with m_s = (O (s - h) - f) dp.
    // Consecutive taps differ by the factor exp(-2 pi i dp / N), so only the
    // first twiddle and that ratio are evaluated (integer arguments reduced
    // exactly), the others by complex multiplication in FP64.
    int64_t r0 = (((int64_t)O * (-h) - f) * dp) % period;
    if (r0 < 0) r0 += period;
    int64_t q = dp % N;
    if (q < 0) q += N;
    double te, tc, rs, rc;
    sincospi(-2.0 * (double)r0 / (double)period, &te, &tc);
    sincospi(-2.0 * (double)q / (double)N, &rs, &rc);
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      if (s < S) {
        acc_re[s] += are * tc - aim * te;
        acc_im[s] += are * te + aim * tc;
        const double nc = tc * rc - te * rs;
        te = tc * rs + te * rc;
        tc = nc;
      }
    }
  }
  const double invN = 1.0 / (double)N;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    if (s < S) {
      double re = block_sum(acc_re[s], sh);
      double im = block_sum(acc_im[s], sh);
      if (threadIdx.x == 0)
        out[((int64_t)k * O + fi) * S + s] = make_float2((float)(re * invN), (float)(im * invN));
    }
  }
}

// ---- derived layouts of the tables (same values, kernel-friendly storage) ----

__global__ void pad_table_kernel(const float2* __restrict__ tab, const float* __restrict__ scale,
                                 int O, int S, int alternate, float2* __restrict__ out) {
  // one block per (plane, sub-cell row): out row of L entries
  const int L = padded_len(S), c = kRegion + 1 - S;
  const int row = blockIdx.x, k = row / O;
  const float f0 = scale ? scale[k] : 1.f;
  for (int x = threadIdx.x; x < L; x += blockDim.x) {
    const int s = x - (c - 1);
    float2 v = make_float2(0.f, 0.f);
    if (s >= 0 && s < S) {
      const float f = (alternate && (s & 1)) ? -f0 : f0;
      v = tab[(int64_t)row * S + s];
      v.x *= f;
      v.y *= f;
    }
    out[(int64_t)row * L + x] = v;
  }
}

// 16-bit padded tables: row of L dwords per (plane, sub-cell row), tap s of
// the row at c - 1 + s as (Re, Im) rounded to nearest even (FP16, or BF16 high
// parts); BF16 low parts, bf16(x - hi), at + tab_len.
__device__ inline uint32_t f16_bits(float x) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
}
__device__ inline uint32_t bf16_bits(float x) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ inline float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

__global__ void lp_table_kernel(const float2* __restrict__ tab, int S, int bf16, int tab_len,
                                uint32_t* __restrict__ out) {
  const int L = padded_len(S), c = kRegion + 1 - S;
  const int row = blockIdx.x;
  for (int x = threadIdx.x; x < L; x += blockDim.x) {
    const int s = x - (c - 1);
    float2 t = make_float2(0.f, 0.f);
    if (s >= 0 && s < S) t = tab[(int64_t)row * S + s];
    const int64_t i = (int64_t)row * L + x;
    if (bf16) {
      const uint32_t hr = bf16_bits(t.x), hi = bf16_bits(t.y);
      out[i] = hr | (hi << 16);
      out[i + tab_len] = bf16_bits(t.x - bf16_value(hr)) | (bf16_bits(t.y - bf16_value(hi)) << 16);
    } else {
      out[i] = f16_bits(t.x) | (f16_bits(t.y) << 16);
    }
  }
}

}  // namespace

hipError_t launch_taper(const double* d_coef, int ncoef, double norm, int N, double* c1,
                        hipStream_t s) {
  hipLaunchKernelGGL(taper_kernel, dim3((N + 255) / 256), dim3(256), 0, s, d_coef, ncoef,
                     1.0 / norm, N, c1);
  return hipGetLastError();
}

hipError_t launch_ones(double* c1, int N, hipStream_t s) {
  hipLaunchKernelGGL(ones_kernel, dim3((N + 255) / 256), dim3(256), 0, s, c1, N);
  return hipGetLastError();
}

hipError_t launch_pad_table(const float2* tab, const float* scale, int P, int O, int S, float2* out,
                            hipStream_t s, bool alternate) {
  hipLaunchKernelGGL(pad_table_kernel, dim3(P * O), dim3(32), 0, s, tab, scale, O, S,
                     alternate ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_lp_table(const float2* tab, int P, int O, int S, int bf16, int tab_len,
                           uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(lp_table_kernel, dim3(P * O), dim3(32), 0, s, tab, S, bf16, tab_len, out);
  return hipGetLastError();
}

hipError_t launch_tables(const double* c1, int N, double fov, int P, int O, int S, double w_lo,
                         double w_hi, double a, double b, float2* out, hipStream_t s) {
  if (S <= 16) {
    hipLaunchKernelGGL(table_kernel<16>, dim3(P * O), dim3(kTabThreads), 0, s, c1, N, fov, P, O, S,
                       w_lo, w_hi, a, b, out);
  } else {
    hipLaunchKernelGGL(table_kernel<32>, dim3(P * O), dim3(kTabThreads), 0, s, c1, N, fov, P, O, S,
                       w_lo, w_hi, a, b, out);
  }
  return hipGetLastError();
}

}  // namespace sepw
