// Generation of the correction table F_w - F~_w (Section 6's proposal: store
// the difference between the exact GCF and its separable approximation as a
// small full 2D table).
//
// Entry (k, fu, fv, su, sv) is the double sum over the N x N image pixels
//   C = (1/N^2) sum_{q,p} A_k(q, p) E_{d_i}(p) E_{d_j}(q),
//   A_k(q, p) = c1(l_p) c1(m_q) [exp(2 pi i w_k (n - 1)) - exp(-2 pi i w_k (phi_u(l_p) + phi_v(m_q)))],
//   E_d(p) = exp(-2 pi i d (p - N/2) / (O_c N)),
// with phi(l) = a l^2 + b l^4 the separable screen's exponent per axis, d_i =
// (su - h_c) O_c - (fu - O_c/2) the tap offset in 1/O_c cells (d_j likewise
// with sv, fv) and n - 1 written as -(l^2 + m^2) / (1 + n), which is equal and
// free of cancellation.  Everything is FP64; the table is stored complex64.
//
// The screen is even in l and in m (the taper must be symmetric), so the sums
// fold about the centre: pixels N/2 + c and N/2 - c (0 < c < N/2) share A and
// their weights add to Wt_|d|(c) = 2 cos(2 pi d c / (O_c N)) (Wt(0) = 1);
// pixel 0 has no partner and weight e_d = exp(i pi d / O_c).  With folded
// columns c in [0, N/2] (c = N/2 standing for pixel 0) and D = max |d| + 1:
//   Rcos[b][c] = sum_{r < N/2} Wt_b(r) A(N/2 + r, p(c))     (fold_kernel; b = |d_j|)
//   A0[c]      = A(0, p(c))                                 (the unpaired row)
//   M[a][b]    = sum_{c < N/2} Wt_a(c) Rcos[b][c],  V[a] = sum_{c < N/2} Wt_a(c) A0[c]
//   C(i, j)    = (M[|d_i|][|d_j|] + e_{d_j} V[|d_i|] + e_{d_i} (Rcos[|d_j|][N/2] + e_{d_j} A0[N/2])) / N^2
// which takes a quarter of the screen evaluations and an eighth of the
// multiply-adds of the direct double sum.
#include "internal.h"

namespace sepw {

namespace {

constexpr int kFoldWaves = 4;
constexpr int kMaxDW = kCorrMaxD / kFoldWaves;   // |d| values per wave

// Wt[a][r] = 2 cos(2 pi a r / (Oc N)) (1 at r = 0), integer argument reduced exactly.
__global__ void corr_weights_kernel(int D, int N, int Oc, double* __restrict__ wt) {
  const int half = N / 2;
  const int64_t total = (int64_t)D * half;
  const int64_t period = (int64_t)Oc * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(i / half), r = (int)(i - (int64_t)a * half);
    const int64_t m = ((int64_t)a * r) % period;
    wt[i] = r == 0 ? 1.0 : 2.0 * cospi(2.0 * (double)m / (double)period);
  }
}

struct ScreenCol {
  double l2, phi_u, c1p;
};

// A_k(q, p) for the lane's column (l^2, phi_u and c1 of pixel p precomputed).
__device__ inline double2 screen(const ScreenCol& col, int q, const double* __restrict__ c1, int N,
                                 double fov, double wk, double a_v, double b_v) {
  const double m = (double)(q - N / 2) * fov / (double)N;
  const double m2 = m * m;
  const double r2 = col.l2 + m2;
  const double n = sqrt(1.0 - r2);
  const double ce = wk * (-r2 / (1.0 + n));                        // exact screen, cycles
  const double cs = wk * (col.phi_u + (a_v * m2 + b_v * m2 * m2)); // separable exponent, cycles
  double se, cee, ss, css;
  sincospi(2.0 * (ce - rint(ce)), &se, &cee);
  sincospi(-2.0 * (cs - rint(cs)), &ss, &css);
  const double t = col.c1p * c1[q];
  return make_double2(t * (cee - css), t * (se - ss));
}

// Rcos[kb][b][c] and A0[kb][c] for 64 folded columns per workgroup.  The four
// waves take turns evaluating one folded row each (through LDS, double
// buffered) and each wave accumulates its own range of |d| values for all
// rows; the weights are wave-uniform (scalar loads).
__global__ __launch_bounds__(64 * kFoldWaves) void corr_fold_kernel(
    const double* __restrict__ c1, const double* __restrict__ wt, int N, double fov, int k0, int P,
    double w_lo, double w_hi, double a_u, double b_u, double a_v, double b_v, int D,
    double2* __restrict__ rcos, double2* __restrict__ a0) {
  __shared__ double2 As[2][kFoldWaves][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kb = blockIdx.y, k = k0 + kb;
  const double wk = w_lo + ((double)k + 0.5) * (w_hi - w_lo) / (double)P;
  const int half = N / 2, M1 = half + 1;
  const int c = blockIdx.x * 64 + lane;
  const bool col_ok = c < M1;
  const int p = c < half ? half + c : 0;
  ScreenCol col;
  {
    const double l = (double)(p - half) * fov / (double)N;
    col.l2 = l * l;
    col.phi_u = a_u * col.l2 + b_u * col.l2 * col.l2;
    col.c1p = col_ok ? c1[p] : 0.0;
  }
  const int dw = (D + kFoldWaves - 1) / kFoldWaves;
  const int b0 = wave * dw;
  double acc_re[kMaxDW], acc_im[kMaxDW];
#pragma unroll
  for (int i = 0; i < kMaxDW; ++i) acc_re[i] = acc_im[i] = 0.0;

  for (int r0 = 0, buf = 0; r0 < half; r0 += kFoldWaves, buf ^= 1) {
    const int r = r0 + wave;
    As[buf][wave][lane] = r < half ? screen(col, half + r, c1, N, fov, wk, a_v, b_v)
                                   : make_double2(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kFoldWaves; ++rr) {
      const int row = r0 + rr;
      if (row >= half) break;
      const double2 av = As[buf][rr][lane];
#pragma unroll
      for (int i = 0; i < kMaxDW; ++i) {
        if (i < dw && b0 + i < D) {
          const double wgt = wt[(int64_t)(b0 + i) * half + row];
          acc_re[i] += wgt * av.x;
          acc_im[i] += wgt * av.y;
        }
      }
    }
  }
  if (!col_ok) return;
  const int64_t base = (int64_t)kb * D * M1;
#pragma unroll
  for (int i = 0; i < kMaxDW; ++i)
    if (i < dw && b0 + i < D) rcos[base + (int64_t)(b0 + i) * M1 + c] = make_double2(acc_re[i], acc_im[i]);
  if (wave == 0) a0[(int64_t)kb * M1 + c] = screen(col, 0, c1, N, fov, wk, a_v, b_v);
}

// M[kb][a][b] and V[kb][a] (complex) for one plane per workgroup: 4 x 4
// output blocks per thread over 32-column LDS tiles of Wt, Rcos and A0.
constexpr int kTile = 32;
__global__ __launch_bounds__(256) void corr_matrix_kernel(const double* __restrict__ wt,
                                                          const double2* __restrict__ rcos,
                                                          const double2* __restrict__ a0, int N,
                                                          int D, double2* __restrict__ mv) {
  __shared__ double ws[kCorrMaxD][kTile];
  __shared__ double2 rs[kCorrMaxD + 1][kTile];
  const int kb = blockIdx.x, t = threadIdx.x;
  const int half = N / 2, M1 = half + 1;
  const double2* R = rcos + (int64_t)kb * D * M1;
  const double2* Z = a0 + (int64_t)kb * M1;
  const int ab = (t >> 4) * 4, bb = (t & 15) * 4;   // this thread's a and b blocks
  double mre[4][4], mim[4][4], vre = 0.0, vim = 0.0;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) mre[x][y] = mim[x][y] = 0.0;
  for (int c0 = 0; c0 < half; c0 += kTile) {
    for (int e = t; e < kCorrMaxD * kTile; e += 256) {
      const int a = e / kTile, cc = e % kTile, c = c0 + cc;
      const bool ok = a < D && c < half;
      ws[a][cc] = ok ? wt[(int64_t)a * half + c] : 0.0;
      rs[a][cc] = ok ? R[(int64_t)a * M1 + c] : make_double2(0.0, 0.0);
    }
    for (int cc = t; cc < kTile; cc += 256)
      rs[kCorrMaxD][cc] = c0 + cc < half ? Z[c0 + cc] : make_double2(0.0, 0.0);
    __syncthreads();
    for (int cc = 0; cc < kTile; ++cc) {
      double wa[4];
      double2 rb[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) wa[x] = ws[ab + x][cc];
#pragma unroll
      for (int y = 0; y < 4; ++y) rb[y] = rs[bb + y][cc];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          mre[x][y] += wa[x] * rb[y].x;
          mim[x][y] += wa[x] * rb[y].y;
        }
    }
    if (t < kCorrMaxD) {
      for (int cc = 0; cc < kTile; ++cc) {
        vre += ws[t][cc] * rs[kCorrMaxD][cc].x;
        vim += ws[t][cc] * rs[kCorrMaxD][cc].y;
      }
    }
    __syncthreads();
  }
  double2* out = mv + (int64_t)kb * D * (D + 1);   // rows a: M[a][0..D) then V[a]
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
      if (ab + x < D && bb + y < D)
        out[(int64_t)(ab + x) * (D + 1) + bb + y] = make_double2(mre[x][y], mim[x][y]);
  if (t < D) out[(int64_t)t * (D + 1) + D] = make_double2(vre, vim);
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// e_d = exp(i pi d / Oc)
__device__ inline double2 unpaired_weight(int d, int Oc) {
  double s, c;
  sincospi((double)d / (double)Oc, &s, &c);
  return make_double2(c, s);
}

// out[k][fu][fv][sv][su] from M, V, the last folded column of Rcos and A0.
__global__ void corr_assemble_kernel(const double2* __restrict__ mv, const double2* __restrict__ rcos,
                                     const double2* __restrict__ a0, int nkb, int k0, int N, int Sc,
                                     int Oc, int D, float2* __restrict__ out) {
  const int half = N / 2, M1 = half + 1, hc = Sc / 2;
  const int per = Oc * Oc * Sc * Sc;
  const int64_t total = (int64_t)nkb * per;
  const double inv = 1.0 / ((double)N * (double)N);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int kb = (int)(e / per);
    int r = (int)(e - (int64_t)kb * per);
    const int su = r % Sc;
    r /= Sc;
    const int sv = r % Sc;
    r /= Sc;
    const int fv = r % Oc;
    const int fu = r / Oc;
    const int di = (su - hc) * Oc - (fu - Oc / 2);
    const int dj = (sv - hc) * Oc - (fv - Oc / 2);
    const int ai = di < 0 ? -di : di, bj = dj < 0 ? -dj : dj;
    const double2* m = mv + (int64_t)kb * D * (D + 1);
    const double2 ei = unpaired_weight(di, Oc), ej = unpaired_weight(dj, Oc);
    const double2 rl = rcos[((int64_t)kb * D + bj) * M1 + half];
    const double2 zl = a0[(int64_t)kb * M1 + half];
    const double2 inner = make_double2(rl.x + (ej.x * zl.x - ej.y * zl.y), rl.y + (ej.x * zl.y + ej.y * zl.x));
    const double2 t1 = m[(int64_t)ai * (D + 1) + bj];
    const double2 t2 = cmul(ej, m[(int64_t)ai * (D + 1) + D]);
    const double2 t3 = cmul(ei, inner);
    out[(int64_t)(k0 + kb) * per + ((fu * Oc + fv) * Sc + sv) * Sc + su] =
        make_float2((float)((t1.x + t2.x + t3.x) * inv), (float)((t1.y + t2.y + t3.y) * inv));
  }
}

inline unsigned blocks_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (unsigned)b;
}

}  // namespace

int corr_dmax(int Sc, int Oc) { return (Sc / 2) * Oc + Oc / 2; }

// weights (padded to an even count so that the complex arrays after them stay
// 16-byte aligned), then per plane Rcos, A0 and M / V (complex = 2 doubles)
int64_t corr_wt_doubles(int N, int D) { return ((int64_t)D * (N / 2) + 1) & ~(int64_t)1; }

int64_t corr_tmp_doubles(int N, int Sc, int Oc, int nkb) {
  const int D = corr_dmax(Sc, Oc) + 1;
  const int64_t M1 = N / 2 + 1;
  return corr_wt_doubles(N, D) + 2 * (int64_t)nkb * ((int64_t)D * M1 + M1 + (int64_t)D * (D + 1));
}

hipError_t launch_corr_tables(const double* c1, int N, double fov, int P, double w_lo, double w_hi,
                              double a_u, double b_u, double a_v, double b_v, int Sc, int Oc,
                              int nkb, double* tmp, float2* out, hipStream_t s) {
  const int D = corr_dmax(Sc, Oc) + 1;
  if (D > kCorrMaxD || nkb < 1 || N < 2) return hipErrorInvalidValue;
  const int half = N / 2, M1 = half + 1;
  double* wt = tmp;
  double2* rcos = reinterpret_cast<double2*>(wt + corr_wt_doubles(N, D));
  double2* a0 = rcos + (int64_t)nkb * D * M1;
  double2* mv = a0 + (int64_t)nkb * M1;
  hipLaunchKernelGGL(corr_weights_kernel, dim3(blocks_for((int64_t)D * half, 256)), dim3(256), 0, s, D,
                     N, Oc, wt);
  hipError_t e = hipGetLastError();
  for (int k0 = 0; k0 < P && e == hipSuccess; k0 += nkb) {
    const int nk = P - k0 < nkb ? P - k0 : nkb;
    hipLaunchKernelGGL(corr_fold_kernel, dim3((unsigned)((M1 + 63) / 64), (unsigned)nk),
                       dim3(64 * kFoldWaves), 0, s, c1, wt, N, fov, k0, P, w_lo, w_hi, a_u, b_u, a_v,
                       b_v, D, rcos, a0);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(corr_matrix_kernel, dim3((unsigned)nk), dim3(256), 0, s, wt, rcos, a0, N, D,
                       mv);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(corr_assemble_kernel, dim3(blocks_for((int64_t)nk * Oc * Oc * Sc * Sc, 256)),
                       dim3(256), 0, s, mv, rcos, a0, nk, k0, N, Sc, Oc, D, out);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace sepw
