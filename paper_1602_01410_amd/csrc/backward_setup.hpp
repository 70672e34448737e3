// Final steps of the reverse pass: adjoint of the initialisation (-> dL/dy),
// the lambda-gradient reduction and the map of the spectral blur gradient to
// the kernel taps.  Included by the host translation unit only.
#pragma once
#include "backward.hpp"

namespace dcv {

// --------------------------------------------------------------------------
// initialisation adjoint: ytilde^0 = E(y), v^0 = D ytilde^0, d^0 = 0
// --------------------------------------------------------------------------

// e = zb + D^T vb on unobserved pixels; observed pixels take D^T vb into yb
__global__ void init_adj_a_kernel(const ImgMeta* meta, const uint8_t* __restrict__ mask, const float2* vb,
                                  const float* zb, float* yb, float* e) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  const long long n = (long long)mt.m * mt.n;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p / mt.n), j = (int)(p - (long long)i * mt.n);
    const long long c = mt.px + p;
    const float2 w = vb[c];
    const float wl = vb[mt.px + (long long)i * mt.n + (j == 0 ? mt.n - 1 : j - 1)].x;
    const float wu = vb[mt.px + (long long)(i == 0 ? mt.m - 1 : i - 1) * mt.n + j].y;
    const float a = wl - w.x + wu - w.y;
    if (observed(mt, mask, i, j)) { yb[c] += a; e[c] = 0.f; }
    else e[c] = zb[c] + a;
  }
}

// band pixels copy the nearest central pixel: gather their adjoints onto it;
// then observed central pixels take it into yb, unobserved central pixels
// add it to the adjoint of the mean (per-block partial)
__global__ void __launch_bounds__(kNT) init_adj_b_kernel(const ImgMeta* meta, const uint8_t* __restrict__ mask,
                                                         const float* e, float* yb, double* mean_part,
                                                         int nblk) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  const int b = mt.b, M = mt.m, N = mt.n;
  const long long n = (long long)M * N;
  double macc = 0.0;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p / N), j = (int)(p - (long long)i * N);
    if (!(i >= b && i < M - b && j >= b && j < N - b)) continue;
    double s = e[mt.px + p];
    const int i_lo = (i == b) ? 0 : i, i_hi = (i == M - b - 1) ? M - 1 : i;
    const int j_lo = (j == b) ? 0 : j, j_hi = (j == N - b - 1) ? N - 1 : j;
    if (i_lo != i_hi || j_lo != j_hi) {
      for (int ii = i_lo; ii <= i_hi; ++ii)
        for (int jj = j_lo; jj <= j_hi; ++jj) {
          if (ii >= b && ii < M - b && jj >= b && jj < N - b) continue;   // central: not band
          if (observed(mt, mask, ii, jj)) continue;
          s += e[mt.px + (long long)ii * N + jj];
        }
    }
    if (observed(mt, mask, i, j)) yb[mt.px + p] += (float)s;
    else macc += s;
  }
  __shared__ double red[3 * (kNT / 64)];
  double z0 = 0, z1 = 0;
  block_sum3(macc, z0, z1, red);
  if (threadIdx.x == 0) mean_part[(long long)img * nblk + blockIdx.x] = macc;
}

// observed pixels: + mean adjoint / count; unobserved: 0
__global__ void __launch_bounds__(kNT) init_adj_c_kernel(const ImgMeta* meta, const uint8_t* __restrict__ mask,
                                                         const double* mean_part, int nblk, const double* obs_part,
                                                         int nobs, const float* yb, float* grad_y) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  // the mean adjoint, spread over the observed pixels (their count comes
  // from the forward run's observed-sum partials: sum, count per block)
  __shared__ float add;
  if (threadIdx.x == 0) {
    double s = 0, c = 0;
    for (int k = 0; k < nblk; ++k) s += mean_part[(long long)img * nblk + k];
    for (int k = 0; k < nobs; ++k) c += obs_part[2 * ((long long)img * nobs + k) + 1];
    add = c > 0 ? (float)(s / c) : 0.f;
  }
  __syncthreads();
  for (int i = blockIdx.x; i < mt.m; i += gridDim.x) {
    const RowObs ro = row_observed(mt, i);
    const uint8_t* mrow = ro.explicit_mask ? mask + mt.px + (long long)i * mt.n : nullptr;
    for (int j = threadIdx.x; j < mt.n; j += kNT) {
      const long long q = mt.px + (long long)i * mt.n + j;
      grad_y[q] = pixel_observed(mt, ro, mrow, j) ? yb[q] + add : 0.f;
    }
  }
}

// dL/dh[b+p][b+q] = (1/(m'n')) sum_k w(kx) Re(S_k exp(-2 pi i (ky p / m' + kx q / n')))
// over the stored half spectrum (w = 1 for kx = 0 and kx = n'/2, 2 otherwise:
// S is Hermitian), in two separable stages: T[ky][q] = sum_kx w S_k
// exp(-2 pi i kx q / n'), then sum_ky Re(T[ky][q] exp(-2 pi i ky p / m')).
// FP64 throughout, with exact phase tables (index products reduced modulo
// the length).  Stage 1: one thread per (ky, q); T has `tstride` entries per
// image.
__global__ void __launch_bounds__(kNT) grad_taps_rows_kernel(const ImgMeta* meta, const double2* __restrict__ S,
                                                            const double2* __restrict__ tw64, double2* T,
                                                            long long tstride) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  const int K = 2 * mt.b + 1;
  const int t = blockIdx.x * kNT + threadIdx.x;
  if (t >= mt.m * K) return;
  const int ky = t / K, qi = t - ky * K;
  const int qq = qi - mt.b, qn = qq < 0 ? qq + mt.n : qq;
  const double2* TN = tw64 + mt.twr;   // exp(-2 pi i k / n'), k < n'
  double ar = 0.0, ai = 0.0;
  int ph = 0;   // kx * qn mod n', stepped
  for (int kx = 0; kx < mt.nh; ++kx) {
    const double2 sv = S[mt.hh + ((long long)(kx >> mt.logC) * mt.m + ky) * mt.C + (kx & (mt.C - 1))];
    const double2 e = TN[ph];
    const double w = (kx == 0 || 2 * kx == mt.n) ? 1.0 : 2.0;
    ar += w * (sv.x * e.x - sv.y * e.y);
    ai += w * (sv.x * e.y + sv.y * e.x);
    ph += qn;
    if (ph >= mt.n) ph -= mt.n;
  }
  T[img * tstride + t] = make_double2(ar, ai);
}

// Stage 2: one workgroup per (tap, image), a sum over the m' rows.
__global__ void __launch_bounds__(kNT) grad_taps_cols_kernel(const ImgMeta* meta, const double2* __restrict__ T,
                                                            long long tstride, const double2* __restrict__ tw64,
                                                            float* grad_h, const long long* hoff) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  const int K = 2 * mt.b + 1;
  const int t = blockIdx.x;
  if (t >= K * K) return;
  const int pi = t / K, qi = t % K;
  const int pp = pi - mt.b, pm = pp < 0 ? pp + mt.m : pp;
  const double2* TM = tw64 + mt.twc;   // exp(-2 pi i k / m'), k < m'
  double acc = 0.0;
  int ph = (int)(((long long)threadIdx.x * pm) % mt.m);          // ky * pm mod m', stepped
  const int step = (int)(((long long)kNT * pm) % mt.m);
  for (int ky = threadIdx.x; ky < mt.m; ky += kNT) {
    const double2 v = T[img * tstride + (long long)ky * K + qi];
    const double2 e = TM[ph];
    acc += v.x * e.x - v.y * e.y;
    ph += step;
    if (ph >= mt.m) ph -= mt.m;
  }
  __shared__ double red[3 * (kNT / 64)];
  double z0 = 0, z1 = 0;
  block_sum3(acc, z0, z1, red);
  if (threadIdx.x == 0) grad_h[hoff[img] + t] = (float)(acc / ((double)mt.m * (double)mt.n));
}

// per image: sum of the per-tile dL/dlambda partials
__global__ void __launch_bounds__(kNT) lam_reduce_kernel(const ImgMeta* meta, const double* part, float* out) {
  const int img = blockIdx.x;
  const ImgMeta mt = meta[img];
  double a = 0, z0 = 0, z1 = 0;
  for (int t = threadIdx.x; t < mt.nrt; t += kNT) a += part[mt.rt0 + t];
  __shared__ double red[3 * (kNT / 64)];
  block_sum3(a, z0, z1, red);
  if (threadIdx.x == 0) out[img] = (float)a;
}

}  // namespace dcv
