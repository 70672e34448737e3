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
                                                         const double* mean_part, int nblk, const float* yb,
                                                         float* grad_y) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  const long long n = (long long)mt.m * mt.n;
  __shared__ double tot[2];
  if (threadIdx.x == 0) {
    double s = 0;
    for (int k = 0; k < nblk; ++k) s += mean_part[(long long)img * nblk + k];
    tot[0] = s;
  }
  // count observed pixels
  double cnt = 0;
  for (long long p = threadIdx.x; p < n; p += kNT) {
    const int i = (int)(p / mt.n), j = (int)(p - (long long)i * mt.n);
    if (observed(mt, mask, i, j)) cnt += 1.0;
  }
  __shared__ double red[3 * (kNT / 64)];
  double z0 = 0, z1 = 0;
  block_sum3(cnt, z0, z1, red);
  if (threadIdx.x == 0) tot[1] = cnt;
  __syncthreads();
  const float add = tot[1] > 0 ? (float)(tot[0] / tot[1]) : 0.f;
  for (long long p = threadIdx.x; p < n; p += kNT) {
    const int i = (int)(p / mt.n), j = (int)(p - (long long)i * mt.n);
    grad_y[mt.px + p] = observed(mt, mask, i, j) ? yb[mt.px + p] + add : 0.f;
  }
}

// Hermitian completion of the accumulated half spectrum S into a full
// complex m' x n' grid (for the final transform to the kernel taps)
__global__ void unpack_half_kernel(const ImgMeta* meta, const float2* __restrict__ S, float2* grid,
                                   const long long* goff) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  const long long n = (long long)mt.m * mt.n;
  float2* g = grid + goff[img];
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int ky = (int)(p / mt.n), kx = (int)(p - (long long)ky * mt.n);
    float2 v;
    if (kx < mt.nh) {
      v = S[mt.hh + ((long long)(kx / mt.C) * mt.m + ky) * mt.C + kx % mt.C];
    } else {
      const int kx2 = mt.n - kx, ky2 = ky == 0 ? 0 : mt.m - ky;
      const float2 w = S[mt.hh + ((long long)(kx2 / mt.C) * mt.m + ky2) * mt.C + kx2 % mt.C];
      v = make_float2(w.x, -w.y);
    }
    g[p] = v;
  }
}

// dL/dh[b+p][b+q] = Re(F(S))[p mod m', q mod n'] / (m' n')
__global__ void gather_taps_kernel(const ImgMeta* meta, const float2* grid, const long long* goff,
                                   const long long* hoff, float* grad_h) {
  const int img = blockIdx.x;
  const ImgMeta mt = meta[img];
  const int K = 2 * mt.b + 1;
  const float2* g = grid + goff[img];
  const float inv = 1.0f / ((float)mt.m * (float)mt.n);
  for (int t = threadIdx.x; t < K * K; t += blockDim.x) {
    const int pp = t / K - mt.b, qq = t % K - mt.b;
    const int i = ((pp % mt.m) + mt.m) % mt.m, j = ((qq % mt.n) + mt.n) % mt.n;
    grad_h[hoff[img] + t] = g[(long long)i * mt.n + j].x * inv;
  }
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
