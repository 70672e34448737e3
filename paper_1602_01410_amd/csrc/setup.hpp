// Setup, initialisation and reduction kernels of the partial ADMM (blur
// spectrum, initial state, FP64 residuals) and the plain batched 2-D FFT used
// by the setup and the diagnostic entry point.  Included by the host
// translation unit only.
#pragma once
#include "kernels.hpp"

namespace dcv {

// ---------------------------------------------------------------------------
// plain batched 2-D FFT passes (setup of the blur spectrum, diagnostics)
// data: float2 [count][H][W] row-major
// ---------------------------------------------------------------------------
template <int L>  // L = W
__global__ void __launch_bounds__(kNT) fft_rows_kernel(float2* data, long long nrows_total,
                                                       const float2* tw_glob, int inverse) {
  extern __shared__ float2 lds[];
  constexpr int LPW = 4096 / L < 1 ? 1 : (4096 / L > 32 ? 32 : 4096 / L);
  constexpr int LS = lstride(L);
  float2* tw = lds + LPW * LS;
  load_twiddles<L, kNT>(tw, tw_glob);
  const long long row0 = (long long)blockIdx.x * LPW;
  const int nl = (int)min((long long)LPW, nrows_total - row0);
  for (int q = threadIdx.x; q < nl * L; q += kNT) {
    const int l = q / L, j = q - l * L;
    lds[l * LS + lpad(j)] = data[(row0 + l) * L + j];
  }
  __syncthreads();
  if (inverse) fft_lines<L, true, kNT, LPW>(lds, nl, tw);
  else fft_lines<L, false, kNT, LPW>(lds, nl, tw);
  for (int q = threadIdx.x; q < nl * L; q += kNT) {
    const int l = q / L, j = q - l * L;
    data[(row0 + l) * L + j] = lds[l * LS + lpad(j)];
  }
}

template <int L>  // L = H
__global__ void __launch_bounds__(kNT) fft_cols_kernel(float2* data, int W, int count,
                                                       const float2* tw_glob, int inverse) {
  extern __shared__ float2 lds[];
  constexpr int CW = c_for(L) * 2;   // columns per workgroup
  constexpr int LS = lstride(L);
  float2* tw = lds + CW * LS;
  load_twiddles<L, kNT>(tw, tw_glob);
  const int nblk = (W + CW - 1) / CW;
  const int img = blockIdx.x / nblk, blk = blockIdx.x - img * nblk;
  if (img >= count) return;
  float2* base = data + (long long)img * L * W;
  const int c0 = blk * CW;
  const int nc = min(CW, W - c0);
  for (int q = threadIdx.x; q < L * CW; q += kNT) {
    const int i = q / CW, c = q - i * CW;
    if (c < nc) lds[c * LS + lpad(i)] = base[(long long)i * W + c0 + c];
  }
  __syncthreads();
  if (inverse) fft_lines<L, true, kNT, CW>(lds, nc, tw);
  else fft_lines<L, false, kNT, CW>(lds, nc, tw);
  for (int q = threadIdx.x; q < L * CW; q += kNT) {
    const int i = q / CW, c = q - i * CW;
    if (c < nc) base[(long long)i * W + c0 + c] = lds[c * LS + lpad(i)];
  }
}

// ---------------------------------------------------------------------------
// setup and initialisation
// ---------------------------------------------------------------------------

// scatter kernel b circularly centred at the origin into a zeroed complex
// m' x n' grid (2b < min(m', n'), so the taps land on distinct positions)
__global__ void embed_psf_kernel(const ImgMeta* meta, const float* __restrict__ h, const long long* hoff,
                                 float2* grid, const long long* goff) {
  const int img = blockIdx.x;
  const ImgMeta mt = meta[img];
  const int K = 2 * mt.b + 1;
  float2* g = grid + goff[img];
  for (int t = threadIdx.x; t < K * K; t += blockDim.x) {
    const int pp = t / K - mt.b, qq = t % K - mt.b;
    const int i = pp < 0 ? pp + mt.m : pp, j = qq < 0 ? qq + mt.n : qq;
    g[(long long)i * mt.n + j] = make_float2(h[hoff[img] + t], 0.f);
  }
}

// Blur half spectrum by direct summation (setup).  For the (2b+1)^2 kernel
// centred at the origin (as embed_psf_kernel places it),
//   H(ky, kx) = sum_p w_m^(ky p) T(p, kx),  T(p, kx) = sum_q h(p, q) w_n^(kx q),
// p, q = -b..b, w_L = exp(-2 pi i / L) read from the twiddle tables (phase
// indices reduced exactly).  One workgroup per image, block of kBlurCols
// spectrum columns and block of kBlurRows rows: T of its columns in LDS,
// then its rows; written in the tiled half layout the column pass reads
// (zero past nh), or, with full, as the whole m' x n' spectrum (row-major at
// the image's pixel offset); H(0, 0) into hsum.  Kernels up to kBlurMaxK
// taps a side; FP32 sums of K terms.
constexpr int kBlurCols = 32;
constexpr int kBlurRows = 64;
constexpr int kBlurMaxK = 65;
// With sep (nullable; half spectrum only) an image whose sep flag is set
// takes H(ky, kx) = U(ky) V(kx) from its 1-D spectra in hsep (written by
// separable_psf_kernel beforehand) instead of the sums over its taps.
__global__ void __launch_bounds__(kNT) blur_half_kernel(const ImgMeta* meta, const float* __restrict__ h,
                                                       const long long* hoff, const float2* __restrict__ tw,
                                                       float2* hh, float2* hsum, float2* full,
                                                       const float2* hsep, const int* sep) {
  const int img = blockIdx.z;
  const ImgMeta mt = meta[img];
  const int ncol = full ? mt.n : mt.nb * mt.C;
  const int nval = full ? mt.n : mt.nh;   // columns with values (zero past them)
  const int kx0 = blockIdx.x * kBlurCols;
  const int ky0 = blockIdx.y * kBlurRows;
  if (kx0 >= ncol || ky0 >= mt.m) return;
  const int nrow = min(kBlurRows, mt.m - ky0);
  if (!full && sep && sep[img]) {
    const float2* __restrict__ U = hsep + mt.tab;
    const float2* __restrict__ V = U + mt.m;
    for (int t = threadIdx.x; t < nrow * kBlurCols; t += kNT) {
      const int ky = ky0 + t / kBlurCols, kx = kx0 + t % kBlurCols;
      if (kx >= ncol) continue;
      const float2 H = kx < nval ? cmul(U[ky], V[kx]) : make_float2(0.f, 0.f);
      hh[mt.hh + ((long long)(kx >> mt.logC) * mt.m + ky) * mt.C + (kx & (mt.C - 1))] = H;
      if (kx == 0 && ky == 0) hsum[img] = H;
    }
    return;
  }
  const int b = mt.b, K = 2 * b + 1;
  const float* __restrict__ hk = h + hoff[img];
  const float2* __restrict__ twn = tw + mt.twr;
  const float2* __restrict__ twm = tw + mt.twc;
  __shared__ float2 T[kBlurMaxK * kBlurCols];
  for (int t = threadIdx.x; t < K * kBlurCols; t += kNT) {
    const int p = t / kBlurCols, kx = kx0 + t % kBlurCols;
    float re = 0.f, im = 0.f;
    if (kx < nval) {
      // r = kx (q - b) mod n', stepped by kx
      int r = (int)(((long long)kx * (mt.n - b)) % mt.n);
      for (int q = 0; q < K; ++q) {
        const float2 w = twn[r];
        const float hv = hk[p * K + q];
        re = fmaf(hv, w.x, re);
        im = fmaf(hv, w.y, im);
        r += kx;
        if (r >= mt.n) r -= mt.n;
      }
    }
    T[t] = make_float2(re, im);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nrow * kBlurCols; t += kNT) {
    const int ky = ky0 + t / kBlurCols, c = t % kBlurCols, kx = kx0 + c;
    if (kx >= ncol) continue;
    float re = 0.f, im = 0.f;
    if (kx < nval) {
      int r = (int)(((long long)ky * (mt.m - b)) % mt.m);
      for (int p = 0; p < K; ++p) {
        const float2 w = twm[r];
        const float2 tv = T[p * kBlurCols + c];
        re = fmaf(tv.x, w.x, fmaf(-tv.y, w.y, re));
        im = fmaf(tv.x, w.y, fmaf(tv.y, w.x, im));
        r += ky;
        if (r >= mt.m) r -= mt.m;
      }
    }
    if (full) full[mt.px + (long long)ky * mt.n + kx] = make_float2(re, im);
    else hh[mt.hh + ((long long)(kx >> mt.logC) * mt.m + ky) * mt.C + (kx & (mt.C - 1))] = make_float2(re, im);
    if (kx == 0 && ky == 0) hsum[img] = make_float2(re, im);
  }
}

// Separable blurs.  If the (2b+1)^2 kernel of an image is the outer product
// h(p, q) = u(p) v(q) (to within 1e-6 of its largest tap), its spectrum is
// H(ky, kx) = U(ky) V(kx) with the 1-D spectra
//   U(ky) = sum_p u(p) w_m^(ky p),  V(kx) = sum_q v(q) w_n^(kx q),
// p, q = -b..b (the kernel centred at the origin, as embed_psf_kernel places
// it; w_L from the twiddle tables).  Pivot at the largest |h| (first on ties),
// u = its column, v = its row over the pivot; the rank-one test; then U and V.
// Grid: (blocks of kNT outputs, images); each workgroup repeats the test and
// writes its share of U[m'] then V[nb C] at the |D|^2 table's offset (tab);
// sep[img] = 1 when used (enable and the test passes), else 0.
constexpr int kSepMaxK = 65;
__global__ void __launch_bounds__(kNT) separable_psf_kernel(const ImgMeta* meta, const float* __restrict__ h,
                                                           const long long* hoff, const float2* __restrict__ tw,
                                                           float2* out, int* sep, int enable) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  const int nout = mt.m + mt.nb * mt.C;
  if ((int)blockIdx.x * kNT >= nout) return;
  const int b = mt.b, K = 2 * b + 1;
  const float* __restrict__ hk = h + hoff[img];
  __shared__ float u[kSepMaxK], v[kSepMaxK];
  __shared__ float best_v[kNT / 64];
  __shared__ int best_i[kNT / 64];
  __shared__ int ok;
  const bool fits = enable && K <= kSepMaxK;
  // pivot: largest |h|, smallest index on ties (wave maxima, then the waves)
  float bv = -1.f;
  int bi = 0x7fffffff;
  for (int t = threadIdx.x; fits && t < K * K; t += kNT) {
    const float a = fabsf(hk[t]);
    if (a > bv) { bv = a; bi = t; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(bv, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  if ((threadIdx.x & 63) == 0) { best_v[threadIdx.x >> 6] = bv; best_i[threadIdx.x >> 6] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kNT / 64; ++w)
      if (best_v[w] > bv || (best_v[w] == bv && best_i[w] < bi)) { bv = best_v[w]; bi = best_i[w]; }
    best_i[0] = bi;
    ok = fits && bv > 0.f;
  }
  __syncthreads();
  if (!ok) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sep[img] = 0;
    return;
  }
  const int pivot = best_i[0];
  const int pr = pivot / K, pc = pivot % K;
  const float hp = hk[pivot];
  for (int t = threadIdx.x; t < K; t += kNT) {
    u[t] = hk[t * K + pc];
    v[t] = hk[pr * K + t] / hp;
  }
  __syncthreads();
  const float tol = 1e-6f * fabsf(hp);
  for (int t = threadIdx.x; t < K * K; t += kNT)
    if (fabsf(hk[t] - u[t / K] * v[t % K]) > tol) ok = 0;
  __syncthreads();
  if (!ok) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sep[img] = 0;
    return;
  }
  const int t = blockIdx.x * kNT + threadIdx.x;
  if (t < nout) {
    const bool isu = t < mt.m;
    const int k = isu ? t : t - mt.m;
    const int len = isu ? mt.m : mt.n;
    const float* w = isu ? u : v;
    const float2* __restrict__ twl = tw + (isu ? mt.twc : mt.twr);
    float re = 0.f, im = 0.f;
    if (isu || k < mt.nh) {
      int r = (int)(((long long)k * (len - b)) % len);
      for (int p = 0; p < K; ++p) {
        const float2 e = twl[r];
        re = fmaf(w[p], e.x, re);
        im = fmaf(w[p], e.y, im);
        r += k;
        if (r >= len) r -= len;
      }
    }
    (isu ? out[mt.tab + k] : out[mt.tab + mt.m + k]) = make_float2(re, im);
  }
  if (threadIdx.x == 0 && blockIdx.x == 0) sep[img] = 1;
}

// copy the spectrum columns kx < nh into the tiled half layout
__global__ void pack_half_kernel(const ImgMeta* meta, const float2* __restrict__ grid,
                                 const long long* goff, float2* hh) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  const float2* g = grid + goff[img];
  const int ncol = mt.nb * mt.C;
  for (int ky = blockIdx.x; ky < mt.m; ky += gridDim.x)
    for (int kx = threadIdx.x; kx < ncol; kx += blockDim.x)
      hh[mt.hh + ((long long)(kx >> mt.logC) * mt.m + ky) * mt.C + (kx & (mt.C - 1))] =
          kx < mt.nh ? g[(long long)ky * mt.n + kx] : make_float2(0.f, 0.f);
}

constexpr int kMeanBlocks = 256;   // blocks of rows per image (partial sums of the observed mean)

// per image and block of rows: FP64 sum and count of the observed pixels
__global__ void __launch_bounds__(kNT) observed_sum_kernel(const ImgMeta* meta, const float* __restrict__ y,
                                                          const uint8_t* __restrict__ mask, double* part) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  double s = 0.0, c = 0.0, dummy = 0.0;
  for (int i = blockIdx.x; i < mt.m; i += gridDim.x)
    for (int j = threadIdx.x; j < mt.n; j += kNT)
      if (observed(mt, mask, i, j)) { s += y[mt.px + (long long)i * mt.n + j]; c += 1.0; }
  __shared__ double red[3 * (kNT / 64)];
  block_sum3(s, c, dummy, red);
  if (threadIdx.x == 0) {
    part[2 * ((long long)img * gridDim.x + blockIdx.x)] = s;
    part[2 * ((long long)img * gridDim.x + blockIdx.x) + 1] = c;
  }
}

__device__ __forceinline__ float init_value(const ImgMeta& mt, const float* __restrict__ y,
                                            const uint8_t* __restrict__ mask, float mean, int i, int j) {
  if (observed(mt, mask, i, j)) return y[mt.px + (long long)i * mt.n + j];
  const bool in_c = i >= mt.b && i < mt.m - mt.b && j >= mt.b && j < mt.n - mt.b;
  if (in_c) return mean;
  const int si = min(max(i, mt.b), mt.m - mt.b - 1), sj = min(max(j, mt.b), mt.n - mt.b - 1);
  return observed(mt, mask, si, sj) ? y[mt.px + (long long)si * mt.n + sj] : mean;
}

// ytilde^0, v^0 = D ytilde^0, d^0 = 0 (one row per block and step; every
// block sums the partials of the observed mean in the same order)
__global__ void __launch_bounds__(kNT) init_state_kernel(const ImgMeta* meta, const float* __restrict__ y,
                                                        const uint8_t* __restrict__ mask, const double* part,
                                                        int nparts, float* yt, float2* v, float2* d) {
  const int img = blockIdx.y;
  const ImgMeta mt = meta[img];
  __shared__ float smean;
  __shared__ double red[3 * (kNT / 64)];
  double s = 0.0, c = 0.0, dummy = 0.0;
  for (int k = threadIdx.x; k < nparts; k += kNT) {
    s += part[2 * ((long long)img * nparts + k)];
    c += part[2 * ((long long)img * nparts + k) + 1];
  }
  block_sum3(s, c, dummy, red);
  if (threadIdx.x == 0) smean = c > 0 ? (float)(s / c) : 0.f;
  __syncthreads();
  const float mn = smean;
  for (int i = blockIdx.x; i < mt.m; i += gridDim.x) {
    const int id = i + 1 == mt.m ? 0 : i + 1;
    for (int j = threadIdx.x; j < mt.n; j += kNT) {
      const long long p = mt.px + (long long)i * mt.n + j;
      const float c = init_value(mt, y, mask, mn, i, j);
      const float r = init_value(mt, y, mask, mn, i, j + 1 == mt.n ? 0 : j + 1);
      const float dn = init_value(mt, y, mask, mn, id, j);
      yt[p] = c;
      v[p] = make_float2(r - c, dn - c);
      d[p] = make_float2(0.f, 0.f);
    }
  }
}

// n 32-bit words of zeros (instead of a memset node where a graph may be
// captured)
__global__ void __launch_bounds__(kNT) zero_words_kernel(unsigned* p, long long n) {
  for (long long i = (long long)blockIdx.x * kNT + threadIdx.x; i < n; i += (long long)gridDim.x * kNT) p[i] = 0u;
}

// per image: FP64 sum of the row-tile partials -> |d'-d|, |v'-v|, |z'-z|;
// with stop_test, sets the stop flag when both tolerances hold; with
// adapt_t > 0, the penalty update of eq. (varying_penalty): mu doubles (d
// halves) when |d'-d| > t |v'-v|, mu halves (d doubles) when |v'-v| >
// t |d'-d|; dscale receives the factor for d.
// For a colour group |d'-d| and |v'-v| run over all its channels (the joint
// prox leaves them in the partials of the group's first image), so every
// channel takes the same stop and penalty decisions.
__global__ void __launch_bounds__(kNT) residual_kernel(const ImgMeta* meta, const double* partials,
                                                       double* res, int* done, int* nonfinite,
                                                       int* iters_done, int iters_since, int stop_test,
                                                       double tol_p, double tol_d, double adapt_t,
                                                       float* mu_cur, float* dscale, int* stop_buf,
                                                       int cur_d) {
  const int img = blockIdx.x;
  const ImgMeta mt = meta[img];
  const ImgMeta mg = meta[mt.group];
  double a = 0, b = 0, c = 0;
  for (int t = threadIdx.x; t < mg.nrt; t += kNT) {
    const double* p = partials + 3 * (mg.rt0 + t);
    a += p[0]; b += p[1];
  }
  for (int t = threadIdx.x; t < mt.nrt; t += kNT) c += partials[3 * (mt.rt0 + t) + 2];
  __shared__ double red[3 * (kNT / 64)];
  block_sum3(a, b, c, red);
  if (threadIdx.x == 0) {
    if (record_residuals(mt, img, a, b, c, res, done, nonfinite, iters_done, iters_since, stop_test, tol_p, tol_d,
                         stop_buf, cur_d))
      return;
    const double nd = sqrt(a), nv = sqrt(b);
    if (adapt_t > 0) {
      float f = 1.f;
      if (nd > adapt_t * nv) { mu_cur[img] *= 2.f; f = 0.5f; }
      else if (nv > adapt_t * nd) { mu_cur[img] *= 0.5f; f = 2.f; }
      dscale[img] = f;
    }
  }
}

// After a run with early stopping: copy the d of each stopped image from the
// buffer it stopped in to the current one (no-op for the others).
__global__ void __launch_bounds__(kNT) stopped_d_kernel(const ImgMeta* meta, const int* done, const int* stop_buf,
                                                        int cur_d, float2* d0, float2* d1) {
  const int img = blockIdx.y;
  if (!done[img] || stop_buf[img] == cur_d) return;
  const ImgMeta mt = meta[img];
  const float2* src = (cur_d == 0 ? d1 : d0) + mt.px;
  float2* dst = (cur_d == 0 ? d0 : d1) + mt.px;
  const long long n = (long long)mt.m * mt.n;
  for (long long i = (long long)blockIdx.x * kNT + threadIdx.x; i < n; i += (long long)gridDim.x * kNT) dst[i] = src[i];
}

// Joint prox of a colour group (vectorial TV of Sec. III-C): at each pixel one
// vector soft threshold over the 2C components u^c = D x^c + d^c of the
// group's C channels, whose images follow each other in the packed arrays.
// u arrives in d_new (ROW_UONLY pass); d_new and v receive d^{i+1}, v^{i+1}.
// One block per row tile of the group's first image; with check, |d'-d|^2
// and |v'-v|^2 of the tile go to its partials.  tau = lambda / mu of the
// first channel.
constexpr int kMaxChannels = 4;
// 1024 threads per row tile: a colour image has few row tiles (288 rows: 36),
// so each workgroup must keep many loads in flight (288 x 256 x 3 image: 31 us
// per launch with 256 threads and one pixel per step, 9 us with 1024 threads
// and every load of two pixels issued before their stores)
constexpr int kNTProx = 1024;
__global__ void __launch_bounds__(kNTProx) group_prox_kernel(const ImgMeta* meta, const float* lam, const float* mu,
                                                            const float2* __restrict__ d_old, float2* d_new,
                                                            float2* v, double* partials, int check, const int* done) {
  const int g0 = blockIdx.y * meta[0].nch;
  const ImgMeta mt = meta[g0];
  if (done && done[g0]) return;
  const int t = blockIdx.x;
  if (t >= mt.nrt) return;
  const float tau = lam[g0] / mu[g0];
  const float tau2 = tau * tau;
  const int r0 = t * mt.rt, nr = min(mt.rt, mt.m - r0);
  const long long plane = (long long)mt.m * mt.n;
  const int npx = nr * mt.n;
  float rd = 0.f, rv = 0.f;
  // kProxPix pixels per thread and step, every load issued before the
  // first store (the stores could alias the next loads as far as the
  // compiler knows)
  constexpr int kProxPix = 2;
  for (int p0 = threadIdx.x; p0 < npx; p0 += kNTProx * kProxPix) {
    float2 u[kProxPix][kMaxChannels], d0[kProxPix][kMaxChannels], v0[kProxPix][kMaxChannels];
#pragma unroll
    for (int e = 0; e < kProxPix; ++e) {
      const int p = p0 + e * kNTProx;
      const long long pix = mt.px + (long long)r0 * mt.n + p;
#pragma unroll
      for (int c = 0; c < kMaxChannels; ++c)
        if (p < npx && c < mt.nch) {
          u[e][c] = d_new[pix + c * plane];
          if (check) {
            d0[e][c] = d_old[pix + c * plane];
            v0[e][c] = v[pix + c * plane];
          }
        }
    }
#pragma unroll
    for (int e = 0; e < kProxPix; ++e) {
      const int p = p0 + e * kNTProx;
      if (p >= npx) continue;
      const long long pix = mt.px + (long long)r0 * mt.n + p;
      float n2 = 0.f;
#pragma unroll
      for (int c = 0; c < kMaxChannels; ++c)
        if (c < mt.nch) n2 += u[e][c].x * u[e][c].x + u[e][c].y * u[e][c].y;
      const float s = vsoft_scale(n2, tau, tau2);
#pragma unroll
      for (int c = 0; c < kMaxChannels; ++c)
        if (c < mt.nch) {
          const long long q = pix + c * plane;
          const float2 vn = make_float2(s * u[e][c].x, s * u[e][c].y);
          const float2 dn = make_float2(u[e][c].x - vn.x, u[e][c].y - vn.y);
          if (check) {
            const float2 a = d0[e][c], b = v0[e][c];
            rd += (dn.x - a.x) * (dn.x - a.x) + (dn.y - a.y) * (dn.y - a.y);
            rv += (vn.x - b.x) * (vn.x - b.x) + (vn.y - b.y) * (vn.y - b.y);
          }
          v[q] = vn;
          d_new[q] = dn;
        }
    }
  }
  if (check) {
    __shared__ double red[3 * (kNTProx / 64)];
    double a = rd, b = rv, z = 0.0;
    block_sum3(a, b, z, red);
    if (threadIdx.x == 0) {
      partials[3 * (mt.rt0 + t)] = a;
      partials[3 * (mt.rt0 + t) + 1] = b;
    }
  }
}

}  // namespace dcv
