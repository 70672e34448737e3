// Whole-image-in-LDS path for small images: one workgroup runs every
// iteration of a check period of one image without leaving the compute unit.
//
// The iteration is that of the two-pass kernels (Sec. II-B, eqs.
// (admm_aprox_1)-(admm_aprox_4) with the x-step solved per frequency as in
// eq. (dual_x_iter_resolved_boundaries), the over-relaxed z-step and the
// vector soft threshold of Sec. III-B), but the whole m' x n' complex array
// sits in LDS, so the 2-D transforms need no HBM round trip: the state
// (ytilde, v, d) and the per-frequency constants live in registers, the state
// goes to HBM once per launch.
//
// Per iteration, with C the LDS array and W the LDS field of w = v - d:
//   W <- v - d;  C <- ytilde + i mu D^T W          (g from the neighbours in W)
//   C <- DFT2(C)                                   (row DFTs, then column DFTs)
//   per frequency pair (k, -k):  Y, G from C(k), conj C(-k);
//     X = (conj(H) Y + G) / (|H|^2 + mu |D|^2) / (m'n'),  Q = H X,
//     C(k) <- X + i Q, C(-k) <- conj X + i conj Q
//   C <- IDFT2(C)  ->  x + i H x
//   z-step, u = D x + d (neighbours in C), v' = shrink(u), d' = u - v'.
#pragma once
#include "kernels.hpp"

namespace dcv {

constexpr int kNTS = 1024;   // threads of a small-image workgroup

struct SmallArgs {
  const ImgMeta* meta;
  const int* imgs;           // images of this launch
  float* yt;
  float2* d;                 // d, updated in place (one workgroup owns the image)
  float2* v;                 // v: read at the start, written by the last iteration
  const float2* hh;          // blur half spectrum (tiled like the column pass)
  const float* tab;          // |D_v|^2[m'], |D_h|^2[nb C]
  const uint8_t* mask;
  const float* lam;
  const float* mu;
  const float2* tw;
  int* done;                 // per image: stop flag (read at the start, set by a check)
  float* x_out;
  // a check (the workgroup holds the whole image, so it finishes the
  // residuals itself): per image |d'-d|, |v'-v|, |z'-z|, the non-finite
  // flag, iterations done, the d buffer of a stop
  double* res;
  int* nonfinite;
  int* iters_done;
  int* stop_buf;
  double tol_p, tol_d;
  int cur_d;
  int iters;                 // iterations of this launch
  int check_every;           // residuals after every check_every-th iteration of the launch (0: none)
  int stop_test;             // 1: apply the tolerances at those checks
  int store_x;               // 1: x of the last iteration into x_out
  float alpha;
};

// One Stockham pass over the N columns (length M) of a row-major array in
// LDS: element e of column q at buf[e * LSN + lpad(q)].  Consecutive threads
// take consecutive columns.
template <int M, int N, int R, int NS, bool INV, int NT, int LSN>
__device__ __forceinline__ void col_stockham_pass(float2* buf, const float2* tw, unsigned tid) {
  constexpr int NB = M / R;
  constexpr int S = M / (NS * R);
  constexpr int TOTAL = N * NB;
  constexpr int MAXB = (TOTAL + NT - 1) / NT;
  float2 v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = (int)tid + q * NT;
    if (idx < TOTAL) {
      const int col = idx % N, j = idx / N;
#pragma unroll
      for (int k = 0; k < R; ++k) v[q][k] = buf[(j + k * NB) * LSN + lpad(col)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = (int)tid + q * NT;
    if (idx < TOTAL) {
      const int col = idx % N, j = idx / N;
      const int jm = j % NS;
      if constexpr (NS > 1) apply_twiddles<R, S, INV>(v[q], jm, tw);
      Dft<R, INV>::run(v[q]);
      const int base = (j / NS) * NS * R + jm;
#pragma unroll
      for (int k = 0; k < R; ++k) buf[(base + k * NS) * LSN + lpad(col)] = v[q][k];
    }
  }
  __syncthreads();
}

template <int M, int N, bool INV, int NT, int LSN, int P = 0>
__device__ __forceinline__ void fft_cols_lds(float2* buf, const float2* tw, unsigned tid) {
  if constexpr (P < RadixPlan<M>::npass) {
    col_stockham_pass<M, N, RadixPlan<M>::radix(P), RadixPlan<M>::ns(P), INV, NT, LSN>(buf, tw, tid);
    fft_cols_lds<M, N, INV, NT, LSN, P + 1>(buf, tw, tid);
  }
}

// Keeps the compiler from hoisting the loads of later pixels above this
// point: bounds the loads in flight (and the registers they hold) per thread.
__device__ __forceinline__ void small_group_fence() { __asm__ volatile("" ::: "memory"); }

template <int M, int N>
struct SmallShape {
  static constexpr int LSN = lstride(N);
  static constexpr int NPX = M * N;
  static constexpr int KP = (NPX + kNTS - 1) / kNTS;                // pixels per thread
  static constexpr int NHALF = M * (N / 2 + 1);                      // half-spectrum frequencies
  static constexpr int KF = (NHALF + kNTS - 1) / kNTS;               // frequencies per thread
  // C, W, the twiddle tables of both lengths, then (where it fits) the
  // per-frequency constants (H, |D|^2) of the x-step as float4
  static constexpr size_t base_bytes = ((size_t)2 * M * LSN + M + N) * sizeof(float2);
  static constexpr bool kConstLds = base_bytes + (size_t)NHALF * sizeof(float4) <= 160 * 1024;
  static constexpr size_t lds_bytes = base_bytes + (kConstLds ? (size_t)NHALF * sizeof(float4) : 0);
};

template <int M, int N>
__device__ __forceinline__ void small_image(const SmallArgs& a, int img, float2* lds);

template <int M, int N>
__global__ void __launch_bounds__(kNTS) small_kernel(SmallArgs a) {
  extern __shared__ float2 lds[];
  const int img = a.imgs[blockIdx.x];
  if (a.done && a.done[img]) return;
  small_image<M, N>(a, img, lds);
}

// one launch for images of several sides: each workgroup dispatches on its
// image's side (square images)
template <int S0, int... Ss>
__device__ __forceinline__ void small_dispatch(const SmallArgs& a, int side, int img, float2* lds) {
  if (side == S0) {
    small_image<S0, S0>(a, img, lds);
    return;
  }
  if constexpr (sizeof...(Ss) > 0) small_dispatch<Ss...>(a, side, img, lds);
}

template <int... Ss>
__global__ void __launch_bounds__(kNTS) small_kernel_multi(SmallArgs a) {
  extern __shared__ float2 lds[];
  const int img = a.imgs[blockIdx.x];
  if (a.done && a.done[img]) return;
  small_dispatch<Ss...>(a, a.meta[img].m, img, lds);
}

template <int M, int N>
__device__ __forceinline__ void small_image(const SmallArgs& a, int img, float2* lds) {
  using SS = SmallShape<M, N>;
  constexpr int LSN = SS::LSN, KP = SS::KP, KF = SS::KF, NH = N / 2 + 1;
  static_assert(KP <= 32 && KF <= 32, "per-thread flags are kept in one word");
  float2* C = lds;                 // the complex image / spectrum
  float2* W = lds + M * LSN;       // w = v - d, kept here between iterations
  const ImgMeta mt = a.meta[img];
  float* __restrict__ yt = a.yt + mt.px;
  float2* __restrict__ dg = a.d + mt.px;
  float2* __restrict__ vg = a.v + mt.px;
  const float2* __restrict__ hh = a.hh + mt.hh;
  const float* __restrict__ tab = a.tab + mt.tab;
  const float mu = a.mu[img];
  const float tau = a.lam[img] / mu;
  const float tau2 = tau * tau;
  const float alpha = a.alpha;
  // the twiddle tables in LDS: every transform pass reads them on its
  // critical path
  float2* twr = lds + 2 * M * LSN;
  float2* twc = twr + N;
  for (int t = (int)threadIdx.x; t < N; t += kNTS) twr[t] = a.tw[mt.twr + t];
  for (int t = (int)threadIdx.x; t < M; t += kNTS) twc[t] = a.tw[mt.twc + t];
  // per frequency f of the half spectrum (ky = f / NH, kx = f mod NH): H and
  // |D_h|^2 + |D_v|^2, in LDS where they fit (else read per iteration)
  float4* HT = reinterpret_cast<float4*>(twc + M);
  if constexpr (SS::kConstLds) {
    for (int f = (int)threadIdx.x; f < SS::NHALF; f += kNTS) {
      const int ky = f / NH, kx = f - ky * NH;
      const float2 H = hh[((kx >> mt.logC) * M + ky) * mt.C + (kx & (mt.C - 1))];
      HT[f] = make_float4(H.x, H.y, tab[ky] + tab[M + kx], 0.f);
    }
  }

  // registers: ytilde and d of the thread's pixels p = tid + k kNTS, which
  // of them are observed; w = v - d lives in W.  Each pixel's LDS offset
  // i LSN + lpad(j) and the flags that give its neighbours' offsets (the
  // last / first column and row, and where lpad steps by 2) are computed
  // once, so that the loop does no division.
  float yv[KP];
  float2 dv[KP];
  int poff[KP];
  unsigned obs = 0, jlast = 0, jfirst = 0, ilast = 0, ifirst = 0, padr = 0, padl = 0;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int p = (int)threadIdx.x + k * kNTS;
    poff[k] = 0;
    if (p < SS::NPX) {
      const int i = p / N, j = p - i * N;
      poff[k] = i * LSN + lpad(j);
      yv[k] = yt[p];
      dv[k] = dg[p];
      const float2 v0 = vg[p];
      W[poff[k]] = make_float2(v0.x - dv[k].x, v0.y - dv[k].y);
      if (observed(mt, a.mask, i, j)) obs |= 1u << k;
      if (j == N - 1) jlast |= 1u << k;
      if (j == 0) jfirst |= 1u << k;
      if (i == M - 1) ilast |= 1u << k;
      if (i == 0) ifirst |= 1u << k;
      if ((j & 15) == 15) padr |= 1u << k;   // lpad(j + 1) = lpad(j) + 2
      if ((j & 15) == 0) padl |= 1u << k;    // lpad(j - 1) = lpad(j) - 2 (j > 0)
    }
  }
  // the thread's frequencies f = tid + k kNTS of the half spectrum (kx <=
  // N/2; on the columns kx = 0 and kx = N/2 only ky <= M/2, whose partner
  // (-ky, kx) lies in the same column): offsets of (ky, kx) and (-ky, -kx),
  // which of them take part and which are their own partner
  int foff[KF], fmoff[KF];
  unsigned fact = 0, fself = 0;
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int f = (int)threadIdx.x + k * kNTS;
    foff[k] = 0;
    fmoff[k] = 0;
    if (f < SS::NHALF) {
      const int ky = f / NH, kx = f - ky * NH;
      const bool edge = kx == 0 || 2 * kx == N;
      const int ny = ky == 0 ? 0 : M - ky, nx = kx == 0 ? 0 : N - kx;
      foff[k] = ky * LSN + lpad(kx);
      fmoff[k] = ny * LSN + lpad(nx);
      if (!edge || 2 * ky <= M) fact |= 1u << k;
      if (ny == ky && nx == kx) fself |= 1u << k;
    }
  }
  const float scale = 1.0f / ((float)M * (float)N);
  float rd = 0.f, rv = 0.f, rz = 0.f;

  for (int it = 0; it < a.iters; ++it) {
    const bool last = it + 1 == a.iters;
    const bool chk = a.check_every > 0 && (it + 1) % a.check_every == 0;
    // the offsets and the thread index made opaque per iteration: addresses
    // derived from them are formed where they are used rather than kept in
    // registers across the loop
    unsigned tid = threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
#pragma unroll
    for (int k = 0; k < KP; ++k) __asm__ volatile("" : "+v"(poff[k]));
#pragma unroll
    for (int k = 0; k < KF; ++k) __asm__ volatile("" : "+v"(foff[k]), "+v"(fmoff[k]));
    __syncthreads();   // W written (before the loop or by the last epilogue)
    // C <- ytilde + i mu D^T w: g = w_h[i, j-1] - w_h[i, j] + w_v[i-1, j] - w_v[i, j]
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int p = (int)tid + k * kNTS;
      if (p < SS::NPX) {
        const int o = poff[k];
        const int ol = (jfirst >> k) & 1u ? o + lpad(N - 1) : o - 1 - (int)((padl >> k) & 1u);
        const int ou = (ifirst >> k) & 1u ? o + (M - 1) * LSN : o - LSN;
        const float2 w = W[o];
        const float wl = W[ol].x;
        const float wu = W[ou].y;
        C[o] = make_float2(yv[k], mu * (wl - w.x + wu - w.y));
      }
      if (k % 2 == 1) small_group_fence();
    }
    __syncthreads();
    fft_lines<N, false, kNTS, M>(C, M, twr, tid);
    fft_cols_lds<M, N, false, kNTS, LSN>(C, twc, tid);
    // x-step per frequency pair (C holds F(ytilde) + i F(mu g)); each slot
    // is read and written by one thread
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int f = (int)tid + k * kNTS;
      if ((fact >> k) & 1u) {
        float2 H;
        float ds;
        if constexpr (SS::kConstLds) {
          const float4 t = HT[f];
          H = make_float2(t.x, t.y);
          ds = t.z;
        } else {
          const int ky = f / NH, kx = f - ky * NH;
          H = hh[((kx >> mt.logC) * M + ky) * mt.C + (kx & (mt.C - 1))];
          ds = tab[ky] + tab[M + kx];
        }
        const float2 c = C[foff[k]];
        const float2 cm = C[fmoff[k]];
        // Y = (c + conj cm) / 2, G = (c - conj cm) / 2i
        const float2 Y = make_float2(0.5f * (c.x + cm.x), 0.5f * (c.y - cm.y));
        const float2 G = make_float2(0.5f * (c.y + cm.y), 0.5f * (cm.x - c.x));
        const float inv = scale * frcp(H.x * H.x + H.y * H.y + mu * ds);
        const float2 X = make_float2((H.x * Y.x + H.y * Y.y + G.x) * inv, (H.x * Y.y - H.y * Y.x + G.y) * inv);
        const float2 Q = cmul(H, X);
        C[foff[k]] = make_float2(X.x - Q.y, X.y + Q.x);
        if (!((fself >> k) & 1u)) C[fmoff[k]] = make_float2(X.x + Q.y, Q.x - X.y);
      }
      small_group_fence();
    }
    __syncthreads();
    fft_cols_lds<M, N, true, kNTS, LSN>(C, twc, tid);
    fft_lines<N, true, kNTS, M>(C, M, twr, tid);
    // z-step, TV prox, dual update (C = x + i H x); w' = v' - d' into W
    // (W's last readers finished before the forward transforms)
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int p = (int)tid + k * kNTS;
      if (p < SS::NPX) {
        const int o = poff[k];
        const int orr = (jlast >> k) & 1u ? o - lpad(N - 1) : o + 1 + (int)((padr >> k) & 1u);
        const int od = (ilast >> k) & 1u ? o - (M - 1) * LSN : o + LSN;
        const float2 c = C[o];
        const float x = c.x;
        const float xr = C[orr].x;
        const float xd = C[od].x;
        if (!((obs >> k) & 1u)) {
          const float yn = yv[k] + alpha * (c.y - yv[k]);
          if (chk) rz += (yn - yv[k]) * (yn - yv[k]);
          yv[k] = yn;
        }
        const float uh = xr - x + dv[k].x, uv = xd - x + dv[k].y;
        const float sc = vsoft_scale(uh * uh + uv * uv, tau, tau2);
        const float vh = sc * uh, vw = sc * uv;
        const float dh = uh - vh, dw = uv - vw;
        float2* wp = W + o;
        if (chk) {
          const float2 w0 = *wp;   // v = w + d of the previous iteration
          const float v0h = w0.x + dv[k].x, v0v = w0.y + dv[k].y;
          rd += (dh - dv[k].x) * (dh - dv[k].x) + (dw - dv[k].y) * (dw - dv[k].y);
          rv += (vh - v0h) * (vh - v0h) + (vw - v0v) * (vw - v0v);
        }
        *wp = make_float2(vh - dh, vw - dw);
        dv[k] = make_float2(dh, dw);
        if (last) {
          vg[p] = make_float2(vh, vw);
          if (a.store_x) a.x_out[mt.px + p] = x;
        }
      }
      if (k % 2 == 1) small_group_fence();
    }
    if (chk) {
      // a check: the workgroup holds the whole image, so it records the
      // image's residuals (and the stop decision) itself
      __shared__ double red[3 * (kNTS / 64)];
      double s0 = rd, s1 = rv, s2 = rz;
      block_sum3(s0, s1, s2, red);
      if (threadIdx.x == 0)
        record_residuals(mt, img, s0, s1, s2, a.res, a.done, a.nonfinite, a.iters_done, a.check_every, a.stop_test,
                         a.tol_p, a.tol_d, a.stop_buf, a.cur_d);
      rd = rv = rz = 0.f;
    }
  }
  // the state back to HBM (v was written by the last iteration); the
  // addresses computed here, not kept live through the loop
  unsigned tid_end = threadIdx.x;
  __asm__ volatile("" : "+v"(tid_end));
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int p = (int)tid_end + k * kNTS;
    if (p < SS::NPX) {
      yt[p] = yv[k];
      dg[p] = dv[k];
    }
  }
}

}  // namespace dcv
