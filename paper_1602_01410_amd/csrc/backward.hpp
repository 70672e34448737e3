// Reverse mode through unrolled partial-ADMM iterations (not in the paper;
// derived from the forward steps of Sec. II-B / III-B).
//
// Forward iteration i maps the state (ytilde^i, v^i, d^i) to
//   x = A^{-1}(H^T ytilde + mu D^T (v - d)),  A = H^T H + mu D^T D,
//   z' = z + alpha (M_z H x - z),  u = D x + d,  v' = S_tau(u),  d' = u - v'.
// Given the adjoints (zb, vb, db) of the new state and xb_direct = dL/dx (only
// for the output iterate), one reverse step is
//   t  = vb - db,           ub = db + J_S(u)^T t,   lambda_b -= <u/|u|, t>/mu,
//   xb = xb_direct + D^T ub + H^T (alpha M_z^T zb),
//   rb = A^{-1} xb          (A is symmetric: the same spectral solve),
//   y_b += (H rb) on observed pixels,
//   zb <- (1 - alpha) zb + (H rb) on unobserved pixels,
//   vb <- mu D rb,          db <- ub - mu D rb,
// and the blur gradient collects, in the frequency domain, per frequency k
//   S_k += conj(QB_k) X_k + conj(Y_k) RB_k - 2 conj(H_k) Re(conj(RB_k) X_k)
//        = X_k conj(QB_k - H_k RB_k) + RB_k conj(Y_k - H_k X_k)
// (QB = DFT(alpha M_z^T zb), X = DFT(x), Y = DFT(ytilde^i), RB = DFT(rb));
// dL/dh[p] = Re(sum_k S_k exp(-2 pi i k.p / N)) / N at the kernel taps.
//
// The kernels mirror the forward ones: a column pass (spectral solve + S
// accumulation) and a row pass that finishes reverse step i (inverse row DFT
// -> rb, H rb) and starts reverse step i-1 (forward row DFT of
// D^T ub + i alpha M_z^T zb), with one halo row on each side.
#pragma once
#include "kernels.hpp"

namespace dcv {

enum { BWD_ITER = 0, BWD_START = 1, BWD_END = 2 };

struct BwdRowArgs {
  const ImgMeta* meta;
  const int4* tiles;
  const float4* spec_in;   // (RB, H RB) column-pass output
  float4* spec_out;        // (DFT_row(xb), DFT_row(qb)) for the next column pass
  const float2* ub_in;     // ub of the step being finished (halo rows read)
  float2* ub_out;          // ub of the step being started
  float2* vb;              // adjoint state at segment boundaries
  float2* db;
  float* zb;               // adjoint of z (unobserved pixels)
  float* yb;               // accumulated dL/dy (observed pixels)
  const float2* u;         // u = D x + d of the forward step being started
  const float* grad_x;     // dL/dx^N (first reverse step only), nullable
  const uint8_t* mask;
  const float* lam;
  const float* mu;
  const float2* tw;
  double* lam_part;        // per row tile, accumulated dL/dlambda
  float alpha;
  int mode;
};

struct BwdColArgs {
  const ImgMeta* meta;
  const int4* tiles;
  const float4* spec_in;
  float4* spec_out;
  const float2* hh;
  const float* tab;
  const float* mu;
  const float2* tw;
  const float4* fwd_spec;  // (Y, X / (m'n')) stored by the forward recompute
  double2* S;              // accumulated spectral blur gradient (half, tiled, FP64)
};

// J^T t for the vector soft threshold at u (J is symmetric); also returns the
// derivative of <S_tau(u), t> with respect to tau.  The active set is the one
// of the forward shrink (|u|^2 > tau^2); with r = 1/|u|:
// J^T t = (1 - tau r) t + tau r^3 <u, t> u,  d<S,t>/dtau = -r <u, t>.
__device__ __forceinline__ float2 vsoft_vjp(float2 u, float2 t, float tau, float tau2, float& dtau) {
  const float n2 = u.x * u.x + u.y * u.y;
  if (!(n2 > tau2)) { dtau = 0.f; return make_float2(0.f, 0.f); }
  const float r = __builtin_amdgcn_rsqf(n2);
  const float ut = u.x * t.x + u.y * t.y;
  const float s = 1.f - tau * r;
  const float c = ut * tau * r * r * r;
  dtau = -ut * r;
  return make_float2(s * t.x + c * u.x, s * t.y + c * u.y);
}

// reverse row pass: issue the epilogue's state loads before the inverse
// transform (1: more registers) or after it (0)
#ifndef DCV_BWD_EARLY_STATE
#define DCV_BWD_EARLY_STATE 0
#endif

template <int L>
__device__ __forceinline__ void bwd_row_tile(const BwdRowArgs& a, int img, int r0, float2* lds) {
  using PM = PixMap<L>;
  constexpr int RT = rt_for(L);
  constexpr int LS = row_lstride(L, RT);
  constexpr int KP = ((RT + 1) * L + kNTR - 1) / kNTR;
  static_assert(KP <= 32, "observed flags of a thread's pixels are kept in one word");
  const unsigned tid = threadIdx.x;
  __builtin_assume(tid < (unsigned)kNTR);
  const ImgMeta mt = a.meta[img];
  const int M = mt.m;
  const int nr = min(RT, M - r0);
  const int C = mt.C, logC = mt.logC, nh = mt.nh, nb = mt.nb;
  float2* buf = lds;
  float2* lds_tw = lds + (RT + 1) * LS;
  const float2* tw_glob = a.tw + mt.twr;
  TwCopy<L, kNTR, kTwLdsRow> twc;
  const float2* tw = tw_glob;
  const float mu = a.mu[img];
  const float tau = a.lam[img] / mu;
  const float tau2 = tau * tau;
  const bool start = a.mode == BWD_START, end = a.mode == BWD_END;
  float2* __restrict__ vb = a.vb + mt.px;
  float2* __restrict__ db = a.db + mt.px;
  float* __restrict__ zb = a.zb + mt.px;
  float* __restrict__ yb = a.yb + mt.px;
  const float2* __restrict__ ubin = start ? nullptr : a.ub_in + mt.px;
  const float2* __restrict__ uin = end ? nullptr : a.u + mt.px;
  float2* __restrict__ ubout = end ? nullptr : a.ub_out + mt.px;
  float2 ureg[KP];
  float qreg[KP];
  float lsum = 0.f;

  // state loads of the epilogue, issued before the transform: ub (or vb, db
  // at the start), u, and z-bar or y-bar of the own rows
  float2 s0[KP], s1[KP], su[KP];
  float sz[KP];
  unsigned obsbits = 0;
  if (!start) {
    // the twiddle table's reads travel with the spectra
    gather_rows<L, RT>(a.spec_in + mt.sp, buf, M, r0, nr, nh, nb, C, logC, mt.rb,
                       [&]() { twc.issue(tw_glob, tid); });
    tw = twc.commit(lds_tw, tw_glob, tid);
#if !DCV_BWD_EARLY_STATE
    // finish reverse step: rb + i H rb on the own rows, rb on the halo rows
    __syncthreads();
    fft_lines<L, true, kNTR, RT + 1, kEarlyTwRow, LS>(buf, nr + 1, tw);
#endif
  }
  if (start) {
    twc.issue(tw_glob, tid);
    tw = twc.commit(lds_tw, tw_glob, tid);
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int l = PM::row(k, tid), j = PM::col(k, tid);
    if (l <= nr) {
      const int i = wrapi(r0 - 1 + l, M);
      const unsigned pix = (unsigned)(i * L + j);
      if (start) {
        s0[k] = vb[pix];
        s1[k] = db[pix];
      } else {
        s0[k] = ubin[pix];
      }
      if (!end) su[k] = uin[pix];
      if (l >= 1) {
        const RowObs ro = row_observed(mt, i);
        const bool obs = pixel_observed(mt, ro, ro.explicit_mask ? a.mask + mt.px + i * L : nullptr, j);
        obsbits |= (obs ? 1u : 0u) << k;
        sz[k] = obs ? yb[pix] : zb[pix];
      }
    }
  }
#if DCV_BWD_EARLY_STATE
  if (!start) {
    // finish reverse step: rb + i H rb on the own rows, rb on the halo rows
    __syncthreads();
    fft_lines<L, true, kNTR, RT + 1, kEarlyTwRow, LS>(buf, nr + 1, tw);
  }
#endif

#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int l = PM::row(k, tid), j = PM::col(k, tid);
    if (l <= nr) {
      const int i = wrapi(r0 - 1 + l, M);
      const unsigned pix = (unsigned)(i * L + j);
      float2 vbv, dbv;
      float hr = 0.f;
      if (start) {
        vbv = s0[k];
        dbv = s1[k];
      } else {
        const int lj = lpad(j);
        const float r = row_x<LS>(buf, l, nr, lj);
        if (l >= 1) hr = buf[(l - 1) * LS + lj].y;
        const float rr = row_x<LS>(buf, l, nr, lpad(j + 1 == L ? 0 : j + 1));
        const float rd = row_x<LS>(buf, l + 1, nr, lj);
        vbv = make_float2(mu * (rr - r), mu * (rd - r));
        dbv = make_float2(s0[k].x - vbv.x, s0[k].y - vbv.y);
      }
      float qb = 0.f;
      if (l >= 1) {
        const bool obs = (obsbits >> k) & 1u;
        if (start) {
          if (!obs) qb = a.alpha * sz[k];
        } else {
          if (obs) {
            yb[pix] = sz[k] + hr;
          } else {
            const float zn = (1.f - a.alpha) * sz[k] + hr;
            zb[pix] = zn;
            qb = a.alpha * zn;
          }
          if (end) { vb[pix] = vbv; db[pix] = dbv; }
        }
      }
      if (!end) {
        const float2 t = make_float2(vbv.x - dbv.x, vbv.y - dbv.y);
        float dt;
        const float2 jt = vsoft_vjp(su[k], t, tau, tau2, dt);
        const float2 ub = make_float2(dbv.x + jt.x, dbv.y + jt.y);
        ureg[k] = ub;
        if (l >= 1) {
          ubout[pix] = ub;
          lsum += dt;
        }
      }
      qreg[k] = qb;
    }
  }

  if (!end) {
    __shared__ double red[3 * (kNTR / 64)];
    double ls = lsum, z0 = 0.0, z1 = 0.0;
    block_sum3(ls, z0, z1, red);
    if (threadIdx.x == 0) a.lam_part[mt.rt0 + r0 / RT] += ls / (double)mu;
  } else {
    return;
  }

  // start the next reverse step: xb = D^T ub (+ grad_x), qb, forward row DFT
  const float* __restrict__ gx = a.grad_x ? a.grad_x + mt.px : nullptr;
  row_prologue<L, RT, KP>(buf, ureg, nr, tw, a.spec_out + mt.sp, M, r0, nh, nb, C, logC,
                          [&](int k, int l, int j, float g) {
                            const float xb = gx ? g + gx[(r0 - 1 + l) * L + j] : g;
                            return make_float2(xb, qreg[k]);
                          });
}

template <int L>
__global__ void __launch_bounds__(kNTR) bwd_row_kernel(BwdRowArgs a) {
  extern __shared__ float2 lds[];
  const int4 t = a.tiles[blockIdx.x];
  if (t.x < 0) return;
  bwd_row_tile<L>(a, t.x, t.y, lds);
}

template <int L0, int... Ls>
__device__ __forceinline__ void bwd_row_dispatch(const BwdRowArgs& a, int L, int img, int r0, float2* lds) {
  if (L == L0) {
    bwd_row_tile<L0>(a, img, r0, lds);
    return;
  }
  if constexpr (sizeof...(Ls) > 0) bwd_row_dispatch<Ls...>(a, L, img, r0, lds);
}

template <int... Ls>
__global__ void __launch_bounds__(kNTR, DCV_MULTI_ROW_WAVES) bwd_row_kernel_multi(BwdRowArgs a) {
  extern __shared__ float2 lds[];
  const int4 t = a.tiles[blockIdx.x];
  if (t.x < 0) return;
  bwd_row_dispatch<Ls...>(a, a.meta[t.x].n, t.x, t.y, lds);
}

template <int L>
__device__ __forceinline__ void bwd_col_tile(const BwdColArgs& a, int img, int blk, float2* lds) {
  constexpr int C = c_for(L);
  constexpr int LS = lstride(L);
  const ImgMeta mt = a.meta[img];
  float2* buf = lds;
  const float2* tw = twiddle_table<L, kNTC, kTwLdsCol>(lds + 2 * C * LS, a.tw + mt.twc);
  const long long base = mt.sp + (long long)blk * L * C;
  const float4* __restrict__ sin = a.spec_in + base;
  for (int q = threadIdx.x; q < L * C; q += kNTC) {
    const int i = q / C, c = q - i * C;
    const float4 v = sin[q];
    buf[(2 * c) * LS + lpad(i)] = make_float2(v.x, v.y);
    buf[(2 * c + 1) * LS + lpad(i)] = make_float2(v.z, v.w);
  }
  __syncthreads();
  fft_lines<L, false, kNTC, 2 * C, kEarlyTwCol>(buf, 2 * C, tw);
  const float mu = a.mu[img];
  const float mn = (float)L * (float)mt.n;
  const float scale = 1.0f / mn;
  const float2* __restrict__ hh = a.hh + mt.hh + (long long)blk * L * C;
  const float* __restrict__ dv2 = a.tab + mt.tab;
  const float* __restrict__ dh2 = dv2 + L;
  const float4* __restrict__ fs = a.fwd_spec + base;
  double2* S = a.S + mt.hh + (long long)blk * L * C;
  for (int q = threadIdx.x; q < L * C; q += kNTC) {
    const int ky = q / C, c = q - ky * C;
    const int kx = blk * C + c;
    const float2 XB = buf[(2 * c) * LS + lpad(ky)];
    const float2 QB = buf[(2 * c + 1) * LS + lpad(ky)];
    float2 R = make_float2(0.f, 0.f), HR = R;
    if (kx < mt.nh) {
      const float2 Hk = hh[q];
      const float den = Hk.x * Hk.x + Hk.y * Hk.y + mu * (dh2[kx] + dv2[ky]);
      // xb_hat = XB + conj(H) QB ; rb_hat = xb_hat / den
      const float2 xbh = make_float2(XB.x + Hk.x * QB.x + Hk.y * QB.y, XB.y + Hk.x * QB.y - Hk.y * QB.x);
      const float rden = frcp(den);
      const float2 rb = make_float2(xbh.x * rden, xbh.y * rden);
      const float4 f = fs[q];
      const float2 Y = make_float2(f.x, f.y);
      const float2 X = make_float2(f.z * mn, f.w * mn);
      // conj(QB) X + conj(Y) rb - 2 conj(H) Re(conj(rb) X), evaluated as
      // X conj(QB - H rb) + rb conj(Y - H X): the differences are the
      // spectra of the adjoint and data residuals; accumulated in FP64
      const float2 hr = cmul(Hk, rb), hx = cmul(Hk, X);
      const float2 a1 = make_float2(QB.x - hr.x, QB.y - hr.y);
      const float2 a2 = make_float2(Y.x - hx.x, Y.y - hx.y);
      double2 acc = S[q];
      acc.x += (double)X.x * a1.x + (double)X.y * a1.y + (double)rb.x * a2.x + (double)rb.y * a2.y;
      acc.y += (double)X.y * a1.x - (double)X.x * a1.y + (double)rb.y * a2.x - (double)rb.x * a2.y;
      S[q] = acc;
      R = make_float2(rb.x * scale, rb.y * scale);
      HR = cmul(Hk, R);
    }
    buf[(2 * c) * LS + lpad(ky)] = R;
    buf[(2 * c + 1) * LS + lpad(ky)] = HR;
  }
  __syncthreads();
  fft_lines<L, true, kNTC, 2 * C, kEarlyTwCol>(buf, 2 * C, tw);
  float4* __restrict__ sout = a.spec_out + mt.sp + (unsigned)(blk * C * mt.rb);
  const unsigned nbc = (unsigned)(mt.nb * C);
  for (int q = threadIdx.x; q < L * C; q += kNTC) {
    const int i = q / C, c = q - i * C;
    const float2 X = buf[(2 * c) * LS + lpad(i)];
    const float2 Q = buf[(2 * c + 1) * LS + lpad(i)];
    sout[row_block_index(mt, i, nbc) + c * mt.rb] = make_float4(X.x, X.y, Q.x, Q.y);
  }
}

template <int L>
__global__ void __launch_bounds__(kNTC) bwd_col_kernel(BwdColArgs a) {
  extern __shared__ float2 lds[];
  const int4 t = a.tiles[blockIdx.x];
  if (t.x < 0) return;
  bwd_col_tile<L>(a, t.x, t.y, lds);
}

template <int L0, int... Ls>
__device__ __forceinline__ void bwd_col_dispatch(const BwdColArgs& a, int L, int img, int blk, float2* lds) {
  if (L == L0) {
    bwd_col_tile<L0>(a, img, blk, lds);
    return;
  }
  if constexpr (sizeof...(Ls) > 0) bwd_col_dispatch<Ls...>(a, L, img, blk, lds);
}

template <int... Ls>
__global__ void __launch_bounds__(kNTC, DCV_MULTI_COL_WAVES) bwd_col_kernel_multi(BwdColArgs a) {
  extern __shared__ float2 lds[];
  const int4 t = a.tiles[blockIdx.x];
  if (t.x < 0) return;
  bwd_col_dispatch<Ls...>(a, a.meta[t.x].m, t.x, t.y, lds);
}

}  // namespace dcv
