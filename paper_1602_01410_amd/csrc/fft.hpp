// Device-side mixed-radix Stockham FFT for gfx950, staged in LDS.
//
// The x-step of the partial ADMM (eq. dual_x_iter_resolved_boundaries) is a
// BCCB solve, diagonal after a 2-D DFT (Sec. II-B); every transform of the
// library goes through the routines below.  A workgroup transforms a batch of
// "lines" (rows or columns) that sit in LDS, all of one compile-time length L
// = 2^a 3^c.  Each pass of radix R reads R values at stride L/R, applies the
// twiddles and an R-point DFT in registers, and writes them back in
// self-sorting (Stockham) order, so no bit reversal is needed.  Passes are
// radix 16/8/4/2 for the power-of-two part, radix 9 for each factor 3^2 and
// radix 3 for a last factor 3.
//
// Conventions: forward = exp(-2 pi i jk/L), inverse = exp(+2 pi i jk/L), both
// unnormalised (scaling is folded into the spectral solve).
#pragma once
#include <hip/hip_runtime.h>

namespace dcv {

// ---------------------------------------------------------------------------
// compile-time radix plan
// ---------------------------------------------------------------------------
constexpr int count3(int L) { int c = 0; while (L % 3 == 0) { L /= 3; ++c; } return c; }
constexpr int pow3(int c) { int p = 1; while (c-- > 0) p *= 3; return p; }
constexpr int ilog2(int v) { int a = 0; while ((1 << a) < v) ++a; return a; }

template <int L>
struct RadixPlan {
  static constexpr int c3 = count3(L);
  static constexpr int a = ilog2(L / pow3(c3));
  static constexpr int np2 = a > 0 ? (a + 3) / 4 : 0;   // radix <= 16 passes
  static constexpr int npass = np2 + c3 / 2 + c3 % 2;   // each 3^2 in one radix-9 pass
  static constexpr int radix(int k) {
    return k < np2 ? (1 << (a / np2 + (k < a % np2 ? 1 : 0))) : (k - np2 < c3 / 2 ? 9 : 3);
  }
  static constexpr int ns(int k) { int n = 1; for (int q = 0; q < k; ++q) n *= radix(q); return n; }
  static_assert((1 << a) * pow3(c3) == L, "length must be 2^a 3^c");
};

// LDS layout of one line: one padding slot every 16 complex values spreads
// the power-of-two strides of the Stockham writes over the banks.
#ifndef DCV_PAD_SHIFT
#define DCV_PAD_SHIFT 4
#endif
constexpr int kPadShift = DCV_PAD_SHIFT;
__host__ __device__ constexpr int lpad(int i) { return i + (i >> kPadShift); }
__host__ __device__ constexpr int lstride(int L) { return lpad(L) + 1; }

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by exp(-+ 2 pi i m / 16) with a constant m
template <int M, bool INV>
__device__ __forceinline__ float2 tw16(float2 a) {
  constexpr int m = M & 15;
  if constexpr (m == 0) return a;
  else if constexpr (m == 4) return mul_mi<INV>(a);
  else if constexpr (m == 8) return make_float2(-a.x, -a.y);
  else {
    // cos / sin of 2 pi m / 16, m = 0..15
    constexpr double kc[16] = {1, 0.92387953251128674, 0.70710678118654757, 0.38268343236508984, 6.123233995736766e-17, -0.38268343236508973, -0.70710678118654746, -0.92387953251128674, -1, -0.92387953251128685, -0.70710678118654768, -0.38268343236509034, -1.8369701987210297e-16, 0.38268343236509, 0.70710678118654735, 0.92387953251128652};
    constexpr double ks[16] = {0, 0.38268343236508978, 0.70710678118654746, 0.92387953251128674, 1, 0.92387953251128674, 0.70710678118654757, 0.38268343236508989, 1.2246467991473532e-16, -0.38268343236508967, -0.70710678118654746, -0.92387953251128652, -1, -0.92387953251128663, -0.70710678118654768, -0.38268343236509039};
    constexpr float c = (float)kc[m];
    constexpr float s = (float)ks[m];
    constexpr float sg = INV ? s : -s;   // forward exp(-i theta)
    return make_float2(a.x * c - a.y * sg, a.x * sg + a.y * c);
  }
}

// ---------------------------------------------------------------------------
// small DFTs in registers
// ---------------------------------------------------------------------------
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  }
};

template <bool INV> struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float h = 0.86602540378443864676f;   // sqrt(3)/2
    float2 a0 = v[0], s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    float2 m = make_float2(a0.x - 0.5f * s.x, a0.y - 0.5f * s.y);
    // forward: y1 = m - i h d, y2 = m + i h d; inverse swaps the signs
    float2 ihd = make_float2(-h * d.y, h * d.x);
    v[0] = cadd(a0, s);
    v[1] = INV ? cadd(m, ihd) : csub(m, ihd);
    v[2] = INV ? csub(m, ihd) : cadd(m, ihd);
  }
};

// multiply by exp(-+ 2 pi i m / 9) with a constant m (m = 1, 2, 4)
template <int M, bool INV>
__device__ __forceinline__ float2 tw9(float2 a) {
  // cos / sin of 2 pi m / 9
  constexpr double kc[5] = {1, 0.76604444311897801, 0.17364817766693041, -0.5, -0.93969262078590832};
  constexpr double ks[5] = {0, 0.64278760968653925, 0.98480775301220802, 0.86602540378443871,
                            0.34202014332566888};
  constexpr float c = (float)kc[M];
  constexpr float s = (float)ks[M];
  constexpr float sg = INV ? s : -s;   // forward exp(-i theta)
  return make_float2(a.x * c - a.y * sg, a.x * sg + a.y * c);
}

// 9 = 3 x 3: inner 3-point DFTs over n1 (stride 3), twiddle W9^(n2 k1), outer
// 3-point DFTs over n2; output index k1 + 3 k2.
template <bool INV> struct Dft<9, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t[3][3];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
      t[n2][0] = v[n2]; t[n2][1] = v[n2 + 3]; t[n2][2] = v[n2 + 6];
      Dft<3, INV>::run(t[n2]);
    }
    t[1][1] = tw9<1, INV>(t[1][1]); t[1][2] = tw9<2, INV>(t[1][2]);
    t[2][1] = tw9<2, INV>(t[2][1]); t[2][2] = tw9<4, INV>(t[2][2]);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      float2 u[3] = {t[0][k1], t[1][k1], t[2][k1]};
      Dft<3, INV>::run(u);
      v[k1] = u[0]; v[k1 + 3] = u[1]; v[k1 + 6] = u[2];
    }
  }
};

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2); a2 = csub(t0, t2); a1 = cadd(t1, t3); a3 = csub(t1, t3);
}

template <bool INV> struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }
};

template <bool INV> struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    o1 = tw16<2, INV>(o1); o2 = tw16<4, INV>(o2); o3 = tw16<6, INV>(o3);
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
  }
};

// 16 = 4 x 4: inner 4-point DFTs over n1 (stride 4), twiddle W16^(n2 k1),
// outer 4-point DFTs over n2; output index k1 + 4 k2.
template <bool INV> struct Dft<16, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      t[n2][0] = v[n2]; t[n2][1] = v[4 + n2]; t[n2][2] = v[8 + n2]; t[n2][3] = v[12 + n2];
      dft4<INV>(t[n2][0], t[n2][1], t[n2][2], t[n2][3]);
    }
    t[1][1] = tw16<1, INV>(t[1][1]); t[1][2] = tw16<2, INV>(t[1][2]); t[1][3] = tw16<3, INV>(t[1][3]);
    t[2][1] = tw16<2, INV>(t[2][1]); t[2][2] = tw16<4, INV>(t[2][2]); t[2][3] = tw16<6, INV>(t[2][3]);
    t[3][1] = tw16<3, INV>(t[3][1]); t[3][2] = tw16<6, INV>(t[3][2]); t[3][3] = tw16<9, INV>(t[3][3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 a0 = t[0][k1], a1 = t[1][k1], a2 = t[2][k1], a3 = t[3][k1];
      dft4<INV>(a0, a1, a2, a3);
      v[k1] = a0; v[k1 + 4] = a1; v[k1 + 8] = a2; v[k1 + 12] = a3;
    }
  }
};

// ---------------------------------------------------------------------------
// v[k] *= w^k with w = exp(-+2 pi i jm S / L), k = 1..R-1.  The powers w, w^2,
// w^4, w^8 come from the table (exact up to the float rounding of the table);
// the others are products of at most three of them.  twiddle_base reads the
// table entries, twiddle_mul forms the other powers and applies them, so that
// a pass can issue the reads before it waits on the workgroup barrier.
// ---------------------------------------------------------------------------
template <int R>
struct TwBase {
  static constexpr int n = R == 2 ? 1 : (R <= 4 ? 2 : (R == 8 ? 3 : 4));
  float2 w[n];   // w, w^2, w^4, w^8 (as many as radix R needs)
};
template <int R, int S>
__device__ __forceinline__ void twiddle_base(TwBase<R>& b, int jm, const float2* tw) {
  b.w[0] = tw[jm * S];
  if constexpr (TwBase<R>::n > 1) b.w[1] = tw[2 * jm * S];
  if constexpr (TwBase<R>::n > 2) b.w[2] = tw[4 * jm * S];
  if constexpr (TwBase<R>::n > 3) b.w[3] = tw[8 * jm * S];
}
template <int R, bool INV>
__device__ __forceinline__ void twiddle_mul(float2* v, const TwBase<R>& b) {
  float2 w[R];
  w[1] = b.w[0];
  if constexpr (R > 2) w[2] = b.w[1];
  if constexpr (R == 3) {
  } else if constexpr (R == 9) {
    w[3] = cmul(w[1], w[2]);
    w[4] = b.w[2];
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
    w[8] = b.w[3];
  } else if constexpr (R >= 4) {
    w[3] = cmul(w[1], w[2]);
    if constexpr (R >= 8) {
      w[4] = b.w[2];
      w[5] = cmul(w[4], w[1]);
      w[6] = cmul(w[4], w[2]);
      w[7] = cmul(w[4], w[3]);
    }
    if constexpr (R >= 16) {
      w[8] = b.w[3];
#pragma unroll
      for (int k = 9; k < 16; ++k) w[k] = cmul(w[8], w[k - 8]);
    }
  }
#pragma unroll
  for (int k = 1; k < R; ++k) {
    float2 t = w[k];
    if (INV) t.y = -t.y;
    v[k] = cmul(v[k], t);
  }
}
template <int R, int S, bool INV>
__device__ __forceinline__ void apply_twiddles(float2* v, int jm, const float2* tw) {
  TwBase<R> b;
  twiddle_base<R, S>(b, jm, tw);
  twiddle_mul<R, INV>(v, b);
}

// ---------------------------------------------------------------------------
// one Stockham pass over `nlines` lines of length L stored in LDS
// (line q at buf + q * LS, LS >= lstride(L)); NT threads cooperate, each takes up to
// MAXB butterflies.  tw is the LDS table exp(-2 pi i t / L), t < L.
// The caller must have synchronised after the last write of buf.
// ---------------------------------------------------------------------------
// (tid: the thread's index in the workgroup, threadIdx.x unless the caller
// passes a copy the compiler cannot see through).  With EARLY_TW the twiddle
// reads are issued together with the data reads, before the barrier, so that
// a table read from global memory waits on the barrier rather than after it.
template <int L, int R, int NS, bool INV, int NT, int MAXLINES, bool EARLY_TW = false, int LS = lstride(L)>
__device__ __forceinline__ void stockham_pass(float2* buf, int nlines, const float2* tw,
                                              unsigned tid = threadIdx.x) {
  constexpr int NB = L / R;
  constexpr int MAXB = (MAXLINES * NB + NT - 1) / NT;
  constexpr int S = L / (NS * R);
  const int total = nlines * NB;
  float2 v[MAXB][R];
  TwBase<R> wb[EARLY_TW && NS > 1 ? MAXB : 1];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = (int)tid + q * NT;
    if (idx < total) {
      const int line = idx / NB, j = idx - line * NB;
      const float2* src = buf + line * LS;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        // a stride that is a multiple of the padding period pads uniformly
        if constexpr (NB % (1 << kPadShift) == 0) v[q][k] = src[lpad(j) + k * lpad(NB)];
        else v[q][k] = src[lpad(j + k * NB)];
      }
      if constexpr (EARLY_TW && NS > 1) twiddle_base<R, S>(wb[q], j % NS, tw);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = (int)tid + q * NT;
    if (idx < total) {
      const int line = idx / NB, j = idx - line * NB;
      const int jm = j % NS;
      if constexpr (EARLY_TW && NS > 1) twiddle_mul<R, INV>(v[q], wb[q]);
      else if constexpr (NS > 1) apply_twiddles<R, S, INV>(v[q], jm, tw);
      Dft<R, INV>::run(v[q]);
      float2* dst = buf + line * LS;
      const int base = (j / NS) * NS * R + jm;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if constexpr (NS % (1 << kPadShift) == 0) dst[lpad(base) + k * lpad(NS)] = v[q][k];
        else dst[lpad(base + k * NS)] = v[q][k];
      }
    }
  }
  __syncthreads();
}

template <int L, bool INV, int NT, int MAXLINES, bool EARLY_TW = false, int LS = lstride(L), int P = 0>
__device__ __forceinline__ void fft_lines(float2* buf, int nlines, const float2* tw, unsigned tid = threadIdx.x) {
  if constexpr (P < RadixPlan<L>::npass) {
    stockham_pass<L, RadixPlan<L>::radix(P), RadixPlan<L>::ns(P), INV, NT, MAXLINES, EARLY_TW, LS>(buf, nlines, tw,
                                                                                                   tid);
    fft_lines<L, INV, NT, MAXLINES, EARLY_TW, LS, P + 1>(buf, nlines, tw, tid);
  }
}

// copy the global twiddle table of length L into LDS (caller synchronises)
template <int L, int NT>
__device__ __forceinline__ void load_twiddles(float2* tw_lds, const float2* __restrict__ tw_glob) {
  for (int t = threadIdx.x; t < L; t += NT) tw_lds[t] = tw_glob[t];
}

}  // namespace dcv
