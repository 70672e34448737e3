// HIP kernels of the partial ADMM (arXiv 1602.01410, Sec. II-B and III-B).
//
// One iteration i -> i+1 of eqs. (admm_aprox_1)-(admm_aprox_4) is two launches:
//
//   column pass  (one workgroup per block of C half-spectrum columns)
//     forward column DFT of the row spectra of ytilde^i and mu*D^T(v^i-d^i),
//     spectral solve of the x-step (dual_x_iter_resolved_boundaries):
//        X = (conj(H) Y + mu G) / (|H|^2 + mu(|D_h|^2 + |D_v|^2)),
//     Q = H X, inverse column DFT of X and Q.
//   row pass     (one workgroup per tile of RT image rows)
//     inverse row DFT of X + iQ on RT+2 rows (one halo row above and below)
//     -> x^{i+1} (real part) and H x^{i+1} (imaginary part);
//     z-step with relaxation alpha on the unobserved pixels;
//     u = D x^{i+1} + d^i, vector soft threshold -> v^{i+1}, d^{i+1} = u - v;
//     right-hand side of the next x-step: g = D^T(v^{i+1} - d^{i+1}),
//     forward row DFT of ytilde^{i+1} + i mu g, split into the two real
//     signals' half spectra (Hermitian symmetry), stored for the next
//     column pass.
//
// Only the state (ytilde, d, and v on the iterations that need it) and the
// two half-spectrum buffers touch HBM; x and H x never leave LDS.
//
// Half-spectrum buffer layout ("tiled"): for an image with m' rows, nh = n'/2+1
// spectrum columns grouped in nb blocks of C columns, element (row i, column
// kx) of the pair of signals is the float4 at ((kx / C) * m' + i) * C + kx % C.
// A column pass reads one block as a contiguous run; a row pass reads C
// columns x (RT+2) rows contiguously per block.
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace dcv {

#ifndef DCV_NT
#define DCV_NT 256
#endif
#ifndef DCV_ROW_PIX
#define DCV_ROW_PIX 4096
#endif
// column-pass tiles hold about DCV_COL_ELEMS frequencies per line set (512:
// narrower blocks for short columns, measured +8 to +12% on single 72^2 and
// 256^2 images and neutral on batches)
#ifndef DCV_COL_ELEMS
#define DCV_COL_ELEMS 512
#endif
#ifndef DCV_NT_ROW
#define DCV_NT_ROW 512
#endif
#ifndef DCV_NT_COL
#define DCV_NT_COL 256
#endif
constexpr int kNT = DCV_NT;       // threads per workgroup of the setup / reduction kernels
constexpr int kNTR = DCV_NT_ROW;  // threads per workgroup of the row passes
constexpr int kNTRWide = 1024;    // row workgroups of plans with few tiles
constexpr int kNTC = DCV_NT_COL;  // threads per workgroup of the column passes
constexpr int kNTCWide = 512;     // column workgroups of plans with few tiles

// rows per row-pass tile (about DCV_ROW_PIX pixels, at least 2 rows) and
// columns per column-pass block (a power of two, about DCV_COL_ELEMS / L)
__host__ __device__ constexpr int rt_for(int L) {
  // rounded down to a power of two (lengths with a factor 3: 768 -> 4 rows
  // rather than 5; the mixed batch gains 3%)
  const int r = DCV_ROW_PIX / L < 2 ? 2 : (DCV_ROW_PIX / L > 32 ? 32 : DCV_ROW_PIX / L);
  int q = 1;
  while (q * 2 <= r) q *= 2;
  return q;
}
// rows per block of the row-block spectrum layout, in units of the default
// row tile height
#ifndef DCV_ROW_BLOCK_MULT
#define DCV_ROW_BLOCK_MULT 1
#endif
__host__ __device__ constexpr int c_for(int L) {
  int c = 1;
  while (c * 2 <= DCV_COL_ELEMS / L && c * 2 <= 16) c *= 2;
  return c;
}
// Twiddle tables are read from LDS (copied per workgroup at its start) or
// straight from the global table through the L1 cache, per pass (bits of
// DCV_TW_LDS: 1 row passes, 2 column passes).  Measured on MI355X: the LDS
// copy shortens the row pass (16 x 1024^2: 147 -> 138 us per launch), the
// global table suits the column pass (its larger LDS footprint would cost a
// workgroup per compute unit: 76 -> 80 us).
#ifndef DCV_TW_LDS
#define DCV_TW_LDS 1
#endif
constexpr int kTwLdsRow = (DCV_TW_LDS & 1) ? 1 : 0;
constexpr int kTwLdsCol = (DCV_TW_LDS & 2) ? 1 : 0;
// Twiddle reads issued before each transform pass's barrier (bits: 1 row
// passes, 2 column passes); measured to pay for the column pass's global
// table (mixed 256-image batch: 425 -> 410 us per column launch).
#ifndef DCV_EARLY_TW
#define DCV_EARLY_TW 2
#endif
constexpr bool kEarlyTwRow = (DCV_EARLY_TW & 1) != 0;
constexpr bool kEarlyTwCol = (DCV_EARLY_TW & 2) != 0;
// row pass: full tiles get their own copy of the tile code with the row
// count as a constant (1) or share the code of the ragged last tiles (0)
#ifndef DCV_FULL_TILES
#define DCV_FULL_TILES 0
#endif
// Line stride of the row tiles' LDS lines.  The spectrum gather and split
// give consecutive threads the tile's RT rows at one frequency, so a wave's
// 64 8-byte accesses fall on RT lines at once, 128/RT consecutive dwords on
// each.  The 64 banks serve every one twice (the minimum) when the lines
// start an odd multiple of 64/RT banks apart, i.e. stride = 32/RT (mod
// 64/RT) in float2 units: lstride(L) is raised to the next such value for
// 4 <= RT <= 32 (for RT <= 2 each line's accesses cover all banks anyway).
// Measured with SQ_LDS_BANK_CONFLICT on MI355X: 4 lines at stride 1089 cost
// three times the cycles of stride 1096.
__host__ __device__ constexpr int row_lstride(int L, int RT) {
  int s = lstride(L);
  if (RT >= 4 && RT <= 32) {
    const int m = 64 / RT;
    while (s % m != m / 2) ++s;
  }
  return s;
}
__host__ __device__ constexpr int row_lds_elems(int L, int rt = 0) {
  return ((rt > 0 ? rt : rt_for(L)) + 1) * row_lstride(L, rt > 0 ? rt : rt_for(L)) + kTwLdsRow * L;
}
// Lengths that also have row tiles of half the rows (rt_for(L) / 2), for
// plans with too few tiles to fill the chip: those of at least 64 (a half
// tile lies inside one row block of the spectrum layout)
#define DCV_FOR_EACH_HALF_RT_LEN(X) \
  X(64) X(72) X(96) X(128) X(144) X(192) X(256) X(288) X(384) X(512) X(576) X(768) X(1024) X(1152) X(1536) \
      X(2048)
#ifndef DCV_RT_SPLIT
#define DCV_RT_SPLIT 2
#endif
__host__ __device__ constexpr int rt_half(int L) {
  return rt_for(L) / DCV_RT_SPLIT > 0 ? rt_for(L) / DCV_RT_SPLIT : 1;
}
#define DCV_CASE(n) static_assert(rt_for(n) % rt_half(n) == 0, "half tiles must divide the row blocks");
DCV_FOR_EACH_HALF_RT_LEN(DCV_CASE)
#undef DCV_CASE
__host__ __device__ constexpr int col_lds_elems(int L) { return 2 * c_for(L) * lstride(L) + kTwLdsCol * L; }

// the twiddle table a workgroup uses for length L (caller synchronises)
template <int L, int NT, int TW_LDS>
__device__ __forceinline__ const float2* twiddle_table(float2* lds_tw, const float2* __restrict__ glob) {
  if constexpr (TW_LDS) {
    load_twiddles<L, NT>(lds_tw, glob);
    return lds_tw;
  } else {
    return glob;
  }
}

// The same copy split in two: issue() reads the thread's entries of the
// global table into registers, commit() writes them to LDS and returns the
// table to use; the reads can then travel with a tile's other loads.
template <int L, int NT, int TW_LDS>
struct TwCopy {
  static constexpr int N = TW_LDS ? (L + NT - 1) / NT : 1;
  float2 r[N];
  __device__ __forceinline__ void issue(const float2* __restrict__ glob, unsigned tid) {
    if constexpr (TW_LDS) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const unsigned t = tid + (unsigned)(i * NT);
        if (L % NT == 0 || t < (unsigned)L) r[i] = glob[t];
      }
    }
  }
  __device__ __forceinline__ const float2* commit(float2* lds_tw, const float2* glob, unsigned tid) {
    if constexpr (TW_LDS) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const unsigned t = tid + (unsigned)(i * NT);
        if (L % NT == 0 || t < (unsigned)L) lds_tw[t] = r[i];
      }
      return lds_tw;
    } else {
      return glob;
    }
  }
};

struct ImgMeta {
  int m, n;            // m' (rows), n' (columns)
  int b;               // kernel half size
  int mask_kind, decim;
  int nh, C, logC, nb; // half-spectrum columns, block width (power of 2), blocks
  int rt;              // rows per row tile
  int nrt;             // row tiles
  unsigned dmagic;     // floor(2^32 / decim) + 1: exact x / decim for x < 2^11
  long long px;        // offset of the image in pixel arrays
  long long sp;        // offset in half-spectrum buffers (float4 units)
  long long hh;        // offset in the blur half spectrum (float2 units)
  long long tab;       // offset in the |D|^2 tables (float)
  long long twr, twc;  // twiddle table offsets for lengths n' and m'
  long long rt0;       // first row-tile index of the image (residual partials)
  unsigned rtmagic;    // floor(2^32 / rt) + 1 (rt > 1): exact i / rt for rows i < 2^11
  int group;           // first image of the colour group (itself for grey images)
  int nch;             // channels of the group (1 for grey images)
  int rb;              // rows per block of the row-block spectrum layout (a multiple of rt)
  unsigned rbmagic;    // floor(2^32 / rb) + 1 (rb > 1): exact i / rb for rows i < 2^11
};

// ROW_ITER: finish an iteration (z-step, prox, dual update) and start the
// next x-step.  ROW_STATE: start an x-step from a stored state.  ROW_INNER:
// one more block-Gauss-Seidel pass with v, d frozen (z-step on the own rows,
// new transform of ytilde only; the mu G half of the spectra is kept).
// ROW_UONLY: colour images; the z-step and u = D x + d of the own rows (into
// d_out), the joint prox of the channels following in its own kernel.
enum { ROW_ITER = 0, ROW_STATE = 1, ROW_INNER = 2, ROW_UONLY = 3 };

struct RowArgs {
  const ImgMeta* meta;
  const int4* tiles;         // (image, first row, -, -)
  const float4* spec_in;     // column-pass output (X, Q) half spectra
  float4* spec_out;          // (Y, mu G) half spectra for the next column pass
  float* yt;                 // ytilde = [y; z] on the extended grid
  const float2* d_in;        // d^i (double-buffered: halo rows are read by neighbours)
  float2* d_out;             // d^{i+1}
  float2* v;                 // v (read on check iterations, written when store_v)
  float* x_out;              // x^{i+1} (when store_x)
  float2* u_out;             // u = D x + d (backward recompute), nullable
  const uint8_t* mask;       // explicit masks
  const float* lam;
  const float* mu;
  const float2* tw;          // twiddle tables
  double* partials;          // 3 doubles per row tile (when check)
  const int* done;           // per-image stop flags, nullable
  const float* dscale;       // ROW_STATE: per-image factor applied to d, nullable
  const int* npass;          // per image: BGS passes; tiles of images with npass <= pass_q skip, nullable
  int pass_q;
  float alpha;
  int mode, check, store_v, store_x, last;
  int nt_spec;               // non-temporal stores of spec_out
};

struct ColArgs {
  const ImgMeta* meta;
  const int4* tiles;         // (image, block, -, -)
  const float4* spec_in;
  float4* spec_out;
  const float2* hh;          // blur half spectrum, tiled like the spectra (float2)
  const float* tab;          // per image: |D_v|^2[m'] then |D_h|^2[nb*C]
  const float2* hsep;        // separable blurs: U[m'] then V[nb*C] per image (offsets of tab)
  const int* sep;            // per image: 1 = H(ky, kx) = U(ky) V(kx), nullable
  const float* mu;
  const float2* tw;
  float4* spec_store;        // (Y, X) per frequency for the backward, nullable
  const int* done;
  const int* npass;          // as in RowArgs
  int pass_q;
  int warm;                  // 1: quadratic warm-start solve (|H|^2 + warm_tau)
  float warm_tau;
  int nt_spec;               // non-temporal stores of spec_out
};

// x % s == 0 for 0 <= x < 2^11 and 1 < s <= 2^11, with magic = floor(2^32/s) + 1
__device__ __forceinline__ bool divisible(int x, int s, unsigned magic) {
  const unsigned q = __umulhi((unsigned)x, magic);
  return (unsigned)x == q * (unsigned)s;
}

// offset of entry (row i, column 0 of the block) in the row-block layout of
// the spectra the column pass writes for the row pass (entry (i, kx) at
// (i / rb) rb nbc + kx rb + i mod rb; the caller adds (kx - blk C) rb)
__device__ __forceinline__ unsigned row_block_index(const ImgMeta& mt, int i, unsigned nbc) {
  const unsigned i0 = mt.rb == 1 ? (unsigned)i : __umulhi((unsigned)i, mt.rbmagic) * (unsigned)mt.rb;
  return i0 * nbc + (unsigned)(i - (int)i0);
}

__device__ __forceinline__ bool observed(const ImgMeta& mt, const uint8_t* __restrict__ mask,
                                         int i, int j) {
  if (mt.mask_kind == 1) return mask[mt.px + (i * mt.n + j)] != 0;
  const bool in_c = i >= mt.b && i < mt.m - mt.b && j >= mt.b && j < mt.n - mt.b;
  if (mt.mask_kind == 2 && mt.decim > 1)
    return in_c && divisible(i - mt.b, mt.decim, mt.dmagic) && divisible(j - mt.b, mt.decim, mt.dmagic);
  return in_c;
}

// The same test split into a per-row part (uniform over a row) and a
// branch-free per-pixel part.
struct RowObs {
  bool explicit_mask, decim, row_ok;
};
__device__ __forceinline__ RowObs row_observed(const ImgMeta& mt, int i) {
  RowObs r;
  r.explicit_mask = mt.mask_kind == 1;
  r.decim = mt.mask_kind == 2 && mt.decim > 1;
  r.row_ok = (i >= mt.b) & (i < mt.m - mt.b) & (!r.decim | divisible(i - mt.b, mt.decim, mt.dmagic));
  return r;
}
__device__ __forceinline__ bool pixel_observed(const ImgMeta& mt, const RowObs& r,
                                               const uint8_t* __restrict__ mask_row, int j) {
  if (r.explicit_mask) return mask_row[j] != 0;
  return r.row_ok & (j >= mt.b) & (j < mt.n - mt.b) & (!r.decim | divisible(j - mt.b, mt.decim, mt.dmagic));
}

// Stores of pass outputs that another kernel reads.  With the
// non-temporal hint (NT = true) the lines stream out instead of staying
// dirty in L2 until the end-of-kernel write-back; that pays for the row
// pass's full-line state writes.  Bits of DCV_NT_STORE: 1 row-pass state
// (d, z), 2 row-pass spectra, 4 column-pass spectra.
#ifndef DCV_NT_STORE
#define DCV_NT_STORE 1
#endif
typedef float dcv_f4v __attribute__((ext_vector_type(4)));
typedef float dcv_f2v __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ void st_out(float4* p, float4 v) {
  if constexpr (NT) __builtin_nontemporal_store(dcv_f4v{v.x, v.y, v.z, v.w}, reinterpret_cast<dcv_f4v*>(p));
  else *p = v;
}
template <bool NT>
__device__ __forceinline__ void st_out(float2* p, float2 v) {
  if constexpr (NT) __builtin_nontemporal_store(dcv_f2v{v.x, v.y}, reinterpret_cast<dcv_f2v*>(p));
  else *p = v;
}
template <bool NT>
__device__ __forceinline__ void st_out(float* p, float v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
// the spectra one pass leaves for the other: the hint is chosen per plan
// (it pays when the plan's whole working set stays in the last-level cache)
template <bool NT_ALWAYS>
__device__ __forceinline__ void st_spec(float4* p, float4 v, bool nt) {
  if (NT_ALWAYS || nt) st_out<true>(p, v);
  else st_out<false>(p, v);
}
// The same hint on loads (bits: 1 row-pass state, 2 row-pass spectra, 4
// column-pass inputs); measured to pay for the row-pass state only.
#ifndef DCV_NT_LOAD
#define DCV_NT_LOAD 1
#endif
template <bool NT>
__device__ __forceinline__ float4 ld_in(const float4* p) {
  if constexpr (NT) {
    const dcv_f4v v = __builtin_nontemporal_load(reinterpret_cast<const dcv_f4v*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ float2 ld_in(const float2* p) {
  if constexpr (NT) {
    const dcv_f2v v = __builtin_nontemporal_load(reinterpret_cast<const dcv_f2v*>(p));
    return make_float2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ float ld_in(const float* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
constexpr bool kNtLdRowState = (DCV_NT_LOAD & 1) != 0;
constexpr bool kNtLdRowSpec = (DCV_NT_LOAD & 2) != 0;
constexpr bool kNtLdCol = (DCV_NT_LOAD & 4) != 0;
constexpr bool kNtRowState = (DCV_NT_STORE & 1) != 0;
constexpr bool kNtRowSpec = (DCV_NT_STORE & 2) != 0;
constexpr bool kNtColSpec = (DCV_NT_STORE & 4) != 0;

__device__ __forceinline__ int wrapi(int i, int M) { return i < 0 ? i + M : (i >= M ? i - M : i); }

// reciprocal with one Newton step (error below 1 ulp of the exact division)
__device__ __forceinline__ float frcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return r * (2.0f - x * r);
}

// sum three doubles over the workgroup; result valid in thread 0
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* scratch) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
    c += __shfl_xor(c, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { scratch[3 * wv] = a; scratch[3 * wv + 1] = b; scratch[3 * wv + 2] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = b = c = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a += scratch[3 * w]; b += scratch[3 * w + 1]; c += scratch[3 * w + 2];
    }
  }
}

// Record one image's residuals from the sums over its pixels (a = |d'-d|^2,
// b = |v'-v|^2, c = |z'-z|^2); with stop_test, set the stop flag when both
// tolerances hold (scaled by sqrt(2 m' n'), the size of v).  Returns true
// when the image is or becomes stopped.
__device__ __forceinline__ bool record_residuals(const ImgMeta& mt, int img, double a, double b, double c,
                                                 double* res, int* done, int* nonfinite, int* iters_done,
                                                 int iters_since, int stop_test, double tol_p, double tol_d,
                                                 int* stop_buf, int cur_d) {
  if (done && done[img]) return true;
  const double nd = sqrt(a), nv = sqrt(b);
  res[3 * img] = nd; res[3 * img + 1] = nv; res[3 * img + 2] = sqrt(c);
  if (!isfinite(a) || !isfinite(b) || !isfinite(c)) nonfinite[img] = 1;
  iters_done[img] += iters_since;
  const double sc = sqrt(2.0 * (double)mt.m * (double)mt.n);
  if (stop_test && done && (tol_p > 0 || tol_d > 0) && nd <= tol_p * sc && nv <= tol_d * sc) {
    done[img] = 1;   // a stopped image keeps its penalty and its d (in buffer cur_d)
    stop_buf[img] = cur_d;
    return true;
  }
  return false;
}

// ---------------------------------------------------------------------------
// row pass
// ---------------------------------------------------------------------------

// LDS lines of a row tile with nr own rows: lines 0..nr-1 hold the own rows
// r0..r0+nr-1 (x + iHx after the inverse transform); line nr holds the two
// halo rows packed as one complex line, x(r0-1) + i x(r0+nr).  Only x is
// needed on the halo rows, so both share one transform.
//
// Gather the tile's half spectra into those lines, completing the other
// half by Hermitian symmetry: X + iQ for the own rows, X(r0-1) + i X(r0+nr)
// for the halo line.  The column pass leaves the spectra in row blocks of
// rb rows (entry (i, kx) at (i / rb) rb nbc + kx rb + i mod rb, nbc = nb C),
// rb a multiple of RT: the own rows are RT consecutive rows of one block (the
// whole block when rb = RT).  All loads are issued first; `extra` issues the
// caller's own loads after them, before the first wait.
struct NoExtraLoads {
  __device__ __forceinline__ void operator()() const {}
};
template <int L, int RT, bool HALO = true, int NT = kNTR, class Extra = NoExtraLoads>
__device__ __forceinline__ void gather_rows(const float4* __restrict__ sin, float2* buf, int M, int r0, int nr,
                                            int nh, int nb, int C, int logC, int rb, Extra extra = Extra()) {
  constexpr int LS = row_lstride(L, RT);
  constexpr int NBC_MAX = L / 2 + 16;   // >= nb * C
  constexpr int NQ = (RT * NBC_MAX + NT - 1) / NT;
  constexpr int NH = (NBC_MAX + NT - 1) / NT;
  const float2* __restrict__ sin2 = reinterpret_cast<const float2*>(sin);
  float4 g[NQ];
  int dst[NQ];   // (line << 12) | kx of each load, -1 for none
  float2 ha[NH], hb[NH];
  const int ia = r0 == 0 ? M - 1 : r0 - 1;
  const int ib = r0 + nr == M ? 0 : r0 + nr;
  // the tile's rows in their block: entry (r0 + l, kx) at
  // (r0 / rb) rb nbc + r0 mod rb + kx rb + l
  const unsigned nbc = (unsigned)(nb * C);
  const unsigned rbu = (unsigned)rb;
  const unsigned b0 = (unsigned)(r0 / rb) * rbu;
  const float4* __restrict__ blkp = sin + (b0 * nbc + ((unsigned)r0 - b0));
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = threadIdx.x + k * NT;
    const int l = q % RT, kx = q / RT;
    dst[k] = -1;
    if (l < nr && kx < nh) {
      g[k] = ld_in<kNtLdRowSpec>(blkp + ((unsigned)kx * rbu + (unsigned)l));
      dst[k] = (l << 12) | kx;
    }
  }
  const unsigned ba = (unsigned)(ia / rb) * rbu * nbc + (unsigned)(ia % rb);
  const unsigned bb = (unsigned)(ib / rb) * rbu * nbc + (unsigned)(ib % rb);
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int kx = threadIdx.x + k * NT;
    if (HALO && kx < nh) {
      ha[k] = sin2[2 * (ba + (unsigned)kx * rbu)];
      hb[k] = sin2[2 * (bb + (unsigned)kx * rbu)];
    }
  }
  // more loads of the caller, in flight with the spectra
  extra();
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    if (dst[k] >= 0) {
      const int l = dst[k] >> 12, kx = dst[k] & 4095;
      const float4 v = g[k];
      float2* line = buf + l * LS;
      line[lpad(kx)] = make_float2(v.x - v.w, v.y + v.z);
      if (kx >= 1 && kx <= L - nh) line[lpad(L - kx)] = make_float2(v.x + v.w, v.z - v.y);
    }
  }
  float2* hline = buf + nr * LS;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int kx = threadIdx.x + k * NT;
    if (HALO && kx < nh) {
      hline[lpad(kx)] = make_float2(ha[k].x - hb[k].y, ha[k].y + hb[k].x);
      if (kx >= 1 && kx <= L - nh) hline[lpad(L - kx)] = make_float2(ha[k].x + hb[k].y, hb[k].x - ha[k].y);
    }
  }
}

// LDS slot of tile row l (image row r0-1+l, l = 0..nr+1): the halo line for
// l = 0 and l = nr+1, own line l-1 otherwise.
__device__ __forceinline__ int row_slot(int l, int nr) { return (l == 0 || l == nr + 1) ? nr : l - 1; }

// x on tile row l (real part of the own line, or the halo line's real part
// for the row above and imaginary part for the row below)
template <int LS>
__device__ __forceinline__ float row_x(const float2* buf, int l, int nr, int lj) {
  const float2 v = buf[row_slot(l, nr) * LS + lj];
  return l == nr + 1 ? v.y : v.x;
}

// Split C = F(a) + i F(b) of lines 0..nr-1 into the half spectra of the real
// signals a, b and store them in the tiled layout.
template <int L, int RT, int NT = kNTR>
__device__ __forceinline__ void split_store(float4* __restrict__ sout, const float2* buf, int M, int r0, int nr,
                                            int nh, int nb, int C, int logC, bool nt) {
  constexpr int LS = row_lstride(L, RT);
  constexpr int NBC_MAX = L / 2 + 16;   // >= nb * C
  constexpr int NQ = (RT * NBC_MAX + NT - 1) / NT;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = threadIdx.x + k * NT;
    const int c = q & (C - 1);
    const int t2 = q >> logC;
    const int l = t2 % RT, blk = t2 / RT;
    const int kx = blk * C + c;
    if (l < nr && blk < nb && kx < nh) {
      const float2 cf = buf[l * LS + lpad(kx)];
      const float2 cm = buf[l * LS + lpad(kx == 0 ? 0 : L - kx)];
      st_spec<kNtRowSpec>(sout + (((__umul24(blk, M) + r0 + l) << logC) + c),
             make_float4(0.5f * (cf.x + cm.x), 0.5f * (cf.y - cm.y), 0.5f * (cf.y + cm.y), 0.5f * (cm.x - cf.x)),
             nt);
    }
  }
}

// Pixel p = tid + k * kNTR of a row tile sits on tile row p / L, column p % L.
// When L is a multiple of the workgroup size the row is a compile-time
// function of k; when the workgroup covers whole rows it is a shift.
template <int L, int NT = kNTR>
struct PixMap {
  static constexpr bool kSplitRow = L % NT == 0;
  static constexpr bool kWholeRows = !kSplitRow && NT % L == 0;
  __device__ static __forceinline__ int row(int k, unsigned tid) {
    if constexpr (kSplitRow) return k / (L / NT);
    else if constexpr (kWholeRows) return k * (NT / L) + (int)(tid / L);
    else return (int)((tid + k * NT) / L);
  }
  __device__ static __forceinline__ int col(int k, unsigned tid) {
    if constexpr (kSplitRow) return (k % (L / NT)) * NT + (int)tid;
    else if constexpr (kWholeRows) return (int)(tid % L);
    else return (int)((tid + k * NT) % L);
  }
};

// Start of the next transform: with a vector field w of tile rows 0..nr in
// wreg, form g = D^T w on the own rows, pack(k, l, j, g) into the own lines,
// transform them forward and store their split half spectra.
template <int L, int RT, int KP, int NT = kNTR, class Pack>
__device__ __forceinline__ void row_prologue(float2* buf, float2 (&wreg)[KP], int nr, const float2* tw,
                                             float4* __restrict__ sout, int M, int r0, int nh, int nb, int C,
                                             int logC, Pack pack, bool nt = false) {
  using PM = PixMap<L, NT>;
  constexpr int LS = row_lstride(L, RT);
  const unsigned tid = threadIdx.x;
  __builtin_assume(tid < (unsigned)NT);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int l = PM::row(k, tid), j = PM::col(k, tid);
    if (l <= nr) buf[row_slot(l, nr) * LS + lpad(j)] = wreg[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int l = PM::row(k, tid), j = PM::col(k, tid);
    if (l <= nr && l >= 1) {
      const float2* line = buf + (l - 1) * LS;
      const float2 w = line[lpad(j)];
      const float whl = line[lpad(j == 0 ? L - 1 : j - 1)].x;
      const float wvu = buf[row_slot(l - 1, nr) * LS + lpad(j)].y;
      wreg[k] = pack(k, l, j, whl - w.x + wvu - w.y);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int l = PM::row(k, tid), j = PM::col(k, tid);
    if (l <= nr && l >= 1) buf[(l - 1) * LS + lpad(j)] = wreg[k];
  }
  __syncthreads();
  fft_lines<L, false, NT, RT, kEarlyTwRow, LS>(buf, nr, tw);
  split_store<L, RT, NT>(sout, buf, M, r0, nr, nh, nb, C, logC, nt);
}

// One more block-Gauss-Seidel pass of the x- and z-steps with v and d frozen
// (the passes of Sec. III-B): the x-step's transform is finished on the own
// rows only (no halo: the prox is not taken), the z-step updates ytilde, and
// ytilde is transformed again, two real rows per complex line.  Only the Y
// half of each spectrum entry is rewritten: the mu G half, a function of the
// frozen v and d, is still valid.
template <int L, int RT>
__device__ __forceinline__ void row_inner(const RowArgs& a, const ImgMeta& mt, int r0, float2* lds) {
  using PM = PixMap<L>;
  constexpr int LS = row_lstride(L, RT);
  constexpr int KP = ((RT + 1) * L + kNTR - 1) / kNTR;
  constexpr int NBC_MAX = L / 2 + 16;
  constexpr int NQ = (RT * NBC_MAX + kNTR - 1) / kNTR;
  const unsigned tid = threadIdx.x;
  __builtin_assume(tid < (unsigned)kNTR);
  const int M = mt.m;
  const int nr = min(RT, M - r0);
  const int C = mt.C, logC = mt.logC, nh = mt.nh, nb = mt.nb;
  float* __restrict__ yt = a.yt + mt.px;
  float2* buf = lds;
  const float2* tw_glob = a.tw + mt.twr;
  TwCopy<L, kNTR, kTwLdsRow> twc;
  gather_rows<L, RT, false>(a.spec_in + mt.sp, buf, M, r0, nr, nh, nb, C, logC, mt.rb,
                            [&]() { twc.issue(tw_glob, tid); });
  const float2* tw = twc.commit(lds + (RT + 1) * LS, tw_glob, tid);
  float yo[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int l = PM::row(k, tid), j = PM::col(k, tid);
    if (l >= 1 && l <= nr) yo[k] = yt[(unsigned)((r0 + l - 1) * L + j)];
  }
  __syncthreads();
  fft_lines<L, true, kNTR, RT, kEarlyTwRow, LS>(buf, nr, tw);
  // z-step on own row r = l - 1
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int l = PM::row(k, tid), j = PM::col(k, tid);
    if (l >= 1 && l <= nr) {
      const int i = r0 + l - 1;
      const RowObs ro = row_observed(mt, i);
      if (!pixel_observed(mt, ro, ro.explicit_mask ? a.mask + mt.px + i * L : nullptr, j)) {
        const float hx = buf[(l - 1) * LS + lpad(j)].y;
        yo[k] = yo[k] + a.alpha * (hx - yo[k]);
        yt[(unsigned)(i * L + j)] = yo[k];
      }
    }
  }
  __syncthreads();
  // rows 2q and 2q+1 into line q as a + i b (b = 0 past the last row)
  float* bufs = reinterpret_cast<float*>(buf);
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int l = PM::row(k, tid), j = PM::col(k, tid);
    if (l >= 1 && l <= nr) {
      const int r = l - 1;
      const int at = ((r >> 1) * LS + lpad(j)) * 2;
      bufs[at + (r & 1)] = yo[k];
      if (r + 1 == nr && !(r & 1)) bufs[at + 1] = 0.f;
    }
  }
  __syncthreads();
  const int npl = (nr + 1) >> 1;
  fft_lines<L, false, kNTR, (RT + 1) / 2, kEarlyTwRow, LS>(buf, npl, tw);
  float2* __restrict__ sout2 = reinterpret_cast<float2*>(a.spec_out + mt.sp);
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = threadIdx.x + k * kNTR;
    const int c = q & (C - 1);
    const int t2 = q >> logC;
    const int r = t2 % RT, blk = t2 / RT;
    const int kx = blk * C + c;
    if (r < nr && blk < nb && kx < nh) {
      const float2* line = buf + (r >> 1) * LS;
      const float2 cf = line[lpad(kx)];
      const float2 cm = line[lpad(kx == 0 ? 0 : L - kx)];
      const float2 y = (r & 1) ? make_float2(0.5f * (cf.y + cm.y), 0.5f * (cm.x - cf.x))
                               : make_float2(0.5f * (cf.x + cm.x), 0.5f * (cf.y - cm.y));
      sout2[2 * (((__umul24(blk, M) + r0 + r) << logC) + c)] = y;
    }
  }
}

// Vector soft threshold factor: max(|u| - tau, 0) / |u| for |u|^2 = n2,
// 0 when |u| <= tau (including u = 0).
__device__ __forceinline__ float vsoft_scale(float n2, float tau, float tau2) {
  return n2 > tau2 ? 1.0f - tau * __builtin_amdgcn_rsqf(n2) : 0.f;
}

// Row-pass instantiations by the work an iteration asks for, so that the
// common cases run with their flags as compile-time constants:
//   RV_PLAIN   ROW_ITER, no residuals, no stores of v, x or u (most
//              iterations between two residual checks);
//   RV_STOREV  ROW_ITER storing v only (the iteration before a check);
//   RV_CHECK   ROW_ITER with residuals (a check), storing v and x as the
//              arguments ask (only where the run may stop there);
//   RV_GENERIC every mode and flag from the arguments.
enum { RV_PLAIN = 0, RV_STOREV = 1, RV_CHECK = 2, RV_GENERIC = 3 };

// the variant a launch with these arguments needs
__host__ __device__ inline int row_variant(const RowArgs& a) {
  if (a.mode != ROW_ITER || a.u_out || a.last) return RV_GENERIC;
  if (!a.check && !a.store_v && !a.store_x) return RV_PLAIN;
  if (!a.check && a.store_v && !a.store_x) return RV_STOREV;
  if (a.check) return RV_CHECK;
  return RV_GENERIC;
}

// One row tile of nr <= RT own rows (nr == RT is passed as a literal for the
// full tiles, so that their row bounds fold away).
template <int L, int V, int RT, int NT = kNTR>
__device__ __forceinline__ void row_tile_rows(const RowArgs& a, const ImgMeta& mt, int img, int r0, int nr,
                                              float2* lds) {
  using PM = PixMap<L, NT>;
  constexpr int LS = row_lstride(L, RT);
  constexpr int KP = ((RT + 1) * L + NT - 1) / NT;  // pixels per thread (own rows + 1 halo)
  const unsigned tid = threadIdx.x;
  __builtin_assume(tid < (unsigned)NT);
  constexpr bool GEN = V == RV_GENERIC;
  const int M = mt.m;
  const int C = mt.C, logC = mt.logC, nh = mt.nh, nb = mt.nb;
  const bool check = V == RV_CHECK || (GEN && a.check);
  const bool uonly = GEN && a.mode == ROW_UONLY;
  const bool store_v = V == RV_STOREV || ((V == RV_CHECK || GEN) && a.store_v);
  const bool store_x = (V == RV_CHECK || GEN) && a.store_x;
  // image-local bases (uniform) with 32-bit offsets below
  const float2* __restrict__ d_in = a.d_in + mt.px;
  float2* __restrict__ d_out = a.d_out + mt.px;
  float* __restrict__ yt = a.yt + mt.px;
  float2* __restrict__ vst = a.v + mt.px;
  float* __restrict__ x_out = store_x ? a.x_out + mt.px : nullptr;
  float2* __restrict__ u_out = (GEN && a.u_out) ? a.u_out + mt.px : nullptr;
  float2* buf = lds;
  float2* lds_tw = lds + (RT + 1) * LS;
  const float2* tw_glob = a.tw + mt.twr;
  TwCopy<L, NT, kTwLdsRow> twc;
  const float2* tw = tw_glob;
  const float mu = a.mu[img];
  const float tau = a.lam[img] / mu;
  const float tau2 = tau * tau;
  const float alpha = a.alpha;
  float ynew[KP];
  float2 wreg[KP];
  float rd = 0.f, rv = 0.f, rz = 0.f;

  if (!GEN || a.mode == ROW_ITER || uonly) {
    float2 dd[KP];
    float yo[KP];
    // the twiddle table's reads travel with the spectra; the state loads
    // follow the inverse transform (issued before it, they slowed one 1024^2
    // image's row pass by 5% even when every wave's spectra had arrived)
    gather_rows<L, RT, true, NT>(a.spec_in + mt.sp, buf, M, r0, nr, nh, nb, C, logC, mt.rb,
                                 [&]() { twc.issue(tw_glob, tid); });
    tw = twc.commit(lds_tw, tw_glob, tid);
    __syncthreads();
    fft_lines<L, true, NT, RT + 1, kEarlyTwRow, LS>(buf, nr + 1, tw);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int l = PM::row(k, tid), j = PM::col(k, tid);
      if (l <= nr) {
        const unsigned pix = (unsigned)(wrapi(r0 - 1 + l, M) * L + j);
        dd[k] = ld_in<kNtLdRowState>(d_in + pix);
        if (l >= 1) yo[k] = ld_in<kNtLdRowState>(yt + pix);
      }
    }

    // epilogue: z-step, TV prox, dual update for tile rows 0..nr
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int l = PM::row(k, tid), j = PM::col(k, tid);
      if (l <= nr) {
        const int i = wrapi(r0 - 1 + l, M);
        const unsigned pix = (unsigned)(i * L + j);
        const int lj = lpad(j), ljr = lpad(j + 1 == L ? 0 : j + 1);
        const float x = row_x<LS>(buf, l, nr, lj);
        const float xr = row_x<LS>(buf, l, nr, ljr);
        const float xd = row_x<LS>(buf, l + 1, nr, lj);
        const float uh = xr - x + dd[k].x, uv = xd - x + dd[k].y;
        const float sc = vsoft_scale(uh * uh + uv * uv, tau, tau2);
        const float vh = sc * uh, vv = sc * uv;
        const float dh = uh - vh, dv = uv - vv;
        wreg[k] = make_float2(vh - dh, vv - dv);
        if (l >= 1) {
          st_out<kNtRowState>(d_out + pix, uonly ? make_float2(uh, uv) : make_float2(dh, dv));
          if (check && !uonly) {
            rd += (dh - dd[k].x) * (dh - dd[k].x) + (dv - dd[k].y) * (dv - dd[k].y);
            const float2 vo = vst[pix];
            rv += (vh - vo.x) * (vh - vo.x) + (vv - vo.y) * (vv - vo.y);
          }
          if (store_v && !uonly) vst[pix] = make_float2(vh, vv);
          float yn = yo[k];
          const RowObs ro = row_observed(mt, i);
          if (!pixel_observed(mt, ro, ro.explicit_mask ? a.mask + mt.px + i * L : nullptr, j)) {
            const float hx = buf[(l - 1) * LS + lj].y;
            yn = yo[k] + alpha * (hx - yo[k]);
            st_out<kNtRowState>(yt + pix, yn);
            if (check) rz += (yn - yo[k]) * (yn - yo[k]);
          }
          ynew[k] = yn;
          if (store_x) x_out[pix] = x;
          if (u_out) u_out[pix] = make_float2(uh, uv);
        }
      }
    }
  } else {
    // ROW_STATE: start from a stored state (v, d, ytilde); d is rescaled by
    // dscale (penalty update of eq. (varying_penalty))
    twc.issue(tw_glob, tid);
    tw = twc.commit(lds_tw, tw_glob, tid);
    const float ds = a.dscale ? a.dscale[img] : 1.f;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int l = PM::row(k, tid), j = PM::col(k, tid);
      if (l <= nr) {
        const unsigned pix = (unsigned)(wrapi(r0 - 1 + l, M) * L + j);
        const float2 vv = vst[pix], d0 = d_in[pix];
        const float2 dd = make_float2(ds * d0.x, ds * d0.y);
        wreg[k] = make_float2(vv.x - dd.x, vv.y - dd.y);
        if (l >= 1) {
          ynew[k] = yt[pix];
          d_out[pix] = dd;
        }
      }
    }
  }

  if (check) {
    __shared__ double red[3 * (NT / 64)];
    double rdd = rd, rvd = rv, rzd = rz;
    block_sum3(rdd, rvd, rzd, red);
    if (threadIdx.x == 0) {
      double* out = a.partials + 3 * (mt.rt0 + r0 / RT);
      out[0] = rdd; out[1] = rvd; out[2] = rzd;
    }
  }
  if (GEN && (a.last || uonly)) return;
  // prologue of the next x-step: pack ytilde + i mu D^T(v - d)
  row_prologue<L, RT, KP, NT>(buf, wreg, nr, tw, a.spec_out + mt.sp, M, r0, nh, nb, C, logC,
                          [&](int k, int, int, float g) { return make_float2(ynew[k], mu * g); }, a.nt_spec != 0);
}

template <int L, int V, int RT = rt_for(L), int NT = kNTR>
__device__ __forceinline__ void row_tile(const RowArgs& a, int img, int r0, float2* lds) {
  const ImgMeta mt = a.meta[img];
  if constexpr (V == RV_GENERIC) {
    if (a.mode == ROW_INNER) {
      row_inner<L, RT>(a, mt, r0, lds);
      return;
    }
  }
#if DCV_FULL_TILES
  if (r0 + RT <= mt.m) {
    row_tile_rows<L, V, RT>(a, mt, img, r0, RT, lds);
    return;
  }
#endif
  row_tile_rows<L, V, RT, NT>(a, mt, img, r0, min(RT, mt.m - r0), lds);
}

// Tile tables are built on the host in dispatch order (XCD-interleaved, see
// deconv.hip); entries with image -1 are padding.
// minimum waves per SIMD the row kernels are compiled for: 6 = three
// workgroups of 512 threads per compute unit (at most 80 registers); the
// 1024-thread kernels: 4 = one workgroup per compute unit, 128 registers
#ifndef DCV_ROW_WAVES
#define DCV_ROW_WAVES 6
#endif
#ifndef DCV_ROW_WAVES_WIDE
#define DCV_ROW_WAVES_WIDE 4
#endif
// NT = kNTR, or kNTRWide for plans with few row tiles (half-height tiles on
// one image: a shorter dependent chain per tile; plain and before-check
// iterations only)
template <int L, int V, int RT = rt_for(L), int NT = kNTR>
__global__ void __launch_bounds__(NT, NT == kNTR ? DCV_ROW_WAVES : DCV_ROW_WAVES_WIDE) row_kernel(RowArgs a) {
  static_assert(NT == kNTR || V != RV_GENERIC, "the generic variant runs kNTR threads");
  extern __shared__ float2 lds[];
  const int4 t = a.tiles[blockIdx.x];
  if (t.x < 0 || (a.done && a.done[t.x]) || (a.npass && a.pass_q >= a.npass[t.x])) return;
  row_tile<L, V, RT, NT>(a, t.x, t.y, lds);
}

// one launch for tiles of every line length: dispatch on the tile's length
template <int V, int L0, int... Ls>
__device__ __forceinline__ void row_dispatch(const RowArgs& a, int L, int img, int r0, float2* lds) {
  if (L == L0) {
    row_tile<L0, V>(a, img, r0, lds);
    return;
  }
  if constexpr (sizeof...(Ls) > 0) row_dispatch<V, Ls...>(a, L, img, r0, lds);
}

// The multi-length kernels hold the code of every length they dispatch to;
// left alone the register allocator sizes them for the union, which can
// cost a workgroup per compute unit.  They are held to the occupancy of the
// single-length kernels instead.
#ifndef DCV_MULTI_ROW_WAVES
#define DCV_MULTI_ROW_WAVES 4
#endif
#ifndef DCV_MULTI_COL_WAVES
#define DCV_MULTI_COL_WAVES 4
#endif
template <int V, int... Ls>
__global__ void __launch_bounds__(kNTR, DCV_MULTI_ROW_WAVES) row_kernel_multi(RowArgs a) {
  extern __shared__ float2 lds[];
  const int4 t = a.tiles[blockIdx.x];
  if (t.x < 0 || (a.done && a.done[t.x]) || (a.npass && a.pass_q >= a.npass[t.x])) return;
  row_dispatch<V, Ls...>(a, a.meta[t.x].n, t.x, t.y, lds);
}

// ---------------------------------------------------------------------------
// column pass
// ---------------------------------------------------------------------------
// Registers of one column tile between its loads and its use: the (Y, mu G)
// column spectra, the blur spectrum and the |D|^2 sums of its frequencies.
template <int L, int NT = kNTC>
struct ColLoad {
  static constexpr int C = c_for(L);
  static constexpr int NQ = (L * C + NT - 1) / NT;
  float4 g[NQ];
  float2 Hk[NQ];   // blur spectrum, or U(ky) for a separable blur
  float dv[NQ];    // |D_v|^2(ky)
  // a thread's column c = tid mod C is the same for all its entries (NT is
  // a multiple of C): one V(kx) and one |D_h|^2(kx) per thread
  float2 Hv;       // V(kx) for a separable blur
  float dh;
  static_assert(NT % C == 0, "a thread keeps one column of its tile");
};

// issue every load of tile (img, blk).  A separable blur (sep) takes its
// spectrum as the product of the two 1-D spectra, U(ky) V(kx): per image m'
// + nb C values that stay in the caches, instead of one stored value per
// frequency.
template <int L, int NT>
__device__ __forceinline__ void col_load(const ColArgs& a, const ImgMeta& mt, int blk, bool sep,
                                         ColLoad<L, NT>& r) {
  constexpr int C = c_for(L);
  constexpr int NQ = ColLoad<L, NT>::NQ;
  const long long base = mt.sp + (long long)blk * L * C;
  const float4* __restrict__ sin = a.spec_in + base;
  const float2* __restrict__ hh = a.hh + mt.hh + (long long)blk * L * C;
  const float2* __restrict__ hu = a.hsep + mt.tab;
  const float2* __restrict__ hv = hu + L;
  const float* __restrict__ dv2 = a.tab + mt.tab;
  const float* __restrict__ dh2 = dv2 + L;
  // (products and sums of these values are formed where they are used,
  // after the forward transform: formed here they would wait on every load
  // in flight)
  const int kx = blk * C + (int)(threadIdx.x % C);
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = threadIdx.x + k * NT;
    if (q < L * C) {
      const int ky = q / C;
      r.g[k] = ld_in<kNtLdCol>(sin + q);
      if (sep) r.Hk[k] = hu[ky];
      else r.Hk[k] = ld_in<kNtLdCol>(hh + q);
      r.dv[k] = dv2[ky];
    }
  }
  if (sep) r.Hv = hv[kx];
  r.dh = dh2[kx];
}

// the column spectra into the LDS lines (Y in line 2c, mu G in line 2c+1)
template <int L, int NT>
__device__ __forceinline__ void col_fill(const ColLoad<L, NT>& r, float2* buf) {
  constexpr int C = c_for(L);
  constexpr int LS = lstride(L);
#pragma unroll
  for (int k = 0; k < ColLoad<L, NT>::NQ; ++k) {
    const int q = threadIdx.x + k * NT;
    if (q < L * C) {
      const int i = q / C, c = q - i * C;
      buf[(2 * c) * LS + lpad(i)] = make_float2(r.g[k].x, r.g[k].y);
      buf[(2 * c + 1) * LS + lpad(i)] = make_float2(r.g[k].z, r.g[k].w);
    }
  }
}

// forward column DFTs, x-step solve, Q = H X, inverse DFTs, store (X, Q);
// the caller has filled the lines (not yet synchronised)
template <int L, int NT>
__device__ __forceinline__ void col_solve_store(const ColArgs& a, const ImgMeta& mt, int blk, float muv,
                                                const float2* Hk, float2 Hv, bool sep, const float* dv, float dh,
                                                float2* buf, const float2* tw) {
  constexpr int C = c_for(L);
  constexpr int LS = lstride(L);
  constexpr int NQ = ColLoad<L, NT>::NQ;
  const long long base = mt.sp + (long long)blk * L * C;
  __syncthreads();
  fft_lines<L, false, NT, 2 * C, kEarlyTwCol>(buf, 2 * C, tw);
  const float scale = 1.0f / ((float)L * (float)mt.n);
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = threadIdx.x + k * NT;
    if (q < L * C) {
      const int ky = q / C, c = q - ky * C;
      const int kx = blk * C + c;
      const float2 Y = buf[(2 * c) * LS + lpad(ky)];
      const float2 G = buf[(2 * c + 1) * LS + lpad(ky)];
      float2 X = make_float2(0.f, 0.f), Q = X;
      if (kx < mt.nh) {
        const float2 H = sep ? cmul(Hk[k], Hv) : Hk[k];
        const float h2 = H.x * H.x + H.y * H.y;
        // x-step: (conj(H) Y + G) / (|H|^2 + mu |D|^2); warm start (eq. (ini_x)):
        // conj(H) Y / (|H|^2 + tau)
        const float2 Gk = a.warm ? make_float2(0.f, 0.f) : G;
        const float den = a.warm ? h2 + a.warm_tau : h2 + muv * (dh + dv[k]);
        const float inv = scale * frcp(den);
        X = make_float2((H.x * Y.x + H.y * Y.y + Gk.x) * inv, (H.x * Y.y - H.y * Y.x + Gk.y) * inv);
        Q = cmul(H, X);
        if (a.spec_store) a.spec_store[base + q] = make_float4(Y.x, Y.y, X.x, X.y);
      }
      buf[(2 * c) * LS + lpad(ky)] = X;
      buf[(2 * c + 1) * LS + lpad(ky)] = Q;
    }
  }
  __syncthreads();
  fft_lines<L, true, NT, 2 * C, kEarlyTwCol>(buf, 2 * C, tw);
  // output in the row-block layout the row pass reads (runs of rt rows)
  float4* __restrict__ sout = a.spec_out + mt.sp + (unsigned)(blk * C * mt.rb);
  const unsigned nbc = (unsigned)(mt.nb * C);
  const bool nt = a.nt_spec != 0;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = threadIdx.x + k * NT;
    if (q < L * C) {
      const int i = q / C, c = q - i * C;
      const float2 X = buf[(2 * c) * LS + lpad(i)];
      const float2 Q = buf[(2 * c + 1) * LS + lpad(i)];
      st_spec<kNtColSpec>(sout + (row_block_index(mt, i, nbc) + c * mt.rb), make_float4(X.x, X.y, Q.x, Q.y),
                          nt);
    }
  }
}

// NT threads per tile: kNTC, or kNTCWide for plans with few tiles (a shorter
// dependent chain per tile when a compute unit has no other tile to overlap)
template <int L, int NT = kNTC>
__device__ __forceinline__ void col_tile(const ColArgs& a, int img, int blk, float2* lds) {
  constexpr int C = c_for(L);
  const ImgMeta mt = a.meta[img];
  float2* buf = lds;
  const float2* tw = twiddle_table<L, NT, kTwLdsCol>(lds + 2 * C * lstride(L), a.tw + mt.twc);
  ColLoad<L, NT> r;
  const bool sep = a.sep != nullptr && a.sep[img] != 0;
  col_load<L, NT>(a, mt, blk, sep, r);
  col_fill<L, NT>(r, buf);
  col_solve_store<L, NT>(a, mt, blk, a.mu[img], r.Hk, r.Hv, sep, r.dv, r.dh, buf, tw);
}

template <int L, int NT = kNTC>
__global__ void __launch_bounds__(NT) col_kernel(ColArgs a) {
  extern __shared__ float2 lds[];
  const int4 t = a.tiles[blockIdx.x];
  if (t.x < 0 || (a.done && a.done[t.x]) || (a.npass && a.pass_q >= a.npass[t.x])) return;
  col_tile<L, NT>(a, t.x, t.y, lds);
}

template <int L0, int... Ls>
__device__ __forceinline__ void col_dispatch(const ColArgs& a, int L, int img, int blk, float2* lds) {
  if (L == L0) {
    col_tile<L0>(a, img, blk, lds);
    return;
  }
  if constexpr (sizeof...(Ls) > 0) col_dispatch<Ls...>(a, L, img, blk, lds);
}

template <int... Ls>
__global__ void __launch_bounds__(kNTC, DCV_MULTI_COL_WAVES) col_kernel_multi(ColArgs a) {
  extern __shared__ float2 lds[];
  const int4 t = a.tiles[blockIdx.x];
  if (t.x < 0 || (a.done && a.done[t.x]) || (a.npass && a.pass_q >= a.npass[t.x])) return;
  col_dispatch<Ls...>(a, a.meta[t.x].m, t.x, t.y, lds);
}

}  // namespace dcv
