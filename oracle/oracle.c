/*
 * FP64 CPU oracle for the partial ADMM of Simoes, Almeida, Bioucas-Dias and
 * Chanussot, "A Framework for Fast Image Deconvolution with Incomplete
 * Observations" (arXiv 1602.01410).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * Everything is double precision and written for readability, not speed: the
 * DFT is this file's own iterative radix-2 FFT, with Bluestein's chirp-z
 * reduction (through the same radix-2 FFT) for lengths that are not powers of
 * two, and a direct O(n^2) DFT kept for cross-checks.  OpenMP only splits
 * independent rows / columns over threads; it never changes the arithmetic.
 *
 * Conventions (all images row-major, M rows by N columns, M = m', N = n'):
 *   forward DFT   X[k] = sum_j x[j] exp(-2 pi i jk / n), unnormalised;
 *   inverse DFT   x[j] = (1/n) sum_k X[k] exp(+2 pi i jk / n).
 *   Blur (Sec. I-A, model (4)): (Hx)[i,j] = sum_{p,q=-b..b} h[b+p][b+q]
 *   x[i-p, j-q], indices modulo (M, N); h is (2b+1)^2, centred at (b, b).
 *   Differences (Sec. III-B, isotropic TV): periodic forward differences
 *   (D_h x)[i,j] = x[i,j+1]-x[i,j], (D_v x)[i,j] = x[i+1,j]-x[i,j].
 *   Mask: 1 = observed, over the whole extended grid.  For unknown
 *   boundaries (Sec. I-A) the caller's mask is 0 on the band of width b
 *   around the central m x n region; the oracle takes the mask as given so
 *   that the fully observed special cases can be exercised too.
 *
 * Parity pins (tests/test_oracle_pins.py, tests/test_oracle_color.py): each
 * exported function is checked against something other than itself.
 *   or_fft1, or_fft2, or_dft2_direct  numpy.fft, each other, Parseval
 *   or_psf_spectrum       the kappa(H) values printed in Table I and the
 *                         appendix tables (256^2 domain, sigma = sqrt(l))
 *   or_conv_direct, or_conv_fft  scipy.signal.convolve2d on the valid part,
 *                         each other, the adjoint identity
 *   or_grad, or_gradT     numpy.roll differences, the adjoint identity, the
 *                         4 sin^2 spectrum of the stencil
 *   or_init_state         numpy.pad(mode='edge') of the central region (holes
 *                         at numpy's mean of the observed pixels), numpy.roll
 *                         differences for v^0
 *   or_admm_iterate       closed forms (lambda = 0; quadratic phi: Tikhonov
 *                         and dense normal equations), a dense standard ADMM,
 *                         Lemmas 2 and 3, the x-step normal equations; passes:
 *                         the dense joint (x, z) minimiser; penalty update:
 *                         the decisions of eq. (varying_penalty) on built
 *                         states and the invariance of mu d
 *   or_admm_iterate_vec   reduces to or_admm_iterate (C = 1, lambda = 0,
 *                         equal channels)
 *   or_warm_start         the dense minimiser of f + tau/2 |x|^2
 *   or_objective          decreases to the dense minimum
 *   or_admm_backward      central finite differences of or_admm_iterate
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* 1-D FFT: radix-2 (powers of two) and Bluestein (everything else).         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;          /* transform length */
    int pow2;       /* 1 if n is a power of two */
    cplx* tw;       /* radix-2: exp(-2 pi i k/n), k < n/2 */
    /* Bluestein data */
    int m;          /* power-of-two convolution length >= 2n-1 */
    cplx* chirp;    /* exp(-i pi k^2 / n), k < n */
    cplx* bhat;     /* forward FFT (length m) of conj(chirp), wrapped */
    void* sub;      /* radix-2 plan of length m */
} offt;

static int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

static offt* offt_new(int n);

static void fft_radix2(const offt* p, cplx* a, int sign)
{
    /* iterative decimation-in-time: bit-reversal permutation, then stages */
    int n = p->n;
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int step = n / len;
        for (int s = 0; s < n; s += len) {
            for (int k = 0; k < len / 2; ++k) {
                cplx w = p->tw[k * step];
                if (sign > 0) w = conj(w);
                cplx u = a[s + k], v = a[s + k + len / 2] * w;
                a[s + k] = u + v;
                a[s + k + len / 2] = u - v;
            }
        }
    }
}

/* Unnormalised DFT with exponent sign `sign` (-1 forward, +1 inverse). */
static void offt_exec(const offt* p, cplx* a, int sign, cplx* scratch /* >= m */)
{
    if (p->n == 1) return;
    if (p->pow2) { fft_radix2(p, a, sign); return; }
    /* Bluestein: jk = (j^2 + k^2 - (k-j)^2)/2 turns the DFT into a
       convolution with the chirp, done with length-m radix-2 FFTs. */
    const offt* q = (const offt*)p->sub;
    int n = p->n, m = p->m;
    for (int j = 0; j < m; ++j) scratch[j] = 0;
    for (int j = 0; j < n; ++j) {
        cplx c = sign < 0 ? p->chirp[j] : conj(p->chirp[j]);
        scratch[j] = a[j] * c;
    }
    fft_radix2(q, scratch, -1);
    for (int j = 0; j < m; ++j) {
        cplx b = p->bhat[j];
        /* bhat holds the transform for sign -1; for sign +1 the kernel is
           conj(conj(chirp)) = chirp, whose transform is conj(bhat[-j]) */
        if (sign > 0) b = conj(p->bhat[(m - j) % m]);
        scratch[j] *= b;
    }
    fft_radix2(q, scratch, +1);
    for (int k = 0; k < n; ++k) {
        cplx c = sign < 0 ? p->chirp[k] : conj(p->chirp[k]);
        a[k] = c * scratch[k] / (double)m;
    }
}

static offt* offt_new(int n)
{
    offt* p = (offt*)calloc(1, sizeof(offt));
    p->n = n;
    p->pow2 = is_pow2(n);
    if (p->pow2) {
        int h = n / 2 > 0 ? n / 2 : 1;
        p->tw = (cplx*)malloc(sizeof(cplx) * h);
        for (int k = 0; k < h; ++k) {
            double a = -2.0 * M_PI * (double)k / (double)n;
            p->tw[k] = cos(a) + I * sin(a);
        }
        return p;
    }
    int m = 1;
    while (m < 2 * n - 1) m <<= 1;
    p->m = m;
    p->sub = offt_new(m);
    p->chirp = (cplx*)malloc(sizeof(cplx) * n);
    for (int k = 0; k < n; ++k) {
        /* k^2 mod 2n keeps the angle small and exact */
        long long kk = ((long long)k * k) % (2LL * n);
        double a = -M_PI * (double)kk / (double)n;
        p->chirp[k] = cos(a) + I * sin(a);
    }
    p->bhat = (cplx*)calloc(m, sizeof(cplx));
    p->bhat[0] = conj(p->chirp[0]);
    for (int k = 1; k < n; ++k) {
        p->bhat[k] = conj(p->chirp[k]);
        p->bhat[m - k] = conj(p->chirp[k]);
    }
    fft_radix2((const offt*)p->sub, p->bhat, -1);
    return p;
}

static void offt_free(offt* p)
{
    if (!p) return;
    free(p->tw);
    free(p->chirp);
    free(p->bhat);
    offt_free((offt*)p->sub);
    free(p);
}

static int offt_scratch_len(const offt* p) { return p->pow2 ? 1 : p->m; }

/* 2-D unnormalised DFT of an M x N complex array, in place.  Rows first,
   then columns; the 2-D DFT is separable so the order is immaterial. */
static void dft2(int M, int N, cplx* a, int sign)
{
    offt* pr = offt_new(N);
    offt* pc = (M == N) ? pr : offt_new(M);
    int sr = offt_scratch_len(pr), sc = offt_scratch_len(pc);
#pragma omp parallel
    {
        cplx* scr = (cplx*)malloc(sizeof(cplx) * (sr > sc ? sr : sc));
        cplx* col = (cplx*)malloc(sizeof(cplx) * M);
#pragma omp for schedule(static)
        for (int i = 0; i < M; ++i) offt_exec(pr, a + (size_t)i * N, sign, scr);
#pragma omp for schedule(static)
        for (int j = 0; j < N; ++j) {
            for (int i = 0; i < M; ++i) col[i] = a[(size_t)i * N + j];
            offt_exec(pc, col, sign, scr);
            for (int i = 0; i < M; ++i) a[(size_t)i * N + j] = col[i];
        }
        free(col);
        free(scr);
    }
    if (pc != pr) offt_free(pc);
    offt_free(pr);
}

/* ------------------------------------------------------------------------ */
/* Exported transforms (used by the tests to pin the FFT itself).           */
/* ------------------------------------------------------------------------ */

/* 1-D DFT of n complex values (re/im split), sign -1 forward, +1 inverse
   (unnormalised). */
void or_fft1(int n, double* re, double* im, int sign)
{
    offt* p = offt_new(n);
    cplx* a = (cplx*)malloc(sizeof(cplx) * n);
    cplx* s = (cplx*)malloc(sizeof(cplx) * offt_scratch_len(p));
    for (int j = 0; j < n; ++j) a[j] = re[j] + I * im[j];
    offt_exec(p, a, sign, s);
    for (int j = 0; j < n; ++j) { re[j] = creal(a[j]); im[j] = cimag(a[j]); }
    free(s); free(a); offt_free(p);
}

/* 2-D DFT of an M x N complex array (re/im split), unnormalised. */
void or_fft2(int M, int N, double* re, double* im, int sign)
{
    size_t n = (size_t)M * N;
    cplx* a = (cplx*)malloc(sizeof(cplx) * n);
    for (size_t j = 0; j < n; ++j) a[j] = re[j] + I * im[j];
    dft2(M, N, a, sign);
    for (size_t j = 0; j < n; ++j) { re[j] = creal(a[j]); im[j] = cimag(a[j]); }
    free(a);
}

/* Direct O((MN)^2)-free separable DFT: the textbook double sum, evaluated
   per output frequency with exact angle reduction.  For cross-checks on
   small sizes only. */
void or_dft2_direct(int M, int N, const double* re, const double* im,
                    double* ore, double* oim, int sign)
{
    for (int ky = 0; ky < M; ++ky)
        for (int kx = 0; kx < N; ++kx) {
            cplx s = 0;
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < N; ++j) {
                    /* angle = sign 2 pi (ky i / M + kx j / N), reduced exactly */
                    long long a = ((long long)ky * i) % M;
                    long long b = ((long long)kx * j) % N;
                    double ang = sign * 2.0 * M_PI *
                                 ((double)a / (double)M + (double)b / (double)N);
                    s += (re[(size_t)i * N + j] + I * im[(size_t)i * N + j]) *
                         (cos(ang) + I * sin(ang));
                }
            ore[(size_t)ky * N + kx] = creal(s);
            oim[(size_t)ky * N + kx] = cimag(s);
        }
}

/* ------------------------------------------------------------------------ */
/* Operators of the observation model and of the regulariser.               */
/* ------------------------------------------------------------------------ */

/* Spectrum of the BCCB blur (Sec. II-B: products by T~ via the FFT): embed the
   (2b+1)^2 kernel circularly centred at the origin, take its 2-D DFT. */
static void psf_spectrum(int M, int N, int K, const double* h, cplx* Hs)
{
    int b = K / 2;
    size_t n = (size_t)M * N;
    for (size_t j = 0; j < n; ++j) Hs[j] = 0;
    for (int p = -b; p <= b; ++p)
        for (int q = -b; q <= b; ++q) {
            int i = ((p % M) + M) % M, j = ((q % N) + N) % N;
            Hs[(size_t)i * N + j] += h[(size_t)(b + p) * K + (b + q)];
        }
    dft2(M, N, Hs, -1);
}

void or_psf_spectrum(int M, int N, int K, const double* h, double* re, double* im)
{
    size_t n = (size_t)M * N;
    cplx* Hs = (cplx*)malloc(sizeof(cplx) * n);
    psf_spectrum(M, N, K, h, Hs);
    for (size_t j = 0; j < n; ++j) { re[j] = creal(Hs[j]); im[j] = cimag(Hs[j]); }
    free(Hs);
}

/* Periodic convolution written as the defining double sum (model (4)). */
void or_conv_direct(int M, int N, int K, const double* h, const double* x, double* out)
{
    int b = K / 2;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            double s = 0;
            for (int p = -b; p <= b; ++p)
                for (int q = -b; q <= b; ++q) {
                    int ii = (((i - p) % M) + M) % M, jj = (((j - q) % N) + N) % N;
                    s += h[(size_t)(b + p) * K + (b + q)] * x[(size_t)ii * N + jj];
                }
            out[(size_t)i * N + j] = s;
        }
}

/* y = H x through the FFT (the route the method takes). */
static void apply_H(int M, int N, const cplx* Hs, const double* x, double* out, int adjoint)
{
    size_t n = (size_t)M * N;
    cplx* a = (cplx*)malloc(sizeof(cplx) * n);
    for (size_t j = 0; j < n; ++j) a[j] = x[j];
    dft2(M, N, a, -1);
    for (size_t j = 0; j < n; ++j) a[j] *= adjoint ? conj(Hs[j]) : Hs[j];
    dft2(M, N, a, +1);
    for (size_t j = 0; j < n; ++j) out[j] = creal(a[j]) / (double)n;
    free(a);
}

void or_conv_fft(int M, int N, int K, const double* h, const double* x, double* out, int adjoint)
{
    size_t n = (size_t)M * N;
    cplx* Hs = (cplx*)malloc(sizeof(cplx) * n);
    psf_spectrum(M, N, K, h, Hs);
    apply_H(M, N, Hs, x, out, adjoint);
    free(Hs);
}

/* D = [D_h; D_v]: periodic forward differences. */
void or_grad(int M, int N, const double* x, double* gh, double* gv)
{
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            double c = x[(size_t)i * N + j];
            gh[(size_t)i * N + j] = x[(size_t)i * N + (j + 1) % N] - c;
            gv[(size_t)i * N + j] = x[(size_t)((i + 1) % M) * N + j] - c;
        }
}

/* D^T [w_h; w_v] (the adjoint of or_grad). */
void or_gradT(int M, int N, const double* wh, const double* wv, double* out)
{
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            size_t c = (size_t)i * N + j;
            out[c] = wh[(size_t)i * N + (j + N - 1) % N] - wh[c] +
                     wv[(size_t)((i + M - 1) % M) * N + j] - wv[c];
        }
}

static int in_valid(int M, int N, int b, int i, int j)
{
    return i >= b && i < M - b && j >= b && j < N - b;
}

static int observed(int M, int N, int b, const uint8_t* mask, int i, int j)
{
    (void)M; (void)b;
    return mask[(size_t)i * N + j] != 0;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* Initial state (Sec. III-B: the observed image padded by repeating its    */
/* border pixels, used for x^0 and z^0).                                    */
/* ------------------------------------------------------------------------ */

/* ytilde^0: observed pixels keep y; unobserved pixels inside the central
   region take the mean of the observed pixels; unobserved pixels of the band
   of width b copy the nearest pixel of the central region (edge
   replication).
   v^0 = D x^0 with x^0 = ytilde^0, d^0 = 0. */
void or_init_state(int M, int N, int K, const double* y, const uint8_t* mask,
                   double* yt, double* vh, double* vv, double* dh, double* dv)
{
    int b = K / 2;
    double s = 0;
    long long cnt = 0;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j)
            if (observed(M, N, b, mask, i, j)) { s += y[(size_t)i * N + j]; ++cnt; }
    double mean = cnt ? s / (double)cnt : 0.0;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j)
            if (in_valid(M, N, b, i, j))
                yt[(size_t)i * N + j] = observed(M, N, b, mask, i, j) ? y[(size_t)i * N + j] : mean;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j)
            if (!in_valid(M, N, b, i, j)) {
                int si = clampi(i, b, M - b - 1), sj = clampi(j, b, N - b - 1);
                yt[(size_t)i * N + j] = observed(M, N, b, mask, i, j) ? y[(size_t)i * N + j]
                                                                       : yt[(size_t)si * N + sj];
            }
    or_grad(M, N, yt, vh, vv);
    size_t n = (size_t)M * N;
    for (size_t j = 0; j < n; ++j) { dh[j] = 0; dv[j] = 0; }
}

/* ------------------------------------------------------------------------ */
/* Partial ADMM, eqs. (admm_aprox_1)-(admm_aprox_4), closed forms of        */
/* Sec. II-B (x-step (dual_x_iter_resolved_boundaries), z-step with         */
/* over-relaxation), isotropic-TV prox of Sec. III-B.                       */
/* ------------------------------------------------------------------------ */

enum { OR_PHI_TV = 0, OR_PHI_QUAD = 1 };

/* Proximal step (admm_aprox_3) at one pixel: v = argmin phi(v) +
   mu/2 |v - u|^2 with u = D x^{i+1} + d^i.
   TV: vector soft threshold with tau = lambda/mu (|u| <= tau gives 0).
   Quadratic phi = lambda/2 |v|^2: v = mu u / (lambda + mu). */
static void prox(int phi, double lam, double mu, double uh, double uv, double* vh, double* vv)
{
    if (phi == OR_PHI_QUAD) {
        double s = mu / (lam + mu);
        *vh = s * uh; *vv = s * uv;
        return;
    }
    double tau = lam / mu;
    double nrm = sqrt(uh * uh + uv * uv);
    double s = nrm > tau ? (nrm - tau) / nrm : 0.0;
    *vh = s * uh; *vv = s * uv;
}

typedef struct {
    int M, N, K;
    const uint8_t* mask;
    cplx* Hs;       /* blur spectrum */
    double* den;    /* |H|^2 + mu |D|^2 */
    double mu;
} ctx_t;

/* |D_h^|^2 + |D_v^|^2 for forward periodic differences. */
static double dsq(int M, int N, int ky, int kx)
{
    double sx = sin(M_PI * (double)kx / (double)N), sy = sin(M_PI * (double)ky / (double)M);
    return 4.0 * sx * sx + 4.0 * sy * sy;
}

/* One x-step (admm_aprox_1) followed by one z-step (admm_aprox_2 with
   relaxation alpha).  G holds DFT(D^T (v - d)).  On return x holds x^{i+1}
   and yt the updated extended image; ytold receives the image before the
   z-step. */
static void bgs_pass(const ctx_t* c, const cplx* G, double alpha, double* yt, double* x,
                     double* q, cplx* Y, cplx* X, double* max_imag)
{
    int M = c->M, N = c->N, b = c->K / 2;
    size_t n = (size_t)M * N;
    for (size_t j = 0; j < n; ++j) Y[j] = yt[j];
    dft2(M, N, Y, -1);
    for (size_t j = 0; j < n; ++j)
        X[j] = (conj(c->Hs[j]) * Y[j] + c->mu * G[j]) / c->den[j];
    /* x = IDFT(X); Hx = IDFT(H X) */
    for (size_t j = 0; j < n; ++j) Y[j] = c->Hs[j] * X[j];
    dft2(M, N, X, +1);
    dft2(M, N, Y, +1);
    double mi = 0;
    for (size_t j = 0; j < n; ++j) {
        x[j] = creal(X[j]) / (double)n;
        q[j] = creal(Y[j]) / (double)n;
        double a = fabs(cimag(X[j])) / (double)n, bq = fabs(cimag(Y[j])) / (double)n;
        if (a > mi) mi = a;
        if (bq > mi) mi = bq;
    }
    if (max_imag && mi > *max_imag) *max_imag = mi;
    /* z^{i+1} = z^i + alpha (M_z H x^{i+1} - z^i) on the unobserved pixels */
    for (int i = 0; i < M; ++i)
        for (int jj = 0; jj < N; ++jj) {
            size_t k = (size_t)i * N + jj;
            if (!observed(M, N, b, c->mask, i, jj)) yt[k] = yt[k] + alpha * (q[k] - yt[k]);
        }
}

/*
 * Run `iters` partial-ADMM iterations from the state (yt, vh, vv, dh, dv),
 * which is updated in place.  On return x holds x^{iters} (the output of the
 * last x-step).  hist (nullable) receives per iteration
 *   [ |d'-d|, |v'-v|, |z'-z|, |w'-w|_G^2, mu ]
 * where w = [z; v_x; d_x] and G = diag(I, mu I, mu I) (Appendix B).
 * passes = number of block-Gauss-Seidel passes per iteration.
 * adapt_t > 0 enables the penalty update (varying_penalty) with threshold t;
 * mu_io then holds the final mu.
 * Returns the largest imaginary residue seen after an inverse DFT.
 */
double or_admm_iterate(int M, int N, int K, const double* h, const uint8_t* mask,
                       double lam, double* mu_io, double alpha, int passes, int phi,
                       int iters, double adapt_t,
                       double* yt, double* vh, double* vv, double* dh, double* dv,
                       double* x, double* hist)
{
    size_t n = (size_t)M * N;
    int b = K / 2;
    double mu = *mu_io;
    ctx_t c = {M, N, K, mask, NULL, NULL, mu};
    c.Hs = (cplx*)malloc(sizeof(cplx) * n);
    c.den = (double*)malloc(sizeof(double) * n);
    psf_spectrum(M, N, K, h, c.Hs);
    cplx* G = (cplx*)malloc(sizeof(cplx) * n);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * n);
    cplx* X = (cplx*)malloc(sizeof(cplx) * n);
    double* g = (double*)malloc(sizeof(double) * n);
    double* wh = (double*)malloc(sizeof(double) * n);
    double* wv = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    double* zold = (double*)malloc(sizeof(double) * n);
    double max_imag = 0;
    for (int it = 0; it < iters; ++it) {
        c.mu = mu;
        for (int ky = 0; ky < M; ++ky)
            for (int kx = 0; kx < N; ++kx) {
                size_t k = (size_t)ky * N + kx;
                double h2 = creal(c.Hs[k]) * creal(c.Hs[k]) + cimag(c.Hs[k]) * cimag(c.Hs[k]);
                c.den[k] = h2 + mu * dsq(M, N, ky, kx);
            }
        /* right-hand side term mu D^T (v - d) */
        for (size_t j = 0; j < n; ++j) { wh[j] = vh[j] - dh[j]; wv[j] = vv[j] - dv[j]; }
        or_gradT(M, N, wh, wv, g);
        for (size_t j = 0; j < n; ++j) G[j] = g[j];
        dft2(M, N, G, -1);
        memcpy(zold, yt, sizeof(double) * n);
        for (int p = 0; p < passes; ++p) bgs_pass(&c, G, alpha, yt, x, q, Y, X, &max_imag);
        /* v, d steps (admm_aprox_3), (admm_aprox_4) */
        double rd = 0, rv = 0, rz = 0;
        for (int i = 0; i < M; ++i)
            for (int jj = 0; jj < N; ++jj) {
                size_t k = (size_t)i * N + jj;
                double xc = x[k];
                double uh = x[(size_t)i * N + (jj + 1) % N] - xc + dh[k];
                double uv = x[(size_t)((i + 1) % M) * N + jj] - xc + dv[k];
                double nvh, nvv;
                prox(phi, lam, mu, uh, uv, &nvh, &nvv);
                double ndh = uh - nvh, ndv = uv - nvv;
                rd += (ndh - dh[k]) * (ndh - dh[k]) + (ndv - dv[k]) * (ndv - dv[k]);
                rv += (nvh - vh[k]) * (nvh - vh[k]) + (nvv - vv[k]) * (nvv - vv[k]);
                if (!observed(M, N, b, mask, i, jj)) rz += (yt[k] - zold[k]) * (yt[k] - zold[k]);
                vh[k] = nvh; vv[k] = nvv; dh[k] = ndh; dv[k] = ndv;
            }
        if (hist) {
            hist[5 * it + 0] = sqrt(rd);
            hist[5 * it + 1] = sqrt(rv);
            hist[5 * it + 2] = sqrt(rz);
            hist[5 * it + 3] = rz + mu * rv + mu * rd;
            hist[5 * it + 4] = mu;
        }
        if (adapt_t > 0) {
            /* penalty update (varying_penalty) and rescaling of d */
            double nd = sqrt(rd), nv = sqrt(rv);
            if (nd > adapt_t * nv) {
                mu *= 2.0;
                for (size_t j = 0; j < n; ++j) { dh[j] *= 0.5; dv[j] *= 0.5; }
            } else if (nv > adapt_t * nd) {
                mu *= 0.5;
                for (size_t j = 0; j < n; ++j) { dh[j] *= 2.0; dv[j] *= 2.0; }
            }
        }
    }
    *mu_io = mu;
    free(zold); free(q); free(wv); free(wh); free(g); free(X); free(Y); free(G);
    free(c.den); free(c.Hs);
    return max_imag;
}

/*
 * Colour images (Sec. III-C, demosaicing): C channels x^1..x^C observed
 * through the same blur, each with its own mask, data [y^j; z^j] and x-step.
 * The data term is the sum of the per-channel terms, so the x- and z-steps
 * are those of one channel, applied to each.  The regulariser is the
 * vectorial TV, lambda times the per-pixel Euclidean norm of all 2C
 * differences, so the v-step is one vector soft threshold over the 2C
 * components of u = D x + d at each pixel.
 * Arrays hold the channels one after the other (C * M * N values); v and d
 * likewise per component (vh, vv, dh, dv each C * M * N).  Residuals and the
 * penalty update use norms over all channels.  hist as or_admm_iterate.
 * Parity: pinned by reduction to or_admm_iterate (C = 1, and lambda = 0 where
 * the channels decouple) and by the identity that C equal channels behave as
 * one channel with lambda / sqrt(C).
 */
double or_admm_iterate_vec(int M, int N, int K, int C, const double* h, const uint8_t* masks,
                           double lam, double* mu_io, double alpha, int passes, int iters,
                           double adapt_t, double* yt, double* vh, double* vv, double* dh,
                           double* dv, double* x, double* hist)
{
    size_t n = (size_t)M * N;
    double mu = *mu_io;
    ctx_t c = {M, N, K, masks, NULL, NULL, mu};
    c.Hs = (cplx*)malloc(sizeof(cplx) * n);
    c.den = (double*)malloc(sizeof(double) * n);
    psf_spectrum(M, N, K, h, c.Hs);
    cplx* G = (cplx*)malloc(sizeof(cplx) * n);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * n);
    cplx* X = (cplx*)malloc(sizeof(cplx) * n);
    double* g = (double*)malloc(sizeof(double) * n);
    double* wh = (double*)malloc(sizeof(double) * n);
    double* wv = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    double* zold = (double*)malloc(sizeof(double) * n * C);
    double max_imag = 0;
    for (int it = 0; it < iters; ++it) {
        c.mu = mu;
        for (int ky = 0; ky < M; ++ky)
            for (int kx = 0; kx < N; ++kx) {
                size_t k = (size_t)ky * N + kx;
                double h2 = creal(c.Hs[k]) * creal(c.Hs[k]) + cimag(c.Hs[k]) * cimag(c.Hs[k]);
                c.den[k] = h2 + mu * dsq(M, N, ky, kx);
            }
        memcpy(zold, yt, sizeof(double) * n * C);
        /* x- and z-steps, channel by channel */
        for (int ch = 0; ch < C; ++ch) {
            size_t o = (size_t)ch * n;
            c.mask = masks + o;
            for (size_t j = 0; j < n; ++j) { wh[j] = vh[o + j] - dh[o + j]; wv[j] = vv[o + j] - dv[o + j]; }
            or_gradT(M, N, wh, wv, g);
            for (size_t j = 0; j < n; ++j) G[j] = g[j];
            dft2(M, N, G, -1);
            for (int p = 0; p < passes; ++p) bgs_pass(&c, G, alpha, yt + o, x + o, q, Y, X, &max_imag);
        }
        /* joint v- and d-steps over the 2C components */
        double rd = 0, rv = 0, rz = 0;
        double tau = lam / mu;
        for (int i = 0; i < M; ++i)
            for (int jj = 0; jj < N; ++jj) {
                size_t k = (size_t)i * N + jj;
                size_t kr = (size_t)i * N + (jj + 1) % N, kd = (size_t)((i + 1) % M) * N + jj;
                double nrm2 = 0;
                for (int ch = 0; ch < C; ++ch) {
                    size_t o = (size_t)ch * n;
                    double uh = x[o + kr] - x[o + k] + dh[o + k];
                    double uv = x[o + kd] - x[o + k] + dv[o + k];
                    nrm2 += uh * uh + uv * uv;
                }
                double nrm = sqrt(nrm2);
                double s = nrm > tau ? (nrm - tau) / nrm : 0.0;
                for (int ch = 0; ch < C; ++ch) {
                    size_t o = (size_t)ch * n;
                    double uh = x[o + kr] - x[o + k] + dh[o + k];
                    double uv = x[o + kd] - x[o + k] + dv[o + k];
                    double nvh = s * uh, nvv = s * uv;
                    double ndh = uh - nvh, ndv = uv - nvv;
                    rd += (ndh - dh[o + k]) * (ndh - dh[o + k]) + (ndv - dv[o + k]) * (ndv - dv[o + k]);
                    rv += (nvh - vh[o + k]) * (nvh - vh[o + k]) + (nvv - vv[o + k]) * (nvv - vv[o + k]);
                    /* u reads d at this pixel only, so v and d update in place */
                    vh[o + k] = nvh; vv[o + k] = nvv;
                    dh[o + k] = ndh; dv[o + k] = ndv;
                }
            }
        for (int ch = 0; ch < C; ++ch) {
            size_t o = (size_t)ch * n;
            for (int i = 0; i < M; ++i)
                for (int jj = 0; jj < N; ++jj) {
                    size_t k = (size_t)i * N + jj;
                    if (!observed(M, N, K / 2, masks + o, i, jj))
                        rz += (yt[o + k] - zold[o + k]) * (yt[o + k] - zold[o + k]);
                }
        }
        if (hist) {
            hist[5 * it + 0] = sqrt(rd);
            hist[5 * it + 1] = sqrt(rv);
            hist[5 * it + 2] = sqrt(rz);
            hist[5 * it + 3] = rz + mu * rv + mu * rd;
            hist[5 * it + 4] = mu;
        }
        if (adapt_t > 0) {
            double nd = sqrt(rd), nv = sqrt(rv);
            if (nd > adapt_t * nv) {
                mu *= 2.0;
                for (size_t j = 0; j < n * C; ++j) { dh[j] *= 0.5; dv[j] *= 0.5; }
            } else if (nv > adapt_t * nd) {
                mu *= 0.5;
                for (size_t j = 0; j < n * C; ++j) { dh[j] *= 2.0; dv[j] *= 2.0; }
            }
        }
    }
    *mu_io = mu;
    free(zold); free(q); free(wv); free(wh); free(g); free(X); free(Y); free(G);
    free(c.den); free(c.Hs);
    return max_imag;
}

/* Quadratic warm start for z (eqs. (ini_x), (ini_z)): `iters` alternations of
   x = (H^T H + tau I)^{-1} H^T [y; z],  z = M_z H x,  from yt in place. */
void or_warm_start(int M, int N, int K, const double* h, const uint8_t* mask,
                   double tau, int iters, double* yt)
{
    size_t n = (size_t)M * N;
    int b = K / 2;
    cplx* Hs = (cplx*)malloc(sizeof(cplx) * n);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * n);
    psf_spectrum(M, N, K, h, Hs);
    for (int it = 0; it < iters; ++it) {
        for (size_t j = 0; j < n; ++j) Y[j] = yt[j];
        dft2(M, N, Y, -1);
        for (size_t j = 0; j < n; ++j) {
            double h2 = creal(Hs[j]) * creal(Hs[j]) + cimag(Hs[j]) * cimag(Hs[j]);
            /* H x with x = conj(H) Y / (|H|^2 + tau) */
            Y[j] = Hs[j] * conj(Hs[j]) * Y[j] / (h2 + tau);
        }
        dft2(M, N, Y, +1);
        for (int i = 0; i < M; ++i)
            for (int jj = 0; jj < N; ++jj) {
                size_t k = (size_t)i * N + jj;
                if (!observed(M, N, b, mask, i, jj)) yt[k] = creal(Y[k]) / (double)n;
            }
    }
    free(Y); free(Hs);
}

/* Objective f(x, z) + phi(D x) of (problem_xz) with f from (new_model). */
double or_objective(int M, int N, int K, const double* h, const double* yt, const double* x,
                    double lam, int phi)
{
    size_t n = (size_t)M * N;
    double* hx = (double*)malloc(sizeof(double) * n);
    or_conv_fft(M, N, K, h, x, hx, 0);
    double f = 0, r = 0;
    for (size_t j = 0; j < n; ++j) f += 0.5 * (yt[j] - hx[j]) * (yt[j] - hx[j]);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            double c = x[(size_t)i * N + j];
            double gh = x[(size_t)i * N + (j + 1) % N] - c;
            double gv = x[(size_t)((i + 1) % M) * N + j] - c;
            r += phi == OR_PHI_QUAD ? 0.5 * (gh * gh + gv * gv) : sqrt(gh * gh + gv * gv);
        }
    free(hx);
    return f + lam * r;
}

/* ------------------------------------------------------------------------ */
/* Reverse mode through `iters` unrolled iterations (one BGS pass, fixed mu) */
/* of the run that or_init_state + or_admm_iterate perform.  Derived by hand */
/* from the forward steps; every h-gradient term is written as the spatial   */
/* correlation that differentiating the defining sum of H gives.             */
/* ------------------------------------------------------------------------ */

/* Correlation term: out[b+p][b+q] += sum_{i,j} a[i,j] c[i-p, j-q]. */
static void corr_acc(int M, int N, int K, const double* a, const double* c, double sgn, double* out)
{
    int b = K / 2;
#pragma omp parallel for collapse(2) schedule(static)
    for (int p = -b; p <= b; ++p)
        for (int q = -b; q <= b; ++q) {
            double s = 0;
            for (int i = 0; i < M; ++i) {
                int ii = (((i - p) % M) + M) % M;
                for (int j = 0; j < N; ++j) {
                    int jj = (((j - q) % N) + N) % N;
                    s += a[(size_t)i * N + j] * c[(size_t)ii * N + jj];
                }
            }
            out[(size_t)(b + p) * K + (b + q)] += sgn * s;
        }
}

/*
 * Loss L depends on the output x^{iters}; grad_x = dL/dx^{iters}.
 * Produces dL/dy (zero at unobserved pixels), dL/dlambda and dL/dh.
 * The run starts from or_init_state (the gradient flows through the
 * initialisation as well).
 */
void or_admm_backward(int M, int N, int K, const double* h, const double* y, const uint8_t* mask,
                      double lam, double mu, double alpha, int phi, int iters,
                      const double* grad_x, double* grad_y, double* grad_lam, double* grad_h)
{
    size_t n = (size_t)M * N;
    int b = K / 2;
    /* forward, keeping every state */
    double* YT = (double*)malloc(sizeof(double) * n * (iters + 1)); /* ytilde^i */
    double* XS = (double*)malloc(sizeof(double) * n * (iters + 1)); /* x^{i+1} at slot i */
    double* UH = (double*)malloc(sizeof(double) * n * (iters + 1)); /* u^{i+1} */
    double* UV = (double*)malloc(sizeof(double) * n * (iters + 1));
    double *vh = malloc(sizeof(double) * n), *vv = malloc(sizeof(double) * n);
    double *dh = malloc(sizeof(double) * n), *dv = malloc(sizeof(double) * n);
    double* yt = (double*)malloc(sizeof(double) * n);
    or_init_state(M, N, K, y, mask, yt, vh, vv, dh, dv);
    for (int it = 0; it < iters; ++it) {
        memcpy(YT + n * it, yt, sizeof(double) * n);
        double muc = mu;
        double* xx = XS + n * it;
        /* u^{i+1} = D x^{i+1} + d^i, recorded before the step overwrites d */
        double* dh0 = (double*)malloc(sizeof(double) * n);
        double* dv0 = (double*)malloc(sizeof(double) * n);
        memcpy(dh0, dh, sizeof(double) * n);
        memcpy(dv0, dv, sizeof(double) * n);
        or_admm_iterate(M, N, K, h, mask, lam, &muc, alpha, 1, phi, 1, 0.0, yt, vh, vv, dh, dv, xx, NULL);
        double *gh = UH + n * it, *gv = UV + n * it;
        or_grad(M, N, xx, gh, gv);
        for (size_t j = 0; j < n; ++j) { gh[j] += dh0[j]; gv[j] += dv0[j]; }
        free(dh0); free(dv0);
    }
    memcpy(YT + n * iters, yt, sizeof(double) * n);

    cplx* Hs = (cplx*)malloc(sizeof(cplx) * n);
    psf_spectrum(M, N, K, h, Hs);
    /* adjoint state of (z, v, d) after the current iteration */
    double* zb = (double*)calloc(n, sizeof(double));
    double* vbh = (double*)calloc(n, sizeof(double));
    double* vbv = (double*)calloc(n, sizeof(double));
    double* dbh = (double*)calloc(n, sizeof(double));
    double* dbv = (double*)calloc(n, sizeof(double));
    double* ybar = (double*)calloc(n, sizeof(double));
    double* ubh = (double*)malloc(sizeof(double) * n);
    double* ubv = (double*)malloc(sizeof(double) * n);
    double* xb = (double*)malloc(sizeof(double) * n);
    double* qb = (double*)malloc(sizeof(double) * n);
    double* tmp = (double*)malloc(sizeof(double) * n);
    double* rb = (double*)malloc(sizeof(double) * n);
    double* hrb = (double*)malloc(sizeof(double) * n);
    double* hx = (double*)malloc(sizeof(double) * n);
    double* drh = (double*)malloc(sizeof(double) * n);
    double* drv = (double*)malloc(sizeof(double) * n);
    cplx* F = (cplx*)malloc(sizeof(cplx) * n);
    for (int k = 0; k < K * K; ++k) grad_h[k] = 0;
    double lbar = 0;

    for (int it = iters - 1; it >= 0; --it) {
        const double* xx = XS + n * it;
        const double* yti = YT + n * it;
        /* d^{i+1} = u - v^{i+1}, v^{i+1} = prox(u) */
        for (size_t j = 0; j < n; ++j) {
            double uh = UH[n * it + j], uv = UV[n * it + j];
            double th = vbh[j] - dbh[j], tv = vbv[j] - dbv[j]; /* adjoint reaching prox output */
            double jh, jv; /* J^T t */
            if (phi == OR_PHI_QUAD) {
                double s = mu / (lam + mu);
                jh = s * th; jv = s * tv;
                /* d prox / d lambda = -mu u / (lam+mu)^2 */
                lbar += -(mu / ((lam + mu) * (lam + mu))) * (uh * th + uv * tv);
            } else {
                double tau = lam / mu;
                double nr = sqrt(uh * uh + uv * uv);
                if (nr > tau) {
                    double s = 1.0 - tau / nr;
                    double ut = (uh * th + uv * tv) * tau / (nr * nr * nr);
                    jh = s * th + ut * uh;
                    jv = s * tv + ut * uv;
                    /* d prox / d tau = -u/|u|, tau = lambda / mu */
                    lbar += -(uh * th + uv * tv) / nr / mu;
                } else {
                    jh = 0; jv = 0;
                }
            }
            ubh[j] = dbh[j] + jh;
            ubv[j] = dbv[j] + jv;
        }
        /* x-bar = grad (last iterate only) + D^T u-bar + H^T q-bar,
           q-bar = alpha M_z^T z-bar (the z-step's use of Hx) */
        or_gradT(M, N, ubh, ubv, xb);
        if (it == iters - 1)
            for (size_t j = 0; j < n; ++j) xb[j] += grad_x[j];
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < N; ++j) {
                size_t k = (size_t)i * N + j;
                qb[k] = observed(M, N, b, mask, i, j) ? 0.0 : alpha * zb[k];
            }
        apply_H(M, N, Hs, qb, tmp, 1);
        for (size_t j = 0; j < n; ++j) xb[j] += tmp[j];
        /* r-bar = A^{-1} x-bar, A = H^T H + mu D^T D (symmetric) */
        for (size_t j = 0; j < n; ++j) F[j] = xb[j];
        dft2(M, N, F, -1);
        for (int ky = 0; ky < M; ++ky)
            for (int kx = 0; kx < N; ++kx) {
                size_t k = (size_t)ky * N + kx;
                double h2 = creal(Hs[k]) * creal(Hs[k]) + cimag(Hs[k]) * cimag(Hs[k]);
                F[k] /= (h2 + mu * dsq(M, N, ky, kx));
            }
        dft2(M, N, F, +1);
        for (size_t j = 0; j < n; ++j) rb[j] = creal(F[j]) / (double)n;
        apply_H(M, N, Hs, rb, hrb, 0);
        apply_H(M, N, Hs, xx, hx, 0);
        /* dL/dh: q = Hx, r = H^T ytilde, A = H^T H */
        corr_acc(M, N, K, qb, xx, +1.0, grad_h);
        corr_acc(M, N, K, yti, rb, +1.0, grad_h);
        corr_acc(M, N, K, hx, rb, -1.0, grad_h);
        corr_acc(M, N, K, hrb, xx, -1.0, grad_h);
        /* ytilde^i feeds r through H^T: its adjoint is H r-bar.
           observed part -> y; unobserved part -> z (plus the relaxation's
           (1 - alpha) z^i term). v^i, d^i feed r through mu D^T (v - d). */
        or_grad(M, N, rb, drh, drv);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < N; ++j) {
                size_t k = (size_t)i * N + j;
                if (observed(M, N, b, mask, i, j)) {
                    ybar[k] += hrb[k];
                    zb[k] = 0;
                } else {
                    zb[k] = (1.0 - alpha) * zb[k] + hrb[k];
                }
                vbh[k] = mu * drh[k];
                vbv[k] = mu * drv[k];
                dbh[k] = ubh[k] - mu * drh[k];
                dbv[k] = ubv[k] - mu * drv[k];
            }
    }
    /* initialisation: ytilde^0 = E(y), v^0 = D ytilde^0, d^0 = 0 */
    or_gradT(M, N, vbh, vbv, tmp);
    double* e = (double*)calloc(n, sizeof(double));
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            size_t k = (size_t)i * N + j;
            if (observed(M, N, b, mask, i, j)) ybar[k] += tmp[k];
            else e[k] = zb[k] + tmp[k];
        }
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j)
            if (!in_valid(M, N, b, i, j) && !observed(M, N, b, mask, i, j)) {
                int si = clampi(i, b, M - b - 1), sj = clampi(j, b, N - b - 1);
                e[(size_t)si * N + sj] += e[(size_t)i * N + j];
            }
    double madj = 0;
    long long cnt = 0;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            size_t k = (size_t)i * N + j;
            if (observed(M, N, b, mask, i, j)) { ybar[k] += e[k]; ++cnt; }
            else if (in_valid(M, N, b, i, j)) madj += e[k];
        }
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            size_t k = (size_t)i * N + j;
            grad_y[k] = observed(M, N, b, mask, i, j) ? ybar[k] + (cnt ? madj / (double)cnt : 0.0) : 0.0;
        }
    *grad_lam = lbar;
    free(e);
    free(F); free(drv); free(drh); free(hx); free(hrb); free(rb); free(tmp); free(qb); free(xb);
    free(ubv); free(ubh); free(ybar); free(dbv); free(dbh); free(vbv); free(vbh); free(zb);
    free(Hs); free(yt); free(dv); free(dh); free(vv); free(vh);
    free(UV); free(UH); free(XS); free(YT);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the parallel loops that follow (timing only; the arithmetic
   does not depend on it) */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
