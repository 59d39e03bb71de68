// Host side of the C ABI: operator setup (extraction, on-device Pade factors),
// the remainder evaluation, exp / phi1 actions and the Lawson / ERK step sequences.
// Everything that computes on grid data runs in the kernels of contract.hip,
// stencil.hip and spectral.hip; this file only validates arguments, allocates, and
// enqueues (and, for periodic problems, sums the first columns of the circulant
// factors from their Fourier symbols at setup).
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>

#include "mm_internal.h"

using namespace mm;

namespace {

void set_err(mm_ctx* ctx, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->last_error = buf;
}

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_err(ctx, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return MM_EDEVICE;                                                                   \
    }                                                                                      \
  } while (0)

// q-point Gauss-Legendre rule on [0, 1]: Newton iteration on the Legendre polynomial
// P_q (three-term recurrence) from the Chebyshev-like initial guesses.
void gauss_legendre(int q, double* theta, double* w) {
  for (int i = 0; i < q; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = x; p0 = 1.0; }
      dp = q * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= q; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p1 = x; p0 = 1.0; }
    dp = q * (x * p1 - p0) / (x * x - 1.0);
    theta[q - 1 - i] = 0.5 * (x + 1.0);
    w[q - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);  // 2/((1-x^2)P'^2) halved for [0,1]
  }
}

hipError_t gemm_sq(int n, const double* X, const double* Y, double* Z, hipStream_t s) {
  GemmArgs g{};
  g.A[0] = X;
  g.B[0] = Y;
  g.C[0] = Z;
  g.Cadd[0] = nullptr;
  g.M = g.N = g.K = n;
  g.lda = g.ldb = g.ldc = n;
  g.inner = 1;
  g.groups = 1;
  g.b_trans = 1;
  g.alpha = 1.0;
  g.beta = 0.0;
  return launch_gemm(MM_FP64, g, s);
}

// Q^{-1} P by the Newton-Schulz iteration X <- X (2I - Q X) from X0 = Q^T/(|Q|_1 |Q|_inf)
// (quadratic convergence once |I - Q X| < 1; Pan and Schreiber, SIAM J. Sci. Stat.
// Comput. 12(5), 1991), all products on the FP64 MFMA GEMM. The Pade denominator of
// a matrix with |A|_1 <= theta_13 is well conditioned, so a handful of iterations
// reach the rounding floor. On success the result overwrites P; Q is never written.
// X, R, Y are n x n scratch. Returns MM_NOT_READY, with P untouched, if the residual
// does not fall below 1e-10 within 60 iterations (the caller then uses Gaussian
// elimination).
mm_status newton_schulz_solve(mm_ctx* ctx, int n, const double* Q, double* P, double* X, double* R,
                              double* Y) {
  hipStream_t st = ctx->stream;
  double* scal = ctx->reduce_buf;   // two doubles of device scratch
  double h[2];
  HIPCHK(ctx, launch_norms(Q, n, scal, st));
  HIPCHK(ctx, hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  if (!(h[0] > 0.0) || !(h[1] > 0.0) || !std::isfinite(h[0] * h[1])) return MM_NOT_READY;
  HIPCHK(ctx, launch_scaled_transpose(X, Q, n, 1.0 / (h[0] * h[1]), st));
  int extra = -1;
  for (int it = 0; it < 60; ++it) {
    HIPCHK(ctx, gemm_sq(n, Q, X, R, st));                 // R = Q X
    HIPCHK(ctx, launch_resid(R, n, scal, st));
    double res = 0.0;
    HIPCHK(ctx, hipMemcpyAsync(&res, scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    if (!std::isfinite(res)) return MM_NOT_READY;
    if (extra < 0 && res < 1e-10) extra = 1;              // one more step reaches the floor
    else if (extra == 0) break;
    else if (extra > 0) --extra;
    HIPCHK(ctx, launch_combo(R, n, -1.0, R, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, 2.0, st));  // 2I - QX
    HIPCHK(ctx, gemm_sq(n, X, R, Y, st));                 // X (2I - QX)
    std::swap(X, Y);
    if (it == 59) return MM_NOT_READY;
  }
  HIPCHK(ctx, gemm_sq(n, X, P, Y, st));                   // Q^{-1} P
  HIPCHK(ctx, hipMemcpyAsync(P, Y, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  return MM_OK;
}

// exp(T) for the n x n tridiagonal Toeplitz T = tridiag(sub, diag, sup) by the [13/13]
// Pade approximant with scaling and squaring (Higham, SIAM J. Matrix Anal. Appl. 26(4),
// 2005): s = max(0, ceil(log2(||T||_1 / theta_13))), X = r_13(T/2^s), then s squarings.
// The Pade numerator coefficients are b_j = (26 - j)! / (j! (13 - j)!).
// neumann: the last row is [.., sub + sup, diag] (the mirror ghost of a zero normal
// derivative at x = 1), which adds at most |sub + sup| to a column sum.
mm_status pade_expm(mm_ctx* ctx, int n, double sub, double diag, double sup, bool neumann, double* out, int* s_out,
                    double* ws) {
  hipStream_t st = ctx->stream;
  const double last_sub = (neumann && n >= 2) ? sub + sup : sub;
  double nrm = std::fabs(diag);
  if (n == 2) nrm += std::fmax(std::fabs(last_sub), std::fabs(sup));
  if (n >= 3) nrm += std::fabs(sub) + std::fabs(sup) + (neumann ? std::fabs(last_sub) : 0.0);
  const double theta13 = 5.371920351148152;
  int s = 0;
  if (nrm > theta13) s = (int)std::ceil(std::log2(nrm / theta13));
  const double sc = std::ldexp(1.0, -s);
  double b[14];
  for (int j = 0; j <= 13; ++j) {
    unsigned __int128 num = 1;
    for (int k = 13 - j + 1; k <= 26 - j; ++k) num *= (unsigned __int128)k;  // (26-j)!/(13-j)!
    unsigned __int128 den = 1;
    for (int k = 2; k <= j; ++k) den *= (unsigned __int128)k;
    b[j] = (double)(num / den);
  }
  const int64_t nn = (int64_t)n * n;
  double *A = ws, *A2 = ws + nn, *A4 = ws + 2 * nn, *A6 = ws + 3 * nn, *T1 = ws + 4 * nn, *U = ws + 5 * nn,
         *V = ws + 6 * nn;
  HIPCHK(ctx, launch_build_tridiag(A, n, sub * sc, diag * sc, sup * sc, last_sub * sc, st));
  HIPCHK(ctx, gemm_sq(n, A, A, A2, st));
  HIPCHK(ctx, gemm_sq(n, A2, A2, A4, st));
  HIPCHK(ctx, gemm_sq(n, A4, A2, A6, st));
  // U = A [A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I]
  HIPCHK(ctx, launch_combo(T1, n, b[13], A6, b[11], A4, b[9], A2, 0.0, nullptr, 0.0, st));
  HIPCHK(ctx, gemm_sq(n, A6, T1, V, st));
  HIPCHK(ctx, launch_combo(V, n, 1.0, V, b[7], A6, b[5], A4, b[3], A2, b[1], st));
  HIPCHK(ctx, gemm_sq(n, A, V, U, st));
  // V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
  HIPCHK(ctx, launch_combo(T1, n, b[12], A6, b[10], A4, b[8], A2, 0.0, nullptr, 0.0, st));
  HIPCHK(ctx, gemm_sq(n, A6, T1, V, st));
  HIPCHK(ctx, launch_combo(V, n, 1.0, V, b[6], A6, b[4], A4, b[2], A2, b[0], st));
  // (V - U) X = (V + U): P in A2, Q in A4
  HIPCHK(ctx, launch_combo(A2, n, 1.0, V, 1.0, U, 0.0, nullptr, 0.0, nullptr, 0.0, st));
  HIPCHK(ctx, launch_combo(A4, n, 1.0, V, -1.0, U, 0.0, nullptr, 0.0, nullptr, 0.0, st));
  mm_status rs = newton_schulz_solve(ctx, n, A4, A2, A6, T1, U);
  if (rs == MM_NOT_READY) {   // not converged: Gaussian elimination (Q and P are intact)
    HIPCHK(ctx, launch_lu_solve(A4, A2, n, 1, st));
  } else if (rs != MM_OK) {
    return rs;
  }
  double* X = A2;
  double* Y = A6;
  for (int i = 0; i < s; ++i) {
    HIPCHK(ctx, gemm_sq(n, X, X, Y, st));
    double* t = X;
    X = Y;
    Y = t;
  }
  HIPCHK(ctx, hipMemcpyAsync(out, X, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (s_out) *s_out = s;
  return MM_OK;
}

// Device memory of ops comes from the stream-ordered pool on the context's stream, so
// that creating and releasing ops does not synchronise the device (plain hipFree may),
// which keeps admission in the request server from stalling on running requests.
template <typename T>
mm_status dev_alloc(mm_op* op, T** p, int64_t count) {
  const size_t bytes = (size_t)count * sizeof(T);
  hipError_t e = hipMallocAsync((void**)p, bytes, op->ctx->stream);
  if (e != hipSuccess) {
    set_err(op->ctx, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    *p = nullptr;
    return MM_ENOMEM;
  }
  op->bytes += (int64_t)bytes;
  return MM_OK;
}

int last_axis(const mm_op* op) { return op->d - 1; }

void dev_free(mm_op* op, void* p) {
  if (p) hipFreeAsync(p, op->ctx->stream);
}

// Bracket one launch with events on its stream when the context is timing.
template <typename F>
hipError_t timed_launch(mm_ctx* ctx, int kind, double work, hipStream_t s, F&& launch) {
  if (!ctx || !ctx->timing) return launch();
  if (ctx->timed_used == ctx->timed.size()) {
    mm_timed t{};
    if (hipEventCreate(&t.start) != hipSuccess || hipEventCreate(&t.stop) != hipSuccess)
      return hipErrorOutOfMemory;
    ctx->timed.push_back(t);
  }
  mm_timed& t = ctx->timed[ctx->timed_used++];
  t.kind = kind;
  t.work = work;
  hipError_t e = hipEventRecord(t.start, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  return hipEventRecord(t.stop, s);
}

// Floating-point operations of a mode-product launch: 2 M N K, or for a folded product the
// two half-size products (2 f x f factor values against the grid's other dimension).
double gemm_work(const GemmArgs& g, int prec) {
  if (use_fold(g, prec)) {
    // each of the fold_blocks stacked n x n factors contributes a half-size pair
    const int G = g.fold_blocks > 1 ? g.fold_blocks : 1;
    const int n = g.K / G;
    const double f = n - n / 2;
    return 4.0 * f * f * G * (g.b_trans ? (double)g.N : (double)g.M) * g.inner * g.groups;
  }
  return 2.0 * g.M * (double)g.N * g.K * g.inner * g.groups;
}

hipError_t gemm(const mm_op* op, GemmArgs& g, hipStream_t s) {
  const double work = gemm_work(g, op->prec);
  g.tile = op->ctx ? op->ctx->gemm_tile : 0;
  g.vdig = op->vdig;
  g.vexp = op->vexp;
  g.vdig_cap = op->vdig_len;
  g.vexp_cap = op->vexp_len;
  return timed_launch(op->ctx, g.b_trans ? MM_KIND_GEMM_N : MM_KIND_GEMM_K, work, s,
                      [&] { return launch_gemm(op->prec, g, s); });
}

// FP64 mode product along axis mu with a dense n_mu x n_mu matrix M (out_i = sum_j M_ij
// in_j along the axis), out = M x_mu in (+ add): the layouts of the three mode passes.
hipError_t mode_product64(const mm_op* op, int mu, const double* M, const double* in, double* out,
                          const double* add, hipStream_t s) {
  const int n = op->n[mu];
  const int64_t dof = op->dof;
  GemmArgs g{};
  g.groups = 1;
  g.alpha = 1.0;
  g.beta = add ? 1.0 : 0.0;
  g.Cadd[0] = add;
  g.C[0] = out;
  g.inner = 1;
  if (mu == 0) {
    g.A[0] = in;
    g.B[0] = M;
    g.M = (int)(dof / n);
    g.N = g.K = n;
    g.lda = g.ldb = g.ldc = n;
    g.b_trans = 0;
  } else if (mu == op->d - 1) {
    const int P = (int)(dof / n);
    g.A[0] = M;
    g.B[0] = in;
    g.M = g.K = n;
    g.N = P;
    g.lda = n;
    g.ldb = g.ldc = P;
    g.b_trans = 1;
  } else {   // x2 of a 3D grid: per x3 slab
    g.A[0] = M;
    g.B[0] = in;
    g.M = g.K = n;
    g.N = op->n[0];
    g.lda = n;
    g.ldb = g.ldc = op->n[0];
    g.inner = op->n[2];
    g.sA = 0;
    g.sB = g.sC = (int64_t)op->n[0] * op->n[1];
    g.b_trans = 1;
  }
  g.tile = op->ctx ? op->ctx->gemm_tile : 0;
  const double work = 2.0 * g.M * (double)g.N * g.K * g.inner;
  return timed_launch(op->ctx, g.b_trans ? MM_KIND_GEMM_N : MM_KIND_GEMM_K, work, s,
                      [&] { return launch_gemm(MM_FP64, g, s); });
}

// Remainder of a periodic problem (pseudo-spectral, FP64 whatever the op's precision):
// G = r(u); per axis T1 = D x_mu u, the pointwise pass, G += D1 x_mu T2; for F also
// G += A_mu x_mu u; then the stage outputs of `a` from G (the stencil's contract).
// The chains of the axes are independent up to the stage outputs: axis 0 runs on s, every
// further axis on a side stream of its own (forked from and joined back to s with events,
// so the calls stay stream-ordered and capturable) into its own accumulator. A mode
// product of a 256-point axis has only sixteen workgroups, so running the chains side by
// side fills more of the chip than running them one after another.
hipError_t spectral_remainder(const mm_op* op, const StencilArgs& a, hipStream_t s) {
  const int64_t dof = op->dof;
  // the pointwise pass writes FP64 or FP32 stage outputs only (no digit planes)
  if (a.dig || (!a.out0 && !a.out0f)) return hipErrorInvalidValue;
  const bool nondiv = op->form == MM_FORM_NONDIV;
  hipError_t e = hipSuccess;
  if (op->d > 1) {
    e = hipEventRecord(op->spec_fork, s);
    for (int mu = 1; mu < op->d && e == hipSuccess; ++mu) e = hipStreamWaitEvent(op->spec_side[mu - 1], op->spec_fork, 0);
  }
  const double* Gs[3] = {nullptr, nullptr, nullptr};
  for (int mu = 0; mu < op->d && e == hipSuccess; ++mu) {
    const hipStream_t sm = mu == 0 ? s : op->spec_side[mu - 1];
    double* G = op->spec_ws + 3 * mu * dof;
    double* T1 = G + dof;
    double* T2 = T1 + dof;
    Gs[mu] = G;
    const int64_t nn = (int64_t)op->n[mu] * op->n[mu];
    const double* D1 = op->dmat[mu];
    const double* D2 = D1 + nn;
    if ((e = mu == 0 ? launch_spec_react(G, a.u, dof, op->r, sm) : launch_fill(G, 0.0, dof, sm)) != hipSuccess) break;
    if ((e = mode_product64(op, mu, nondiv ? D2 : D1, a.u, T1, nullptr, sm)) != hipSuccess) break;
    SpecMidArgs m{};
    m.G = G;
    m.T2 = T2;
    m.T1 = T1;
    m.u = a.u;
    m.a = op->a + mu * dof;
    m.vel = op->vel ? op->vel + mu * dof : nullptr;
    m.lam_amax = op->lam * op->amax_mu[mu];
    m.beta = op->beta[mu];
    m.beta_bar = op->beta_bar[mu];
    m.n = dof;
    m.nondiv = nondiv;
    if ((e = launch_spec_mid(m, sm)) != hipSuccess) break;
    // the outer derivative: of the flux, or (non-divergence form) of the advected u only
    if (!nondiv || op->vel || op->beta[mu] != op->beta_bar[mu])
      if ((e = mode_product64(op, mu, D1, T2, G, G, sm)) != hipSuccess) break;
    if (a.full && (e = mode_product64(op, mu, D1 + 2 * nn, a.u, G, G, sm)) != hipSuccess) break;
    if (mu > 0 && (e = hipEventRecord(op->spec_join[mu - 1], sm)) == hipSuccess)
      e = hipStreamWaitEvent(s, op->spec_join[mu - 1], 0);
  }
  if (e != hipSuccess) return e;
  return launch_spec_combine(Gs, a, dof, s);
}

hipError_t stencil(const mm_op* op, const StencilArgs& a, hipStream_t s) {
  if (op->periodic) return spectral_remainder(op, a, s);
  return timed_launch(op->ctx, MM_KIND_STENCIL, (double)op->dof, s,
                      [&] { return launch_stencil(op->d, a, s); });
}

// ---------------------------------------------------------------- mode passes
// Operand formats of one mode pass: the grid operand is read as float (in_f32) or
// double, C is written as float (out_f32) or double. FP64 ops always use double.
struct PassIO {
  bool in_f32 = false, out_f32 = false;
  bool ready = false;   // MM_SLICED mode 1: the grid operand is already split (by the stencil)
};

// Low-precision modes pass FP32 values between the passes of an action.
bool lowp(const mm_op* op) { return op->prec == MM_FP32 || op->prec == MM_BF16X3 || op->prec == MM_BF16X6; }

// padded row stride of the factor operand for contraction length k
int factor_ld(const mm_op* op, int k) {
  return op->prec == MM_FP64 ? k : op->prec == MM_SLICED ? slice_ld(k) : fac_ld(k);
}

// elements per slice plane of a rows x k factor operand (0 for single-plane formats)
int64_t factor_slice_stride(const mm_op* op, int rows, int k) {
  if (op->prec == MM_FP64 || op->prec == MM_FP32) return 0;
  return (int64_t)rows * factor_ld(op, k);
}

// bytes of one n x n factor operand in the op's precision, all slices
int64_t factor_bytes(const mm_op* op, int n) {
  switch (op->prec) {
    case MM_FP64: return (int64_t)n * n * 8;
    case MM_FP32: return (int64_t)n * fac_ld(n) * 4;
    case MM_SLICED: return (int64_t)n * slice_ld(n) * op->slices;
    default: return (int64_t)n * fac_ld(n) * 2 * factor_slices(op->prec);
  }
}

// the factor operand of axis mu, coefficient index j, in the op's precision
const void* factor_op(const mm_op* op, int mu, int j) {
  if (op->prec == MM_FP64) return op->fac[mu] + (int64_t)j * op->n[mu] * op->n[mu];
  return (const char*)op->fac_lp[mu] + j * factor_bytes(op, op->n[mu]);
}

// per-row exponents of that factor (MM_SLICED only, else null)
const int* factor_exp(const mm_op* op, int mu, int j) {
  if (op->prec != MM_SLICED) return nullptr;
  return op->fac_exp[mu] + (int64_t)j * op->n[mu];
}

// the folded form [Es; Ed] of exp factor j of axis mu (FP64 centrosymmetric axes), else
// null; rows of n_mu - n_mu/2 values
const double* folded(const mm_op* op, int mu, int j) {
  if (op->prec != MM_FP64 || mu >= (int)op->ffold.size() || !op->ffold[mu] || j < 0 || j >= op->nfold) return nullptr;
  const int64_t f = op->n[mu] - op->n[mu] / 2;
  return op->ffold[mu] + (int64_t)j * 2 * f * fold_ld(op->n[mu]);
}

// (call with the launch's shape set). The grouped passes of one op (its φ1 quadrature
// nodes and ERK stage groups) fold when all groups together have at least 512 folded
// tiles (127^3 ETD2RK: five groups of 127 tiles, 0.383 -> 0.345 ms/step), whatever each
// group alone has; single launches follow the launcher's per-problem rule. The server's
// grouped launches (group_pass) keep the per-problem rule: theirs must not depend on the
// group count.
void set_fold(const mm_op* op, GemmArgs& g, int mu) {
  g.ldf = (g.fold_blocks > 1 ? g.fold_blocks : 1) * fold_ld(op->n[mu]);
  g.fold = op->ctx ? op->ctx->fold : 1;
  if (g.fold == 1 && g.groups > 1) g.fold = fold_tiles(g) * g.groups >= 512 ? 2 : 0;
}

// the stacked last-axis factor of an ERK stage in the op's precision
const void* stacked(const mm_op* op, int which) {
  if (op->prec == MM_FP64) return which == 1 ? op->f3_stage1 : which == 2 ? op->f3_stage2 : op->f3_phi;
  return which == 1 ? op->f3_stage1_lp : which == 2 ? op->f3_stage2_lp : op->f3_phi_lp;
}

const int* stacked_exp(const mm_op* op, int which) {
  return which == 1 ? op->f3_stage1_exp : which == 2 ? op->f3_stage2_exp : op->f3_phi_exp;
}

// Memory layout of a grid operand: x1 rows of `ld` values (ld >= n1; larger for the
// padded stage vectors of the Lawson steps) and `vs` values between stacked vectors.
// Every layout here is dense above the rows: plane stride n2 ld, vs = n2 n3 ld.
struct Layout {
  int ld;
  int64_t vs;
};
Layout natural(const mm_op* op) { return Layout{op->n[0], op->dof}; }
Layout staged(const mm_op* op) { return Layout{op->ld1, op->dofp}; }

// mode 1: C (rows x n1) = A (rows x n1) . E1^T, per group (input, factor, output);
// galpha: optional per-group output scales (sliced mode only)
hipError_t pass_mode1(const mm_op* op, int groups, const void* const* in, const int* fidx,
                      void* const* out, int rows, PassIO io, hipStream_t s, const double* galpha = nullptr,
                      Layout li = Layout{0, 0}, Layout lo = Layout{0, 0}) {
  const int n1 = op->n[0];
  GemmArgs g{};
  for (int i = 0; i < groups; ++i) {
    g.A[i] = in[i];
    g.B[i] = factor_op(op, 0, fidx[i]);
    g.Ff[i] = folded(op, 0, fidx[i]);
    g.fexp[i] = factor_exp(op, 0, fidx[i]);
    g.galpha[i] = galpha ? galpha[i] : 0.0;
    g.C[i] = out[i];
    g.Cadd[i] = nullptr;
  }
  g.slices = op->slices;
  g.M = rows;
  g.N = n1;
  g.K = n1;
  g.lda = li.ld ? li.ld : n1;
  g.ldb = factor_ld(op, n1);
  g.ldc = lo.ld ? lo.ld : n1;
  g.inner = 1;
  g.groups = groups;
  g.b_trans = 0;
  g.alpha = 1.0;
  g.beta = 0.0;
  g.in_f32 = io.in_f32;
  g.out_f32 = io.out_f32;
  g.fac_slice = factor_slice_stride(op, n1, n1);
  g.vready = io.ready;
  set_fold(op, g, 0);
  return gemm(op, g, s);
}

// mode 2 of a 3D grid: per x3-slab (n2 x n1), C = E2 . slab, `slabs` slabs per group
hipError_t pass_mode2(const mm_op* op, int groups, const int* fidx, const void* const* in, void* const* out,
                      int slabs, PassIO io, hipStream_t s, Layout li = Layout{0, 0}, Layout lo = Layout{0, 0}) {
  const int ldi = li.ld ? li.ld : op->n[0], ldo = lo.ld ? lo.ld : op->n[0];
  GemmArgs g{};
  for (int i = 0; i < groups; ++i) {
    g.A[i] = factor_op(op, 1, fidx[i]);
    g.Ff[i] = folded(op, 1, fidx[i]);
    g.fexp[i] = factor_exp(op, 1, fidx[i]);
    g.B[i] = in[i];
    g.C[i] = out[i];
    g.Cadd[i] = nullptr;
  }
  g.slices = op->slices;
  g.M = op->n[1];
  g.N = op->n[0];
  g.K = op->n[1];
  g.lda = factor_ld(op, op->n[1]);
  g.ldb = ldi;
  g.ldc = ldo;
  g.inner = slabs;
  g.sA = 0;
  g.sB = (int64_t)ldi * op->n[1];
  g.sC = (int64_t)ldo * op->n[1];
  g.groups = groups;
  g.b_trans = 1;
  g.alpha = 1.0;
  g.beta = 0.0;
  g.in_f32 = io.in_f32;
  g.out_f32 = io.out_f32;
  g.fac_slice = factor_slice_stride(op, op->n[1], op->n[1]);
  set_fold(op, g, 1);
  return gemm(op, g, s);
}

// last mode: C (nl x P) = alpha * F (nl x K) . B (K x P) + beta * add, K = kmul * nl,
// P = dof / nl; `inner` stacked vectors of stride dof (same factor). F is the factor
// operand in the op's precision (row stride factor_ld(K)), Fexp its row exponents
// (MM_SLICED).
// With layouts: stacked vectors `vs` apart; in 3D a padded layout makes the columns the
// (x2, x1) positions including the row padding (computed, never read as data), and
// input and output layouts that differ take one launch per vector, batched over x2.
hipError_t pass_last(const mm_op* op, const void* F, const int* Fexp, int kmul, const void* in, void* out,
                     const double* add, double alpha, double beta, int inner, PassIO io, hipStream_t s,
                     Layout li = Layout{0, 0}, Layout lo = Layout{0, 0}, const double* Ffold = nullptr) {
  const int nl = op->n[last_axis(op)];
  const int P = (int)(op->dof / nl);
  if (li.ld && lo.ld && (li.ld != op->n[0] || lo.ld != op->n[0])) {
    const size_t ib = io.in_f32 ? 4 : 8, ob = io.out_f32 ? 4 : 8;
    GemmArgs g{};
    g.A[0] = F;
    g.Ff[0] = Ffold;
    g.fold_blocks = kmul;
    set_fold(op, g, last_axis(op));
    g.fexp[0] = Fexp;
    g.slices = op->slices;
    g.Cadd[0] = nullptr;
    g.M = nl;
    g.K = kmul * nl;
    g.lda = factor_ld(op, kmul * nl);
    g.groups = 1;
    g.b_trans = 1;
    g.alpha = alpha;
    g.beta = 0.0;
    g.in_f32 = io.in_f32;
    g.out_f32 = io.out_f32;
    g.fac_slice = factor_slice_stride(op, nl, kmul * nl);
    if (add) return hipErrorInvalidValue;   // not needed by the padded schemes
    if (op->d == 2 || li.ld == lo.ld) {
      // rows of the operand are the last axis: N = (2D) x1 or (3D) the padded plane
      const int ncols = op->d == 2 ? op->n[0] : op->n[1] * li.ld;
      g.B[0] = in;
      g.C[0] = out;
      g.N = ncols;
      g.ldb = op->d == 2 ? li.ld : op->n[1] * li.ld;
      g.ldc = op->d == 2 ? lo.ld : op->n[1] * lo.ld;
      g.inner = inner;
      g.sA = 0;
      g.sB = li.vs;
      g.sC = lo.vs;
      return gemm(op, g, s);
    }
    // 3D with different row strides: per vector, batched over the x2 rows
    for (int v = 0; v < inner; ++v) {
      g.B[0] = (const char*)in + (size_t)v * li.vs * ib;
      g.C[0] = (char*)out + (size_t)v * lo.vs * ob;
      g.N = op->n[0];
      g.ldb = op->n[1] * li.ld;
      g.ldc = op->n[1] * lo.ld;
      g.inner = op->n[1];
      g.sA = 0;
      g.sB = li.ld;
      g.sC = lo.ld;
      const hipError_t e = gemm(op, g, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  GemmArgs g{};
  g.A[0] = F;
  g.Ff[0] = Ffold;
  g.fold_blocks = kmul;
  set_fold(op, g, last_axis(op));
  g.fexp[0] = Fexp;
  g.slices = op->slices;
  g.B[0] = in;
  g.C[0] = out;
  g.Cadd[0] = add;
  g.M = nl;
  g.N = P;
  g.K = kmul * nl;
  g.lda = factor_ld(op, kmul * nl);
  g.ldb = P;
  g.ldc = P;
  g.inner = inner;
  g.sA = 0;
  g.sB = g.sC = op->dof;
  g.groups = 1;
  g.b_trans = 1;
  g.alpha = alpha;
  g.beta = beta;
  g.in_f32 = io.in_f32;
  g.out_f32 = io.out_f32;
  g.fac_slice = factor_slice_stride(op, nl, kmul * nl);
  return gemm(op, g, s);
}

const double* factor(const mm_op* op, int mu, int j) {
  return op->fac[mu] + (int64_t)j * op->n[mu] * op->n[mu];
}

// out = exp(c_j tau A) in for `nvec` stacked vectors (stride dof): in -> t0 [-> t1] -> out.
// in_f32: the input is float (mixed modes only); out is always double. In the mixed
// modes the intermediates t0, t1 hold floats.
// out = alpha exp(c_j tau A) in + beta add (add optional).
// li, lt, lo: layouts of in, of the intermediates t0/t1 and of out (default: unpadded).
hipError_t exp_action(const mm_op* op, int j, const void* in, bool in_f32, double* out, int nvec, double* t0,
                      double* t1, hipStream_t s, const double* add = nullptr, double alpha = 1.0,
                      double beta = 1.0, Layout li = Layout{0, 0}, Layout lt = Layout{0, 0},
                      Layout lo = Layout{0, 0}, bool in_digits = false) {
  const bool mixed = lowp(op);
  PassIO first{in_f32, mixed, in_digits}, mid{mixed, mixed}, last_io{mixed, false};
  const int fj[1] = {j};
  const void* i1[1] = {in};
  void* o1[1] = {t0};
  const int la = last_axis(op);
  const void* Fl = factor_op(op, la, j);
  const int* Fe = factor_exp(op, la, j);
  if (op->d == 3) {
    hipError_t e = pass_mode1(op, 1, i1, fj, o1, (int)(op->dof / op->n[0]) * nvec, first, s, nullptr, li, lt);
    if (e != hipSuccess) return e;
    const void* i2[1] = {t0};
    void* o2[1] = {t1};
    e = pass_mode2(op, 1, fj, i2, o2, op->n[2] * nvec, mid, s, lt, lt);
    if (e != hipSuccess) return e;
    return pass_last(op, Fl, Fe, 1, t1, out, add, alpha, add ? beta : 0.0, nvec, last_io, s, lt, lo,
                     folded(op, la, j));
  }
  hipError_t e = pass_mode1(op, 1, i1, fj, o1, (int)(op->dof / op->n[0]) * nvec, first, s, nullptr, li, lt);
  if (e != hipSuccess) return e;
  PassIO l2{mixed, false};
  return pass_last(op, Fl, Fe, 1, t0, out, add, alpha, add ? beta : 0.0, nvec, l2, s, lt, lo, folded(op, la, j));
}

// out = stacked-last-factor contraction over G groups: group g applies modes 1..d-1 with
// factor index fidx[g] to the FP64 input ins[g] (scaled by w1[g] when given); the last
// mode sums the groups with the stacked factor F3 (nl x G*nl, in the op's precision)
// and adds beta*add. t0 and t1 hold G grid functions each (floats in the mixed modes).
hipError_t grouped_action(const mm_op* op, int G, const double* const* ins, const int* fidx, const void* F3,
                          const int* F3exp, double* out, const double* add, double beta, double* t0, double* t1,
                          hipStream_t s, const double* w1 = nullptr) {
  const bool mixed = lowp(op);
  const int64_t esz = mixed ? 4 : 8;
  // the folded form of the stacked factor, when it has one
  const double* F3fold = F3 == op->f3_stage1 ? op->f3_stage1_fold
                         : F3 == op->f3_stage2 ? op->f3_stage2_fold
                         : F3 == op->f3_phi    ? op->f3_phi_fold
                                               : nullptr;
  const void* in1[kMaxGroups];
  void* o1[kMaxGroups];
  for (int g = 0; g < G; ++g) {
    in1[g] = ins[g];
    o1[g] = (char*)t0 + g * op->dof * esz;
  }
  hipError_t e = pass_mode1(op, G, in1, fidx, o1, (int)(op->dof / op->n[0]), PassIO{false, mixed}, s, w1);
  if (e != hipSuccess) return e;
  if (op->d == 3) {
    const void* i2[kMaxGroups];
    void* o2[kMaxGroups];
    for (int g = 0; g < G; ++g) {
      i2[g] = (const char*)t0 + g * op->dof * esz;
      o2[g] = (char*)t1 + g * op->dof * esz;
    }
    e = pass_mode2(op, G, fidx, i2, o2, op->n[2], PassIO{mixed, mixed}, s);
    if (e != hipSuccess) return e;
    return pass_last(op, F3, F3exp, G, t1, out, add, 1.0, beta, 1, PassIO{mixed, false}, s, Layout{0, 0},
                     Layout{0, 0}, F3fold);
  }
  return pass_last(op, F3, F3exp, G, t0, out, add, 1.0, beta, 1, PassIO{mixed, false}, s, Layout{0, 0},
                   Layout{0, 0}, F3fold);
}

// Sliced mode keeps the stacked last-axis blocks unweighted (so that one row exponent
// suits every block) and applies the stage's quadrature weights as per-group scales of
// the first pass instead; other precisions fold the weights into the stacked factor.
// which: 1 stage one (ETD2RK: [1, tau w_j]; ERK2P1: [tau w_j]), 2 stage two
// ([tau/2 w_j]), 3 phi1 ([w_j]). Returns null when the weights are in the factor.
const double* stage_weights(const mm_op* op, int which, double* w) {
  if (op->prec != MM_SLICED) return nullptr;
  int k = 0;
  if (which == 1 && op->scheme == MM_ETD2RK) w[k++] = 1.0;
  const double c = (which == 3) ? 1.0 : (which == 2) ? 0.5 * op->tau : op->tau;
  for (int j = 1; j <= op->q; ++j) w[k++] = c * op->weight[j];
  return w;
}

// exact phi1: factor slots of the eigenvector matrices (A_mu = L diag(ev) R)
constexpr int kFacR = 1, kFacL = 2;

hipError_t eig_scale(const mm_op* op, double* out, const double* a, double ca, int fa, const double* b, double cb,
                     int fb, hipStream_t s) {
  if (op->periodic)
    return launch_spec_eig_scale(out, a, ca, fa, b, cb, fb, op->ev[0], op->ev[1], op->d == 3 ? op->ev[2] : nullptr,
                                 op->n[0], op->n[1], op->d == 3 ? op->n[2] : 1, op->tau, s);
  return launch_eig_scale(out, a, ca, fa, b, cb, fb, op->ev[0], op->ev[1], op->d == 3 ? op->ev[2] : nullptr,
                          op->n[0], op->n[1], op->d == 3 ? op->n[2] : 1, op->tau, s);
}

// mesh width of axis mu: n unknowns at i/(n+1) (Dirichlet data at both ends) or at i/n
// (zero normal derivative at x = 1)
double mesh_h(const mm_op* op, int mu) {
  if (op->bc[mu] == MM_BC_PERIODIC) return op->length[mu] / op->n[mu];
  return op->bc[mu] == MM_BC_NEUMANN ? 1.0 / op->n[mu] : 1.0 / (op->n[mu] + 1);
}

// First column of the real circulant n x n matrix whose eigenvalue on the Fourier mode
// e^{2 pi i m j / n} is sym(m, nyquist): c_j = (1/n) sum_m sym(m) e^{2 pi i m j / n}, m the
// signed wavenumber (|m| <= n/2; nyquist marks m = n/2 of even n). Summed in long double
// with an exact twiddle index (m j mod n).
template <typename F>
std::vector<double> circulant_column(int n, F sym) {
  typedef std::complex<long double> cl;
  std::vector<cl> tw(n), f(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < n; ++k) {
    const long double t = 2.0L * pi * (long double)k / (long double)n;
    tw[k] = cl(std::cos(t), std::sin(t));
  }
  for (int m = 0; m < n; ++m) {
    const int ms = (m <= (n - 1) / 2) ? m : m - n;
    f[m] = sym(ms, n % 2 == 0 && m == n / 2);
  }
  std::vector<double> col(n);
  for (int j = 0; j < n; ++j) {
    cl acc = 0;
    for (int m = 0; m < n; ++m) acc += f[m] * tw[(int64_t)m * j % n];
    col[j] = (double)(acc.real() / (long double)n);
  }
  return col;
}

StencilArgs stencil_args(const mm_op* op, const double* u, bool full) {
  StencilArgs a{};
  a.u = u;
  a.a = op->a;
  a.n1 = op->n[0];
  a.n2 = op->n[1];
  a.n3 = (op->d == 3) ? op->n[2] : 1;
  for (int mu = 0; mu < 3; ++mu) {
    const double h = mesh_h(op, mu);
    a.ih2[mu] = 1.0 / (h * h);
    a.neu[mu] = (mu < op->d) && op->bc[mu] == MM_BC_NEUMANN;
    const double b = full ? op->beta[mu] : op->beta[mu] - op->beta_bar[mu];
    a.cadv[mu] = (mu < op->d) ? b / (2.0 * h) : 0.0;
  }
  a.lam_amax = full ? 0.0 : op->lam * op->a_max;
  a.r0 = op->r[0];
  a.r1 = op->r[1];
  a.r2 = op->r[2];
  a.r3 = op->r[3];
  a.c0 = 1.0;
  a.c1 = 1.0;
  a.flag = op->flag;
  a.nondiv = op->form == MM_FORM_NONDIV;
  a.full = full;
  return a;
}

// Real orthonormal Fourier basis of n equispaced points, Q[j][k] (row-major): column 0
// the constant 1/sqrt(n); columns 2m - 1, 2m for 1 <= m < n/2 sqrt(2/n) cos(2 pi m j/n) and
// sqrt(2/n) sin(2 pi m j/n); for even n column n - 1 the Nyquist mode (-1)^j/sqrt(n).
// Angles from the exact residue m j mod n, in long double.
void fourier_basis(int n, std::vector<double>& Q) {
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double c0 = 1.0L / std::sqrt((long double)n), c1 = std::sqrt(2.0L / n);
  Q.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Q[(size_t)j * n] = (double)c0;
    for (int m = 1; 2 * m < n; ++m) {
      const long double t = 2.0L * pi * (long double)(((int64_t)m * j) % n) / n;
      Q[(size_t)j * n + 2 * m - 1] = (double)(c1 * std::cos(t));
      Q[(size_t)j * n + 2 * m] = (double)(c1 * std::sin(t));
    }
    if (n % 2 == 0 && n > 1) Q[(size_t)j * n + n - 1] = (double)((j % 2 ? -c0 : c0));
  }
}

// Closed-form eigen-decomposition of the tridiagonal Toeplitz matrix with sub-diagonal
// s, diagonal delta and super-diagonal t (s t > 0, or s = t = 0): with rho = sqrt(s/t),
// D = diag(rho^j), the similar matrix D^-1 A D is symmetric tridiagonal with off-diagonal
// sigma = sign(t) sqrt(s t), diagonalised by the orthogonal symmetric sine matrix
// S[j][k] = sqrt(2/(n+1)) sin(j k pi/(n+1)), eigenvalues delta + 2 sigma cos(k pi/(n+1)).
// Hence A = L diag(ev) R with L = D S and R = S D^-1 (R L = I), both row-major n x n.
// The eigenvalues are evaluated as (delta + 2 sigma) - 4 sigma sin^2(k pi/(2(n+1))) with
// delta + 2 sigma = (delta^2 - 4 s t)/(delta - 2 sigma): equal in real arithmetic to
// delta + 2 sigma cos(k pi/(n+1)), whose small eigenvalues lose about 2 |delta| u to
// cancellation (for the stiff exponentials of large grids, 1e-13 relative in exp).
bool eigen_closed_form(int n, double s, double delta, double t, std::vector<double>& ev, std::vector<double>& R,
                       std::vector<double>& L) {
  double rho = 1.0, sigma = 0.0;
  if (s * t > 0.0) {
    rho = std::sqrt(s / t);
    sigma = (t > 0.0 ? 1.0 : -1.0) * std::sqrt(s * t);
  } else if (!(s == 0.0 && t == 0.0)) {
    return false;
  }
  const double pi = 3.14159265358979323846;
  const double c = std::sqrt(2.0 / (n + 1));
  const int64_t per = 2 * (int64_t)(n + 1);             // sin(m pi/(n+1)) has period 2(n+1) in m
  ev.resize(n);
  R.resize((size_t)n * n);
  L.resize((size_t)n * n);
  std::vector<double> dpow(n);
  for (int j = 0; j < n; ++j) dpow[j] = std::pow(rho, j + 1);
  // The operators here are a second difference plus a centred first difference, so
  // delta = -(s + t) up to the rounding of s and t, and delta^2 - 4 s t = (s - t)^2.
  const double dm = delta - 2.0 * sigma;
  const bool second_difference = std::fabs(delta + s + t) <= 1e-15 * std::fabs(delta);
  const double c0 = (dm != 0.0 && second_difference) ? (s - t) * (s - t) / dm : delta + 2.0 * sigma;
  for (int k = 0; k < n; ++k) {
    const double h = std::sin((k + 1) * pi / (2.0 * (n + 1)));
    ev[k] = c0 - 4.0 * sigma * h * h;
  }
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) {
      const int64_t m = ((int64_t)(j + 1) * (k + 1)) % per;   // exact argument reduction
      const double sjk = c * std::sin(m * pi / (n + 1));
      L[(size_t)j * n + k] = dpow[j] * sjk;                  // (D S)[j][k]
      R[(size_t)k * n + j] = sjk / dpow[j];                  // (S D^-1)[k][j]
    }
  return true;
}

// The same for A = diff T_N on an axis with a zero normal derivative at x = 1: T_N is the
// second difference whose last row, through the mirror ghost, reads [.., 2, -2] (just -2
// for n = 1). With D = diag(1, .., 1, 1/sqrt(2)), D T_N D^-1 is symmetric, with the
// orthonormal eigenvectors Q[j][k] = sqrt(2/n) D_jj sin((2k+1)(j+1) pi/(2n)) (the
// sine modes that vanish at x = 0 and are flat at x = 1) and the eigenvalues
// -4 sin^2((2k+1) pi/(4n)). Hence A = L diag(ev) R with L = D^-1 Q and R = Q^T D.
void eigen_closed_form_neumann(int n, double diff, std::vector<double>& ev, std::vector<double>& R,
                               std::vector<double>& L) {
  const double pi = 3.14159265358979323846;
  const double c = std::sqrt(2.0 / n);
  const int64_t per = 4 * (int64_t)n;                    // sin(m pi/(2n)) has period 4n in m
  ev.resize(n);
  R.resize((size_t)n * n);
  L.resize((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    const double h = std::sin((2 * k + 1) * pi / (4.0 * n));
    ev[k] = -4.0 * diff * h * h;
  }
  for (int j = 0; j < n; ++j) {
    const double w = (j == n - 1) ? std::sqrt(0.5) : 1.0;   // D_jj
    for (int k = 0; k < n; ++k) {
      const int64_t m = ((int64_t)(2 * k + 1) * (j + 1)) % per;   // exact argument reduction
      const double q = c * w * std::sin(m * pi / (2.0 * n));
      L[(size_t)j * n + k] = q / w;                             // (D^-1 Q)[j][k]
      R[(size_t)k * n + j] = q * w;                             // (Q^T D)[k][j]
    }
  }
}

// MM_SLICED Lawson steps: the first stencil pass writes its stage vectors (nvec of them,
// stacked as operand rows) straight into the digit workspace of the mode-1 product, so
// that product skips its split pass. Needs rows that one stencil wave covers.
bool stencil_digits(const mm_op* op) {
  return op->prec == MM_SLICED && !op->periodic && stencil_row_in_one_wave(op->n[0]);
}

void set_stencil_digits(StencilArgs& a, const mm_op* op, signed char* dig, int* dexp, int nvec) {
  const int64_t rows = op->dof / op->n[0];   // operand rows of one stage vector
  a.dig = dig;
  a.dexp = dexp;
  a.dS = op->slices;
  a.dplane = rows * nvec * slice_ld(op->n[0]);
  a.drow1 = nvec > 1 ? rows : 0;
  a.out0 = nullptr;
  a.out1 = nullptr;
}

// MM_SLICED Lawson-Euler / Lawson2b on finite-difference grids whose axes all fit one
// chained workgroup's 256 fibers: the exp action can run as chained mode products (the
// stencil writes the first product's digits, every product but the last writes the
// next one's). Decided at setup (it needs the second digit workspace).
bool chain_capable(const mm_op* op) {
  if (!stencil_digits(op) || op->family != MM_LAWSON ||
      (op->scheme != MM_LAWSON_EULER && op->scheme != MM_LAWSON2B))
    return false;
  for (int mu = 0; mu < op->d; ++mu)
    if (op->n[mu] > 256) return false;
  return true;
}

// whether this op's Lawson steps take the chained action under the context's mode
bool chain_active(const mm_op* op) {
  const int mode = op->ctx ? op->ctx->sliced_chain : 0;
  if (mode == 0 || !op->vdig2 || !chain_capable(op)) return false;
  if (mode == 1)
    for (int mu = 0; mu < op->d; ++mu)
      if (op->n[mu] <= 128) return false;
  return true;
}

// out = exp(tau A) v for the nvec stage vectors whose digit planes and fiber exponents the
// stencil wrote into op->vdig / op->vexp (chain layout, groups of n2 fibers). Product mu contracts
// axis mu; its fiber groups run along the next axis (F = n_(mu+1), Gv = dof / (n_mu F)
// groups per vector), and its output rows are the next product's fibers, written to the
// other workspace. The last product writes FP64 into out (layout lo).
hipError_t chain_action(const mm_op* op, int j, int nvec, double* out, Layout lo, hipStream_t s) {
  signed char* dig[2] = {op->vdig, op->vdig2};
  int* ex[2] = {op->vexp, op->vexp2};
  const int64_t dcap[2] = {op->vdig_len, op->vdig2_len}, ecap[2] = {op->vexp_len, op->vexp2_len};
  const int mode = op->ctx->sliced_chain;
  for (int mu = 0; mu < op->d; ++mu) {
    const int cur = mu & 1;
    const int n = op->n[mu], nf = op->n[(mu + 1) % op->d];
    ChainArgs c{};
    c.fdig = (const signed char*)factor_op(op, mu, j);
    c.fexp = factor_exp(op, mu, j);
    c.fplane = factor_slice_stride(op, n, n);
    c.vdig = dig[cur];
    c.vexp = ex[cur];
    c.vcap = dcap[cur];
    c.vexp_cap = ecap[cur];
    c.M = c.K = n;
    c.F = nf;
    c.Gv = (int)(op->dof / ((int64_t)n * nf));
    c.nvec = nvec;
    c.slices = op->slices;
    c.wide = mode == 3;
    if (mu + 1 < op->d) {
      c.odig = dig[cur ^ 1];
      c.oexp = ex[cur ^ 1];
      c.ocap = dcap[cur ^ 1];
      c.oexp_cap = ecap[cur ^ 1];
      c.Fn = op->n[(mu + 2) % op->d];   // the next product's fibers per group
    } else {
      c.out = out;
      c.ldo = lo.ld;
      c.ovs = lo.vs;
    }
    const double work = 2.0 * n * (double)op->dof * nvec;
    const hipError_t e = timed_launch(op->ctx, mu == 0 ? MM_KIND_GEMM_K : MM_KIND_GEMM_N, work, s,
                                      [&] { return launch_gemm_sliced_chain(c, s); });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}


mm_status check_op(mm_ctx* ctx, const mm_op* op) {
  if (!ctx) return MM_EINVAL;
  if (!op) {
    set_err(ctx, "null op");
    return MM_EINVAL;
  }
  if (op->ctx != ctx) {
    set_err(ctx, "op belongs to another context");
    return MM_EINVAL;
  }
  return MM_OK;
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

const char* mm_version(void) { return "mumode-gfx950 1.0"; }

mm_status mm_ctx_create(int device, mm_ctx** out) {
  if (!out) return MM_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MM_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return MM_EDEVICE;
  mm_ctx* ctx = new mm_ctx();
  ctx->device = device;
  if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return MM_EDEVICE;
  }
  // keep freed pool memory for reuse instead of returning it to the driver
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t keep = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  // the device address of the allocation-free entry point's scratch array, on this device
  if (noalloc_resolve(device) != hipSuccess) {
    hipStreamDestroy(ctx->stream);
    delete ctx;
    return MM_EDEVICE;
  }
  ctx->reduce_parts = 1024;
  if (hipMalloc((void**)&ctx->reduce_buf, (ctx->reduce_parts + 1) * sizeof(double)) != hipSuccess) {
    hipStreamDestroy(ctx->stream);
    delete ctx;
    return MM_ENOMEM;
  }
  *out = ctx;
  return MM_OK;
}

void mm_ctx_destroy(mm_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  if (!ctx->bws.empty()) {
    // grouped sliced workspaces: their streams' work must be over before the release
    hipDeviceSynchronize();
    for (auto& w : ctx->bws) {
      if (w.vdig) hipFreeAsync(w.vdig, ctx->stream);
      if (w.vexp) hipFreeAsync(w.vexp, ctx->stream);
    }
  }
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  if (ctx->reduce_buf) hipFree(ctx->reduce_buf);
  for (auto& t : ctx->timed) {
    hipEventDestroy(t.start);
    hipEventDestroy(t.stop);
  }
  if (ctx->stream) hipStreamDestroy(ctx->stream);
  if (ctx->capture) hipStreamDestroy(ctx->capture);
  delete ctx;
}

const char* mm_last_error(const mm_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->last_error.c_str();
}

void mumode_destroy(mm_op* op) {
  if (!op) return;
  if (!op->ctx) {
    delete op;
    return;
  }
  hipSetDevice(op->ctx->device);
  dev_free(op, op->a);
  for (size_t i = 0; i < op->fac.size(); ++i)
    if (op->fac_owned[i]) dev_free(op, op->fac[i]);
  for (size_t i = 0; i < op->ffold.size(); ++i)
    if (op->ffold_owned[i]) dev_free(op, op->ffold[i]);
  dev_free(op, op->f3_stage1);
  dev_free(op, op->f3_stage2);
  dev_free(op, op->f3_phi);
  dev_free(op, op->f3_stage1_fold);
  dev_free(op, op->f3_stage2_fold);
  dev_free(op, op->f3_phi_fold);
  for (size_t i = 0; i < op->fac_lp.size(); ++i)
    if (op->fac_owned[i]) dev_free(op, op->fac_lp[i]);
  dev_free(op, op->f3_stage1_lp);
  dev_free(op, op->f3_stage2_lp);
  dev_free(op, op->f3_phi_lp);
  for (size_t i = 0; i < op->fac_exp.size(); ++i)
    if (op->fac_owned[i]) dev_free(op, op->fac_exp[i]);
  dev_free(op, op->f3_stage1_exp);
  dev_free(op, op->f3_stage2_exp);
  dev_free(op, op->f3_phi_exp);
  for (int mu = 0; mu < 3; ++mu) dev_free(op, op->ev[mu]);
  for (int mu = 0; mu < 3; ++mu)
    if (op->dmat_owned[mu]) dev_free(op, op->dmat[mu]);
  dev_free(op, op->vel);
  dev_free(op, op->spec_ws);
  for (int i = 0; i < 2; ++i) {
    if (op->spec_side[i]) hipStreamDestroy(op->spec_side[i]);
    if (op->spec_join[i]) hipEventDestroy(op->spec_join[i]);
  }
  if (op->spec_fork) hipEventDestroy(op->spec_fork);
  for (int i = 0; i < 6; ++i) dev_free(op, op->buf[i]);
  dev_free(op, op->vdig);
  dev_free(op, op->vexp);
  dev_free(op, op->vdig2);
  dev_free(op, op->vexp2);
  dev_free(op, op->flag);
  if (op->gexec) hipGraphExecDestroy(op->gexec);
  delete op;
}

mm_status mumode_setup(mm_ctx* ctx, const mm_problem* prob, double tau, int family, int scheme,
                       int quad_nodes, int prec, int slices, mm_op** out) {
  if (!ctx) return MM_EINVAL;
  if (!prob || !out) {
    set_err(ctx, "null problem or output pointer");
    return MM_EINVAL;
  }
  *out = nullptr;
  if (prob->d != 2 && prob->d != 3) {
    set_err(ctx, "d must be 2 or 3 (got %d)", prob->d);
    return MM_EINVAL;
  }
  for (int mu = 0; mu < prob->d; ++mu)
    if (prob->n[mu] < 1 || prob->n[mu] > 4096) {
      set_err(ctx, "n[%d] = %d out of range 1..4096", mu, prob->n[mu]);
      return MM_EINVAL;
    }
  if (!(tau > 0.0) || !std::isfinite(tau)) {
    set_err(ctx, "tau must be finite and positive");
    return MM_EINVAL;
  }
  if (!prob->a) {
    set_err(ctx, "null diffusion coefficient");
    return MM_EINVAL;
  }
  for (int mu = 0; mu < prob->d; ++mu)
    if (prob->bc[mu] != MM_BC_DIRICHLET && prob->bc[mu] != MM_BC_NEUMANN && prob->bc[mu] != MM_BC_PERIODIC) {
      set_err(ctx, "bc[%d] = %d is not a boundary type", mu, prob->bc[mu]);
      return MM_EINVAL;
    }
  const bool periodic = prob->bc[0] == MM_BC_PERIODIC;
  for (int mu = 0; mu < prob->d; ++mu) {
    if ((prob->bc[mu] == MM_BC_PERIODIC) != periodic) {
      set_err(ctx, "periodic axes cannot be mixed with Dirichlet or Neumann axes");
      return MM_EINVAL;
    }
    if (periodic && !(prob->length[mu] > 0.0 && std::isfinite(prob->length[mu]))) {
      set_err(ctx, "length[%d] must be finite and positive for a periodic axis", mu);
      return MM_EINVAL;
    }
  }
  if (prob->form != MM_FORM_FLUX && prob->form != MM_FORM_NONDIV) {
    set_err(ctx, "form = %d is not a diffusion form", prob->form);
    return MM_EINVAL;
  }
  if (family != MM_LAWSON && family != MM_ERK) {
    set_err(ctx, "unknown family %d", family);
    return MM_EINVAL;
  }
  if (family == MM_LAWSON && (scheme < MM_LAWSON_EULER || scheme > MM_SL2)) {
    set_err(ctx, "unknown Lawson scheme %d", scheme);
    return MM_EINVAL;
  }
  if (family == MM_ERK && scheme != MM_ETD2RK && scheme != MM_ERK2P1 && scheme != MM_EE && scheme != MM_ERK2P2) {
    set_err(ctx, "unknown ERK scheme %d", scheme);
    return MM_EINVAL;
  }
  if (family == MM_ERK && (scheme == MM_EE || scheme == MM_ERK2P2) && quad_nodes != 0) {
    set_err(ctx, "exponential Euler and ERK2 with phi2 need exact phi functions (quad_nodes = 0)");
    return MM_EINVAL;
  }
  if (family == MM_ERK && (quad_nodes < 0 || quad_nodes > kMaxGroups - 1)) {
    set_err(ctx, "quad_nodes must be 0 (exact phi1) or 1..%d", kMaxGroups - 1);
    return MM_EINVAL;
  }
  if (family == MM_ERK && quad_nodes == 0 && prec != MM_FP64) {
    set_err(ctx, "exact phi1 (quad_nodes = 0) is FP64 only");
    return MM_EINVAL;
  }
  if (family == MM_ERK && quad_nodes == 0)
    for (int mu = 0; mu < prob->d; ++mu)
      if (prob->bc[mu] == MM_BC_NEUMANN && prob->beta_bar[mu] != 0.0) {
        set_err(ctx, "exact phi1 (quad_nodes = 0) on an axis with a zero normal derivative needs beta_bar = 0 there "
                     "(closed-form eigenbasis)");
        return MM_EINVAL;
      }
  if (prec < MM_FP64 || prec > MM_SLICED) {
    set_err(ctx, "unknown precision %d", prec);
    return MM_EINVAL;
  }
  if (prec == MM_SLICED && slices != 0 && (slices < kMinSlices || slices > kMaxSlices)) {
    set_err(ctx, "slices must be 0 or %d..%d", kMinSlices, kMaxSlices);
    return MM_EINVAL;
  }
  if (prec == MM_SLICED) {
    // exact int32 level sums need S * 2^14 * K < 2^31 for every contraction length K
    int64_t kmax = 0;
    for (int mu = 0; mu < prob->d; ++mu) kmax = std::max<int64_t>(kmax, prob->n[mu]);
    if (family == MM_ERK) kmax = std::max<int64_t>(kmax, (int64_t)(quad_nodes + 1) * prob->n[prob->d - 1]);
    const int S = slices ? slices : kDefaultSlices;
    if (kmax * S * 16384 >= ((int64_t)1 << 31)) {
      set_err(ctx, "contraction length %lld too long for exact %d-digit slicing", (long long)kmax, S);
      return MM_EINVAL;
    }
  }
  if (!std::isfinite(prob->lambda) || prob->lambda < 0.0) {
    set_err(ctx, "lambda must be finite and >= 0");
    return MM_EINVAL;
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;

  mm_op* op = new mm_op();
  op->ctx = ctx;
  op->d = prob->d;
  for (int mu = 0; mu < 3; ++mu) {
    op->n[mu] = (mu < prob->d) ? prob->n[mu] : 1;
    op->beta[mu] = (mu < prob->d) ? prob->beta[mu] : 0.0;
    op->beta_bar[mu] = (mu < prob->d) ? prob->beta_bar[mu] : 0.0;
    op->bc[mu] = (mu < prob->d) ? prob->bc[mu] : MM_BC_DIRICHLET;
  }
  op->form = prob->form;
  op->periodic = periodic;
  for (int mu = 0; mu < 3; ++mu) op->length[mu] = (periodic && mu < prob->d) ? prob->length[mu] : 0.0;
  for (int i = 0; i < 4; ++i) op->r[i] = prob->r[i];
  op->lam = prob->lambda;
  op->tau = tau;
  op->family = family;
  op->scheme = scheme;
  op->q = (family == MM_ERK) ? quad_nodes : 0;
  op->exact = (family == MM_ERK && quad_nodes == 0);
  op->prec = prec;
  op->slices = (prec == MM_SLICED) ? (slices ? slices : kDefaultSlices) : 0;
  op->dof = (int64_t)op->n[0] * op->n[1] * op->n[2];
  int64_t na = 1;
  for (int mu = 0; mu < op->d; ++mu) na *= op->n[mu] + 2;
  if (periodic) na = op->d * op->dof;   // the d diagonal diffusion fields

  auto fail = [&](mm_status s) {
    mumode_destroy(op);
    return s;
  };
  mm_status rc;
  if ((rc = dev_alloc(op, &op->a, na)) != MM_OK) return fail(rc);
  if (hipMemcpyAsync(op->a, prob->a, na * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess) {
    set_err(ctx, "copy of the diffusion coefficient failed (device pointer expected)");
    return fail(MM_EINVAL);
  }
  if ((rc = dev_alloc(op, &op->flag, 1)) != MM_OK) return fail(rc);
  if (hipMemsetAsync(op->flag, 0, sizeof(int), st) != hipSuccess) return fail(MM_EDEVICE);
  if (periodic && prob->velocity) {
    if ((rc = dev_alloc(op, &op->vel, op->d * op->dof)) != MM_OK) return fail(rc);
    if (hipMemcpyAsync(op->vel, prob->velocity, op->d * op->dof * sizeof(double), hipMemcpyDeviceToDevice, st) !=
        hipSuccess) {
      set_err(ctx, "copy of the velocity field failed (device pointer expected)");
      return fail(MM_EINVAL);
    }
  }

  // a_max = max over all nodes (eq. (eq:amaxbeta)); periodic problems: the maximum of each
  // diagonal entry a_mumu of the diffusion tensor
  const int nred = periodic ? op->d : 1;
  const int64_t lred = periodic ? op->dof : na;
  double amax = 0.0;
  for (int i = 0; i < nred; ++i) {
    double m = 0.0;
    if (launch_max_reduce(op->a + i * lred, lred, ctx->reduce_buf, ctx->reduce_parts,
                          ctx->reduce_buf + ctx->reduce_parts, st) != hipSuccess ||
        hipMemcpyAsync(&m, ctx->reduce_buf + ctx->reduce_parts, sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_err(ctx, "a_max reduction failed");
      return fail(MM_EDEVICE);
    }
    if (!std::isfinite(m)) {
      set_err(ctx, "diffusion coefficient is not finite");
      return fail(MM_EINVAL);
    }
    op->amax_mu[i] = m;
    amax = (i == 0) ? m : std::max(amax, m);
  }
  if (!periodic)
    for (int mu = 0; mu < 3; ++mu) op->amax_mu[mu] = amax;
  op->a_max = amax;

  // coefficients c of the factors exp(c tau A_mu): c_0 = 1, c_j = theta_j
  // Pade factors exp(c tau A_mu) for c = 1 and the quadrature nodes; the exact-phi1 mode
  // stores two more per axis, the eigenvector matrices R and L (A_mu = L diag(ev) R)
  int nf = 1 + op->q;
  double cs[kMaxGroups];
  cs[0] = 1.0;
  if (op->q > 0) {
    gauss_legendre(op->q, op->theta + 1, op->weight + 1);
    for (int j = 1; j <= op->q; ++j) cs[j] = op->theta[j];
  }
  // Lawson2a uses exp(tau A / 2) too; stabilized Lawson2 exp(tau A / 2) and exp(alpha tau A)
  if (family == MM_LAWSON && (scheme == MM_LAWSON2A || scheme == MM_SL2)) {
    cs[nf++] = 0.5;
    if (scheme == MM_SL2) cs[nf++] = kAlphaSL2;
    for (int j = 1; j < nf; ++j) op->theta[j] = cs[j];
  }
  op->nfac = op->exact ? 3 : nf;
  op->theta[0] = 1.0;
  op->weight[0] = 1.0;

  int nmax = 0;
  for (int mu = 0; mu < op->d; ++mu) nmax = std::max(nmax, op->n[mu]);
  double* ws = nullptr;
  if (hipMallocAsync((void**)&ws, (size_t)7 * nmax * nmax * sizeof(double), st) != hipSuccess) {
    set_err(ctx, "Pade workspace allocation failed");
    return fail(MM_ENOMEM);
  }
  op->fac.assign(op->d, nullptr);
  op->fac_owned.assign(op->d, false);
  for (int mu = 0; mu < op->d; ++mu) {
    int same = -1;
    for (int nu = 0; nu < mu; ++nu)
      if (op->n[nu] == op->n[mu] && op->beta_bar[nu] == op->beta_bar[mu] && op->bc[nu] == op->bc[mu] &&
          op->length[nu] == op->length[mu] && op->amax_mu[nu] == op->amax_mu[mu])
        same = nu;
    if (same >= 0) {
      op->fac[mu] = op->fac[same];
      op->squarings[mu] = op->squarings[same];
      continue;
    }
    const int n = op->n[mu];
    if ((rc = dev_alloc(op, &op->fac[mu], (int64_t)op->nfac * n * n)) != MM_OK) {
      hipFreeAsync(ws, st);
      return fail(rc);
    }
    op->fac_owned[mu] = true;
    if (periodic) {
      // exp(c tau A_mu) is circulant: its first column from the symbol of A_mu
      const double kap = 2.0 * M_PI / op->length[mu];
      const long double la = (long double)op->lam * op->amax_mu[mu], bb = op->beta_bar[mu];
      for (int j = 0; j < nf; ++j) {
        const long double ct = (long double)cs[j] * tau;
        std::vector<double> col = circulant_column(n, [&](int m, bool nyq) {
          const long double k = (long double)kap * m;
          const long double re = -la * k * k, im = nyq ? 0.0L : bb * k;
          const long double mag = std::exp(ct * re);
          return std::complex<long double>(mag * std::cos(ct * im), mag * std::sin(ct * im));
        });
        if (hipMemcpyAsync(ws, col.data(), n * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
            launch_build_circulant(op->fac[mu] + (int64_t)j * n * n, n, ws, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
          hipFreeAsync(ws, st);
          set_err(ctx, "circulant factor setup failed");
          return fail(MM_EDEVICE);
        }
      }
      continue;
    }
    const double h = mesh_h(op, mu);
    const double diff = op->lam * op->a_max / (h * h);
    const double adv = op->beta_bar[mu] / (2.0 * h);
    if (op->bc[mu] == MM_BC_DIRICHLET && adv == 0.0) {
      // symmetric A_mu: exp(c tau A_mu) = S diag(exp(c tau ev)) S with the orthogonal sine
      // matrix S (closed form, no squarings): one FP64 product per factor, accurate to
      // rounding however stiff c tau A_mu is -- scaling and squaring doubles the error of
      // the scaled exponential with every squaring (about 2^s u relative)
      std::vector<double> ev, Sm, Lm;
      eigen_closed_form(n, diff, -2.0 * diff, diff, ev, Sm, Lm);
      const int64_t nn = (int64_t)n * n;
      std::vector<double> W((size_t)nn);
      bool ok = hipMemcpy(ws, Sm.data(), nn * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
      for (int j = 0; j < nf && ok; ++j) {
        const double ct = cs[j] * tau;
        std::vector<double> w(n);
        for (int k = 0; k < n; ++k) w[k] = std::exp(ct * ev[k]);
        for (int r = 0; r < n; ++r)
          for (int k = 0; k < n; ++k) W[(size_t)r * n + k] = Sm[(size_t)r * n + k] * w[k];
        ok = hipMemcpy(ws + nn, W.data(), nn * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
             gemm_sq(n, ws + nn, ws, op->fac[mu] + (int64_t)j * nn, st) == hipSuccess &&
             hipStreamSynchronize(st) == hipSuccess;
      }
      if (!ok) {
        hipFreeAsync(ws, st);
        set_err(ctx, "closed-form factor setup failed");
        return fail(MM_EDEVICE);
      }
      op->squarings[mu] = 0;
      continue;
    }
    for (int j = 0; j < nf; ++j) {
      const double ct = cs[j] * tau;
      int sq = 0;
      rc = pade_expm(ctx, n, ct * (diff - adv), ct * (-2.0 * diff), ct * (diff + adv), op->bc[mu] == MM_BC_NEUMANN,
                     op->fac[mu] + (int64_t)j * n * n, &sq, ws);
      if (rc != MM_OK) {
        hipFreeAsync(ws, st);
        return fail(rc);
      }
      if (j == 0) op->squarings[mu] = sq;
    }
  }
  if (periodic) {
    // per axis [D1 | D2 | A_mu]: the Fourier derivatives and the extracted operator
    for (int mu = 0; mu < op->d; ++mu) {
      int same = -1;
      for (int nu = 0; nu < mu; ++nu)
        if (op->n[nu] == op->n[mu] && op->beta_bar[nu] == op->beta_bar[mu] && op->length[nu] == op->length[mu] &&
            op->amax_mu[nu] == op->amax_mu[mu])
          same = nu;
      if (same >= 0) {
        op->dmat[mu] = op->dmat[same];
        continue;
      }
      const int n = op->n[mu];
      const int64_t nn = (int64_t)n * n;
      if ((rc = dev_alloc(op, &op->dmat[mu], 3 * nn)) != MM_OK) {
        hipFreeAsync(ws, st);
        return fail(rc);
      }
      op->dmat_owned[mu] = true;
      const long double kap = 2.0L * (long double)M_PI / op->length[mu];
      const long double la = (long double)op->lam * op->amax_mu[mu], bb = op->beta_bar[mu];
      typedef std::complex<long double> cl;
      const std::vector<double> cols[3] = {
          circulant_column(n, [&](int m, bool nyq) { return cl(0.0L, nyq ? 0.0L : kap * m); }),
          circulant_column(n, [&](int m, bool) { return cl(-(kap * m) * (kap * m), 0.0L); }),
          circulant_column(n, [&](int m, bool nyq) { return cl(-la * (kap * m) * (kap * m), nyq ? 0.0L : bb * kap * m); })};
      for (int k = 0; k < 3; ++k)
        if (hipMemcpyAsync(ws, cols[k].data(), n * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
            launch_build_circulant(op->dmat[mu] + k * nn, n, ws, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
          hipFreeAsync(ws, st);
          set_err(ctx, "circulant derivative setup failed");
          return fail(MM_EDEVICE);
        }
    }
    if ((rc = dev_alloc(op, &op->spec_ws, 3 * (int64_t)op->d * op->dof)) != MM_OK) {
      hipFreeAsync(ws, st);
      return fail(rc);
    }
    for (int mu = 1; mu < op->d; ++mu)
      if (hipStreamCreateWithFlags(&op->spec_side[mu - 1], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&op->spec_join[mu - 1], hipEventDisableTiming) != hipSuccess) {
        hipFreeAsync(ws, st);
        set_err(ctx, "stream or event creation failed");
        return fail(MM_EDEVICE);
      }
    if (op->d > 1 && hipEventCreateWithFlags(&op->spec_fork, hipEventDisableTiming) != hipSuccess) {
      hipFreeAsync(ws, st);
      set_err(ctx, "event creation failed");
      return fail(MM_EDEVICE);
    }
  }
  hipFreeAsync(ws, st);
  if (hipStreamSynchronize(st) != hipSuccess) {
    set_err(ctx, "factor setup failed on the device");
    return fail(MM_EDEVICE);
  }
  if (op->exact && periodic) {
    // real orthonormal Fourier basis of every axis (R = Q^T, L = Q, uploaded next to E(1))
    // and the symbol of A_mu at the wavenumbers 0 .. n/2
    for (int mu = 0; mu < op->d; ++mu) {
      const int n = op->n[mu];
      const int64_t nn = (int64_t)n * n;
      std::vector<double> R((size_t)nn), L((size_t)nn), sym(2 * (n / 2 + 1));
      fourier_basis(n, L);
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) R[(size_t)k * n + j] = L[(size_t)j * n + k];
      const long double kap = 2.0L * 3.141592653589793238462643383279502884L / op->length[mu];
      for (int m = 0; m <= n / 2; ++m) {
        const long double km = kap * m;
        sym[2 * m] = (double)(-(long double)op->lam * op->amax_mu[mu] * km * km);
        sym[2 * m + 1] = (n % 2 == 0 && m == n / 2) ? 0.0 : (double)((long double)op->beta_bar[mu] * km);
      }
      if ((rc = dev_alloc(op, &op->ev[mu], (int64_t)sym.size())) != MM_OK) return fail(rc);
      if (hipMemcpy(op->ev[mu], sym.data(), sym.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
          (op->fac_owned[mu] &&
           (hipMemcpy(op->fac[mu] + nn, R.data(), nn * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(op->fac[mu] + 2 * nn, L.data(), nn * sizeof(double), hipMemcpyHostToDevice) != hipSuccess))) {
        set_err(ctx, "upload of the Fourier basis failed");
        return fail(MM_EDEVICE);
      }
    }
  } else if (op->exact) {
    // closed-form eigen-decomposition of every 1D operator (uploaded next to E(1))
    for (int mu = 0; mu < op->d; ++mu) {
      const int n = op->n[mu];
      const double h = mesh_h(op, mu);
      const double diff = op->lam * op->a_max / (h * h);
      const double adv = op->beta_bar[mu] / (2.0 * h);
      std::vector<double> ev, R, L;
      if (op->bc[mu] == MM_BC_NEUMANN)
        eigen_closed_form_neumann(n, diff, ev, R, L);   // beta_bar = 0 there (checked)
      else if (!eigen_closed_form(n, diff - adv, -2.0 * diff, diff + adv, ev, R, L)) {
        set_err(ctx, "exact phi1 needs |beta_bar| h < 2 lambda a_max on every axis (real eigenvalues)");
        return fail(MM_EINVAL);
      }
      if ((rc = dev_alloc(op, &op->ev[mu], n)) != MM_OK) return fail(rc);
      const int64_t nn = (int64_t)n * n;
      if (hipMemcpy(op->ev[mu], ev.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
          (op->fac_owned[mu] &&
           (hipMemcpy(op->fac[mu] + nn, R.data(), nn * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(op->fac[mu] + 2 * nn, L.data(), nn * sizeof(double), hipMemcpyHostToDevice) != hipSuccess))) {
        set_err(ctx, "upload of the eigen-decomposition failed");
        return fail(MM_EDEVICE);
      }
    }
  }
  // other precisions: FP32, BF16-slice or digit-plane forms with zero-padded rows
  op->fac_lp.assign(op->d, nullptr);
  op->fac_exp.assign(op->d, nullptr);
  // convert `rows` x k (row stride lds) FP64 into the op's factor format at dst (exps:
  // per-row exponents for MM_SLICED)
  auto convert = [&](void* dst, int* exps, const double* src, int rows, int k, int lds) -> hipError_t {
    if (prec == MM_SLICED)
      return launch_slice_rows((signed char*)dst, exps, src, rows, k, lds, slice_ld(k), op->slices, st);
    return launch_convert_factor(prec, dst, src, rows, k, lds, st);
  };
  // bytes of a rows x k factor operand in the op's format
  auto op_bytes = [&](int rows, int k) -> int64_t {
    if (prec == MM_SLICED) return (int64_t)rows * slice_ld(k) * op->slices;
    if (prec == MM_FP32) return (int64_t)rows * fac_ld(k) * 4;
    return (int64_t)rows * fac_ld(k) * 2 * factor_slices(prec);
  };
  if (prec != MM_FP64) {
    for (int mu = 0; mu < op->d; ++mu) {
      if (!op->fac_owned[mu]) {
        for (int nu = 0; nu < mu; ++nu)
          if (op->fac[nu] == op->fac[mu]) {
            op->fac_lp[mu] = op->fac_lp[nu];
            op->fac_exp[mu] = op->fac_exp[nu];
          }
        continue;
      }
      const int n = op->n[mu];
      const int64_t per = op_bytes(n, n);
      char* dst = nullptr;
      if ((rc = dev_alloc(op, &dst, nf * per)) != MM_OK) return fail(rc);
      op->fac_lp[mu] = dst;
      if (prec == MM_SLICED && (rc = dev_alloc(op, &op->fac_exp[mu], (int64_t)nf * n)) != MM_OK) return fail(rc);
      for (int j = 0; j < nf; ++j)
        HIPCHK(ctx, convert(dst + j * per, prec == MM_SLICED ? op->fac_exp[mu] + j * n : nullptr,
                            op->fac[mu] + (int64_t)j * n * n, n, n, n));
    }
  }

  // FP64 axes whose operator is a symmetric Toeplitz matrix (zero Dirichlet data at both
  // ends, no advection moved into A): every exp(c tau A_mu) is centrosymmetric, and the
  // mode products of the exp actions can run folded, at half the multiply-adds
  op->ffold.assign(op->d, nullptr);
  op->ffold_owned.assign(op->d, false);
  op->nfold = nf;
  if (prec == MM_FP64 && !periodic) {
    for (int mu = 0; mu < op->d; ++mu) {
      if (op->bc[mu] != MM_BC_DIRICHLET || op->beta_bar[mu] != 0.0) continue;
      int same = -1;
      for (int nu = 0; nu < mu; ++nu)
        if (op->fac[nu] == op->fac[mu] && op->ffold[nu]) same = nu;
      if (same >= 0) {
        op->ffold[mu] = op->ffold[same];
        continue;
      }
      const int n = op->n[mu], f = n - n / 2;
      if ((rc = dev_alloc(op, &op->ffold[mu], (int64_t)nf * 2 * f * fold_ld(n))) != MM_OK) return fail(rc);
      op->ffold_owned[mu] = true;
      HIPCHK(ctx, launch_fold_factor(op->ffold[mu], op->fac[mu], n, nf, st));
    }
  }

  const int la = last_axis(op);
  const int nl = op->n[la];
  const int64_t dof = op->dof;
  if (family == MM_ERK && op->exact) {
    // buffers: 0 [u, g0] (or [-, F0]), 1 and 2 pairs of scratch, 3 U, 4 D, 5 F0
    const int64_t lens[6] = {2 * dof, 2 * dof, 2 * dof, dof, dof, scheme != MM_ETD2RK ? dof : 0};
    for (int i = 0; i < 6; ++i) {
      op->buf_len[i] = lens[i];
      if (lens[i] > 0 && (rc = dev_alloc(op, &op->buf[i], lens[i])) != MM_OK) return fail(rc);
    }
  } else if (family == MM_ERK) {
    const int q = op->q;
    // stage 1: ETD2RK [E(1) | tau w_j E(theta_j)], ERK2P1 [tau w_j E(theta_j)]
    const int g1 = (scheme == MM_ETD2RK) ? q + 1 : q;
    if ((rc = dev_alloc(op, &op->f3_stage1, (int64_t)nl * g1 * nl)) != MM_OK) return fail(rc);
    if ((rc = dev_alloc(op, &op->f3_stage2, (int64_t)nl * q * nl)) != MM_OK) return fail(rc);
    if ((rc = dev_alloc(op, &op->f3_phi, (int64_t)nl * q * nl)) != MM_OK) return fail(rc);
    int col = 0;
    if (scheme == MM_ETD2RK) {
      HIPCHK(ctx, launch_place_scaled(op->f3_stage1, g1 * nl, 0, factor(op, la, 0), nl, 1.0, st));
      col = nl;
    }
    // sliced mode: unweighted blocks (the weights scale the first pass instead)
    const bool unit = prec == MM_SLICED;
    for (int j = 1; j <= q; ++j) {
      HIPCHK(ctx, launch_place_scaled(op->f3_stage1, g1 * nl, col + (j - 1) * nl, factor(op, la, j), nl,
                                      unit ? 1.0 : tau * op->weight[j], st));
      HIPCHK(ctx, launch_place_scaled(op->f3_stage2, q * nl, (j - 1) * nl, factor(op, la, j), nl,
                                      unit ? 1.0 : 0.5 * tau * op->weight[j], st));
      HIPCHK(ctx, launch_place_scaled(op->f3_phi, q * nl, (j - 1) * nl, factor(op, la, j), nl,
                                      unit ? 1.0 : op->weight[j], st));
    }
    // the stacked factors' blocks are weighted exp factors of the last axis: they fold
    // where that axis's factors do
    if (prec == MM_FP64 && op->ffold[la]) {
      const int64_t fb = (int64_t)2 * (nl - nl / 2) * fold_ld(nl);
      if ((rc = dev_alloc(op, &op->f3_stage1_fold, fb * g1)) != MM_OK) return fail(rc);
      if ((rc = dev_alloc(op, &op->f3_stage2_fold, fb * q)) != MM_OK) return fail(rc);
      if ((rc = dev_alloc(op, &op->f3_phi_fold, fb * q)) != MM_OK) return fail(rc);
      HIPCHK(ctx, launch_fold_stacked(op->f3_stage1_fold, op->f3_stage1, nl, g1, st));
      HIPCHK(ctx, launch_fold_stacked(op->f3_stage2_fold, op->f3_stage2, nl, q, st));
      HIPCHK(ctx, launch_fold_stacked(op->f3_phi_fold, op->f3_phi, nl, q, st));
    }
    if (prec != MM_FP64) {
      const int64_t s1 = op_bytes(nl, g1 * nl), s2 = op_bytes(nl, q * nl);
      char *d1 = nullptr, *d2 = nullptr, *d3 = nullptr;
      if ((rc = dev_alloc(op, &d1, s1)) != MM_OK) return fail(rc);
      op->f3_stage1_lp = d1;
      if ((rc = dev_alloc(op, &d2, s2)) != MM_OK) return fail(rc);
      op->f3_stage2_lp = d2;
      if ((rc = dev_alloc(op, &d3, s2)) != MM_OK) return fail(rc);
      op->f3_phi_lp = d3;
      if (prec == MM_SLICED) {
        if ((rc = dev_alloc(op, &op->f3_stage1_exp, nl)) != MM_OK) return fail(rc);
        if ((rc = dev_alloc(op, &op->f3_stage2_exp, nl)) != MM_OK) return fail(rc);
        if ((rc = dev_alloc(op, &op->f3_phi_exp, nl)) != MM_OK) return fail(rc);
      }
      HIPCHK(ctx, convert(d1, op->f3_stage1_exp, op->f3_stage1, nl, g1 * nl, g1 * nl));
      HIPCHK(ctx, convert(d2, op->f3_stage2_exp, op->f3_stage2, nl, q * nl, q * nl));
      HIPCHK(ctx, convert(d3, op->f3_phi_exp, op->f3_phi, nl, q * nl, q * nl));
    }
    // buffers: 0 g0, 1 T1 ((q+1) dof), 2 T2 ((q+1) dof), 3 U, 4 D, 5 F0 (ERK2P1)
    const int64_t lens[6] = {dof, (q + 1) * dof, (q + 1) * dof, dof, dof, scheme == MM_ERK2P1 ? dof : 0};
    for (int i = 0; i < 6; ++i) {
      op->buf_len[i] = lens[i];
      if (lens[i] > 0 && (rc = dev_alloc(op, &op->buf[i], lens[i])) != MM_OK) return fail(rc);
    }
  } else {
    // buffers: 0 and 1 hold two stacked grid functions each; stabilized Lawson2 needs a
    // fifth grid function (buffer 2). Lawson-Euler and Lawson2b on finite differences keep
    // them with x1 rows padded to whole 128-byte lines (16 values) from n1 = 32 on: rows
    // of n1 = 255 values start 2040 bytes apart, so most rows begin and end inside a
    // line, and the mode products read and write partial lines. The padding is zeroed
    // here and stays zero (no pass writes it except with products of zeros).
    op->ld1 = op->n[0];
    if (!periodic && (scheme == MM_LAWSON_EULER || scheme == MM_LAWSON2B) && op->n[0] >= 32)
      op->ld1 = (op->n[0] + 15) / 16 * 16;
    op->dofp = dof / op->n[0] * op->ld1;
    for (int i = 0; i < 2; ++i) {
      op->buf_len[i] = 2 * op->dofp;
      if ((rc = dev_alloc(op, &op->buf[i], 2 * op->dofp)) != MM_OK) return fail(rc);
      if (hipMemsetAsync(op->buf[i], 0, 2 * op->dofp * sizeof(double), st) != hipSuccess) return fail(MM_EDEVICE);
    }
    if (scheme == MM_SL2) {
      op->buf_len[2] = dof;
      if ((rc = dev_alloc(op, &op->buf[2], dof)) != MM_OK) return fail(rc);
    }
  }
  if (prec == MM_SLICED) {
    // the grid operand of the largest sliced launch: G groups or stacked vectors per
    // mode product (ERK: the q + 1 stage groups, Lawson: the stacked pair), and the
    // stacked last mode of the ERK stages (K = G n_last)
    const int S = op->slices;
    const int64_t G = std::max(2, op->q + 1);
    int64_t dig = 0, ex = 0;
    for (int mu = 0; mu < op->d; ++mu) {
      // fibers of the largest launch along mu (padded stage vectors count their padding)
      const int64_t fib = std::max(dof, op->dofp) / op->n[mu];
      dig = std::max(dig, G * fib * S * slice_ld(op->n[mu]));
      ex = std::max(ex, G * fib);
    }
    if (family == MM_ERK) {
      dig = std::max(dig, (dof / nl) * S * (int64_t)slice_ld((int)G * nl));
      ex = std::max(ex, dof / nl);
    }
    // chained actions: the chain layout of every product's input, two stacked vectors,
    // groups of 256 fibers (padded), in two workspaces
    int64_t cdig = 0, cex = 0;
    if (chain_capable(op)) {
      for (int mu = 0; mu < op->d; ++mu) {
        const int64_t groups = 2 * (dof / ((int64_t)op->n[mu] * op->n[(mu + 1) % op->d]));
        cdig = std::max(cdig, groups * 256 * S * slice_ld(op->n[mu]));
        cex = std::max(cex, groups * 256);
      }
    }
    dig = std::max(dig, cdig);
    ex = std::max(ex, cex);
    op->vdig_len = dig;
    op->vexp_len = ex;
    if ((rc = dev_alloc(op, &op->vdig, dig)) != MM_OK) return fail(rc);
    if ((rc = dev_alloc(op, &op->vexp, ex)) != MM_OK) return fail(rc);
    if (cdig > 0) {
      op->vdig2_len = cdig;
      op->vexp2_len = cex;
      if ((rc = dev_alloc(op, &op->vdig2, cdig)) != MM_OK) return fail(rc);
      if ((rc = dev_alloc(op, &op->vexp2, cex)) != MM_OK) return fail(rc);
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    set_err(ctx, "setup failed on the device");
    return fail(MM_EDEVICE);
  }
  *out = op;
  return MM_OK;
}

mm_status mumode_info(const mm_op* op, double* a_max, int* squarings) {
  if (!op) return MM_EINVAL;
  if (a_max) *a_max = op->a_max;
  if (squarings)
    for (int mu = 0; mu < op->d; ++mu) squarings[mu] = op->squarings[mu];
  return MM_OK;
}

mm_status mumode_get_factor(const mm_op* op, int mu, int j, double* host_out) {
  if (!op || !host_out || mu < 0 || mu >= op->d || j < 0 || j >= op->nfac) return MM_EINVAL;
  hipSetDevice(op->ctx->device);
  const int64_t nn = (int64_t)op->n[mu] * op->n[mu];
  if (hipMemcpy(host_out, factor(op, mu, j), nn * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return MM_EDEVICE;
  return MM_OK;
}

mm_status remainder_eval(mm_ctx* ctx, const mm_op* op, const double* u, double* g, double* F, void* stream) {
  mm_status rc = check_op(ctx, op);
  if (rc != MM_OK) return rc;
  if (!u || !g) {
    set_err(ctx, "null u or g");
    return MM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  StencilArgs a = stencil_args(op, u, false);
  a.out0 = g;
  a.flag = nullptr;
  HIPCHK(ctx, stencil(op, a, s));
  if (F) {
    StencilArgs b = stencil_args(op, u, true);
    b.out0 = F;
    b.flag = nullptr;
    HIPCHK(ctx, stencil(op, b, s));
  }
  return MM_OK;
}

mm_status mumode_expv(mm_ctx* ctx, const mm_op* op, int j, const double* in, double* out, void* stream) {
  mm_status rc = check_op(ctx, op);
  if (rc != MM_OK) return rc;
  if (!in || !out || j < 0 || j >= op->nfac) {
    set_err(ctx, "bad arguments to mumode_expv");
    return MM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  double* t0 = (op->family == MM_ERK) ? op->buf[1] : op->buf[0];
  double* t1 = (op->family == MM_ERK) ? op->buf[2] : op->buf[1];
  HIPCHK(ctx, exp_action(op, j, in, false, out, 1, t0, t1, s));
  return MM_OK;
}

mm_status mumode_phi1v(mm_ctx* ctx, const mm_op* op, const double* in, double* out, void* stream) {
  mm_status rc = check_op(ctx, op);
  if (rc != MM_OK) return rc;
  if (op->family != MM_ERK) {
    set_err(ctx, "mumode_phi1v needs an MM_ERK operator (quadrature factors)");
    return MM_EINVAL;
  }
  if (!in || !out) {
    set_err(ctx, "null input or output");
    return MM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (op->exact) {
    // R transform, scale by phi1(tau Lambda), L transform
    double* S1 = op->buf[1];
    double* S2 = op->buf[2];
    HIPCHK(ctx, exp_action(op, kFacR, in, false, S2, 1, S1, S1 + op->dof, s));
    HIPCHK(ctx, eig_scale(op, S2, S2, 1.0, MM_EIG_PHI1, nullptr, 0.0, MM_EIG_ONE, s));
    HIPCHK(ctx, exp_action(op, kFacL, S2, false, out, 1, S1, S1 + op->dof, s));
    return MM_OK;
  }
  const double* ins[kMaxGroups];
  int fidx[kMaxGroups];
  for (int g = 0; g < op->q; ++g) {
    ins[g] = in;
    fidx[g] = g + 1;
  }
  double w[kMaxGroups];
  HIPCHK(ctx, grouped_action(op, op->q, ins, fidx, stacked(op, 3), stacked_exp(op, 3), out, nullptr, 0.0,
                                 op->buf[1], op->buf[2], s, stage_weights(op, 3, w)));
  return MM_OK;
}

}  // extern "C"

namespace {

// Enqueue nsteps Lawson steps on s (arguments already validated).
mm_status enqueue_lawson(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, hipStream_t s) {
  const double tau = op->tau;
  const int64_t dof = op->dof;
  double* b0 = op->buf[0];
  double* b1 = op->buf[1];
  const bool mixed = lowp(op);
  // (the one-workgroup solver implements the flux form with Dirichlet data only)
  if (ctx->small_fused && op->prec == MM_FP64 && small2d_fits(op->d, op->n[0], op->n[1]) &&
      op->form == MM_FORM_FLUX && op->bc[0] == MM_BC_DIRICHLET && op->bc[1] == MM_BC_DIRICHLET &&
      (op->scheme == MM_LAWSON_EULER || op->scheme == MM_LAWSON2B)) {
    // the whole time loop in one workgroup
    if (nsteps == 0) return MM_OK;
    const StencilArgs sa = stencil_args(op, u, false);
    SmallArgs a{};
    a.u = u;
    a.a = op->a;
    a.E1 = factor(op, 0, 0);
    a.E2 = factor(op, 1, 0);
    a.n1 = op->n[0];
    a.n2 = op->n[1];
    a.nsteps = nsteps;
    a.tau = tau;
    for (int mu = 0; mu < 2; ++mu) {
      a.ih2[mu] = sa.ih2[mu];
      a.cadv[mu] = sa.cadv[mu];
    }
    a.lam_amax = sa.lam_amax;
    a.r0 = sa.r0;
    a.r1 = sa.r1;
    a.r2 = sa.r2;
    a.r3 = sa.r3;
    a.flag = op->flag;
    const double work = (double)nsteps * (op->scheme == MM_LAWSON2B ? 2 : 1) * 2.0 *
                        (double)op->dof * (op->n[0] + op->n[1]);
    HIPCHK(ctx, timed_launch(ctx, MM_KIND_FUSED, work, s,
                             [&] { return launch_lawson_small2d(a, op->scheme == MM_LAWSON2B, s); }));
    return MM_OK;
  }
  for (int it = 0; it < nsteps; ++it) {
    if (op->scheme == MM_LAWSON_EULER) {
      // u+ = e^{tau A}(u + tau g(u)); the stage vector in the padded layout
      StencilArgs a = stencil_args(op, u, false);
      a.base0 = u;
      a.c0 = tau;
      a.ldo = op->ld1;
      const bool dg = stencil_digits(op);
      if (dg) {
        set_stencil_digits(a, op, op->vdig, op->vexp, 1);
        a.dchain = chain_active(op);
      } else if (mixed)
        a.out0f = (float*)b0;
      else
        a.out0 = b0;
      HIPCHK(ctx, stencil(op, a, s));
      if (dg && chain_active(op))
        HIPCHK(ctx, chain_action(op, 0, 1, u, natural(op), s));
      else
        HIPCHK(ctx, exp_action(op, 0, b0, mixed, u, 1, b1, b0, s, nullptr, 1.0, 1.0, staged(op), staged(op),
                               natural(op), dg));
    } else if (op->scheme == MM_SLE) {
      // u+ = u + tau e^{tau A} F(u)
      StencilArgs f = stencil_args(op, u, true);
      f.out0 = b0;
      HIPCHK(ctx, stencil(op, f, s));
      HIPCHK(ctx, exp_action(op, 0, b0, false, u, 1, b1, b1 + dof, s, u, tau, 1.0));
    } else if (op->scheme == MM_LAWSON2A) {
      // U = e^{tau/2 A}(u + tau/2 g(u)); u+ = e^{tau A} u + tau e^{tau/2 A} g(U)
      StencilArgs a = stencil_args(op, u, false);
      a.base0 = u;
      a.c0 = 0.5 * tau;
      a.out0 = b0;
      HIPCHK(ctx, stencil(op, a, s));
      double* U = b0 + dof;
      HIPCHK(ctx, exp_action(op, 1, b0, false, U, 1, b1, b1 + dof, s));
      StencilArgs c = stencil_args(op, U, false);
      c.out0 = b0;
      HIPCHK(ctx, stencil(op, c, s));
      HIPCHK(ctx, exp_action(op, 1, b0, false, U, 1, b1, b1 + dof, s));
      HIPCHK(ctx, exp_action(op, 0, u, false, u, 1, b1, b1 + dof, s, U, 1.0, tau));
    } else if (op->scheme == MM_SL2) {
      // U = u + alpha tau e^{alpha tau A} F(u);
      // u+ = u + tau e^{tau/2 A} F(u) + tau/(2 alpha) e^{tau A}(g(U) - g(u))
      double *F0 = b0, *g0 = b0 + dof, *U = op->buf[2];
      StencilArgs f = stencil_args(op, u, true);
      f.out0 = F0;
      HIPCHK(ctx, stencil(op, f, s));
      StencilArgs a = stencil_args(op, u, false);
      a.out0 = g0;
      HIPCHK(ctx, stencil(op, a, s));
      HIPCHK(ctx, exp_action(op, 2, F0, false, U, 1, b1, b1 + dof, s, u, kAlphaSL2 * tau, 1.0));
      StencilArgs c = stencil_args(op, U, false);   // D = g(U) - g0, in place of g0
      c.sub = g0;
      c.out0 = g0;
      HIPCHK(ctx, stencil(op, c, s));
      HIPCHK(ctx, exp_action(op, 1, F0, false, U, 1, b1, b1 + dof, s, u, tau, 1.0));   // W (over U)
      HIPCHK(ctx, exp_action(op, 0, g0, false, u, 1, b1, b1 + dof, s, U, 0.5 * tau / kAlphaSL2, 1.0));
    } else {
      // v1 = u + tau g(u), v2 = u + tau/2 g(u); [U, W] = e^{tau A}[v1, v2]; u+ = W + tau/2 g(U)
      // (v1, v2, U, W in the padded layout: rows of ld1, dofp apart)
      const int64_t dp = op->dofp;
      StencilArgs a = stencil_args(op, u, false);
      a.base0 = u;
      a.c0 = tau;
      a.base1 = u;
      a.c1 = 0.5 * tau;
      a.ldo = op->ld1;
      const bool dg = stencil_digits(op);
      if (dg) {
        set_stencil_digits(a, op, op->vdig, op->vexp, 2);
        a.dchain = chain_active(op);
      } else if (mixed) {
        a.out0f = (float*)b0;
        a.out1f = (float*)b0 + dp;
      } else {
        a.out0 = b0;
        a.out1 = b0 + dp;
      }
      HIPCHK(ctx, stencil(op, a, s));
      double* res = (op->d == 3) ? b1 : b0;
      if (dg && chain_active(op))
        HIPCHK(ctx, chain_action(op, 0, 2, res, staged(op), s));
      else
        HIPCHK(ctx, exp_action(op, 0, b0, mixed, res, 2, b1, b0, s, nullptr, 1.0, 1.0, staged(op), staged(op),
                               staged(op), dg));
      StencilArgs c = stencil_args(op, res, false);
      c.base0 = res + dp;
      c.c0 = 0.5 * tau;
      c.ldi = op->ld1;
      c.out0 = u;
      HIPCHK(ctx, stencil(op, c, s));
    }
  }
  return MM_OK;
}

// ERK steps with exact phi functions through the joint eigenbasis (A = L diag(Lambda) R
// per axis): every phi or exponential action is an R transform, a diagonal scaling and
// an L transform, so an ETD2RK step is 12 mode products instead of the quadrature's 2q+1
// actions.
mm_status enqueue_erk_exact(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, hipStream_t s) {
  const double tau = op->tau;
  const int64_t dof = op->dof;
  double *TG = op->buf[0], *S1 = op->buf[1], *S2 = op->buf[2], *U = op->buf[3], *D = op->buf[4], *F0 = op->buf[5];
  double* g0 = TG + dof;
  const int sch = op->scheme;
  for (int it = 0; it < nsteps; ++it) {
    if (sch != MM_EE) {
      // g0 = g(u); ETD2RK also copies u alongside so that [u, g0] transform together
      StencilArgs a = stencil_args(op, u, false);
      a.out0 = g0;
      if (sch == MM_ETD2RK) {
        a.base1 = u;
        a.c1 = 0.0;
        a.out1 = TG;
      }
      HIPCHK(ctx, stencil(op, a, s));
    }
    // first stage into U (exponential Euler: straight into u)
    double* U1 = (sch == MM_EE) ? u : U;
    if (sch == MM_ETD2RK) {
      // U = L (e^{tau Lambda} R u + tau phi1(tau Lambda) R g0). The transformed pair H
      // comes out of the last pass: S1 in 3D (TG -> S1 -> S2 -> S1), S2 in 2D (TG -> S1
      // -> S2); the scaled combination goes to the other buffer.
      double* H = (op->d == 3) ? S1 : S2;
      double* W = (op->d == 3) ? S2 : S1;
      HIPCHK(ctx, exp_action(op, kFacR, TG, false, H, 2, S1, S2, s));
      HIPCHK(ctx, eig_scale(op, W, H, 1.0, MM_EIG_EXP, H + dof, tau, MM_EIG_PHI1, s));
      HIPCHK(ctx, exp_action(op, kFacL, W, false, U1, 1, H, H + dof, s));
    } else {
      // U = u + L tau phi1(tau Lambda) R F(u)
      StencilArgs f = stencil_args(op, u, true);
      f.out0 = F0;
      HIPCHK(ctx, stencil(op, f, s));
      HIPCHK(ctx, exp_action(op, kFacR, F0, false, S2, 1, S1, S1 + dof, s));
      HIPCHK(ctx, eig_scale(op, S2, S2, tau, MM_EIG_PHI1, nullptr, 0.0, MM_EIG_ONE, s));
      HIPCHK(ctx, exp_action(op, kFacL, S2, false, U1, 1, S1, S1 + dof, s, u));
    }
    if (sch == MM_EE) continue;
    // D = g(U) - g0;  u+ = U + L c f(tau Lambda) R D with c f = tau/2 phi1 (ETD2RK,
    // ERK2P1) or tau phi2 (ERK2P2)
    StencilArgs b = stencil_args(op, U, false);
    b.sub = g0;
    b.out0 = D;
    HIPCHK(ctx, stencil(op, b, s));
    HIPCHK(ctx, exp_action(op, kFacR, D, false, S2, 1, S1, S1 + dof, s));
    if (sch == MM_ERK2P2)
      HIPCHK(ctx, eig_scale(op, S2, S2, tau, MM_EIG_PHI2, nullptr, 0.0, MM_EIG_ONE, s));
    else
      HIPCHK(ctx, eig_scale(op, S2, S2, 0.5 * tau, MM_EIG_PHI1, nullptr, 0.0, MM_EIG_ONE, s));
    HIPCHK(ctx, exp_action(op, kFacL, S2, false, u, 1, S1, S1 + dof, s, U));
  }
  return MM_OK;
}

// Enqueue nsteps ERK steps on s (arguments already validated).
mm_status enqueue_erk(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, hipStream_t s) {
  if (op->exact) return enqueue_erk_exact(ctx, op, u, nsteps, s);
  const double tau = op->tau;
  const int q = op->q;
  double *g0 = op->buf[0], *T1 = op->buf[1], *T2 = op->buf[2], *U = op->buf[3], *D = op->buf[4],
         *F0 = op->buf[5];
  const double* ins[kMaxGroups];
  int fidx[kMaxGroups];
  double w1[kMaxGroups], w2[kMaxGroups];
  for (int it = 0; it < nsteps; ++it) {
    StencilArgs a = stencil_args(op, u, false);
    a.out0 = g0;
    HIPCHK(ctx, stencil(op, a, s));
    if (op->scheme == MM_ETD2RK) {
      // U = e^{tau A} u + tau sum_j w_j e^{theta_j tau A} g0
      ins[0] = u;
      fidx[0] = 0;
      for (int j = 1; j <= q; ++j) {
        ins[j] = g0;
        fidx[j] = j;
      }
      HIPCHK(ctx, grouped_action(op, q + 1, ins, fidx, stacked(op, 1), stacked_exp(op, 1), U, nullptr, 0.0, T1, T2,
                                 s, stage_weights(op, 1, w1)));
    } else {
      // U = u + tau sum_j w_j e^{theta_j tau A} F(u)
      StencilArgs f = stencil_args(op, u, true);
      f.out0 = F0;
      HIPCHK(ctx, stencil(op, f, s));
      for (int j = 0; j < q; ++j) {
        ins[j] = F0;
        fidx[j] = j + 1;
      }
      HIPCHK(ctx, grouped_action(op, q, ins, fidx, stacked(op, 1), stacked_exp(op, 1), U, u, 1.0, T1, T2, s,
                                 stage_weights(op, 1, w1)));
    }
    // D = g(U) - g0;  u+ = U + tau/2 sum_j w_j e^{theta_j tau A} D
    StencilArgs b = stencil_args(op, U, false);
    b.sub = g0;
    b.out0 = D;
    HIPCHK(ctx, stencil(op, b, s));
    for (int j = 0; j < q; ++j) {
      ins[j] = D;
      fidx[j] = j + 1;
    }
    HIPCHK(ctx, grouped_action(op, q, ins, fidx, stacked(op, 2), stacked_exp(op, 2), u, U, 1.0, T1, T2, s,
                               stage_weights(op, 2, w2)));
  }
  return MM_OK;
}

mm_status enqueue_steps(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, hipStream_t s) {
  return op->family == MM_LAWSON ? enqueue_lawson(ctx, op, u, nsteps, s) : enqueue_erk(ctx, op, u, nsteps, s);
}

// Record `gs` steps on state u into the op's graph (capture runs nothing). A previous
// graph of the op may still be replaying on the stream it was last launched on: wait for
// that stream before destroying it.
mm_status record_graph(mm_ctx* ctx, const mm_op* op, double* u, int gs) {
  if (!ctx->capture) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
  if (op->gexec) {
    HIPCHK(ctx, hipStreamSynchronize(op->gstream));
    HIPCHK(ctx, hipGraphExecDestroy(op->gexec));
    op->gexec = nullptr;
  }
  HIPCHK(ctx, hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
  mm_status rc = enqueue_steps(ctx, op, u, gs, ctx->capture);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->capture, &graph);
  if (rc != MM_OK) {
    if (graph) hipGraphDestroy(graph);
    return rc;
  }
  HIPCHK(ctx, e);
  const hipError_t ei = hipGraphInstantiate(&op->gexec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  HIPCHK(ctx, ei);
  op->gu = u;
  op->gsteps = gs;
  return MM_OK;
}

// Steps through recorded graphs when the context asks for them (and is not timing
// individual kernels), else by direct launches.
mm_status run_steps(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, hipStream_t s) {
  const int gs = ctx->graph_steps;
  if (gs <= 0 || ctx->timing || nsteps < gs) return enqueue_steps(ctx, op, u, nsteps, s);
  if (!op->gexec || op->gu != u || op->gsteps != gs) {
    mm_status rc = record_graph(ctx, op, u, gs);
    if (rc != MM_OK) return rc;
  }
  const int reps = nsteps / gs;
  op->gstream = s;
  for (int i = 0; i < reps; ++i) HIPCHK(ctx, hipGraphLaunch(op->gexec, s));
  return enqueue_steps(ctx, op, u, nsteps - reps * gs, s);
}

// One mode pass of the exponential for `count` problems of one class, as a single
// grouped launch: group i applies problem i's factor exp(tau_i A_mu) to its own
// `nvec` stacked grid functions (in[i] -> out[i], layouts li -> lo as in pass_mode1,
// pass_mode2 and pass_last).
hipError_t group_pass(mm_ctx* ctx, const mm_op* const* ops, int count, int mu, int nvec, const void* const* in,
                      void* const* out, PassIO io, const mm_batch_ws* ws, hipStream_t s, Layout li, Layout lo) {
  const mm_op* o0 = ops[0];
  const int d = o0->d, n = o0->n[mu];
  const int64_t dof = o0->dof;
  GemmArgs g{};
  for (int i = 0; i < count; ++i) {
    const void* F = factor_op(ops[i], mu, 0);
    g.Ff[i] = folded(ops[i], mu, 0);
    g.fexp[i] = factor_exp(ops[i], mu, 0);
    g.galpha[i] = 0.0;
    g.Cadd[i] = nullptr;
    g.C[i] = out[i];
    if (mu == 0) {
      g.A[i] = in[i];
      g.B[i] = F;
    } else {
      g.A[i] = F;
      g.B[i] = in[i];
    }
  }
  g.groups = count;
  g.slices = o0->slices;
  g.alpha = 1.0;
  g.beta = 0.0;
  g.in_f32 = io.in_f32;
  g.out_f32 = io.out_f32;
  g.fac_slice = factor_slice_stride(o0, n, n);
  g.tile = ctx->gemm_tile;
  g.vready = io.ready;
  g.ldf = fold_ld(n);
  g.fold = ctx->fold;
  if (ws) {
    g.vdig = ws->vdig;
    g.vexp = ws->vexp;
    g.vdig_cap = ws->vdig_cap;
    g.vexp_cap = ws->vexp_cap;
  }
  auto launch = [&]() {
    const double work = gemm_work(g, o0->prec);
    return timed_launch(ctx, g.b_trans ? MM_KIND_GEMM_N : MM_KIND_GEMM_K, work, s,
                        [&] { return launch_gemm(o0->prec, g, s); });
  };
  if (mu == 0) {
    g.M = (int)(dof / n) * nvec;
    g.N = g.K = n;
    g.lda = li.ld;
    g.ldc = lo.ld;
    g.ldb = factor_ld(o0, n);
    g.inner = 1;
    g.b_trans = 0;
    return launch();
  }
  g.M = g.K = n;
  g.lda = factor_ld(o0, n);
  g.sA = 0;
  g.b_trans = 1;
  if (mu < d - 1) {   // x2 of a 3D grid: per x3 slab
    g.N = o0->n[0];
    g.ldb = li.ld;
    g.ldc = lo.ld;
    g.inner = o0->n[2] * nvec;
    g.sB = (int64_t)li.ld * o0->n[1];
    g.sC = (int64_t)lo.ld * o0->n[1];
    return launch();
  }
  if (d == 2 || li.ld == lo.ld) {
    // the last axis: columns are x1 (2D) or the whole padded (x2, x1) plane (3D)
    g.N = d == 2 ? o0->n[0] : o0->n[1] * li.ld;
    g.ldb = d == 2 ? li.ld : o0->n[1] * li.ld;
    g.ldc = d == 2 ? lo.ld : o0->n[1] * lo.ld;
    g.inner = nvec;
    g.sB = li.vs;
    g.sC = lo.vs;
    return launch();
  }
  // 3D with different row strides: per vector, batched over the x2 rows
  const size_t ib = io.in_f32 ? 4 : 8, ob = io.out_f32 ? 4 : 8;
  for (int v = 0; v < nvec; ++v) {
    for (int i = 0; i < count; ++i) {
      g.B[i] = (const char*)in[i] + (size_t)v * li.vs * ib;
      g.C[i] = (char*)out[i] + (size_t)v * lo.vs * ob;
    }
    g.N = o0->n[0];
    g.ldb = o0->n[1] * li.ld;
    g.ldc = o0->n[1] * lo.ld;
    g.inner = o0->n[1];
    g.sB = li.ld;
    g.sC = lo.ld;
    const hipError_t e = launch();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The digit-plane workspace of grouped sliced launches on stream s, at least dig bytes
// and ex exponents (stream-ordered reallocation when it has to grow).
mm_status group_workspace(mm_ctx* ctx, hipStream_t s, int64_t dig, int64_t ex, mm_batch_ws** out) {
  mm_batch_ws* w = nullptr;
  for (auto& b : ctx->bws)
    if (b.stream == s) w = &b;
  if (!w) {
    ctx->bws.push_back(mm_batch_ws{});
    w = &ctx->bws.back();
    w->stream = s;
  }
  if (w->vdig_cap < dig) {
    if (w->vdig) hipFreeAsync(w->vdig, s);
    w->vdig = nullptr;
    w->vdig_cap = 0;
    if (hipMallocAsync((void**)&w->vdig, (size_t)dig, s) != hipSuccess) {
      w->vdig = nullptr;
      set_err(ctx, "grouped sliced workspace allocation (%lld bytes) failed", (long long)dig);
      return MM_ENOMEM;
    }
    w->vdig_cap = dig;
  }
  if (w->vexp_cap < ex) {
    if (w->vexp) hipFreeAsync(w->vexp, s);
    w->vexp = nullptr;
    w->vexp_cap = 0;
    if (hipMallocAsync((void**)&w->vexp, (size_t)ex * sizeof(int), s) != hipSuccess) {
      w->vexp = nullptr;
      set_err(ctx, "grouped sliced workspace allocation failed");
      return MM_ENOMEM;
    }
    w->vexp_cap = ex;
  }
  *out = w;
  return MM_OK;
}

}  // namespace

namespace mm {

bool lawson_groupable(const mm_op* op) {
  return op && op->family == MM_LAWSON && !op->periodic &&
         (op->scheme == MM_LAWSON_EULER || op->scheme == MM_LAWSON2B);
}

bool small2d_fusable(const mm_ctx* ctx, const mm_op* op) {
  return ctx->small_fused && op->family == MM_LAWSON && op->prec == MM_FP64 && !op->periodic &&
         small2d_fits(op->d, op->n[0], op->n[1]) && op->form == MM_FORM_FLUX && op->bc[0] == MM_BC_DIRICHLET &&
         op->bc[1] == MM_BC_DIRICHLET && (op->scheme == MM_LAWSON_EULER || op->scheme == MM_LAWSON2B);
}

bool same_class(const mm_op* a, const mm_op* b) {
  return a->d == b->d && a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->n[2] == b->n[2] && a->prec == b->prec &&
         a->slices == b->slices && a->family == b->family && a->scheme == b->scheme;
}

// Steps of `count` problems of one class (Lawson-Euler or Lawson2b, the pass sequence
// of enqueue_lawson): per pass one stencil launch for all problems and one grouped
// launch per mode, every problem with its own factors, coefficients, tau and scratch.
// Each output is computed by the same kernels in the same order as for the problem
// alone (the stencil per point; a mode product per output, whatever the tile), so the
// results are bit-identical to lawson_step's.
mm_status enqueue_lawson_group(mm_ctx* ctx, const mm_op* const* ops, double* const* u, int count, int nsteps,
                               hipStream_t s) {
  const mm_op* o0 = ops[0];
  const int64_t dof = o0->dof;
  const int d = o0->d;
  const bool mixed = lowp(o0);
  const bool l2b = o0->scheme == MM_LAWSON2B;
  const int nvec = l2b ? 2 : 1;
  const int64_t dp = o0->dofp;   // stage-vector stride (padded rows, equal across the class)
  mm_batch_ws* ws = nullptr;
  if (o0->prec == MM_SLICED) {
    // the largest grid-operand split over the modes of one grouped action (padded
    // stage vectors count their padding)
    int64_t dig = 0, ex = 0;
    for (int mu = 0; mu < d; ++mu) {
      const int64_t fib = (int64_t)count * nvec * (o0->dofp / o0->n[mu]);
      dig = std::max(dig, fib * o0->slices * slice_ld(o0->n[mu]));
      ex = std::max(ex, fib);
    }
    mm_status rc = group_workspace(ctx, s, dig, ex, &ws);
    if (rc != MM_OK) return rc;
  }
  StencilArgs sa[kMaxGroups];
  const void* in[kMaxGroups];
  void *t0[kMaxGroups], *t1[kMaxGroups], *out[kMaxGroups];
  for (int i = 0; i < count; ++i) {
    in[i] = ops[i]->buf[0];
    t0[i] = ops[i]->buf[1];
    t1[i] = ops[i]->buf[0];
    out[i] = l2b ? (d == 3 ? ops[i]->buf[1] : ops[i]->buf[0]) : u[i];
  }
  // sliced: the first stencil pass writes the mode-1 operand's digits into each
  // problem's slot of the group workspace (group i at i S plane bytes, i F exponents)
  const bool dg = stencil_digits(o0);
  const int64_t fib1 = (int64_t)nvec * (dof / o0->n[0]);
  for (int it = 0; it < nsteps; ++it) {
    // v1 = u + tau g(u) (and for Lawson2b v2 = u + tau/2 g(u)) into buf[0]
    for (int i = 0; i < count; ++i) {
      const mm_op* op = ops[i];
      double* b0 = op->buf[0];
      StencilArgs a = stencil_args(op, u[i], false);
      a.base0 = u[i];
      a.c0 = op->tau;
      a.ldo = op->ld1;
      if (l2b) {
        a.base1 = u[i];
        a.c1 = 0.5 * op->tau;
      }
      if (dg) {
        set_stencil_digits(a, op, ws->vdig + (int64_t)i * o0->slices * fib1 * slice_ld(o0->n[0]), ws->vexp + i * fib1,
                           nvec);
      } else if (mixed) {
        a.out0f = (float*)b0;
        if (l2b) a.out1f = (float*)b0 + dp;
      } else {
        a.out0 = b0;
        if (l2b) a.out1 = b0 + dp;
      }
      sa[i] = a;
    }
    HIPCHK(ctx, timed_launch(ctx, MM_KIND_STENCIL, (double)dof * count, s,
                             [&] { return launch_stencil_batch(d, sa, count, s); }));
    // e^{tau A}: buf[0] -> buf[1] (-> buf[0]) -> out, stage vectors padded
    const Layout lp = staged(o0), lout = l2b ? lp : natural(o0);
    HIPCHK(ctx, group_pass(ctx, ops, count, 0, nvec, in, t0, PassIO{mixed, mixed, dg}, ws, s, lp, lp));
    if (d == 3) {
      HIPCHK(ctx, group_pass(ctx, ops, count, 1, nvec, (const void* const*)t0, t1, PassIO{mixed, mixed}, ws, s,
                             lp, lp));
      HIPCHK(ctx, group_pass(ctx, ops, count, 2, nvec, (const void* const*)t1, out, PassIO{mixed, false}, ws, s,
                             lp, lout));
    } else {
      HIPCHK(ctx, group_pass(ctx, ops, count, 1, nvec, (const void* const*)t0, out, PassIO{mixed, false}, ws, s,
                             lp, lout));
    }
    if (!l2b) continue;
    // u+ = W + tau/2 g(U) with [U, W] the transformed pair
    for (int i = 0; i < count; ++i) {
      const mm_op* op = ops[i];
      const double* res = (const double*)out[i];
      StencilArgs c = stencil_args(op, res, false);
      c.base0 = res + dp;
      c.c0 = 0.5 * op->tau;
      c.ldi = op->ld1;
      c.out0 = u[i];
      sa[i] = c;
    }
    HIPCHK(ctx, timed_launch(ctx, MM_KIND_STENCIL, (double)dof * count, s,
                             [&] { return launch_stencil_batch(d, sa, count, s); }));
  }
  return MM_OK;
}

// Whole solves of small 2D problems, one workgroup each (any sizes up to 64 x 64 and any
// step counts), each computed exactly as by the one-problem launch.
mm_status enqueue_small2d_group(mm_ctx* ctx, const mm_op* const* ops, double* const* u, const int* nsteps,
                                int count, hipStream_t s) {
  if (count < 1 || count > kMaxSmallBatch) return MM_EINVAL;
  const bool l2b = ops[0]->scheme == MM_LAWSON2B;
  SmallArgs args[kMaxSmallBatch];
  double work = 0.0;
  for (int i = 0; i < count; ++i) {
    const mm_op* op = ops[i];
    if ((op->scheme == MM_LAWSON2B) != l2b) return MM_EINVAL;
    const StencilArgs sa = stencil_args(op, u[i], false);
    SmallArgs& a = args[i];
    a = SmallArgs{};
    a.u = u[i];
    a.a = op->a;
    a.E1 = factor(op, 0, 0);
    a.E2 = factor(op, 1, 0);
    a.n1 = op->n[0];
    a.n2 = op->n[1];
    a.nsteps = nsteps[i];
    a.tau = op->tau;
    for (int mu = 0; mu < 2; ++mu) {
      a.ih2[mu] = sa.ih2[mu];
      a.cadv[mu] = sa.cadv[mu];
    }
    a.lam_amax = sa.lam_amax;
    a.r0 = sa.r0;
    a.r1 = sa.r1;
    a.r2 = sa.r2;
    a.r3 = sa.r3;
    a.flag = op->flag;
    work += (double)nsteps[i] * (l2b ? 2 : 1) * 2.0 * (double)op->dof * (op->n[0] + op->n[1]);
  }
  HIPCHK(ctx, timed_launch(ctx, MM_KIND_FUSED, work, s,
                           [&] { return launch_lawson_small2d_batch(args, count, l2b, s); }));
  return MM_OK;
}

}  // namespace mm

extern "C" {

mm_status lawson_step_batch(mm_ctx* ctx, const mm_op* const* ops, double* const* u, int count, int nsteps,
                            void* stream) {
  if (!ctx) return MM_EINVAL;
  if (!ops || !u || count < 1 || count > kMaxGroups || nsteps < 0) {
    set_err(ctx, "lawson_step_batch: null arrays, count outside 1..%d or nsteps < 0", kMaxGroups);
    return MM_EINVAL;
  }
  for (int i = 0; i < count; ++i) {
    mm_status rc = check_op(ctx, ops[i]);
    if (rc != MM_OK) return rc;
    if (!u[i]) {
      set_err(ctx, "lawson_step_batch: null state %d", i);
      return MM_EINVAL;
    }
    if (!lawson_groupable(ops[i])) {
      set_err(ctx, "lawson_step_batch: op %d is not a finite-difference Lawson-Euler or Lawson2b operator", i);
      return MM_EINVAL;
    }
    if (!same_class(ops[0], ops[i])) {
      set_err(ctx, "lawson_step_batch: op %d differs from op 0 in shape, precision, digits or scheme", i);
      return MM_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (ops[j] == ops[i] || u[j] == u[i]) {
        set_err(ctx, "lawson_step_batch: entries %d and %d share an operator or a state", j, i);
        return MM_EINVAL;
      }
  }
  if (nsteps == 0) return MM_OK;
  hipStream_t s = (hipStream_t)stream;
  if (small2d_fusable(ctx, ops[0])) {
    int ns[kMaxGroups];
    for (int i = 0; i < count; ++i) ns[i] = nsteps;
    return enqueue_small2d_group(ctx, ops, u, ns, count, s);
  }
  return enqueue_lawson_group(ctx, ops, u, count, nsteps, s);
}

}  // extern "C"

extern "C" {

mm_status lawson_step(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, void* stream) {
  mm_status rc = check_op(ctx, op);
  if (rc != MM_OK) return rc;
  if (op->family != MM_LAWSON) {
    set_err(ctx, "lawson_step needs an MM_LAWSON operator");
    return MM_EINVAL;
  }
  if (!u || nsteps < 0) {
    set_err(ctx, "bad arguments to lawson_step");
    return MM_EINVAL;
  }
  return run_steps(ctx, op, u, nsteps, (hipStream_t)stream);
}

mm_status erk_step(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, void* stream) {
  mm_status rc = check_op(ctx, op);
  if (rc != MM_OK) return rc;
  if (op->family != MM_ERK) {
    set_err(ctx, "erk_step needs an MM_ERK operator");
    return MM_EINVAL;
  }
  if (!u || nsteps < 0) {
    set_err(ctx, "bad arguments to erk_step");
    return MM_EINVAL;
  }
  return run_steps(ctx, op, u, nsteps, (hipStream_t)stream);
}

mm_status mm_set_small_fused(mm_ctx* ctx, int enable) {
  if (!ctx) return MM_EINVAL;
  ctx->small_fused = enable != 0;
  return MM_OK;
}

mm_status mm_set_graph_steps(mm_ctx* ctx, int steps) {
  if (!ctx) return MM_EINVAL;
  if (steps < 0 || steps > 4096) {
    set_err(ctx, "graph steps must be in [0, 4096]");
    return MM_EINVAL;
  }
  ctx->graph_steps = steps;
  return MM_OK;
}

mm_status mm_synchronize(mm_ctx* ctx) {
  if (!ctx) return MM_EINVAL;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipDeviceSynchronize());
  return MM_OK;
}

mm_status mm_timing_enable(mm_ctx* ctx, int enable) {
  if (!ctx) return MM_EINVAL;
  ctx->timing = enable != 0;
  ctx->timed_used = 0;
  return MM_OK;
}

mm_status mm_set_sliced_chain(mm_ctx* ctx, int mode) {
  if (!ctx) return MM_EINVAL;
  if (mode < 0 || mode > 3) {
    set_err(ctx, "sliced chain mode must be 0, 1, 2 or 3");
    return MM_EINVAL;
  }
  ctx->sliced_chain = mode;
  return MM_OK;
}

mm_status mm_set_fold(mm_ctx* ctx, int mode) {
  if (!ctx) return MM_EINVAL;
  if (mode < 0 || mode > 2) {
    set_err(ctx, "fold mode must be 0, 1 or 2");
    return MM_EINVAL;
  }
  ctx->fold = mode;
  return MM_OK;
}

mm_status mm_set_gemm_tile(mm_ctx* ctx, int tile) {
  if (!ctx) return MM_EINVAL;
  if (tile != 0 && tile != 32 && tile != 64 && tile != 128) {
    set_err(ctx, "gemm tile must be 0, 32, 64 or 128");
    return MM_EINVAL;
  }
  ctx->gemm_tile = tile;
  return MM_OK;
}

mm_status mm_timing_read(mm_ctx* ctx, int kind, int64_t* launches, double* total_ms, double* work) {
  if (!ctx) return MM_EINVAL;
  int64_t cnt = 0;
  double ms = 0.0, wk = 0.0;
  for (size_t i = 0; i < ctx->timed_used; ++i) {
    mm_timed& t = ctx->timed[i];
    if (t.kind != kind) continue;
    HIPCHK(ctx, hipEventSynchronize(t.stop));
    float e = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&e, t.start, t.stop));
    ++cnt;
    ms += e;
    wk += t.work;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (work) *work = wk;
  return MM_OK;
}

mm_status mm_check(mm_ctx* ctx, const mm_op* op, void* stream) {
  mm_status rc = check_op(ctx, op);
  if (rc != MM_OK) return rc;
  int flag = 0;
  HIPCHK(ctx, hipStreamSynchronize((hipStream_t)stream));
  HIPCHK(ctx, hipMemcpy(&flag, op->flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) {
    set_err(ctx, "non-finite values in the solution");
    return MM_EUNSTABLE;
  }
  return MM_OK;
}

}  // extern "C"
