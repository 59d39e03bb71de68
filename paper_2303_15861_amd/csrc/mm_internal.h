// Internal declarations shared by the HIP sources of the mu-mode library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mumode.h"

namespace mm {

constexpr int kMaxGroups = 8;   // quadrature nodes + 1
// stabilized Lawson2: the alpha of Theorem thm:stablawson2 (stability bound 0.182)
constexpr double kAlphaSL2 = 0.327;

// One batched/grouped GEMM  C[g][b] = alpha * A[g][b] . B'[g][b] + beta * Cadd[g][b]
// with row-major operands: A[m][k] at m*lda + k; C[m][n] at m*ldc + n;
// B'[n][k] at n*ldb + k (b_trans = 0) or at k*ldb + n (b_trans = 1).
// Group g selects base pointers; the inner batch index b adds b*s{A,B,C}.
// FP64 mode: every operand is double. Mixed modes: the factor operand (B' when
// b_trans = 0, A when b_trans = 1) is pre-converted at setup -- FP32, or S BF16 slices
// `fac_slice` elements apart -- with its rows zero-padded to a multiple of 32 in k;
// the grid operand is float (in_f32) or double, C is float (out_f32) or double.
struct GemmArgs {
  const void* A[kMaxGroups];
  const void* B[kMaxGroups];
  void* C[kMaxGroups];
  const double* Cadd[kMaxGroups];
  int M, N, K;
  int lda, ldb, ldc;
  int inner;
  int64_t sA, sB, sC;
  int groups;
  int b_trans;
  double alpha, beta;
  int in_f32, out_f32;
  int64_t fac_slice;
  int tile;             // workgroup tile: 0 = chosen by the launcher, 64 or 128
  // MM_SLICED: digit count and per-row exponents of the factor operand of each group
  int slices;
  const int* fexp[kMaxGroups];
  double galpha[kMaxGroups];   // MM_SLICED: extra per-group output scale (0 = none)
  // MM_SLICED: workspace for the digit planes and fiber exponents of the grid operand
  // (sliced_workspace() bytes and ints for this launch); vready: the grid operand's
  // digits and exponents are already there (written by the stencil), so the launch
  // skips its split pass and does not read the FP64 operand
  signed char* vdig;
  int* vexp;
  int64_t vdig_cap, vexp_cap;
  int vready;
  // FP64 with a centrosymmetric factor (every group's factor E = J E J): Ff[g] is the
  // folded factor [Es; Ed] of launch_fold_factor (2f rows of f = K - K/2 values, row
  // stride ldf = fold_ld(K)); fold: 0 plain product, 1 folded from 192 tiles per group, 2 always
  const double* Ff[kMaxGroups];
  int ldf;
  int fold;
  // modes 2/3 only: the factor stacks fold_blocks n x n blocks along k (K = fold_blocks n,
  // each block centrosymmetric; the grid operand stacks as many vectors), folded block by
  // block side by side (launch_fold_stacked; ldf = fold_blocks fold_ld(n)); 0 or 1: one
  int fold_blocks;
  // filled by the launcher
  int tiles_m, tiles_n, total, per_xcd;
};

constexpr int kFacPad = 32;   // k padding of pre-converted factors
inline int fac_ld(int k) { return (k + kFacPad - 1) / kFacPad * kFacPad; }
// digit planes of MM_SLICED: rows zero-padded to a multiple of 64 in k
constexpr int kMinSlices = 3, kMaxSlices = 7, kDefaultSlices = 6;
__host__ __device__ inline int slice_ld(int k) { return (k + 63) / 64 * 64; }
// Workspace of a sliced launch: digit bytes and exponent count for the grid operand
// (groups x fibers x S x slice_ld(K) bytes; groups x fibers exponents). Fibers are the
// M rows (mode 1) or the inner x N columns (modes 2 and 3).
__host__ __device__ inline int64_t sliced_fibers(const GemmArgs& g) { return g.b_trans ? (int64_t)g.inner * g.N : (int64_t)g.M; }
__host__ __device__ inline int64_t sliced_digit_bytes(const GemmArgs& g) {
  return (int64_t)g.groups * sliced_fibers(g) * g.slices * slice_ld(g.K);
}

// Stencil launch parameters (remainder g and fused stage updates).
struct StencilArgs {
  const double* u;      // input grid function
  const double* a;      // nodal coefficient, (n+2)^d
  int n1, n2, n3;       // n3 = 1 for d = 2
  double ih2[3];        // 1/h_mu^2
  double cadv[3];       // (beta - beta_bar)/(2 h)
  double lam_amax;      // lambda * a_max (0 for the unsplit F)
  double r0, r1, r2, r3;
  const double* sub;    // nullable: s = g - sub
  const double* base0;  // nullable
  double c0;
  double* out0;         // out0 = base0 + c0 * s
  float* out0f;         // if set, out0 is written here as float instead
  const double* base1;  // nullable
  double c1;
  double* out1;         // nullable: out1 = base1 + c1 * s
  float* out1f;         // if set, out1 is written here as float instead
  int* flag;            // nullable: set to 1 if out0 is not finite
  int neu[3];           // per axis: zero normal derivative at x = 1 (mirror ghost)
  int nondiv;           // diffusion a Lap u instead of div(a grad u)
  int full;             // F(u) requested instead of g(u) (periodic problems read this;
                        // the stencil gets F through lam_amax = 0 and cadv)
  int ldi, ldo;         // x1 row strides of u/sub/base* and of out* (0: n1, unpadded)
  // MM_SLICED, rows of n1 <= 64 P values (one wave per row): out0 (and out1) are written
  // not in FP64 but as the grid operand of the mode-1 product, split into dS digit
  // planes of rows slice_ld(n1) (dplane bytes per plane) with one exponent per row in
  // dexp, the layout and definition of the separate grid split; out0 of grid row r is
  // operand row r, out1 operand row drow1 + r
  signed char* dig;
  int* dexp;
  int dS;
  int64_t dplane, drow1;
  // with dig: write the chain layout of the chained mode products instead (operand row r
  // is fiber r % n2 of group r / n2, exponent at (r / n2) 256 + r % n2; needs n2 <= 256)
  int dchain;
};
// whether every x1 row of n1 points is covered by one wave of the stencil (the condition
// of the digit output)
bool stencil_row_in_one_wave(int n1);

// Up to kMaxGroups stencil problems of one grid shape, launched together.
struct StencilBatch {
  StencilArgs a[kMaxGroups];
};

// One axis of the pointwise pass of the spectral remainder (spectral.hip).
struct SpecMidArgs {
  double* G;            // remainder accumulator (nondiv: += (a - lam a_max) T1)
  double* T2;           // operand of the outer derivative
  const double* T1;     // inner derivative of u along the axis
  const double* u;
  const double* a;      // a_mumu on the grid
  const double* vel;    // nullable: velocity b_mu on the grid (else the constant beta)
  double lam_amax, beta, beta_bar;
  int64_t n;
  int nondiv;
};

// Whole small 2D Lawson solves in one workgroup (n1, n2 <= 64, FP64).
struct SmallArgs {
  double* u;            // n2 x n1, advanced in place
  const double* a;      // (n2+2) x (n1+2)
  const double* E1;     // n1 x n1 factor exp(tau A_1)
  const double* E2;     // n2 x n2 factor exp(tau A_2)
  int n1, n2, nsteps;
  double tau;
  double ih2[2], cadv[2], lam_amax;
  double r0, r1, r2, r3;
  int* flag;
};
bool small2d_fits(int d, int n1, int n2);
hipError_t launch_lawson_small2d(const SmallArgs& a, bool l2b, hipStream_t s);
// Up to kMaxSmallBatch whole solves in one launch, one workgroup each.
constexpr int kMaxSmallBatch = 16;
struct SmallBatch {
  SmallArgs a[kMaxSmallBatch];
};
hipError_t launch_lawson_small2d_batch(const SmallArgs* a, int count, bool l2b, hipStream_t s);

hipError_t launch_gemm(int prec, GemmArgs& g, hipStream_t s);
// Row stride of a folded factor: f = n - n/2 rounded up to even (16-byte aligned pairs).
__host__ __device__ inline int fold_ld(int n) {
  const int f = n - n / 2;
  return f + (f & 1);
}
// Folded factor of a centrosymmetric n x n matrix E (row-major, row stride n) into Ff:
// rows 0..f-1 Es, rows f..2f-1 Ed, each of f = n - n/2 values (row stride fold_ld(n),
// padding zero), with
// m = n/2: Es_ir = (E_ir + E_i,n-1-r)/2 and Ed_ir = (E_ir - E_i,n-1-r)/2 for r < m, and for
// odd n Es_im = E_im, Ed_im = 0. `count` matrices n^2 apart in E, 2 f fold_ld(n) apart in Ff.
hipError_t launch_fold_factor(double* Ff, const double* E, int n, int count, hipStream_t s);
// Folded form of a stacked factor [E_0 | ... | E_{G-1}] (n rows, row stride G n, every
// block centrosymmetric) into Ff: 2f rows of G fold_ld(n) values, block g's Es and Ed in
// columns g fold_ld(n) .. +fold_ld(n).
hipError_t launch_fold_stacked(double* Ff, const double* E, int n, int G, hipStream_t s);
// Whether launch_gemm runs g as a folded product (FP64, a folded factor for every group,
// a square factor, and fold = 2 or enough tiles to fill the chip).
bool use_fold(const GemmArgs& g, int prec);
// 128 x 64 folded tiles of one group of g.
int64_t fold_tiles(const GemmArgs& g);
// Tile size the launcher takes for g in precision prec (g.tile if set, else 64 when
// 128-tiles would not fill the chip once, and in FP64 32 when 64-tiles would not give
// every compute unit one).
int choose_tile(const GemmArgs& g, int prec);
// MM_SLICED mode product (64 x 64 tiles; factor operand as digit planes).
hipError_t launch_gemm_sliced(GemmArgs& g, hipStream_t s);
// MM_SLICED chained mode product: C (M x F per fiber group) = F_mu (M x K) . V^T, with the
// grid operand V given as digit planes of whole fibers in the chain layout and one
// exponent per fiber. Fiber group g = v Gv + gi of stacked vector v holds F <= 256 fibers.
// A tile computes 32 factor rows against all fibers of one group, so every output row m
// is a whole fiber of the next product: the epilogue writes it as that product's digits
// (linear fiber (v M + m) Gv + gi, i.e. fiber lin % Fn of group lin / Fn with Fn that
// product's fibers per group; positions j; exponent from the row's maximum: the definition
// of the grid split) or, for the last mode, as FP64 values out[v ovs + (m Gv + gi) ldo + j].
// The launcher refuses launches whose chain-layout input or output would not fit the
// given workspace capacities.
struct ChainArgs {
  const signed char* fdig;   // factor digit planes (row stride slice_ld(K), fplane apart)
  const int* fexp;           // factor row exponents
  int64_t fplane;
  const signed char* vdig;   // input fibers' digits in the chain layout (slice_digits.h),
  const int* vexp;           // exponent of fiber j of group g at g 256 + j
  int M, K, F, Gv, nvec;
  int slices;
  signed char* odig;         // digit output in the chain layout (null: FP64 output)
  int* oexp;
  int Fn;                    // fibers per group of the next product (digit output)
  int64_t vcap, vexp_cap;    // bytes and exponents of the input workspace
  int64_t ocap, oexp_cap;    // bytes and exponents of the output workspace
  double* out;               // FP64 output
  int ldo;
  int64_t ovs;
  int wide;                  // 0: eight waves of 32 fibers; 1: four waves of 64 fibers
  // filled by the launcher
  int tiles_m, total, per_xcd;
};
hipError_t launch_gemm_sliced_chain(ChainArgs& c, hipStream_t s);
// Split rows x k (row stride lds) into S digit planes of row stride ldd (plane stride
// rows*ldd bytes, zero for k <= c < ldd) and per-row exponents.
hipError_t launch_slice_rows(signed char* dst, int* exps, const double* src, int rows, int k, int lds, int ldd,
                             int S, hipStream_t s);
hipError_t launch_stencil(int d, const StencilArgs& a, hipStream_t s);
// count (1..kMaxGroups) problems with equal n1, n2, n3 in one launch; each problem's
// outputs are bit-identical to launch_stencil's.
hipError_t launch_stencil_batch(int d, const StencilArgs* a, int count, hipStream_t s);
hipError_t launch_build_circulant(double* M, int n, const double* col, hipStream_t s);
hipError_t launch_spec_react(double* G, const double* u, int64_t n, const double* r, hipStream_t s);
hipError_t launch_spec_mid(const SpecMidArgs& a, hipStream_t s);
hipError_t launch_spec_combine(const double* const (&G)[3], const StencilArgs& a, int64_t n, hipStream_t s);
hipError_t launch_max_reduce(const double* x, int64_t n, double* partial, int nparts, double* out,
                             hipStream_t s);
// last_sub: the entry (n-1, n-2) (sub for a Toeplitz matrix)
hipError_t launch_build_tridiag(double* M, int n, double sub, double diag, double sup, double last_sub,
                                hipStream_t s);
// out = c0*X0 + c1*X1 + c2*X2 + c3*X3 + cI*I (any X may be null); n x n
hipError_t launch_combo(double* out, int n, double c0, const double* X0, double c1, const double* X1,
                        double c2, const double* X2, double c3, const double* X3, double cI,
                        hipStream_t s);
// out = X + s*Y elementwise over count values
hipError_t launch_axpy(double* out, const double* X, double s, const double* Y, int64_t count,
                       hipStream_t st);
// Solve Q X = P in place (X overwrites P); Q is destroyed. `count` independent systems
// with stride n*n each, one workgroup per system (Gaussian elimination, partial pivoting).
hipError_t launch_lu_solve(double* Q, double* P, int n, int count, hipStream_t s);
// dst[r][c0 + c] = w * src[r][c] for an n x n src into a row-major dst with leading dim ldd
hipError_t launch_place_scaled(double* dst, int ldd, int col0, const double* src, int n, double w,
                               hipStream_t s);
hipError_t launch_fill(double* dst, double v, int64_t count, hipStream_t s);
// Joint-eigenbasis scaling: out = ca f_a(tau L) a + cb f_b(tau L) b elementwise, with
// L(k3,k2,k1) = ev1[k1] + ev2[k2] + ev3[k3] (ev3 null in 2D, n3 = 1); b may be null.
enum { MM_EIG_ONE = 0, MM_EIG_EXP = 1, MM_EIG_PHI1 = 2, MM_EIG_PHI2 = 3 };
hipError_t launch_eig_scale(double* out, const double* a, double ca, int fa, const double* b, double cb, int fb,
                            const double* ev1, const double* ev2, const double* ev3, int n1, int n2, int n3,
                            double tau, hipStream_t s);
// The same for periodic axes in the real orthonormal Fourier basis (cos/sin pairs are
// 2 x 2 blocks): sym_mu holds (alpha(m), omega(m)), the symbol of A_mu at wavenumber
// m = 0 .. n_mu/2 (sym3 null in 2D).
hipError_t launch_spec_eig_scale(double* out, const double* a, double ca, int fa, const double* b, double cb, int fb,
                                 const double* sym1, const double* sym2, const double* sym3, int n1, int n2, int n3,
                                 double tau, hipStream_t s);
// out[0] = ||Q||_1, out[1] = ||Q||_inf (device); X = alpha Q^T; out[0] = max |R - I|
hipError_t launch_norms(const double* Q, int n, double* out, hipStream_t s);
hipError_t launch_scaled_transpose(double* X, const double* Q, int n, double alpha, hipStream_t s);
hipError_t launch_resid(const double* R, int n, double* out, hipStream_t s);
// Pre-convert an FP64 factor (rows x k, leading dim lds) for the mixed modes into
// dst (rows x fac_ld(k), zero-padded): prec MM_FP32 -> float, MM_BF16X3/X6 -> S BF16
// slices, slice s at dst + s*rows*fac_ld(k) (elements).
hipError_t launch_convert_factor(int prec, void* dst, const double* src, int rows, int k, int lds,
                                 hipStream_t s);
int factor_slices(int prec);

// Allocation-free exponential action (noalloc.hip): grid values per intermediate of the
// file-scope scratch array, and the per-device resolution of its address (called by
// mm_ctx_create with the device current).
constexpr int64_t kNoAllocMaxDof = (int64_t)1 << 21;
hipError_t noalloc_resolve(int device);

// Grouped stepping (used by lawson_step_batch and the request server). A problem can be
// advanced together with others of its class when it is a finite-difference problem
// (not periodic) stepped by Lawson-Euler or Lawson2b; a class is (d, n, precision,
// digit count, scheme). Small 2D problems that the one-workgroup solver takes run one
// workgroup each, any mix of sizes and step counts.
bool lawson_groupable(const mm_op* op);
bool small2d_fusable(const mm_ctx* ctx, const mm_op* op);
bool same_class(const mm_op* a, const mm_op* b);
mm_status enqueue_lawson_group(mm_ctx* ctx, const mm_op* const* ops, double* const* u, int count, int nsteps,
                               hipStream_t s);
mm_status enqueue_small2d_group(mm_ctx* ctx, const mm_op* const* ops, double* const* u, const int* nsteps,
                                int count, hipStream_t s);

}  // namespace mm

struct mm_timed {
  int kind;
  double work;
  hipEvent_t start, stop;
};

// Digit-plane workspace of grouped sliced launches on one stream (grown on demand).
struct mm_batch_ws {
  hipStream_t stream = nullptr;
  signed char* vdig = nullptr;
  int* vexp = nullptr;
  int64_t vdig_cap = 0, vexp_cap = 0;
};

struct mm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // setup stream
  std::string last_error;
  double* reduce_buf = nullptr;   // partial maxima
  int reduce_parts = 0;
  bool timing = false;            // per-kernel event timing
  int gemm_tile = 0;              // 0 = automatic, else forced 64 or 128
  int graph_steps = 0;            // >0: step calls replay captured graphs of this many steps
  bool small_fused = true;        // small 2D Lawson solves as one-workgroup kernels
  int sliced_chain = 1;           // MM_SLICED chained actions (mm_set_sliced_chain)
  int fold = 1;                   // FP64 folded mode products (mm_set_fold)
  hipStream_t capture = nullptr;  // private stream used only to record graphs
  std::vector<mm_timed> timed;
  size_t timed_used = 0;
  std::vector<mm_batch_ws> bws;   // per stream: grouped sliced launches
};

struct mm_op {
  mm_ctx* ctx = nullptr;
  int d = 3;
  int n[3] = {1, 1, 1};
  int64_t dof = 0;
  double tau = 0, lam = 1, a_max = 0;
  double beta[3] = {0, 0, 0}, beta_bar[3] = {0, 0, 0}, r[4] = {0, 0, 0, 0};
  int family = 0, scheme = 0, q = 0, prec = 0;
  int slices = 0;                      // MM_SLICED digit count
  int bc[3] = {0, 0, 0};               // MM_BC_* per axis
  int form = 0;                        // MM_FORM_*
  // periodic (pseudo-spectral) problems: every axis MM_BC_PERIODIC
  bool periodic = false;
  double length[3] = {0, 0, 0};        // periods
  double amax_mu[3] = {0, 0, 0};       // max of each diagonal diffusion entry
  double* vel = nullptr;               // nullable: d velocity fields (dof each)
  double* dmat[3] = {nullptr, nullptr, nullptr};   // per axis [D1 | D2 | A], n x n each
  bool dmat_owned[3] = {false, false, false};
  double* spec_ws = nullptr;           // per axis G, T1, T2 (dof each)
  hipStream_t spec_side[2] = {nullptr, nullptr};   // streams of the x2 and x3 chains
  hipEvent_t spec_fork = nullptr, spec_join[2] = {nullptr, nullptr};
  bool exact = false;                  // MM_ERK with exact phi1 through the eigenbasis
  int nfac = 1;                        // factors stored per axis
  double* ev[3] = {nullptr, nullptr, nullptr};   // exact: 1D eigenvalues per axis
  int squarings[3] = {0, 0, 0};
  double theta[8] = {0}, weight[8] = {0};
  // device memory owned by the op
  double* a = nullptr;                 // nodal coefficient copy
  std::vector<double*> fac;            // fac[mu] = (1 + q) stacked n_mu x n_mu FP64 factors
  std::vector<bool> fac_owned;
  // FP64 centrosymmetric axes: the first nfold factors of fac[mu] folded ([Es; Ed], 2f rows
  // of stride fold_ld(n_mu), f = n_mu - n_mu/2; launch_fold_factor), null on other axes
  std::vector<double*> ffold;
  std::vector<bool> ffold_owned;
  int nfold = 0;
  // folded forms of the stacked last-axis ERK factors (null unless that axis folds)
  double* f3_stage1_fold = nullptr;
  double* f3_stage2_fold = nullptr;
  double* f3_phi_fold = nullptr;
  double* f3_stage1 = nullptr;         // ERK: [E3(1) | tau w_j E3(theta_j)] or [tau w_j E3]
  double* f3_stage2 = nullptr;         // ERK: [tau/2 w_j E3(theta_j)]
  double* f3_phi = nullptr;            // [w_j E3(theta_j)] for mumode_phi1v
  // mixed modes: pre-converted copies (see GemmArgs), same stacking
  std::vector<void*> fac_lp;
  void* f3_stage1_lp = nullptr;
  void* f3_stage2_lp = nullptr;
  void* f3_phi_lp = nullptr;
  // MM_SLICED: per-row exponents of the digit-plane factors (same stacking)
  std::vector<int*> fac_exp;
  int* f3_stage1_exp = nullptr;
  int* f3_stage2_exp = nullptr;
  int* f3_phi_exp = nullptr;
  double* buf[6] = {nullptr};          // scratch
  int64_t buf_len[6] = {0};
  // Lawson-Euler and Lawson2b keep their stage vectors (buf[0], buf[1]) with x1 rows of
  // ld1 >= n1 values (padded to whole 128-byte lines), dofp values per grid function
  int ld1 = 0;
  int64_t dofp = 0;
  // MM_SLICED: digit planes and fiber exponents of the grid operand of one launch
  signed char* vdig = nullptr;
  int* vexp = nullptr;
  int64_t vdig_len = 0, vexp_len = 0;
  // MM_SLICED Lawson steps: the second digit workspace of chained actions (the mode
  // products alternate between the two)
  signed char* vdig2 = nullptr;
  int* vexp2 = nullptr;
  int64_t vdig2_len = 0, vexp2_len = 0;
  int* flag = nullptr;                 // sticky non-finite flag
  int64_t bytes = 0;                   // device footprint
  // recorded step graph: `gsteps` steps on state `gu` (rebuilt when either changes)
  mutable hipGraphExec_t gexec = nullptr;
  mutable double* gu = nullptr;
  mutable int gsteps = 0;
  mutable hipStream_t gstream = nullptr;   // stream of the last replay
};
