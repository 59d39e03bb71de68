/*
 * mumode.h -- C ABI of the mu-mode exponential-integrator library for MI355X (gfx950).
 *
 * Problem (Sec. 3, eq. (eq:adr) with a scalar diffusion coefficient and constant
 * velocity, on the unit cube with homogeneous Dirichlet data):
 *
 *     u_t = div(a(x) grad u) + beta . grad u + r(u),     r(u) = r0 + r1 u + r2 u^2 + r3 u^3,
 *
 * split as u_t = A u + g(u) (eqs. (eq:adr_equiv), (eq:linop), (eq:nonlin)) with the
 * extracted constant-coefficient operator A = lambda*a_max*Laplacian + beta_bar . grad
 * and a_max = max over the sampled nodes of a (eq. (eq:amaxbeta)). Second-order centred
 * finite differences make A a Kronecker sum A_d (+) ... (+) A_1 of tridiagonal 1D
 * matrices (Sec. 5.2), whose exponential acts on a grid tensor V as the mu-mode
 * product V x_1 exp(tau A_1) x_2 exp(tau A_2) (x_3 exp(tau A_3)) (Sec. 1, Sec. 5.2).
 *
 * Memory layout (all grid functions, device memory, FP64 unless noted):
 *   interior unknowns u[i3][i2][i1], x1 fastest, n1*n2*n3 values (d = 2: n3 = 1);
 *   diffusion coefficient a on all nodes including the boundary,
 *   (n3+2)*(n2+2)*(n1+2) values, x1 fastest; node (i1,i2,i3) sits at (i1 h1, i2 h2, i3 h3),
 *   h_mu = 1/(n_mu + 1).
 *
 * Ownership: the caller owns every grid buffer it passes (u, a, g, F, in, out) and keeps
 * it alive until the work enqueued on it has finished. The library owns mm_ctx, mm_op
 * and mm_server and everything they allocate. mumode_setup copies a.
 *
 * Errors: every call returns an mm_status; none aborts the process. A message for the
 * last failure of a context is available from mm_last_error(ctx). Step and apply calls
 * are stream-ordered and asynchronous: they return MM_OK once the work is enqueued; a
 * device fault or a non-finite solution surfaces at mm_check(op) or a later call.
 * An mm_ctx (and any mm_op made from it) must be used from one host thread at a time.
 * The server calls are thread-safe.
 */
#ifndef MUMODE_H
#define MUMODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MM_OK = 0,
  MM_NOT_READY = 1,   /* solve_poll: the request has not finished                  */
  MM_EINVAL = -1,     /* invalid argument                                          */
  MM_ENOMEM = -2,     /* device allocation failed, or a request exceeds the budget */
  MM_EDEVICE = -3,    /* a HIP runtime call failed                                 */
  MM_EUNSTABLE = -4,  /* the solution became non-finite                            */
  MM_EBUSY = -5,      /* server queue full                                         */
  MM_ENOTFOUND = -6   /* unknown request id                                        */
} mm_status;

/* Arithmetic of the mu-mode contractions. Setup (factors in FP64), the remainder
 * stencil and the stage updates are FP64 in every mode, and so is the state u.
 *   MM_FP64      FP64 MFMA, FP64 accumulation (the plain baseline).
 *   MM_FP32      factors rounded to FP32 at setup, grid operands rounded to FP32
 *                (nearest even) while staged; FP32 MFMA with FP32 accumulation. The
 *                values passed between the passes of one action are FP32.
 *   MM_BF16X3    factors split at setup, grid operands while staged, into two BF16
 *                values x = hi + lo (each nearest even); hi*hi + hi*lo + lo*hi on the
 *                BF16 MFMA with FP32 accumulation; FP32 between passes.
 *   MM_BF16X6    three BF16 slices x = s0 + s1 + s2; the six products s_i*s_j with
 *                i + j <= 2, otherwise as MM_BF16X3.
 *   MM_SLICED    exact slicing: every operand row gets a power-of-two scale and is
 *                written as S balanced base-256 digits in [-128, 127] (S = `slices`,
 *                3..7, default 6); the digit products s + t < S run on the int8
 *                MFMA, where the int32 accumulation is exact, and are combined in
 *                FP64. Error about 2^(-8S) relative to the row scales, whatever K;
 *                FP64 between passes. Needs S * 2^14 * K < 2^31 for every
 *                contraction length K (n, or (q+1) n for the ERK stacked mode). */
typedef enum { MM_FP64 = 0, MM_FP32 = 1, MM_BF16X3 = 2, MM_BF16X6 = 3, MM_SLICED = 4 } mm_prec;

/* Scheme families and members (Appendix).
 *   family MM_LAWSON: MM_LAWSON_EULER  u+ = e^{tau A}(u + tau g(u))
 *                     MM_LAWSON2B      U = e^{tau A}(u + tau g(u)),
 *                                      u+ = e^{tau A}(u + tau/2 g(u)) + tau/2 g(U)
 *                     MM_SLE           stabilized Lawson-Euler u+ = u + tau e^{tau A} F(u)
 *                     MM_LAWSON2A      U = e^{tau/2 A}(u + tau/2 g(u)),
 *                                      u+ = e^{tau A} u + tau e^{tau/2 A} g(U)
 *                     MM_SL2           stabilized Lawson2, alpha = 0.327:
 *                                      U = u + alpha tau e^{alpha tau A} F(u),
 *                                      u+ = u + tau e^{tau/2 A} F(u)
 *                                           + tau/(2 alpha) e^{tau A}(g(U) - g(u))
 *   family MM_ERK:    MM_ETD2RK        second-order ERK with phi1, c2 = 1, in the form
 *                                      U = e^{tau A}u + tau phi1(tau A) g(u),
 *                                      u+ = U + tau/2 phi1(tau A)(g(U) - g(u))
 *                     MM_ERK2P1        the same scheme in the Appendix form
 *                                      U = u + tau phi1(tau A) F(u),
 *                                      u+ = U + tau/2 phi1(tau A)(g(U) - g(u))
 *                     MM_EE            exponential Euler u+ = u + tau phi1(tau A) F(u)
 *                     MM_ERK2P2        second-order ERK with phi2 (Appendix, c2 = 1):
 *                                      U = u + tau phi1(tau A) F(u),
 *                                      u+ = U + tau phi2(tau A)(g(U) - g(u))
 *                                      (MM_EE and MM_ERK2P2 need exact phi, q = 0)
 * phi1(tau A) is replaced by the q-node Gauss-Legendre rule
 *   phi1(tau A) v ~ sum_j w_j exp(theta_j tau A) v,  theta_j, w_j on [0, 1],
 * or (q = 0) evaluated exactly in the joint eigenbasis of the Kronecker sum: with
 * A_mu = L_mu diag(ev_mu) R_mu (closed form for the tridiagonal Toeplitz A_mu),
 *   f(tau A) v = (v x_mu R_mu over mu) scaled by f(tau (ev_1 + ev_2 + ev_3)) x_mu L_mu.
 * On periodic axes L_mu = Q_mu is the real orthonormal Fourier basis (the constant, the
 * cos/sin pair of every wavenumber 0 < m < n/2, the alternating Nyquist vector for even
 * n) and R_mu = Q_mu^T; A_mu is block diagonal there, with 2 x 2 blocks for the pairs
 * (the advection's imaginary symbol), and f acts on the up to eight coefficients of one
 * wavenumber triple through their complex amplitudes.                                */
enum { MM_LAWSON = 0, MM_ERK = 1 };
enum { MM_LAWSON_EULER = 0, MM_LAWSON2B = 1, MM_SLE = 2, MM_LAWSON2A = 3, MM_SL2 = 4 };
enum { MM_ETD2RK = 0, MM_ERK2P1 = 1, MM_EE = 2, MM_ERK2P2 = 3 };

/* Boundary data per axis (Sec. 5.2, eq. (eq:adr3d)): MM_BC_DIRICHLET is zero data at
 * x = 0 and x = 1 (n unknowns at i/(n+1)); MM_BC_NEUMANN is zero data at x = 0 and a zero
 * normal derivative at x = 1 (n unknowns at i/n, i = 1..n, the value beyond x = 1 taken as
 * the mirror u_{n+1} = u_{n-1}, so the 1D operator's last row reads [.., 2, -2]/h^2 and
 * its centred advection vanishes there). Diffusion form: MM_FORM_FLUX is div(a grad u)
 * with face means of the nodal a (eq. (eq:nonlin)); MM_FORM_NONDIV is a Lap u, the form
 * of eq. (eq:adr3d), which reads a at the unknowns only.
 *
 * MM_BC_PERIODIC (every axis at once; Sec. 4.1, 4.2 and 5.1) selects the Fourier
 * pseudo-spectral discretization on n equispaced points per period length[mu]: a is then
 * the diagonal diffusion tensor, d fields of n1 n2 (n3) values (a_11 first) on those
 * points, and `velocity` (nullable) holds d fields b_mu entering as div(b u) (without it
 * the constant beta enters as beta . grad u). The derivatives along an axis multiply the
 * discrete Fourier coefficients by i kappa (zero at the Nyquist wavenumber of even n) and
 * by -kappa^2, kappa = 2 pi m / length; the library applies them, and the exponentials
 * of A = sum_mu lam a_mumu^max d_mumu + beta_bar_mu d_mu (a^max the grid maximum of each
 * a_mumu), as mode products with dense circulant n x n matrices whose first columns it
 * sums from their Fourier symbols in FP64 at setup (no FFT on the step path). g follows
 * eq. (eq:nonlin): sum_mu d_mu((a_mumu - lam a^max_mumu) d_mu u) (MM_FORM_NONDIV:
 * (a_mumu - lam a^max_mumu) d_mumu u) + sum_mu d_mu((b_mu - beta_bar_mu) u) + r(u), and
 * F = A u + g. Exact phi (q = 0) goes through the Fourier basis (above). Their remainder
 * works in scratch held by the op (three grid functions per axis) and runs the chain of
 * every axis after the first on a side stream of the op, forked from and joined back to
 * the call's stream with events (so it stays stream-ordered and can be captured); calls
 * on one periodic op must not overlap (on different streams), as for the step calls of
 * every op.                                                                          */
enum { MM_BC_DIRICHLET = 0, MM_BC_NEUMANN = 1, MM_BC_PERIODIC = 2 };
enum { MM_FORM_FLUX = 0, MM_FORM_NONDIV = 1 };

typedef struct {
  int d;                 /* 2 or 3                                                    */
  int n[3];              /* unknowns per axis, x1 first (n[2] ignored if d=2)         */
  const double* a;       /* device, nodal diffusion coefficient on the padded nodes
                            (n3+2)(n2+2)(n1+2): the unknowns plus one node per side;
                            beyond a Neumann face the flux form reads the extra node,
                            which should hold the mirror value a(x_{n-1})             */
  double beta[3];        /* constant velocity                                         */
  double r[4];           /* reaction coefficients r0..r3                              */
  double lambda;         /* extraction factor, eq. (eq:linop)                         */
  double beta_bar[3];    /* advection moved into A, eq. (eq:linop)                    */
  int bc[3];             /* MM_BC_* per axis (zero: Dirichlet)                        */
  int form;              /* MM_FORM_* (zero: flux form)                               */
  double length[3];      /* MM_BC_PERIODIC: period of each axis (ignored otherwise)   */
  const double* velocity;/* MM_BC_PERIODIC: nullable device pointer, d velocity fields
                            of n1 n2 (n3) values (ignored otherwise)                  */
} mm_problem;

typedef struct mm_ctx mm_ctx;
typedef struct mm_op mm_op;
typedef struct mm_server mm_server;

/* Create a context on HIP device `device` (it becomes current on the calling thread).
 * *out is set to NULL first, so it is NULL after any failure. MM_EINVAL for out ==
 * NULL, MM_EDEVICE for a device that does not exist, MM_ENOMEM. */
mm_status mm_ctx_create(int device, mm_ctx** out);
void mm_ctx_destroy(mm_ctx* ctx);
/* Message of the last failure on this context (static storage, never NULL). */
const char* mm_last_error(const mm_ctx* ctx);
/* Library version string (static storage). */
const char* mm_version(void);

/* Build the operator for one problem and time step (Sec. 3 extraction, Sec. 5.2
 * Kronecker factors): a_max by a device reduction, the tridiagonal A_mu, and on the
 * device in FP64 the dense factors E_mu(c) = exp(c tau A_mu) by [13/13] Pade
 * scaling-and-squaring for every c the scheme needs (c = 1 and the quadrature nodes
 * theta_j for MM_ERK), plus the FP32, BF16-slice or digit-plane forms the precision
 * needs. Returns after the setup has finished. quad_nodes (q) is 1..7 for MM_ERK and
 * ignored for MM_LAWSON; q = 0 selects exact phi1 through the eigenbasis (FP64 only;
 * Dirichlet axes need |beta_bar_mu| h_mu < 2 lambda a_max so that the eigenvalues are
 * real, axes with a zero normal derivative at x = 1 need beta_bar_mu = 0, periodic axes
 * take any beta_bar_mu), and the op then also stores R_mu and L_mu. slices: digit count of MM_SLICED (0 = 6,
 * else 3..7), ignored by the other precisions. `a` must be complete when the call is
 * made (the copy runs on the context's own stream, which does not wait for others).
 * Errors: MM_EINVAL (d, n < 1, tau <= 0 or not finite, unknown family/scheme/prec/bc/form,
 * exact phi1 with beta_bar_mu != 0 on an axis with a zero normal derivative,
 * slices out of range, exact phi1 with another precision or complex eigenvalues,
 * a == NULL), MM_ENOMEM, MM_EDEVICE. */
mm_status mumode_setup(mm_ctx* ctx, const mm_problem* prob, double tau, int family, int scheme,
                       int quad_nodes, int prec, int slices, mm_op** out);
/* Release the op. Work enqueued with it must have completed (synchronise first). */
void mumode_destroy(mm_op* op);

/* Wait until all work on the context's device has completed (hipDeviceSynchronize). */
mm_status mm_synchronize(mm_ctx* ctx);

/* The extracted maximum a_max and the scaling exponent s used for factor c = 1 along
 * axis mu (diagnostics). Periodic problems: a_max is the largest of the per-axis maxima
 * a_mumu^max, and s = 0 (their factors come from the Fourier symbol, not from Pade). */
mm_status mumode_info(const mm_op* op, double* a_max, int* squarings);

/* Copy the FP64 factor of index j of axis mu into host memory (n_mu*n_mu values,
 * row-major E[row][col]): exp(c tau A_mu) with c = 1 (j = 0) or c = theta_j (j = 1..q);
 * with exact phi1 (q = 0), j = 1 is R_mu and j = 2 is L_mu; Lawson2a and stabilized
 * Lawson2 add c = 1/2 (j = 1) and, for the latter, c = alpha (j = 2). */
mm_status mumode_get_factor(const mm_op* op, int mu, int j, double* host_out);

/* Remainder (eq. (eq:nonlin)) on the grid, flux-form centred differences, face
 * coefficient = mean of the two nodal values, zero Dirichlet ghosts:
 *   g(u) = sum_mu [(abar+ - lambda a_max)(u+ - u) - (abar- - lambda a_max)(u - u-)]/h_mu^2
 *        + sum_mu (beta_mu - beta_bar_mu)(u+ - u-)/(2 h_mu) + r(u).
 * F (nullable) receives the unsplit right-hand side F(u) = A u + g(u).
 * u, g, F: device, n1*n2*n3 values; must not alias. Enqueued on `stream`. */
mm_status remainder_eval(mm_ctx* ctx, const mm_op* op, const double* u, double* g, double* F,
                         void* stream);

/* out = in x_mu M_mu over all axes, three (two) mu-mode passes in the op's precision,
 * with M the factors of index j (see mumode_get_factor): exp(c tau A) in for j = 0 and
 * the quadrature nodes, the eigenbasis transforms R and L with exact phi1. in/out:
 * device, may alias. */
mm_status mumode_expv(mm_ctx* ctx, const mm_op* op, int j, const double* in, double* out,
                      void* stream);

/* out = phi1(tau A) in (MM_ERK): the q-node quadrature sum_j w_j exp(theta_j tau A) in,
 * or exact through the eigenbasis when q = 0. */
mm_status mumode_phi1v(mm_ctx* ctx, const mm_op* op, const double* in, double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * allocation-free serving loops, harnesses that forbid hipMalloc): the FP64 exponential
 * action of mumode_expv, out = in x_1 E_1 x_2 E_2 (x_3 E_3), with caller-owned factors
 * and no operator. E[mu]: device, row-major n[mu] x n[mu] (for instance exp(tau A_mu)
 * from mumode_get_factor, uploaded); n: d sizes, x1 first; in, out: device,
 * n1*n2(*n3) values, may alias. The two intermediates live in a scratch array of
 * 2 x 2^21 doubles (32 MiB) that the library holds on each device from the first
 * mm_ctx_create on it until the process ends; the call allocates nothing. Limit:
 * n1*n2*n3 <= 2^21 (2,097,152 grid values), else MM_EINVAL with a message. The scratch is
 * fully written before it is read in every call, so no state carries over, but every
 * call on one device shares it: calls that overlap in time on one device (on different
 * streams or threads) race, and the caller must serialise them. Results are
 * bit-identical to mumode_expv with the same factors. Enqueued on `stream`;
 * MM_EDEVICE if a launch fails. */
mm_status mumode_expv_noalloc(mm_ctx* ctx, int d, const int* n, const double* const* E, const double* in,
                              double* out, void* stream);

/* Advance u (device, in place) by nsteps Lawson steps (family MM_LAWSON). */
mm_status lawson_step(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, void* stream);

/* Grouped Lawson steps (Appendix, the Lawson-Euler and Lawson2b schemes): advance u[i]
 * (device, in place, n1*n2*n3 values each) by nsteps steps of ops[i], for i < count
 * (1..8). Every op must come from ctx, be a finite-difference (not periodic) MM_LAWSON
 * operator with scheme MM_LAWSON_EULER or MM_LAWSON2B, and share op 0's d, n, precision,
 * digit count and scheme; each op keeps its own coefficients, tau and factors. No two
 * entries may share an op or a state. Each pass of a step is one launch for all count
 * problems (the stencil, and one grouped mode product per axis), so problems too small
 * to fill the GPU alone fill it together; small 2D problems that lawson_step solves in
 * one workgroup run one workgroup each in a single launch. Results are bit-identical to
 * lawson_step on each op alone. MM_SLICED groups use a digit workspace the context
 * keeps per stream (allocated stream-ordered on first use and grown when a larger group
 * needs it). Errors: MM_EINVAL (mismatched or invalid entries), MM_ENOMEM, MM_EDEVICE;
 * enqueued on `stream`, asynchronous like lawson_step. */
mm_status lawson_step_batch(mm_ctx* ctx, const mm_op* const* ops, double* const* u, int count, int nsteps,
                            void* stream);

/* Advance u (device, in place) by nsteps ERK steps (family MM_ERK). */
mm_status erk_step(mm_ctx* ctx, const mm_op* op, double* u, int nsteps, void* stream);

/* Wait for the op's work on `stream` and report MM_EUNSTABLE if any step produced a
 * non-finite value since the op was created (the flag is sticky). */
mm_status mm_check(mm_ctx* ctx, const mm_op* op, void* stream);

/* Per-kernel timing (diagnostics). While enabled, every kernel launch the context
 * enqueues is bracketed by two HIP events recorded on the launch's own stream, and the
 * launch's algorithmic work is recorded with it (mode products: 2*M*N*K flops per
 * batch, padding excluded; stencil: grid points). kind: MM_KIND_STENCIL, MM_KIND_GEMM_K
 * (mode-1 kernel, both operands read along k), MM_KIND_GEMM_N (modes 2..d, the grid
 * operand read along n) or MM_KIND_FUSED (whole small-2D solves, work = mode-product
 * flops). mm_timing_read synchronises the recorded events and returns
 * the totals since the last enable. */
enum { MM_KIND_STENCIL = 0, MM_KIND_GEMM_K = 1, MM_KIND_GEMM_N = 2, MM_KIND_FUSED = 3 };
mm_status mm_timing_enable(mm_ctx* ctx, int enable);
mm_status mm_timing_read(mm_ctx* ctx, int kind, int64_t* launches, double* total_ms, double* work);

/* Workgroup tile of the mode-product kernels launched through this context (tuning and
 * tests). tile = 0 (default): 128 x 128 tiles, or 64 x 64 when a launch has fewer
 * 128-tiles than the chip holds at once, or in FP64 32 x 32 when it has fewer 64-tiles
 * than the chip has compute units; 32, 64 or 128 force that size (32 applies to FP64
 * launches, the other precisions take 64 then). FP64 results are bit-identical across
 * tile sizes (every output's sum over k runs in the same order); in the other precisions
 * 64 and 128 agree likewise. Other values: MM_EINVAL. Takes effect for launches enqueued
 * after the call. */
mm_status mm_set_gemm_tile(mm_ctx* ctx, int tile);

/* Small 2D Lawson solves (n1, n2 <= 64, FP64, Lawson-Euler or Lawson2b) run their whole
 * time loop in one workgroup: state and stage vectors in LDS, the same stencil
 * arithmetic and mode products on the FP64 matrix cores, one launch per lawson_step
 * call. enable = 0 launches them step by step like larger problems (tests, timing).
 * Default: enabled. Results agree with the launched path to rounding. */
mm_status mm_set_small_fused(mm_ctx* ctx, int enable);

/* Exact-slice (MM_SLICED) Lawson-Euler and Lawson2b steps on finite-difference grids with
 * every n_mu <= 256 can run their exponential action as a chain of mode products whose
 * epilogues write the next product's digit planes directly (no separate split passes):
 * a workgroup covers 32 factor rows against a whole fiber group, so the exponent of every
 * next-mode fiber is taken from the complete fiber, as the split pass takes it, and the
 * results are bit-identical to the unchained path. mode = 0: off; 1 (default): on when
 * every n_mu > 128 (smaller axes leave most of a 256-fiber tile idle); 2: on wherever
 * possible (eight waves of 32 fibers); 3: as 2 with four waves of 64 fibers. Other modes:
 * MM_EINVAL. */
mm_status mm_set_sliced_chain(mm_ctx* ctx, int mode);

/* FP64 mode products along axes whose extracted operator is a symmetric Toeplitz matrix
 * (zero Dirichlet data at both ends, beta_bar_mu = 0, Sec. 2, eq. (eq:linop)): there
 * every factor exp(c tau A_mu) is centrosymmetric (E_ij = E_{n-1-i,n-1-j}), so a product
 * y = E x splits into the sums and differences of mirrored entries of x and two products
 * with half-size factors, at half the multiply-adds; the results agree with the plain
 * product to rounding. Applies to the exp actions of the Lawson and ERK steps and of
 * mumode_expv (not to stacked quadrature factors). mode = 0: off; 1 (default): on for
 * products with at least 192 folded tiles (128 grid rows or columns x 64 folded
 * positions) per problem, smaller ones keep the plain kernel's smaller tiles; 2: always.
 * The decision does not depend on how many problems share a launch. Other modes:
 * MM_EINVAL. */
mm_status mm_set_fold(mm_ctx* ctx, int mode);

/* Step replay through HIP graphs (launch-bound small problems). steps = 0 (default):
 * lawson_step / erk_step launch their kernels one by one. steps = G > 0: a call with
 * nsteps >= G records G steps on that state buffer into a graph once (kept by the op and
 * recorded again when the buffer or G changes) and replays it nsteps / G times on the
 * call's stream, then launches the remaining steps directly. Kernels, their order and
 * therefore the results are the same as without graphs. Ignored while per-kernel timing
 * is enabled. steps outside [0, 4096]: MM_EINVAL. */
mm_status mm_set_graph_steps(mm_ctx* ctx, int steps);

/* ---------------------------------------------------------------------------------
 * Serving: continuous batching of Lawson2b solves. Four admission threads, each with
 * its own context and stream, copy a request's data to the device and build its
 * operator as soon as a slot and its device-memory footprint fit. A step thread then
 * batches at the granularity of steps: finite-difference requests of equal (d, n,
 * precision, digit count) form a class on one of four streams, and each tick enqueues
 * the next few steps of every member together through grouped launches (lawson_step_batch's
 * kernels, up to eight requests per launch), so requests join and leave the group
 * between ticks as they arrive and finish; at most two ticks per class are in flight.
 * Small 2D requests (the one-workgroup solver's sizes, FP64) run whole, up to sixteen
 * per launch; periodic requests run alone on the least loaded stream. Finished
 * requests are retired (result copied back, memory released) as their events fire.
 * A request's result does not depend on what else is being served (bit for bit).
 * ------------------------------------------------------------------------------- */
typedef struct {
  int d;
  int n[3];
  const double* a;       /* HOST, nodal coefficient incl. boundary (copied)           */
  const double* u0;      /* HOST, interior initial data (copied)                      */
  double beta[3];
  double r[4];
  double lambda;
  double beta_bar[3];
  double tau;
  int steps;
  int prec;              /* mm_prec                                                   */
  int slices;            /* digit count for MM_SLICED (0 = 6)                          */
  int bc[3];             /* MM_BC_* per axis (zero: Dirichlet), as in mm_problem      */
  int form;              /* MM_FORM_* (zero: flux form)                               */
  double length[3];      /* MM_BC_PERIODIC: periods, as in mm_problem                 */
  const double* velocity;/* MM_BC_PERIODIC: nullable HOST pointer, d velocity fields
                            (copied); for periodic requests `a` holds the d diagonal
                            diffusion fields of n1 n2 (n3) values each                */
} mm_request;

typedef struct {
  double t_submit;       /* seconds on the server clock                               */
  double t_admit;
  double t_done;
  int64_t bytes;         /* device footprint charged at admission                     */
  int steps;
  int status;            /* mm_status of the solve                                    */
} mm_stats;

/* max_active: concurrent solves on the device; hbm_budget: bytes the active solves may
 * hold (0 = 90% of free device memory at creation). *out is set to NULL first (when out
 * is not NULL). MM_EINVAL for out == NULL or max_active < 1. */
mm_status mm_server_create(int device, int max_active, int64_t hbm_budget, mm_server** out);
/* Stop taking requests, run every queued and running request to its end, then release
 * the server; results that were not polled are discarded. */
void mm_server_destroy(mm_server* srv);
/* Copy the request in and queue it; returns its id. MM_ENOMEM if the request alone
 * exceeds the budget, MM_EINVAL for a malformed request. */
mm_status solve_submit(mm_server* srv, const mm_request* req, uint64_t* id);
/* MM_NOT_READY while queued or running; otherwise the request's final status. On
 * MM_OK the solution is copied to u_out (HOST, may be NULL) and stats filled (may be
 * NULL); the request is forgotten after a non-NOT_READY return. */
mm_status solve_poll(mm_server* srv, uint64_t id, double* u_out, mm_stats* stats);
/* Seconds on the server clock (same clock as mm_stats). */
double mm_server_clock(const mm_server* srv);

/* What the step thread has launched since the server was created (diagnostics):
 * problem_steps / group_steps is the mean number of requests per grouped launch. */
typedef struct {
  int64_t ticks;           /* class ticks enqueued                                      */
  int64_t group_launches;  /* grouped step sequences (per tick, per group of up to 8)   */
  int64_t group_steps;     /* steps those sequences enqueued                            */
  int64_t problem_steps;   /* request-steps they advanced                               */
  int64_t small_launches;  /* launches of the one-workgroup small-2D solver             */
  int64_t small_solves;    /* whole solves in those launches                            */
  int64_t single_solves;   /* requests stepped on their own (periodic problems)         */
} mm_server_counters;
mm_status mm_server_read_counters(mm_server* srv, mm_server_counters* out);

#ifdef __cplusplus
}
#endif
#endif /* MUMODE_H */
