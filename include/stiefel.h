/*
 * stiefel.h - C ABI of the MI355X (gfx950) PLAM / PCAL solver library.
 *
 * Solves  min f(X)  s.t.  X^T X = I_p,  X in R^{n x p}, 2p <= n  (Section 1 of
 * Gao, Liu, Yuan, "Parallelizable Algorithms for Optimization Problems with
 * Orthogonality Constraints") with
 *   PLAM (Algorithm 2): X <- X - grad_X L_beta(X, Lam) / eta,
 *                       Lam = Psi(grad f(X)^T X)        (Section 3.1)
 *   PCAL (Algorithm 3): the same point with every column scaled to unit
 *                       2-norm, Lam optionally corrected by
 *                       Phi(X^T grad_X L_beta(X, Psi(.)))  (Section 3.2)
 * and one CholeskyQR2 orthonormalization of the last iterate (the
 * post-process of Section 5.3 / Table 2).
 *
 * Objective families (the test problems of Section 5.2):
 *   f(X) = 1/2 tr(X^T (L + Diag v) X) + alpha/4 rho^T L^{-1} rho,
 *   rho  = diag(X X^T),
 * with L the unscaled 1D Dirichlet Laplacian tridiag(-1,2,-1)
 * (STF_KIND_STENCIL1D) or the 7-point Dirichlet Laplacian on an nx*ny*nz grid
 * (STF_KIND_STENCIL3D), or the quadratic f(X) = 1/2 tr(X^T A X) with a dense
 * symmetric A (STF_KIND_DENSE).
 *
 * Conventions for every entry point
 *   - Matrices are row-major.  X is n x p with row r holding grid point r;
 *     for 3D grids r = x + nx*(y + ny*z).
 *   - Pointers are DEVICE pointers unless marked "host".  The caller owns all
 *     memory; the library never allocates or frees device memory and keeps no
 *     global state, so calls on different streams with different workspaces
 *     are independent.
 *   - All device work is enqueued on `stream`; the solve entry points return
 *     after the final status has been read back (host-synchronous).
 *   - Return codes: STF_OK (0), STF_MAX_ITER (1) or STF_TOL_UNMET (2) (a
 *     result is still filled), or a negative STF_E_* code; stf_strerror()
 *     names them.  No C++ exception crosses this boundary.
 */
#ifndef STIEFEL_H
#define STIEFEL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- enums ------------------------------------------------------------- */
#define STF_KIND_STENCIL1D 0
#define STF_KIND_STENCIL3D 1
#define STF_KIND_DENSE     2

#define STF_F64 0
#define STF_F32 1

/* algorithm: PLAM (Algorithm 2), PCAL (Algorithm 3), or the retraction-based
 * comparator MOptQR of Table 1 with the Cholesky-QR retraction of Section 5.5
 * (float64 only; mult_rule and beta are not used) */
#define STF_PLAM   0
#define STF_PCAL   1
#define STF_MOPTQR 2

/* multiplier: eq. (Lambda1) Psi(G^T X); eq. (lambda2) adds the Phi term (PCAL);
 * DUAL is the dual ascent of the augmented Lagrangian method, eq. (Lambda-alm),
 * Lam^k = Lam^{k-1} - beta (X^k^T X^k - I) from Lam^0 = Psi(G^0^T X^0): Step 3
 * of Algorithms 2 / 3 replaced as in PLAM-DA / PCAL-DA of Section 5.3 */
#define STF_MULT_PSI     0
#define STF_MULT_PSI_PHI 1
#define STF_MULT_DUAL    2

/* proximal parameter eta (Section 5.1): constant, differential, BB1, BB2,
 * alternating BB (BB1 at odd k, BB2 at even k) */
#define STF_ETA_CONST 0
#define STF_ETA_DIFF  1
#define STF_ETA_BB1   2
#define STF_ETA_BB2   3
#define STF_ETA_ABB   4

/* BB pair: STANDARD uses S = X^k - X^{k-1}, Y = gradL^k - gradL^{k-1} for
 * eta^k; LAGGED uses S^{k-1}, Y^{k-1} in the BB quotients as printed in
 * Section 5.1.  The differential rule is printed with the newest pair and
 * uses it under both settings. */
#define STF_BB_STANDARD 0
#define STF_BB_LAGGED   1

/* arithmetic of the iteration:
 *   FP64  - X, G in float64, float64 MFMA / VALU everywhere;
 *   FP32  - X, G in float32 with a float64 master iterate, float32 MFMA
 *           products, float64 accumulation of every reduction over n,
 *           float64 p x p stage;
 *   MIXED - as FP32, but the Gram products use the two-way bf16 split (three
 *           bf16 MFMA products, float32 tile accumulation) and the row-block
 *           product X M_L the exact three-way bf16 split (six products).
 * Both float32 forms stall near relative KKT 5e-6 (see switch_tol).  The
 * p x p multiplier stage, the KKT test and CholeskyQR2 are float64 in every
 * mode. */
#define STF_PREC_FP64    0
#define STF_PREC_FP32    1
#define STF_PREC_MIXED   2
/* MIXED32 - the MIXED kernels with the iterate kept in float32 only (no
 *           float64 master: the stencil and the update read and write the
 *           float32 X); the float64 hand-over starts from that X. */
#define STF_PREC_MIXED32 3

/* ---- return codes -------------------------------------------------------- */
#define STF_OK               0   /* the float64 check of the returned point meets tol */
#define STF_MAX_ITER         1
#define STF_TOL_UNMET        2   /* the in-loop stop test was met, but the float64
                                    KKT of the returned point is above tol */
#define STF_E_INVALID       -1   /* bad argument: p <= 0, n < 2p, NULL, dtype, sizes */
#define STF_E_DIVERGED      -2   /* non-finite values or ||X^T X - I||_F above feas_blowup */
#define STF_E_HIP           -3   /* a HIP runtime call failed */
#define STF_E_UNSUPPORTED   -4   /* option combination not supported */
#define STF_E_WORKSPACE     -5   /* workspace smaller than stf_workspace_size() */
#define STF_E_CHOLESKY      -6   /* CholeskyQR2 met a non-positive pivot (rank-deficient X) */
#define STF_E_SCRATCH       -7   /* the problem needs more than the library's static
                                    scratch buffer (stf_gram_noalloc) */

/* ---- problem descriptor ---------------------------------------------------
 * The objective is
 *   f(X) = 1/2 tr(X^T H0 X B) + tr(Glin^T X) + alpha/4 rho^T L^{-1} rho
 *          - 3/4 gamma rho^T rho^{1/3},        rho = diag(X X^T),
 * with H0 = L + Diag v (stencil kinds) or A (dense kind), B = I when NULL:
 * Problems 1 and 3 of Section 5.2 (Glin, B NULL, gamma 0), Problem 2 (Glin),
 * Problem 4 (B) and Problem 6 (gamma, the exchange term).
 * kind   : STF_KIND_*
 * n, p   : sizes, 1 <= p, 2p <= n (Section 1); p <= 4096
 * grid   : (nx, ny, nz); STENCIL1D requires (n, 1, 1); STENCIL3D nx*ny*nz == n
 * alpha  : weight of the Hartree-like term alpha/4 rho^T L^{-1} rho (stencil kinds)
 * v      : device, float64, length n: diagonal potential added to L; may be NULL
 * A      : device, dense symmetric n x n (STF_KIND_DENSE), dtype A_dtype
 *          (STF_F64 or STF_F32); its symmetry is assumed, not checked.  A
 *          float32 A serves every precision form (the float64 form widens it
 *          exactly; the MIXED forms take A X in split bf16, three bf16 MFMA
 *          products with float32 accumulation); a float64 A only STF_PREC_FP64.
 * block  : STENCIL1D only: L = Diag(L_1, ..., L_s) with tridiag(-1,2,-1)
 *          blocks of this order (the last one shorter when it does not divide
 *          n), the operator of the parallel experiments of Section 5.5;
 *          0 = one block (the whole tridiagonal matrix)
 * gamma  : exchange weight of Problem 6 (stencil kinds); 0 = no exchange term.
 *          Its gradient -2 gamma Diag(rho^{1/3}) X enters the row diagonal.
 * Glin   : device, float64, n x p row-major, or NULL: the linear term of
 *          Problem 2 (gradient Glin)
 * B      : device, float64, p x p symmetric, or NULL: the right factor of
 *          Problem 4 (gradient H0 X B); only with alpha = gamma = 0.
 * With Glin or B the product X^T grad f(X) is not symmetric: the iteration
 * then forms the whole of X^T G instead of its upper blocks.                */
typedef struct stf_problem {
    int32_t kind;
    int32_t p;
    int64_t n;
    int32_t grid[3];
    int32_t A_dtype;
    double alpha;
    const double* v;
    const void* A;
    int32_t block;
    int32_t reserved;
    double gamma;
    const double* Glin;
    const double* B;
} stf_problem;

/* ---- options --------------------------------------------------------------
 * beta        : penalty parameter of L_beta (Section 5.1)
 * eta0        : eta at k = 0 (the paper leaves it open; an input here)
 * eta_const   : gamma of STF_ETA_CONST
 * tol         : stop when ||G - X Psi(G^T X)||_F <= tol * (same at X^0)
 *               (Section 5.1; 0 runs exactly max_iter updates)
 * max_iter    : number of updates at most
 * kkt_every   : evaluate the stop test every kkt_every iterations (>= 1)
 * orth_final  : 1 = CholeskyQR2 of the returned iterate (float64)
 * check_every : the host reads the device "done" flag every check_every
 *               iterations (>= 1); iterations after "done" are no-ops
 * use_graph   : 1 = replay the iteration chunk as a captured HIP graph
 *               (ignored on the legacy default stream, which cannot be captured)
 * profile     : 1 = bracket every kernel group of every iteration with HIP
 *               events (no graph) and report per-group times in
 *               stf_result.kernel_ms / prof_iters
 * fused       : 1 = single-pass iteration: eta^k and the PCAL column norms
 *               nu^k are found before the row-block pass from p x p float64
 *               quantities (the lagged Barzilai-Borwein pair of Section 5.1,
 *               and ||X_c - gradL_c / eta||^2 expanded through X^T X, X^T G,
 *               M_L and the column sums of G^2 taken with the Gram products),
 *               so that the pass that forms gradL^k also writes X^{k+1} and
 *               its row sums of squares: one read of X, G and gradL^{k-1} per
 *               iteration instead of two.  Needs bb_index = STF_BB_LAGGED,
 *               eta_rule other than STF_ETA_DIFF, PLAM or PCAL, p > 64, and
 *               precision STF_PREC_FP64 or STF_PREC_MIXED32 (the latter with
 *               p <= 384); else STF_E_UNSUPPORTED.  The iterates are those of
 *               the two-pass form up to rounding.  0 = two passes.
 * feas_blowup : divergence threshold on ||X^T X - I||_F (e.g. 1e3)
 * switch_tol  : STF_PREC_FP32 / STF_PREC_MIXED only; 0 = never.  Once the
 *               stop test of iteration k finds ||G - X Psi||_F <= switch_tol
 *               times the same at X^0 (and above tol), iteration k is redone
 *               in float64 from the float64 master iterate, with the eta,
 *               column norms and previous gradL carried over, and the solve
 *               continues in float64 (stf_result.switch_iter = k).  The float32
 *               forms stall where the rounding noise of their products (the
 *               row-block product X M_L and the Grams) dominates the
 *               Barzilai-Borwein quotients; this finishes the descent exactly.
 *               The hand-over also happens, above switch_tol, once 100
 *               iterations have passed without a new smallest stop-test value
 *               (a float32 descent that wanders instead of converging).  If
 *               the stop-test value at such a hand-over exceeds the one at X^0
 *               (the float32 iterate has left the neighbourhood of the
 *               manifold), the float32 iterate is discarded and the float64
 *               phase restarts from X^0 (stf_result.restarted = 1): the solve
 *               then returns what the float64 form returns from X^0 rounded
 *               to float32.  The workspace keeps a float32 copy of X^0 for it.
 * history     : device, (max_iter + 1) x 4 float64, or NULL: row k receives
 *               { ||G - X Psi||_F (NaN when the stop test was not due),
 *                 ||X^T X - I||_F, eta^k (NaN on the last row), k } as
 *               iteration k finishes (the per-iteration record of Figs. 1-5) */
typedef struct stf_options {
    int32_t variant;
    int32_t mult_rule;
    int32_t eta_rule;
    int32_t bb_index;
    int32_t precision;
    int32_t max_iter;
    int32_t kkt_every;
    int32_t orth_final;
    int32_t check_every;
    int32_t use_graph;
    int32_t profile;
    int32_t fused;
    double beta;
    double eta0;
    double eta_const;
    double tol;
    double feas_blowup;
    double switch_tol;
    double* history;
} stf_options;

/* ---- result (host struct) -------------------------------------------------
 * status  : STF_OK / STF_MAX_ITER / STF_TOL_UNMET / STF_E_DIVERGED
 * iters   : index k of the returned iterate X^k (number of updates made)
 * kkt0    : ||G - X Psi(G^T X)||_F at X^0 (iteration precision)
 * kkt_abs : the same at the returned point, float64 (after CholeskyQR2 if
 *           orth_final), kkt_rel = kkt_abs / kkt0
 * feas    : ||X^T X - I||_F at the returned point, float64
 * fval    : f at the returned point, float64
 * eta_last: the last eta used
 * ms_loop : wall time of the iteration loop (device events)
 * ms_orth : wall time of CholeskyQR2 + the float64 final evaluation
 * kernel_ms[STF_NPROF] : with opt->profile, summed device time of each
 *           kernel group (STF_PROF_*) over prof_iters iterations.  GRAD, GRAM,
 *           RESIDUAL and UPDATE each bracket exactly one kernel launch;
 *           HARTREE brackets the six sine-transform passes; STAGE1 the
 *           reduction of the Gram partials, the p x p stage, the p x p KKT
 *           products (and the split of M_L in the mixed form); STAGE2 the
 *           column-dot reduction and the step-size / stop stage.  In the
 *           single-pass form (fused) STAGE1 also holds the S M_L product and
 *           the eta / nu stage, and UPDATE brackets the reduction of the row
 *           sums of squares into rho (no launch when no term needs rho)
 * switch_iter : iteration at which a float32 / mixed solve continued in
 *           float64 (see switch_tol), or -1
 * restarted : 1 when that float64 phase restarted from X^0 (see switch_tol):
 *           iters then counts the float64 iterations from X^0, after the
 *           switch_iter discarded float32 ones; history holds the float64
 *           rows from 0 (later rows of the float32 phase are left); 0 else
 * reserved  : set to 0                                                       */
#define STF_PROF_HARTREE  0
#define STF_PROF_GRAD     1
#define STF_PROF_GRAM     2
#define STF_PROF_STAGE1   3
#define STF_PROF_RESIDUAL 4
#define STF_PROF_STAGE2   5
#define STF_PROF_UPDATE   6
#define STF_NPROF         7
typedef struct stf_result {
    int32_t status;
    int32_t iters;
    double kkt0;
    double kkt_abs;
    double kkt_rel;
    double feas;
    double fval;
    double eta_last;
    double ms_loop;
    double ms_orth;
    double kernel_ms[8];
    int32_t prof_iters;
    int32_t switch_iter;
    int32_t restarted;
    int32_t reserved;
} stf_result;

/* Bytes of device workspace needed by stf_solve / plam_solve / pcal_solve and
 * by every step-level entry point for this problem (opt may be NULL: then the
 * largest requirement over the precision modes is returned). */
size_t stf_workspace_size(const stf_problem* prob, const stf_options* opt);

/* Run PLAM or PCAL (opt->variant) from X^0.
 *   X       : device, n x p, float64 (precision FP64) or float32 (FP32 and
 *             MIXED); in: X^0, out: the returned iterate (after CholeskyQR2
 *             when orth_final, rounded to X's dtype)
 *   X64_out : device, n x p float64, may be NULL: the float64 result
 *   Lam_out : device, p x p float64, may be NULL: Psi(grad f(X)^T X) at the
 *             returned point (the multiplier of eq. (closed-multi))
 *   ws      : device workspace of ws_bytes >= stf_workspace_size(prob, opt)
 *   res     : host, filled on return codes >= 0 and on STF_E_DIVERGED */
int stf_solve(const stf_problem* prob, void* X, const stf_options* opt,
              void* ws, size_t ws_bytes, double* X64_out, double* Lam_out,
              stf_result* res, hipStream_t stream);

/* stf_solve with opt->variant forced to STF_PLAM / STF_PCAL (Algorithms 2, 3). */
int plam_solve(const stf_problem* prob, void* X, const stf_options* opt,
               void* ws, size_t ws_bytes, double* X64_out, double* Lam_out,
               stf_result* res, hipStream_t stream);
int pcal_solve(const stf_problem* prob, void* X, const stf_options* opt,
               void* ws, size_t ws_bytes, double* X64_out, double* Lam_out,
               stf_result* res, hipStream_t stream);

/* ---- step-level entry points (each is one step of the iteration) --------- */

/* G = grad f(X) = (L + Diag v) X + alpha Diag(L^{-1} rho) X, or A X (dense):
 * the gradients of Problem 1 (the simplified Kohn-Sham energy, with the
 * operators of the workloads) and Problem 3 (Rayleigh-Ritz) of Section 5.2,
 * "Func" in Table 1.
 * X, G: device n x p of dtype (STF_F64 / STF_F32); a float32 A serves both
 * dtypes (widened exactly for float64), a float64 A only dtype STF_F64.
 * Computes rho and the Hartree solve internally (in the workspace).  Errors:
 * STF_E_INVALID (NULL, bad dtype), STF_E_UNSUPPORTED (float64 A with a
 * float32 X), STF_E_WORKSPACE, STF_E_HIP.  Host-synchronous. */
int stf_gradient(const stf_problem* prob, const void* X, void* G, int32_t dtype,
                 void* ws, size_t ws_bytes, hipStream_t stream);

/* phi = L^{-1} rho for the stencil kinds (the L^dagger of eq. (KS-energy) and
 * of Problem 1, Section 5.2);
 * rho, phi: device float64 length n.  1D: closed-form Green's function by
 * two scans; 3D: sine transforms along each axis. */
int stf_hartree(const stf_problem* prob, const double* rho, double* phi,
                void* ws, size_t ws_bytes, hipStream_t stream);

/* S = X^T X and W = X^T G (both p x p float64, full, row-major), the Gram
 * products of Table 1 ("feasibility" and "KKT" rows) that feed the
 * multiplier of eq. (Lambda1).  X, G: device n x p of dtype.  precision
 * selects the product arithmetic (STF_PREC_*; FP64 needs dtype F64, the
 * others F32).  Host-synchronous. */
int stf_gram(const stf_problem* prob, const void* X, const void* G, int32_t dtype,
             int32_t precision, double* S, double* W, void* ws, size_t ws_bytes,
             hipStream_t stream);

/* In-place CholeskyQR2 of a float64 n x p X (full column rank): the
 * orthonormalization post-process of Section 5.3 (Table 2), Cholesky-based as
 * in the parallel experiments of Section 5.5, applied twice.  Returns
 * STF_E_CHOLESKY (X unchanged in its first pass, or partly transformed) when a
 * pivot is not positive (X rank-deficient to working precision). */
int stf_cholqr2(const stf_problem* prob, double* X, void* ws, size_t ws_bytes,
                hipStream_t stream);

/* out3 (host, 3 doubles) = { f(X), ||G - X Psi(G^T X)||_F, ||X^T X - I||_F }
 * in float64 for a float64 X: the objective, the KKT violation of the stop
 * test of Section 5.1 (with X Psi in place of X G^T X, as Section 3.3 notes)
 * and the feasibility violation, the three columns of Table 2 (a float32 A is
 * widened exactly).  Host-synchronous. */
int stf_eval(const stf_problem* prob, const double* X, double* out3,
             void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- adjoint (implicit differentiation of the stationary point) ---------
 * d l(X*) / dV for the diagonal potential V of the objective, given the
 * Euclidean gradient gradX = dl/dX* of a loss that is invariant under
 * X* -> X* Q (Q orthogonal).  Differentiating the stationarity condition
 * grad f(X) = X Lam (eq. (kkt)) on the horizontal space {xi : X^T xi = 0}
 * gives Hess[zeta] = P(gradX) with Hess[xi] = P(grad^2 f(X)[xi] - xi Lam),
 * P = I - X X^T (the form of (son)); then dl/dV = -rowdot(zeta, X*).
 * The system is solved by float64 conjugate gradients on the device.
 *   Xstar  : device n x p float64, orthonormal stationary point (e.g. X64_out of stf_solve)
 *   Lam    : device p x p float64, Psi(grad f(X*)^T X*) (Lam_out of stf_solve)
 *   gradX  : device n x p float64;  gradV: device n float64 (output)
 *   cg_tol : relative residual target of CG;  cg_maxit: iteration cap
 *   ws     : device workspace of ws_bytes >= stf_adjoint_workspace_size(prob)
 *   cg_iters, cg_relres : host outputs (may be NULL)
 * Returns STF_OK, STF_MAX_ITER (cap reached, gradV still written),
 * STF_E_DIVERGED (the Hessian is not positive definite on the horizontal
 * space: X* is not a strict local minimizer), or another STF_E_* code. */
size_t stf_adjoint_workspace_size(const stf_problem* prob);
int pcal_adjoint_v(const stf_problem* prob, const double* Xstar, const double* Lam,
                   const double* gradX, double* gradV, double cg_tol, int32_t cg_maxit,
                   void* ws, size_t ws_bytes, int32_t* cg_iters, double* cg_relres,
                   hipStream_t stream);

/* ---- batched solve: many independent problems of uneven n and p --------
 * Each problem runs the iteration of stf_solve (Algorithms 2 / 3 with the
 * step-size rules of Section 5.1) on its own; the library advances all of them
 * together, every stage of an iteration being one grouped launch over the
 * whole batch, captured in a HIP graph (opt->use_graph) and replayed.  A
 * problem that meets its stop test stops; the others go on.
 *   nprob  : number of problems (>= 1)
 *   probs  : host array of nprob descriptors; kind STF_KIND_STENCIL1D only
 *            (STF_E_UNSUPPORTED otherwise)
 *   X      : host array of nprob device pointers, each n_b x p_b row-major,
 *            float64 (STF_PREC_FP64) or float32 (STF_PREC_FP32 / MIXED);
 *            X^0 on entry, the returned iterate on exit (CholeskyQR2'd when
 *            opt->orth_final)
 *   opts   : host array of nprob option sets, one per problem (beta, eta0,
 *            tol, step rule, variant, max_iter may differ); precision must
 *            be the same for all, use_graph and check_every are taken from
 *            opts[0]; history is ignored; MIXED needs p <= 384; fused must
 *            be 0 (STF_E_UNSUPPORTED otherwise).  switch_tol
 *            acts as in stf_solve, per problem: in the float32 forms a problem
 *            that reaches it (or stalls) continues in float64 at once while
 *            the others go on in float32 in the same iterations
 *            (stf_result.switch_iter per problem); a problem always continues
 *            from its float32 iterate here (restarted = 0: no restart from X^0)
 *   ws     : device workspace of ws_bytes >= stf_batched_workspace_size()
 *   res    : host array of nprob results (ms_loop / ms_orth: the whole batch)
 * Returns the first STF_E_* met, else STF_MAX_ITER when some problem reached
 * max_iter, else STF_TOL_UNMET when some problem's float64 check is above its
 * tol, else STF_OK (every problem converged). */
size_t stf_batched_workspace_size(int32_t nprob, const stf_problem* probs,
                                  const stf_options* opts);
int stf_solve_batched(int32_t nprob, const stf_problem* probs, void* const* X,
                      const stf_options* opts, void* ws, size_t ws_bytes, stf_result* res,
                      hipStream_t stream);
/* The same with every variant = STF_PCAL. */
int pcal_solve_batched(int32_t nprob, const stf_problem* probs, void* const* X,
                       const stf_options* opts, void* ws, size_t ws_bytes, stf_result* res,
                       hipStream_t stream);
/* stf_solve_batched with explicit batch-wide workgroup budgets of the Gram
 * pass and of the residual pass (<= 0: defaults), which set every problem's
 * split-K chunk count and residual row blocks in proportion to its n p^2;
 * ms_per_iter (host, may be NULL) receives the loop time per iteration. */
int stf_solve_batched_ex(int32_t nprob, const stf_problem* probs, void* const* X,
                         const stf_options* opts, void* ws, size_t ws_bytes, stf_result* res,
                         int32_t budget_gram, int32_t budget_res, double* ms_per_iter,
                         hipStream_t stream);
/* Autotuner of the two budgets: times `iters` iterations of the batch for each
 * candidate pair and returns the fastest in *best_gram / *best_res.  The
 * iterations are real: X is advanced by 9 * iters iterations (reload X^0
 * before solving). */
int stf_batched_tune(int32_t nprob, const stf_problem* probs, void* const* X,
                     const stf_options* opts, void* ws, size_t ws_bytes, int32_t iters,
                     int32_t* best_gram, int32_t* best_res, double* best_ms_per_iter,
                     hipStream_t stream);

/* ---- no allocation -------------------------------------------------------
 * stf_gram without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same inputs, outputs and arithmetic as stf_gram;
 * the split-K partial sums go to a static device buffer of
 * STF_NOALLOC_SCRATCH_BYTES that the library owns on each GPU it runs on (held
 * until the process ends), so the call allocates nothing.  Calls that overlap
 * on one GPU (other streams or threads) share that buffer and race: serialize
 * them.  When even one split-K chunk of the Gram tiles does not fit the
 * buffer (p above about 2048) it returns STF_E_SCRATCH; the chunk count is
 * otherwise capped to fit, so the summation order can differ from stf_gram's
 * (results equal to rounding).  Host-synchronous. */
#define STF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int stf_gram_noalloc(const stf_problem* prob, const void* X, const void* G, int32_t dtype,
                     int32_t precision, double* S, double* W, hipStream_t stream);

/* Human-readable name of a return code (static string). */
const char* stf_strerror(int code);

/* Library version string. */
const char* stf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STIEFEL_H */
