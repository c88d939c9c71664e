// Internal declarations of the gfx950 PLAM / PCAL library: device-resident
// iteration state, workspace layout and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/stiefel.h"

namespace stf {

// Iteration state kept in device memory so that no host round trip is needed
// inside an iteration.  Written by the p x p stage kernels only.
struct DevState {
    double kkt0;          // ||G - X Psi||_F at X^0
    double kkt;           // the last evaluated ||G - X Psi||_F
    double feas;          // ||X^T X - I||_F of the current iterate
    double eta;           // eta^k (valid after the stage-2 kernel of iteration k)
    double ss, sy, yy;    // <S,S>, <S,Y>, <Y,Y> of the current iteration (standard pair)
    double ss_l, sy_l, yy_l;  // the same from the previous iteration (lagged pair)
    double fval;          // scratch for the evaluation kernels
    double red[8];        // scratch for reductions
    int32_t iter;         // k of the iteration being processed
    int32_t done;         // 1 once converged / max_iter / diverged
    int32_t status;       // STF_OK / STF_MAX_ITER / STF_E_DIVERGED
    int32_t final_iter;   // index of the returned iterate
    int32_t info;         // Cholesky failure pivot + 1, or 0
    int32_t k_best;       // iteration of the smallest stop-test value so far
    int32_t pad[2];
    double kkt_best;      // that value
    double eta_next;      // single-pass form: eta^k, set before the pass of iteration k
};

// Parameters the device kernels read (copied once per solve into the workspace).
struct DevParams {
    double beta, eta0, eta_const, tol, feas_blowup;
    int32_t variant, mult_rule, eta_rule, bb_index, max_iter, kkt_every;
    int32_t n_scal_parts;   // number of scalar partial slots written by the residual pass
    int32_t n_col_parts;    // number of row-block column partials
    int32_t kkt_identity;   // 1: stop test from the float64 p x p identity (no second product)
    int32_t switch_stall;   // hand over also after this many iterations without a new
                            // smallest stop-test value (with switch_tol > 0; 0 = never)
    double switch_tol;      // relative KKT at which a reduced-precision solve hands over
    double* history;        // optional per-iteration record, (max_iter + 1) x 4
    int32_t fused;          // 1: single-pass update (eta, nu before the residual pass)
    int32_t pad_f;
};

// Terms of the gradient beyond (L + Diag v + alpha Diag phi) X: the linear
// term of Problem 2, the exchange term -2 gamma Diag(rho^{1/3}) X of Problem 6
// and the block structure of the 1D operator of Section 5.5.
struct GradExtra {
    const double* glin;   // n x p float64, added to G, or null
    const double* rho;    // the density rho = diag(X X^T) (read when gamma != 0)
    double gamma;         // exchange weight
    int32_t block;        // 1D: order of the tridiagonal blocks (0: one block)
    int32_t dense_prod;   // dense float32 A X: 0 = float32 MFMA, 3 = split bf16
    void* xsplit;         // split bf16 X^T (2 x p x dense_npad(n) bf16); required with dense_prod 3
};
// k padding of the split X^T of the split-bf16 dense product
inline int64_t dense_npad(int64_t n) { return (n + 63) / 64 * 64; }

// Internal status of a reduced-precision phase that reached switch_tol, and
// (batched solves) of one whose float64 continuation has taken over.
#define STF_SWITCH 16
#define STF_SWITCHED 17
// Iterations without a new smallest stop-test value after which a
// reduced-precision phase hands over even above switch_tol.
constexpr int kSwitchStall = 100;

// Tiling of the split-K Gram pass.
struct GramPlan {
    int wm;          // MFMA 16x16 tiles per wave per dimension (1, 2 or 4)
    int bt;          // workgroup tile = 32 * wm
    int nb;          // ceil(p / bt)
    int n_s_tiles;   // upper-triangular blocks of S
    int n_tiles;     // n_s_tiles + the W blocks (nb*nb, or n_s_tiles when wup)
    int wup;         // 1: W symmetric, only its upper blocks are computed
    int nchunks;     // split-K chunks over the n rows
    int64_t chunk;   // rows per chunk (multiple of 4)
};

// Tiling of the row-block x (p x p) product pass (square tiles of `tile`;
// tile 256 is the LDS-resident split-bf16 kernel: 256-row tiles, 64-column blocks).
struct ResPlan {
    int tile;        // 128 (float64 / float32), 64 or 256 (split-bf16 kernels)
    int nrb;         // row-block workgroups (each strides over row tiles)
    int ncb;         // ceil(p / 64) column blocks of 64 columns
    int64_t nrt;     // ceil(n / tile) row tiles
};

// Row-block groups of the column-dot reduction after the residual pass (the
// last step sums the groups): one group per 64 row blocks, at most 32.
__host__ __device__ inline int col_groups(int nrb) {
    const int g = nrb / 64;
    return g < 1 ? 1 : (g > 32 ? 32 : g);
}

// Byte offsets of every buffer inside the caller's workspace.
struct Layout {
    size_t state, state_eval, params, params_eval;
    size_t state64, params64;  // batched float32 forms: the float64 continuation's
    size_t g[2];          // G / gradL double buffer, n*p elements of the iteration dtype
    size_t x64, g64;      // float64 n*p buffers: master iterate (float32 forms) and scratch
    size_t g64b;          // second float64 n*p buffer (float32 forms): float64 continuation
    size_t x0keep;        // n*p float32 (float32 forms, solver layout): X^0 for a float64 restart
    size_t rho, phi, hscr;
    size_t S, W, Psi, ML, Rm, Rinv, Lam, Bm, T1, fpart;  // T1: p x p product-pass partials
    size_t nu, colpart;   // colpart: col_groups(res.nrb) x 2p column-dot partials
    size_t gram_part;
    size_t res_col, res_scal, dots;
    size_t dst;           // sine tables and 1D eigenvalues (3D Hartree solve)
    size_t mix;           // split-bf16 copies of M_L^T and Psi^T (MIXED precision)
    size_t lam2;          // two p x p float64: the dual-ascent multiplier, by iteration parity
    size_t cwork;         // p x p float64: the working matrix of the blocked Cholesky
    size_t gtmp;          // n x p (iteration dtype): H0 X before the right factor B
    size_t xalt;          // n x p float64 (MOptQR, single-pass form): the other iterate buffer
    size_t vbuf;          // n x p float64 (MOptQR): V = X - D / eta before the retraction
    size_t colsq;         // single-pass form: Gram chunks x 4 x p column sums of G^2
    size_t nu2;           // single-pass form: nu^k (p float64), found before the pass
    size_t rhopart;       // single-pass form: row partials of rho, slots x n float64
    size_t xsplit;        // dense kind, reduced precision: split bf16 X^T (2 x p x npad)
    size_t total;
    GramPlan gram;        // plan for the iteration dtype
    GramPlan gram64;      // plan for float64 (CholeskyQR2 / evaluation)
    ResPlan res;          // float64 / float32 residual pass
    ResPlan res64;        // split-bf16 residual pass (MIXED), M_L from global memory
    ResPlan resmx;        // split-bf16 residual pass (MIXED), M_L resident in LDS (pk <= 384)
    const ResPlan& mixed_plan() const { return resmx.nrb > 0 ? resmx : res64; }
};

// One problem of a batched solve, as the grouped kernels see it: its sizes,
// operator data, plans and the addresses inside its share of the workspace.
struct BDesc {
    int64_t n;
    int32_t p, pad0;
    double alpha;
    const double* v;
    void* X;           // iterate in the storage dtype (caller's buffer)
    double* Xm;        // float64 master iterate (float32 forms), else null
    void* g[2];        // G / gradL double buffer
    double *rho, *phi, *S, *W, *Psi, *ML, *Bm, *T1, *fpart;
    double *nu, *colpart, *gram_part, *res_col, *res_scal;
    __bf16* mix;
    DevState* st;
    DevParams* prm;
    GramPlan gram;
    ResPlan res;
    int32_t nblk_rows;  // workgroups of the row-parallel passes (gradient, update)
    int32_t pad1;
};

// A grouped launch: workgroups [off[j], off[j+1]) belong to problem list[j].
struct BGroup {
    const int32_t* list;
    const int32_t* off;
    int32_t cnt;
    int32_t total;     // off[cnt]
};

// Grouped launches of one batched iteration stage (stf_kernels.hip).
enum BStage {
    BS_HARTREE = 0, BS_GRAD, BS_GRAM, BS_REDUCE, BS_STAGE1, BS_PPGEMM, BS_SPLIT, BS_RESID,
    BS_COLRED, BS_STAGE2, BS_UPDATE, BS_ROWSQ
};
void launch_batched(int stage, int dtype, int precision, int variant_key, const BDesc* d,
                    const BGroup& grp, int parity, hipStream_t s);
void launch_gather_states(const BDesc* d, int nprob, DevState* out, hipStream_t s);
// Batched per-problem hand-over: every problem whose reduced-precision state d32
// reports STF_SWITCH gets its previous gradL (float32 buffer parity ^ 1)
// converted into its float64 continuation's buffer parity ^ 1 and its state
// copied to d64's (resumed) while d32's is marked STF_SWITCHED.
void launch_batched_switch(const BDesc* d32, const BDesc* d64, int nprob, int parity,
                           hipStream_t s);

int elem_size(int dtype);
// target_wg: workgroups the plan aims at (the single-problem defaults when omitted)
GramPlan make_gram_plan(int64_t n, int p, int64_t target_wg = 512, bool wup = false);
ResPlan make_res_plan(int64_t n, int p, int tile, int64_t target_wg = 0);
// fused: the buffers of the single-pass form (and the second iterate buffer xalt)
// solver = true: the layout of stf_solve (with the float32 copy of X^0 that
// a float64 restart needs in the float32 forms)
Layout make_layout(const stf_problem* prob, int precision, bool moptqr = false,
                   bool fused = false, bool solver = false);
size_t align256(size_t x);

// A problem's workspace: base address and layout.
struct Ws {
    char* base;
    Layout L;
    template <typename T> T* at(size_t o) const { return (T*)(base + o); }
};

// Shared by the single-problem and batched drivers (stf_api.hip).
int check_problem(const stf_problem* prob);
bool has_hartree(const stf_problem* prob);
// the density rho is needed by the gradient (Hartree or exchange term)
bool needs_rho(const stf_problem* prob);
// X^T grad f(X) is symmetric (no linear term, no right factor)
bool w_symmetric(const stf_problem* prob);
GradExtra grad_extra(const stf_problem* prob, const double* rho);
int last_launch();
// In-place CholeskyQR2 of a float64 X (tmp: n x p float64 scratch).
int enqueue_cholqr2(const stf_problem* prob, const Ws& w, double* X, double* tmp,
                    DevState* st, hipStream_t s);
// f, KKT and feasibility of a float64 X into w's evaluation state (G64 overwritten).
int enqueue_eval(const stf_problem* prob, const Ws& w, const double* X, double* G64,
                 hipStream_t s);

// ---- launchers (stf_kernels.hip); all enqueue on `s` -----------------------
void launch_rowsq(int dtype, const void* X, int64_t n, int p, double* rho,
                  const DevState* st, hipStream_t s);
// stencil kinds: the right factor B of Problem 4 applied after the stencil
// (tmp: n x p of dtype); G = tmp B.  Dense: the same with A X in tmp.
void launch_hartree(const stf_problem* prob, const double* rho, double* phi,
                    double* scratch, double* dst_tables, const DevState* st,
                    hipStream_t s);
void launch_dst_init(const stf_problem* prob, double* dst_tables, hipStream_t s);
// Xm (float32 G only): the stencil reads this float64 copy of X instead of X.
// ex: the further gradient terms (grad_extra); with a right factor B the
// caller applies it afterwards (launch_apply).
void launch_grad(const stf_problem* prob, int dtype, const void* X, void* G,
                 const double* phi, const GradExtra& ex, const DevState* st, hipStream_t s,
                 const double* Xm = nullptr);
// S = X^T X (if S) and W = X^T G (if W), float64 p x p, full
void launch_gram(int dtype, int precision, const GramPlan& gp, const void* X,
                 const void* G, int64_t n, int p, double* part, double* S,
                 double* W, const DevState* st, hipStream_t s,
                 hipEvent_t after_main = nullptr, bool w_sym = false,
                 double* colsq = nullptr);
// colsq (single-pass form, W wanted, p > 64): per chunk, gram_colsq_slots
// partial column sums of G^2 at colsq[(chunk * 4 + slot) * p + c]
int gram_colsq_slots(int dtype);
// lam2: two p x p buffers of the dual-ascent multiplier (STF_MULT_DUAL), else null
void launch_stage1(const DevParams* prm, const double* S, const double* W,
                   double* Psi, double* ML, double* Bm, double* feas_part, int p,
                   DevState* st, hipStream_t s, double* lam2 = nullptr);
// per-tile partials of <B, S B - 2 (W - S M_L)> into part[kkt_partials(p)]
// (64 x 64 float64 MFMA tiles of one product, split over K, from p = kPPWide
// on, else 16 x 16 tiles of two)
constexpr int kPPWide = 128;
int kkt_partials(int p);
void launch_kkt_products(const double* S, const double* ML, const double* Bm, const double* W,
                         double* part, int p, DevState* st, hipStream_t s);
void launch_residual(int dtype, int precision, const ResPlan& rp, const void* X,
                     void* G, const void* Gprev, const double* ML, const double* Psi,
                     const double* nu, int64_t n, int p, double* part_col,
                     double* part_scal, const DevParams* prm, DevState* st,
                     int mode, void* mix, hipStream_t s, hipEvent_t before_main = nullptr,
                     const void* Xprev = nullptr);
// pp_part: the ((p+15)/16)^2 tile partials of the KKT identity's p x p term
void launch_stage2(const DevParams* prm, const ResPlan& rp, const double* part_col,
                   const double* part_scal, const double* S, const double* pp_part,
                   const double* feas_part, double* colpart, double* nu, int p, DevState* st,
                   hipStream_t s, const double* nu_cur = nullptr);
// ---- single-pass form (stf_options.fused) ----
// SM = S M_L (float64 MFMA), then eta^k into st->eta_next and the PCAL column
// norms nu^k into nu_cur, from S, W, M_L, SM and the Gram pass's column sums
void launch_fused_pre(const DevParams* prm, const double* S, const double* W, const double* ML,
                      double* SM, const double* colsq, int nchunks, int nsl, double* nu_cur,
                      int p, DevState* st, hipStream_t s);
// the row-block pass of the single-pass form: gradL over G, the Barzilai-
// Borwein and column dots as in launch_residual, X^{k+1} into Xn and per-slot
// row sums of its squares into rho_part[fused_rho_slots][n].  float64 (plan
// res) or float32 with split-bf16 products (plan resmx; M_L split into mix)
int fused_rho_slots(int dtype, const ResPlan& rp);
void launch_residual_fused(int dtype, const ResPlan& rp, const void* X, void* Xn, void* G,
                           const void* Gprev, const double* ML, const double* nu,
                           const double* nu_cur, int64_t n, int p, double* part_col,
                           double* part_scal, double* rho_part, const DevParams* prm,
                           DevState* st, void* mix, hipStream_t s,
                           hipEvent_t before_main = nullptr);
// rho[r] = sum of the nslots row partials
void launch_rho_reduce(const double* part, int nslots, int64_t n, double* rho,
                       const DevState* st, hipStream_t s);
// Xm (float32 X only): float64 master iterate, read and written; X gets its rounding
void launch_update(int dtype, void* X, const void* GL, int64_t n, int p,
                   const double* nu, double* rho, const DevState* st, hipStream_t s,
                   double* Xm = nullptr);
// Out = X M (subtract = 0) or Out -= X M (subtract = 1); M float64 p x p;
// nothing once st (if given) says "done"
void launch_apply(int dtype, const ResPlan& rp, const void* X, void* Out,
                  const double* M, int64_t n, int p, hipStream_t s, int subtract = 0,
                  const DevState* st = nullptr);
// Blocked Cholesky S = R^T R (R upper) and Rinv = R^{-1}, float64, on the device
// (work: p x p scratch).  A non-positive pivot sets st->info to its index + 1;
// with stop_on_fail it also ends the iteration (st->done, STF_E_DIVERGED).
// Every kernel returns at once when st->done is already set.
void launch_chol_inv(const double* S, double* R, double* Rinv, double* work, int p,
                     DevState* st, hipStream_t s, int stop_on_fail = 0);
// MOptQR: V = X - D / eta (eta from the state), out of place, float64
void launch_vform(const double* X, const double* D, double* V, int64_t n, int p,
                  const DevState* st, hipStream_t s);
void launch_convert(int to_dtype, const void* in, int in_dtype, void* out, size_t count,
                    hipStream_t s);
// feas_part: the p row sums of (S - I)^2 written by stage 1
void launch_eval_finish(const stf_problem* prob, const double* X, const double* G,
                        const double* rho, const double* phi, const double* feas_part,
                        int64_t n, int p, double* dots, const double* part_scal, int nps,
                        DevState* st, hipStream_t s);
void launch_init_state(DevState* st, hipStream_t s);
void launch_resume_state(DevState* st, hipStream_t s);

// residual modes
enum { RES_ITERATE = 0, RES_KKT_ONLY = 1 };

}  // namespace stf
