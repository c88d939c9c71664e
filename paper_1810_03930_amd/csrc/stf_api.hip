// C ABI and host driver of the PLAM / PCAL solver (declared in include/stiefel.h).
//
// The driver enqueues whole iterations without reading anything back; the
// device state (stf::DevState) decides convergence.  Every `check_every`
// iterations the host copies the state once and stops when it says "done".
// With use_graph, a chunk of check_every iterations (an even count, so the
// G double-buffer parity repeats) is captured once and replayed.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "stf_internal.h"

namespace stf {

int elem_size(int dtype) { return dtype == STF_F64 ? 8 : 4; }

GramPlan make_gram_plan(int64_t n, int p, int64_t target_wg, bool wup) {
    GramPlan g;
    g.wm = (p <= 32) ? 1 : (p <= 64 ? 2 : 4);
    g.bt = 32 * g.wm;
    g.nb = (p + g.bt - 1) / g.bt;
    g.n_s_tiles = g.nb * (g.nb + 1) / 2;
    g.wup = wup ? 1 : 0;
    g.n_tiles = g.n_s_tiles + (wup ? g.n_s_tiles : g.nb * g.nb);
    // whole rounds of workgroups: never more than target_wg (a few extra
    // workgroups would cost a whole extra round of the longest ones)
    int64_t nch = target_wg / g.n_tiles;
    const int64_t max_ch = std::max<int64_t>(1, n / 256);
    nch = std::min(nch, max_ch);
    nch = std::max<int64_t>(nch, 1);
    int64_t chunk = (n + nch - 1) / nch;
    chunk = (chunk + 3) / 4 * 4;
    // the Gram kernels address a chunk's rows with 32-bit byte offsets
    const int64_t max_chunk = std::max<int64_t>(4, ((int64_t(1) << 31) - 1) / (8 * (int64_t)p) / 4 * 4);
    chunk = std::min(chunk, max_chunk);
    g.chunk = chunk;
    g.nchunks = (int)((n + chunk - 1) / chunk);
    return g;
}

ResPlan make_res_plan(int64_t n, int p, int tile, int64_t target_wg) {
    ResPlan r;
    r.tile = tile;
    if (tile == 256) {
        // one workgroup per CU (the M_L slice fills most of the LDS), 64-column blocks
        r.ncb = (p + 63) / 64;
        r.nrt = (n + 255) / 256;
        const int64_t pk = (p + 31) / 32 * 32;
        if (pk > 384) {
            r.nrb = 0;
            return r;
        }
        int64_t nrb = ((target_wg > 0 ? target_wg : 256) + r.ncb - 1) / r.ncb;
        nrb = std::min<int64_t>(nrb, r.nrt);
        r.nrb = (int)std::max<int64_t>(nrb, 1);
        return r;
    }
    // tile 128: 128-row tiles of 64 columns (float64 / float32 kernels); 64: square
    r.ncb = (p + 63) / 64;
    r.nrt = (n + tile - 1) / tile;
    const int64_t target = target_wg > 0 ? target_wg : ((tile == 128) ? 1024 : 2048);
    int64_t nrb = (target + r.ncb - 1) / r.ncb;
    nrb = std::min<int64_t>(nrb, r.nrt);
    r.nrb = (int)std::max<int64_t>(nrb, 1);
    return r;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(const stf_problem* prob, int precision, bool moptqr, bool fused,
                   bool solver) {
    Layout L;
    memset(&L, 0, sizeof(L));
    const int64_t n = prob->n;
    const int p = prob->p;
    const int dt = (precision == STF_PREC_FP64) ? STF_F64 : STF_F32;
    const size_t np = (size_t)n * p;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.state = take(sizeof(DevState));
    L.state_eval = take(sizeof(DevState));
    L.params = take(sizeof(DevParams));
    L.params_eval = take(sizeof(DevParams));
    L.state64 = take(sizeof(DevState));
    L.params64 = take(sizeof(DevParams));
    L.g[0] = take(np * elem_size(dt));
    L.g[1] = take(np * elem_size(dt));
    if (dt == STF_F64) {
        L.x64 = (size_t)-1;  // X itself
        L.g64 = L.g[0];
        L.x0keep = (size_t)-1;
    } else {
        L.x64 = take(np * 8);
        L.g64 = take(np * 8);
        L.g64b = take(np * 8);
        L.x0keep = solver ? take(np * 4) : (size_t)-1;
    }
    L.rho = take((size_t)n * 8);
    L.phi = take((size_t)n * 8);
    L.hscr = take((size_t)n * 8);
    const size_t pp = (size_t)p * p * 8;
    L.S = take(pp);
    L.W = take(pp);
    L.Psi = take(pp);
    L.ML = take(pp);
    L.Rm = take(pp);
    L.Rinv = take(pp);
    L.Lam = take(pp);
    L.Bm = take(pp);
    L.T1 = take(pp);
    L.fpart = take((size_t)p * 8);
    L.nu = take((size_t)p * 8);
    L.colpart = take((size_t)32 * 2 * p * 8);
    // iterations: W symmetric (upper blocks); evaluation / CholeskyQR2 / step API: full
    L.gram = make_gram_plan(n, p, 512, true);   // one round at two workgroups per CU
    L.gram64 = make_gram_plan(n, p);
    {
        // room for any tile set (S upper + all of W) at either plan's chunk count
        const size_t tiles = (size_t)L.gram64.n_s_tiles + (size_t)L.gram64.nb * L.gram64.nb;
        const size_t nch = (size_t)std::max(L.gram.nchunks, L.gram64.nchunks);
        L.gram_part = take(nch * tiles * L.gram64.bt * L.gram64.bt * 8);
    }
    L.res = make_res_plan(n, p, 128);
    L.res64 = make_res_plan(n, p, 64);
    L.resmx = make_res_plan(n, p, 256);
    const size_t nrb_max = (size_t)std::max({L.res.nrb, L.res64.nrb, L.resmx.nrb});
    const size_t nwg_max = std::max({(size_t)L.res.nrb * L.res.ncb,
                                     (size_t)L.res64.nrb * L.res64.ncb,
                                     (size_t)L.resmx.nrb * L.resmx.ncb});
    L.res_col = take(nrb_max * p * 2 * 8);
    L.res_scal = take(nwg_max * 4 * 8);
    L.dots = take(512 * 4 * 8);
    if (prob->kind == STF_KIND_STENCIL3D) {
        const size_t nx = prob->grid[0], ny = prob->grid[1], nz = prob->grid[2];
        L.dst = take((nx * nx + ny * ny + nz * nz + nx + ny + nz) * 8);
    } else {
        L.dst = take(8);
    }
    {
        const size_t prow = (size_t)L.res64.ncb * 64, pk = (size_t)(p + 31) / 32 * 32;
        L.mix = take(2 * 3 * prow * pk * 2);
    }
    L.lam2 = take(2 * pp);
    L.cwork = take(pp);
    L.gtmp = prob->B ? take(np * 8) : (size_t)-1;  // room for either dtype
    L.xalt = (moptqr || fused) ? take(np * 8) : (size_t)-1;
    L.vbuf = moptqr ? take(np * 8) : (size_t)-1;
    if (fused) {
        L.colsq = take((size_t)L.gram.nchunks * 4 * p * 8);
        L.nu2 = take((size_t)p * 8);
        const size_t slots = (size_t)std::max(2 * L.res.ncb, L.resmx.ncb);
        L.rhopart = take(slots * (size_t)n * 8);
    } else {
        L.colsq = L.nu2 = L.rhopart = (size_t)-1;
    }
    L.xsplit = (prob->kind == STF_KIND_DENSE && precision != STF_PREC_FP64)
                   ? take((size_t)4 * p * dense_npad(n))
                   : (size_t)-1;
    L.total = off;
    return L;
}

// ------------------------------------------------------------ helpers ----

int check_problem(const stf_problem* prob) {
    if (!prob) return STF_E_INVALID;
    if (prob->p <= 0 || prob->p > 4096) return STF_E_INVALID;
    if (prob->n < 2 * (int64_t)prob->p) return STF_E_INVALID;
    if (prob->kind == STF_KIND_STENCIL1D) {
        if (prob->grid[0] != prob->n || prob->grid[1] != 1 || prob->grid[2] != 1)
            return STF_E_INVALID;
    } else if (prob->kind == STF_KIND_STENCIL3D) {
        if (prob->grid[0] <= 0 || prob->grid[1] <= 0 || prob->grid[2] <= 0) return STF_E_INVALID;
        if ((int64_t)prob->grid[0] * prob->grid[1] * prob->grid[2] != prob->n)
            return STF_E_INVALID;
    } else if (prob->kind == STF_KIND_DENSE) {
        if (!prob->A) return STF_E_INVALID;
        if (prob->A_dtype != STF_F64 && prob->A_dtype != STF_F32) return STF_E_INVALID;
        if (prob->n > 2147483647LL) return STF_E_INVALID;
    } else {
        return STF_E_INVALID;
    }
    if (!isfinite(prob->alpha) || !isfinite(prob->gamma)) return STF_E_INVALID;
    if (prob->block < 0) return STF_E_INVALID;
    if (prob->block > 0 && prob->kind != STF_KIND_STENCIL1D) return STF_E_INVALID;
    if (prob->gamma != 0.0 && prob->kind == STF_KIND_DENSE) return STF_E_INVALID;
    // the right factor of Problem 4 only for quadratic objectives
    if (prob->B && (prob->alpha != 0.0 || prob->gamma != 0.0)) return STF_E_UNSUPPORTED;
    return STF_OK;
}

bool has_hartree(const stf_problem* prob) {
    return prob->kind != STF_KIND_DENSE && prob->alpha != 0.0;
}

bool needs_rho(const stf_problem* prob) {
    return prob->kind != STF_KIND_DENSE && (prob->alpha != 0.0 || prob->gamma != 0.0);
}

bool w_symmetric(const stf_problem* prob) { return !prob->Glin && !prob->B; }

GradExtra grad_extra(const stf_problem* prob, const double* rho) {
    GradExtra e;
    memset(&e, 0, sizeof(e));
    e.glin = prob->Glin;
    e.rho = rho;
    e.gamma = (prob->kind != STF_KIND_DENSE) ? prob->gamma : 0.0;
    e.block = (prob->kind == STF_KIND_STENCIL1D && prob->block < prob->n) ? prob->block : 0;
    return e;
}

#define HIPCHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return STF_E_HIP;   \
    } while (0)

int last_launch() { return hipGetLastError() == hipSuccess ? STF_OK : STF_E_HIP; }

// G = grad f(X) given rho / phi of X in the workspace; with the right factor B
// of Problem 4, H0 X goes to the workspace's gtmp and G = gtmp B.  Xm: the
// float64 master copy the float32 forms evaluate the stencil on.
static void enqueue_grad_core(const stf_problem* prob, const Ws& w, int dtype, const void* X,
                              void* G, const DevState* st, hipStream_t s,
                              const double* Xm = nullptr, int dense_prod = 0) {
    GradExtra ex = grad_extra(prob, needs_rho(prob) ? w.at<double>(w.L.rho) : nullptr);
    ex.dense_prod = dense_prod;
    if (dense_prod == 3 && w.L.xsplit != (size_t)-1) ex.xsplit = w.base + w.L.xsplit;
    if (prob->B) {
        void* T = w.base + w.L.gtmp;
        launch_grad(prob, dtype, X, T, w.at<double>(w.L.phi), ex, st, s, Xm);
        launch_apply(dtype, w.L.res, T, G, prob->B, prob->n, prob->p, s, 0, st);
    } else {
        launch_grad(prob, dtype, X, G, w.at<double>(w.L.phi), ex, st, s, Xm);
    }
}

// G = grad f(X) using the workspace's rho / phi (no device state).
static int enqueue_gradient(const stf_problem* prob, const Ws& w, int dtype, const void* X,
                            void* G, const DevState* st, hipStream_t s) {
    if (needs_rho(prob)) launch_rowsq(dtype, X, prob->n, prob->p, w.at<double>(w.L.rho), st, s);
    if (has_hartree(prob))
        launch_hartree(prob, w.at<double>(w.L.rho), w.at<double>(w.L.phi),
                       w.at<double>(w.L.hscr), w.at<double>(w.L.dst), st, s);
    enqueue_grad_core(prob, w, dtype, X, G, st, s);
    return last_launch();
}

// In-place CholeskyQR2 of a float64 X using tmp (n x p float64).
int enqueue_cholqr2(const stf_problem* prob, const Ws& w, double* X, double* tmp,
                           DevState* st, hipStream_t s) {
    const int64_t n = prob->n;
    const int p = prob->p;
    double* a = X;
    double* b = tmp;
    for (int pass = 0; pass < 2; ++pass) {
        launch_gram(STF_F64, STF_PREC_FP64, w.L.gram64, a, a, n, p, w.at<double>(w.L.gram_part),
                    w.at<double>(w.L.S), nullptr, nullptr, s);
        launch_chol_inv(w.at<double>(w.L.S), w.at<double>(w.L.Rm), w.at<double>(w.L.Rinv),
                        w.at<double>(w.L.cwork), p, st, s);
        launch_apply(STF_F64, w.L.res, a, b, w.at<double>(w.L.Rinv), n, p, s);
        std::swap(a, b);
    }
    return last_launch();
}

// f, KKT and feasibility of a float64 X in float64 (G64 is overwritten).
int enqueue_eval(const stf_problem* prob, const Ws& w, const double* X, double* G64,
                        hipStream_t s) {
    const int64_t n = prob->n;
    const int p = prob->p;
    DevState* st = w.at<DevState>(w.L.state_eval);
    DevParams* prm = w.at<DevParams>(w.L.params_eval);
    launch_init_state(st, s);
    DevParams hp;
    memset(&hp, 0, sizeof(hp));
    hp.beta = 0.0;
    hp.variant = STF_PLAM;
    hp.mult_rule = STF_MULT_PSI;
    hp.kkt_every = 1;
    hp.max_iter = 0;
    hp.feas_blowup = INFINITY;
    HIPCHK(hipMemcpyAsync(prm, &hp, sizeof(hp), hipMemcpyHostToDevice, s));
    int rc = enqueue_gradient(prob, w, STF_F64, X, G64, nullptr, s);
    if (rc) return rc;
    launch_gram(STF_F64, STF_PREC_FP64, w.L.gram64, X, G64, n, p, w.at<double>(w.L.gram_part),
                w.at<double>(w.L.S), w.at<double>(w.L.W), nullptr, s);
    launch_stage1(prm, w.at<double>(w.L.S), w.at<double>(w.L.W), w.at<double>(w.L.Psi),
                  w.at<double>(w.L.ML), nullptr, w.at<double>(w.L.fpart), p, st, s);
    // the dot products read G before the KKT pass (which does not write in this mode)
    launch_residual(STF_F64, STF_PREC_FP64, w.L.res, X, G64, nullptr, w.at<double>(w.L.ML),
                    w.at<double>(w.L.Psi), nullptr, n, p, w.at<double>(w.L.res_col),
                    w.at<double>(w.L.res_scal), prm, st, RES_KKT_ONLY, nullptr, s);
    launch_eval_finish(prob, X, G64, w.at<double>(w.L.rho), w.at<double>(w.L.phi),
                       w.at<double>(w.L.fpart), n, p, w.at<double>(w.L.dots),
                       w.at<double>(w.L.res_scal), w.L.res.nrb * w.L.res.ncb, st, s);
    return last_launch();
}

struct IterCtx {
    const stf_problem* prob;
    Ws w;
    int dtype, precision;
    void* X;
    double* Xm;  // float64 master iterate of the float32 forms (null in float64)
    size_t g[2]; // G / gradL double buffer (workspace offsets)
    DevState* st;
    DevParams* prm;
    bool moptqr;
    bool fused;     // single-pass form (stf_options.fused)
    // MOptQR and the single-pass form: X^k lives in xb[k & 1] (the caller's X
    // and the workspace's xalt, or the float64 continuation's x64 and xalt)
    void* xb[2];
};

// ev (optional): STF_NPROF + 1 events bracketing the kernel groups.
static void enqueue_iteration(const IterCtx& c, int parity, hipStream_t s,
                              hipEvent_t* ev = nullptr) {
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    };
    const stf_problem* prob = c.prob;
    const Ws& w = c.w;
    const int64_t n = prob->n;
    const int p = prob->p;
    void* Gc = w.base + c.g[parity];
    void* Gp = w.base + c.g[parity ^ 1];
    double* rho = needs_rho(prob) ? w.at<double>(w.L.rho) : nullptr;
    // MOptQR and the single-pass form iterate between two buffers; the others
    // update X in place
    void* X = (c.moptqr || c.fused) ? c.xb[parity] : c.X;
    mark(0);
    if (has_hartree(prob))
        launch_hartree(prob, rho, w.at<double>(w.L.phi), w.at<double>(w.L.hscr),
                       w.at<double>(w.L.dst), c.st, s);
    mark(1);
    // the MIXED forms take the dense product A X in split bf16 too
    enqueue_grad_core(prob, w, c.dtype, X, Gc, c.st, s,
                      prob->kind == STF_KIND_DENSE ? nullptr : c.Xm,
                      c.precision == STF_PREC_MIXED ? 3 : 0);
    mark(2);
    // groups 2..4: the Gram kernel | chunk reduction, p x p stage, KKT products,
    // split of M_L | the residual kernel (events 3 and 4 recorded by the launchers)
    // (the single-pass form also takes the column sums of G^2 from this pass)
    launch_gram(c.dtype, c.precision, w.L.gram, X, Gc, n, p, w.at<double>(w.L.gram_part),
                w.at<double>(w.L.S), w.at<double>(w.L.W), c.st, s, ev ? ev[3] : nullptr,
                /*w_sym=*/w_symmetric(prob), c.fused ? w.at<double>(w.L.colsq) : nullptr);
    launch_stage1(c.prm, w.at<double>(w.L.S), w.at<double>(w.L.W), w.at<double>(w.L.Psi),
                  w.at<double>(w.L.ML), w.at<double>(w.L.Bm), w.at<double>(w.L.fpart), p, c.st, s,
                  w.at<double>(w.L.lam2));
    launch_kkt_products(w.at<double>(w.L.S), w.at<double>(w.L.ML), w.at<double>(w.L.Bm),
                        w.at<double>(w.L.W), w.at<double>(w.L.T1), p, c.st, s);
    const ResPlan& rp = (c.precision == STF_PREC_MIXED) ? w.L.mixed_plan() : w.L.res;
    if (c.fused) {
        // eta^k and nu^k first (p x p work), then one pass that forms gradL^k,
        // the step-size and stop-test dots, X^{k+1} (into the other buffer)
        // and the row sums of its squares
        launch_fused_pre(c.prm, w.at<double>(w.L.S), w.at<double>(w.L.W), w.at<double>(w.L.ML),
                         w.at<double>(w.L.Rm), w.at<double>(w.L.colsq), w.L.gram.nchunks,
                         gram_colsq_slots(c.dtype), w.at<double>(w.L.nu2), p, c.st, s);
        launch_residual_fused(c.dtype, rp, X, c.xb[parity ^ 1], Gc, Gp, w.at<double>(w.L.ML),
                              w.at<double>(w.L.nu), w.at<double>(w.L.nu2), n, p,
                              w.at<double>(w.L.res_col), w.at<double>(w.L.res_scal),
                              w.at<double>(w.L.rhopart), c.prm, c.st, w.base + w.L.mix, s,
                              ev ? ev[4] : nullptr);
        mark(5);
        launch_stage2(c.prm, rp, w.at<double>(w.L.res_col), w.at<double>(w.L.res_scal),
                      w.at<double>(w.L.S), w.at<double>(w.L.T1), w.at<double>(w.L.fpart),
                      w.at<double>(w.L.colpart), w.at<double>(w.L.nu), p, c.st, s,
                      w.at<double>(w.L.nu2));
        mark(6);
        if (rho)
            launch_rho_reduce(w.at<double>(w.L.rhopart), fused_rho_slots(c.dtype, rp), n, rho,
                              c.st, s);
        mark(7);
        return;
    }
    launch_residual(c.dtype, c.precision, rp, X, Gc, Gp, w.at<double>(w.L.ML),
                    w.at<double>(w.L.Psi), w.at<double>(w.L.nu), n, p,
                    w.at<double>(w.L.res_col), w.at<double>(w.L.res_scal), c.prm, c.st,
                    RES_ITERATE, w.base + w.L.mix, s, ev ? ev[4] : nullptr,
                    c.moptqr ? (const void*)c.xb[parity ^ 1] : nullptr);
    mark(5);
    launch_stage2(c.prm, rp, w.at<double>(w.L.res_col), w.at<double>(w.L.res_scal),
                  w.at<double>(w.L.S), w.at<double>(w.L.T1), w.at<double>(w.L.fpart),
                  w.at<double>(w.L.colpart), w.at<double>(w.L.nu), p, c.st, s);
    mark(6);
    if (c.moptqr) {
        // the Cholesky-QR retraction (Table 1, Section 5.5): V = X - D / eta,
        // V^T V = R^T R, X^{k+1} = V R^{-1} into the buffer of X^{k-1}
        double* V = w.at<double>(w.L.vbuf);
        double* Xn = (double*)c.xb[parity ^ 1];
        launch_vform((const double*)X, (const double*)Gc, V, n, p, c.st, s);
        launch_gram(STF_F64, STF_PREC_FP64, w.L.gram64, V, V, n, p, w.at<double>(w.L.gram_part),
                    w.at<double>(w.L.Rm), nullptr, c.st, s);
        launch_chol_inv(w.at<double>(w.L.Rm), w.at<double>(w.L.Lam), w.at<double>(w.L.Rinv),
                        w.at<double>(w.L.cwork), p, c.st, s, /*stop_on_fail=*/1);
        launch_apply(STF_F64, w.L.res, V, Xn, w.at<double>(w.L.Rinv), n, p, s, 0, c.st);
        if (rho) launch_rowsq(STF_F64, Xn, n, p, rho, c.st, s);
    } else {
        launch_update(c.dtype, c.X, Gc, n, p, w.at<double>(w.L.nu), rho, c.st, s, c.Xm);
    }
    mark(7);
}

static int solve_impl(const stf_problem* prob, void* X, const stf_options* opt, void* ws,
                      size_t ws_bytes, double* X64_out, double* Lam_out, stf_result* res,
                      hipStream_t s) {
    int rc = check_problem(prob);
    if (rc) return rc;
    if (!X || !opt || !ws || !res) return STF_E_INVALID;
    if (opt->variant != STF_PLAM && opt->variant != STF_PCAL && opt->variant != STF_MOPTQR)
        return STF_E_INVALID;
    const bool moptqr = opt->variant == STF_MOPTQR;
    if (!moptqr) {
        if (opt->mult_rule != STF_MULT_PSI && opt->mult_rule != STF_MULT_PSI_PHI &&
            opt->mult_rule != STF_MULT_DUAL)
            return STF_E_INVALID;
        if (opt->mult_rule == STF_MULT_PSI_PHI && opt->variant != STF_PCAL)
            return STF_E_UNSUPPORTED;
    } else if (opt->precision != STF_PREC_FP64) {
        return STF_E_UNSUPPORTED;  // the comparator runs in float64 only
    }
    if (opt->eta_rule < STF_ETA_CONST || opt->eta_rule > STF_ETA_ABB) return STF_E_INVALID;
    if (opt->bb_index != STF_BB_STANDARD && opt->bb_index != STF_BB_LAGGED) return STF_E_INVALID;
    if (opt->precision < STF_PREC_FP64 || opt->precision > STF_PREC_MIXED32) return STF_E_INVALID;
    // MIXED32: the split-bf16 kernels of MIXED with the iterate kept in float32 only
    const bool nomaster = opt->precision == STF_PREC_MIXED32;
    if (opt->max_iter < 0 || opt->kkt_every < 1 || opt->check_every < 1) return STF_E_INVALID;
    if (!(opt->eta0 > 0.0) || !(opt->tol >= 0.0) || !isfinite(opt->beta)) return STF_E_INVALID;
    if (opt->eta_rule == STF_ETA_CONST && !(opt->eta_const > 0.0)) return STF_E_INVALID;
    const bool fused = opt->fused != 0;
    if (fused) {
        // the single-pass form needs eta^k before the pass (the lagged pair),
        // the Gram kernel with column sums (p > 64), and a row-block pass with
        // the update in its epilogue (float64, or split bf16 with M_L in LDS)
        if (moptqr || opt->bb_index != STF_BB_LAGGED || opt->eta_rule == STF_ETA_DIFF ||
            prob->p <= 64)
            return STF_E_UNSUPPORTED;
        if (opt->precision != STF_PREC_FP64 &&
            !(opt->precision == STF_PREC_MIXED32 && make_res_plan(prob->n, prob->p, 256).nrb > 0))
            return STF_E_UNSUPPORTED;
    }
    const int dtype = (opt->precision == STF_PREC_FP64) ? STF_F64 : STF_F32;
    // a float32 A serves every form (the float64 form widens it exactly); a
    // float64 A only the float64 form
    if (prob->kind == STF_KIND_DENSE && prob->A_dtype == STF_F64 && dtype != STF_F64)
        return STF_E_UNSUPPORTED;

    Ws w;
    w.base = (char*)ws;
    w.L = make_layout(prob, opt->precision, moptqr, fused, true);
    if (ws_bytes < w.L.total) return STF_E_WORKSPACE;
    memset(res, 0, sizeof(*res));
    const int64_t n = prob->n;
    const int p = prob->p;

    IterCtx c;
    c.prob = prob;
    c.w = w;
    c.dtype = dtype;
    c.precision = nomaster ? STF_PREC_MIXED : opt->precision;
    c.X = X;
    c.Xm = (dtype == STF_F32 && !nomaster) ? w.at<double>(w.L.x64) : nullptr;
    c.g[0] = w.L.g[0];
    c.g[1] = w.L.g[1];
    c.st = w.at<DevState>(w.L.state);
    c.prm = w.at<DevParams>(w.L.params);
    c.moptqr = moptqr;
    c.fused = fused;
    c.xb[0] = X;
    c.xb[1] = (moptqr || fused) ? w.at<double>(w.L.xalt) : nullptr;
    void* xb64[2] = {c.xb[0], c.xb[1]};  // where the float64 phase keeps X^k

    DevParams hp;
    memset(&hp, 0, sizeof(hp));
    hp.beta = opt->beta;
    hp.eta0 = opt->eta0;
    hp.eta_const = opt->eta_const;
    hp.tol = opt->tol;
    hp.feas_blowup = opt->feas_blowup > 0.0 ? opt->feas_blowup : INFINITY;
    hp.variant = opt->variant;
    hp.mult_rule = moptqr ? STF_MULT_PSI : opt->mult_rule;
    hp.eta_rule = opt->eta_rule;
    hp.bb_index = opt->bb_index;
    hp.max_iter = opt->max_iter;
    hp.kkt_every = opt->kkt_every;
    hp.kkt_identity = 1;
    hp.switch_tol = (opt->precision == STF_PREC_FP64) ? 0.0 : std::max(0.0, opt->switch_tol);
    hp.switch_stall = kSwitchStall;
    hp.history = opt->history;
    hp.fused = fused ? 1 : 0;
    HIPCHK(hipMemcpyAsync(c.prm, &hp, sizeof(hp), hipMemcpyHostToDevice, s));
    launch_init_state(c.st, s);
    if (prob->kind == STF_KIND_STENCIL3D) launch_dst_init(prob, w.at<double>(w.L.dst), s);
    // X^0 of the float32 forms is kept for a float64 restart (see below)
    if (dtype == STF_F32)
        HIPCHK(hipMemcpyAsync(w.at<float>(w.L.x0keep), X, (size_t)n * p * 4,
                              hipMemcpyDeviceToDevice, s));
    // the float32 forms iterate on a float64 master copy; X holds its rounding
    if (c.Xm) launch_convert(STF_F64, X, STF_F32, c.Xm, (size_t)n * p, s);
    if (needs_rho(prob))
        launch_rowsq(c.Xm ? STF_F64 : dtype, c.Xm ? (const void*)c.Xm : X, n, p,
                     w.at<double>(w.L.rho), c.st, s);
    if ((rc = last_launch())) return rc;

    hipEvent_t e0, e1, e2;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventCreate(&e2));
    HIPCHK(hipEventRecord(e0, s));

    int chunk = std::max(1, opt->check_every);
    if (opt->use_graph && (chunk & 1)) chunk += 1;
    const bool prof = opt->profile != 0;
    std::vector<hipEvent_t> pev;
    if (prof) {
        pev.resize((size_t)chunk * (STF_NPROF + 1));
        for (auto& e : pev) HIPCHK(hipEventCreate(&e));
    }
    double kms[STF_NPROF] = {0};
    int prof_iters = 0;
    DevState hs;
    memset(&hs, 0, sizeof(hs));
    const int64_t limit = (int64_t)opt->max_iter + 1;

    // Enqueue iterations k0, k0+1, ... of context cc in chunks until the
    // device state says "done"; returns nonzero on a HIP error.
    auto run_phase = [&](const IterCtx& cc, int64_t k0) -> int {
        hipGraphExec_t gexec = nullptr;
        hipGraph_t graph = nullptr;
        // the legacy default stream cannot be captured: run uncaptured there
        if (opt->use_graph && !prof && s != nullptr) {
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return 1;
            for (int i = 0; i < chunk; ++i) enqueue_iteration(cc, (int)((k0 + i) & 1), s);
            if (hipStreamEndCapture(s, &graph) != hipSuccess) return 1;
            if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
                hipGraphDestroy(graph);
                return 1;
            }
        }
        int64_t enq = k0;
        int64_t last_todo = 0;
        int err = 0;
        while (true) {
            if (gexec) {
                if (hipGraphLaunch(gexec, s) != hipSuccess) { err = 1; break; }
                enq += chunk;
                last_todo = chunk;
            } else {
                // no iterations past max_iter: the last uncaptured chunk is clamped
                const int todo = (int)std::max<int64_t>(1, std::min<int64_t>(chunk, limit - enq));
                for (int i = 0; i < todo; ++i)
                    enqueue_iteration(cc, (int)((enq + i) & 1), s,
                                      prof ? &pev[(size_t)i * (STF_NPROF + 1)] : nullptr);
                enq += todo;
                last_todo = todo;
                if (last_launch()) { err = 1; break; }
            }
            if (hipMemcpyAsync(&hs, cc.st, sizeof(hs), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                err = 1;
                break;
            }
            if (prof) {
                // iterations after "done" are no-ops; count only the ones that ran
                const int64_t first = enq - last_todo;
                const int64_t last = hs.done ? (int64_t)hs.final_iter : enq - 1;
                for (int i = 0; i < last_todo && first + i <= last; ++i) {
                    hipEvent_t* e = &pev[(size_t)i * (STF_NPROF + 1)];
                    for (int g = 0; g < STF_NPROF; ++g) {
                        float ms = 0.f;
                        (void)hipEventElapsedTime(&ms, e[g], e[g + 1]);
                        kms[g] += ms;
                    }
                    ++prof_iters;
                }
            }
            if (hs.done) break;
            if (enq > limit + 2 * chunk) { err = 1; break; }  // stage 2 ends every run by max_iter
        }
        if (gexec) hipGraphExecDestroy(gexec);
        if (graph) hipGraphDestroy(graph);
        return err;
    };

    int hip_err = run_phase(c, 0);
    res->switch_iter = -1;
    res->restarted = 0;
    if (!hip_err && hs.done && hs.status == STF_SWITCH && hs.kkt > hs.kkt0 &&
        hs.kkt > hp.switch_tol * hs.kkt0) {
        // A reduced-precision descent that stalled at a point worse than X^0
        // has left the neighbourhood of the manifold (typically its columns
        // have collapsed onto a few directions, which float32 iterates cannot
        // separate again): its iterate is discarded and the float64 phase
        // starts over from X^0, so that the solve reaches what the float64
        // form reaches from the same start.
        res->switch_iter = (int)hs.final_iter;
        res->restarted = 1;
        IterCtx c64 = c;
        c64.dtype = STF_F64;
        c64.precision = STF_PREC_FP64;
        c64.X = w.at<double>(w.L.x64);
        c64.Xm = nullptr;
        launch_convert(STF_F64, w.at<float>(w.L.x0keep), STF_F32, c64.X, (size_t)n * p, s);
        if (fused) {
            c64.xb[0] = c64.X;
            c64.xb[1] = w.at<double>(w.L.xalt);
            xb64[0] = c64.xb[0];
            xb64[1] = c64.xb[1];
        }
        c64.g[0] = w.L.g64;
        c64.g[1] = w.L.g64b;
        hp.switch_tol = 0.0;
        if (hipMemcpyAsync(c.prm, &hp, sizeof(hp), hipMemcpyHostToDevice, s) != hipSuccess)
            hip_err = 1;
        launch_init_state(c.st, s);
        if (needs_rho(prob))
            launch_rowsq(STF_F64, c64.X, n, p, w.at<double>(w.L.rho), c.st, s);
        if (!hip_err && last_launch()) hip_err = 1;
        if (!hip_err) hip_err = run_phase(c64, 0);
    } else if (!hip_err && hs.done && hs.status == STF_SWITCH) {
        // Redo iteration k in float64 from the master iterate: the previous
        // gradL (float32, exact in float64) seeds the Barzilai-Borwein pair.
        const int64_t k = hs.final_iter;
        res->switch_iter = (int)k;
        IterCtx c64 = c;
        c64.dtype = STF_F64;
        c64.precision = STF_PREC_FP64;
        if (nomaster)  // the float64 phase starts from the float32 iterate
            launch_convert(STF_F64, fused ? c.xb[k & 1] : X, STF_F32, w.at<double>(w.L.x64),
                           (size_t)n * p, s);
        c64.X = w.at<double>(w.L.x64);
        if (fused) {
            // X^k (now in x64) and X^{k+1} alternate between x64 and xalt
            c64.xb[k & 1] = w.at<double>(w.L.x64);
            c64.xb[(k & 1) ^ 1] = w.at<double>(w.L.xalt);
            xb64[0] = c64.xb[0];
            xb64[1] = c64.xb[1];
        }
        c64.Xm = nullptr;
        c64.g[k & 1] = w.L.g64;
        c64.g[(k & 1) ^ 1] = w.L.g64b;
        if (k >= 1)
            launch_convert(STF_F64, w.base + c.g[(k & 1) ^ 1], STF_F32,
                           w.base + c64.g[(k & 1) ^ 1], (size_t)n * p, s);
        hp.switch_tol = 0.0;
        if (hipMemcpyAsync(c.prm, &hp, sizeof(hp), hipMemcpyHostToDevice, s) != hipSuccess)
            hip_err = 1;
        launch_resume_state(c.st, s);
        if (!hip_err) hip_err = run_phase(c64, k);
    }
    for (auto& e : pev) (void)hipEventDestroy(e);
    for (int g = 0; g < STF_NPROF; ++g) res->kernel_ms[g] = kms[g];
    res->prof_iters = prof_iters;
    if (hip_err) return STF_E_HIP;
    HIPCHK(hipEventRecord(e1, s));

    res->status = hs.status;
    res->iters = hs.final_iter;
    res->kkt0 = hs.kkt0;
    res->eta_last = hs.eta;
    if (hs.status == STF_E_DIVERGED) {
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        res->ms_loop = ms;
        res->kkt_abs = res->kkt_rel = res->feas = res->fval = NAN;
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        hipEventDestroy(e2);
        return STF_E_DIVERGED;
    }

    // MOptQR and the single-pass form: the returned iterate X^k sits in buffer
    // k & 1 (of the float64 phase, if the solve continued in float64)
    const int kf1 = hs.final_iter & 1;
    if (moptqr && kf1)
        HIPCHK(hipMemcpyAsync(X, c.xb[1], (size_t)n * p * 8, hipMemcpyDeviceToDevice, s));
    if (fused && (dtype == STF_F64 || res->switch_iter >= 0)) {
        // float64 iterates: into X (float64 form) or x64 (after a hand-over);
        // a float32 final iterate is converted from its buffer below
        void* dst = (dtype == STF_F64) ? X : (void*)w.at<double>(w.L.x64);
        if (xb64[kf1] != dst)
            HIPCHK(hipMemcpyAsync(dst, xb64[kf1], (size_t)n * p * 8, hipMemcpyDeviceToDevice, s));
    }
    // float64 copy of the returned iterate, CholeskyQR2, float64 evaluation
    double* Xd;
    double* tmp;
    if (dtype == STF_F64) {
        Xd = (double*)X;
        tmp = w.at<double>(w.L.g[1]);
    } else {
        Xd = w.at<double>(w.L.x64);
        tmp = w.at<double>(w.L.g64);
        // without a master, the float64 copy is the float32 iterate (unless a
        // float64 phase has taken over, which iterates on that copy)
        if (nomaster && res->switch_iter < 0)
            launch_convert(STF_F64, fused ? c.xb[kf1] : X, STF_F32, Xd, (size_t)n * p, s);
    }
    DevState* st_eval = w.at<DevState>(w.L.state_eval);
    launch_init_state(st_eval, s);
    if (opt->orth_final) {
        if ((rc = enqueue_cholqr2(prob, w, Xd, tmp, st_eval, s))) return rc;
    }
    DevState he;
    HIPCHK(hipMemcpyAsync(&he, st_eval, sizeof(he), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (opt->orth_final && he.info != 0) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        hipEventDestroy(e2);
        return STF_E_CHOLESKY;
    }
    double* G64 = (dtype == STF_F64) ? w.at<double>(w.L.g[0]) : w.at<double>(w.L.g64);
    if ((rc = enqueue_eval(prob, w, Xd, G64, s))) return rc;
    if (Lam_out)
        HIPCHK(hipMemcpyAsync(Lam_out, w.at<double>(w.L.Psi), (size_t)p * p * 8,
                              hipMemcpyDeviceToDevice, s));
    if (dtype == STF_F32) launch_convert(STF_F32, Xd, STF_F64, X, (size_t)n * p, s);
    if (X64_out)
        HIPCHK(hipMemcpyAsync(X64_out, Xd, (size_t)n * p * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(&he, st_eval, sizeof(he), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(e2, s));
    HIPCHK(hipStreamSynchronize(s));
    if ((rc = last_launch())) return rc;
    float ms1 = 0.f, ms2 = 0.f;
    hipEventElapsedTime(&ms1, e0, e1);
    hipEventElapsedTime(&ms2, e1, e2);
    res->ms_loop = ms1;
    res->ms_orth = ms2;
    res->fval = he.red[0];
    res->kkt_abs = he.red[1];
    res->feas = he.red[2];
    res->kkt_rel = (hs.kkt0 > 0.0) ? he.red[1] / hs.kkt0 : 0.0;
    // the in-loop stop test ran in the iteration's arithmetic on the iterate;
    // "converged" is reported only when the float64 check of the returned
    // point agrees
    if (res->status == STF_OK && hs.kkt0 > 0.0 && !(he.red[1] <= opt->tol * hs.kkt0))
        res->status = STF_TOL_UNMET;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipEventDestroy(e2);
    return res->status;
}

}  // namespace stf

using namespace stf;

extern "C" {

size_t stf_workspace_size(const stf_problem* prob, const stf_options* opt) {
    if (check_problem(prob) != STF_OK) return 0;
    if (opt)
        return make_layout(prob, opt->precision, opt->variant == STF_MOPTQR, opt->fused != 0,
                           true)
            .total;
    const size_t a = make_layout(prob, STF_PREC_FP64, true, true, true).total;
    const size_t b = make_layout(prob, STF_PREC_FP32, false, true, true).total;
    return a > b ? a : b;
}

int stf_solve(const stf_problem* prob, void* X, const stf_options* opt, void* ws,
              size_t ws_bytes, double* X64_out, double* Lam_out, stf_result* res,
              hipStream_t stream) {
    return solve_impl(prob, X, opt, ws, ws_bytes, X64_out, Lam_out, res, stream);
}

int plam_solve(const stf_problem* prob, void* X, const stf_options* opt, void* ws,
               size_t ws_bytes, double* X64_out, double* Lam_out, stf_result* res,
               hipStream_t stream) {
    if (!opt) return STF_E_INVALID;
    stf_options o = *opt;
    o.variant = STF_PLAM;
    return solve_impl(prob, X, &o, ws, ws_bytes, X64_out, Lam_out, res, stream);
}

int pcal_solve(const stf_problem* prob, void* X, const stf_options* opt, void* ws,
               size_t ws_bytes, double* X64_out, double* Lam_out, stf_result* res,
               hipStream_t stream) {
    if (!opt) return STF_E_INVALID;
    stf_options o = *opt;
    o.variant = STF_PCAL;
    return solve_impl(prob, X, &o, ws, ws_bytes, X64_out, Lam_out, res, stream);
}

static int step_ws(const stf_problem* prob, void* ws, size_t ws_bytes, Ws& w) {
    int rc = check_problem(prob);
    if (rc) return rc;
    if (!ws) return STF_E_INVALID;
    w.base = (char*)ws;
    w.L = make_layout(prob, STF_PREC_FP32);  // the larger layout (has float64 scratch)
    if (ws_bytes < w.L.total) return STF_E_WORKSPACE;
    return STF_OK;
}

int stf_gradient(const stf_problem* prob, const void* X, void* G, int32_t dtype, void* ws,
                 size_t ws_bytes, hipStream_t stream) {
    Ws w;
    int rc = step_ws(prob, ws, ws_bytes, w);
    if (rc) return rc;
    if (!X || !G || (dtype != STF_F64 && dtype != STF_F32)) return STF_E_INVALID;
    if (prob->kind == STF_KIND_DENSE && prob->A_dtype == STF_F64 && dtype != STF_F64)
        return STF_E_UNSUPPORTED;
    if (prob->kind == STF_KIND_STENCIL3D) launch_dst_init(prob, w.at<double>(w.L.dst), stream);
    rc = enqueue_gradient(prob, w, dtype, X, G, nullptr, stream);
    if (rc) return rc;
    return hipStreamSynchronize(stream) == hipSuccess ? last_launch() : STF_E_HIP;
}

int stf_hartree(const stf_problem* prob, const double* rho, double* phi, void* ws,
                size_t ws_bytes, hipStream_t stream) {
    Ws w;
    int rc = step_ws(prob, ws, ws_bytes, w);
    if (rc) return rc;
    if (!rho || !phi || prob->kind == STF_KIND_DENSE) return STF_E_INVALID;
    if (prob->kind == STF_KIND_STENCIL3D) launch_dst_init(prob, w.at<double>(w.L.dst), stream);
    launch_hartree(prob, rho, phi, w.at<double>(w.L.hscr), w.at<double>(w.L.dst), nullptr,
                   stream);
    return hipStreamSynchronize(stream) == hipSuccess ? last_launch() : STF_E_HIP;
}

int stf_gram(const stf_problem* prob, const void* X, const void* G, int32_t dtype,
             int32_t precision, double* S, double* W, void* ws, size_t ws_bytes,
             hipStream_t stream) {
    Ws w;
    int rc = step_ws(prob, ws, ws_bytes, w);
    if (rc) return rc;
    if (!X || !G || !S || !W) return STF_E_INVALID;
    if (dtype != STF_F64 && dtype != STF_F32) return STF_E_INVALID;
    if (precision < STF_PREC_FP64 || precision > STF_PREC_MIXED) return STF_E_INVALID;
    if ((precision == STF_PREC_FP64) != (dtype == STF_F64)) return STF_E_UNSUPPORTED;
    launch_gram(dtype, precision, w.L.gram64, X, G, prob->n, prob->p,
                w.at<double>(w.L.gram_part), S, W, nullptr, stream);
    return hipStreamSynchronize(stream) == hipSuccess ? last_launch() : STF_E_HIP;
}

int stf_cholqr2(const stf_problem* prob, double* X, void* ws, size_t ws_bytes,
                hipStream_t stream) {
    Ws w;
    int rc = step_ws(prob, ws, ws_bytes, w);
    if (rc) return rc;
    if (!X) return STF_E_INVALID;
    DevState* st = w.at<DevState>(w.L.state_eval);
    launch_init_state(st, stream);
    rc = enqueue_cholqr2(prob, w, X, w.at<double>(w.L.g64), st, stream);
    if (rc) return rc;
    DevState he;
    HIPCHK(hipMemcpyAsync(&he, st, sizeof(he), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (he.info != 0) return STF_E_CHOLESKY;
    return last_launch();
}

int stf_eval(const stf_problem* prob, const double* X, double* out3, void* ws, size_t ws_bytes,
             hipStream_t stream) {
    Ws w;
    int rc = step_ws(prob, ws, ws_bytes, w);
    if (rc) return rc;
    if (!X || !out3) return STF_E_INVALID;

    if (prob->kind == STF_KIND_STENCIL3D) launch_dst_init(prob, w.at<double>(w.L.dst), stream);
    rc = enqueue_eval(prob, w, X, w.at<double>(w.L.g64), stream);
    if (rc) return rc;
    DevState he;
    HIPCHK(hipMemcpyAsync(&he, w.at<DevState>(w.L.state_eval), sizeof(he),
                          hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    out3[0] = he.red[0];
    out3[1] = he.red[1];
    out3[2] = he.red[2];
    return last_launch();
}

const char* stf_strerror(int code) {
    switch (code) {
        case STF_OK: return "converged";
        case STF_MAX_ITER: return "maximum number of iterations reached";
        case STF_TOL_UNMET:
            return "stop test met in the iteration, float64 check of the returned point above tol";
        case STF_E_INVALID: return "invalid argument";
        case STF_E_DIVERGED: return "iteration diverged (non-finite values or infeasibility blow-up)";
        case STF_E_HIP: return "HIP runtime error";
        case STF_E_UNSUPPORTED: return "unsupported option combination";
        case STF_E_WORKSPACE: return "workspace too small";
        case STF_E_CHOLESKY: return "CholeskyQR2 met a non-positive pivot";
        case STF_E_SCRATCH: return "problem too large for the static scratch buffer";
        default: return "unknown status";
    }
}

const char* stf_version(void) { return "stiefel-gfx950 0.1"; }

}  // extern "C"
