// Batched PLAM / PCAL driver (declared in include/stiefel.h): many independent
// 1D Kohn-Sham-type problems of uneven n and p solved together.
//
// Every stage of an iteration is ONE grouped launch over all problems (the
// Gram pass and the mixed residual pass: one launch per tile-shape bucket);
// workgroups find their problem through a prefix table, and each problem keeps
// its own device state, so a converged problem's workgroups return at once.
// A chunk of iterations is captured once as a HIP graph and replayed; the host
// reads every problem's state once per chunk and stops when all are done.  In
// the float32 forms with a switch_tol, every iteration runs the float32 groups,
// a per-problem hand-over and the float64 groups (second descriptors: the
// float64 master, float64 gradient buffers, own state and parameters): a
// problem that reaches its switch_tol continues in float64 in the same
// iteration, as a single solve does, while the others go on in float32.
// Tile shapes per problem: the Gram bucket (MFMA tiles per wave) follows p;
// the number of split-K chunks and residual row blocks follows the problem's
// share of the batch's n p^2 work, from a batch-wide workgroup budget that
// stf_batched_tune() can pick by timing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "stf_internal.h"

namespace stf {

namespace {

constexpr int kGramBudget = 2048;   // default batch-wide Gram workgroups
constexpr int kResBudget = 2048;    // default batch-wide residual workgroups (tile 128)
constexpr int kMixBudget = 512;     // default batch-wide mixed residual workgroups (tile 256)

struct Group {
    std::vector<int32_t> list, off;
    int key = 0;
    size_t dev_list = 0, dev_off = 0;  // workspace offsets of the tables
};

struct BatchPlan {
    int nprob = 0;
    int precision = STF_PREC_FP64;
    int dtype = STF_F64;
    std::vector<size_t> pbase;      // workspace offset of each problem's share
    std::vector<Layout> L;          // per-problem single-problem layouts
    std::vector<GramPlan> gram;     // batched plans
    std::vector<ResPlan> res;
    std::vector<int32_t> nblk_rows;
    std::vector<Group> groups[BS_ROWSQ + 1];
    // float32 forms: the float64 continuation after a hand-over (switch_tol)
    std::vector<ResPlan> res64;
    std::vector<Group> groups64[BS_ROWSQ + 1];
    size_t desc = 0;                // BDesc[nprob]
    size_t states = 0;              // DevState[nprob]: gathered device states
    size_t desc64 = 0;              // float32 forms: BDesc[nprob] of the float64 continuation
    size_t states64 = 0;            //   and its gathered states
    size_t tables = 0, table_bytes = 0;
    size_t total = 0;
};

// opts: host array of nprob option sets, or null (sizes only).
int batch_check(int32_t nprob, const stf_problem* probs, const stf_options* opts) {
    if (nprob <= 0 || !probs) return STF_E_INVALID;
    for (int b = 0; b < nprob; ++b) {
        const int rc = check_problem(&probs[b]);
        if (rc) return rc;
        // the grouped Hartree and gradient passes are the 1D ones of Problem 1
        if (probs[b].kind != STF_KIND_STENCIL1D) return STF_E_UNSUPPORTED;
        if (probs[b].Glin || probs[b].B || probs[b].gamma != 0.0 || probs[b].block != 0)
            return STF_E_UNSUPPORTED;
    }
    if (opts) {
        const int prec = opts[0].precision;
        if (prec < STF_PREC_FP64 || prec > STF_PREC_MIXED) return STF_E_INVALID;
        for (int b = 0; b < nprob; ++b) {
            const stf_options& o = opts[b];
            // one storage dtype and kernel set for the whole batch
            if (o.precision != prec) return STF_E_INVALID;
            if (o.variant != STF_PLAM && o.variant != STF_PCAL) return STF_E_INVALID;
            if (o.mult_rule != STF_MULT_PSI && o.mult_rule != STF_MULT_PSI_PHI)
                return STF_E_INVALID;
            if (o.mult_rule == STF_MULT_PSI_PHI && o.variant != STF_PCAL) return STF_E_UNSUPPORTED;
            if (o.eta_rule < STF_ETA_CONST || o.eta_rule > STF_ETA_ABB) return STF_E_INVALID;
            if (o.bb_index != STF_BB_STANDARD && o.bb_index != STF_BB_LAGGED) return STF_E_INVALID;
            if (o.max_iter < 0 || o.kkt_every < 1 || o.check_every < 1) return STF_E_INVALID;
            if (!(o.eta0 > 0.0) || !(o.tol >= 0.0) || !isfinite(o.beta)) return STF_E_INVALID;
            if (o.eta_rule == STF_ETA_CONST && !(o.eta_const > 0.0)) return STF_E_INVALID;
            if (o.fused) return STF_E_UNSUPPORTED;  // the single-pass form: one problem only
            if (prec == STF_PREC_MIXED && (probs[b].p + 31) / 32 * 32 > 384)
                return STF_E_UNSUPPORTED;
        }
    }
    return STF_OK;
}

// Shapes and workspace of a batch.  budget_* <= 0 selects the defaults.
BatchPlan make_batch_plan(int32_t nprob, const stf_problem* probs, int precision,
                          int budget_gram, int budget_res) {
    BatchPlan P;
    P.nprob = nprob;
    P.precision = precision;
    P.dtype = (precision == STF_PREC_FP64) ? STF_F64 : STF_F32;
    const bool mixed = precision == STF_PREC_MIXED;
    const int bg = budget_gram > 0 ? budget_gram : kGramBudget;
    const int br = budget_res > 0 ? budget_res : (mixed ? kMixBudget : kResBudget);
    double wsum = 0.0;
    for (int b = 0; b < nprob; ++b) wsum += (double)probs[b].n * probs[b].p * probs[b].p;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    P.desc = take(sizeof(BDesc) * (size_t)nprob);
    P.states = take(sizeof(DevState) * (size_t)nprob);
    if (P.dtype == STF_F32) {
        P.desc64 = take(sizeof(BDesc) * (size_t)nprob);
        P.states64 = take(sizeof(DevState) * (size_t)nprob);
    }
    P.L.resize(nprob);
    P.gram.resize(nprob);
    P.res.resize(nprob);
    P.res64.resize(nprob);
    P.nblk_rows.resize(nprob);
    P.pbase.resize(nprob);
    for (int b = 0; b < nprob; ++b) {
        const stf_problem& pr = probs[b];
        const double share = (double)pr.n * pr.p * pr.p / wsum;
        P.L[b] = make_layout(&pr, precision);
        // batched plans never exceed the single-problem ones the layout is sized for
        // W = X^T grad f(X) is symmetric here: upper blocks only
        const GramPlan g0 = make_gram_plan(pr.n, pr.p, 1024, true);
        const int64_t tg = std::max<int64_t>(g0.n_tiles, (int64_t)llround(bg * share));
        P.gram[b] = make_gram_plan(pr.n, pr.p, std::min<int64_t>(tg, 1024), true);
        {
            const ResPlan r0 = make_res_plan(pr.n, pr.p, 128);
            const int64_t tr = std::max<int64_t>(r0.ncb, (int64_t)llround(kResBudget * share));
            P.res64[b] = make_res_plan(pr.n, pr.p, 128, std::min<int64_t>(tr, 1024));
        }
        if (mixed) {
            const ResPlan r0 = make_res_plan(pr.n, pr.p, 256);
            const int64_t tr = std::max<int64_t>(r0.ncb, (int64_t)llround(br * share));
            P.res[b] = make_res_plan(pr.n, pr.p, 256, std::min<int64_t>(tr, 256));
        } else {
            const ResPlan r0 = make_res_plan(pr.n, pr.p, 128);
            const int64_t tr = std::max<int64_t>(r0.ncb, (int64_t)llround(br * share));
            P.res[b] = make_res_plan(pr.n, pr.p, 128, std::min<int64_t>(tr, 1024));
        }
        const int64_t rows4 = std::max<int64_t>(1, (pr.n + 3) / 4);
        const int64_t want = std::max<int64_t>(1, ((int64_t)pr.n * pr.p + 8191) / 8192);
        P.nblk_rows[b] = (int32_t)std::min<int64_t>(std::min<int64_t>(rows4, want), 65536);
    }
    // grouped-launch tables, for the batch's form and (float32 forms) for the
    // float64 continuation
    std::vector<Group>* G = nullptr;
    auto add = [&](int stage, int key, const std::vector<int>& members,
                   const std::vector<int32_t>& wgs) {
        Group g;
        g.key = key;
        g.off.push_back(0);
        for (size_t i = 0; i < members.size(); ++i) {
            if (wgs[i] <= 0) continue;
            g.list.push_back(members[i]);
            g.off.push_back(g.off.back() + wgs[i]);
        }
        if (!g.list.empty()) G[stage].push_back(g);
    };
    std::vector<int> all(nprob), hart;
    std::iota(all.begin(), all.end(), 0);
    for (int b = 0; b < nprob; ++b)
        if (probs[b].alpha != 0.0) hart.push_back(b);
    auto wg_of = [&](const std::vector<int>& m, auto f) {
        std::vector<int32_t> w;
        for (int b : m) w.push_back((int32_t)f(b));
        return w;
    };
    auto build = [&](bool mx, const std::vector<ResPlan>& RP) {
        add(BS_HARTREE, 0, hart, wg_of(hart, [&](int) { return 1; }));
        add(BS_ROWSQ, 0, hart, wg_of(hart, [&](int b) { return P.nblk_rows[b]; }));
        add(BS_GRAD, 0, all, wg_of(all, [&](int b) { return P.nblk_rows[b]; }));
        for (int wm : {1, 2, 4}) {
            std::vector<int> m;
            for (int b = 0; b < nprob; ++b)
                if (P.gram[b].wm == wm) m.push_back(b);
            add(BS_GRAM, wm, m, wg_of(m, [&](int b) { return P.gram[b].n_tiles * P.gram[b].nchunks; }));
        }
        add(BS_REDUCE, 0, all, wg_of(all, [&](int b) {
                const GramPlan& g = P.gram[b];
                return ((int64_t)g.n_tiles * g.bt * g.bt + 63) / 64;
            }));
        add(BS_STAGE1, 0, all, wg_of(all, [&](int b) { return probs[b].p; }));
        add(BS_PPGEMM, 0, all, wg_of(all, [&](int b) {
                const int t = (probs[b].p + 15) / 16;
                return t * t;
            }));
        if (mx) {
            add(BS_SPLIT, 0, all, wg_of(all, [&](int b) {
                    const int64_t prow = (int64_t)RP[b].ncb * 64, pk = (probs[b].p + 31) / 32 * 32;
                    return (prow * pk + 255) / 256;
                }));
            for (int pkmax : {128, 256, 384}) {
                std::vector<int> m;
                for (int b = 0; b < nprob; ++b) {
                    const int pk = (probs[b].p + 31) / 32 * 32;
                    const int key = pk <= 128 ? 128 : (pk <= 256 ? 256 : 384);
                    if (key == pkmax) m.push_back(b);
                }
                add(BS_RESID, pkmax, m, wg_of(m, [&](int b) { return RP[b].nrb * RP[b].ncb; }));
            }
        } else {
            add(BS_RESID, 0, all, wg_of(all, [&](int b) { return RP[b].nrb * RP[b].ncb; }));
        }
        add(BS_COLRED, 0, all, wg_of(all, [&](int b) {
                return (2 * probs[b].p + 63) / 64 * col_groups(RP[b].nrb);
            }));
        add(BS_STAGE2, 0, all, wg_of(all, [&](int) { return 1; }));
        add(BS_UPDATE, 0, all, wg_of(all, [&](int b) { return P.nblk_rows[b]; }));
    };
    G = P.groups;
    build(mixed, P.res);
    if (P.dtype == STF_F32) {
        G = P.groups64;
        build(false, P.res64);
    }
    // table storage
    P.tables = off;
    size_t tb = 0;
    for (auto* GS : {P.groups, P.groups64})
        for (int st = 0; st <= BS_ROWSQ; ++st)
            for (auto& g : GS[st]) {
                g.dev_list = P.tables + tb;
                tb += g.list.size() * 4;
                g.dev_off = P.tables + tb;
                tb += g.off.size() * 4;
            }
    P.table_bytes = tb;
    off = align256(P.tables + tb);
    for (int b = 0; b < nprob; ++b) P.pbase[b] = take(P.L[b].total);
    P.total = off;
    return P;
}

// One iteration of every problem: the grouped launches of `groups` with the
// kernels of (dtype, precision) on the descriptors d.
void enqueue_batched_iteration(const BatchPlan& P, const std::vector<Group>* groups, int dtype,
                               int precision, const BDesc* d, char* ws, int parity,
                               hipStream_t s) {
    auto run = [&](int stage) {
        for (const Group& g : groups[stage]) {
            BGroup bg;
            bg.list = (const int32_t*)(ws + g.dev_list);
            bg.off = (const int32_t*)(ws + g.dev_off);
            bg.cnt = (int32_t)g.list.size();
            bg.total = g.off.back();
            launch_batched(stage, dtype, precision, g.key, d, bg, parity, s);
        }
    };
    run(BS_HARTREE);
    run(BS_GRAD);
    run(BS_GRAM);
    run(BS_REDUCE);
    run(BS_STAGE1);
    run(BS_PPGEMM);
    if (precision == STF_PREC_MIXED) run(BS_SPLIT);
    run(BS_RESID);
    run(BS_COLRED);
    run(BS_STAGE2);
    run(BS_UPDATE);
}

#define HIPCHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return STF_E_HIP;   \
    } while (0)

// Host copies of the per-problem descriptors and tables, and device parameters.
int setup_batch(const BatchPlan& P, const stf_problem* probs, void* const* X,
                const stf_options* opts, char* ws, std::vector<BDesc>& hd,
                std::vector<int32_t>& htab, std::vector<DevParams>& hp, hipStream_t s) {
    hd.resize(P.nprob);
    for (int b = 0; b < P.nprob; ++b) {
        const Layout& L = P.L[b];
        char* base = ws + P.pbase[b];
        auto at = [&](size_t o) { return (double*)(base + o); };
        BDesc& d = hd[b];
        memset(&d, 0, sizeof(d));
        d.n = probs[b].n;
        d.p = probs[b].p;
        d.alpha = probs[b].alpha;
        d.v = probs[b].v;
        d.X = X[b];
        d.Xm = (P.dtype == STF_F32) ? at(L.x64) : nullptr;
        d.g[0] = base + L.g[0];
        d.g[1] = base + L.g[1];
        d.rho = at(L.rho);
        d.phi = at(L.phi);
        d.S = at(L.S);
        d.W = at(L.W);
        d.Psi = at(L.Psi);
        d.ML = at(L.ML);
        d.Bm = at(L.Bm);
        d.T1 = at(L.T1);
        d.fpart = at(L.fpart);
        d.nu = at(L.nu);
        d.colpart = at(L.colpart);
        d.gram_part = at(L.gram_part);
        d.res_col = at(L.res_col);
        d.res_scal = at(L.res_scal);
        d.mix = (__bf16*)(base + L.mix);
        d.st = (DevState*)(base + L.state);
        d.prm = (DevParams*)(base + L.params);
        d.gram = P.gram[b];
        d.res = P.res[b];
        d.nblk_rows = P.nblk_rows[b];
    }
    HIPCHK(hipMemcpyAsync(ws + P.desc, hd.data(), sizeof(BDesc) * hd.size(),
                          hipMemcpyHostToDevice, s));
    htab.assign(P.table_bytes / 4, 0);
    for (const auto* GS : {P.groups, P.groups64})
        for (int st = 0; st <= BS_ROWSQ; ++st)
            for (const auto& g : GS[st]) {
                memcpy((char*)htab.data() + (g.dev_list - P.tables), g.list.data(),
                       g.list.size() * 4);
                memcpy((char*)htab.data() + (g.dev_off - P.tables), g.off.data(),
                       g.off.size() * 4);
            }
    if (P.table_bytes)
        HIPCHK(hipMemcpyAsync(ws + P.tables, htab.data(), P.table_bytes, hipMemcpyHostToDevice,
                              s));
    hp.assign(P.nprob, DevParams{});
    for (int b = 0; b < P.nprob; ++b) {
        const stf_options* opt = &opts[b];
        DevParams& q = hp[b];
        memset(&q, 0, sizeof(q));
        q.beta = opt->beta;
        q.eta0 = opt->eta0;
        q.eta_const = opt->eta_const;
        q.tol = opt->tol;
        q.feas_blowup = opt->feas_blowup > 0.0 ? opt->feas_blowup : INFINITY;
        q.variant = opt->variant;
        q.mult_rule = opt->mult_rule;
        q.eta_rule = opt->eta_rule;
        q.bb_index = opt->bb_index;
        q.max_iter = opt->max_iter;
        q.kkt_every = opt->kkt_every;
        q.kkt_identity = 1;
        q.switch_tol = (P.dtype == STF_F32) ? std::max(0.0, opt->switch_tol) : 0.0;
        q.switch_stall = kSwitchStall;
        q.history = nullptr;
        HIPCHK(hipMemcpyAsync(hd[b].prm, &q, sizeof(q), hipMemcpyHostToDevice, s));
        launch_init_state(hd[b].st, s);
        if (hd[b].Xm)
            launch_convert(STF_F64, X[b], STF_F32, hd[b].Xm, (size_t)hd[b].n * hd[b].p, s);
    }
    // row sums of squares of X^0 for the first Hartree solve
    {
        const char* w = ws;
        for (const Group& g : P.groups[BS_ROWSQ]) {
            BGroup bg;
            bg.list = (const int32_t*)(w + g.dev_list);
            bg.off = (const int32_t*)(w + g.dev_off);
            bg.cnt = (int32_t)g.list.size();
            bg.total = g.off.back();
            launch_batched(BS_ROWSQ, P.dtype, P.precision, 0, (const BDesc*)(ws + P.desc), bg,
                           0, s);
        }
    }
    // the host arrays are read by the copies above: finish them before returning
    HIPCHK(hipStreamSynchronize(s));
    return last_launch();
}

int batched_impl(int32_t nprob, const stf_problem* probs, void* const* X,
                 const stf_options* opts, void* ws, size_t ws_bytes, stf_result* res,
                 hipStream_t s, int budget_gram, int budget_res, double* ms_per_iter) {
    if (!opts) return STF_E_INVALID;
    int rc = batch_check(nprob, probs, opts);
    if (rc) return rc;
    if (!X || !ws || !res) return STF_E_INVALID;
    for (int b = 0; b < nprob; ++b)
        if (!X[b]) return STF_E_INVALID;
    // loop-level settings come from the first option set
    const stf_options* opt = &opts[0];
    const BatchPlan P = make_batch_plan(nprob, probs, opt->precision, budget_gram, budget_res);
    if (ws_bytes < P.total) return STF_E_WORKSPACE;
    char* w = (char*)ws;
    for (int b = 0; b < nprob; ++b) memset(&res[b], 0, sizeof(stf_result));
    std::vector<BDesc> hd;
    std::vector<int32_t> htab;
    std::vector<DevParams> hpv;
    if ((rc = setup_batch(P, probs, X, opts, w, hd, htab, hpv, s))) return rc;

    hipEvent_t e0, e1, e2;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventCreate(&e2));
    HIPCHK(hipEventRecord(e0, s));
    int chunk = std::max(1, opt->check_every);
    if (opt->use_graph && (chunk & 1)) chunk += 1;
    std::vector<DevState> hs(nprob);
    int64_t limit = 1;
    for (int b = 0; b < nprob; ++b) limit = std::max<int64_t>(limit, (int64_t)opts[b].max_iter + 1);
    int64_t iters_run = 0;

    // float32 forms with a hand-over: every problem that reaches its switch_tol
    // (or stalls) continues in float64 at once, on its own, while the others go
    // on in float32: each iteration runs the float32 kernels on the float32
    // descriptors, the per-problem hand-over, then the float64 kernels on the
    // continuation descriptors (their states start done, so those workgroups
    // return at once until a problem hands over).
    bool any_sw = false;
    for (int b = 0; b < nprob; ++b) any_sw = any_sw || (hpv[b].switch_tol > 0.0);
    const bool two = (P.dtype == STF_F32) && any_sw;
    const BDesc* d32 = (const BDesc*)(w + P.desc);
    const BDesc* d64 = two ? (const BDesc*)(w + P.desc64) : nullptr;
    std::vector<DevState> hs64(nprob);
    if (two) {
        std::vector<BDesc> hd64 = hd;
        for (int b = 0; b < nprob; ++b) {
            const Layout& L = P.L[b];
            char* base = w + P.pbase[b];
            BDesc& d = hd64[b];
            d.X = d.Xm;  // the float64 master
            d.Xm = nullptr;
            d.g[0] = base + L.g64;
            d.g[1] = base + L.g64b;
            d.res = P.res64[b];
            d.st = (DevState*)(base + L.state64);
            d.prm = (DevParams*)(base + L.params64);
            DevParams q = hpv[b];
            q.switch_tol = 0.0;
            HIPCHK(hipMemcpyAsync(d.prm, &q, sizeof(q), hipMemcpyHostToDevice, s));
            DevState z;
            memset(&z, 0, sizeof(z));
            z.done = 1;
            HIPCHK(hipMemcpyAsync(d.st, &z, sizeof(z), hipMemcpyHostToDevice, s));
        }
        HIPCHK(hipMemcpyAsync(w + P.desc64, hd64.data(), sizeof(BDesc) * hd64.size(),
                              hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));  // the host arrays above are read by the copies
    }
    auto enqueue = [&](int parity) {
        enqueue_batched_iteration(P, P.groups, P.dtype, P.precision, d32, w, parity, s);
        if (two) {
            launch_batched_switch(d32, d64, nprob, parity, s);
            enqueue_batched_iteration(P, P.groups64, STF_F64, STF_PREC_FP64, d64, w, parity, s);
        }
    };
    // the state that describes problem b now
    auto cur = [&](int b) -> const DevState& {
        return (two && hs[b].status == STF_SWITCHED) ? hs64[b] : hs[b];
    };

    // Enqueue iterations until every problem is done; nonzero on a HIP error.
    auto run_phase = [&]() -> int {
        hipGraphExec_t gexec = nullptr;
        hipGraph_t graph = nullptr;
        if (opt->use_graph && s != nullptr) {
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return 1;
            for (int i = 0; i < chunk; ++i) enqueue(i & 1);
            if (hipStreamEndCapture(s, &graph) != hipSuccess) return 1;
            if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
                hipGraphDestroy(graph);
                return 1;
            }
        }
        int64_t enq = 0;
        int err = 0;
        while (true) {
            if (gexec) {
                if (hipGraphLaunch(gexec, s) != hipSuccess) { err = 1; break; }
                enq += chunk;
            } else {
                const int todo = (int)std::max<int64_t>(1, std::min<int64_t>(chunk, limit - enq));
                for (int i = 0; i < todo; ++i) enqueue((int)((enq + i) & 1));
                enq += todo;
                if (last_launch()) { err = 1; break; }
            }
            launch_gather_states(d32, nprob, (DevState*)(w + P.states), s);
            if (two) launch_gather_states(d64, nprob, (DevState*)(w + P.states64), s);
            if (hipMemcpyAsync(hs.data(), w + P.states, sizeof(DevState) * (size_t)nprob,
                               hipMemcpyDeviceToHost, s) != hipSuccess ||
                (two && hipMemcpyAsync(hs64.data(), w + P.states64,
                                       sizeof(DevState) * (size_t)nprob,
                                       hipMemcpyDeviceToHost, s) != hipSuccess) ||
                hipStreamSynchronize(s) != hipSuccess) {
                err = 1;
                break;
            }
            bool all = true;
            int64_t mx = 0;
            for (int b = 0; b < nprob; ++b) {
                const DevState& c = cur(b);
                all = all && c.done;
                mx = std::max<int64_t>(mx, c.done ? c.final_iter : c.iter);
            }
            iters_run = mx;
            if (all) break;
            if (enq > limit + 2 * chunk) { err = 1; break; }
        }
        if (gexec) hipGraphExecDestroy(gexec);
        if (graph) hipGraphDestroy(graph);
        return err;
    };

    if (run_phase()) return STF_E_HIP;
    std::vector<int> switched(nprob, -1);
    for (int b = 0; b < nprob; ++b)
        if (two && hs[b].status == STF_SWITCHED) switched[b] = hs[b].final_iter;
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms_loop = 0.f;
    hipEventElapsedTime(&ms_loop, e0, e1);
    if (ms_per_iter) *ms_per_iter = iters_run > 0 ? ms_loop / (double)iters_run : 0.0;

    // per problem: CholeskyQR2 and the float64 evaluation, as in a single
    // solve, all enqueued back to back with one read-back after each phase
    int worst = STF_OK;
    std::vector<Ws> pws(nprob);
    std::vector<double*> xds(nprob);
    std::vector<char> live(nprob, 0);
    std::vector<DevState> he(nprob);
    for (int b = 0; b < nprob; ++b) {
        stf_result& r = res[b];
        const DevState& hb = cur(b);
        r.status = hb.status;
        r.iters = hb.final_iter;
        r.kkt0 = hb.kkt0;
        r.eta_last = hb.eta;
        r.ms_loop = ms_loop;
        r.switch_iter = switched[b];
        if (hb.status == STF_E_DIVERGED) {
            r.kkt_abs = r.kkt_rel = r.feas = r.fval = NAN;
            worst = STF_E_DIVERGED;
            continue;
        }
        live[b] = 1;
        Ws& pw = pws[b];
        pw.base = w + P.pbase[b];
        pw.L = P.L[b];
        xds[b] = (P.dtype == STF_F64) ? (double*)X[b]
                                      : pw.at<double>(pw.L.x64);  // the float64 master
        double* tmp = (P.dtype == STF_F64) ? pw.at<double>(pw.L.g[1]) : pw.at<double>(pw.L.g64);
        DevState* st_eval = pw.at<DevState>(pw.L.state_eval);
        launch_init_state(st_eval, s);
        if (opts[b].orth_final && (rc = enqueue_cholqr2(&probs[b], pw, xds[b], tmp, st_eval, s)))
            return rc;
        HIPCHK(hipMemcpyAsync(&he[b], st_eval, sizeof(DevState), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    for (int b = 0; b < nprob; ++b) {
        if (!live[b]) continue;
        if (opts[b].orth_final && he[b].info != 0) {
            res[b].status = STF_E_CHOLESKY;
            worst = std::min(worst, (int)STF_E_CHOLESKY);
            live[b] = 0;
            continue;
        }
        const Ws& pw = pws[b];
        double* G64 = (P.dtype == STF_F64) ? pw.at<double>(pw.L.g[0]) : pw.at<double>(pw.L.g64);
        if ((rc = enqueue_eval(&probs[b], pw, xds[b], G64, s))) return rc;
        if (P.dtype == STF_F32)
            launch_convert(STF_F32, xds[b], STF_F64, X[b], (size_t)probs[b].n * probs[b].p, s);
        HIPCHK(hipMemcpyAsync(&he[b], pw.at<DevState>(pw.L.state_eval), sizeof(DevState),
                              hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    for (int b = 0; b < nprob; ++b) {
        if (!live[b]) continue;
        stf_result& r = res[b];
        r.fval = he[b].red[0];
        r.kkt_abs = he[b].red[1];
        r.feas = he[b].red[2];
        r.kkt_rel = (cur(b).kkt0 > 0.0) ? he[b].red[1] / cur(b).kkt0 : 0.0;
        if (r.status == STF_OK && cur(b).kkt0 > 0.0 &&
            !(he[b].red[1] <= opts[b].tol * cur(b).kkt0))
            r.status = STF_TOL_UNMET;
        // aggregate: the first error, else MAX_ITER, else TOL_UNMET, else OK
        if (worst >= 0 && r.status > 0)
            worst = (worst == STF_MAX_ITER || r.status == STF_MAX_ITER) ? STF_MAX_ITER : r.status;
    }
    HIPCHK(hipEventRecord(e2, s));
    HIPCHK(hipEventSynchronize(e2));
    float ms_orth = 0.f;
    hipEventElapsedTime(&ms_orth, e1, e2);
    for (int b = 0; b < nprob; ++b) res[b].ms_orth = ms_orth;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipEventDestroy(e2);
    if ((rc = last_launch())) return rc;
    return worst;
}

}  // namespace

}  // namespace stf

using namespace stf;

extern "C" {

size_t stf_batched_workspace_size(int32_t nprob, const stf_problem* probs,
                                  const stf_options* opts) {
    if (batch_check(nprob, probs, opts) != STF_OK) return 0;
    if (opts) return make_batch_plan(nprob, probs, opts[0].precision, 0, 0).total;
    size_t m = 0;
    for (int prec : {STF_PREC_FP64, STF_PREC_FP32, STF_PREC_MIXED}) {
        bool ok = true;
        if (prec == STF_PREC_MIXED)
            for (int b = 0; b < nprob; ++b)
                ok = ok && (probs[b].p + 31) / 32 * 32 <= 384;
        if (ok) m = std::max(m, make_batch_plan(nprob, probs, prec, 0, 0).total);
    }
    return m;
}

int stf_solve_batched(int32_t nprob, const stf_problem* probs, void* const* X,
                      const stf_options* opts, void* ws, size_t ws_bytes, stf_result* res,
                      hipStream_t stream) {
    return batched_impl(nprob, probs, X, opts, ws, ws_bytes, res, stream, 0, 0, nullptr);
}

int stf_solve_batched_ex(int32_t nprob, const stf_problem* probs, void* const* X,
                         const stf_options* opts, void* ws, size_t ws_bytes, stf_result* res,
                         int32_t budget_gram, int32_t budget_res, double* ms_per_iter,
                         hipStream_t stream) {
    return batched_impl(nprob, probs, X, opts, ws, ws_bytes, res, stream, budget_gram,
                        budget_res, ms_per_iter);
}

int stf_batched_tune(int32_t nprob, const stf_problem* probs, void* const* X,
                     const stf_options* opts, void* ws, size_t ws_bytes, int32_t iters,
                     int32_t* best_gram, int32_t* best_res, double* best_ms_per_iter,
                     hipStream_t stream) {
    if (!opts || !best_gram || !best_res || iters < 1 || nprob <= 0) return STF_E_INVALID;
    std::vector<stf_options> ov(opts, opts + nprob);
    for (auto& o : ov) {
        o.tol = 0.0;
        o.max_iter = iters;
        o.orth_final = 0;
        o.check_every = iters;
        o.history = nullptr;
    }
    std::vector<stf_result> r((size_t)nprob);
    const bool mixed = opts[0].precision == STF_PREC_MIXED;
    const int gram_c[] = {2048, 4096, 8192};
    const int res_c[] = {mixed ? 512 : 2048, mixed ? 1024 : 4096, mixed ? 2048 : 8192};
    double best = INFINITY;
    for (int bg : gram_c)
        for (int br : res_c) {
            double ms = 0.0;
            // every candidate starts from the iterate the previous one left: same work per iteration
            const int rc = batched_impl(nprob, probs, X, ov.data(), ws, ws_bytes, r.data(),
                                        stream, bg, br, &ms);
            if (rc < 0) return rc;
            if (ms > 0.0 && ms < best) {
                best = ms;
                *best_gram = bg;
                *best_res = br;
            }
        }
    if (best_ms_per_iter) *best_ms_per_iter = best;
    return STF_OK;
}

int pcal_solve_batched(int32_t nprob, const stf_problem* probs, void* const* X,
                       const stf_options* opts, void* ws, size_t ws_bytes, stf_result* res,
                       hipStream_t stream) {
    if (!opts || nprob <= 0) return STF_E_INVALID;
    std::vector<stf_options> ov(opts, opts + nprob);
    for (auto& o : ov) o.variant = STF_PCAL;
    return batched_impl(nprob, probs, X, ov.data(), ws, ws_bytes, res, stream, 0, 0, nullptr);
}

}  // extern "C"
