// Adjoint of the PCAL solution with respect to the diagonal potential V.
//
// X* is a stationary point (grad f(X) = X Lam, X^T X = I, eq. (kkt)) of
// f(X) = 1/2 tr(X^T (L + Diag V) X) + alpha/4 rho^T L^{-1} rho.  f and the
// losses it is used with are invariant under X -> X Q (Q orthogonal), so the
// implicit derivative lives in the horizontal space {xi : X^T xi = 0}.  With
// P = I - X X^T and the second-order form of (son),
//     Hess[xi] = P(grad^2 f(X)[xi] - xi Lam),
//     grad^2 f(X)[xi] = (L + Diag V + alpha Diag phi) xi + alpha Diag(L^{-1} drho) X,
//     drho = 2 rowdot(X, xi),  phi = L^{-1} rho(X),
// the adjoint zeta solves Hess[zeta] = P(g) for the loss gradient g = dl/dX*,
// and dl/dV_j = -rowdot(zeta, X)_j  (d grad f / dV along dV is Diag(dV) X).
// Hess is symmetric on the horizontal space; conjugate gradients runs on it in
// float64, every vector operation and both step scalars on the device, with one
// 16-byte read-back per step (<d, Hd> for the positivity check and the new
// <r, r> for the stop test).
#include <math.h>
#include <string.h>

#include <algorithm>

#include "stf_internal.h"

namespace stf {

__device__ __forceinline__ double wave_sum_a(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// out_r = scale * sum_c X_rc Z_rc; one wave per row.
__global__ __launch_bounds__(256) void k_rowdot(const double* __restrict__ X,
                                                const double* __restrict__ Z, int64_t n, int p,
                                                double scale, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n;
         r += (int64_t)gridDim.x * 4) {
        const double* xr = X + (size_t)r * p;
        const double* zr = Z + (size_t)r * p;
        double s = 0.0;
        for (int c = lane; c < p; c += 64) s += xr[c] * zr[c];
        s = wave_sum_a(s);
        if (lane == 0) out[r] = scale * s;
    }
}

// T_rc += alpha * dphi_r * X_rc
__global__ __launch_bounds__(256) void k_add_diag_x(double* __restrict__ T,
                                                    const double* __restrict__ X,
                                                    const double* __restrict__ dphi, int64_t n,
                                                    int p, double alpha) {
    const size_t np = (size_t)n * p;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < np;
         e += (size_t)gridDim.x * blockDim.x)
        T[e] += alpha * dphi[e / p] * X[e];
}

// partial sums of <a, b> and <c, d> (second pair optional) per workgroup
__global__ __launch_bounds__(256) void k_dot2(const double* __restrict__ a,
                                              const double* __restrict__ b,
                                              const double* __restrict__ c,
                                              const double* __restrict__ d, size_t m,
                                              double* __restrict__ part) {
    __shared__ double sh[2][4];
    double s0 = 0.0, s1 = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (size_t)gridDim.x * blockDim.x) {
        s0 += a[e] * b[e];
        if (c) s1 += c[e] * d[e];
    }
    s0 = wave_sum_a(s0);
    s1 = wave_sum_a(s1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wave] = s0;
        sh[1][wave] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x * 2] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        part[blockIdx.x * 2 + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

__global__ __launch_bounds__(256) void k_dot_finish(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out, int nout) {
    __shared__ double sh[2][256];
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        s0 += part[2 * i];
        s1 += part[2 * i + 1];
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0][0];
        if (nout > 1) out[1] = sh[1][0];
    }
}

// CG scalars on the device: sc[0] = <r, r>, sc[1] = <d, Hd>, sc[2] = the new <r, r>.
// z += a d;  r -= a Hd  with a = sc[0] / sc[1]
__global__ __launch_bounds__(256) void k_cg_step(double* __restrict__ z, double* __restrict__ r,
                                                 const double* __restrict__ d,
                                                 const double* __restrict__ Hd,
                                                 const double* __restrict__ sc, size_t m) {
    const double a = sc[0] / sc[1];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (size_t)gridDim.x * blockDim.x) {
        z[e] += a * d[e];
        r[e] -= a * Hd[e];
    }
}

// d = r + b d  with b = sc[2] / sc[0]
__global__ __launch_bounds__(256) void k_cg_dir(double* __restrict__ d,
                                                const double* __restrict__ r,
                                                const double* __restrict__ sc, size_t m) {
    const double b = sc[2] / sc[0];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (size_t)gridDim.x * blockDim.x)
        d[e] = r[e] + b * d[e];
}

// sc[0] = sc[2] (after every thread of k_cg_dir has read both)
__global__ void k_cg_shift(double* __restrict__ sc) { sc[0] = sc[2]; }

struct AdjLayout {
    size_t z, r, d, hd, t;             // n x p float64
    size_t rho, phi, drho, dphi, hscr;  // n float64
    size_t wt;                         // p x p float64
    size_t gram_part, dst, dots, dot2;
    size_t total;
    GramPlan gram;
    ResPlan res;
};

static AdjLayout make_adj_layout(const stf_problem* prob) {
    AdjLayout L;
    memset(&L, 0, sizeof(L));
    const int64_t n = prob->n;
    const int p = prob->p;
    const size_t np = (size_t)n * p;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    L.z = take(np * 8);
    L.r = take(np * 8);
    L.d = take(np * 8);
    L.hd = take(np * 8);
    L.t = take(np * 8);
    L.rho = take((size_t)n * 8);
    L.phi = take((size_t)n * 8);
    L.drho = take((size_t)n * 8);
    L.dphi = take((size_t)n * 8);
    L.hscr = take((size_t)n * 8);
    L.wt = take((size_t)p * p * 8);
    L.gram = make_gram_plan(n, p);
    L.gram_part = take((size_t)L.gram.nchunks * L.gram.n_tiles * L.gram.bt * L.gram.bt * 8);
    L.res = make_res_plan(n, p, 128);
    if (prob->kind == STF_KIND_STENCIL3D) {
        const size_t nx = prob->grid[0], ny = prob->grid[1], nz = prob->grid[2];
        L.dst = take((nx * nx + ny * ny + nz * nz + nx + ny + nz) * 8);
    } else {
        L.dst = take(8);
    }
    L.dots = take(1024 * 2 * 8);
    L.dot2 = take(4 * 8);
    L.total = off;
    return L;
}

static unsigned grid_elems(size_t m) {
    size_t g = (m + 255) / 256;
    if (g > 8192) g = 8192;
    return (unsigned)std::max<size_t>(g, 1);
}

static unsigned grid_rows_a(int64_t n) {
    int64_t g = (n + 3) / 4;
    if (g > 65536) g = 65536;
    return (unsigned)std::max<int64_t>(g, 1);
}

struct AdjCtx {
    const stf_problem* prob;
    char* base;
    AdjLayout L;
    const double* X;
    const double* Lam;
    template <typename T> T* at(size_t o) const { return (T*)(base + o); }
};

// out = P(in) = in - X (X^T in), in place on `in` (float64 n x p)
static void project_inplace(const AdjCtx& c, double* v, hipStream_t s) {
    const int64_t n = c.prob->n;
    const int p = c.prob->p;
    launch_gram(STF_F64, STF_PREC_FP64, c.L.gram, c.X, v, n, p, c.at<double>(c.L.gram_part),
                nullptr, c.at<double>(c.L.wt), nullptr, s);
    launch_apply(STF_F64, c.L.res, c.X, v, c.at<double>(c.L.wt), n, p, s, 1);
}

// Hd = P(grad^2 f(X)[d] - d Lam)
static void hess_apply(const AdjCtx& c, const double* d, double* Hd, hipStream_t s) {
    const stf_problem* prob = c.prob;
    const int64_t n = prob->n;
    const int p = prob->p;
    // H0 d + alpha Diag(phi) d (the operator's block structure, no other terms)
    GradExtra ex;
    memset(&ex, 0, sizeof(ex));
    ex.block = grad_extra(prob, nullptr).block;
    launch_grad(prob, STF_F64, d, Hd, c.at<double>(c.L.phi), ex, nullptr, s);
    if (prob->kind != STF_KIND_DENSE && prob->alpha != 0.0) {
        k_rowdot<<<grid_rows_a(n), 256, 0, s>>>(c.X, d, n, p, 2.0, c.at<double>(c.L.drho));
        launch_hartree(prob, c.at<double>(c.L.drho), c.at<double>(c.L.dphi),
                       c.at<double>(c.L.hscr), c.at<double>(c.L.dst), nullptr, s);
        k_add_diag_x<<<grid_elems((size_t)n * p), 256, 0, s>>>(Hd, c.X, c.at<double>(c.L.dphi), n,
                                                             p, prob->alpha);
    }
    launch_apply(STF_F64, c.L.res, d, Hd, c.Lam, n, p, s, 1);
    project_inplace(c, Hd, s);
}

// <a, b> into the device scalar *out (no read-back)
static void dot_dev(const AdjCtx& c, const double* a, const double* b, double* out,
                    hipStream_t s) {
    const size_t m = (size_t)c.prob->n * c.prob->p;
    const int nb = 1024;
    k_dot2<<<nb, 256, 0, s>>>(a, b, nullptr, nullptr, m, c.at<double>(c.L.dots));
    k_dot_finish<<<1, 256, 0, s>>>(c.at<double>(c.L.dots), nb, out, 1);
}

// read `cnt` device scalars back to the host (the one synchronization of a CG step)
static int read_scalars(const double* dev, double* host, int cnt, hipStream_t s) {
    if (hipMemcpyAsync(host, dev, (size_t)cnt * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
        return STF_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return STF_E_HIP;
    return hipGetLastError() == hipSuccess ? STF_OK : STF_E_HIP;
}

static int adjoint_impl(const stf_problem* prob, const double* X, const double* Lam,
                        const double* gradX, double* gradV, double cg_tol, int32_t cg_maxit,
                        void* ws, size_t ws_bytes, int32_t* cg_iters, double* cg_relres,
                        hipStream_t s) {
    if (!prob || !X || !Lam || !gradX || !gradV || !ws) return STF_E_INVALID;
    if (prob->p <= 0 || prob->p > 1024 || prob->n < 2 * (int64_t)prob->p) return STF_E_INVALID;
    if (prob->kind == STF_KIND_DENSE && prob->A_dtype != STF_F64) return STF_E_UNSUPPORTED;
    if (check_problem(prob) != STF_OK) return STF_E_INVALID;
    // the Hessian products cover Problem 1 / 3 objectives (no linear, exchange or
    // right-factor terms)
    if (prob->Glin || prob->B || prob->gamma != 0.0) return STF_E_UNSUPPORTED;
    if (!(cg_tol > 0.0) || cg_maxit < 1) return STF_E_INVALID;
    AdjCtx c;
    c.prob = prob;
    c.base = (char*)ws;
    c.L = make_adj_layout(prob);
    c.X = X;
    c.Lam = Lam;
    if (ws_bytes < c.L.total) return STF_E_WORKSPACE;
    const int64_t n = prob->n;
    const int p = prob->p;
    const size_t m = (size_t)n * p;
    double* z = c.at<double>(c.L.z);
    double* r = c.at<double>(c.L.r);
    double* d = c.at<double>(c.L.d);
    double* hd = c.at<double>(c.L.hd);
    // phi = L^{-1} rho(X*) for the Hessian
    if (prob->kind == STF_KIND_STENCIL3D) launch_dst_init(prob, c.at<double>(c.L.dst), s);
    if (prob->kind != STF_KIND_DENSE && prob->alpha != 0.0) {
        launch_rowsq(STF_F64, X, n, p, c.at<double>(c.L.rho), nullptr, s);
        launch_hartree(prob, c.at<double>(c.L.rho), c.at<double>(c.L.phi), c.at<double>(c.L.hscr),
                       c.at<double>(c.L.dst), nullptr, s);
    }
    // b = P(g); z = 0; r = b; d = r
    if (hipMemcpyAsync(r, gradX, m * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) return STF_E_HIP;
    project_inplace(c, r, s);
    if (hipMemcpyAsync(d, r, m * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) return STF_E_HIP;
    if (hipMemsetAsync(z, 0, m * 8, s) != hipSuccess) return STF_E_HIP;
    double* sc = c.at<double>(c.L.dot2);
    double dd[2];
    dot_dev(c, r, r, sc, s);
    int rc = read_scalars(sc, dd, 1, s);
    if (rc) return rc;
    const double b2 = dd[0];
    double rr = b2;
    int it = 0;
    if (b2 > 0.0) {
        for (it = 1; it <= cg_maxit; ++it) {
            hess_apply(c, d, hd, s);
            dot_dev(c, d, hd, sc + 1, s);
            k_cg_step<<<grid_elems(m), 256, 0, s>>>(z, r, d, hd, sc, m);
            dot_dev(c, r, r, sc + 2, s);
            if ((rc = read_scalars(sc + 1, dd, 2, s))) return rc;
            const double dHd = dd[0], rr_new = dd[1];
            if (!(dHd > 0.0) || !isfinite(dHd)) return STF_E_DIVERGED;  // not positive definite
            if (rr_new <= cg_tol * cg_tol * b2) {
                rr = rr_new;
                break;
            }
            k_cg_dir<<<grid_elems(m), 256, 0, s>>>(d, r, sc, m);
            k_cg_shift<<<1, 1, 0, s>>>(sc);
            rr = rr_new;
        }
    }
    // dl/dV = -rowdot(zeta, X)
    k_rowdot<<<grid_rows_a(n), 256, 0, s>>>(X, z, n, p, -1.0, gradV);
    if (hipStreamSynchronize(s) != hipSuccess) return STF_E_HIP;
    if (hipGetLastError() != hipSuccess) return STF_E_HIP;
    if (cg_iters) *cg_iters = std::min(it, cg_maxit);
    if (cg_relres) *cg_relres = b2 > 0.0 ? sqrt(rr / b2) : 0.0;
    return (it > cg_maxit) ? STF_MAX_ITER : STF_OK;
}

}  // namespace stf

extern "C" {

size_t stf_adjoint_workspace_size(const stf_problem* prob) {
    if (!prob || prob->p <= 0 || prob->n < 2 * (int64_t)prob->p) return 0;
    return stf::make_adj_layout(prob).total;
}

int pcal_adjoint_v(const stf_problem* prob, const double* Xstar, const double* Lam,
                   const double* gradX, double* gradV, double cg_tol, int32_t cg_maxit,
                   void* ws, size_t ws_bytes, int32_t* cg_iters, double* cg_relres,
                   hipStream_t stream) {
    return stf::adjoint_impl(prob, Xstar, Lam, gradX, gradV, cg_tol, cg_maxit, ws, ws_bytes,
                             cg_iters, cg_relres, stream);
}

}  // extern "C"
