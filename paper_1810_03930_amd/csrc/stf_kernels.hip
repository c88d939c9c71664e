// gfx950 kernels of the PLAM / PCAL iteration.
//
// One iteration k (Algorithms 2 and 3 of the paper) is the kernel sequence
//   hartree  : phi = L^{-1} rho                       (stencil kinds with alpha != 0)
//   grad     : G = (L + Diag v + alpha Diag phi) X   or   G = A X (dense)
//   gram     : split-K partials of S = X^T X (upper blocks) and W = X^T G
//   gram_red : deterministic sum of the partials
//   stage1   : Psi = (W + W^T)/2, C = S - I, d (PCAL Phi term), M_L = Psi - beta C + Diag d
//   residual : gradL = G - X M_L (written over G), optional KKT product G - X Psi,
//              Barzilai-Borwein inner products, column dots for the PCAL norms
//   colred   : deterministic sum of the column partials
//   stage2   : KKT stop test, eta^k, column norms nu
//   update   : X <- (X - gradL / eta) / nu, rho <- diag(X X^T)
// All kernels read the device iteration state and return immediately once it
// says "done", so a captured chunk of iterations can run past convergence
// without touching the returned iterate.
//
// MFMA operand layout used throughout (v_mfma_f64_16x16x4f64 and
// v_mfma_f32_16x16x4f32, one block): lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Element v of the 16x16 result sits in column l%16 and row
// Mma<T>::row(l/16, v): 4*(l/16)+v for float32, (l/16)+4*v for float64.
#include "stf_internal.h"

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace stf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<double> {
    typedef d4 acc;
    static __device__ __forceinline__ d4 run(double a, double b, d4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mma<float> {
    typedef f4 acc;
    static __device__ __forceinline__ f4 run(float a, float b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

// ---- split-bf16 helpers (MIXED precision) ---------------------------------
// v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8*(l/16)+e] and
// B[8*(l/16)+e][l%16] for e = 0..7; the float32 result has the float32 layout
// above.  A float32 x splits exactly as x = h + m + l with h = bf16(x),
// m = bf16(x - h), l = bf16(x - h - m) (each difference is exact in float32 and
// the last one has at most 8 significant bits).
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mma_bf(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void split2(const float (&x)[8], bf8& h, bf8& l) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 hb = (__bf16)x[e];
        h[e] = hb;
        l[e] = (__bf16)(x[e] - (float)hb);
    }
}

__device__ __forceinline__ void split3(const float (&x)[8], bf8& h, bf8& m, bf8& l) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 hb = (__bf16)x[e];
        const float r = x[e] - (float)hb;
        const __bf16 mb = (__bf16)r;
        h[e] = hb;
        m[e] = mb;
        l[e] = (__bf16)(r - (float)mb);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 256 threads of a workgroup; the result is valid in thread 0.
// `sh` must hold at least 4 doubles.
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

// Sum over the NW waves of a workgroup; the result is valid in thread 0.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
#pragma unroll
        for (int w = 0; w < NW; ++w) r += sh[w];
    return r;
}

// Map a hardware workgroup id to a logical id so that consecutive logical ids
// run on the same XCD (workgroups are dealt to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_remap(int b, int nwg) {
    const int q = nwg / 8, r = nwg % 8;
    const int x = b % 8, pos = b / 8;
    const int start = (x < r) ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return start + pos;
}

// Raw buffer resource over [base, base + bytes) (bytes < 2^31): a load whose
// byte offset is at or past `bytes` returns zero (the hardware range check), so
// edge tiles need no branches.  The whole offset goes in the VGPR operand,
// which the range check covers; kBufOob is an offset past every range.
constexpr uint32_t kBufOob = 0x80000000u;
typedef uint32_t u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ float buf_ldf(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <typename T>
__device__ __forceinline__ T buf_ld1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
// 16 bytes (offset a multiple of 16) as a vector of T
template <typename T>
__device__ __forceinline__ T __attribute__((ext_vector_type(16 / sizeof(T))))
buf_ld16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef T tv __attribute__((ext_vector_type(16 / sizeof(T))));
    return __builtin_bit_cast(tv, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// ---------------------------------------------------------------- state ----
// Clear the stop flag after a precision hand-over (iteration k is redone).
__global__ void k_resume_state(DevState* st) {
    if (threadIdx.x == 0) {
        st->done = 0;
        st->status = 0;
    }
}

__global__ void k_init_state(DevState* st) {
    if (threadIdx.x == 0) {
        DevState z;
        memset(&z, 0, sizeof(z));
        *st = z;
    }
}

// -------------------------------------------------------------- density ----
// rho_r = sum_c X_rc^2 (float64 accumulation); one wave per row.
template <typename T>
__device__ __forceinline__ void body_rowsq(const T* __restrict__ X, int64_t n, int p,
                                               double* __restrict__ rho,
                                               const DevState* __restrict__ st, int bid_, int nblk_) {
    if (st && st->done) return;
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)bid_ * 4 + (threadIdx.x >> 6); r < n;
         r += (int64_t)nblk_ * 4) {
        const T* xr = X + (size_t)r * p;
        double s = 0.0;
        for (int c = lane; c < p; c += 64) {
            double x = (double)xr[c];
            s += x * x;
        }
        s = wave_sum(s);
        if (lane == 0) rho[r] = s;
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_rowsq(const T* __restrict__ X, int64_t n, int p,
                                               double* __restrict__ rho,
                                               const DevState* __restrict__ st) {
    body_rowsq<T>(X, n, p, rho, st, blockIdx.x, gridDim.x);
}


// ------------------------------------------------------------- Hartree ----
// 1D: phi = T^{-1} rho with T = tridiag(-1,2,-1) of order n, through the
// closed-form Green's function (T^{-1})_ij = min(i,j)(n+1-max(i,j))/(n+1)
// (1-based), i.e. phi_i = ((n+1-i) A_i + i B_i) / (n+1) with the prefix sum
// A_i = sum_{j<=i} j rho_j and the suffix sum B_i = sum_{j>i} (n+1-j) rho_j.
// One workgroup of 1024 threads; each thread owns a contiguous chunk.
__device__ __forceinline__ void body_hartree1d(const double* __restrict__ rho,
                                                    double* __restrict__ phi, int64_t n,
                                                    const DevState* __restrict__ st, int bid_, int nblk_) {
    if (st && st->done) return;
    __shared__ double sa[1024], sb[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    const int64_t chunk = (n + nt - 1) / nt;
    const int64_t i0 = (int64_t)t * chunk, i1 = min(n, i0 + chunk);
    const double np1 = (double)(n + 1);
    double a = 0.0, b = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const double j = (double)(i + 1);
        a += j * rho[i];
        b += (np1 - j) * rho[i];
    }
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    // inclusive scans: sa forward (prefix), sb backward (suffix)
    for (int off = 1; off < nt; off <<= 1) {
        double va = (t >= off) ? sa[t - off] : 0.0;
        double vb = (t + off < nt) ? sb[t + off] : 0.0;
        __syncthreads();
        sa[t] += va;
        sb[t] += vb;
        __syncthreads();
    }
    const double a_excl = (t > 0) ? sa[t - 1] : 0.0;        // sum over chunks before t
    const double b_excl = (t + 1 < nt) ? sb[t + 1] : 0.0;   // sum over chunks after t
    double A = a_excl;
    for (int64_t i = i0; i < i1; ++i) {
        const double j = (double)(i + 1);
        A += j * rho[i];
        phi[i] = (np1 - j) * A;
    }
    double B = b_excl;  // sum_{j > i}
    for (int64_t i = i1 - 1; i >= i0; --i) {
        const double j = (double)(i + 1);
        phi[i] = (phi[i] + j * B) / np1;
        B += (np1 - j) * rho[i];
    }
}
__global__ __launch_bounds__(1024) void k_hartree1d(const double* __restrict__ rho,
                                                    double* __restrict__ phi, int64_t n,
                                                    const DevState* __restrict__ st) {
    body_hartree1d(rho, phi, n, st, blockIdx.x, gridDim.x);
}
// Block-diagonal L = Diag(L_1, ..., L_s) (blocks of order `block`, the last one
// shorter): L^{-1} is block-diagonal and each block is the Green's function
// above of the block's order.  Long blocks: one workgroup per block (the scan
// above on the block's range); short blocks: one thread per block, the two
// sums of the Green's function formula taken serially.
__global__ __launch_bounds__(1024) void k_hartree1d_wg(const double* __restrict__ rho,
                                                       double* __restrict__ phi, int64_t n,
                                                       int64_t block,
                                                       const DevState* __restrict__ st) {
    const int64_t b0 = (int64_t)blockIdx.x * block;
    if (b0 >= n) return;
    const int64_t m = min(block, n - b0);
    body_hartree1d(rho + b0, phi + b0, m, st, 0, 1);
}
__global__ __launch_bounds__(256) void k_hartree1d_short(const double* __restrict__ rho,
                                                         double* __restrict__ phi, int64_t n,
                                                         int block,
                                                         const DevState* __restrict__ st) {
    if (st && st->done) return;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b0 = b * block;
    if (b0 >= n) return;
    const int m = (int)min((int64_t)block, n - b0);
    const double mp1 = (double)(m + 1);
    // phi_i = ((m+1-i) sum_{j<=i} j rho_j + i sum_{j>i} (m+1-j) rho_j) / (m+1), 1-based
    double A = 0.0;
    for (int i = 0; i < m; ++i) {
        const double j = (double)(i + 1);
        A += j * rho[b0 + i];
        phi[b0 + i] = (mp1 - j) * A;
    }
    double B = 0.0;
    for (int i = m - 1; i >= 0; --i) {
        const double j = (double)(i + 1);
        phi[b0 + i] = (phi[b0 + i] + j * B) / mp1;
        B += (mp1 - j) * rho[b0 + i];
    }
}


// 3D: the orthonormal DST-I matrix S_m[k][j] = sqrt(2/(m+1)) sin(pi (k+1)(j+1)/(m+1))
// diagonalizes tridiag(-1,2,-1) of order m with eigenvalues 4 sin^2(pi (k+1) / (2(m+1))).
__global__ void k_dst_init(double* __restrict__ S, double* __restrict__ lam, int m) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const double sc = sqrt(2.0 / (double)(m + 1));
    if (e < m * m) {
        const int k = e / m, j = e % m;
        const long q = ((long)(k + 1) * (long)(j + 1)) % (2L * (m + 1));
        S[e] = sc * sin(M_PI * (double)q / (double)(m + 1));
    }
    if (e < m) {
        const double s = sin(M_PI * (double)(e + 1) / (2.0 * (m + 1)));
        lam[e] = 4.0 * s * s;
    }
}

// out = (S_m applied along one axis) in; if lam3 is set, out is then divided
// elementwise by lam_x + lam_y + lam_z.
__global__ __launch_bounds__(256) void k_dst_axis(const double* __restrict__ in,
                                                  double* __restrict__ out,
                                                  const double* __restrict__ S, int m,
                                                  int64_t stride, int64_t n,
                                                  const double* __restrict__ lx,
                                                  const double* __restrict__ ly,
                                                  const double* __restrict__ lz, int nx,
                                                  int ny, const DevState* __restrict__ st) {
    if (st && st->done) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t k = (e / stride) % m;
    const int64_t base = e - k * stride;
    const double* srow = S + k * m;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += srow[j] * in[base + (int64_t)j * stride];
    if (lx) {
        const int64_t x = e % nx, y = (e / nx) % ny, z = e / ((int64_t)nx * ny);
        s /= (lx[x] + ly[y]) + lz[z];
    }
    out[e] = s;
}

// The same 3D solve in three passes with the planes staged in LDS (grids with
// nx, ny, nz <= 64).  k_dst_xy applies S_x along x and S_y along y to one
// z-plane per workgroup: out_plane = S_y in_plane S_x^T (S symmetric);
// k_dst_z applies, for one y and all x, S_z along z, the division by
// lx + ly + lz and S_z again (the forward and inverse z transforms fused).
// Each 64 x 64 product is sixteen 16 x 16 tiles of float64 MFMA, one per wave
// of the 1024-thread workgroup; the operands sit in LDS zero-padded to 64 x 64
// with a 65-double row pitch (the 16 rows an MFMA operand reads then fall in
// different banks).
constexpr int kDstMax = 64;
constexpr int kDP = kDstMax + 1;

// 16 x 16 tile (ti, tj) of L R over the padded 64-long inner dimension; the
// lane holds rows 16 ti + Mma<double>::row(lk, q), column 16 tj + lr.
__device__ __forceinline__ d4 dst_tile(const double* L, const double* R, int ti, int tj,
                                       int lr, int lk) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = 0; k < kDstMax; k += 4) {
        const double a = L[(16 * ti + lr) * kDP + k + lk];
        const double b = R[(k + lk) * kDP + 16 * tj + lr];
        acc = Mma<double>::run(a, b, acc);
    }
    return acc;
}

// m x m matrix (row-major, global) into a zero-padded 64 x kDP LDS array
__device__ __forceinline__ void dst_stage(double* D, const double* M, int rows, int cols,
                                          int ld) {
    for (int e = threadIdx.x; e < kDstMax * kDstMax; e += blockDim.x) {
        const int r = e / kDstMax, c = e % kDstMax;
        D[r * kDP + c] = (r < rows && c < cols) ? M[(size_t)r * ld + c] : 0.0;
    }
}

__global__ __launch_bounds__(1024) void k_dst_xy(const double* __restrict__ in,
                                                double* __restrict__ out,
                                                const double* __restrict__ Sx,
                                                const double* __restrict__ Sy, int nx, int ny,
                                                const DevState* __restrict__ st) {
    if (st && st->done) return;
    __shared__ double A[kDstMax * kDP], T[kDstMax * kDP];
    __shared__ double Mx[kDstMax * kDP], My[kDstMax * kDP];
    const int nxy = nx * ny;
    const double* src = in + (size_t)blockIdx.x * nxy;
    double* dst = out + (size_t)blockIdx.x * nxy;
    dst_stage(A, src, ny, nx, nx);
    dst_stage(Mx, Sx, nx, nx, nx);
    dst_stage(My, Sy, ny, ny, ny);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int ti = wave >> 2, tj = wave & 3;
    // T[y][k] = sum_x A[y][x] Sx[x][k]  (S symmetric)
    {
        const d4 t = dst_tile(A, Mx, ti, tj, lr, lk);
#pragma unroll
        for (int q = 0; q < 4; ++q) T[(16 * ti + Mma<double>::row(lk, q)) * kDP + 16 * tj + lr] = t[q];
    }
    __syncthreads();
    // out[k][x] = sum_y Sy[k][y] T[y][x]
    const d4 o = dst_tile(My, T, ti, tj, lr, lk);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = 16 * ti + Mma<double>::row(lk, q), x = 16 * tj + lr;
        if (k < ny && x < nx) dst[k * nx + x] = o[q];
    }
}
__global__ __launch_bounds__(1024) void k_dst_z(const double* in, double* out,
                                               const double* __restrict__ Sz,
                                               const double* __restrict__ lx,
                                               const double* __restrict__ ly,
                                               const double* __restrict__ lz, int nx, int ny,
                                               int nz, const DevState* __restrict__ st) {
    if (st && st->done) return;
    __shared__ double A[kDstMax * kDP], U[kDstMax * kDP], Mz[kDstMax * kDP];
    const int y = blockIdx.x;
    const size_t sxy = (size_t)nx * ny;
    for (int e = threadIdx.x; e < kDstMax * kDstMax; e += blockDim.x) {
        const int z = e / kDstMax, x = e % kDstMax;
        A[z * kDP + x] = (z < nz && x < nx) ? in[(size_t)z * sxy + (size_t)y * nx + x] : 0.0;
    }
    dst_stage(Mz, Sz, nz, nz, nz);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int ti = wave >> 2, tj = wave & 3;
    // U[k][x] = (sum_z Sz[k][z] A[z][x]) / (lx[x] + ly[y] + lz[k])
    {
        const d4 u = dst_tile(Mz, A, ti, tj, lr, lk);
        const int x = 16 * tj + lr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 16 * ti + Mma<double>::row(lk, q);
            U[k * kDP + x] = (k < nz && x < nx) ? u[q] / ((lx[x] + ly[y]) + lz[k]) : 0.0;
        }
    }
    __syncthreads();
    // out[z][x] = sum_k Sz[z][k] U[k][x]  (every read of this slab is done)
    const d4 o = dst_tile(Mz, U, ti, tj, lr, lk);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int z = 16 * ti + Mma<double>::row(lk, q), x = 16 * tj + lr;
        if (z < nz && x < nx) out[(size_t)z * sxy + (size_t)y * nx + x] = o[q];
    }
}

// ------------------------------------------------------------ gradient ----
// G = (L + Diag v + alpha Diag phi) X for the 1D (ND = 2 neighbours) and 3D
// (ND = 6) Dirichlet stencils, computed in the arithmetic of the input X and
// stored as TO.  One wave per grid point (row) at a time; lanes take 16-byte
// vectors of the row, and the loads of the row and of all its neighbours are
// issued before any use (a neighbour missing at the boundary reads the row
// itself with weight 0).  Workgroups keep the hardware round-robin over the
// XCDs, so the y- and z-neighbours of a row (nx and nx*ny rows away) are read
// by the same XCD a few hundred rows later and come from its L2.
template <typename T, typename TO, int ND>
__device__ __forceinline__ void body_grad_stencil(const T* __restrict__ X,
                                                      TO* __restrict__ G, int64_t n, int p,
                                                      int nx, int ny, int nz,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ phi,
                                                      double alpha, const GradExtra ex,
                                                      const DevState* __restrict__ st, int bid_, int nblk_) {
    if (st && st->done) return;
    constexpr int V = 16 / (int)sizeof(T);
    typedef T tv __attribute__((ext_vector_type(V)));
    const int lane = threadIdx.x & 63;
    const bool vec = (p % V) == 0;
    const int rpb = blockDim.x >> 6;  // rows per workgroup: one per wave
    for (int64_t r = (int64_t)bid_ * rpb + (threadIdx.x >> 6); r < n;
         r += (int64_t)nblk_ * rpb) {
        double dg = (ND == 6) ? 6.0 : 2.0;
        if (v) dg += v[r];
        if (phi) dg += alpha * phi[r];
        // exchange term of Problem 6: -2 gamma rho_r^{1/3} on the row diagonal
        if (ex.gamma != 0.0) dg -= 2.0 * ex.gamma * cbrt(ex.rho[r]);
        int64_t nb[ND];
        T w[ND];
        if (ND == 2) {
            // blocks of order ex.block: no coupling across a block boundary
            const bool lo = r > 0 && (ex.block <= 0 || r % ex.block != 0);
            const bool hi = r + 1 < n && (ex.block <= 0 || (r + 1) % ex.block != 0);
            nb[0] = lo ? r - 1 : r;
            w[0] = lo ? (T)1 : (T)0;
            nb[1] = hi ? r + 1 : r;
            w[1] = hi ? (T)1 : (T)0;
        } else {
            const int64_t sxy = (int64_t)nx * ny;
            const int64_t x = r % nx, y = (r / nx) % ny, z = r / sxy;
            const bool has[6] = {x > 0, x + 1 < nx, y > 0, y + 1 < ny, z > 0, z + 1 < nz};
            const int64_t d[6] = {-1, 1, -(int64_t)nx, (int64_t)nx, -sxy, sxy};
#pragma unroll
            for (int q = 0; q < ND; ++q) {
                nb[q] = has[q] ? r + d[q] : r;
                w[q] = has[q] ? (T)1 : (T)0;
            }
        }
        const T tdg = (T)dg;
        const T* xr = X + (size_t)r * p;
        TO* gr = G + (size_t)r * p;
        if (vec) {
            for (int c = lane * V; c < p; c += 64 * V) {
                tv xc = *(const tv*)(xr + c);
                tv xn[ND];
#pragma unroll
                for (int q = 0; q < ND; ++q) xn[q] = *(const tv*)(X + (size_t)nb[q] * p + c);
                tv acc = tdg * xc;
#pragma unroll
                for (int q = 0; q < ND; ++q) acc -= w[q] * xn[q];
                if (ex.glin) {
                    // linear term of Problem 2
                    const double* gl = ex.glin + (size_t)r * p + c;
#pragma unroll
                    for (int e = 0; e < V; ++e) acc[e] += (T)gl[e];
                }
                typedef TO ov __attribute__((ext_vector_type(V)));
                ov o;
#pragma unroll
                for (int e = 0; e < V; ++e) o[e] = (TO)acc[e];
                __builtin_nontemporal_store(o, (ov*)(gr + c));  // streamed: keep L2 for X
            }
        } else {
            for (int c = lane; c < p; c += 64) {
                T acc = tdg * xr[c];
#pragma unroll
                for (int q = 0; q < ND; ++q) acc -= w[q] * X[(size_t)nb[q] * p + c];
                if (ex.glin) acc += (T)ex.glin[(size_t)r * p + c];
                gr[c] = (TO)acc;
            }
        }
    }
}
template <typename T, typename TO, int ND>
__global__ __launch_bounds__(256) void k_grad_stencil(const T* __restrict__ X,
                                                      TO* __restrict__ G, int64_t n, int p,
                                                      int nx, int ny, int nz,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ phi,
                                                      double alpha, const GradExtra ex,
                                                      const DevState* __restrict__ st) {
    body_grad_stencil<T, TO, ND>(X, G, n, p, nx, ny, nz, v, phi, alpha, ex, st, blockIdx.x,
                                 gridDim.x);
}

// Line-walking form of the same gradient for rows whose length is a multiple
// of the 16-byte vector.  A wave owns R consecutive rows (a run along x) and
// slides over them with the rows r-1, r, r+1 held in registers, so each row
// costs one new x-row load plus its y- and z-neighbours (ND - 2 of them)
// instead of ND + 1 loads; the loads of row r+1 are issued before the
// arithmetic of row r.  The diagonal (ND + v + alpha phi) of the R rows is
// read once per run, one row per lane, and broadcast with readlane.
// The terms are added in the order of the one-wave-per-row form above.
// Workgroups deal the runs to the XCDs in contiguous slabs (xcd_remap), so a
// run's y-neighbours, one line away, are read by the same XCD at about the
// same time.
template <typename T, typename TO, int ND, int R>
__device__ __forceinline__ void body_grad_line(const T* __restrict__ X, TO* __restrict__ G,
                                               int64_t n, int p, int nx, int ny, int nz,
                                               const double* __restrict__ v,
                                               const double* __restrict__ phi, double alpha,
                                               const DevState* __restrict__ st, int bid_,
                                               int nblk_) {
    static_assert(R >= 2 && R <= 64, "a run is at most one row per lane");
    if (st && st->done) return;
    constexpr int V = 16 / (int)sizeof(T);
    constexpr int NB = ND - 2;  // neighbours off the x line
    typedef T tv __attribute__((ext_vector_type(V)));
    typedef TO ov __attribute__((ext_vector_type(V)));
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int64_t nseg = (n + R - 1) / R;
    const int64_t sxy = (int64_t)nx * ny;
    const int bid = xcd_remap(bid_, nblk_);
    for (int64_t sg = (int64_t)bid * wpb + (threadIdx.x >> 6); sg < nseg;
         sg += (int64_t)nblk_ * wpb) {
        const int64_t r0 = sg * R;
        const int rn = (int)((n - r0) < R ? (n - r0) : R);
        double dgl = (ND == 6) ? 6.0 : 2.0;
        if (lane < rn) {
            if (v) dgl += v[r0 + lane];
            if (phi) dgl += alpha * phi[r0 + lane];
        }
        // grid coordinates of the first row; later rows step x and carry
        int x0 = 0, y0 = 0, z0 = 0;
        if (ND == 6) {
            x0 = (int)(r0 % nx);
            y0 = (int)((r0 / nx) % ny);
            z0 = (int)(r0 / sxy);
        }
        for (int c = lane * V; c < p; c += 64 * V) {
            const T* xc = X + c;
            auto ld = [&](int64_t r) { return *(const tv*)(xc + (size_t)r * p); };
            // neighbours of row r off the x line (the row itself at the boundary)
            auto ldnb = [&](int64_t r, int x, int y, int z, tv (&o)[NB > 0 ? NB : 1]) {
                if (ND == 6) {
                    o[0] = ld(y > 0 ? r - nx : r);
                    o[1] = ld(y + 1 < ny ? r + nx : r);
                    o[2] = ld(z > 0 ? r - sxy : r);
                    o[3] = ld(z + 1 < nz ? r + sxy : r);
                }
            };
            tv xm = ld(r0 > 0 ? r0 - 1 : r0);
            tv xx = ld(r0);
            tv xp = ld(r0 + 1 < n ? r0 + 1 : r0);
            tv nb[NB > 0 ? NB : 1];
            ldnb(r0, x0, y0, z0, nb);
            int x = x0, y = y0, z = z0;
            for (int i = 0; i < rn; ++i) {
                const int64_t r = r0 + i;
                // coordinates of row r + 1 (clamped to the run) and its loads
                int x1 = x, y1 = y, z1 = z;
                if (ND == 6 && i + 1 < rn) {
                    if (++x1 == nx) {
                        x1 = 0;
                        if (++y1 == ny) {
                            y1 = 0;
                            ++z1;
                        }
                    }
                }
                const int64_t r1 = (i + 1 < rn) ? r + 1 : r;
                const tv xq = ld(r1 + 1 < n ? r1 + 1 : r1);
                tv nq[NB > 0 ? NB : 1];
                ldnb(r1, x1, y1, z1, nq);
                // row r
                // (lanes past the row's last vector are off in this loop, so
                // read the run's diagonal with readlane, which ignores them)
                const T tdg = (T)__hiloint2double(
                    __builtin_amdgcn_readlane(__double2hiint(dgl), i),
                    __builtin_amdgcn_readlane(__double2loint(dgl), i));
                T wxm, wxp;
                if (ND == 6) {
                    wxm = x > 0 ? (T)1 : (T)0;
                    wxp = x + 1 < nx ? (T)1 : (T)0;
                } else {
                    wxm = r > 0 ? (T)1 : (T)0;
                    wxp = r + 1 < n ? (T)1 : (T)0;
                }
                tv acc = tdg * xx;
                acc -= wxm * xm;
                acc -= wxp * xp;
                if (ND == 6) {
                    acc -= (y > 0 ? (T)1 : (T)0) * nb[0];
                    acc -= (y + 1 < ny ? (T)1 : (T)0) * nb[1];
                    acc -= (z > 0 ? (T)1 : (T)0) * nb[2];
                    acc -= (z + 1 < nz ? (T)1 : (T)0) * nb[3];
                }
                ov o;
#pragma unroll
                for (int e = 0; e < V; ++e) o[e] = (TO)acc[e];
                __builtin_nontemporal_store(o, (ov*)(G + (size_t)r * p + c));
                xm = xx;
                xx = xp;
                xp = xq;
#pragma unroll
                for (int q = 0; q < NB; ++q) nb[q] = nq[q];
                x = x1;
                y = y1;
                z = z1;
            }
        }
    }
}
template <typename T, typename TO, int ND, int R>
__global__ __launch_bounds__(256) void k_grad_line(const T* __restrict__ X, TO* __restrict__ G,
                                                   int64_t n, int p, int nx, int ny, int nz,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ phi, double alpha,
                                                   const DevState* __restrict__ st) {
    body_grad_line<T, TO, ND, R>(X, G, n, p, nx, ny, nz, v, phi, alpha, st, blockIdx.x,
                                 gridDim.x);
}


// ------------------------------------------------- transposed products ----
// acc[i][j] += sum_{k0 <= k < k1} Z[k][zc0 + 16 i + (row in tile)] * Y[k][yc0 + 16 j + ...]
// i.e. one wave accumulates a (16 WM) x (16 WM) block of Z^T Y.  Fragments are
// read straight from global memory: for a fixed k the 16 lanes of a quarter
// wave read 16 consecutive elements of one row, so every load is coalesced
// for row-major Z and Y.
template <typename T, int WM, typename TZ = T>
__device__ __forceinline__ void tn_mac(const TZ* __restrict__ Z, int64_t ldz, int zc0, int zlim,
                                       const T* __restrict__ Y, int64_t ldy, int yc0, int ylim,
                                       int64_t k0, int64_t k1,
                                       typename Mma<T>::acc (&acc)[WM][WM]) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    bool zok[WM], yok[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        zok[i] = (zc0 + i * 16 + lr) < zlim;
        yok[i] = (yc0 + i * 16 + lr) < ylim;
    }
    const TZ* zp = Z + zc0 + lr;
    const T* yp = Y + yc0 + lr;
    constexpr int U = 4;
    int64_t k = k0;
    for (; k + 4 * U <= k1; k += 4 * U) {
        T a[U][WM], b[U][WM];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = k + u * 4 + lk;
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                a[u][i] = zok[i] ? (T)zp[row * ldz + i * 16] : (T)0;
                b[u][i] = yok[i] ? yp[row * ldy + i * 16] : (T)0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WM; ++j) acc[i][j] = Mma<T>::run(a[u][i], b[u][j], acc[i][j]);
    }
    for (; k < k1; k += 4) {
        const int64_t row = k + lk;
        const bool rok = row < k1;
        T a[WM], b[WM];
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            a[i] = (rok && zok[i]) ? (T)zp[row * ldz + i * 16] : (T)0;
            b[i] = (rok && yok[i]) ? yp[row * ldy + i * 16] : (T)0;
        }
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WM; ++j) acc[i][j] = Mma<T>::run(a[i], b[j], acc[i][j]);
    }
}

// Decode tile index t of the Gram pass into (bi, bj, is_S): the upper blocks
// of S first, then the blocks of W (only the upper ones when wup: W is
// symmetric in exact arithmetic for every f here, grad f(X) = H(X) X with H
// symmetric, so its lower blocks are mirrored from the upper ones).
__device__ __forceinline__ void upper_block(int u, int nb, int& bi, int& bj) {
    int row = 0;
    while (u >= nb - row) {
        u -= nb - row;
        ++row;
    }
    bi = row;
    bj = row + u;
}
__device__ __forceinline__ void gram_tile(int t, int nb, int n_s_tiles, int wup, int& bi,
                                          int& bj, bool& isS) {
    isS = t < n_s_tiles;
    if (isS) {
        upper_block(t, nb, bi, bj);
    } else if (wup) {
        upper_block(t - n_s_tiles, nb, bi, bj);
    } else {
        const int u = t - n_s_tiles;
        bi = u / nb;
        bj = u % nb;
    }
}

// Split-K Gram pass: part[chunk][tile][bt][bt] (float64) holds the chunk's
// contribution to the tile of S (upper blocks, Y = X) or W (Y = G).
template <typename T, int WM>
__device__ __forceinline__ void body_gram(const T* __restrict__ X, const T* __restrict__ G,
                                              int64_t n, int p, int nb, int n_s_tiles,
                                              int n_tiles, int wup, int64_t chunk,
                                              double* __restrict__ part,
                                              const DevState* __restrict__ st, int bid_, int nblk_) {
    if (st && st->done) return;
    constexpr int WT = 16 * WM, BT = 2 * WT;
    const int nwg = nblk_;
    const int lid = xcd_remap(bid_, nwg);
    // consecutive logical ids share a chunk (same rows: L2 reuse inside one XCD)
    const int tile = lid % n_tiles, c = lid / n_tiles;
    int bi, bj;
    bool isS;
    gram_tile(tile, nb, n_s_tiles, wup, bi, bj, isS);
    const T* Y = isS ? X : G;
    const int wave = threadIdx.x >> 6, wi = wave >> 1, wj = wave & 1;
    // below the diagonal of a diagonal block of a symmetric result: nothing to do
    if ((bi == bj) && (isS || wup) && (wi > wj)) return;
    const int zc0 = bi * BT + wi * WT, yc0 = bj * BT + wj * WT;
    const int64_t k0 = (int64_t)c * chunk, k1 = min(n, k0 + chunk);
    typename Mma<T>::acc acc[WM][WM];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][j][q] = 0;
    if (zc0 < p && yc0 < p && k0 < k1) tn_mac<T, WM>(X, p, zc0, p, Y, p, yc0, p, k0, k1, acc);
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    double* out = part + ((size_t)c * n_tiles + tile) * (size_t)(BT * BT);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ii = wi * WT + i * 16 + Mma<T>::row(lk, q);
                const int jj = wj * WT + j * 16 + lr;
                out[ii * BT + jj] = (double)acc[i][j][q];
            }
}
template <typename T, int WM>
__global__ __launch_bounds__(256) void k_gram(const T* __restrict__ X, const T* __restrict__ G,
                                              int64_t n, int p, int nb, int n_s_tiles,
                                              int n_tiles, int wup, int64_t chunk,
                                              double* __restrict__ part,
                                              const DevState* __restrict__ st) {
    body_gram<T, WM>(X, G, n, p, nb, n_s_tiles, n_tiles, wup, chunk, part, st, blockIdx.x, gridDim.x);
}


// LDS-staged split-K Gram pass for 128 x 128 tiles (p > 64): the workgroup
// walks its chunk of rows KC at a time, staging the tile's 128 columns of Z
// (= X) and of Y (= X or G) for those rows in LDS, prefetched one step ahead
// into registers; four waves of 64 x 64.  float32 tiles are added into float64
// every 256 rows.  Partials as in k_gram.
template <typename T>
__device__ __forceinline__ void body_gram_lds(const T* __restrict__ X,
                                                  const T* __restrict__ G, int64_t n, int p,
                                                  int nb, int n_s_tiles, int n_tiles, int wup,
                                                  int64_t chunk, double* __restrict__ part,
                                                  const DevState* __restrict__ st, int bid_, int nblk_,
                                                  double* __restrict__ colsq = nullptr) {
    if (st && st->done) return;
    constexpr int KC = (sizeof(T) == 8) ? 16 : 32;
    constexpr int LS = 128 + 4;
    constexpr int VX = 16 / (int)sizeof(T);
    constexpr int NV = KC * 128 / VX / 256;
    constexpr int FLUSH = 256 / KC;
    // float64: the chunk's 16 rows of the Z and Y panels go straight from
    // global memory into two LDS buffers (buffer_load ... lds; one 1 KiB wave
    // load per panel row, a lane's 16 bytes at its lane's place), the next
    // chunk in flight while this one is used, one barrier per chunk.  Row k
    // holds its column pair c at slot c ^ ((k & 1) << 3), so the four rows of
    // an MFMA operand read spread over both halves of the banks.
    constexpr bool DL = sizeof(T) == 8;
    __shared__ T Zs[DL ? 1 : KC * LS];
    __shared__ T Ys[DL ? 1 : KC * LS];
    __shared__ __attribute__((aligned(16))) double ZsD[DL ? 2 * 16 * 128 : 2];
    __shared__ __attribute__((aligned(16))) double YsD[DL ? 2 * 16 * 128 : 2];
    const int nwg = nblk_;
    const int lid = xcd_remap(bid_, nwg);
    const int tile = lid % n_tiles, c = lid / n_tiles;
    int bi, bj;
    bool isS;
    gram_tile(tile, nb, n_s_tiles, wup, bi, bj, isS);
    const T* Y = isS ? X : G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wi = wave >> 1, wj = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    const int zc = bi * 128, yc = bj * 128;
    const int64_t k0 = (int64_t)c * chunk, k1 = min(n, k0 + chunk);
    const bool vec = (p % VX) == 0;
    // the chunk's rows as raw buffers (the plan keeps chunk * p * 8 < 2^31):
    // rows past k1 and columns past p read zero
    constexpr uint32_t ES = sizeof(T);
    const uint32_t rowb = (uint32_t)p * ES;
    const uint32_t cbytes = (k1 > k0) ? (uint32_t)(k1 - k0) * rowb : 0u;
    const __amdgpu_buffer_rsrc_t rz = buf_rsrc(X + (size_t)k0 * p, cbytes);
    const __amdgpu_buffer_rsrc_t ry = buf_rsrc(Y + (size_t)k0 * p, cbytes);
    T zr[NV][VX], yr[NV][VX];
    auto load = [&](int64_t kb) {
        const uint32_t ob = (uint32_t)(kb - k0) * rowb;
#pragma unroll
        for (int s2 = 0; s2 < NV; ++s2) {
            const int e = tid + 256 * s2;
            const int kk = e / (128 / VX), col = (e % (128 / VX)) * VX;
            const int zcol = zc + col, ycol = yc + col;
            const uint32_t orow = ob + (uint32_t)kk * rowb;
            if (vec) {
                // p is a multiple of VX: a vector is wholly inside the row or past it
                const auto w = buf_ld16<T>(rz, zcol < p ? orow + (uint32_t)zcol * ES : kBufOob);
                const auto u = buf_ld16<T>(ry, ycol < p ? orow + (uint32_t)ycol * ES : kBufOob);
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    zr[s2][v] = w[v];
                    yr[s2][v] = u[v];
                }
            } else {
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    zr[s2][v] = buf_ld1<T>(rz, zcol + v < p ? orow + (uint32_t)(zcol + v) * ES : kBufOob);
                    yr[s2][v] = buf_ld1<T>(ry, ycol + v < p ? orow + (uint32_t)(ycol + v) * ES : kBufOob);
                }
            }
        }
    };
    typename Mma<T>::acc acc[4][4];
    double dacc[sizeof(T) == 4 ? 4 : 1][4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][j][q] = 0;
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) dacc[i][j][q] = 0.0;
    }
    const bool active = (zc < p) && (yc < p) && (k0 < k1);
    // in a diagonal block of a symmetric result the wave below the diagonal has
    // nothing to compute (it still stages its share of the panels)
    const bool below = (bi == bj) && (isS || wup) && (wi > wj);
    // single-pass form: the diagonal blocks of W also sum the squares of their
    // G columns (each thread always loads the same VX columns of the block)
    const bool csq = colsq && !isS && bi == bj;
    double sq[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) sq[v] = 0.0;
    const int wu = __builtin_amdgcn_readfirstlane(wave);
    auto issue = [&](int64_t kb, int b) {
        if constexpr (DL) {
            const uint32_t ob = (uint32_t)(kb - k0) * rowb;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kr = wu * 4 + u;
                const int cps = lane ^ ((kr & 1) << 3);
                const uint32_t oz = ob + (uint32_t)kr * rowb + (uint32_t)(zc + 2 * cps) * 8u;
                const uint32_t oy = ob + (uint32_t)kr * rowb + (uint32_t)(yc + 2 * cps) * 8u;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rz, (__attribute__((address_space(3))) void*)(ZsD + b * 2048 + kr * 128), 16,
                    oz, 0, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    ry, (__attribute__((address_space(3))) void*)(YsD + b * 2048 + kr * 128), 16,
                    oy, 0, 0, 0);
            }
        }
    };
    if constexpr (DL) {
        // rows past the chunk and columns past the row (the next row's values,
        // or zero past the range) only reach partial entries the reduction skips
        int dbuf = 0;
        if (active) issue(k0, 0);
        for (int64_t kb = k0; active && kb < k1; kb += 16) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            const double* zs = ZsD + dbuf * 2048;
            const double* ys = YsD + dbuf * 2048;
            if (csq) {
                // rows wave, wave + 4, ... of the lane's column pair
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    const int kr = wave + 4 * s2;
                    const int slot = lane ^ ((kr & 1) << 3);
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        const double y = ys[kr * 128 + 2 * slot + v];
                        sq[v] += (yc + 2 * lane + v < p) ? y * y : 0.0;
                    }
                }
            }
            // the chunk's operands into registers before the next chunk's
            // loads are issued (LDS reads after them would wait for them)
            double a[4][4], b[4][4];
            if (!below) {
#pragma unroll
                for (int kq = 0; kq < 4; ++kq) {
                    const int k = 4 * kq + lk;
                    const int sw = (k & 1) << 3;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int col = wi * 64 + i * 16 + lr;
                        a[kq][i] = zs[k * 128 + (((col >> 1) ^ sw) << 1) + (col & 1)];
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int col = wj * 64 + j * 16 + lr;
                        b[kq][j] = ys[k * 128 + (((col >> 1) ^ sw) << 1) + (col & 1)];
                    }
                }
            }
            if (kb + 16 < k1) issue(kb + 16, dbuf ^ 1);
            if (!below) {
#pragma unroll
                for (int kq = 0; kq < 4; ++kq)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = Mma<T>::run((T)a[kq][i], (T)b[kq][j], acc[i][j]);
            }
            dbuf ^= 1;
        }
    } else {
    if (active) load(k0);
    int step = 0;
    for (int64_t kb = k0; active && kb < k1; kb += KC, ++step) {
        __syncthreads();
#pragma unroll
        for (int s2 = 0; s2 < NV; ++s2) {
            const int e = tid + 256 * s2;
            const int kk = e / (128 / VX), col = (e % (128 / VX)) * VX;
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                Zs[kk * LS + col + v] = zr[s2][v];
                Ys[kk * LS + col + v] = yr[s2][v];
                if (csq) sq[v] += (double)yr[s2][v] * (double)yr[s2][v];
            }
        }
        __syncthreads();
        if (kb + KC < k1) load(kb + KC);
        if (below) continue;
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Zs[(kk + lk) * LS + wi * 64 + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Ys[(kk + lk) * LS + wj * 64 + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = Mma<T>::run(a[i], b[j], acc[i][j]);
        }
        if constexpr (sizeof(T) == 4) {
            if ((step % FLUSH) == FLUSH - 1) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            dacc[i][j][q] += (double)acc[i][j][q];
                            acc[i][j][q] = 0;
                        }
            }
        }
    }
    }  // !DL
    if (csq) {
        // [chunk][wave][column] partials (4 threads share a column pair)
        const int col = (tid % (128 / VX)) * VX;
#pragma unroll
        for (int v = 0; v < VX; ++v)
            if (yc + col + v < p) colsq[((size_t)c * 4 + wave) * p + yc + col + v] = sq[v];
    }
    if (below) return;
    double* out = part + ((size_t)c * n_tiles + tile) * (size_t)(128 * 128);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ii = wi * 64 + i * 16 + Mma<T>::row(lk, q);
                const int jj = wj * 64 + j * 16 + lr;
                if constexpr (sizeof(T) == 4)
                    out[ii * 128 + jj] = dacc[i][j][q] + (double)acc[i][j][q];
                else
                    out[ii * 128 + jj] = (double)acc[i][j][q];
            }
}
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 1) void k_gram_lds(const T* __restrict__ X,
                                                  const T* __restrict__ G, int64_t n, int p,
                                                  int nb, int n_s_tiles, int n_tiles, int wup,
                                                  int64_t chunk, double* __restrict__ part,
                                                  const DevState* __restrict__ st,
                                                  double* __restrict__ colsq = nullptr) {
    body_gram_lds<T>(X, G, n, p, nb, n_s_tiles, n_tiles, wup, chunk, part, st, blockIdx.x, gridDim.x,
                     colsq);
}


// Split-bf16 Gram pass (MIXED): Z^T Y ~ Zh^T Yh + Zh^T Yl + Zl^T Yh, three
// bf16 MFMA products with float32 accumulation over 256-row segments that are
// then added into float64 registers; partials as in k_gram.
template <int WM>
__device__ __forceinline__ void body_gram_bf3(const float* __restrict__ X,
                                                  const float* __restrict__ G, int64_t n, int p,
                                                  int nb, int n_s_tiles, int n_tiles, int wup,
                                                  int64_t chunk, double* __restrict__ part,
                                                  const DevState* __restrict__ st, int bid_, int nblk_) {
    if (st && st->done) return;
    constexpr int WT = 16 * WM, BT = 2 * WT;
    const int nwg = nblk_;
    const int lid = xcd_remap(bid_, nwg);
    const int tile = lid % n_tiles, c = lid / n_tiles;
    int bi, bj;
    bool isS;
    gram_tile(tile, nb, n_s_tiles, wup, bi, bj, isS);
    const float* Y = isS ? X : G;
    const int wave = threadIdx.x >> 6, wi = wave >> 1, wj = wave & 1;
    // below the diagonal of a diagonal block of a symmetric result: nothing to do
    if ((bi == bj) && (isS || wup) && (wi > wj)) return;
    const int zc0 = bi * BT + wi * WT, yc0 = bj * BT + wj * WT;
    const int64_t k0 = (int64_t)c * chunk, k1 = min(n, k0 + chunk);
    const int lane = threadIdx.x & 63, lr = lane & 15, g = lane >> 4;
    double dacc[WM][WM][4];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) dacc[i][j][q] = 0.0;
    if (zc0 < p && yc0 < p) {
        bool zok[WM], yok[WM];
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            zok[i] = (zc0 + i * 16 + lr) < p;
            yok[i] = (yc0 + i * 16 + lr) < p;
        }
        for (int64_t ks = k0; ks < k1; ks += 256) {
            const int64_t ke = min(k1, ks + 256);
            f4 acc[WM][WM];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WM; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[i][j][q] = 0.f;
            for (int64_t k = ks; k < ke; k += 32) {
                bf8 ah[WM], al[WM], bh[WM], bl[WM];
#pragma unroll
                for (int i = 0; i < WM; ++i) {
                    float a[8], b[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int64_t row = k + 8 * g + e;
                        const bool rok = row < ke;
                        a[e] = (rok && zok[i]) ? X[row * p + zc0 + i * 16 + lr] : 0.f;
                        b[e] = (rok && yok[i]) ? Y[row * p + yc0 + i * 16 + lr] : 0.f;
                    }
                    split2(a, ah[i], al[i]);
                    split2(b, bh[i], bl[i]);
                }
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WM; ++j) {
                        acc[i][j] = mma_bf(ah[i], bh[j], acc[i][j]);
                        acc[i][j] = mma_bf(ah[i], bl[j], acc[i][j]);
                        acc[i][j] = mma_bf(al[i], bh[j], acc[i][j]);
                    }
            }
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WM; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) dacc[i][j][q] += (double)acc[i][j][q];
        }
    }
    double* out = part + ((size_t)c * n_tiles + tile) * (size_t)(BT * BT);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ii = wi * WT + i * 16 + Mma<float>::row(g, q);
                const int jj = wj * WT + j * 16 + lr;
                out[ii * BT + jj] = dacc[i][j][q];
            }
}
template <int WM>
__global__ __launch_bounds__(256) void k_gram_bf3(const float* __restrict__ X,
                                                  const float* __restrict__ G, int64_t n, int p,
                                                  int nb, int n_s_tiles, int n_tiles, int wup,
                                                  int64_t chunk, double* __restrict__ part,
                                                  const DevState* __restrict__ st) {
    body_gram_bf3<WM>(X, G, n, p, nb, n_s_tiles, n_tiles, wup, chunk, part, st, blockIdx.x, gridDim.x);
}


// LDS-staged split-K Gram pass of the MIXED form for 128 x 128 tiles (p > 64).
// The workgroup walks its chunk of rows KS at a time.  Each thread loads KS/2
// rows of one column of Z (= X) and of Y (= X or G) -- 256-byte coalesced
// loads per wave, prefetched one step ahead -- splits them into bf16 pairs
// h + l and stores them transposed (K contiguous, 80-byte pitch, so that the
// 16-byte operand reads of 16 lanes hit distinct banks).  Four waves of 64 x 64
// accumulate hh + hl + lh in float32 over the whole chunk (one rounding per
// 32-row MFMA step, ~56 per entry: ~5e-7 relative on a chunk's partial, below
// the 2^-16 of the split); with no float64 accumulators two workgroups fit on
// a CU.  Partials as in k_gram.
template <typename TP = double>
__device__ __forceinline__ void body_gram_bf3_lds(const float* __restrict__ X,
                                                  const float* __restrict__ G, int64_t n, int p,
                                                  int nb, int n_s_tiles, int n_tiles, int wup,
                                                  int64_t chunk, TP* __restrict__ part,
                                                  const DevState* __restrict__ st, int bid_,
                                                  int nblk_, double* __restrict__ colsq = nullptr) {
    if (st && st->done) return;
    constexpr int KS = 32;            // rows per step
    constexpr int KP = KS + 8;        // LDS pitch in bf16
    constexpr int RH = KS / 2;        // rows per loader thread
    __shared__ __attribute__((aligned(16))) __bf16 Ls[4][128 * KP];  // Zh, Zl, Yh, Yl
    const int lid = xcd_remap(bid_, nblk_);
    const int tile = lid % n_tiles, c = lid / n_tiles;
    int bi, bj;
    bool isS;
    gram_tile(tile, nb, n_s_tiles, wup, bi, bj, isS);
    const float* Y = isS ? X : G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wi = wave >> 1, wj = wave & 1;
    const int lr = lane & 15, g = lane >> 4;
    const int zc = bi * 128, yc = bj * 128;
    const int64_t k0 = (int64_t)c * chunk, k1 = min(n, k0 + chunk);
    // loader role: column lc of the tile, rows RH * lh .. RH * lh + RH - 1 of a step
    const int lc = tid & 127, lh = tid >> 7;
    const bool zok = zc + lc < p, yok = yc + lc < p;
    // the chunk's rows as raw buffers (the plan keeps chunk * p * 8 < 2^31):
    // rows past k1 and columns past p read zero
    const uint32_t rowb = (uint32_t)p * 4u;
    const uint32_t cbytes = (k1 > k0) ? (uint32_t)(k1 - k0) * rowb : 0u;
    const __amdgpu_buffer_rsrc_t rz = buf_rsrc(X + (size_t)k0 * p, cbytes);
    const __amdgpu_buffer_rsrc_t ry = buf_rsrc(Y + (size_t)k0 * p, cbytes);
    const uint32_t oz = zok ? (uint32_t)(zc + lc) * 4u + (uint32_t)(RH * lh) * rowb : kBufOob;
    const uint32_t oy = yok ? (uint32_t)(yc + lc) * 4u + (uint32_t)(RH * lh) * rowb : kBufOob;
    float zr[RH], yr[RH];
    auto load = [&](int64_t kb) {
        const uint32_t ob = (uint32_t)(kb - k0) * rowb;
#pragma unroll
        for (int e = 0; e < RH; ++e) {
            zr[e] = buf_ldf(rz, oz + ob + (uint32_t)e * rowb);
            yr[e] = buf_ldf(ry, oy + ob + (uint32_t)e * rowb);
        }
    };
    // single-pass form: the diagonal blocks of W also sum the squares of their
    // G columns (the loader thread owns column yc + lc)
    const bool csq = colsq && !isS && bi == bj;
    double sq = 0.0;
    auto store = [&]() {
        if (csq) {
#pragma unroll
            for (int e = 0; e < RH; ++e) sq += (double)yr[e] * (double)yr[e];
        }
#pragma unroll
        for (int q = 0; q < RH / 8; ++q) {
            float a[8], b[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = zr[8 * q + e];
                b[e] = yr[8 * q + e];
            }
            bf8 ah, al, bh, bl;
            split2(a, ah, al);
            split2(b, bh, bl);
            const int o = lc * KP + RH * lh + 8 * q;
            *(bf8*)&Ls[0][o] = ah;
            *(bf8*)&Ls[1][o] = al;
            *(bf8*)&Ls[2][o] = bh;
            *(bf8*)&Ls[3][o] = bl;
        }
    };
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][j][q] = 0.f;
    const bool active = (zc < p) && (yc < p) && (k0 < k1);
    // in a diagonal block of a symmetric result the wave below the diagonal has
    // nothing to compute (it still stages its share of the panels)
    const bool below = (bi == bj) && (isS || wup) && (wi > wj);
    if (active) load(k0);
    for (int64_t kb = k0; active && kb < k1; kb += KS) {
        __syncthreads();
        store();
        __syncthreads();
        if (kb + KS < k1) load(kb + KS);
        if (below) continue;
#pragma unroll
        for (int ks = 0; ks < KS; ks += 32) {
            bf8 ah[4], al[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = (wi * 64 + i * 16 + lr) * KP + ks + 8 * g;
                ah[i] = *(const bf8*)&Ls[0][o];
                al[i] = *(const bf8*)&Ls[1][o];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = (wj * 64 + j * 16 + lr) * KP + ks + 8 * g;
                const bf8 bh = *(const bf8*)&Ls[2][o];
                const bf8 bl = *(const bf8*)&Ls[3][o];
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf(ah[i], bh, acc[i][j]);
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf(ah[i], bl, acc[i][j]);
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf(al[i], bh, acc[i][j]);
            }
        }
    }
    if (csq && yok) colsq[((size_t)c * 4 + lh) * p + yc + lc] = sq;
    if (below) return;
    TP* out = part + ((size_t)c * n_tiles + tile) * (size_t)(128 * 128);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ii = wi * 64 + i * 16 + Mma<float>::row(g, q);
                const int jj = wj * 64 + j * 16 + lr;
                out[ii * 128 + jj] = (TP)acc[i][j][q];
            }
}
// The chunk partials are float32 sums, stored as float32 (exactly what a
// float64 copy would hold, in half the bytes).
__global__ __launch_bounds__(256, 2) void k_gram_bf3_lds(const float* __restrict__ X,
                                                      const float* __restrict__ G, int64_t n,
                                                      int p, int nb, int n_s_tiles, int n_tiles, int wup,
                                                      int64_t chunk, float* __restrict__ part,
                                                      const DevState* __restrict__ st,
                                                      double* __restrict__ colsq = nullptr) {
    body_gram_bf3_lds(X, G, n, p, nb, n_s_tiles, n_tiles, wup, chunk, part, st, blockIdx.x,
                      gridDim.x, colsq);
}


// out[s][c][k] (s = 0, 1, 2: the exact bf16 split h, m, l of float(M[k][c])),
// rows c < prow, columns k < pk, zero outside p x p: the transposed, padded
// operand layout the split-bf16 row-block product reads with 16-byte loads.
__device__ __forceinline__ void body_split3_t(const double* __restrict__ M,
                                                  __bf16* __restrict__ out, int p, int prow,
                                                  int pk, const DevState* __restrict__ st, int bid_, int nblk_) {
    if (st && st->done) return;
    const int64_t e = (int64_t)bid_ * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)prow * pk;
    if (e >= tot) return;
    const int c = (int)(e / pk), k = (int)(e % pk);
    const float x = (c < p && k < p) ? (float)M[(size_t)k * p + c] : 0.f;
    const __bf16 hb = (__bf16)x;
    const float r = x - (float)hb;
    const __bf16 mb = (__bf16)r;
    out[e] = hb;
    out[tot + e] = mb;
    out[2 * tot + e] = (__bf16)(r - (float)mb);
}
__global__ __launch_bounds__(256) void k_split3_t(const double* __restrict__ M,
                                                  __bf16* __restrict__ out, int p, int prow,
                                                  int pk, const DevState* __restrict__ st) {
    body_split3_t(M, out, p, prow, pk, st, blockIdx.x, gridDim.x);
}


// MIXED form of k_residual: the same epilogue, with X M computed as six
// split-bf16 MFMA products sum_{a+b<=2} X_a M_b (X split on the fly, M from
// k_split3_t), i.e. float32-level accuracy (relative error ~2^-23).
template <bool APPLY>
__device__ __forceinline__ void body_residual_bf6(
    const float* __restrict__ X, float* __restrict__ G, const float* __restrict__ Gprev,
    const __bf16* __restrict__ MS, const __bf16* __restrict__ PS, int prow, int pk,
    const double* __restrict__ nu, int64_t n, int p, int nrb, int ncb, int64_t nrt,
    double* __restrict__ part_col, double* __restrict__ part_scal,
    const DevParams* __restrict__ prm, const DevState* __restrict__ st, int mode, int bid_, int nblk_) {
    if (st && st->done) return;
    __shared__ float Xs[64][36];
    __shared__ double sh[4];
    __shared__ double scol[2][2][64];
    const int nwg = nblk_;
    const int lid = xcd_remap(bid_, nwg);
    const int rb = lid / ncb, cb = lid % ncb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, g = lane >> 4;
    const int c0 = cb * 64 + wc * 32;
    const size_t tot = (size_t)prow * pk;

    bool kkt_due = false, have_prev = false, iterate = false;
    double eta_prev = 1.0;
    if (!APPLY) {
        const int k = st->iter;
        iterate = (mode == RES_ITERATE);
        kkt_due = PS && ((mode == RES_KKT_ONLY) || (k % prm->kkt_every == 0) ||
                         (k >= prm->max_iter));
        have_prev = iterate && (k >= 1);
        eta_prev = st->eta;
    }
    double cxg[2] = {0.0, 0.0}, cgg[2] = {0.0, 0.0};
    double skk = 0.0, sss = 0.0, ssy = 0.0, syy = 0.0;

    for (int64_t rt = rb; rt < nrt; rt += nrb) {
        const int64_t r0 = rt * 64;
        f4 a1[2][2], a2[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a1[i][j][q] = 0.f;
                    a2[i][j][q] = 0.f;
                }
        for (int kc = 0; kc < p; kc += 32) {
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * 32; e += 256) {
                const int rr = e >> 5, kk = e & 31;
                const int64_t r = r0 + rr;
                const int k = kc + kk;
                Xs[rr][kk] = (r < n && k < p) ? X[(size_t)r * p + k] : 0.f;
            }
            __syncthreads();
            bf8 xh[2], xm[2], xl[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                float xa[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) xa[e] = Xs[wr * 32 + i * 16 + lr][8 * g + e];
                split3(xa, xh[i], xm[i], xl[i]);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int c = c0 + j * 16 + lr;
                if (APPLY || iterate) {
                    const bf8* mp = (const bf8*)(MS + (size_t)c * pk + kc + 8 * g);
                    const bf8 mh = mp[0];
                    const bf8 mm = *(const bf8*)((const __bf16*)mp + tot);
                    const bf8 ml = *(const bf8*)((const __bf16*)mp + 2 * tot);
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        f4 acc = a1[i][j];
                        acc = mma_bf(xh[i], mh, acc);
                        acc = mma_bf(xh[i], mm, acc);
                        acc = mma_bf(xm[i], mh, acc);
                        acc = mma_bf(xh[i], ml, acc);
                        acc = mma_bf(xl[i], mh, acc);
                        acc = mma_bf(xm[i], mm, acc);
                        a1[i][j] = acc;
                    }
                }
                if (kkt_due) {
                    const bf8* pp = (const bf8*)(PS + (size_t)c * pk + kc + 8 * g);
                    const bf8 ph = pp[0];
                    const bf8 pm = *(const bf8*)((const __bf16*)pp + tot);
                    const bf8 pl = *(const bf8*)((const __bf16*)pp + 2 * tot);
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        f4 acc = a2[i][j];
                        acc = mma_bf(xh[i], ph, acc);
                        acc = mma_bf(xh[i], pm, acc);
                        acc = mma_bf(xm[i], ph, acc);
                        acc = mma_bf(xh[i], pl, acc);
                        acc = mma_bf(xl[i], ph, acc);
                        acc = mma_bf(xm[i], pm, acc);
                        a2[i][j] = acc;
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t r = r0 + wr * 32 + i * 16 + Mma<float>::row(g, q);
                    const int c = c0 + j * 16 + lr;
                    if (r >= n || c >= p) continue;
                    const size_t idx = (size_t)r * p + c;
                    if (APPLY) {
                        G[idx] = a1[i][j][q];
                        continue;
                    }
                    const double gv = (double)G[idx];
                    if (kkt_due) {
                        const double rk = gv - (double)a2[i][j][q];
                        skk += rk * rk;
                    }
                    if (!iterate) continue;
                    const float glt = (float)(gv - (double)a1[i][j][q]);
                    G[idx] = glt;
                    const double gl = (double)glt;
                    const double x = (double)X[idx];
                    cxg[j] += x * gl;
                    cgg[j] += gl * gl;
                    if (have_prev) {
                        const double glp = (double)Gprev[idx];
                        const double sd = (1.0 - nu[c]) * x - glp / eta_prev;
                        const double yd = gl - glp;
                        sss += sd * sd;
                        ssy += sd * yd;
                        syy += yd * yd;
                    }
                }
    }
    if (APPLY) return;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        cxg[j] += __shfl_xor(cxg[j], 16, 64);
        cxg[j] += __shfl_xor(cxg[j], 32, 64);
        cgg[j] += __shfl_xor(cgg[j], 16, 64);
        cgg[j] += __shfl_xor(cgg[j], 32, 64);
    }
    if (iterate) {
        if (g == 0) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                scol[wr][0][wc * 32 + j * 16 + lr] = cxg[j];
                scol[wr][1][wc * 32 + j * 16 + lr] = cgg[j];
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int c = cb * 64 + threadIdx.x;
            if (c < p) {
                double* pc = part_col + ((size_t)rb * p + c) * 2;
                pc[0] = scol[0][0][threadIdx.x] + scol[1][0][threadIdx.x];
                pc[1] = scol[0][1][threadIdx.x] + scol[1][1][threadIdx.x];
            }
        }
    }
    const double t0 = block_sum256(skk, sh);
    const double t1 = block_sum256(sss, sh);
    const double t2 = block_sum256(ssy, sh);
    const double t3 = block_sum256(syy, sh);
    if (threadIdx.x == 0) {
        double* ps = part_scal + (size_t)lid * 4;
        ps[0] = t0;
        ps[1] = t1;
        ps[2] = t2;
        ps[3] = t3;
    }
}
template <bool APPLY>
__global__ __launch_bounds__(256) void k_residual_bf6(
    const float* __restrict__ X, float* __restrict__ G, const float* __restrict__ Gprev,
    const __bf16* __restrict__ MS, const __bf16* __restrict__ PS, int prow, int pk, const double* __restrict__ nu, int64_t n, int p, int nrb, int ncb,
    int64_t nrt, double* __restrict__ part_col, double* __restrict__ part_scal,
    const DevParams* __restrict__ prm, const DevState* __restrict__ st, int mode) {
    body_residual_bf6<APPLY>(X, G, Gprev, MS, PS, prow, pk, nu, n, p, nrb, ncb, nrt, part_col, part_scal, prm, st, mode, blockIdx.x, gridDim.x);
}


// Order LDS writes of a wave before its later LDS reads of other lanes' data
// (a wave's LDS operations complete in issue order; this keeps the compiler
// from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Rows per wave of the LDS-resident split-bf16 residual pass (64: four waves
// and one wave per SIMD; 32: eight waves, two per SIMD).
constexpr int kMixRW = 32;

// MIXED residual pass with M_L resident in LDS.  A workgroup owns a column
// block of 64 and keeps its slice of the split M_L^T (3 x 64 x pk bf16) in LDS
// for all its row tiles; 256 / RW waves of RW rows x 64 columns walk row tiles
// of 256 rows.  X fragments come straight from global memory (8 consecutive
// columns of one row per lane, two 16-byte loads), prefetched one K-step
// ahead (the first two K-steps of the next row tile during the epilogue) and
// split into h + m + l in registers; the six products
// sum_{a+b<=2} X_a M_b give float32-level accuracy.  Epilogue, partials and BB
// pair as in k_residual (stop test by the p x p identity, so no product with
// Psi).
// FU = true: the single-pass form, as in body_residual (X^{k+1} to Xn, row
// sums of its squares over the workgroup's 64 columns to rho_part[cb][r]).
// Wide epilogue (PKMAX <= 256, where the LDS has room): a wave stages its
// product rows 16 at a time in LDS and reads them back row-major, so that a
// lane holds 4 consecutive columns and every load and store of G, X,
// gradL^{k-1}, gradL (and X^{k+1}) is a 16-byte vector (a wave instruction
// covers 4 rows x 256 bytes); the G, X and gradL^{k-1} of the first 16 rows
// are loaded before the K loop, those of the next 16 while the first are used.
template <int PKMAX, int RW, bool FU = false>
__device__ __forceinline__ void body_residual_bf6_lds(
    const float* __restrict__ X, float* __restrict__ G, const float* __restrict__ Gprev,
    const __bf16* __restrict__ MS, int prow, int pk, const double* __restrict__ nu, int64_t n,
    int p, int nrb, int ncb, int64_t nrt, double* __restrict__ part_col,
    double* __restrict__ part_scal, const DevParams* __restrict__ prm,
    const DevState* __restrict__ st, int bid_, int nblk_, float* __restrict__ Xn = nullptr,
    const double* __restrict__ nu_cur = nullptr, double* __restrict__ rho_part = nullptr) {
    if (st->done) return;
    constexpr int LP = PKMAX + 8;  // LDS pitch (bf16) of one column's K run
    constexpr int NW = 256 / RW;   // waves
    constexpr int NT = 64 * NW;    // threads
    constexpr int IT = RW / 16;    // 16-row MFMA tiles per wave
    constexpr bool WE = PKMAX <= 256 && RW == 32;
    constexpr int kPP = 68;        // LDS pitch (floats) of the staged product rows
    __shared__ __attribute__((aligned(16))) __bf16 Ms[3 * 64 * LP];
    __shared__ __attribute__((aligned(16))) float Ps[WE ? NW * 16 * kPP : 4];
    __shared__ double sh[8];
    __shared__ double scol[NW][2][64];
    const int lid = xcd_remap(bid_, nblk_);
    const int rb = lid / ncb, cb = lid % ncb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const int cblk = cb * 64;
    const size_t tot = (size_t)prow * pk;
    // wide epilogue: lane (rq, cq) takes rows 4 s + rq of a 16-row group and
    // the 4 columns cw .. cw + 3
    const int rq = lane >> 4, cq = lane & 15;
    const int cw = cblk + 4 * cq;
    {
        const int nv = pk / 8;
        for (int e = tid; e < 3 * 64 * nv; e += NT) {
            const int sp = e / (64 * nv), rem = e % (64 * nv), cc = rem / nv, kv = rem % nv;
            *(bf8*)&Ms[(sp * 64 + cc) * LP + kv * 8] =
                *(const bf8*)(MS + sp * tot + (size_t)(cblk + cc) * pk + kv * 8);
        }
    }
    __syncthreads();
    const int k = st->iter;
    const bool have_prev = k >= 1;
    const double rinv_eta = 1.0 / st->eta;
    // per-column constants: columns cblk + 16 j + lr (MFMA layout), or, in the
    // wide epilogue, cw + j.  The single-pass form updates in float32
    // arithmetic (the iterate is float32) with the reciprocals of eta^k, nu^k
    bool cok[4];
    double onu[4];
    float rnu[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = WE ? cw + j : cblk + j * 16 + lr;
        cok[j] = c < p;
        onu[j] = (have_prev && cok[j]) ? 1.0 - nu[c] : 0.0;
        rnu[j] = (FU && cok[j]) ? (float)(1.0 / nu_cur[c]) : 1.f;
    }
    const float reta_cur = FU ? (float)(1.0 / st->eta_next) : 1.f;
    double cxg[4] = {0.0, 0.0, 0.0, 0.0}, cgg[4] = {0.0, 0.0, 0.0, 0.0};
    double sss = 0.0, ssy = 0.0, syy = 0.0;
    const bool vec = (p % 4) == 0;
    const uint32_t rowb = (uint32_t)p * 4u;
    float xa[2][IT][8];
    for (int64_t rt = rb; rt < nrt; rt += nrb) {
        const int64_t r0 = rt * 256 + wave * RW;
        // the wave's rows of X, G and grad L^{k-1} as raw buffers: rows past n
        // read zero and stores to them are dropped
        const int nvr = (int)max<int64_t>(0, min<int64_t>(RW, n - r0));
        const size_t rbase = (size_t)min<int64_t>(r0, n) * p;
        const __amdgpu_buffer_rsrc_t bx = buf_rsrc(X + rbase, (uint32_t)nvr * rowb);
        const __amdgpu_buffer_rsrc_t bg = buf_rsrc(G + rbase, (uint32_t)nvr * rowb);
        const __amdgpu_buffer_rsrc_t bp = buf_rsrc(Gprev + rbase, (uint32_t)nvr * rowb);
        const __amdgpu_buffer_rsrc_t bn = buf_rsrc(FU ? Xn + rbase : X + rbase,
                                                   FU ? (uint32_t)nvr * rowb : 0u);
        // X fragments (16 rows x 8 consecutive columns per MFMA tile) of two
        // K-chunks in flight: chunk kc is split while kc + 64 is loaded
        auto load_x = [&](int kc, float (&dst)[IT][8], int64_t rbase) {
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const int64_t r = rbase + i * 16 + lr;
                const int c = kc + 8 * g;
                const float* src = X + (size_t)r * p + c;
                if (vec && r < n && c + 8 <= p) {
                    const f4 u = *(const f4*)src;
                    const f4 v = *(const f4*)(src + 4);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        dst[i][e] = u[e];
                        dst[i][4 + e] = v[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) dst[i][e] = (r < n && c + e < p) ? src[e] : 0.f;
                }
            }
        };
        f4 acc[IT][4];
#pragma unroll
        for (int i = 0; i < IT; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][j][q] = 0.f;
        auto step = [&](int kc, float (&buf)[IT][8]) {
            bf8 xh[IT], xm[IT], xl[IT];
#pragma unroll
            for (int i = 0; i < IT; ++i) split3(buf[i], xh[i], xm[i], xl[i]);
            if (kc + 64 < pk) load_x(kc + 64, buf, r0);
#pragma unroll
            for (int j0 = 0; j0 < 4; j0 += 2) {
                bf8 mh[2], mm[2], ml[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int o = ((j0 + u) * 16 + lr) * LP + kc + 8 * g;
                    mh[u] = *(const bf8*)&Ms[o];
                    mm[u] = *(const bf8*)&Ms[64 * LP + o];
                    ml[u] = *(const bf8*)&Ms[2 * 64 * LP + o];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < IT; ++i) acc[i][j0 + u] = mma_bf(xh[i], mh[u], acc[i][j0 + u]);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < IT; ++i) acc[i][j0 + u] = mma_bf(xh[i], mm[u], acc[i][j0 + u]);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < IT; ++i) acc[i][j0 + u] = mma_bf(xm[i], mh[u], acc[i][j0 + u]);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < IT; ++i) acc[i][j0 + u] = mma_bf(xh[i], ml[u], acc[i][j0 + u]);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < IT; ++i) acc[i][j0 + u] = mma_bf(xl[i], mh[u], acc[i][j0 + u]);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < IT; ++i) acc[i][j0 + u] = mma_bf(xm[i], mm[u], acc[i][j0 + u]);
            }
        };
        // wide epilogue: 16-byte slices of rows of G, X and gradL^{k-1}
        // (columns past p read zero and their stores are dropped)
        auto wld = [&](__amdgpu_buffer_rsrc_t r, int row) -> f4 {
            const uint32_t rbyte = (uint32_t)row * rowb;
            if (vec) return buf_ld16<float>(r, cok[0] ? rbyte + (uint32_t)cw * 4u : kBufOob);
            f4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[e] = buf_ldf(r, cok[e] ? rbyte + (uint32_t)(cw + e) * 4u : kBufOob);
            return v;
        };
        auto wst = [&](__amdgpu_buffer_rsrc_t r, int row, f4 v) {
            const uint32_t rbyte = (uint32_t)row * rowb;
            if (vec) {
                __builtin_amdgcn_raw_buffer_store_b128(
                    __builtin_bit_cast(v4u, v), r, cok[0] ? rbyte + (uint32_t)cw * 4u : kBufOob,
                    0, 0);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    __builtin_amdgcn_raw_buffer_store_b32(
                        __float_as_uint(v[e]), r,
                        cok[e] ? rbyte + (uint32_t)(cw + e) * 4u : kBufOob, 0, 0);
            }
        };
        f4 wg[IT][4], wx[IT][4], wp[IT][4];
        auto wload = [&](int i) {
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                const int row = i * 16 + 4 * s2 + rq;
                wg[i][s2] = wld(bg, row);
                wx[i][s2] = wld(bx, row);
                wp[i][s2] = have_prev ? wld(bp, row) : f4{0.f, 0.f, 0.f, 0.f};
            }
        };
        if constexpr (WE) wload(0);
        if (rt == rb) {
            load_x(0, xa[0], r0);
            if (32 < pk) load_x(32, xa[1], r0);
        }
        for (int kc = 0; kc < pk; kc += 64) {
            step(kc, xa[0]);
            if (kc + 32 < pk) step(kc + 32, xa[1]);
        }
        // the next row tile's first two K-chunks, in flight during the epilogue
        if (rt + nrb < nrt) {
            const int64_t r0n = (rt + nrb) * 256 + wave * RW;
            load_x(0, xa[0], r0n);
            if (32 < pk) load_x(32, xa[1], r0n);
        }

        // gradL = G - X M_L over G, one 16 x 16 sub-tile per round; the next
        // round's G, X and gradL^{k-1} are loaded before this round's arithmetic.
        // The BB and column dots of the block are summed in float32 per lane
        // (at most 4 IT terms per column, 16 IT per BB dot) and added in float64
        // Entries past n or p read zero (X rows, G, grad L^{k-1}) and have a
        // zero product (M_L is zero-padded), so they add nothing to the dots
        // and their stores fall outside the buffer.
        const float rinv_f = (float)rinv_eta;
        float tss = 0.f, tsy = 0.f, tyy = 0.f;
        float txg[4] = {0.f, 0.f, 0.f, 0.f}, tgg[4] = {0.f, 0.f, 0.f, 0.f};
        if constexpr (WE) {
            float* Pw = Ps + wave * (16 * kPP);
            float onu_f[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) onu_f[e] = (float)onu[e];
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                // the product rows i*16 .. i*16 + 15 of the wave through LDS
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        Pw[(4 * g + q) * kPP + j * 16 + lr] = acc[i][j][q];
                // the next group's loads, in flight during this group's arithmetic
                if (i + 1 < IT) wload(i + 1);
                wave_lds_sync();
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    const int row = i * 16 + 4 * s2 + rq;
                    const f4 pr = *(const f4*)&Pw[(4 * s2 + rq) * kPP + 4 * cq];
                    const f4 gv = wg[i][s2], xv = wx[i][s2], pv = wp[i][s2];
                    f4 gl, xn;
                    float rs = 0.f;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        gl[e] = gv[e] - pr[e];
                        if constexpr (FU) {
                            xn[e] = (xv[e] - gl[e] * reta_cur) * rnu[e];
                            rs += xn[e] * xn[e];
                        }
                        txg[e] += xv[e] * gl[e];
                        tgg[e] += gl[e] * gl[e];
                        if (have_prev) {
                            const float sd = onu_f[e] * xv[e] - pv[e] * rinv_f;
                            const float yd = gl[e] - pv[e];
                            tss += sd * sd;
                            tsy += sd * yd;
                            tyy += yd * yd;
                        }
                    }
                    wst(bg, row, gl);
                    if constexpr (FU) {
                        // columns past p hold x = gl = 0: xn = 0
                        wst(bn, row, xn);
#pragma unroll
                        for (int o = 8; o > 0; o >>= 1) rs += __shfl_xor(rs, o, 16);
                        const int64_t r = r0 + row;
                        if (cq == 0 && r < n) rho_part[(size_t)cb * n + r] = (double)rs;
                    }
                }
                wave_lds_sync();
            }
        } else {
        constexpr int NR = IT * 4;
        float eg[2][4], ex[2][4], ep[2][4];
        auto eoff = [&](int rw, int j) {
            return cok[j] ? (uint32_t)rw * rowb + (uint32_t)(cblk + j * 16 + lr) * 4u : kBufOob;
        };
        auto eload = [&](int rr, int sb) {
            const int i = rr / 4, j = rr % 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t o = eoff(i * 16 + Mma<float>::row(g, q), j);
                eg[sb][q] = buf_ldf(bg, o);
                ex[sb][q] = buf_ldf(bx, o);
                ep[sb][q] = have_prev ? buf_ldf(bp, o) : 0.f;
            }
        };
        eload(0, 0);
        float rsq[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            if (rr + 1 < NR) eload(rr + 1, (rr + 1) & 1);
            const int i = rr / 4, j = rr % 4, sb = rr & 1;
            const float onu_f = (float)onu[j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float gl = eg[sb][q] - acc[i][j][q];
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(gl), bg,
                                                      eoff(i * 16 + Mma<float>::row(g, q), j), 0, 0);
                if constexpr (FU) {
                    // entries past n or p: the store falls outside the buffer and
                    // x = gl = 0 adds nothing to the row sums
                    const float xn = (ex[sb][q] - gl * reta_cur) * rnu[j];
                    __builtin_amdgcn_raw_buffer_store_b32(
                        __float_as_uint(xn), bn, eoff(i * 16 + Mma<float>::row(g, q), j), 0, 0);
                    rsq[q] += cok[j] ? xn * xn : 0.f;
                }
                txg[j] += ex[sb][q] * gl;
                tgg[j] += gl * gl;
                if (have_prev) {
                    const float sd = onu_f * ex[sb][q] - ep[sb][q] * rinv_f;
                    const float yd = gl - ep[sb][q];
                    tss += sd * sd;
                    tsy += sd * yd;
                    tyy += yd * yd;
                }
            }
            if constexpr (FU) {
                if (j == 3) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float v = rsq[q];
#pragma unroll
                        for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
                        const int64_t r = r0 + i * 16 + Mma<float>::row(g, q);
                        if (lr == 0 && r < n) rho_part[(size_t)cb * n + r] = (double)v;
                        rsq[q] = 0.f;
                    }
                }
            }
        }
        }  // !WE
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            cxg[j] += (double)txg[j];
            cgg[j] += (double)tgg[j];
        }
        sss += (double)tss;
        ssy += (double)tsy;
        syy += (double)tyy;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        cxg[j] += __shfl_xor(cxg[j], 16, 64);
        cxg[j] += __shfl_xor(cxg[j], 32, 64);
        cgg[j] += __shfl_xor(cgg[j], 16, 64);
        cgg[j] += __shfl_xor(cgg[j], 32, 64);
    }
    if (g == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cc = WE ? 4 * cq + j : j * 16 + lr;
            scol[wave][0][cc] = cxg[j];
            scol[wave][1][cc] = cgg[j];
        }
    }
    __syncthreads();
    if (tid < 64) {
        const int c = cblk + tid;
        if (c < p) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                a += scol[w][0][tid];
                b += scol[w][1][tid];
            }
            double* pc = part_col + ((size_t)rb * p + c) * 2;
            pc[0] = a;
            pc[1] = b;
        }
    }
    // scalar partials: {||R||^2 (unused: identity), <S,S>, <S,Y>, <Y,Y>}
    double v[3] = {sss, ssy, syy};
#pragma unroll
    for (int q = 0; q < 3; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if (lane == 0) {
        scol[wave][0][0] = v[0];
        scol[wave][0][1] = v[1];
        scol[wave][0][2] = v[2];
    }
    __syncthreads();
    if (tid == 0) {
        double t[3] = {0.0, 0.0, 0.0};
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int q = 0; q < 3; ++q) t[q] += scol[w][0][q];
        double* ps = part_scal + (size_t)lid * 4;
        ps[0] = 0.0;
        ps[1] = t[0];
        ps[2] = t[1];
        ps[3] = t[2];
    }
    (void)sh;
    (void)prm;
}
template <int PKMAX, int RW, bool FU = false>
__global__ __launch_bounds__(64 * (256 / RW)) void k_residual_bf6_lds(
    const float* __restrict__ X, float* __restrict__ G, const float* __restrict__ Gprev,
    const __bf16* __restrict__ MS, int prow, int pk, const double* __restrict__ nu, int64_t n,
    int p, int nrb, int ncb, int64_t nrt, double* __restrict__ part_col,
    double* __restrict__ part_scal, const DevParams* __restrict__ prm,
    const DevState* __restrict__ st, float* __restrict__ Xn = nullptr,
    const double* __restrict__ nu_cur = nullptr, double* __restrict__ rho_part = nullptr) {
    body_residual_bf6_lds<PKMAX, RW, FU>(X, G, Gprev, MS, prow, pk, nu, n, p, nrb, ncb, nrt,
                                         part_col, part_scal, prm, st, blockIdx.x, gridDim.x,
                                         Xn, nu_cur, rho_part);
}


// Sum the chunk partials in a fixed order; S is written from its upper blocks
// (entries with row <= col) and mirrored, so it is exactly symmetric.
template <typename TP = double>
__device__ __forceinline__ void body_gram_reduce(const TP* __restrict__ part,
                                                     int nchunks, int n_tiles, int bt, int nb,
                                                     int n_s_tiles, int wup, int p,
                                                     double* __restrict__ S,
                                                     double* __restrict__ W,
                                                     const DevState* __restrict__ st, int bid_, int nblk_) {
    if (st && st->done) return;
    // 64 consecutive tile elements per workgroup; wave w sums the chunks
    // q = w (mod 4), two loads in flight, and wave 0 adds the four slices
    __shared__ double sred[4][64];
    const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const int64_t per = (int64_t)bt * bt;
    const int64_t e = (int64_t)bid_ * 64 + lane;
    bool live = e < per * n_tiles;
    int r = 0, c = 0;
    bool isS = false, mirrored = false;
    if (live) {
        const int tile = (int)(e / per);
        const int ii = (int)((e % per) / bt), jj = (int)(e % bt);
        int bi, bj;
        gram_tile(tile, nb, n_s_tiles, wup, bi, bj, isS);
        r = bi * bt + ii;
        c = bj * bt + jj;
        mirrored = isS || wup;
        live = r < p && c < p && !(mirrored && r > c) && (isS || W);
    }
    double s0 = 0.0, s1 = 0.0;
    if (live) {
        const size_t stride = (size_t)n_tiles * per;
        int q = slice;
        for (; q + 4 < nchunks; q += 8) {
            s0 += part[(size_t)q * stride + e];
            s1 += part[(size_t)(q + 4) * stride + e];
        }
        if (q < nchunks) s0 += part[(size_t)q * stride + e];
    }
    sred[slice][lane] = s0 + s1;
    __syncthreads();
    if (slice != 0 || !live) return;
    const double sum = (sred[0][lane] + sred[1][lane]) + (sred[2][lane] + sred[3][lane]);
    double* M = isS ? S : W;
    M[(size_t)r * p + c] = sum;
    if (mirrored) M[(size_t)c * p + r] = sum;
}
template <typename TP>
__global__ __launch_bounds__(256) void k_gram_reduce(const TP* __restrict__ part,
                                                     int nchunks, int n_tiles, int bt, int nb,
                                                     int n_s_tiles, int wup, int p,
                                                     double* __restrict__ S,
                                                     double* __restrict__ W,
                                                     const DevState* __restrict__ st) {
    body_gram_reduce(part, nchunks, n_tiles, bt, nb, n_s_tiles, wup, p, S, W, st, blockIdx.x, gridDim.x);
}


// Dense gradient G = A X = A^T X (A symmetric), written straight to G.  A may
// be stored narrower than the arithmetic (TA = float with T = double: the
// float64 form of a problem whose A is given in float32, widened exactly).
template <typename T, int WM, typename TA = T>
__global__ __launch_bounds__(256) void k_dense_grad(const TA* __restrict__ A,
                                                    const T* __restrict__ X, T* __restrict__ G,
                                                    int64_t n, int p, int nbp,
                                                    const double* __restrict__ glin,
                                                    const DevState* __restrict__ st) {
    if (st && st->done) return;
    constexpr int WT = 16 * WM, BT = 2 * WT;
    const int nwg = gridDim.x;
    const int lid = xcd_remap(blockIdx.x, nwg);
    const int bi = lid / nbp, bj = lid % nbp;
    const int wave = threadIdx.x >> 6, wi = wave >> 1, wj = wave & 1;
    const int zc0 = bi * BT + wi * WT, yc0 = bj * BT + wj * WT;
    typename Mma<T>::acc acc[WM][WM];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][j][q] = 0;
    if (zc0 < n && yc0 < p) tn_mac<T, WM, TA>(A, n, zc0, (int)n, X, p, yc0, p, 0, n, acc);
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = zc0 + i * 16 + Mma<T>::row(lk, q);
                const int c = yc0 + j * 16 + lr;
                if (r < n && c < p) {
                    const size_t idx = (size_t)r * p + c;
                    // the linear term of Problem 2 (if any)
                    G[idx] = glin ? (T)((double)acc[i][j][q] + glin[idx]) : acc[i][j][q];
                }
            }
}

// Dense gradient for p > 64 in the arithmetic of T (float64, or float32 on the
// float32 MFMA): G = A X (+ Glin), A stored as TA (a float32 A is widened
// exactly in the float64 form).  A workgroup owns 128 rows x 128 columns of
// G, four waves of 64 x 64 (4 x 4 MFMA tiles); K advances 16 at a time
// through two LDS buffers filled straight from global memory (buffer_load ...
// lds, 16 bytes a lane), the next K step in flight while this one is used,
// one barrier per step.  A panel: 128 rows x 16 k, row r holding its k-group
// s (4 floats or 2 doubles) at slot s ^ ((r >> 2) & 3) (float32) or
// s ^ ((r >> 1) & 7) (float64); X panel: 16 rows x 128 columns, row k holding
// its column pair c at slot c ^ ((k & 1) << 3) (float64) or its column quad
// at slot c ^ ((k & 3) << 2) (float32), so the MFMA operand reads spread over
// the banks.  Rows of A past n and rows of X past n read zero through the
// range check; A's entries past n in a row (the next row's finite values) meet
// X's zero rows, and X's columns past p only reach columns of G that are not
// stored.
template <typename T, typename TA>
__global__ __launch_bounds__(256, 2) void k_dense_mfma(const TA* __restrict__ A,
                                                      const T* __restrict__ X,
                                                      T* __restrict__ G, int64_t n, int p,
                                                      int nbp, const double* __restrict__ glin,
                                                      const DevState* __restrict__ st) {
    if (st && st->done) return;
    constexpr int ES = (int)sizeof(TA);
    constexpr int XE = (int)sizeof(T);
    constexpr int AP = 128 * 16;     // A panel elements (TA) per buffer
    constexpr int XV = 16 / XE;      // X elements per lane load: 2 doubles or 4 floats
    __shared__ __attribute__((aligned(16))) TA As[2 * AP];
    __shared__ __attribute__((aligned(16))) T Xs[2 * 16 * 128];
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int bi = lid / nbp, bj = lid % nbp;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wi = wave >> 1, wj = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    const int wu = __builtin_amdgcn_readfirstlane(wave);
    const int64_t r0 = (int64_t)bi * 128;
    const int c0 = bj * 128;
    const int nvr = (int)max<int64_t>(0, min<int64_t>(128, n - r0));
    const uint32_t arow = (uint32_t)n * (uint32_t)ES;
    const __amdgpu_buffer_rsrc_t ra =
        buf_rsrc(A + (size_t)min<int64_t>(r0, n) * n, (uint32_t)nvr * arow);
    constexpr int RPL = ES == 4 ? 4 : 8;  // lanes per A row (16 k of TA = 64 or 128 bytes)
    constexpr int RPI = 64 / RPL;         // A rows per wave load: 16 or 8
    constexpr int NAI = 128 / RPI / 4;    // A wave loads per wave: 2 or 4
    constexpr int XL = 128 / XV;          // lanes per X row: 64 (float64) or 32 (float32)
    constexpr int XRI = 64 / XL;          // X rows per wave load: 1 or 2
    constexpr int NXI = 16 / XRI / 4;     // X wave loads per wave: 4 or 2
    auto issue = [&](int64_t kb, int b) {
#pragma unroll
        for (int u = 0; u < NAI; ++u) {
            const int t = wu * NAI + u;
            const int row = RPI * t + lane / RPL;
            const int slot = lane % RPL;
            const int sg = (ES == 4) ? (slot ^ ((row >> 2) & 3)) : (slot ^ ((row >> 1) & 7));
            const uint32_t off = (uint32_t)row * arow + (uint32_t)(kb + sg * (16 / ES)) * ES;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                ra, (__attribute__((address_space(3))) void*)(As + b * AP + t * (1024 / ES)), 16,
                off, 0, 0, 0);
        }
        const int nxr = (int)max<int64_t>(0, min<int64_t>(16, n - kb));
        const __amdgpu_buffer_rsrc_t rx =
            buf_rsrc(X + (size_t)min<int64_t>(kb, n) * p, (uint32_t)nxr * (uint32_t)p * XE);
#pragma unroll
        for (int u = 0; u < NXI; ++u) {
            const int t = wu * NXI + u;
            const int kr = XRI * t + lane / XL;
            const int slot = lane % XL;
            const int cg = (XE == 8) ? (slot ^ ((kr & 1) << 3)) : (slot ^ ((kr & 3) << 2));
            const uint32_t off = ((uint32_t)kr * (uint32_t)p + (uint32_t)(c0 + XV * cg)) * XE;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rx, (__attribute__((address_space(3))) void*)(Xs + b * 2048 + t * (1024 / XE)),
                16, off, 0, 0, 0);
        }
    };
    typename Mma<T>::acc acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][j][q] = 0;
    int dbuf = 0;
    issue(0, 0);
    for (int64_t kb = 0; kb < n; kb += 16) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const TA* as = As + dbuf * AP;
        const T* xs = Xs + dbuf * 2048;
        // the chunk's operands into registers before the next chunk's loads
        // are issued (LDS reads after them would wait for them)
        T a[4][4], b[4][4];
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
            const int k = 4 * kq + lk;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = wi * 64 + i * 16 + lr;
                int pos;
                if constexpr (ES == 4)
                    pos = row * 16 + (((k >> 2) ^ ((row >> 2) & 3)) << 2) + (k & 3);
                else
                    pos = row * 16 + (((k >> 1) ^ ((row >> 1) & 7)) << 1) + (k & 1);
                a[kq][i] = (T)as[pos];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = wj * 64 + j * 16 + lr;
                if constexpr (XE == 8)
                    b[kq][j] = xs[k * 128 + (((col >> 1) ^ ((k & 1) << 3)) << 1) + (col & 1)];
                else
                    b[kq][j] = xs[k * 128 + (((col >> 2) ^ ((k & 3) << 2)) << 2) + (col & 3)];
            }
        }
        if (kb + 16 < n) issue(kb + 16, dbuf ^ 1);
#pragma unroll
        for (int kq = 0; kq < 4; ++kq)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = Mma<T>::run(a[kq][i], b[kq][j], acc[i][j]);
        dbuf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = r0 + wi * 64 + i * 16 + Mma<T>::row(lk, q);
                const int c = c0 + wj * 64 + j * 16 + lr;
                if (r < n && c < p) {
                    const size_t idx = (size_t)r * p + c;
                    G[idx] = glin ? (T)((double)acc[i][j][q] + glin[idx]) : acc[i][j][q];
                }
            }
}

// Tile constants of the split-bf16 dense product: 128 rows per workgroup, a
// 32-deep K step, LDS pitch of the A panel (bf16).
constexpr int kDGM = 128, kDGP = 32 + 8;

// X^T split into bf16 h + l for the split-bf16 dense product: XhT, XlT are
// p x npad ([column][k], npad a multiple of 64, zero for k >= n), through a
// 64 x 64 LDS tile (coalesced reads of X rows, coalesced writes of X^T rows).
__global__ __launch_bounds__(256) void k_split_xt(const float* __restrict__ X,
                                                  __bf16* __restrict__ XhT,
                                                  __bf16* __restrict__ XlT, int64_t n, int p,
                                                  int64_t npad, const DevState* __restrict__ st) {
    if (st && st->done) return;
    __shared__ float t[64][65];
    const int64_t k0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int kk = e >> 6, cc = e & 63;
        const int64_t k = k0 + kk;
        const int c = c0 + cc;
        t[kk][cc] = (k < n && c < p) ? X[(size_t)k * p + c] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int cc = e >> 6, kk = e & 63;
        const int c = c0 + cc;
        const int64_t k = k0 + kk;
        if (c < p && k < npad) {
            const float x = t[kk][cc];
            const __bf16 h = (__bf16)x;
            XhT[(size_t)c * npad + k] = h;
            XlT[(size_t)c * npad + k] = (__bf16)(x - (float)h);
        }
    }
}

// Split-bf16 dense product G = A X (+ Glin) with X split beforehand
// (k_split_xt): three products Ah Xh + Ah Xl + Al Xh on the bf16 MFMA with
// float32 accumulation.  A workgroup owns 128 rows x 512 columns (A is
// streamed once for p <= 512), eight waves of 64 x 128; K advances 32 at a
// time.  The A panel (128 x 32) is loaded into registers one step ahead and
// split into LDS when staged; the X panels (512 columns x 32 k, h and l) go
// straight from global memory into two LDS buffers (buffer_load ... lds), a
// column's four 16-byte k-groups at slots g ^ ((col >> 2) & 3) so that the
// operand reads spread over the banks.  Columns past p read zero (range
// check); X^T is zero for k >= n.
constexpr int kDPN = 512;
__global__ __launch_bounds__(512) void k_dense_bfp(const float* __restrict__ A,
                                                   const __bf16* __restrict__ XhT,
                                                   const __bf16* __restrict__ XlT, int64_t npad,
                                                   float* __restrict__ G, int64_t n, int p,
                                                   int ncb, const double* __restrict__ glin,
                                                   const DevState* __restrict__ st) {
    if (st && st->done) return;
    __shared__ __attribute__((aligned(16))) __bf16 La[2][kDGM * kDGP];
    __shared__ __attribute__((aligned(16))) __bf16 Lx[2][2][kDPN * 32];
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int rb = lid / ncb, cb = lid % ncb;
    const int64_t r0 = (int64_t)rb * kDGM;
    const int c0 = cb * kDPN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 2, wj = wave & 3;   // 2 x 4 waves of 64 x 128
    const int lr = lane & 15, g = lane >> 4;
    const int wu = __builtin_amdgcn_readfirstlane(wave);
    // A loader: row (tid >> 2), k offset 8 (tid & 3)
    const int ar = tid >> 2, ak = (tid & 3) * 8;
    const int64_t arow = r0 + ar;
    const bool aok = arow < n;
    float av[8];
    auto load_a = [&](int64_t k0) {
        const float* ap = A + (size_t)arow * n + k0 + ak;
        if (aok && k0 + ak + 8 <= n && (n % 4) == 0) {
            const float4 u = *(const float4*)ap;
            const float4 w = *(const float4*)(ap + 4);
            av[0] = u.x; av[1] = u.y; av[2] = u.z; av[3] = u.w;
            av[4] = w.x; av[5] = w.y; av[6] = w.z; av[7] = w.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = (aok && k0 + ak + e < n) ? ap[e] : 0.f;
        }
    };
    const int ncol = max(0, min(kDPN, p - c0));
    const uint32_t xrange = (uint32_t)ncol * (uint32_t)npad * 2u;
    const __amdgpu_buffer_rsrc_t rxh = buf_rsrc(XhT + (size_t)c0 * npad, xrange);
    const __amdgpu_buffer_rsrc_t rxl = buf_rsrc(XlT + (size_t)c0 * npad, xrange);
    // 32 wave loads per panel (16 columns x 64 bytes each), 4 per wave
    auto issue_x = [&](int64_t k0, int b) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = wu * 4 + u;
            const int col = 16 * t + (lane >> 2);
            const int gs = (lane & 3) ^ ((col >> 2) & 3);
            const uint32_t off = ((uint32_t)col * (uint32_t)npad + (uint32_t)(k0 + 8 * gs)) * 2u;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rxh, (__attribute__((address_space(3))) void*)(&Lx[b][0][t * 512]), 16, off, 0, 0,
                0);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rxl, (__attribute__((address_space(3))) void*)(&Lx[b][1][t * 512]), 16, off, 0, 0,
                0);
        }
    };
    f4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][j][q] = 0.f;
    int dbuf = 0;
    load_a(0);
    issue_x(0, 0);
    for (int64_t k0 = 0; k0 < n; k0 += 32) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        {
            bf8 h, l;
            split2(av, h, l);
            *(bf8*)&La[0][ar * kDGP + ak] = h;
            *(bf8*)&La[1][ar * kDGP + ak] = l;
        }
        if (k0 + 32 < n) load_a(k0 + 32);
        __syncthreads();
        // the step's operands into registers before the next X panels'
        // loads are issued (LDS reads after them would wait for them)
        bf8 ah[4], al[4], bh[8], bl[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = (wi * 64 + i * 16 + lr) * kDGP + 8 * g;
            ah[i] = *(const bf8*)&La[0][o];
            al[i] = *(const bf8*)&La[1][o];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int col = wj * 128 + j * 16 + lr;
            const int o = col * 32 + 8 * (g ^ ((col >> 2) & 3));
            bh[j] = *(const bf8*)&Lx[dbuf][0][o];
            bl[j] = *(const bf8*)&Lx[dbuf][1][o];
        }
        if (k0 + 32 < n) issue_x(k0 + 32, dbuf ^ 1);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf(ah[i], bh[j], acc[i][j]);
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf(ah[i], bl[j], acc[i][j]);
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][j] = mma_bf(al[i], bh[j], acc[i][j]);
        }
        dbuf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = r0 + wi * 64 + i * 16 + Mma<float>::row(g, q);
                const int c = c0 + wj * 128 + j * 16 + lr;
                if (r < n && c < p) {
                    const size_t idx = (size_t)r * p + c;
                    G[idx] = glin ? (float)((double)acc[i][j][q] + glin[idx]) : acc[i][j][q];
                }
            }
}

// -------------------------------------------------------- p x p stage 1 ----
// One workgroup per row i:  Psi = (W + W^T)/2 (eq. (Lambda1)); C = S - I; for
// PCAL with the Phi rule d_i = [X^T grad_X L_beta(X, Psi)]_ii
// = [W - S Psi + beta S C]_ii (eq. (lambda2)); M_L = Psi - beta C + Diag(d), so
// that grad_X L_beta(X, Lam) = G - X M_L; Bm = beta C - Diag(d) (so that
// G - X Psi = gradL - X Bm); feas_part[i] = sum_j C_ij^2.
//
// Dual ascent (STF_MULT_DUAL, PLAM-DA / PCAL-DA of Section 5.3): Step 3 takes
// Lam^k = Lam^{k-1} - beta C (eq. (Lambda-alm)) from Lam^0 = Psi, kept in lam2
// by iteration parity (so that an iteration redone after a precision hand-over
// reads the untouched Lam^{k-1}); M_L = Lam^k - beta C.
// MOptQR (Table 1): D = G - X G^T X = G - X W^T, i.e. M_L = W^T.
// In both, Bm = Psi - M_L (G - X Psi = D - X Bm).
__device__ __forceinline__ void body_stage1(const DevParams* __restrict__ prm,
                                                const double* __restrict__ S,
                                                const double* __restrict__ W,
                                                double* __restrict__ Psi,
                                                double* __restrict__ ML,
                                                double* __restrict__ Bm,
                                                double* __restrict__ feas_part, int p,
                                                const DevState* __restrict__ st, int bid_, int nblk_,
                                                double* __restrict__ lam2 = nullptr) {
    if (st->done) return;
    if (prm->variant == STF_MOPTQR || prm->mult_rule == STF_MULT_DUAL) {
        __shared__ double shf[4];
        const int i = bid_;
        const double beta = prm->beta;
        const bool dual = prm->variant != STF_MOPTQR;
        const int k = st->iter;
        const size_t p2 = (size_t)p * p;
        const double* Lprev = dual ? lam2 + (size_t)((k + 1) & 1) * p2 : nullptr;
        double* Lcur = dual ? lam2 + (size_t)(k & 1) * p2 : nullptr;
        double f2 = 0.0;
        for (int j = threadIdx.x; j < p; j += 256) {
            const size_t e = (size_t)i * p + j;
            const double psi = 0.5 * (W[e] + W[(size_t)j * p + i]);
            const double c = S[e] - (i == j ? 1.0 : 0.0);
            f2 += c * c;
            double ml;
            if (dual) {
                const double lam = (k == 0) ? psi : Lprev[e] - beta * c;
                Lcur[e] = lam;
                ml = lam - beta * c;
            } else {
                ml = W[(size_t)j * p + i];
            }
            Psi[e] = psi;
            ML[e] = ml;
            if (Bm) Bm[e] = psi - ml;
        }
        f2 = block_sum256(f2, shf);
        if (threadIdx.x == 0) feas_part[i] = f2;
        return;
    }
    __shared__ double sh[4];
    __shared__ double s_d;
    const int i = bid_, tid = threadIdx.x;
    const double beta = prm->beta;
    const bool phi_rule = (prm->variant == STF_PCAL) && (prm->mult_rule == STF_MULT_PSI_PHI);
    const double* Si = S + (size_t)i * p;
    const double* Wi = W + (size_t)i * p;
    double sp = 0.0, sc = 0.0, f2 = 0.0;
    for (int j = tid; j < p; j += 256) {
        const double psi = 0.5 * (Wi[j] + W[(size_t)j * p + i]);
        const double c = Si[j] - (i == j ? 1.0 : 0.0);
        sp += Si[j] * psi;   // S symmetric: S_ij Psi_ji = S_ij Psi_ij
        sc += Si[j] * c;
        f2 += c * c;
    }
    sp = block_sum256(sp, sh);
    sc = block_sum256(sc, sh);
    f2 = block_sum256(f2, sh);
    if (tid == 0) {
        s_d = phi_rule ? (Wi[i] - sp + beta * sc) : 0.0;
        feas_part[i] = f2;
    }
    __syncthreads();
    const double d = s_d;
    for (int j = tid; j < p; j += 256) {
        const double psi = 0.5 * (Wi[j] + W[(size_t)j * p + i]);
        const double c = Si[j] - (i == j ? 1.0 : 0.0);
        const double dd = (i == j) ? d : 0.0;
        Psi[(size_t)i * p + j] = psi;
        ML[(size_t)i * p + j] = psi - beta * c + dd;
        if (Bm) Bm[(size_t)i * p + j] = beta * c - dd;
    }
}
__global__ __launch_bounds__(256) void k_stage1(const DevParams* __restrict__ prm,
                                                const double* __restrict__ S,
                                                const double* __restrict__ W,
                                                double* __restrict__ Psi,
                                                double* __restrict__ ML,
                                                double* __restrict__ Bm,
                                                double* __restrict__ feas_part, int p,
                                                const DevState* __restrict__ st,
                                                double* __restrict__ lam2) {
    body_stage1(prm, S, W, Psi, ML, Bm, feas_part, p, st, blockIdx.x, gridDim.x, lam2);
}


// ------------------------------------------------------ residual pass ------
// Columns per workgroup of the float64 / float32 residual kernels: 128 x 64
// tiles keep a wave's accumulators at 64 x 32, so two independent 4-wave
// workgroups share each CU and one's epilogue overlaps the other's MFMAs.
constexpr int kResBC = 64;
// For a tile of 128 rows x kResBC columns (2 x WC waves; X and M_L staged
// through LDS in K-chunks):  gradL = G - X M_L  (written over G), and,
// when KKT and the stop test is due, R = G - X Psi with ||R||_F^2 accumulated.
// The Barzilai-Borwein pair uses the stored gradL^{k-1} (in Gprev) and the
// identity X^{k-1} = nu^{k-1} X^k + gradL^{k-1} / eta^{k-1} (the PCAL scaling
// undone), so S^k = (1 - nu^{k-1}) X^k - gradL^{k-1} / eta^{k-1}.
// APPLY = true computes Out = X M only (CholeskyQR2's X R^{-1}).
// XP = true (MOptQR, whose retraction is not a column scaling) reads the
// previous iterate X^{k-1} from Xprev instead: S^k = X^k - X^{k-1}.
//
// FU = true (the single-pass form) also takes the update of the same iteration
// in the epilogue: X^{k+1} = (X^k - gradL^k / eta^k) / nu^k (eta^k and nu^k
// are known before the pass, see k_fused_pre) written to Xn, and the squared
// entries of X^{k+1} summed per row over the workgroup's columns into
// rho_part[slot][r] (slot = column block x column wave).
template <typename T, typename TG, bool APPLY, bool KKT, int WC, bool XP = false, bool FU = false>
__device__ __forceinline__ void body_residual(
    const T* __restrict__ X, TG* __restrict__ G, const TG* __restrict__ Gprev,
    const double* __restrict__ ML, const double* __restrict__ Psi,
    const double* __restrict__ nu, int64_t n, int p, int nrb, int ncb, int64_t nrt,
    double* __restrict__ part_col, double* __restrict__ part_scal,
    const DevParams* __restrict__ prm, const DevState* __restrict__ st, int mode, int bid_, int nblk_,
    const T* __restrict__ Xprev = nullptr, T* __restrict__ Xn = nullptr,
    const double* __restrict__ nu_cur = nullptr, double* __restrict__ rho_part = nullptr) {
    if (st && st->done) return;
    constexpr int KC = sizeof(T) == 8 ? 16 : 32;  // rows of M_L (columns of X) per LDS stage
    constexpr int XS = KC + 1;
    constexpr int BC = kResBC;         // columns per workgroup
    constexpr int MST = BC + 4;
    constexpr int NT = 128 * WC;       // threads: 2 x WC waves
    constexpr int WTC = BC / WC;       // columns per wave
    constexpr int JT = WTC / 16;       // 16-column MFMA tiles per wave
    // float64: the K-chunks go straight from global memory into two LDS
    // buffers (buffer_load ... lds), so the next chunk is in flight while this
    // one is used, without staging registers and with one barrier per chunk.
    // A wave reads all of a chunk's operands from LDS before it issues the
    // next chunk's loads: an LDS read that follows a load into LDS waits for
    // it (the compiler cannot tell the two buffers apart)
    constexpr bool DL = sizeof(T) == 8 && WC == 2;
    __shared__ T Xs[DL ? 1 : 128 * XS];
    __shared__ T Ms[DL ? 1 : KC * MST];
    __shared__ __attribute__((aligned(16))) double XsD[DL ? 2 * 128 * 16 : 2];
    __shared__ __attribute__((aligned(16))) double MsD[DL ? 2 * 16 * 64 : 2];
    __shared__ double sh[2 * WC];
    __shared__ double scol[2][2][BC];
    const int nwg = nblk_;
    const int lid = xcd_remap(bid_, nwg);
    const int rb = lid / ncb, cb = lid % ncb;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, wr = wave / WC, wc = wave % WC;
    const int lr = lane & 15, lk = lane >> 4;
    const int cblk = cb * BC;
    const int c0 = cblk + wc * WTC;

    // KKT instantiations run only the stop-test product R = G - X Psi
    // (mode RES_KKT_ONLY); the others apply (APPLY) or iterate with M_L
    bool have_prev = false;
    const bool iterate = !APPLY && !KKT && (mode == RES_ITERATE);
    double eta_prev = 1.0;
    if (!APPLY && !KKT) {
        have_prev = iterate && (st->iter >= 1);
        eta_prev = st->eta;
    }
    const double* Mp = KKT ? Psi : ML;
    double cxg[JT], cgg[JT];
#pragma unroll
    for (int j = 0; j < JT; ++j) cxg[j] = cgg[j] = 0.0;
    double skk = 0.0, sss = 0.0, ssy = 0.0, syy = 0.0;
    const double rinv_eta = 1.0 / eta_prev;
    // per-column constants of this lane's four output columns
    bool cok[JT];
    double onu[JT], rnu[JT];
#pragma unroll
    for (int j = 0; j < JT; ++j) {
        const int c = c0 + j * 16 + lr;
        cok[j] = c < p;
        onu[j] = (!APPLY && !XP && have_prev && cok[j]) ? 1.0 - nu[c] : 0.0;
        rnu[j] = (FU && cok[j]) ? 1.0 / nu_cur[c] : 1.0;
    }
    const double reta_cur = FU ? 1.0 / st->eta_next : 1.0;
    const int rslot = cb * WC + wc;
    // staging of one K-chunk: X rows (128 x KC) and M_L / Psi rows (KC x BC),
    // 16-byte vectors when the row pitch allows it, prefetched one chunk ahead
    constexpr int VX = 16 / (int)sizeof(T);          // elements of X per 16-byte load
    constexpr int NXV = 128 * KC / VX / NT;          // X vectors per thread
    constexpr int NMV = KC * BC / 2 / NT;            // float64 pairs of M per thread
    const bool vec = ((p % VX) == 0);
    T xr[NXV][VX];
    T mr[NMV][2];
    auto load_chunk = [&](int64_t r0, int kc) {
#pragma unroll
        for (int s2 = 0; s2 < NXV; ++s2) {
            const int e = tid + NT * s2;
            const int rr = e / (KC / VX), kv = e % (KC / VX);
            const int64_t r = r0 + rr;
            const int k = kc + kv * VX;
            if (vec && r < n && k + VX <= p) {
                // 16-byte aligned: p is a multiple of VX and k of VX
                typedef T tv __attribute__((ext_vector_type(VX)));
                const tv w = *(const tv*)(X + (size_t)r * p + k);
#pragma unroll
                for (int v = 0; v < VX; ++v) xr[s2][v] = w[v];
            } else {
#pragma unroll
                for (int v = 0; v < VX; ++v)
                    xr[s2][v] = (r < n && k + v < p) ? X[(size_t)r * p + k + v] : (T)0;
            }
        }
#pragma unroll
        for (int s2 = 0; s2 < NMV; ++s2) {
            const int e = tid + NT * s2;
            const int kk = e / (BC / 2), cc = (e % (BC / 2)) * 2;
            const int k = kc + kk, c = cblk + cc;
            if ((p & 1) == 0 && k < p && c + 2 <= p) {
                typedef double dv2 __attribute__((ext_vector_type(2)));
                const size_t idx = (size_t)k * p + c;
                const dv2 m = *(const dv2*)(Mp + idx);
                mr[s2][0] = (T)m[0];
                mr[s2][1] = (T)m[1];
            } else {
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    const bool ok = (k < p) && (c + v < p);
                    const size_t idx = (size_t)k * p + c + v;
                    mr[s2][v] = ok ? (T)Mp[idx] : (T)0;
                }
            }
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int s2 = 0; s2 < NXV; ++s2) {
            const int e = tid + NT * s2;
            const int rr = e / (KC / VX), kv = e % (KC / VX);
#pragma unroll
            for (int v = 0; v < VX; ++v) Xs[rr * XS + kv * VX + v] = xr[s2][v];
        }
#pragma unroll
        for (int s2 = 0; s2 < NMV; ++s2) {
            const int e = tid + NT * s2;
            const int kk = e / (BC / 2), cc = (e % (BC / 2)) * 2;
#pragma unroll
            for (int v = 0; v < 2; ++v) Ms[kk * MST + cc + v] = mr[s2][v];
        }
    };

    // Direct chunk loads (float64): the X chunk of a 128-row tile (128 rows x
    // 16 doubles) is 16 wave loads of 8 rows x 128 bytes, the M chunk (16 rows
    // of M x the block's 64 columns) 8 wave loads of 2 rows x 512 bytes; a lane
    // moves 16 bytes (2 doubles) and lands at its lane's place in the wave's
    // 1 KiB of LDS.  Bank spread by XOR: X row r holds its k-pair j at slot
    // j ^ ((r >> 1) & 7), M row k its column pair c at slot c ^ ((k & 1) << 3).
    // Rows past n (X) or p (M) read zero through the buffer range check; the
    // entries of X past p in a row read the next row's (finite) values, which
    // meet M's zero rows, and M's columns past p only reach output columns
    // that are never stored.
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    const __amdgpu_buffer_rsrc_t rm = buf_rsrc(Mp, (uint32_t)((size_t)p * p * 8));
    auto issue = [&](int64_t rtl, int kc, int b) {
        if constexpr (DL) {
            const int64_t rr0 = rtl * 128;
            const int nvr = (int)max<int64_t>(0, min<int64_t>(128, n - rr0));
            const __amdgpu_buffer_rsrc_t rx =
                buf_rsrc((const double*)X + (size_t)min<int64_t>(rr0, n) * p,
                         (uint32_t)nvr * (uint32_t)p * 8u);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = wu * 4 + u;
                const int row = 8 * t + (lane >> 3);
                const int js = (lane & 7) ^ ((row >> 1) & 7);
                const uint32_t off = ((uint32_t)row * (uint32_t)p + (uint32_t)(kc + 2 * js)) * 8u;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rx, (__attribute__((address_space(3))) void*)(XsD + b * 2048 + t * 128), 16,
                    off, 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = wu * 2 + u;
                const int kr = 2 * t + (lane >> 5);
                const int cps = (lane & 31) ^ ((lane >> 5) << 3);
                const uint32_t off =
                    ((uint32_t)(kc + kr) * (uint32_t)p + (uint32_t)(cblk + 2 * cps)) * 8u;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rm, (__attribute__((address_space(3))) void*)(MsD + b * 1024 + t * 128), 16,
                    off, 0, 0, 0);
            }
        }
    };
    int64_t rt = rb;
    int dbuf = 0;
    if constexpr (DL) {
        if (rt < nrt) issue(rt, 0, 0);
    } else {
        if (rt < nrt) load_chunk(rt * 128, 0);
    }
    for (; rt < nrt; rt += nrb) {
        const int64_t r0 = rt * 128;
        typename Mma<T>::acc a1[4][JT];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < JT; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) a1[i][j][q] = 0;
        if constexpr (DL) {
            for (int kc = 0; kc < p; kc += 16) {
                // this chunk landed (every wave's loads), and every wave is done
                // with the other buffer
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                const double* xs = XsD + dbuf * 2048;
                const double* ms = MsD + dbuf * 1024;
                // the whole chunk's operands into registers first: LDS reads
                // issued after the next chunk's loads would wait for them
                double a[4][4], b[4][JT];
#pragma unroll
                for (int kq = 0; kq < 4; ++kq) {
                    const int k = 4 * kq + lk;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = wr * 64 + i * 16 + lr;
                        a[kq][i] = xs[row * 16 + (((k >> 1) ^ ((row >> 1) & 7)) << 1) + (k & 1)];
                    }
#pragma unroll
                    for (int j = 0; j < JT; ++j) {
                        const int col = wc * WTC + j * 16 + lr;
                        b[kq][j] = ms[k * 64 + (((col >> 1) ^ ((k & 1) << 3)) << 1) + (col & 1)];
                    }
                }
                if (kc + 16 < p)
                    issue(rt, kc + 16, dbuf ^ 1);
                else if (rt + nrb < nrt)
                    issue(rt + nrb, 0, dbuf ^ 1);
#pragma unroll
                for (int kq = 0; kq < 4; ++kq)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < JT; ++j)
                            a1[i][j] = Mma<T>::run((T)a[kq][i], (T)b[kq][j], a1[i][j]);
                dbuf ^= 1;
            }
        }
        for (int kc = 0; kc < (DL ? 0 : p); kc += KC) {
            __syncthreads();
            store_chunk();
            __syncthreads();
            // prefetch the next chunk (or the first chunk of the next row tile)
            if (kc + KC < p)
                load_chunk(r0, kc + KC);
            else if (rt + nrb < nrt)
                load_chunk((rt + nrb) * 128, 0);
#pragma unroll
            for (int kk = 0; kk < KC; kk += 4) {
                T a[4], b[JT];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = Xs[(wr * 64 + i * 16 + lr) * XS + kk + lk];
#pragma unroll
                for (int j = 0; j < JT; ++j) b[j] = Ms[(kk + lk) * MST + wc * WTC + j * 16 + lr];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < JT; ++j) a1[i][j] = Mma<T>::run(a[i], b[j], a1[i][j]);
            }
        }
        if (APPLY) {
            // mode 0: Out = X M; mode 1: Out -= X M
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < JT; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t r = r0 + wr * 64 + i * 16 + Mma<T>::row(lk, q);
                        if (r < n && cok[j]) {
                            const size_t idx = (size_t)r * p + c0 + j * 16 + lr;
                            if (mode == 1)
                                G[idx] = (TG)((double)G[idx] - (double)a1[i][j][q]);
                            else
                                G[idx] = (TG)a1[i][j][q];
                        }
                    }
            continue;
        }
        // G, X and gradL^{k-1} of one 16 x 16 sub-tile per round; the loads
        // of the next NB - 1 rounds are in flight during this round's arithmetic
        constexpr int NR = 4 * JT;
        constexpr int NB = 3;  // rounds of loads in flight
        TG eg[NB][4], ep[NB][4];
        T ex[NB][4], exp_[XP ? NB : 1][4];
        auto eload = [&](int rr, int sb) {
            const int i = rr / JT, j = rr % JT;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = r0 + wr * 64 + i * 16 + Mma<T>::row(lk, q);
                const bool ok = (r < n) && cok[j];
                const size_t idx = (size_t)r * p + c0 + j * 16 + lr;
                eg[sb][q] = ok ? G[idx] : (TG)0;
                ex[sb][q] = (ok && iterate) ? X[idx] : (T)0;
                ep[sb][q] = (ok && have_prev) ? Gprev[idx] : (TG)0;
                if constexpr (XP) exp_[sb][q] = (ok && have_prev) ? Xprev[idx] : (T)0;
            }
        };
#pragma unroll
        for (int rr = 0; rr < NB - 1 && rr < NR; ++rr) eload(rr, rr);
        double rsq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            if (rr + NB - 1 < NR) eload(rr + NB - 1, (rr + NB - 1) % NB);
            const int i = rr / JT, j = rr % JT, sb = rr % NB;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = r0 + wr * 64 + i * 16 + Mma<T>::row(lk, q);
                if (r >= n || !cok[j]) continue;
                const double g = (double)eg[sb][q];
                if (KKT) {
                    const double rk = g - (double)a1[i][j][q];
                    skk += rk * rk;
                }
                if (!iterate) continue;
                const TG glt = (TG)(g - (double)a1[i][j][q]);
                G[(size_t)r * p + c0 + j * 16 + lr] = glt;
                const double gl = (double)glt;
                const double x = (double)ex[sb][q];
                if constexpr (FU) {
                    const T xn = (T)((x - gl * reta_cur) * rnu[j]);
                    __builtin_nontemporal_store(xn, &Xn[(size_t)r * p + c0 + j * 16 + lr]);
                    rsq[q] += (double)xn * (double)xn;
                }
                cxg[j] += x * gl;
                cgg[j] += gl * gl;
                if (have_prev) {
                    const double glp = (double)ep[sb][q];
                    double sd;
                    if constexpr (XP)
                        sd = x - (double)exp_[sb][q];
                    else
                        sd = onu[j] * x - glp * rinv_eta;
                    const double yd = gl - glp;
                    sss += sd * sd;
                    ssy += sd * yd;
                    syy += yd * yd;
                }
            }
            if constexpr (FU) {
                if (j == JT - 1) {
                    // the row sums of this 16-row group over the wave's columns
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        double v = rsq[q];
#pragma unroll
                        for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
                        const int64_t r = r0 + wr * 64 + i * 16 + Mma<T>::row(lk, q);
                        if (lr == 0 && r < n) rho_part[(size_t)rslot * n + r] = v;
                        rsq[q] = 0.0;
                    }
                }
            }
        }
    }
    if (APPLY) return;
    // column partials: reduce over the 4 row groups of a wave, then the 2 wave rows
#pragma unroll
    for (int j = 0; j < JT; ++j) {
        cxg[j] += __shfl_xor(cxg[j], 16, 64);
        cxg[j] += __shfl_xor(cxg[j], 32, 64);
        cgg[j] += __shfl_xor(cgg[j], 16, 64);
        cgg[j] += __shfl_xor(cgg[j], 32, 64);
    }
    if (iterate) {
        if (lk == 0) {
#pragma unroll
            for (int j = 0; j < JT; ++j) {
                scol[wr][0][wc * WTC + j * 16 + lr] = cxg[j];
                scol[wr][1][wc * WTC + j * 16 + lr] = cgg[j];
            }
        }
        __syncthreads();
        if (tid < BC) {
            const int c = cblk + tid;
            if (c < p) {
                double* pc = part_col + ((size_t)rb * p + c) * 2;
                pc[0] = scol[0][0][tid] + scol[1][0][tid];
                pc[1] = scol[0][1][tid] + scol[1][1][tid];
            }
        }
    }
    const double t0 = block_sum<2 * WC>(skk, sh);
    const double t1 = block_sum<2 * WC>(sss, sh);
    const double t2 = block_sum<2 * WC>(ssy, sh);
    const double t3 = block_sum<2 * WC>(syy, sh);
    if (tid == 0) {
        double* ps = part_scal + (size_t)lid * 4;
        ps[0] = t0;
        ps[1] = t1;
        ps[2] = t2;
        ps[3] = t3;
    }
}
template <typename T, typename TG, bool APPLY, bool KKT, int WC, bool XP = false, bool FU = false>
__global__ __launch_bounds__(128 * WC, 2) void k_residual(
    const T* __restrict__ X, TG* __restrict__ G, const TG* __restrict__ Gprev,
    const double* __restrict__ ML, const double* __restrict__ Psi,
    const double* __restrict__ nu, int64_t n, int p, int nrb, int ncb, int64_t nrt,
    double* __restrict__ part_col, double* __restrict__ part_scal,
    const DevParams* __restrict__ prm, const DevState* __restrict__ st, int mode,
    const T* __restrict__ Xprev = nullptr, T* __restrict__ Xn = nullptr,
    const double* __restrict__ nu_cur = nullptr, double* __restrict__ rho_part = nullptr) {
    body_residual<T, TG, APPLY, KKT, WC, XP, FU>(X, G, Gprev, ML, Psi, nu, n, p, nrb, ncb, nrt,
                                                 part_col, part_scal, prm, st, mode, blockIdx.x,
                                                 gridDim.x, Xprev, Xn, nu_cur, rho_part);
}


// Column dots of the residual pass summed over row blocks in a fixed order,
// in col_groups(nrb) groups of row blocks (the last step adds the groups).
__device__ __forceinline__ void body_colreduce(const double* __restrict__ part_col, int nrb,
                                                   int p, double* __restrict__ colpart,
                                                   const DevState* __restrict__ st, int bx, int g) {
    if (st->done) return;
    // workgroup (bx, g): 64 consecutive values e of the 2p interleaved column
    // dots, summed over the row blocks of group g; wave w takes the rows
    // b = w (mod 4), two loads in flight
    __shared__ double sred[4][64];
    const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const int ng = col_groups(nrb);
    const int rg = (nrb + ng - 1) / ng;
    const int e = bx * 64 + lane;
    const int b0 = g * rg, b1 = min(nrb, b0 + rg);
    const size_t w2 = (size_t)2 * p;
    double s0 = 0.0, s1 = 0.0;
    if (e < 2 * p) {
        int b = b0 + slice;
        for (; b + 4 < b1; b += 8) {
            s0 += part_col[(size_t)b * w2 + e];
            s1 += part_col[(size_t)(b + 4) * w2 + e];
        }
        if (b < b1) s0 += part_col[(size_t)b * w2 + e];
    }
    sred[slice][lane] = s0 + s1;
    __syncthreads();
    if (slice == 0 && e < 2 * p)
        colpart[(size_t)g * w2 + e] = (sred[0][lane] + sred[1][lane]) + (sred[2][lane] + sred[3][lane]);
}
__global__ __launch_bounds__(256) void k_colreduce(const double* __restrict__ part_col, int nrb,
                                                   int p, double* __restrict__ colpart,
                                                   const DevState* __restrict__ st) {
    body_colreduce(part_col, nrb, p, colpart, st, blockIdx.x, blockIdx.y);
}


// The p x p part of the float64 KKT identity evaluated in stage 2: for one
// 16 x 16 tile (bx, by), T1 = S M_L and T2 = S B on the tile, then the tile's
// share of <B, T2 - 2 (W - T1)> summed in the workgroup and written to
// part[by * tiles + bx] (T1 and T2 themselves are not stored).
__device__ __forceinline__ void body_pp_gemm2(const double* __restrict__ S,
                                              const double* __restrict__ M1,
                                              const double* __restrict__ M2,
                                              const double* __restrict__ W,
                                              double* __restrict__ part, int p,
                                              const DevState* __restrict__ st, int bx, int by) {
    if (st->done) return;
    constexpr int KB = 64;  // K chunk; the next chunk is loaded while this one is used
    __shared__ double As[16][KB + 1], B1[KB][17], B2[KB][17];
    __shared__ double sh[4];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row = by * 16 + ty, col = bx * 16 + tx;
    double a[4], b1[4], b2[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ka = k0 + tx + 16 * q, kb = k0 + ty + 16 * q;
            a[q] = (row < p && ka < p) ? S[(size_t)row * p + ka] : 0.0;
            const bool ok = kb < p && col < p;
            b1[q] = ok ? M1[(size_t)kb * p + col] : 0.0;
            b2[q] = ok ? M2[(size_t)kb * p + col] : 0.0;
        }
    };
    double t1 = 0.0, t2 = 0.0;
    load(0);
    for (int k0 = 0; k0 < p; k0 += KB) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[ty][tx + 16 * q] = a[q];
            B1[ty + 16 * q][tx] = b1[q];
            B2[ty + 16 * q][tx] = b2[q];
        }
        __syncthreads();
        if (k0 + KB < p) load(k0 + KB);
#pragma unroll 16
        for (int k = 0; k < KB; ++k) {
            t1 += As[ty][k] * B1[k][tx];
            t2 += As[ty][k] * B2[k][tx];
        }
        __syncthreads();
    }
    double c = 0.0;
    if (row < p && col < p) {
        const size_t e = (size_t)row * p + col;
        c = M2[e] * (t2 - 2.0 * (W[e] - t1));
    }
    c = block_sum256(c, sh);
    if (threadIdx.x == 0) part[by * ((p + 15) / 16) + bx] = c;
}
__global__ __launch_bounds__(256) void k_pp_gemm2(const double* __restrict__ S,
                                                  const double* __restrict__ M1,
                                                  const double* __restrict__ M2,
                                                  const double* __restrict__ W,
                                                  double* __restrict__ part, int p,
                                                  const DevState* __restrict__ st) {
    body_pp_gemm2(S, M1, M2, W, part, p, st, blockIdx.x, blockIdx.y);
}

// -------------------------------------------------------- p x p stage 2 ----
// Divergence check, stop test (Section 5.1), eta^k (Section 5.1 rules), PCAL
// column norms.  With prm->kkt_identity the stop test uses
//   ||G - X Psi||^2 = ||gradL||^2 - 2 <W - S M_L, Bm> + <Bm, S Bm>
// (G - X Psi = gradL - X Bm and X^T gradL = W - S M_L), whose terms are the
// float64 column dots of the residual pass and p x p products.
__device__ __forceinline__ void body_stage2(const DevParams* __restrict__ prm,
                                                 const double* __restrict__ part_scal,
                                                 int nparts, const double* __restrict__ S,
                                                 const double* __restrict__ pp_part, int npp,
                                                 const double* __restrict__ feas_part,
                                                 double* __restrict__ colpart, int ncolg,
                                                 double* __restrict__ nu, int p,
                                                 DevState* __restrict__ st, int bid_, int nblk_,
                                                 const double* __restrict__ nu_cur = nullptr) {
    if (st->done) return;
    __shared__ double sr[7][1024];
    __shared__ double s_eta;
    __shared__ int s_stop;
    const int t = threadIdx.x;
    const bool ident = prm->kkt_identity != 0;
    // column dots: the ncolg group partials summed into group 0 (x.gradL at
    // 2c, gradL.gradL at 2c + 1), each value by the one thread that reads it
    for (int e = t; e < 2 * p; e += blockDim.x) {
        double a = 0.0;
        for (int g = 0; g < ncolg; ++g) a += colpart[(size_t)g * 2 * p + e];
        colpart[e] = a;
    }
    __syncthreads();
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = t; b < nparts; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += part_scal[(size_t)b * 4 + q];
    for (int i = t; i < p; i += blockDim.x) v[4] += feas_part[i];
    if (ident) {
        for (int i = t; i < p; i += blockDim.x) v[5] += colpart[2 * i + 1];
        // tile partials of <B, S B - 2 (W - S M_L)> from the p x p product pass
        for (int e = t; e < npp; e += blockDim.x) v[6] += pp_part[e];
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) sr[q][t] = v[q];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (t < off)
#pragma unroll
            for (int q = 0; q < 7; ++q) sr[q][t] += sr[q][t + off];
        __syncthreads();
    }
    if (t == 0) {
        const int k = st->iter;
        int stop = 0;
        const double feas = sqrt(sr[4][0]);
        st->feas = feas;
        if (!isfinite(feas) || feas > prm->feas_blowup) {
            st->status = STF_E_DIVERGED;
            stop = 1;
        }
        const bool kkt_due = !stop && ((k % prm->kkt_every == 0) || (k >= prm->max_iter));
        if (kkt_due) {
            const double k2 = ident ? fmax(0.0, sr[5][0] + sr[6][0]) : sr[0][0];
            const double kkt = sqrt(k2);
            if (k == 0) st->kkt0 = kkt;
            st->kkt = kkt;
            const bool best = (k == 0) || kkt < st->kkt_best;
            if (best) {
                st->kkt_best = kkt;
                st->k_best = k;
            }
            if (!isfinite(kkt)) {
                st->status = STF_E_DIVERGED;
                stop = 1;
            } else if (st->kkt0 == 0.0 || kkt <= prm->tol * st->kkt0) {
                st->status = STF_OK;
                stop = 1;
            } else if (prm->switch_tol > 0.0 &&
                       (kkt <= prm->switch_tol * st->kkt0 ||
                        (prm->switch_stall > 0 && k - st->k_best >= prm->switch_stall))) {
                // hand over to float64 (at switch_tol, or when the reduced-precision
                // descent has stopped improving): the state is left as it was
                // before this stage
                st->status = STF_SWITCH;
                stop = 1;
            }
        }
        if (!stop && k >= prm->max_iter) {
            st->status = STF_MAX_ITER;
            stop = 1;
        }
        double eta = st->eta;
        if (!stop) {
            const double ss = sr[1][0], sy = sr[2][0], yy = sr[3][0];
            const int rule = prm->eta_rule;
            if (prm->fused) {
                // single-pass form: eta^k was chosen before the pass
                eta = st->eta_next;
            } else if (rule == STF_ETA_CONST) {
                eta = prm->eta_const;
            } else if (k == 0) {
                eta = prm->eta0;
            } else {
                double pss = ss, psy = sy, pyy = yy;
                bool have = true;
                // eta_D is defined with the newest pair; only the BB quotients
                // are printed with the lagged one (Section 5.1)
                if (prm->bb_index == STF_BB_LAGGED && rule != STF_ETA_DIFF) {
                    pss = st->ss_l;
                    psy = st->sy_l;
                    pyy = st->yy_l;
                    have = (k >= 2);
                }
                if (!have) {
                    eta = prm->eta0;
                } else {
                    double q = NAN;
                    if (rule == STF_ETA_DIFF) {
                        q = (pss > 0.0) ? sqrt(pyy) / sqrt(pss) : NAN;
                    } else if (rule == STF_ETA_BB1 || (rule == STF_ETA_ABB && (k & 1))) {
                        q = (pss > 0.0) ? fabs(psy) / pss : NAN;
                    } else {
                        q = (psy != 0.0) ? pyy / fabs(psy) : NAN;
                    }
                    if (isfinite(q) && q > 0.0) eta = q;
                }
            }
            st->ss_l = ss;
            st->sy_l = sy;
            st->yy_l = yy;
            st->eta = eta;
        }
        if (stop) {
            st->done = 1;
            st->final_iter = k;
        }
        if (prm->history && k <= prm->max_iter) {
            double* h = prm->history + (size_t)k * 4;
            h[0] = kkt_due ? st->kkt : NAN;
            h[1] = feas;
            h[2] = stop ? NAN : eta;
            h[3] = (double)k;
        }
        s_eta = eta;
        s_stop = stop;
    }
    __syncthreads();
    if (s_stop) return;
    const double eta = s_eta;
    const bool pcal = prm->variant == STF_PCAL;
    if (prm->fused) {
        // nu^k was applied in the pass; it is the "previous" nu of the next one
        for (int c = t; c < p; c += blockDim.x) nu[c] = nu_cur[c];
        __syncthreads();
        if (t == 0) st->iter = st->iter + 1;
        return;
    }
    for (int c = t; c < p; c += blockDim.x) {
        double nv = 1.0;
        if (pcal) {
            // ||X_c - gradL_c / eta||_2^2 expanded with float64 column dots
            const double y2 = S[(size_t)c * p + c] - 2.0 * colpart[2 * c] / eta +
                              colpart[2 * c + 1] / (eta * eta);
            nv = sqrt(y2);
        }
        nu[c] = nv;
    }
    __syncthreads();
    if (t == 0) st->iter = st->iter + 1;
}
__global__ __launch_bounds__(1024) void k_stage2(const DevParams* __restrict__ prm,
                                                 const double* __restrict__ part_scal,
                                                 int nparts, const double* __restrict__ S,
                                                 const double* __restrict__ pp_part, int npp,
                                                 const double* __restrict__ feas_part,
                                                 double* __restrict__ colpart, int ncolg,
                                                 double* __restrict__ nu, int p,
                                                 DevState* __restrict__ st,
                                                 const double* __restrict__ nu_cur) {
    body_stage2(prm, part_scal, nparts, S, pp_part, npp, feas_part, colpart, ncolg, nu, p, st,
                blockIdx.x, gridDim.x, nu_cur);
}


// ------------------------------------------------------------- update ------
// X <- (X - gradL / eta) / nu (nu = 1 for PLAM), rho <- diag(X X^T).
template <typename T>
__device__ __forceinline__ void body_update(T* __restrict__ X, double* __restrict__ Xm,
                                                const T* __restrict__ GL,
                                                int64_t n, int p, const double* __restrict__ nu,
                                                double* __restrict__ rho,
                                                const DevState* __restrict__ st, int bid_, int nblk_) {
    if (st->done) return;
    const double eta = st->eta;
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)bid_ * 4 + (threadIdx.x >> 6); r < n;
         r += (int64_t)nblk_ * 4) {
        T* xr = X + (size_t)r * p;
        double* xm = Xm ? Xm + (size_t)r * p : nullptr;
        const T* gr = GL + (size_t)r * p;
        double s = 0.0;
        for (int c = lane; c < p; c += 64) {
            const double x = xm ? xm[c] : (double)xr[c];
            const double y = (x - (double)gr[c] / eta) / nu[c];
            const T yt = (T)y;
            // streamed, not re-read by this pass: non-temporal stores
            __builtin_nontemporal_store(yt, &xr[c]);
            if (xm) __builtin_nontemporal_store(y, &xm[c]);
            s += xm ? y * y : (double)yt * (double)yt;
        }
        if (rho) {
            s = wave_sum(s);
            if (lane == 0) rho[r] = s;
        }
    }
}
// The same update without a master copy for rows whose length is a multiple
// of 4: a lane holds 4 consecutive elements of a row (one 256-column slice per
// wave, so p = 256 is one pass), a wave walks kUR rows at a time with all
// their loads issued before the arithmetic, and the column scale factors nu
// of its slice stay in registers.
constexpr int kUR = 4;
template <typename T>
__global__ __launch_bounds__(256) void k_update_v(T* __restrict__ X, const T* __restrict__ GL,
                                                  int64_t n, int p,
                                                  const double* __restrict__ nu,
                                                  double* __restrict__ rho,
                                                  const DevState* __restrict__ st) {
    if (st->done) return;
    constexpr int V = 4;  // 16 bytes of float32 per lane
    typedef T tv __attribute__((ext_vector_type(V)));
    const double eta = st->eta;
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int c0 = 0; c0 < p; c0 += 64 * V) {
        const int c = c0 + lane * V;
        const bool on = c < p;
        double nuv[V];
#pragma unroll
        for (int e = 0; e < V; ++e) nuv[e] = on ? nu[c + e] : 1.0;
        for (int64_t r0 = wid * kUR; r0 < n; r0 += nw * kUR) {
            tv xv[kUR], gv[kUR];
#pragma unroll
            for (int u = 0; u < kUR; ++u) {
                const int64_t r = r0 + u;
                if (on && r < n) {
                    xv[u] = *(const tv*)(X + (size_t)r * p + c);
                    gv[u] = *(const tv*)(GL + (size_t)r * p + c);
                }
            }
#pragma unroll
            for (int u = 0; u < kUR; ++u) {
                const int64_t r = r0 + u;
                double sq = 0.0;
                if (on && r < n) {
                    tv y;
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        const double v = ((double)xv[u][e] - (double)gv[u][e] / eta) / nuv[e];
                        y[e] = (T)v;
                        sq += (double)y[e] * (double)y[e];
                    }
                    __builtin_nontemporal_store(y, (tv*)(X + (size_t)r * p + c));
                }
                if (rho) {
                    sq = wave_sum(sq);
                    if (lane == 0 && r < n) {
                        if (c0 == 0)
                            rho[r] = sq;
                        else
                            rho[r] += sq;
                    }
                }
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_update(T* __restrict__ X, double* __restrict__ Xm,
                                                const T* __restrict__ GL,
                                                int64_t n, int p, const double* __restrict__ nu,
                                                double* __restrict__ rho,
                                                const DevState* __restrict__ st) {
    body_update<T>(X, Xm, GL, n, p, nu, rho, st, blockIdx.x, gridDim.x);
}


// --------------------------------------------------------- CholeskyQR ------
// Blocked right-looking Cholesky S = R^T R (R upper) and R^{-1}, float64, in
// 64 x 64 blocks (nb = ceil(p / 64) block rows) without a host round trip:
//   k_chol_init        A <- S (working copy), R, Rinv <- 0
//   for j = 0 .. nb-1:
//     k_chol_diag(j)   R_jj = chol(A_jj) and Z_jj = R_jj^{-1}, in LDS (one workgroup)
//     k_chol_step(j)   for every upper block pair j < m <= l of the trailing
//                      matrix: P_m = Z_jj^T A_jm, P_l = Z_jj^T A_jl (the row
//                      panel R_jm, R_jl), A_ml -= P_m^T P_l; the pair (l, l)
//                      writes R_jl
//   k_chol_inv_off(s)  for s = 1 .. nb-1, every block Rinv_{i,i+s} =
//                      -Z_ii sum_{k=i+1}^{i+s} R_ik Rinv_{k,i+s} (blocks of
//                      smaller offset are complete)
// Every 64 x 64 product is sixteen 16 x 16 float64 MFMA tiles (dst_tile), one
// per wave of a 1024-thread workgroup, on zero-padded LDS operands.  Rows and
// columns past p are padded with the identity, so ragged last blocks need no
// special case.
constexpr int kCB = 64;

__global__ __launch_bounds__(256) void k_chol_init(const double* __restrict__ S,
                                                   double* __restrict__ A,
                                                   double* __restrict__ R,
                                                   double* __restrict__ Rinv, int p,
                                                   const DevState* __restrict__ st) {
    if (st && st->done) return;
    const size_t p2 = (size_t)p * p;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < p2;
         e += (size_t)gridDim.x * blockDim.x) {
        A[e] = S[e];
        R[e] = 0.0;
        Rinv[e] = 0.0;
    }
}

// block (bi, bj) of a p x p row-major matrix into a padded LDS tile; rows or
// columns past p read as the identity when `eye`, else as zero; `trans`
// stores the transpose
__device__ __forceinline__ void chol_load(double* D, const double* M, int p, int bi, int bj,
                                          bool eye, bool trans) {
    for (int e = threadIdx.x; e < kCB * kCB; e += blockDim.x) {
        const int r = e / kCB, c = e % kCB;
        const int gr = bi * kCB + r, gc = bj * kCB + c;
        double v;
        if (gr < p && gc < p)
            v = M[(size_t)gr * p + gc];
        else
            v = (eye && gr == gc) ? 1.0 : 0.0;
        if (trans)
            D[c * kDP + r] = v;
        else
            D[r * kDP + c] = v;
    }
}

__global__ __launch_bounds__(1024) void k_chol_diag(double* __restrict__ A,
                                                    double* __restrict__ R,
                                                    double* __restrict__ Rinv, int p, int j,
                                                    DevState* __restrict__ st,
                                                    int stop_on_fail) {
    if (st && st->done) return;
    __shared__ double a[kCB * kDP], z[kCB * kDP];
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    chol_load(a, A, p, j, j, true, false);
    __syncthreads();
    // upper Cholesky of the block, one column at a time
    for (int c = 0; c < kCB; ++c) {
        const double d = a[c * kDP + c];
        const bool ok = d > 0.0 && isfinite(d);
        const double piv = ok ? sqrt(d) : 1.0;
        __syncthreads();
        if (t == 0) {
            a[c * kDP + c] = piv;
            if (!ok && bad == 0) bad = j * kCB + c + 1;
        }
        if (t > c && t < kCB) a[c * kDP + t] /= piv;
        __syncthreads();
        // trailing update of the upper triangle: a[i][l] -= a[c][i] a[c][l], c < i <= l
        for (int e = t; e < kCB * kCB; e += blockDim.x) {
            const int i = e / kCB, l = e % kCB;
            if (i > c && l >= i) a[i * kDP + l] -= a[c * kDP + i] * a[c * kDP + l];
        }
        __syncthreads();
    }
    // Z = R^{-1} (upper), one row at a time from the bottom; 16 threads per
    // column share the dot product z[i][c] = (delta_ic - sum_{i<l<=c} r[i][l] z[l][c]) / r[i][i]
    {
        const int c = t >> 4, part = t & 15;
        for (int e = t; e < kCB * kCB; e += blockDim.x) z[(e / kCB) * kDP + e % kCB] = 0.0;
        __syncthreads();
        for (int i = kCB - 1; i >= 0; --i) {
            double acc = 0.0;
            if (c >= i)
                for (int l = i + 1 + part; l <= c; l += 16) acc += a[i * kDP + l] * z[l * kDP + c];
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
            if (c >= i && part == 0) z[i * kDP + c] = ((i == c ? 1.0 : 0.0) - acc) / a[i * kDP + i];
            __syncthreads();
        }
    }
    // store R_jj and Z_jj (upper parts; the lower parts stay zero)
    for (int e = t; e < kCB * kCB; e += blockDim.x) {
        const int r = e / kCB, c = e % kCB;
        const int gr = j * kCB + r, gc = j * kCB + c;
        if (gr < p && gc < p && c >= r) {
            R[(size_t)gr * p + gc] = a[r * kDP + c];
            Rinv[(size_t)gr * p + gc] = z[r * kDP + c];
        }
    }
    if (t == 0 && st && bad) {
        if (st->info == 0) st->info = bad;
        if (stop_on_fail) {
            st->status = STF_E_DIVERGED;
            st->final_iter = st->iter > 0 ? st->iter - 1 : 0;
            st->done = 1;
        }
    }
}

// one upper block pair (m, l) of the trailing matrix per workgroup
__global__ __launch_bounds__(1024) void k_chol_step(double* __restrict__ A,
                                                    double* __restrict__ R,
                                                    const double* __restrict__ Rinv, int p,
                                                    int j, int nb,
                                                    const DevState* __restrict__ st) {
    if (st && st->done) return;
    __shared__ double zt[kCB * kDP], am[kCB * kDP], al[kCB * kDP];
    // pair index -> (m, l), m <= l, both in (j, nb)
    const int t2 = nb - j - 1;
    int u = blockIdx.x, m = 0;
    while (u >= t2 - m) {
        u -= t2 - m;
        ++m;
    }
    const int bm = j + 1 + m, bl = bm + u;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int ti = wave >> 2, tj = wave & 3;
    chol_load(zt, Rinv, p, j, j, true, true);   // Z_jj^T
    chol_load(am, A, p, j, bm, false, false);
    chol_load(al, A, p, j, bl, false, false);
    __syncthreads();
    const d4 pm = dst_tile(zt, am, ti, tj, lr, lk);
    const d4 pl = (bl == bm) ? pm : dst_tile(zt, al, ti, tj, lr, lk);
    __syncthreads();
    // am <- P_m^T, al <- P_l
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 16 * ti + Mma<double>::row(lk, q), c = 16 * tj + lr;
        am[c * kDP + r] = pm[q];
        al[r * kDP + c] = pl[q];
    }
    __syncthreads();
    const d4 up = dst_tile(am, al, ti, tj, lr, lk);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 16 * ti + Mma<double>::row(lk, q), c = 16 * tj + lr;
        const int gr = bm * kCB + r, gc = bl * kCB + c;
        if (gr < p && gc < p) A[(size_t)gr * p + gc] -= up[q];
        if (bm == bl) {
            const int hr = j * kCB + r;
            if (hr < p && gc < p) R[(size_t)hr * p + gc] = pl[q];
        }
    }
}

// blocks (i, i + s) of R^{-1}, one per workgroup
__global__ __launch_bounds__(1024) void k_chol_inv_off(const double* __restrict__ R,
                                                       double* __restrict__ Rinv, int p,
                                                       int s_off,
                                                       const DevState* __restrict__ st) {
    if (st && st->done) return;
    __shared__ double ra[kCB * kDP], zb[kCB * kDP];
    const int i = blockIdx.x, jb = i + s_off;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int ti = wave >> 2, tj = wave & 3;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k = i + 1; k <= jb; ++k) {
        __syncthreads();
        chol_load(ra, R, p, i, k, false, false);
        chol_load(zb, Rinv, p, k, jb, false, false);
        __syncthreads();
        const d4 t = dst_tile(ra, zb, ti, tj, lr, lk);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += t[q];
    }
    __syncthreads();
    chol_load(ra, Rinv, p, i, i, false, false);  // Z_ii
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 16 * ti + Mma<double>::row(lk, q), c = 16 * tj + lr;
        zb[r * kDP + c] = acc[q];
    }
    __syncthreads();
    const d4 o = dst_tile(ra, zb, ti, tj, lr, lk);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 16 * ti + Mma<double>::row(lk, q), c = 16 * tj + lr;
        const int gr = i * kCB + r, gc = jb * kCB + c;
        if (gr < p && gc < p) Rinv[(size_t)gr * p + gc] = -o[q];
    }
}

// The p x p term of the float64 KKT identity with a single product for wide p:
// <B, S B - 2 (W - S M_L)> = <B, S (B + 2 M_L)> - 2 <B, W>.  Workgroup
// (bx, by, kb) forms the kb-th 64-deep term of the 64 x 64 tile (bx, by) of
// S (B + 2 M_L) (sixteen 16 x 16 float64 MFMA tiles over LDS panels) and its
// share of the inner product (the -2 <B, W> term with kb = 0), reduced in the
// workgroup into part[(kb * nt + by) * nt + bx]: nt^3 workgroups, so that the
// p x p stage spreads over the chip instead of nt^2 workgroups walking K.
__global__ __launch_bounds__(1024) void k_pp_kkt64(const double* __restrict__ S,
                                                   const double* __restrict__ ML,
                                                   const double* __restrict__ Bm,
                                                   const double* __restrict__ W,
                                                   double* __restrict__ part, int p,
                                                   const DevState* __restrict__ st) {
    if (st->done) return;
    __shared__ double sa[kCB * kDP], sb[kCB * kDP];
    __shared__ double sh[16];
    const int bx = blockIdx.x, by = blockIdx.y, kb = blockIdx.z, nt = gridDim.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int ti = wave >> 2, tj = wave & 3;
    chol_load(sa, S, p, by, kb, false, false);
    for (int e = threadIdx.x; e < kCB * kCB; e += blockDim.x) {
        const int r = e / kCB, c = e % kCB;
        const int gr = kb * kCB + r, gc = bx * kCB + c;
        sb[r * kDP + c] = (gr < p && gc < p)
                              ? Bm[(size_t)gr * p + gc] + 2.0 * ML[(size_t)gr * p + gc]
                              : 0.0;
    }
    __syncthreads();
    const d4 acc = dst_tile(sa, sb, ti, tj, lr, lk);
    double c = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int gr = by * kCB + 16 * ti + Mma<double>::row(lk, q);
        const int gc = bx * kCB + 16 * tj + lr;
        if (gr < p && gc < p) {
            const size_t e = (size_t)gr * p + gc;
            c += Bm[e] * (kb == 0 ? acc[q] - 2.0 * W[e] : acc[q]);
        }
    }
    c = block_sum<16>(c, sh);
    if (threadIdx.x == 0) part[((size_t)kb * nt + by) * nt + bx] = c;
}

// C = A B for p x p float64 matrices, 64 x 64 tiles of float64 MFMA.
__global__ __launch_bounds__(1024) void k_pp_mm64(const double* __restrict__ A,
                                                  const double* __restrict__ B,
                                                  double* __restrict__ C, int p,
                                                  const DevState* __restrict__ st) {
    if (st && st->done) return;
    __shared__ double sa[kCB * kDP], sb[kCB * kDP];
    const int bx = blockIdx.x, by = blockIdx.y, nt = gridDim.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int ti = wave >> 2, tj = wave & 3;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int kb = 0; kb < nt; ++kb) {
        __syncthreads();
        chol_load(sa, A, p, by, kb, false, false);
        chol_load(sb, B, p, kb, bx, false, false);
        __syncthreads();
        const d4 t = dst_tile(sa, sb, ti, tj, lr, lk);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += t[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int gr = by * kCB + 16 * ti + Mma<double>::row(lk, q);
        const int gc = bx * kCB + 16 * tj + lr;
        if (gr < p && gc < p) C[(size_t)gr * p + gc] = acc[q];
    }
}

// Single-pass form, before the residual pass of iteration k: eta^k by the
// step-size rule on the lagged pair (S^{k-1}, Y^{k-1}), whose inner products
// the previous pass left in the state, and the PCAL column norms of
// Y = X^k - gradL^k / eta^k without forming gradL^k:
//   ||Y_c||^2 = S_cc - 2 (W - S M_L)_cc / eta + (G^T G - 2 M_L^T W + M_L^T S M_L)_cc / eta^2
// (X^T gradL = W - S M_L, gradL^T gradL = G^T G - W^T M_L - M_L^T W + M_L^T S M_L),
// with diag(G^T G) from the Gram pass's column sums (nsl slots per chunk) and
// SM = S M_L.  A workgroup takes 64 columns (one per lane, coalesced rows of
// M_L, W and SM); its four waves split the sums over j and over the chunks.
// Writes nu_cur and (workgroup 0) st->eta_next.
__global__ __launch_bounds__(256) void k_fused_pre(const DevParams* __restrict__ prm,
                                                   const double* __restrict__ S,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ ML,
                                                   const double* __restrict__ SM,
                                                   const double* __restrict__ colsq,
                                                   int nchunks, int nsl,
                                                   double* __restrict__ nu_cur, int p,
                                                   DevState* __restrict__ st) {
    if (st->done) return;
    __shared__ double red[3][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    // eta^k: the same scalar in every workgroup
    const int k = st->iter;
    const int rule = prm->eta_rule;
    double eta = st->eta;
    if (rule == STF_ETA_CONST) {
        eta = prm->eta_const;
    } else if (k < 2) {
        eta = prm->eta0;   // the lagged pair exists from k = 2 on
    } else {
        const double pss = st->ss_l, psy = st->sy_l, pyy = st->yy_l;
        double q = NAN;
        if (rule == STF_ETA_BB1 || (rule == STF_ETA_ABB && (k & 1)))
            q = (pss > 0.0) ? fabs(psy) / pss : NAN;
        else
            q = (psy != 0.0) ? pyy / fabs(psy) : NAN;
        if (isfinite(q) && q > 0.0) eta = q;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->eta_next = eta;
    if (prm->variant != STF_PCAL) {
        if (wave == 0 && c < p) nu_cur[c] = 1.0;
        return;
    }
    double gg = 0.0, mw = 0.0, msm = 0.0;
    if (c < p) {
        for (int ch = wave; ch < nchunks; ch += 4)
            for (int q = 0; q < nsl; ++q) gg += colsq[((size_t)ch * 4 + q) * p + c];
#pragma unroll 4
        for (int j = wave; j < p; j += 4) {
            const double m = ML[(size_t)j * p + c];
            mw += m * W[(size_t)j * p + c];
            msm += m * SM[(size_t)j * p + c];
        }
    }
    red[0][wave][lane] = gg;
    red[1][wave][lane] = mw;
    red[2][wave][lane] = msm;
    __syncthreads();
    if (wave == 0 && c < p) {
        gg = (red[0][0][lane] + red[0][1][lane]) + (red[0][2][lane] + red[0][3][lane]);
        mw = (red[1][0][lane] + red[1][1][lane]) + (red[1][2][lane] + red[1][3][lane]);
        msm = (red[2][0][lane] + red[2][1][lane]) + (red[2][2][lane] + red[2][3][lane]);
        const double xg = W[(size_t)c * p + c] - SM[(size_t)c * p + c];
        const double y2 = S[(size_t)c * p + c] - 2.0 * xg / eta + (gg - 2.0 * mw + msm) / (eta * eta);
        nu_cur[c] = sqrt(y2);
    }
}

// rho[r] = sum over the slots of the single-pass residual's row partials.
__global__ __launch_bounds__(256) void k_rho_reduce(const double* __restrict__ part, int nslots,
                                                    int64_t n, double* __restrict__ rho,
                                                    const DevState* __restrict__ st) {
    if (st->done) return;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int q = 0; q < nslots; ++q) a += part[(size_t)q * n + r];
        rho[r] = a;
    }
}

// ---------------------------------------------------------- conversions ----
template <typename A, typename B>
__global__ void k_convert(const A* __restrict__ in, B* __restrict__ out, size_t count) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x)
        out[e] = (B)in[e];
}

// --------------------------------------------------------- evaluation ------
// Partial sums of <X, G> over n*p, <rho, phi> over n, <X, Glin> over n*p and
// sum rho^{4/3} over n (each only when its operands are given).
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ X,
                                              const double* __restrict__ G, size_t np,
                                              const double* __restrict__ rho,
                                              const double* __restrict__ phi, int64_t n,
                                              const double* __restrict__ glin, int exch,
                                              double* __restrict__ out) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < np;
         e += (size_t)gridDim.x * blockDim.x) {
        a += X[e] * G[e];
        if (glin) c += X[e] * glin[e];
    }
    if (rho)
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
             e += (int64_t)gridDim.x * blockDim.x) {
            if (phi) b += rho[e] * phi[e];
            if (exch) d += rho[e] * cbrt(rho[e]);
        }
    const double ta = block_sum256(a, sh);
    const double tb = block_sum256(b, sh);
    const double tc = block_sum256(c, sh);
    const double td = block_sum256(d, sh);
    if (threadIdx.x == 0) {
        out[blockIdx.x * 4] = ta;
        out[blockIdx.x * 4 + 1] = tb;
        out[blockIdx.x * 4 + 2] = tc;
        out[blockIdx.x * 4 + 3] = td;
    }
}

// f from <X, G>: with G = H0 X B + Glin + alpha Diag(phi) X - 2 gamma Diag(rho^{1/3}) X,
//   f = 1/2 <X, G> + 1/2 <X, Glin> - alpha/4 rho^T phi + gamma/4 sum rho^{4/3};
// kkt = sqrt(sum of the residual partials), feas = ||S - I||_F from the row
// sums of stage 1.
__global__ __launch_bounds__(256) void k_eval_finish(const double* __restrict__ dots, int nd,
                                                     const double* __restrict__ part_scal,
                                                     int nps,
                                                     const double* __restrict__ feas_part,
                                                     int p, double alpha, double gamma,
                                                     DevState* __restrict__ st) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0, k2 = 0.0, f2 = 0.0;
    for (int i = threadIdx.x; i < nd; i += 256) {
        a += dots[4 * i];
        b += dots[4 * i + 1];
        c += dots[4 * i + 2];
        d += dots[4 * i + 3];
    }
    for (int i = threadIdx.x; i < nps; i += 256) k2 += part_scal[(size_t)i * 4];
    // the rows of ||S - I||_F^2 from stage 1
    for (int i = threadIdx.x; i < p; i += 256) f2 += feas_part[i];
    a = block_sum256(a, sh);
    b = block_sum256(b, sh);
    c = block_sum256(c, sh);
    d = block_sum256(d, sh);
    k2 = block_sum256(k2, sh);
    f2 = block_sum256(f2, sh);
    if (threadIdx.x == 0) {
        st->red[0] = 0.5 * a + 0.5 * c - 0.25 * alpha * b + 0.25 * gamma * d;
        st->red[1] = sqrt(k2);
        st->red[2] = sqrt(f2);
    }
}

// MOptQR: V = X - D / eta^k (out of place).
__global__ __launch_bounds__(256) void k_vform(const double* __restrict__ X,
                                               const double* __restrict__ D,
                                               double* __restrict__ V, size_t np,
                                               const DevState* __restrict__ st) {
    if (st->done) return;
    const double eta = st->eta;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < np;
         e += (size_t)gridDim.x * blockDim.x)
        V[e] = X[e] - D[e] / eta;
}

// ================================================================ batched ===
// Grouped launches for many independent problems: one launch per stage covers
// every problem of a group; workgroup x belongs to the problem whose range
// [off[j], off[j+1]) contains x and runs that problem's body with its own
// sizes, plan, buffers and device state (a finished problem's workgroups
// return at once).  `parity` selects G / gradL^{k-1} in the double buffer:
// all problems of a batch take their iterations in lockstep.

// Index j of the range [off[j], off[j+1]) holding x (off[0] = 0 <= x < off[cnt]).
__device__ __forceinline__ int group_find(const int32_t* __restrict__ off, int cnt, int x) {
    int lo = 0, hi = cnt;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

#define STF_BATCH_PROLOGUE                                              \
    const int j_ = group_find(off, cnt, (int)blockIdx.x);              \
    const BDesc& d = D[list[j_]];                                      \
    const int lid_ = (int)blockIdx.x - off[j_];                        \
    const int nb_ = off[j_ + 1] - off[j_];                             \
    (void)lid_;                                                        \
    (void)nb_;

#define STF_BATCH_ARGS                                                              \
    const BDesc* __restrict__ D, const int32_t* __restrict__ list,                  \
        const int32_t* __restrict__ off, int cnt, int parity

__global__ __launch_bounds__(1024) void kb_hartree1d(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    if (d.alpha == 0.0) return;
    body_hartree1d(d.rho, d.phi, d.n, d.st, 0, 1);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_rowsq(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const T* x = d.Xm ? (const T*)d.Xm : (const T*)d.X;
    body_rowsq<T>(x, d.n, d.p, d.rho, nullptr, lid_, nb_);
}

// 1D stencil gradient; the float32 forms read the float64 master iterate
template <typename T, typename TO>
__global__ __launch_bounds__(256) void kb_grad(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const T* x = d.Xm ? (const T*)d.Xm : (const T*)d.X;
    body_grad_stencil<T, TO, 2>(x, (TO*)d.g[parity], d.n, d.p, (int)d.n, 1, 1, d.v,
                                d.alpha != 0.0 ? d.phi : nullptr, d.alpha, GradExtra{}, d.st,
                                lid_, nb_);
}

template <typename T, int WM>
__global__ __launch_bounds__(256) void kb_gram(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const GramPlan& g = d.gram;
    body_gram<T, WM>((const T*)d.X, (const T*)d.g[parity], d.n, d.p, g.nb, g.n_s_tiles,
                     g.n_tiles, g.wup, g.chunk, d.gram_part, d.st, lid_, nb_);
}

__global__ __launch_bounds__(256, 2) void kb_gram_lds64(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const GramPlan& g = d.gram;
    body_gram_lds<double>((const double*)d.X, (const double*)d.g[parity], d.n, d.p, g.nb,
                          g.n_s_tiles, g.n_tiles, g.wup, g.chunk, d.gram_part, d.st, lid_, nb_);
}

template <int WM>
__global__ __launch_bounds__(256) void kb_gram_bf3(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const GramPlan& g = d.gram;
    body_gram_bf3<WM>((const float*)d.X, (const float*)d.g[parity], d.n, d.p, g.nb,
                      g.n_s_tiles, g.n_tiles, g.wup, g.chunk, d.gram_part, d.st, lid_, nb_);
}

__global__ __launch_bounds__(256) void kb_gram_bf3_lds(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const GramPlan& g = d.gram;
    body_gram_bf3_lds((const float*)d.X, (const float*)d.g[parity], d.n, d.p, g.nb,
                      g.n_s_tiles, g.n_tiles, g.wup, g.chunk, d.gram_part, d.st, lid_, nb_);
}

__global__ __launch_bounds__(256) void kb_gram_reduce(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const GramPlan& g = d.gram;
    body_gram_reduce(d.gram_part, g.nchunks, g.n_tiles, g.bt, g.nb, g.n_s_tiles, g.wup, d.p,
                     d.S, d.W,
                     d.st, lid_, nb_);
}

__global__ __launch_bounds__(256) void kb_stage1(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    body_stage1(d.prm, d.S, d.W, d.Psi, d.ML, d.Bm, d.fpart, d.p, d.st, lid_, nb_);
}

__global__ __launch_bounds__(256) void kb_pp_gemm2(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const int t = (d.p + 15) / 16;
    body_pp_gemm2(d.S, d.ML, d.Bm, d.W, d.T1, d.p, d.st, lid_ % t, lid_ / t);
}

__global__ __launch_bounds__(256) void kb_split3(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const int prow = d.res.ncb * 64, pk = (d.p + 31) / 32 * 32;
    body_split3_t(d.ML, d.mix, d.p, prow, pk, d.st, lid_, nb_);
}

template <typename T>
__global__ __launch_bounds__(256, 2) void kb_residual(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const ResPlan& r = d.res;
    body_residual<T, T, false, false, 2>((const T*)d.X, (T*)d.g[parity], (const T*)d.g[parity ^ 1],
                                   d.ML, d.Psi, d.nu, d.n, d.p, r.nrb, r.ncb, r.nrt, d.res_col,
                                   d.res_scal, d.prm, d.st, RES_ITERATE, lid_, nb_);
}

template <int PKMAX>
__global__ __launch_bounds__(64 * (256 / kMixRW)) void kb_residual_bf6_lds(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const ResPlan& r = d.res;
    const int prow = r.ncb * 64, pk = (d.p + 31) / 32 * 32;
    body_residual_bf6_lds<PKMAX, kMixRW>((const float*)d.X, (float*)d.g[parity],
                                 (const float*)d.g[parity ^ 1], d.mix, prow, pk, d.nu, d.n,
                                 d.p, r.nrb, r.ncb, r.nrt, d.res_col, d.res_scal, d.prm, d.st,
                                 lid_, nb_);
}

__global__ __launch_bounds__(256) void kb_colreduce(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const int nch = (2 * d.p + 63) / 64;
    body_colreduce(d.res_col, d.res.nrb, d.p, d.colpart, d.st, lid_ % nch, lid_ / nch);
}

__global__ __launch_bounds__(1024) void kb_stage2(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    const int npt = (d.p + 15) / 16;
    body_stage2(d.prm, d.res_scal, d.res.nrb * d.res.ncb, d.S, d.T1, npt * npt, d.fpart,
                d.colpart, col_groups(d.res.nrb), d.nu, d.p, d.st, 0, 1);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_update(STF_BATCH_ARGS) {
    STF_BATCH_PROLOGUE
    body_update<T>((T*)d.X, d.Xm, (const T*)d.g[parity], d.n, d.p, d.nu,
                   d.alpha != 0.0 ? d.rho : nullptr, d.st, lid_, nb_);
}

#undef STF_BATCH_PROLOGUE
#undef STF_BATCH_ARGS

// Copy every problem's device state into one array (one read-back per check).
__global__ void kb_gather_states(const BDesc* __restrict__ D, int nprob,
                                 DevState* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nprob) out[b] = *D[b].st;
}

// Per-problem hand-over of a batched float32 solve (see launch_batched_switch):
// kSwitchWg workgroups per problem convert, then one thread per problem moves
// the state (a separate launch, so that no workgroup reads the status after
// it has changed).
constexpr int kSwitchWg = 8;
__global__ __launch_bounds__(256) void kb_switch_convert(const BDesc* __restrict__ D32,
                                                         const BDesc* __restrict__ D64,
                                                         int nprob, int parity) {
    const int b = blockIdx.x / kSwitchWg, part = blockIdx.x % kSwitchWg;
    if (b >= nprob) return;
    const DevState* st = D32[b].st;
    if (!(st->done && st->status == STF_SWITCH)) return;
    const float* src = (const float*)D32[b].g[parity ^ 1];
    double* dst = (double*)D64[b].g[parity ^ 1];
    const int64_t np = D32[b].n * (int64_t)D32[b].p;
    for (int64_t e = (int64_t)part * 256 + threadIdx.x; e < np; e += (int64_t)kSwitchWg * 256)
        dst[e] = (double)src[e];
}
__global__ void kb_switch_state(const BDesc* __restrict__ D32, const BDesc* __restrict__ D64,
                                int nprob) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nprob) return;
    DevState* st = D32[b].st;
    if (!(st->done && st->status == STF_SWITCH)) return;
    DevState t = *st;
    t.done = 0;
    t.status = 0;
    *D64[b].st = t;
    st->status = STF_SWITCHED;
}

// =================================================================== host ===

static inline unsigned grid_rows(int64_t n) {
    int64_t g = (n + 3) / 4;
    if (g > 65536) g = 65536;
    return (unsigned)(g < 1 ? 1 : g);
}

void launch_init_state(DevState* st, hipStream_t s) { k_init_state<<<1, 1, 0, s>>>(st); }
void launch_resume_state(DevState* st, hipStream_t s) { k_resume_state<<<1, 1, 0, s>>>(st); }

void launch_rowsq(int dtype, const void* X, int64_t n, int p, double* rho, const DevState* st,
                  hipStream_t s) {
    if (dtype == STF_F64)
        k_rowsq<double><<<grid_rows(n), 256, 0, s>>>((const double*)X, n, p, rho, st);
    else
        k_rowsq<float><<<grid_rows(n), 256, 0, s>>>((const float*)X, n, p, rho, st);
}

void launch_dst_init(const stf_problem* prob, double* dst, hipStream_t s) {
    const int nx = prob->grid[0], ny = prob->grid[1], nz = prob->grid[2];
    double* Sx = dst;
    double* Sy = Sx + (size_t)nx * nx;
    double* Sz = Sy + (size_t)ny * ny;
    double* lx = Sz + (size_t)nz * nz;
    double* ly = lx + nx;
    double* lz = ly + ny;
    k_dst_init<<<(nx * nx + 255) / 256, 256, 0, s>>>(Sx, lx, nx);
    k_dst_init<<<(ny * ny + 255) / 256, 256, 0, s>>>(Sy, ly, ny);
    k_dst_init<<<(nz * nz + 255) / 256, 256, 0, s>>>(Sz, lz, nz);
}

void launch_hartree(const stf_problem* prob, const double* rho, double* phi, double* scr,
                    double* dst, const DevState* st, hipStream_t s) {
    const int64_t n = prob->n;
    if (prob->kind == STF_KIND_STENCIL1D) {
        const int64_t blk = prob->block;
        if (blk > 0 && blk < n) {
            const int64_t nblk = (n + blk - 1) / blk;
            if (blk <= 256)
                k_hartree1d_short<<<(unsigned)((nblk + 255) / 256), 256, 0, s>>>(rho, phi, n,
                                                                                (int)blk, st);
            else
                k_hartree1d_wg<<<(unsigned)nblk, 1024, 0, s>>>(rho, phi, n, blk, st);
            return;
        }
        k_hartree1d<<<1, 1024, 0, s>>>(rho, phi, n, st);
        return;
    }
    const int nx = prob->grid[0], ny = prob->grid[1], nz = prob->grid[2];
    const double* Sx = dst;
    const double* Sy = Sx + (size_t)nx * nx;
    const double* Sz = Sy + (size_t)ny * ny;
    const double* lx = Sz + (size_t)nz * nz;
    const double* ly = lx + nx;
    const double* lz = ly + ny;
    if (nx <= kDstMax && ny <= kDstMax && nz <= kDstMax) {
        // planes in LDS: xy forward, z forward + divide + z inverse (in place:
        // a workgroup reads its whole slab before writing it), xy inverse
        k_dst_xy<<<nz, 1024, 0, s>>>(rho, scr, Sx, Sy, nx, ny, st);
        k_dst_z<<<ny, 1024, 0, s>>>(scr, scr, Sz, lx, ly, lz, nx, ny, nz, st);
        k_dst_xy<<<nz, 1024, 0, s>>>(scr, phi, Sx, Sy, nx, ny, st);
        return;
    }
    const unsigned g = (unsigned)((n + 255) / 256);
    const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    // forward transform along x, y, z; divide by the eigenvalues; transform back
    k_dst_axis<<<g, 256, 0, s>>>(rho, scr, Sx, nx, sx, n, nullptr, nullptr, nullptr, nx, ny, st);
    k_dst_axis<<<g, 256, 0, s>>>(scr, phi, Sy, ny, sy, n, nullptr, nullptr, nullptr, nx, ny, st);
    k_dst_axis<<<g, 256, 0, s>>>(phi, scr, Sz, nz, sz, n, lx, ly, lz, nx, ny, st);
    k_dst_axis<<<g, 256, 0, s>>>(scr, phi, Sx, nx, sx, n, nullptr, nullptr, nullptr, nx, ny, st);
    k_dst_axis<<<g, 256, 0, s>>>(phi, scr, Sy, ny, sy, n, nullptr, nullptr, nullptr, nx, ny, st);
    k_dst_axis<<<g, 256, 0, s>>>(scr, phi, Sz, nz, sz, n, nullptr, nullptr, nullptr, nx, ny, st);
}

void launch_grad(const stf_problem* prob, int dtype, const void* X, void* G, const double* phi,
                 const GradExtra& ex, const DevState* st, hipStream_t s, const double* Xm) {
    const int64_t n = prob->n;
    const int p = prob->p;
    if (prob->kind == STF_KIND_DENSE) {
        const double* gl = ex.glin;
        if (dtype == STF_F32 && ex.dense_prod == 3) {
            // split-bf16 MFMA products: X^T split once per product (the
            // workspace holds it), then the panels straight to LDS
            const int64_t npad = dense_npad(n);
            __bf16* xh = (__bf16*)ex.xsplit;
            __bf16* xl = xh + (size_t)p * npad;
            k_split_xt<<<dim3((unsigned)(npad / 64), (unsigned)((p + 63) / 64)), 256, 0, s>>>(
                (const float*)X, xh, xl, n, p, npad, st);
            const int ncp = (p + kDPN - 1) / kDPN;
            const unsigned nwp = (unsigned)(((n + kDGM - 1) / kDGM) * ncp);
            k_dense_bfp<<<nwp, 512, 0, s>>>((const float*)prob->A, xh, xl, npad, (float*)G, n, p,
                                            ncp, gl, st);
            return;
        }
        if (p > 64) {
            // 128 x 128 tiles staged through LDS (a float32 A is widened
            // exactly in the float64 form)
            const int nbp = (p + 127) / 128;
            const unsigned nwg = (unsigned)(((n + 127) / 128) * nbp);
            if (dtype == STF_F32)
                k_dense_mfma<float, float><<<nwg, 256, 0, s>>>(
                    (const float*)prob->A, (const float*)X, (float*)G, n, p, nbp, gl, st);
            else if (prob->A_dtype == STF_F32)
                k_dense_mfma<double, float><<<nwg, 256, 0, s>>>(
                    (const float*)prob->A, (const double*)X, (double*)G, n, p, nbp, gl, st);
            else
                k_dense_mfma<double, double><<<nwg, 256, 0, s>>>(
                    (const double*)prob->A, (const double*)X, (double*)G, n, p, nbp, gl, st);
            return;
        }
        // narrow p: 32 x 32 tiles fed from global memory
        const int nbp = (p + 31) / 32;
        const unsigned nwg = (unsigned)(((n + 31) / 32) * nbp);
        if (dtype == STF_F32)
            k_dense_grad<float, 1><<<nwg, 256, 0, s>>>((const float*)prob->A, (const float*)X,
                                                       (float*)G, n, p, nbp, gl, st);
        else if (prob->A_dtype == STF_F32)
            k_dense_grad<double, 1, float><<<nwg, 256, 0, s>>>(
                (const float*)prob->A, (const double*)X, (double*)G, n, p, nbp, gl, st);
        else
            k_dense_grad<double, 1><<<nwg, 256, 0, s>>>((const double*)prob->A, (const double*)X,
                                                        (double*)G, n, p, nbp, gl, st);
        return;
    }
    const double* ph = (prob->alpha != 0.0) ? phi : nullptr;
    const int nx = prob->grid[0], ny = prob->grid[1], nz = prob->grid[2];
    const unsigned g = grid_rows(n);
    auto run = [&](auto ti, auto to, auto nd, const void* XP) {
        typedef decltype(ti) TI;
        typedef decltype(to) TO;
        constexpr int ND = decltype(nd)::value;
        // 3D: runs of kRun rows per wave when the rows split into 16-byte
        // vectors (measured on 64^3 x 256: 0.27 against 0.32 ms for the
        // one-wave-per-row form with a float32 G, 0.324 against 0.333 ms with a
        // float64 G; the 1D problems are too short for runs to fill the chip)
        if constexpr (ND == 6) {
            constexpr int kRun = 64;
            if (p % (16 / (int)sizeof(TI)) == 0 && !ex.glin && ex.gamma == 0.0) {
                const int64_t gl = ((n + kRun - 1) / kRun + 3) / 4;
                const unsigned glr = (unsigned)(gl > 65536 ? 65536 : (gl < 1 ? 1 : gl));
                k_grad_line<TI, TO, ND, kRun><<<glr, 256, 0, s>>>(
                    (const TI*)XP, (TO*)G, n, p, nx, ny, nz, prob->v, ph, prob->alpha, st);
                return;
            }
        }
        k_grad_stencil<TI, TO, ND><<<g, 256, 0, s>>>((const TI*)XP, (TO*)G, n, p, nx, ny, nz,
                                                     prob->v, ph, prob->alpha, ex, st);
    };
    typedef std::integral_constant<int, 6> D3;
    typedef std::integral_constant<int, 2> D1;
    if (prob->kind == STF_KIND_STENCIL3D) {
        if (dtype == STF_F64)
            run(0.0, 0.0, D3(), X);
        else if (Xm)
            // float32 G of the float64 master iterate, stencil evaluated in float64
            run(0.0, 0.0f, D3(), Xm);
        else
            run(0.0f, 0.0f, D3(), X);
    } else {
        if (dtype == STF_F64)
            run(0.0, 0.0, D1(), X);
        else if (Xm)
            run(0.0, 0.0f, D1(), Xm);
        else
            run(0.0f, 0.0f, D1(), X);
    }
}

template <typename T>
static void gram_dispatch(const GramPlan& gp, const T* X, const T* G, int64_t n, int p,
                          double* part, const DevState* st, hipStream_t s, int n_tiles,
                          int wup) {
    const unsigned nwg = (unsigned)(n_tiles * gp.nchunks);
    switch (gp.wm) {
        case 1:
            k_gram<T, 1><<<nwg, 256, 0, s>>>(X, G, n, p, gp.nb, gp.n_s_tiles, n_tiles, wup, gp.chunk,
                                              part, st);
            break;
        case 2:
            k_gram<T, 2><<<nwg, 256, 0, s>>>(X, G, n, p, gp.nb, gp.n_s_tiles, n_tiles, wup, gp.chunk,
                                              part, st);
            break;
        default:
            // float64: LDS-staged with prefetch; float32: direct fragment loads measured faster
            if (sizeof(T) == 8)
                k_gram_lds<T><<<nwg, 256, 0, s>>>(X, G, n, p, gp.nb, gp.n_s_tiles, n_tiles,
                                                   wup, gp.chunk, part, st);
            else
                k_gram<T, 4><<<nwg, 256, 0, s>>>(X, G, n, p, gp.nb, gp.n_s_tiles, n_tiles,
                                                  wup, gp.chunk, part, st);
            break;
    }
}

void launch_gram(int dtype, int precision, const GramPlan& gp, const void* X, const void* G,
                 int64_t n, int p, double* part, double* S, double* W, const DevState* st,
                 hipStream_t s, hipEvent_t after_main, bool w_sym, double* colsq) {
    // tiles: the upper blocks of S (when S is wanted) followed by the blocks of W
    // (the upper ones only when W is known to be symmetric)
    const int nst = S ? gp.n_s_tiles : 0;
    const int wup = (W && w_sym) ? 1 : 0;
    const int n_tiles = nst + (W ? (wup ? gp.n_s_tiles : gp.nb * gp.nb) : 0);
    if (n_tiles == 0) return;
    GramPlan g2 = gp;
    g2.n_s_tiles = nst;
    bool fpart = false;  // float32 chunk partials (the LDS split-bf16 pass)
    if (dtype == STF_F32 && precision == STF_PREC_MIXED) {
        const unsigned nwg = (unsigned)(n_tiles * gp.nchunks);
        const float* x = (const float*)X;
        const float* gg = (const float*)G;
        if (gp.wm == 1)
            k_gram_bf3<1><<<nwg, 256, 0, s>>>(x, gg, n, p, gp.nb, nst, n_tiles, wup, gp.chunk,
                                              part, st);
        else if (gp.wm == 2)
            k_gram_bf3<2><<<nwg, 256, 0, s>>>(x, gg, n, p, gp.nb, nst, n_tiles, wup, gp.chunk,
                                              part, st);
        else {
            k_gram_bf3_lds<<<nwg, 256, 0, s>>>(x, gg, n, p, gp.nb, nst, n_tiles, wup, gp.chunk,
                                               (float*)part, st, colsq);
            fpart = true;
        }
    } else if (dtype == STF_F64) {
        if (colsq && gp.wm == 4)
            k_gram_lds<double><<<(unsigned)(n_tiles * gp.nchunks), 256, 0, s>>>(
                (const double*)X, (const double*)G, n, p, gp.nb, nst, n_tiles, wup, gp.chunk,
                part, st, colsq);
        else
            gram_dispatch<double>(g2, (const double*)X, (const double*)G, n, p, part, st, s,
                                  n_tiles, wup);
    } else {
        gram_dispatch<float>(g2, (const float*)X, (const float*)G, n, p, part, st, s, n_tiles,
                             wup);
    }
    if (after_main) (void)hipEventRecord(after_main, s);
    const int64_t tot = (int64_t)n_tiles * gp.bt * gp.bt;
    if (fpart)
        k_gram_reduce<float><<<(unsigned)((tot + 63) / 64), 256, 0, s>>>(
            (const float*)part, gp.nchunks, n_tiles, gp.bt, gp.nb, nst, wup, p, S, W, st);
    else
        k_gram_reduce<double><<<(unsigned)((tot + 63) / 64), 256, 0, s>>>(
            part, gp.nchunks, n_tiles, gp.bt, gp.nb, nst, wup, p, S, W, st);
}

void launch_stage1(const DevParams* prm, const double* S, const double* W, double* Psi,
                   double* ML, double* Bm, double* feas_part, int p, DevState* st,
                   hipStream_t s, double* lam2) {
    k_stage1<<<p, 256, 0, s>>>(prm, S, W, Psi, ML, Bm, feas_part, p, st, lam2);
}

int kkt_partials(int p) {
    if (p >= kPPWide) {
        const int t = (p + kCB - 1) / kCB;
        return t * t * t;
    }
    const int t = (p + 15) / 16;
    return t * t;
}

void launch_kkt_products(const double* S, const double* ML, const double* Bm, const double* W,
                         double* part, int p, DevState* st, hipStream_t s) {
    if (p >= kPPWide) {
        const int t = (p + kCB - 1) / kCB;
        k_pp_kkt64<<<dim3(t, t, t), 1024, 0, s>>>(S, ML, Bm, W, part, p, st);
        return;
    }
    dim3 grid((p + 15) / 16, (p + 15) / 16);
    k_pp_gemm2<<<grid, 256, 0, s>>>(S, ML, Bm, W, part, p, st);
}

void launch_residual(int dtype, int precision, const ResPlan& rp, const void* X, void* G,
                     const void* Gprev, const double* ML, const double* Psi, const double* nu,
                     int64_t n, int p, double* part_col, double* part_scal,
                     const DevParams* prm, DevState* st, int mode, void* mix, hipStream_t s,
                     hipEvent_t before_main, const void* Xprev) {
    const unsigned nwg = (unsigned)(rp.nrb * rp.ncb);
    auto mark = [&]() {
        if (before_main) (void)hipEventRecord(before_main, s);
    };
    if (dtype == STF_F32 && precision == STF_PREC_MIXED && mode == RES_ITERATE) {
        const int prow = rp.ncb * 64, pk = (p + 31) / 32 * 32;
        __bf16* MS = (__bf16*)mix;
        const unsigned gs = (unsigned)(((size_t)prow * pk + 255) / 256);
        k_split3_t<<<gs, 256, 0, s>>>(ML, MS, p, prow, pk, st);
        mark();
        if (rp.tile == 256) {
            // M_L slice resident in LDS (plans of this shape only exist for pk <= 384)
            if (pk <= 128)
                k_residual_bf6_lds<128, kMixRW><<<nwg, 64 * (256 / kMixRW), 0, s>>>(
                    (const float*)X, (float*)G, (const float*)Gprev, MS, prow, pk, nu, n, p,
                    rp.nrb, rp.ncb, rp.nrt, part_col, part_scal, prm, st);
            else if (pk <= 256)
                k_residual_bf6_lds<256, kMixRW><<<nwg, 64 * (256 / kMixRW), 0, s>>>(
                    (const float*)X, (float*)G, (const float*)Gprev, MS, prow, pk, nu, n, p,
                    rp.nrb, rp.ncb, rp.nrt, part_col, part_scal, prm, st);
            else
                k_residual_bf6_lds<384, kMixRW><<<nwg, 64 * (256 / kMixRW), 0, s>>>(
                    (const float*)X, (float*)G, (const float*)Gprev, MS, prow, pk, nu, n, p,
                    rp.nrb, rp.ncb, rp.nrt, part_col, part_scal, prm, st);
            return;
        }
        // the stop test comes from the p x p identity: no product with Psi
        k_residual_bf6<false><<<nwg, 256, 0, s>>>(
            (const float*)X, (float*)G, (const float*)Gprev, MS, nullptr, prow, pk, nu, n, p, rp.nrb,
            rp.ncb, rp.nrt, part_col, part_scal, prm, st, mode);
        return;
    }
    // iterations evaluate the stop test by the p x p identity (no second product)
    const bool kkt_prod = (mode == RES_KKT_ONLY);
    mark();
    if (Xprev) {
        // MOptQR (float64 only): the BB pair from the stored previous iterate
        k_residual<double, double, false, false, 2, true><<<nwg, 256, 0, s>>>(
            (const double*)X, (double*)G, (const double*)Gprev, ML, Psi, nu, n, p, rp.nrb,
            rp.ncb, rp.nrt, part_col, part_scal, prm, st, mode, (const double*)Xprev);
    } else if (dtype == STF_F64) {
        if (kkt_prod)
            k_residual<double, double, false, true, 2><<<nwg, 256, 0, s>>>(
                (const double*)X, (double*)G, (const double*)Gprev, ML, Psi, nu, n, p, rp.nrb,
                rp.ncb, rp.nrt, part_col, part_scal, prm, st, mode);
        else
            k_residual<double, double, false, false, 2><<<nwg, 256, 0, s>>>(
                (const double*)X, (double*)G, (const double*)Gprev, ML, Psi, nu, n, p, rp.nrb,
                rp.ncb, rp.nrt, part_col, part_scal, prm, st, mode);
    } else if (kkt_prod) {
        k_residual<float, float, false, true, 2><<<nwg, 256, 0, s>>>(
            (const float*)X, (float*)G, (const float*)Gprev, ML, Psi, nu, n, p, rp.nrb, rp.ncb,
            rp.nrt, part_col, part_scal, prm, st, mode);
    } else {
        k_residual<float, float, false, false, 2><<<nwg, 256, 0, s>>>(
            (const float*)X, (float*)G, (const float*)Gprev, ML, Psi, nu, n, p, rp.nrb, rp.ncb,
            rp.nrt, part_col, part_scal, prm, st, mode);
    }
}

int gram_colsq_slots(int dtype) { return dtype == STF_F64 ? 4 : 2; }

int fused_rho_slots(int dtype, const ResPlan& rp) {
    return dtype == STF_F64 ? rp.ncb * 2 : rp.ncb;
}

void launch_fused_pre(const DevParams* prm, const double* S, const double* W, const double* ML,
                      double* SM, const double* colsq, int nchunks, int nsl, double* nu_cur,
                      int p, DevState* st, hipStream_t s) {
    const unsigned t = (unsigned)((p + kCB - 1) / kCB);
    k_pp_mm64<<<dim3(t, t), 1024, 0, s>>>(S, ML, SM, p, st);
    k_fused_pre<<<(unsigned)((p + 63) / 64), 256, 0, s>>>(prm, S, W, ML, SM, colsq, nchunks, nsl,
                                                          nu_cur, p, st);
}

void launch_residual_fused(int dtype, const ResPlan& rp, const void* X, void* Xn, void* G,
                           const void* Gprev, const double* ML, const double* nu,
                           const double* nu_cur, int64_t n, int p, double* part_col,
                           double* part_scal, double* rho_part, const DevParams* prm,
                           DevState* st, void* mix, hipStream_t s, hipEvent_t before_main) {
    const unsigned nwg = (unsigned)(rp.nrb * rp.ncb);
    if (dtype == STF_F64) {
        if (before_main) (void)hipEventRecord(before_main, s);
        k_residual<double, double, false, false, 2, false, true><<<nwg, 256, 0, s>>>(
            (const double*)X, (double*)G, (const double*)Gprev, ML, nullptr, nu, n, p, rp.nrb,
            rp.ncb, rp.nrt, part_col, part_scal, prm, st, RES_ITERATE, nullptr, (double*)Xn,
            nu_cur, rho_part);
        return;
    }
    // float32 iterate, split-bf16 products with the M_L slice resident in LDS
    const int prow = rp.ncb * 64, pk = (p + 31) / 32 * 32;
    __bf16* MS = (__bf16*)mix;
    const unsigned gs = (unsigned)(((size_t)prow * pk + 255) / 256);
    k_split3_t<<<gs, 256, 0, s>>>(ML, MS, p, prow, pk, st);
    if (before_main) (void)hipEventRecord(before_main, s);
    const float* x = (const float*)X;
    float* g = (float*)G;
    const float* gp = (const float*)Gprev;
    float* xn = (float*)Xn;
    if (pk <= 128)
        k_residual_bf6_lds<128, kMixRW, true><<<nwg, 64 * (256 / kMixRW), 0, s>>>(
            x, g, gp, MS, prow, pk, nu, n, p, rp.nrb, rp.ncb, rp.nrt, part_col, part_scal, prm,
            st, xn, nu_cur, rho_part);
    else if (pk <= 256)
        k_residual_bf6_lds<256, kMixRW, true><<<nwg, 64 * (256 / kMixRW), 0, s>>>(
            x, g, gp, MS, prow, pk, nu, n, p, rp.nrb, rp.ncb, rp.nrt, part_col, part_scal, prm,
            st, xn, nu_cur, rho_part);
    else
        k_residual_bf6_lds<384, kMixRW, true><<<nwg, 64 * (256 / kMixRW), 0, s>>>(
            x, g, gp, MS, prow, pk, nu, n, p, rp.nrb, rp.ncb, rp.nrt, part_col, part_scal, prm,
            st, xn, nu_cur, rho_part);
}

void launch_rho_reduce(const double* part, int nslots, int64_t n, double* rho,
                       const DevState* st, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    g = std::min<int64_t>(g, 4096);
    k_rho_reduce<<<(unsigned)g, 256, 0, s>>>(part, nslots, n, rho, st);
}

void launch_stage2(const DevParams* prm, const ResPlan& rp, const double* part_col,
                   const double* part_scal, const double* S, const double* pp_part,
                   const double* feas_part, double* colpart, double* nu, int p, DevState* st,
                   hipStream_t s, const double* nu_cur) {
    const int ng = col_groups(rp.nrb);
    k_colreduce<<<dim3((2 * p + 63) / 64, ng), 256, 0, s>>>(part_col, rp.nrb, p, colpart, st);
    k_stage2<<<1, 1024, 0, s>>>(prm, part_scal, rp.nrb * rp.ncb, S, pp_part, kkt_partials(p),
                                feas_part, colpart, ng, nu, p, st, nu_cur);
}

void launch_update(int dtype, void* X, const void* GL, int64_t n, int p, const double* nu,
                   double* rho, const DevState* st, hipStream_t s, double* Xm) {
    if (dtype == STF_F32 && !Xm && (p % 4) == 0) {
        // float32 rows without a master: 4-element vectors per lane, kUR rows
        // per wave (0.218 -> 0.147 ms on 64^3 x 256; the same form of the
        // float64 update measured 0.274 against 0.255 ms for the row-per-wave one)
        int64_t g = (n + 4 * kUR - 1) / (4 * kUR);
        g = std::min<int64_t>(g, 8192);
        k_update_v<float><<<(unsigned)g, 256, 0, s>>>((float*)X, (const float*)GL, n, p, nu,
                                                      rho, st);
        return;
    }
    if (dtype == STF_F64)
        k_update<double><<<grid_rows(n), 256, 0, s>>>((double*)X, nullptr, (const double*)GL, n,
                                                      p, nu, rho, st);
    else
        k_update<float><<<grid_rows(n), 256, 0, s>>>((float*)X, Xm, (const float*)GL, n, p, nu,
                                                     rho, st);
}

void launch_apply(int dtype, const ResPlan& rp, const void* X, void* Out, const double* M,
                  int64_t n, int p, hipStream_t s, int subtract, const DevState* st) {
    const unsigned nwg = (unsigned)(rp.nrb * rp.ncb);
    if (dtype == STF_F64)
        k_residual<double, double, true, false, 2><<<nwg, 256, 0, s>>>(
            (const double*)X, (double*)Out, nullptr, M, nullptr, nullptr, n, p, rp.nrb, rp.ncb,
            rp.nrt, nullptr, nullptr, nullptr, st, subtract);
    else
        k_residual<float, float, true, false, 2><<<nwg, 256, 0, s>>>(
            (const float*)X, (float*)Out, nullptr, M, nullptr, nullptr, n, p, rp.nrb, rp.ncb,
            rp.nrt, nullptr, nullptr, nullptr, st, subtract);
}

void launch_chol_inv(const double* S, double* R, double* Rinv, double* work, int p,
                     DevState* st, hipStream_t s, int stop_on_fail) {
    const int nb = (p + kCB - 1) / kCB;
    const size_t p2 = (size_t)p * p;
    unsigned gi = (unsigned)((p2 + 255) / 256);
    if (gi > 4096) gi = 4096;
    k_chol_init<<<gi, 256, 0, s>>>(S, work, R, Rinv, p, st);
    for (int j = 0; j < nb; ++j) {
        k_chol_diag<<<1, 1024, 0, s>>>(work, R, Rinv, p, j, st, stop_on_fail);
        const int t = nb - j - 1;
        if (t > 0) k_chol_step<<<(unsigned)(t * (t + 1) / 2), 1024, 0, s>>>(work, R, Rinv, p, j, nb, st);
    }
    for (int so = 1; so < nb; ++so)
        k_chol_inv_off<<<(unsigned)(nb - so), 1024, 0, s>>>(R, Rinv, p, so, st);
}

void launch_vform(const double* X, const double* D, double* V, int64_t n, int p,
                  const DevState* st, hipStream_t s) {
    const size_t np = (size_t)n * p;
    unsigned g = (unsigned)((np + 255) / 256);
    if (g > 8192) g = 8192;
    k_vform<<<g, 256, 0, s>>>(X, D, V, np, st);
}

void launch_convert(int to_dtype, const void* in, int in_dtype, void* out, size_t count,
                    hipStream_t s) {
    unsigned g = (unsigned)((count + 255) / 256);
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    if (in_dtype == STF_F32 && to_dtype == STF_F64)
        k_convert<float, double><<<g, 256, 0, s>>>((const float*)in, (double*)out, count);
    else if (in_dtype == STF_F64 && to_dtype == STF_F32)
        k_convert<double, float><<<g, 256, 0, s>>>((const double*)in, (float*)out, count);
    else if (in_dtype == STF_F64)
        k_convert<double, double><<<g, 256, 0, s>>>((const double*)in, (double*)out, count);
    else
        k_convert<float, float><<<g, 256, 0, s>>>((const float*)in, (float*)out, count);
}

void launch_eval_finish(const stf_problem* prob, const double* X, const double* G,
                        const double* rho, const double* phi, const double* feas_part,
                        int64_t n, int p, double* dots, const double* part_scal, int nps,
                        DevState* st, hipStream_t s) {
    const int nd = 512;
    const bool hart = prob->kind != STF_KIND_DENSE && prob->alpha != 0.0;
    const bool exch = prob->kind != STF_KIND_DENSE && prob->gamma != 0.0;
    k_dots<<<nd, 256, 0, s>>>(X, G, (size_t)n * p, (hart || exch) ? rho : nullptr,
                              hart ? phi : nullptr, n, prob->Glin, exch ? 1 : 0, dots);
    k_eval_finish<<<1, 256, 0, s>>>(dots, nd, part_scal, nps, feas_part, p,
                                    hart ? prob->alpha : 0.0,
                                    exch ? prob->gamma : 0.0, st);
}


void launch_gather_states(const BDesc* d, int nprob, DevState* out, hipStream_t s) {
    kb_gather_states<<<(nprob + 63) / 64, 64, 0, s>>>(d, nprob, out);
}

void launch_batched_switch(const BDesc* d32, const BDesc* d64, int nprob, int parity,
                           hipStream_t s) {
    kb_switch_convert<<<(unsigned)nprob * kSwitchWg, 256, 0, s>>>(d32, d64, nprob, parity);
    kb_switch_state<<<(nprob + 63) / 64, 64, 0, s>>>(d32, d64, nprob);
}

// One grouped launch of a batched stage; variant_key selects the template of
// the stages that have several (Gram: 1/2/4 = MFMA tiles per wave dimension;
// mixed residual: PKMAX).  Grid size is grp.total workgroups.
void launch_batched(int stage, int dtype, int precision, int variant_key, const BDesc* d,
                    const BGroup& grp, int parity, hipStream_t s) {
    if (grp.cnt <= 0 || grp.total <= 0) return;
    const unsigned g = (unsigned)grp.total;
    const int32_t* L = grp.list;
    const int32_t* O = grp.off;
    const int c = grp.cnt;
    const bool f64 = dtype == STF_F64;
    const bool mixed = (dtype == STF_F32) && (precision == STF_PREC_MIXED);
    switch (stage) {
        case BS_HARTREE:
            kb_hartree1d<<<g, 1024, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_ROWSQ:
            // the float32 forms keep their float64 master in Xm: rows of squares in float64
            kb_rowsq<double><<<g, 256, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_GRAD:
            if (f64)
                kb_grad<double, double><<<g, 256, 0, s>>>(d, L, O, c, parity);
            else
                kb_grad<double, float><<<g, 256, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_GRAM:
            if (mixed) {
                if (variant_key == 1)
                    kb_gram_bf3<1><<<g, 256, 0, s>>>(d, L, O, c, parity);
                else if (variant_key == 2)
                    kb_gram_bf3<2><<<g, 256, 0, s>>>(d, L, O, c, parity);
                else
                    kb_gram_bf3_lds<<<g, 256, 0, s>>>(d, L, O, c, parity);
            } else if (f64) {
                if (variant_key == 1)
                    kb_gram<double, 1><<<g, 256, 0, s>>>(d, L, O, c, parity);
                else if (variant_key == 2)
                    kb_gram<double, 2><<<g, 256, 0, s>>>(d, L, O, c, parity);
                else
                    kb_gram_lds64<<<g, 256, 0, s>>>(d, L, O, c, parity);
            } else {
                if (variant_key == 1)
                    kb_gram<float, 1><<<g, 256, 0, s>>>(d, L, O, c, parity);
                else if (variant_key == 2)
                    kb_gram<float, 2><<<g, 256, 0, s>>>(d, L, O, c, parity);
                else
                    kb_gram<float, 4><<<g, 256, 0, s>>>(d, L, O, c, parity);
            }
            break;
        case BS_REDUCE:
            kb_gram_reduce<<<g, 256, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_STAGE1:
            kb_stage1<<<g, 256, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_PPGEMM:
            kb_pp_gemm2<<<g, 256, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_SPLIT:
            kb_split3<<<g, 256, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_RESID:
            if (mixed) {
                if (variant_key <= 128)
                    kb_residual_bf6_lds<128><<<g, 64 * (256 / kMixRW), 0, s>>>(d, L, O, c, parity);
                else if (variant_key <= 256)
                    kb_residual_bf6_lds<256><<<g, 64 * (256 / kMixRW), 0, s>>>(d, L, O, c, parity);
                else
                    kb_residual_bf6_lds<384><<<g, 64 * (256 / kMixRW), 0, s>>>(d, L, O, c, parity);
            } else if (f64) {
                kb_residual<double><<<g, 256, 0, s>>>(d, L, O, c, parity);
            } else {
                kb_residual<float><<<g, 256, 0, s>>>(d, L, O, c, parity);
            }
            break;
        case BS_COLRED:
            kb_colreduce<<<g, 256, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_STAGE2:
            kb_stage2<<<g, 1024, 0, s>>>(d, L, O, c, parity);
            break;
        case BS_UPDATE:
            if (f64)
                kb_update<double><<<g, 256, 0, s>>>(d, L, O, c, parity);
            else
                kb_update<float><<<g, 256, 0, s>>>(d, L, O, c, parity);
            break;
        default:
            break;
    }
}

}  // namespace stf
