// Sparse products on the assembled CSR matrices: y = alpha A x + beta B x for
// two value arrays on one pattern (K and M share theirs). Used for the
// derivative of the quadratic form with respect to u, 2 (K + M) u, and by the
// conjugate-gradient solve of the eddy-current example.
//
// One row per group of G lanes: lane j of a group takes the row's entries j,
// j + G, j + 2G, ... in order and the group adds its lanes by a fixed xor
// tree, so every row is summed in the same order on every call
// (deterministic). The rows of these matrices are short (7 entries in 2D, 13
// to 27 for 3D Nedelec), so G = 8: eight rows per wavefront, and the loads of
// a group are adjacent in the value and column arrays.
#include <algorithm>
#include <cmath>
#include <utility>

#include "fem_internal.h"

namespace fem {

constexpr int MV_G = 8;
constexpr int MV_BLOCK = 256;

template <bool TWO>
__global__ __launch_bounds__(MV_BLOCK) void k_csr_matvec(int64_t n_rows, const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colind,
                                                         const double* __restrict__ A,
                                                         const double* __restrict__ B, double alpha,
                                                         double beta, const double* __restrict__ x,
                                                         double* __restrict__ y) {
    const int64_t t = (int64_t)blockIdx.x * MV_BLOCK + threadIdx.x;
    const int64_t r = t / MV_G;
    const int j = (int)(t % MV_G);
    double sa = 0.0, sb = 0.0;
    if (r < n_rows) {
        const int64_t p1 = rowptr[r + 1];
        for (int64_t p = rowptr[r] + j; p < p1; p += MV_G) {
            const double xv = x[colind[p]];
            sa += A[p] * xv;
            if constexpr (TWO) sb += B[p] * xv;
        }
    }
#pragma unroll
    for (int m = 1; m < MV_G; m <<= 1) {
        sa += __shfl_xor(sa, m, MV_G);
        if constexpr (TWO) sb += __shfl_xor(sb, m, MV_G);
    }
    if (r < n_rows && j == 0) y[r] = TWO ? alpha * sa + beta * sb : alpha * sa;
}

fem_status launch_csr_matvec(int64_t n_rows, const int64_t* rowptr, const int32_t* colind, const double* A,
                             const double* B, double alpha, double beta, const double* x, double* y,
                             hipStream_t s) {
    if (n_rows <= 0) return FEM_OK;
    const int64_t threads = n_rows * MV_G;
    const unsigned grid = (unsigned)((threads + MV_BLOCK - 1) / MV_BLOCK);
    if (B)
        hipLaunchKernelGGL(k_csr_matvec<true>, dim3(grid), dim3(MV_BLOCK), 0, s, n_rows, rowptr, colind, A, B,
                           alpha, beta, x, y);
    else
        hipLaunchKernelGGL(k_csr_matvec<false>, dim3(grid), dim3(MV_BLOCK), 0, s, n_rows, rowptr, colind, A,
                           nullptr, alpha, 0.0, x, y);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

}  // namespace fem

extern "C" {

fem_status fem_csr_matvec(int64_t n_rows, const int64_t* rowptr, const int32_t* colind, const double* A,
                          const double* B, double alpha, double beta, const double* x, double* y,
                          void* stream) {
    if (n_rows < 0) return fem::fail(FEM_EINVAL, "fem_csr_matvec: n_rows < 0");
    if (n_rows > 0 && (!rowptr || !colind || !A || !x || !y))
        return fem::fail(FEM_EINVAL, "fem_csr_matvec: NULL argument");
    if (x == y) return fem::fail(FEM_EINVAL, "fem_csr_matvec: x and y must not be the same buffer");
    return fem::launch_csr_matvec(n_rows, rowptr, colind, A, B, alpha, beta, x, y,
                                  reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

// ===========================================================================
// Conjugate gradients with the Jacobi preconditioner for
// (ca A + cb B) x = rhs, A and B on one CSR pattern (for example K and M of the
// eddy-current problem of Section 4.2, whose matrix K + M is symmetric
// positive definite).
//
// Each iteration is two kernels over a persistent grid of CG_GRID workgroups
// (workgroup g takes row chunks g, g + CG_GRID, ...; a thread sums its
// contributions in chunk order and the workgroup by a fixed tree, so every
// dot product is computed in one fixed order: deterministic):
//   1. q = A' p_new with p_new = z + beta p_old formed on the fly (the update
//      of p fused into the product; p_old and p_new are separate buffers),
//      p_new written, and the dot p_new . q. The last workgroup to finish
//      forms alpha = rz / (p . q).
//   2. x += alpha p, r -= alpha q, z = r / diag(A'), and the dots r . z, r . r.
//      The last workgroup forms beta = rz_new / rz and keeps r . r.
// The "last workgroup" takes a ticket from a device counter after its partial
// is written and fenced; it reads the partials in index order and resets the
// counter. The host reads r . r (the recursive residual) every CG_CHECK
// iterations to test convergence, and the true residual b - A' x of the result
// is formed once at the end. The two differ by the rounding of the recursive
// updates and of A' x itself: for the eddy-current matrices, whose stiffness
// entries grow like h^-2 while A' x stays of the size of b, the true relative
// residual levels off well above the recursive one (restarting from the true
// residual was tried: it tripled the iterations without lowering it).
// ===========================================================================
namespace fem {

constexpr int CG_BLOCK = 256;
constexpr int CG_G = 8;                      // lanes per row in the products
constexpr int CG_ROWS = CG_BLOCK / CG_G;     // rows per chunk of the products
constexpr int CG_GRID = 2048;
constexpr int CG_CHECK = 16;

enum { S_ALPHA = 0, S_BETA, S_RZ, S_RR, S_BB, S_PQ, S_FLAG, S_N };

struct CgArgs {
    int64_t n;
    const int64_t* rowptr;
    const int32_t* colind;
    const double* A;
    const double* B;
    double ca, cb;
    const double* rhs;
    double* x;
    double* r;
    double* z;
    double* q;
    double* dinv;
    double* part;      // [3][CG_GRID] workgroup partials
    double* scal;      // [S_N] scalars
    unsigned* ticket;
};

__device__ __forceinline__ double cg_block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = CG_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// Writes this workgroup's NV partials, takes a ticket; returns true in the last
// workgroup, which then sees every partial.
template <int NV>
__device__ __forceinline__ bool cg_partials(const CgArgs& C, const double (&v)[NV], double* red) {
    __shared__ bool s_last;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = cg_block_sum(v[k], red);
        if (threadIdx.x == 0) C.part[k * CG_GRID + blockIdx.x] = s;
    }
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(C.ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last;
}

// Sum of partial row k in index order (last workgroup only; all threads).
__device__ __forceinline__ double cg_total(const CgArgs& C, int k, double* red) {
    double v = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += CG_BLOCK) v += C.part[k * CG_GRID + i];
    return cg_block_sum(v, red);
}

// Row i of A' x (G lanes per row: lane j takes entries j, j + G, ...; then a
// fixed xor tree); x_j = z_j + beta p_j when P is given.
template <bool FUSED>
__device__ __forceinline__ double cg_row(const CgArgs& C, int64_t i, int j, const double* x, const double* p,
                                         double beta) {
    double sa = 0.0, sb = 0.0;
    if (i < C.n) {
        const int64_t e1 = C.rowptr[i + 1];
        for (int64_t e = C.rowptr[i] + j; e < e1; e += CG_G) {
            const int32_t c = C.colind[e];
            const double xv = FUSED ? fma(beta, p[c], x[c]) : x[c];
            sa += C.A[e] * xv;
            if (C.B) sb += C.B[e] * xv;
        }
    }
    double s = C.ca * sa + C.cb * sb;
#pragma unroll
    for (int m = 1; m < CG_G; m <<= 1) s += __shfl_xor(s, m, CG_G);
    return s;
}

__global__ __launch_bounds__(CG_BLOCK) void k_cg_diag(const CgArgs C) {
    const int64_t i = (int64_t)blockIdx.x * CG_BLOCK + threadIdx.x;
    if (i >= C.n) return;
    double d = 0.0;
    for (int64_t e = C.rowptr[i]; e < C.rowptr[i + 1]; ++e)
        if (C.colind[e] == (int32_t)i) d = C.ca * C.A[e] + (C.B ? C.cb * C.B[e] : 0.0);
    if (!(d > 0.0) || !isfinite(d)) {
        atomicOr(reinterpret_cast<int*>(C.scal + S_FLAG), 1);
        d = 1.0;
    }
    C.dinv[i] = 1.0 / d;
}

// r = rhs - A' x, z = r / d, p_old = 0; dots r . z, r . r, rhs . rhs.
// With FINAL only r . r is formed (true residual of the result).
template <bool FINAL>
__global__ __launch_bounds__(CG_BLOCK) void k_cg_residual(const CgArgs C, double* p_old) {
    __shared__ double red[CG_BLOCK];
    const int lr = threadIdx.x / CG_G, j = threadIdx.x % CG_G;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    const int64_t chunks = (C.n + CG_ROWS - 1) / CG_ROWS;
    for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int64_t i = ch * CG_ROWS + lr;
        const double ax = cg_row<false>(C, i, j, C.x, nullptr, 0.0);
        if (i < C.n && j == 0) {
            const double ri = C.rhs[i] - ax;
            rr += ri * ri;
            if (!FINAL) {
                const double zi = C.dinv[i] * ri;
                C.r[i] = ri;
                C.z[i] = zi;
                p_old[i] = 0.0;
                rz += ri * zi;
                bb += C.rhs[i] * C.rhs[i];
            }
        }
    }
    const double v[3] = {rz, rr, bb};
    if (cg_partials<3>(C, v, red)) {
        const double trz = cg_total(C, 0, red);
        const double trr = cg_total(C, 1, red);
        const double tbb = cg_total(C, 2, red);
        if (threadIdx.x == 0) {
            C.scal[S_RR] = trr;
            if (!FINAL) {
                C.scal[S_RZ] = trz;
                C.scal[S_BB] = tbb;
                C.scal[S_BETA] = 0.0;
            }
            *C.ticket = 0u;
        }
    }
}

// q = A' (z + beta p_old), p_new = z + beta p_old, alpha = rz / (p_new . q)
__global__ __launch_bounds__(CG_BLOCK) void k_cg_product(const CgArgs C, const double* p_old, double* p_new) {
    __shared__ double red[CG_BLOCK];
    const int lr = threadIdx.x / CG_G, j = threadIdx.x % CG_G;
    const double beta = C.scal[S_BETA];
    double pq = 0.0;
    const int64_t chunks = (C.n + CG_ROWS - 1) / CG_ROWS;
    for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int64_t i = ch * CG_ROWS + lr;
        const double qi = cg_row<true>(C, i, j, C.z, p_old, beta);
        if (i < C.n && j == 0) {
            const double pi = fma(beta, p_old[i], C.z[i]);
            p_new[i] = pi;
            C.q[i] = qi;
            pq += pi * qi;
        }
    }
    const double v[1] = {pq};
    if (cg_partials<1>(C, v, red)) {
        const double tpq = cg_total(C, 0, red);
        if (threadIdx.x == 0) {
            C.scal[S_PQ] = tpq;
            if (!(tpq > 0.0) || !isfinite(tpq)) {
                C.scal[S_ALPHA] = 0.0;
                atomicOr(reinterpret_cast<int*>(C.scal + S_FLAG), 2);
            } else {
                C.scal[S_ALPHA] = C.scal[S_RZ] / tpq;
            }
            *C.ticket = 0u;
        }
    }
}

// x += alpha p, r -= alpha q, z = r / d; beta = rz_new / rz
__global__ __launch_bounds__(CG_BLOCK) void k_cg_update(const CgArgs C, const double* p) {
    __shared__ double red[CG_BLOCK];
    const double alpha = C.scal[S_ALPHA];
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * CG_BLOCK + threadIdx.x; i < C.n; i += (int64_t)gridDim.x * CG_BLOCK) {
        C.x[i] = fma(alpha, p[i], C.x[i]);
        const double ri = fma(-alpha, C.q[i], C.r[i]);
        const double zi = C.dinv[i] * ri;
        C.r[i] = ri;
        C.z[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
    const double v[2] = {rz, rr};
    if (cg_partials<2>(C, v, red)) {
        const double trz = cg_total(C, 0, red);
        const double trr = cg_total(C, 1, red);
        if (threadIdx.x == 0) {
            const double old = C.scal[S_RZ];
            C.scal[S_BETA] = old != 0.0 ? trz / old : 0.0;
            C.scal[S_RZ] = trz;
            C.scal[S_RR] = trr;
            *C.ticket = 0u;
        }
    }
}

}  // namespace fem

extern "C" {

fem_status fem_cg_solve(int64_t n_rows, const int64_t* rowptr, const int32_t* colind, const double* A,
                        const double* B, double ca, double cb, const double* rhs, double* x, double rtol,
                        int64_t max_iter, void* stream, int64_t* iters, double* rel_resid) {
    using namespace fem;
    if (n_rows <= 0) return fail(FEM_EINVAL, "fem_cg_solve: n_rows must be positive");
    if (!rowptr || !colind || !A || !rhs || !x) return fail(FEM_EINVAL, "fem_cg_solve: NULL argument");
    if (!(rtol >= 0.0) || max_iter < 0) return fail(FEM_EINVAL, "fem_cg_solve: rtol < 0 or max_iter < 0");
    if (x == rhs) return fail(FEM_EINVAL, "fem_cg_solve: x and rhs must not be the same buffer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = n_rows;
    // workspace: r, z, q, p (two), 1/diag, partials, scalars, ticket
    const size_t vec = (size_t)n * sizeof(double);
    const size_t bytes = 6 * vec + 3 * CG_GRID * sizeof(double) + S_N * sizeof(double) + 256;
    char* ws = nullptr;
    FEM_HIP(hipMalloc(reinterpret_cast<void**>(&ws), bytes));
    struct Free {
        char* p;
        ~Free() { (void)hipFree(p); }
    } guard{ws};
    CgArgs C;
    C.n = n;
    C.rowptr = rowptr;
    C.colind = colind;
    C.A = A;
    C.B = B;
    C.ca = ca;
    C.cb = B ? cb : 0.0;
    C.rhs = rhs;
    C.x = x;
    C.r = reinterpret_cast<double*>(ws);
    C.z = C.r + n;
    C.q = C.z + n;
    double* p0 = C.q + n;
    double* p1 = p0 + n;
    C.dinv = p1 + n;
    C.part = C.dinv + n;
    C.scal = C.part + 3 * CG_GRID;
    C.ticket = reinterpret_cast<unsigned*>(C.scal + S_N);
    FEM_HIP(hipMemsetAsync(C.scal, 0, S_N * sizeof(double) + sizeof(unsigned) * 4, s));
    const int64_t chunks = (n + CG_ROWS - 1) / CG_ROWS;
    const unsigned grid_rows = (unsigned)std::min<int64_t>(CG_GRID, chunks);
    const unsigned grid_elem = (unsigned)std::min<int64_t>(CG_GRID, (n + CG_BLOCK - 1) / CG_BLOCK);
    const unsigned grid_diag = (unsigned)((n + CG_BLOCK - 1) / CG_BLOCK);
    hipLaunchKernelGGL(k_cg_diag, dim3(grid_diag), dim3(CG_BLOCK), 0, s, C);
    hipLaunchKernelGGL(k_cg_residual<false>, dim3(grid_rows), dim3(CG_BLOCK), 0, s, C, p0);
    FEM_HIP(hipGetLastError());
    double host[S_N];
    FEM_HIP(hipMemcpyAsync(host, C.scal, sizeof(host), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    const double bb = host[S_BB];
    int flag = (int)reinterpret_cast<const int*>(&host[S_FLAG])[0];
    if (flag & 1) return fail(FEM_EINVAL, "fem_cg_solve: a diagonal entry is not positive");
    double rr = host[S_RR];
    int64_t it = 0;
    const double target = rtol * rtol * bb;
    bool converged = bb == 0.0 || rr <= target;
    while (!converged && it < max_iter) {
        const int64_t steps = std::min<int64_t>(CG_CHECK, max_iter - it);
        for (int64_t k = 0; k < steps; ++k) {
            hipLaunchKernelGGL(k_cg_product, dim3(grid_rows), dim3(CG_BLOCK), 0, s, C, p0, p1);
            hipLaunchKernelGGL(k_cg_update, dim3(grid_elem), dim3(CG_BLOCK), 0, s, C, p1);
            std::swap(p0, p1);
        }
        FEM_HIP(hipGetLastError());
        it += steps;
        FEM_HIP(hipMemcpyAsync(host, C.scal, sizeof(host), hipMemcpyDeviceToHost, s));
        FEM_HIP(hipStreamSynchronize(s));
        rr = host[S_RR];
        flag = (int)reinterpret_cast<const int*>(&host[S_FLAG])[0];
        if (flag & 2) return fail(FEM_EHIP, "fem_cg_solve: breakdown (p . A p <= 0: the matrix is not positive definite)");
        converged = rr <= target || !std::isfinite(rr);
    }
    // true residual of the result
    hipLaunchKernelGGL(k_cg_residual<true>, dim3(grid_rows), dim3(CG_BLOCK), 0, s, C, p0);
    FEM_HIP(hipGetLastError());
    FEM_HIP(hipMemcpyAsync(host, C.scal, sizeof(host), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    if (iters) *iters = it;
    if (rel_resid) *rel_resid = bb > 0.0 ? std::sqrt(host[S_RR] / bb) : 0.0;
    return FEM_OK;
}

}  // extern "C"
