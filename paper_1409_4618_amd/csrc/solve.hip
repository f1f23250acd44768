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
#include <cstdio>
#include <cstdlib>
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
// One iteration is two kernels:
//   1. q = A' p_new with p_new = z + beta p_old formed on the fly (the update
//      of p fused into the product; p_old and p_new are separate buffers),
//      p_new written, and per-workgroup partials of p_new . q;
//   2. x += alpha p, r -= alpha q, z = r / diag(A'), partials of r . z, r . r.
// Neither scalar has a kernel of its own: every workgroup of a kernel adds the
// partials of the kernel before (at most CG_GRID of them, 16 KB) in the same
// fixed order and forms the scalar itself, so all of them hold the same value
// (beta = rz_k / rz_(k-1) in the product, alpha = rz_k / (p . q) in the
// update). rz_k, which the update needs after the product's partials of it
// are gone, is kept by workgroup 0 of the product in one of two slots chosen
// by the parity of the iteration (the other slot, rz_(k-1), is being read by
// the product's other workgroups). A workgroup takes row chunks g, g + grid,
// ...; a thread adds its contributions in chunk order and the workgroup by a
// fixed tree (wavefront butterflies, then the four wavefront sums): every dot
// product has one fixed order for a given n (deterministic). No atomics on
// the sums.
// A row takes G lanes, G = 4, 8 or 16 by the mean row length (2D Nedelec rows
// have 5 entries, 3D Nedelec rows 13 to 27). The CG_CHECK iterations between
// two convergence tests are captured once in a HIP graph and replayed.
//
// The host reads r . r (the recursive residual) every CG_CHECK iterations to
// test convergence, and the true residual b - A' x of the result is formed
// once at the end. The two differ by the rounding of the recursive updates and
// of A' x itself: for the eddy-current matrices, whose stiffness entries grow
// like h^-2 while A' x stays of the size of b, the true relative residual levels
// off well above the recursive one (restarting from the true residual was
// tried: it tripled the iterations without lowering it).
// ===========================================================================
namespace fem {

constexpr int CG_BLOCK = 256;
// Most workgroups of a grid, and so of partials per dot product: eight per CU
// on 256 CUs, about what is resident at once. Every workgroup of the next
// kernel adds all of them (16 KB), so more would cost more in those sums than
// it gains in loads in flight: at 787,456 rows an iteration took 62 us with the
// scalars in kernels of their own, and 51, 44, 56 and 55 us with 1024, 2048,
// 3072 and 4096 workgroups (512: 67 us).
constexpr int CG_GRID = 2048;
constexpr int CG_CHECK = 16;                 // iterations per convergence test (even: p buffers alternate)

enum { S_RZ0 = 0, S_RZ1, S_RR, S_BB, S_FLAG, S_N };

struct CgArgs {
    int64_t n;
    int64_t nnz;  // for the checked build's bounds checks
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
    double* part;      // [3][CG_GRID] partials of the residual and update kernels (r.z, r.r, b.b)
    double* part_pq;   // [CG_GRID] partials of the product kernel (p.q)
    double* scal;      // [S_N] scalars
};

// Sum over the workgroup, the same value in every thread: a butterfly within
// each wavefront (lane 0's order), then the four wavefront sums in a fixed
// order. red: 4 doubles of LDS.
__device__ __forceinline__ double cg_block_sum(double v, double* red) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

template <int NV>
__device__ __forceinline__ void cg_partials(double* part, const double (&v)[NV], double* red) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = cg_block_sum(v[k], red);
        if (threadIdx.x == 0) part[k * CG_GRID + blockIdx.x] = s;
    }
}

// Sum of the first nb partials of one row in index order per thread, then the
// fixed tree: every workgroup gets the same value.
__device__ __forceinline__ double cg_total(const double* part, int nb, double* red) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += CG_BLOCK) v += part[i];
    return cg_block_sum(v, red);
}

// Row i of A' x (G lanes per row: lane j takes entries j, j + G, ...; then a
// fixed xor tree); x_j = z_j + beta p_j when FUSED.
template <int G, bool FUSED>
__device__ __forceinline__ double cg_row(const CgArgs& C, int64_t i, int j, const double* x, const double* p,
                                         double beta) {
    double sa = 0.0, sb = 0.0;
    if (i < C.n) {
        int64_t e1 = C.rowptr[i + 1];
#if FEM_CHECK
        if (!fem_in_range(e1, C.nnz + 1, reinterpret_cast<int*>(C.scal + S_FLAG))) e1 = 0;
#endif
        for (int64_t e = C.rowptr[i] + j; e < e1; e += G) {
            if (!fem_in_range(e, C.nnz, reinterpret_cast<int*>(C.scal + S_FLAG))) break;
            int32_t c = C.colind[e];
            if (!fem_in_range(c, C.n, reinterpret_cast<int*>(C.scal + S_FLAG))) c = 0;
            const double xv = FUSED ? fma(beta, p[c], x[c]) : x[c];
            sa += C.A[e] * xv;
            if (C.B) sb += C.B[e] * xv;
        }
    }
    double s = C.ca * sa + C.cb * sb;
#pragma unroll
    for (int m = 1; m < G; m <<= 1) s += __shfl_xor(s, m, G);
    return s;
}

// The system's values ca A + cb B, formed once per solve so that an iteration
// reads one value array instead of two (grid-stride: nnz may exceed what one
// work-item per entry can address).
__global__ __launch_bounds__(CG_BLOCK) void k_cg_combine(const double* A, const double* B, double ca, double cb,
                                                         int64_t nnz, double* AB) {
    for (int64_t e = (int64_t)blockIdx.x * CG_BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * CG_BLOCK)
        AB[e] = ca * A[e] + cb * B[e];
}

__global__ __launch_bounds__(CG_BLOCK) void k_cg_diag(const CgArgs C) {
    const int64_t i = (int64_t)blockIdx.x * CG_BLOCK + threadIdx.x;
    if (i >= C.n) return;
    double d = 0.0;
    for (int64_t e = C.rowptr[i]; e < C.rowptr[i + 1]; ++e) {
        if (!fem_in_range(e, C.nnz, reinterpret_cast<int*>(C.scal + S_FLAG))) break;
        if (C.colind[e] == (int32_t)i) d = C.ca * C.A[e] + (C.B ? C.cb * C.B[e] : 0.0);
    }
    if (!(d > 0.0) || !isfinite(d)) {
        atomicOr(reinterpret_cast<int*>(C.scal + S_FLAG), 1);
        d = 1.0;
    }
    C.dinv[i] = 1.0 / d;
}

// r = rhs - A' x, z = r / d, p_old = 0; partials of r . z, r . r, rhs . rhs.
// With FINAL only r . r is formed (true residual of the result).
template <int G, bool FINAL>
__global__ __launch_bounds__(CG_BLOCK) void k_cg_residual(const CgArgs C, double* p_old) {
    constexpr int ROWS = CG_BLOCK / G;
    __shared__ double red[4];
    const int lr = threadIdx.x / G, j = threadIdx.x % G;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    const int64_t chunks = (C.n + ROWS - 1) / ROWS;
    for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int64_t i = ch * ROWS + lr;
        const double ax = cg_row<G, false>(C, i, j, C.x, nullptr, 0.0);
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
    cg_partials<3>(C.part, v, red);
}

// q = A' (z + beta p_old), p_new = z + beta p_old; partials of p_new . q.
// beta = rz_k / rz_(k-1): rz_k from the partials of the kernel before (nb of
// them), rz_(k-1) from slot 1 - par; workgroup 0 keeps rz_k in slot par.
template <int G>
__global__ __launch_bounds__(CG_BLOCK) void k_cg_product(const CgArgs C, const double* p_old, double* p_new,
                                                         int par, int nb) {
    constexpr int ROWS = CG_BLOCK / G;
    __shared__ double red[4];
    const int lr = threadIdx.x / G, j = threadIdx.x % G;
    const double rz = cg_total(C.part, nb, red);
    const double rz_prev = C.scal[S_RZ0 + (1 - par)];
    const double beta = rz_prev != 0.0 ? rz / rz_prev : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) C.scal[S_RZ0 + par] = rz;
    double pq = 0.0;
    const int64_t chunks = (C.n + ROWS - 1) / ROWS;
    for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int64_t i = ch * ROWS + lr;
        const double qi = cg_row<G, true>(C, i, j, C.z, p_old, beta);
        if (i < C.n && j == 0) {
            const double pi = fma(beta, p_old[i], C.z[i]);
            p_new[i] = pi;
            C.q[i] = qi;
            pq += pi * qi;
        }
    }
    const double v[1] = {pq};
    cg_partials<1>(C.part_pq, v, red);
}

// alpha = rz_k / (p . q) from the product's partials (nb of them) and slot
// par; x += alpha p, r -= alpha q, z = r / d; partials of r . z and r . r.
__global__ __launch_bounds__(CG_BLOCK) void k_cg_update(const CgArgs C, const double* p, int par, int nb) {
    __shared__ double red[4];
    const double pq = cg_total(C.part_pq, nb, red);
    const bool ok = pq > 0.0 && isfinite(pq);
    const double alpha = ok ? C.scal[S_RZ0 + par] / pq : 0.0;
    if (!ok && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(reinterpret_cast<int*>(C.scal + S_FLAG), 2);
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
    cg_partials<2>(C.part, v, red);
}

// Scalars for the host (one workgroup): after the first residual r.z (in both
// slots: p_old is zero then, so the first beta only has to be finite), r.r and
// b.b; after the final residual or a run of iterations, r.r.
enum { CG_AFTER_RESIDUAL = 0, CG_AFTER_ITERATIONS };
template <int STAGE>
__global__ __launch_bounds__(CG_BLOCK) void k_cg_scalars(const CgArgs C, int nb) {
    __shared__ double red[4];
    if constexpr (STAGE == CG_AFTER_RESIDUAL) {
        const double trz = cg_total(C.part, nb, red);
        const double trr = cg_total(C.part + CG_GRID, nb, red);
        const double tbb = cg_total(C.part + 2 * CG_GRID, nb, red);
        if (threadIdx.x == 0) {
            C.scal[S_RZ0] = trz;
            C.scal[S_RZ1] = trz;
            C.scal[S_RR] = trr;
            C.scal[S_BB] = tbb;
        }
    } else {
        const double trr = cg_total(C.part + CG_GRID, nb, red);
        if (threadIdx.x == 0) C.scal[S_RR] = trr;
    }
}

// Launch helpers (G selected at run time). The residual runs on the
// elementwise grid, so that its partials and the update's come in the same
// number (the product adds them).
struct CgLaunch {
    CgArgs C;
    int G;
    unsigned grid_rows, grid_elem;
    hipStream_t s;

    void residual(bool final_, double* p_old) const {
        const dim3 g(grid_elem), b(CG_BLOCK);
        if (G == 4) {
            if (final_) hipLaunchKernelGGL((k_cg_residual<4, true>), g, b, 0, s, C, p_old);
            else hipLaunchKernelGGL((k_cg_residual<4, false>), g, b, 0, s, C, p_old);
        } else if (G == 8) {
            if (final_) hipLaunchKernelGGL((k_cg_residual<8, true>), g, b, 0, s, C, p_old);
            else hipLaunchKernelGGL((k_cg_residual<8, false>), g, b, 0, s, C, p_old);
        } else {
            if (final_) hipLaunchKernelGGL((k_cg_residual<16, true>), g, b, 0, s, C, p_old);
            else hipLaunchKernelGGL((k_cg_residual<16, false>), g, b, 0, s, C, p_old);
        }
        if (final_) hipLaunchKernelGGL(k_cg_scalars<CG_AFTER_ITERATIONS>, dim3(1), b, 0, s, C, (int)grid_elem);
        else hipLaunchKernelGGL(k_cg_scalars<CG_AFTER_RESIDUAL>, dim3(1), b, 0, s, C, (int)grid_elem);
    }
    // iteration k, par = k mod 2
    void iteration(const double* p_old, double* p_new, int par) const {
        const dim3 g(grid_rows), b(CG_BLOCK);
        const int nb = (int)grid_elem;
        if (G == 4) hipLaunchKernelGGL(k_cg_product<4>, g, b, 0, s, C, p_old, p_new, par, nb);
        else if (G == 8) hipLaunchKernelGGL(k_cg_product<8>, g, b, 0, s, C, p_old, p_new, par, nb);
        else hipLaunchKernelGGL(k_cg_product<16>, g, b, 0, s, C, p_old, p_new, par, nb);
        hipLaunchKernelGGL(k_cg_update, dim3(grid_elem), b, 0, s, C, p_new, par, (int)grid_rows);
    }
    // r.r of the last iteration, for the host's convergence test
    void residual_norm() const {
        hipLaunchKernelGGL(k_cg_scalars<CG_AFTER_ITERATIONS>, dim3(1), dim3(CG_BLOCK), 0, s, C, (int)grid_elem);
    }
};

}  // namespace fem

namespace fem {

// FEM_CG_LOG=N: one line on stderr at the first convergence test after every N
// iterations (iterations done, recursive relative residual), so that a long
// solve reports its progress; unset or not a positive number: silent.
static int64_t cg_log_every() {
    const char* s = std::getenv("FEM_CG_LOG");
    if (!s) return 0;
    char* end = nullptr;
    const long long v = std::strtoll(s, &end, 10);
    return (end != s && v > 0) ? (int64_t)v : 0;
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
    hipStream_t us = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = n_rows;
    // workspace: r, z, q, p (two), 1/diag, partials, scalars
    const size_t vec = (size_t)n * sizeof(double);
    const size_t bytes = 6 * vec + 4 * CG_GRID * sizeof(double) + S_N * sizeof(double) + 256;
    // The solve runs on a stream of its own (HIP graphs cannot be captured on
    // the null stream), ordered after the caller's work and before anything
    // the caller queues next.
    struct Res {
        char* ws = nullptr;
        double* ab = nullptr;  // ca A + cb B when B is given
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        ~Res() {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            if (s) (void)hipStreamSynchronize(s);
            if (ev) (void)hipEventDestroy(ev);
            if (s) (void)hipStreamDestroy(s);
            if (ws) (void)hipFree(ws);
            if (ab) (void)hipFree(ab);
        }
    } R;
    FEM_HIP(hipMalloc(reinterpret_cast<void**>(&R.ws), bytes));
    FEM_HIP(hipStreamCreateWithFlags(&R.s, hipStreamNonBlocking));
    FEM_HIP(hipEventCreateWithFlags(&R.ev, hipEventDisableTiming));
    FEM_HIP(hipEventRecord(R.ev, us));
    FEM_HIP(hipStreamWaitEvent(R.s, R.ev, 0));
    const hipStream_t s = R.s;
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
    C.r = reinterpret_cast<double*>(R.ws);
    C.z = C.r + n;
    C.q = C.z + n;
    double* p0 = C.q + n;
    double* p1 = p0 + n;
    C.dinv = p1 + n;
    C.part = C.dinv + n;
    C.part_pq = C.part + 3 * CG_GRID;
    C.scal = C.part_pq + CG_GRID;
    FEM_HIP(hipMemsetAsync(C.scal, 0, S_N * sizeof(double), s));
    // lanes per row from the mean row length
    int64_t nnz = 0;
    FEM_HIP(hipMemcpyAsync(&nnz, rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    C.nnz = nnz;
    if (B) {
        FEM_HIP(hipMalloc(reinterpret_cast<void**>(&R.ab), (size_t)std::max<int64_t>(nnz, 1) * sizeof(double)));
        const unsigned gc = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8 * CG_GRID, (nnz + CG_BLOCK - 1) / CG_BLOCK));
        hipLaunchKernelGGL(k_cg_combine, dim3(gc), dim3(CG_BLOCK), 0, s, A, B, ca, cb, nnz, R.ab);
        FEM_HIP(hipGetLastError());
        C.A = R.ab;
        C.B = nullptr;
        C.ca = 1.0;
        C.cb = 0.0;
    }
    CgLaunch L;
    L.C = C;
    L.G = nnz <= 8 * n ? 4 : nnz <= 16 * n ? 8 : 16;
    L.grid_rows = (unsigned)std::min<int64_t>(CG_GRID, (n + CG_BLOCK / L.G - 1) / (CG_BLOCK / L.G));
    L.grid_elem = (unsigned)std::min<int64_t>(CG_GRID, (n + CG_BLOCK - 1) / CG_BLOCK);
    L.s = s;
    hipLaunchKernelGGL(k_cg_diag, dim3((unsigned)((n + CG_BLOCK - 1) / CG_BLOCK)), dim3(CG_BLOCK), 0, s, C);
    L.residual(false, p0);
    FEM_HIP(hipGetLastError());
    double host[S_N];
    FEM_HIP(hipMemcpyAsync(host, C.scal, sizeof(host), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    const double bb = host[S_BB];
    int flag = (int)reinterpret_cast<const int*>(&host[S_FLAG])[0];
    if (flag & ERR_BOUNDS) return fail(FEM_ERANGE, "fem_cg_solve (checked build): a column index outside [0, n_rows)");
    if (flag & 1) return fail(FEM_EINVAL, "fem_cg_solve: a diagonal entry is not positive");
    double rr = host[S_RR];
    int64_t it = 0;
    const double target = rtol * rtol * bb;
    bool converged = bb == 0.0 || rr <= target;
    const int64_t log_every = cg_log_every();
    int64_t next_log = log_every;
    while (!converged && it < max_iter) {
        const int64_t steps = std::min<int64_t>(CG_CHECK, max_iter - it);
        if (steps == CG_CHECK) {
            // CG_CHECK iterations (an even number, so p ends in p0 again) as one graph
            if (!R.exec) {
                // it is a multiple of CG_CHECK here (an even number), so
                // iteration it + k has parity k mod 2
                FEM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < CG_CHECK; ++k) L.iteration(k % 2 ? p1 : p0, k % 2 ? p0 : p1, k % 2);
                L.residual_norm();
                FEM_HIP(hipStreamEndCapture(s, &R.graph));
                FEM_HIP(hipGraphInstantiate(&R.exec, R.graph, nullptr, nullptr, 0));
            }
            FEM_HIP(hipGraphLaunch(R.exec, s));
        } else {
            for (int64_t k = 0; k < steps; ++k) {
                L.iteration(p0, p1, (int)((it + k) % 2));
                std::swap(p0, p1);
            }
            L.residual_norm();
        }
        FEM_HIP(hipGetLastError());
        it += steps;
        FEM_HIP(hipMemcpyAsync(host, C.scal, sizeof(host), hipMemcpyDeviceToHost, s));
        FEM_HIP(hipStreamSynchronize(s));
        rr = host[S_RR];
        flag = (int)reinterpret_cast<const int*>(&host[S_FLAG])[0];
        if (flag & ERR_BOUNDS) return fail(FEM_ERANGE, "fem_cg_solve (checked build): a column index outside [0, n_rows)");
        if (flag & 2) return fail(FEM_EHIP, "fem_cg_solve: breakdown (p . A p <= 0: the matrix is not positive definite)");
        converged = rr <= target || !std::isfinite(rr);
        if (log_every > 0 && it >= next_log) {
            std::fprintf(stderr, "fem_cg_solve: %lld iterations, relative residual %.3e\n", (long long)it,
                         std::sqrt(rr / bb));
            next_log = (it / log_every + 1) * log_every;
        }
    }
    // true residual of the result
    L.residual(true, p0);
    FEM_HIP(hipGetLastError());
    FEM_HIP(hipMemcpyAsync(host, C.scal, sizeof(host), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    // work the caller queues next on its stream runs after the solve
    FEM_HIP(hipEventRecord(R.ev, s));
    FEM_HIP(hipStreamWaitEvent(us, R.ev, 0));
    if (iters) *iters = it;
    if (rel_resid) *rel_resid = bb > 0.0 ? std::sqrt(host[S_RR] / bb) : 0.0;
    return FEM_OK;
}

}  // extern "C"
