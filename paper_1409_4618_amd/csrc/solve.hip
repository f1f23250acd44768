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
