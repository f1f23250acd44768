// Device helpers of the quadrature routines (integrate.hip, p1.hip): the
// catalogue functions, element geometry for quadrature, the loop over the
// points of the conical Gauss-Legendre rule, and a fixed-order workgroup sum.
#pragma once

#include "element.h"
#include "fem_internal.h"

namespace fem {

constexpr int INT_BLOCK = 256;

__device__ __forceinline__ double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// The 2D eddy-current example (Section 4.2) on x1 > x2 (zero elsewhere), with
// g = x2 (x1 - x2)^2 (x1 - 1)^2 and h = dg/dx1 = 2 x2 A B C,
// A = x1 - x2, B = x1 - 1, C = 2 x1 - x2 - 1:
//   E = (sin 2 pi x1 + 2 pi cos(2 pi x1) A,  sin g - sin 2 pi x1),
//   curl E = dE2/dx1 - dE1/dx2 = h cos g,
//   F = curl_vec curl E + E = (d(curl E)/dx2 + E1, -d(curl E)/dx1 + E2),
//   d(curl E)/dx1 = h_1 cos g - h^2 sin g,  d(curl E)/dx2 = h_2 cos g - h g_2 sin g,
//   h_1 = 2 x2 (B C + A C + 2 A B),  h_2 = 2 (A B C - x2 B C - x2 A B),
//   g_2 = dg/dx2 = A B^2 (x1 - 3 x2).
__device__ __forceinline__ void eddy_eval(int fn, double x1, double x2, double* out) {
    if (!(x1 > x2)) {
        out[0] = 0.0;
        out[1] = 0.0;
        return;
    }
    const double A = x1 - x2, B = x1 - 1.0, C = 2.0 * x1 - x2 - 1.0;
    const double g = x2 * A * A * B * B;
    const double h = 2.0 * x2 * A * B * C;
    double sg, cg;
    sincos(g, &sg, &cg);
    if (fn == FEM_FN_EDDY_CURL_E) {
        out[0] = h * cg;
        return;
    }
    double s2, c2;
    sincospi(2.0 * x1, &s2, &c2);
    const double E1 = s2 + 2.0 * M_PI * c2 * A;
    const double E2 = sg - s2;
    if (fn == FEM_FN_EDDY_E) {
        out[0] = E1;
        out[1] = E2;
        return;
    }
    const double h1 = 2.0 * x2 * (B * C + A * C + 2.0 * A * B);
    const double h2 = 2.0 * (A * B * C - x2 * B * C - x2 * A * B);
    const double g2 = A * B * B * (x1 - 3.0 * x2);
    const double dc1 = h1 * cg - h * h * sg;
    const double dc2 = h2 * cg - h * g2 * sg;
    out[0] = dc2 + E1;
    out[1] = -dc1 + E2;
}

// The bubble of the majorant example (Section 4.1), u = prod_i x_i (x_i - 1):
// u, grad u, or f = -Lap u = -2 sum_i prod_{j != i} x_j (x_j - 1).
template <int DIM>
__device__ __forceinline__ void bubble_eval(int fn, const double* x, double* out) {
    double q[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) q[i] = x[i] * (x[i] - 1.0);
    if (fn == FEM_FN_BUBBLE_U) {
        double u = 1.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) u *= q[i];
        out[0] = u;
        return;
    }
    double f = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        double o = 1.0;
#pragma unroll
        for (int j = 0; j < DIM; ++j)
            if (j != i) o *= q[j];
        if (fn == FEM_FN_BUBBLE_GRAD_U) out[i] = (2.0 * x[i] - 1.0) * o;
        f -= 2.0 * o;
    }
    if (fn == FEM_FN_BUBBLE_F) out[0] = f;
}

// Function families of the catalogue: a kernel compiled for one family holds
// only that family's evaluation (and its registers); FN_ANY switches at run
// time.
enum { FN_ANY = 0, FN_POLY = 1, FN_EDDY = 2, FN_BUBBLE = 3 };
inline int fn_family(int fn) {
    return fn == FEM_FN_POLYNOMIAL ? FN_POLY : fn >= FEM_FN_BUBBLE_U ? FN_BUBBLE : FN_EDDY;
}

// f at the physical point x (dim coordinates) into out[0 .. n_comp-1]; FAM the
// family of F.fn, or FN_ANY.
template <int DIM, int FAM = FN_ANY>
__device__ __forceinline__ void eval_fn(const FnArgs& F, const double* x, double* out) {
    if (FAM == FN_BUBBLE || (FAM == FN_ANY && F.fn >= FEM_FN_BUBBLE_U)) {
        bubble_eval<DIM>(F.fn, x, out);
    } else if (FAM == FN_POLY || (FAM == FN_ANY && F.fn == FEM_FN_POLYNOMIAL)) {
        for (int c = 0; c < F.n_comp; ++c) out[c] = 0.0;
        for (int t = 0; t < F.n_terms; ++t) {
            const FnArgs::Term term = F.term[t];
            double v = term.coef;
#pragma unroll
            for (int d = 0; d < DIM; ++d) v *= ipow(x[d], term.expo[d]);
            // the component by uniform branches, not a dynamic register index
            const int c = term.comp;
            if (c == 0) out[0] += v;
            else if (DIM == 2 || c == 1) out[1] += v;
            else out[2] += v;
        }
    } else {
        eddy_eval(F.fn, x[0], x[1], out);
    }
}

// ---------------------------------------------------------------------------
// element geometry for quadrature: vertices, cofactor vectors, J
template <int DIM>
struct QElem {
    double x0[DIM];
    double B[DIM][DIM];     // columns b_j = x_j - x_0
    double c[DIM + 1][DIM]; // c_a = J grad lambda_a
    double J;
};

template <int DIM>
__device__ __forceinline__ QElem<DIM> q_elem(const double* nodes, const int* gid) {
    QElem<DIM> g;
    double x[DIM + 1][DIM];
#pragma unroll
    for (int v = 0; v <= DIM; ++v)
#pragma unroll
        for (int d = 0; d < DIM; ++d) x[v][d] = nodes[(int64_t)gid[v] * DIM + d];
#pragma unroll
    for (int d = 0; d < DIM; ++d) g.x0[d] = x[0][d];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
        for (int d = 0; d < DIM; ++d) g.B[d][j] = x[j + 1][d] - x[0][d];
    if constexpr (DIM == 2) {
        const V2 b1 = {g.B[0][0], g.B[1][0]}, b2 = {g.B[0][1], g.B[1][1]};
        g.J = b1.x * b2.y - b1.y * b2.x;
        g.c[1][0] = b2.y;
        g.c[1][1] = -b2.x;
        g.c[2][0] = -b1.y;
        g.c[2][1] = b1.x;
    } else {
        const V3 b1 = {g.B[0][0], g.B[1][0], g.B[2][0]};
        const V3 b2 = {g.B[0][1], g.B[1][1], g.B[2][1]};
        const V3 b3 = {g.B[0][2], g.B[1][2], g.B[2][2]};
        const V3 c1 = cross(b2, b3), c2 = cross(b3, b1), c3 = cross(b1, b2);
        g.J = dot(b1, c1);
        g.c[1][0] = c1.x; g.c[1][1] = c1.y; g.c[1][2] = c1.z;
        g.c[2][0] = c2.x; g.c[2][1] = c2.y; g.c[2][2] = c2.z;
        g.c[3][0] = c3.x; g.c[3][1] = c3.y; g.c[3][2] = c3.z;
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double s = 0.0;
#pragma unroll
        for (int a = 1; a <= DIM; ++a) s += g.c[a][d];
        g.c[0][d] = -s;
    }
    return g;
}

// Loop over the points of the conical rule: f(xhat, weight).
template <int DIM, class Fn>
__device__ __forceinline__ void for_points(const QuadRule& q, Fn&& f) {
    if constexpr (DIM == 2) {
        for (int i = 0; i < q.m; ++i) {
            const double u = q.x[i];
            for (int j = 0; j < q.m; ++j) {
                const double xh[2] = {u, q.x[j] * (1.0 - u)};
                f(xh, q.w[i] * q.w[j] * (1.0 - u));
            }
        }
    } else {
        for (int i = 0; i < q.m; ++i) {
            const double u = q.x[i];
            for (int j = 0; j < q.m; ++j) {
                const double v = q.x[j];
                for (int k = 0; k < q.m; ++k) {
                    const double xh[3] = {u, v * (1.0 - u), q.x[k] * (1.0 - u) * (1.0 - v)};
                    f(xh, q.w[i] * q.w[j] * q.w[k] * (1.0 - u) * (1.0 - u) * (1.0 - v));
                }
            }
        }
    }
}

template <int DIM>
__device__ __forceinline__ void phys_point(const QElem<DIM>& g, const double* xh, double* x) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double s = g.x0[d];
#pragma unroll
        for (int j = 0; j < DIM; ++j) s += g.B[d][j] * xh[j];
        x[d] = s;
    }
}

template <int DIM>
__device__ __forceinline__ void load_gid(const int32_t* elems, int64_t e, int* gid) {
#pragma unroll
    for (int v = 0; v <= DIM; ++v) gid[v] = elems[e * (DIM + 1) + v];
}

// Fixed-order workgroup sum of v into partials[blockIdx.x].
__device__ __forceinline__ void block_sum(double v, double* partials) {
    __shared__ double red[INT_BLOCK];
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = INT_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}


}  // namespace fem
