// Integration of functions over a mesh (Section 3.1): the squared L2 norm of a
// function, the load vector int F . eta_i of the Nedelec basis, and the
// H(curl) error of a discrete Nedelec field against a given field. These are
// the quadrature steps of the examples of Section 4.
//
// Quadrature: the conical-product (collapsed coordinate) Gauss-Legendre rule
// on the reference simplex. With m Gauss-Legendre points t_i, weights w_i on
// [0, 1] (computed on the host by Newton's method on the Legendre recurrence),
// the points are
//   2D: (u, v (1 - u)),                    weight w_u w_v (1 - u)
//   3D: (u, v (1 - u), t (1 - u)(1 - v)),  weight w_u w_v w_t (1 - u)^2 (1 - v)
// and the rule integrates polynomials of total degree <= 2m - dim exactly. A
// kernel receives the m one-dimensional nodes and weights and forms the
// points itself (m^dim of them; m <= 8).
//
// The elements are evaluated with barycentric coordinates: at the reference
// point x^, lambda_0 = 1 - sum x^_i, lambda_i = x^_i, the physical point is
// x_0 + B x^, grad lambda_a = c_a / J (cofactor vectors, J = det B), and the
// Nedelec basis function of local edge k = (i -> j) is the Whitney form
// s_k (lambda_i grad lambda_j - lambda_j grad lambda_i) (the Piola image of the
// reference basis of Section 2.2), with curl 2 s_k grad lambda_i x grad lambda_j.
//
// Every element's value is computed by one lane; element sums are reduced in a
// fixed order (one partial per workgroup of 256 elements, each a fixed tree,
// then the partials in index order) and load-vector entries are summed over
// each dof's elements in ascending element order: results are deterministic.
#include <cmath>
#include <string>

#include "element.h"
#include "fem_internal.h"
#include "quad.h"

namespace fem {

// ---------------------------------------------------------------------------
// quadrature (host)
fem_status gauss_legendre01(int m, QuadRule* q) {
    if (m < 1 || m > FEM_QUAD_MAX) return fail(FEM_EINVAL, "quadrature: points per direction must be 1..8");
    q->m = m;
    for (int i = 0; i < m; ++i) {
        // Newton's method for the i-th root of P_m from the Chebyshev-like guess
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;  // P_0, P_1
            for (int j = 2; j <= m; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (m == 1) p0 = 1.0, p1 = z;
            // P_m = p1, P_{m-1} = p0; P'_m = m (z P_m - P_{m-1}) / (z^2 - 1)
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute P'_m at the converged root for the weight
        {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= m; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (m == 1) p0 = 1.0, p1 = z;
            dp = m * (z * p1 - p0) / (z * z - 1.0);
        }
        q->x[i] = 0.5 * (1.0 - z);
        q->w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // (2 / ((1 - z^2) P'^2)) / 2
    }
    return FEM_OK;
}

// ---------------------------------------------------------------------------
// functions (device)
fem_status make_fn_args(fem_function fn, int dim, const double* params, int n_params, FnArgs* F) {
    F->fn = (int)fn;
    F->n_terms = 0;
    F->n_comp = 1;
    switch (fn) {
        case FEM_FN_POLYNOMIAL: {
            const int w = 2 + dim;
            if (!params || n_params <= 0 || n_params % w != 0 || n_params / w > FEM_POLY_MAX_TERMS)
                return fail(FEM_EINVAL, "polynomial: params must hold 1.." + std::to_string(FEM_POLY_MAX_TERMS) +
                                            " terms of (coefficient, component, " + std::to_string(dim) +
                                            " exponents)");
            F->n_terms = n_params / w;
            int nc = 1;
            for (int t = 0; t < F->n_terms; ++t) {
                const double* p = params + t * w;
                const double c = p[1];
                if (!(c == 0.0 || c == 1.0 || (c == 2.0 && dim == 3)))
                    return fail(FEM_EINVAL, "polynomial: component must be 0.." + std::to_string(dim - 1));
                for (int d = 0; d < dim; ++d) {
                    const double e = p[2 + d];
                    if (!(e >= 0.0 && e <= 30.0 && e == std::floor(e)))
                        return fail(FEM_EINVAL, "polynomial: exponents must be integers 0..30");
                }
                if ((int)c + 1 > nc) nc = (int)c + 1;
                F->term[t].coef = p[0];
                F->term[t].comp = (int)c;
                for (int d = 0; d < 3; ++d) F->term[t].expo[d] = d < dim ? (int)p[2 + d] : 0;
                F->term[t].pad[0] = F->term[t].pad[1] = 0;
            }
            F->n_comp = nc;
            return FEM_OK;
        }
        case FEM_FN_EDDY_E:
        case FEM_FN_EDDY_F:
            if (dim != 2) return fail(FEM_EINVAL, "the eddy-current functions are two-dimensional");
            F->n_comp = 2;
            return FEM_OK;
        case FEM_FN_EDDY_CURL_E:
            if (dim != 2) return fail(FEM_EINVAL, "the eddy-current functions are two-dimensional");
            F->n_comp = 1;
            return FEM_OK;
        case FEM_FN_BUBBLE_U:
        case FEM_FN_BUBBLE_F:
            F->n_comp = 1;
            return FEM_OK;
        case FEM_FN_BUBBLE_GRAD_U:
            F->n_comp = dim;
            return FEM_OK;
        default:
            return fail(FEM_EINVAL, "unknown function");
    }
}

// ---------------------------------------------------------------------------
// squared L2 norm (Section 3.1): per element sum_q w_q |J| |f(F_K(xhat_q))|^2
template <int DIM, int FAM>
__global__ __launch_bounds__(INT_BLOCK) void k_norm_L2(const int32_t* __restrict__ elems,
                                                        const double* __restrict__ nodes, int64_t T,
                                                        const QuadRule q, const FnArgs F,
                                                        double* __restrict__ per_elem,
                                                        double* __restrict__ partials, int* err_word) {
    const int64_t e = (int64_t)blockIdx.x * INT_BLOCK + threadIdx.x;
    double acc = 0.0;
    if (e < T) {
        int gid[DIM + 1];
        load_gid<DIM>(elems, e, gid);
        const QElem<DIM> g = q_elem<DIM>(nodes, gid);
        const double aJ = fabs(g.J);
        for_points<DIM>(q, [&](const double* xh, double w) {
            double x[DIM], fv[3];
            phys_point<DIM>(g, xh, x);
            eval_fn<DIM, FAM>(F, x, fv);
            double s = 0.0;
            for (int c = 0; c < F.n_comp; ++c) s += fv[c] * fv[c];
            acc += w * s;
        });
        acc *= aJ;
        if (per_elem) per_elem[e] = acc;
        if (!(aJ > 0.0) || !isfinite(g.J)) atomicOr(err_word, ERR_DEGENERATE);
    }
    block_sum(acc, partials);
}

// ---------------------------------------------------------------------------
// Nedelec load vector, local part: loc[e][k] = sum_q w_q |J| F(x_q) . eta_k(x_q)
template <int DIM>
__global__ __launch_bounds__(INT_BLOCK) void k_load_local_ned(const int32_t* __restrict__ elems,
                                                               const double* __restrict__ nodes, int64_t T,
                                                               const QuadRule q, const FnArgs F,
                                                               double* __restrict__ loc, int* err_word) {
    constexpr int NLOC = DIM == 2 ? 3 : 6;
    const int64_t e = (int64_t)blockIdx.x * INT_BLOCK + threadIdx.x;
    if (e >= T) return;
    int gid[DIM + 1];
    load_gid<DIM>(elems, e, gid);
    const QElem<DIM> g = q_elem<DIM>(nodes, gid);
    const double rJ = 1.0 / g.J;
    double s[NLOC];
    if constexpr (DIM == 2) tri_signs(gid, s);
    else ned3_signs(gid, s);
    double acc[NLOC];
#pragma unroll
    for (int k = 0; k < NLOC; ++k) acc[k] = 0.0;
    for_points<DIM>(q, [&](const double* xh, double w) {
        double x[DIM], fv[3] = {0.0, 0.0, 0.0};
        phys_point<DIM>(g, xh, x);
        eval_fn<DIM>(F, x, fv);
        double lam[DIM + 1];
        lam[0] = 1.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            lam[d + 1] = xh[d];
            lam[0] -= xh[d];
        }
        // F . grad lambda_a (times J)
        double fg[DIM + 1];
#pragma unroll
        for (int a = 0; a <= DIM; ++a) {
            double t = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) t += fv[d] * g.c[a][d];
            fg[a] = t;
        }
#pragma unroll
        for (int k = 0; k < NLOC; ++k) {
            const int i = DIM == 2 ? nib(TRI_START, k) : nib(NED3_START, k);
            const int j = DIM == 2 ? nib(TRI_END, k) : nib(NED3_END, k);
            acc[k] += w * (lam[i] * fg[j] - lam[j] * fg[i]);
        }
    });
    // |J| * (1 / J) from grad lambda = c / J
    const double f = fabs(g.J) * rJ;
#pragma unroll
    for (int k = 0; k < NLOC; ++k) loc[e * NLOC + k] = s[k] * acc[k] * f;
    if (!(fabs(g.J) > 0.0) || !isfinite(g.J)) atomicOr(err_word, ERR_DEGENERATE);
}

// f[i] = sum of the local values of dof i's slots, in ascending element order
// (n_slots, err: the checked build's bounds of the slot indices)
__global__ __launch_bounds__(INT_BLOCK) void k_dof_sum(const int32_t* __restrict__ rs_ptr,
                                                        const int32_t* __restrict__ rs_slot,
                                                        const double* __restrict__ loc, int64_t n,
                                                        double* __restrict__ out, int64_t n_slots, int* err) {
    const int64_t i = (int64_t)blockIdx.x * INT_BLOCK + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    const int j1 = rs_ptr[i + 1];
    for (int j = rs_ptr[i]; j < j1; ++j) {
        if (!fem_in_range(j, n_slots, err)) break;
        const int q = rs_slot[j];
        if (fem_in_range(q, n_slots, err)) acc += loc[q];
    }
    out[i] = acc;
}

// ---------------------------------------------------------------------------
// H(curl) error of the Nedelec field with dof values v against (E, curl E):
// per element sum_q w_q |J| (|E - v_h|^2 + |curl E - curl v_h|^2)
template <int DIM>
__global__ __launch_bounds__(INT_BLOCK) void k_hcurl_error(const int32_t* __restrict__ elems,
                                                            const double* __restrict__ nodes,
                                                            const int32_t* __restrict__ elems2dofs,
                                                            const double* __restrict__ v, int64_t T,
                                                            const QuadRule q, const FnArgs FE,
                                                            const FnArgs FC, double* __restrict__ per_elem,
                                                            double* __restrict__ partials, int* err_word) {
    constexpr int NLOC = DIM == 2 ? 3 : 6;
    constexpr int NCURL = DIM == 2 ? 1 : 3;
    const int64_t e = (int64_t)blockIdx.x * INT_BLOCK + threadIdx.x;
    double acc = 0.0;
    if (e < T) {
        int gid[DIM + 1];
        load_gid<DIM>(elems, e, gid);
        const QElem<DIM> g = q_elem<DIM>(nodes, gid);
        const double rJ = 1.0 / g.J;
        double s[NLOC];
        if constexpr (DIM == 2) tri_signs(gid, s);
        else ned3_signs(gid, s);
        double ve[NLOC];
#pragma unroll
        for (int k = 0; k < NLOC; ++k) ve[k] = s[k] * v[elems2dofs[e * NLOC + k]];
        // antisymmetric vertex matrix of the dofs: field = sum_a lambda_a sum_b al_ab grad lambda_b
        double al[DIM + 1][DIM + 1];
#pragma unroll
        for (int a = 0; a <= DIM; ++a)
#pragma unroll
            for (int b = 0; b <= DIM; ++b) al[a][b] = 0.0;
#pragma unroll
        for (int k = 0; k < NLOC; ++k) {
            const int i = DIM == 2 ? nib(TRI_START, k) : nib(NED3_START, k);
            const int j = DIM == 2 ? nib(TRI_END, k) : nib(NED3_END, k);
            al[i][j] = ve[k];
            al[j][i] = -ve[k];
        }
        // R_a = sum_b al_ab c_b (J grad lambda_b); curl v_h = 2 sum_k ve_k grad l_i x grad l_j
        double R[DIM + 1][DIM];
#pragma unroll
        for (int a = 0; a <= DIM; ++a)
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                double t = 0.0;
#pragma unroll
                for (int b = 0; b <= DIM; ++b) t += al[a][b] * g.c[b][d];
                R[a][d] = t * rJ;
            }
        double cv[NCURL];
#pragma unroll
        for (int c = 0; c < NCURL; ++c) cv[c] = 0.0;
#pragma unroll
        for (int k = 0; k < NLOC; ++k) {
            const int i = DIM == 2 ? nib(TRI_START, k) : nib(NED3_START, k);
            const int j = DIM == 2 ? nib(TRI_END, k) : nib(NED3_END, k);
            const double f = 2.0 * ve[k] * rJ * rJ;
            if constexpr (DIM == 2) {
                cv[0] += f * (g.c[i][0] * g.c[j][1] - g.c[i][1] * g.c[j][0]);
            } else {
                cv[0] += f * (g.c[i][1] * g.c[j][2] - g.c[i][2] * g.c[j][1]);
                cv[1] += f * (g.c[i][2] * g.c[j][0] - g.c[i][0] * g.c[j][2]);
                cv[2] += f * (g.c[i][0] * g.c[j][1] - g.c[i][1] * g.c[j][0]);
            }
        }
        for_points<DIM>(q, [&](const double* xh, double w) {
            double x[DIM], ev[3] = {0.0, 0.0, 0.0}, ec[3] = {0.0, 0.0, 0.0};
            phys_point<DIM>(g, xh, x);
            eval_fn<DIM>(FE, x, ev);
            eval_fn<DIM>(FC, x, ec);
            double lam[DIM + 1];
            lam[0] = 1.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                lam[d + 1] = xh[d];
                lam[0] -= xh[d];
            }
            double t = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                double vh = 0.0;
#pragma unroll
                for (int a = 0; a <= DIM; ++a) vh += lam[a] * R[a][d];
                const double dd = ev[d] - vh;
                t += dd * dd;
            }
#pragma unroll
            for (int c = 0; c < NCURL; ++c) {
                const double dc = ec[c] - cv[c];
                t += dc * dc;
            }
            acc += w * t;
        });
        acc *= fabs(g.J);
        if (per_elem) per_elem[e] = acc;
        if (!(fabs(g.J) > 0.0) || !isfinite(g.J)) atomicOr(err_word, ERR_DEGENERATE);
    }
    block_sum(acc, partials);
}

fem_status ensure_int_partials(fem_mesh m) {
    if (!m->int_partials)
        FEM_HIP(dmalloc(m, &m->int_partials, 2 * std::max<int64_t>(1, (m->T + INT_BLOCK - 1) / INT_BLOCK)));
    return FEM_OK;
}

// ---------------------------------------------------------------------------
// Raviart-Thomas quantities of the majorant (Section 4.1). Global basis on an
// element: phi_k = s_k (x - x_(p_k)) / J with p_k the vertex opposite local dof
// k (2D: vertex k; 3D: vertex 3 - k) and J = det B_K signed (the
// contravariant Piola image of the printed basis x^ - p^_k, Section 2.1, with
// which the sign data make the normal component continuous); div phi_k =
// s_k d / J.
template <int DIM>
__device__ __forceinline__ int rt_opp(int k) { return DIM == 2 ? k : 3 - k; }

template <int DIM>
__device__ __forceinline__ void rt_signs_of(const int* gid, double* s) {
    if constexpr (DIM == 2) tri_signs(gid, s);
    else rt3_signs(gid, s);
}

// grad v of the P1 field v on the element
template <int DIM>
__device__ __forceinline__ void p1_grad(const QElem<DIM>& g, const int* gid, const double* v, double rJ, double* gv) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a <= DIM; ++a) t += v[gid[a]] * g.c[a][d];
        gv[d] = t * rJ;
    }
}

// loc[e][k] = c_div int f div phi_k + c_grad int grad v . phi_k
template <int DIM>
__global__ __launch_bounds__(INT_BLOCK) void k_rt_majorant_local(const int32_t* __restrict__ elems,
                                                                  const double* __restrict__ nodes,
                                                                  const double* __restrict__ v, int64_t T,
                                                                  const QuadRule q, const FnArgs F, double c_div,
                                                                  double c_grad, double* __restrict__ loc) {
    constexpr int NLOC = DIM + 1;
    const int64_t e = (int64_t)blockIdx.x * INT_BLOCK + threadIdx.x;
    if (e >= T) return;
    int gid[DIM + 1];
    load_gid<DIM>(elems, e, gid);
    const QElem<DIM> g = q_elem<DIM>(nodes, gid);
    const double rJ = 1.0 / g.J;
    double s[NLOC];
    rt_signs_of<DIM>(gid, s);
    double gv[DIM];
    p1_grad<DIM>(g, gid, v, rJ, gv);
    // vertices x_p = x_0 + B e_p (p >= 1)
    double fint = 0.0;        // int f over the reference element (times the weights)
    double gx[NLOC];          // int grad v . (x - x_p) per opposite vertex p
#pragma unroll
    for (int k = 0; k < NLOC; ++k) gx[k] = 0.0;
    for_points<DIM>(q, [&](const double* xh, double w) {
        double x[DIM], fv[3] = {0.0, 0.0, 0.0};
        phys_point<DIM>(g, xh, x);
        eval_fn<DIM>(F, x, fv);
        fint += w * fv[0];
        // grad v . (x - x_p): x - x_0 = B xh, x_p - x_0 = B e_p
        double gB[DIM];  // grad v . b_j
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double t = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) t += gv[d] * g.B[d][j];
            gB[j] = t;
        }
        double base = 0.0;
#pragma unroll
        for (int j = 0; j < DIM; ++j) base += gB[j] * xh[j];
#pragma unroll
        for (int k = 0; k < NLOC; ++k) {
            const int p = rt_opp<DIM>(k);
            gx[k] += w * (p == 0 ? base : base - gB[p - 1]);
        }
    });
    const double aJ = fabs(g.J);
#pragma unroll
    for (int k = 0; k < NLOC; ++k)
        loc[e * NLOC + k] = s[k] * aJ * rJ * (c_div * DIM * fint + c_grad * gx[k]);
}

// per element ||grad v - y_h||_K^2 and ||div y_h + f||_K^2 into two partial rows
template <int DIM>
__global__ __launch_bounds__(INT_BLOCK) void k_majorant_terms(const int32_t* __restrict__ elems,
                                                               const double* __restrict__ nodes,
                                                               const int32_t* __restrict__ elems2dofs,
                                                               const double* __restrict__ v,
                                                               const double* __restrict__ y, int64_t T,
                                                               const QuadRule q, const FnArgs F,
                                                               double* __restrict__ partials, int64_t nb) {
    constexpr int NLOC = DIM + 1;
    const int64_t e = (int64_t)blockIdx.x * INT_BLOCK + threadIdx.x;
    double a2 = 0.0, b2 = 0.0;
    if (e < T) {
        int gid[DIM + 1];
        load_gid<DIM>(elems, e, gid);
        const QElem<DIM> g = q_elem<DIM>(nodes, gid);
        const double rJ = 1.0 / g.J;
        double s[NLOC];
        rt_signs_of<DIM>(gid, s);
        double gv[DIM];
        p1_grad<DIM>(g, gid, v, rJ, gv);
        double ye[NLOC], ysum = 0.0;
#pragma unroll
        for (int k = 0; k < NLOC; ++k) {
            ye[k] = s[k] * y[elems2dofs[e * NLOC + k]] * rJ;
            ysum += ye[k];
        }
        const double divy = DIM * ysum;
        // y_h(x) = sum_k ye_k (x - x_(p_k)) = ysum (x - x_0) - sum_k ye_k (x_(p_k) - x_0)
        double yoff[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < NLOC; ++k) {
                const int p = rt_opp<DIM>(k);
                if (p > 0) t += ye[k] * g.B[d][p - 1];
            }
            yoff[d] = t;
        }
        for_points<DIM>(q, [&](const double* xh, double w) {
            double x[DIM], fv[3] = {0.0, 0.0, 0.0};
            phys_point<DIM>(g, xh, x);
            eval_fn<DIM>(F, x, fv);
            double t = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const double yh = ysum * (x[d] - g.x0[d]) - yoff[d];
                t += (gv[d] - yh) * (gv[d] - yh);
            }
            a2 += w * t;
            b2 += w * (divy + fv[0]) * (divy + fv[0]);
        });
        const double aJ = fabs(g.J);
        a2 *= aJ;
        b2 *= aJ;
    }
    block_sum(a2, partials);
    block_sum(b2, partials + nb);
}

static unsigned int_grid(int64_t n) { return (unsigned)((n + INT_BLOCK - 1) / INT_BLOCK); }

}  // namespace fem

using namespace fem;

extern "C" {

fem_status fem_norm_L2(fem_mesh m, const double* nodes, fem_function fn, const double* params, int n_params,
                       int quad_m, double* per_elem, double* total, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_norm_L2: mesh is NULL");
    if (!nodes || !total) return fail(FEM_EINVAL, "fem_norm_L2: nodes or total is NULL");
    QuadRule q;
    if (fem_status st = gauss_legendre01(quad_m, &q)) return st;
    FnArgs F;
    if (fem_status st = make_fn_args(fn, m->dim, params, n_params, &F)) return st;
    if (fem_status st = ensure_int_partials(m)) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    const unsigned grid = int_grid(m->T);
    // one kernel per dimension and function family (each holds only its
    // family's evaluation, so the polynomial one keeps few registers)
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, m->T, q, F, per_elem,
                           m->int_partials, m->err_word);
    };
    const int fam = fn_family(F.fn);
    if (m->dim == 2) {
        if (fam == FN_POLY) launch(k_norm_L2<2, FN_POLY>);
        else if (fam == FN_BUBBLE) launch(k_norm_L2<2, FN_BUBBLE>);
        else launch(k_norm_L2<2, FN_EDDY>);
    } else {
        if (fam == FN_POLY) launch(k_norm_L2<3, FN_POLY>);
        else launch(k_norm_L2<3, FN_BUBBLE>);  // the eddy functions are two-dimensional
    }
    FEM_HIP(hipGetLastError());
    return launch_sum_partials(m->int_partials, grid, total, s);
}

fem_status fem_load_vector(fem_mesh m, fem_kind kind, const double* nodes, fem_function fn,
                           const double* params, int n_params, int quad_m, double* f, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_load_vector: mesh is NULL");
    if (kind != FEM_NEDELEC) return fail(FEM_EINVAL, "fem_load_vector: only the Nedelec basis is supported");
    if (!nodes || !f) return fail(FEM_EINVAL, "fem_load_vector: nodes or f is NULL");
    QuadRule q;
    if (fem_status st = gauss_legendre01(quad_m, &q)) return st;
    FnArgs F;
    if (fem_status st = make_fn_args(fn, m->dim, params, n_params, &F)) return st;
    if (F.n_comp > m->dim || (fn != FEM_FN_POLYNOMIAL && F.n_comp != m->dim))
        return fail(FEM_EINVAL, "fem_load_vector: the function must be a vector field of the mesh dimension");
    DofSet& ds = m->edges;
    if (!m->slot_vals) FEM_HIP(dmalloc(m, &m->slot_vals, (size_t)m->T * ds.nloc));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    if (m->dim == 2)
        hipLaunchKernelGGL(k_load_local_ned<2>, dim3(int_grid(m->T)), dim3(INT_BLOCK), 0, s, m->elems, nodes, m->T,
                           q, F, m->slot_vals, m->err_word);
    else
        hipLaunchKernelGGL(k_load_local_ned<3>, dim3(int_grid(m->T)), dim3(INT_BLOCK), 0, s, m->elems, nodes, m->T,
                           q, F, m->slot_vals, m->err_word);
    FEM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dof_sum, dim3(int_grid(ds.n)), dim3(INT_BLOCK), 0, s, ds.rs_ptr, ds.rs_slot, m->slot_vals,
                       ds.n, f, m->T * ds.nloc, m->err_word);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status fem_field_error(fem_mesh m, fem_kind kind, const double* nodes, const double* v, fem_function field,
                           fem_function curl, const double* params, int n_params, int quad_m, double* per_elem,
                           double* total, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_field_error: mesh is NULL");
    if (kind != FEM_NEDELEC) return fail(FEM_EINVAL, "fem_field_error: only the Nedelec basis is supported");
    if (!nodes || !v || !total) return fail(FEM_EINVAL, "fem_field_error: nodes, v or total is NULL");
    QuadRule q;
    if (fem_status st = gauss_legendre01(quad_m, &q)) return st;
    FnArgs FE, FC;
    if (fem_status st = make_fn_args(field, m->dim, params, n_params, &FE)) return st;
    if (fem_status st = make_fn_args(curl, m->dim, params, n_params, &FC)) return st;
    if (FE.n_comp > m->dim || FC.n_comp > (m->dim == 2 ? 1 : 3))
        return fail(FEM_EINVAL, "fem_field_error: field or curl has too many components");
    if (fem_status st = ensure_int_partials(m)) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    const unsigned grid = int_grid(m->T);
    if (m->dim == 2)
        hipLaunchKernelGGL(k_hcurl_error<2>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes,
                           m->edges.elems2dofs, v, m->T, q, FE, FC, per_elem, m->int_partials, m->err_word);
    else
        hipLaunchKernelGGL(k_hcurl_error<3>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes,
                           m->edges.elems2dofs, v, m->T, q, FE, FC, per_elem, m->int_partials, m->err_word);
    FEM_HIP(hipGetLastError());
    return launch_sum_partials(m->int_partials, grid, total, s);
}

fem_status fem_rt_majorant_rhs(fem_mesh m, const double* nodes, const double* v, fem_function f,
                               const double* params, int n_params, int quad_m, double c_div, double c_grad,
                               double* rhs, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_rt_majorant_rhs: mesh is NULL");
    if (!nodes || !v || !rhs) return fail(FEM_EINVAL, "fem_rt_majorant_rhs: nodes, v or rhs is NULL");
    QuadRule q;
    if (fem_status st = gauss_legendre01(quad_m, &q)) return st;
    FnArgs F;
    if (fem_status st = make_fn_args(f, m->dim, params, n_params, &F)) return st;
    if (F.n_comp != 1) return fail(FEM_EINVAL, "fem_rt_majorant_rhs: f must be scalar");
    DofSet& ds = m->dim == 3 ? m->faces : m->edges;
    if (!m->slot_vals) FEM_HIP(dmalloc(m, &m->slot_vals, (size_t)m->T * m->edges.nloc));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    const unsigned grid = int_grid(m->T);
    if (m->dim == 3)
        hipLaunchKernelGGL(k_rt_majorant_local<3>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, v, m->T, q, F,
                           c_div, c_grad, m->slot_vals);
    else
        hipLaunchKernelGGL(k_rt_majorant_local<2>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, v, m->T, q, F,
                           c_div, c_grad, m->slot_vals);
    FEM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dof_sum, dim3(int_grid(ds.n)), dim3(INT_BLOCK), 0, s, ds.rs_ptr, ds.rs_slot, m->slot_vals,
                       ds.n, rhs, m->T * ds.nloc, m->err_word);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status fem_majorant_terms(fem_mesh m, const double* nodes, const double* v, const double* y, fem_function f,
                              const double* params, int n_params, int quad_m, double* terms, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_majorant_terms: mesh is NULL");
    if (!nodes || !v || !y || !terms) return fail(FEM_EINVAL, "fem_majorant_terms: NULL argument");
    QuadRule q;
    if (fem_status st = gauss_legendre01(quad_m, &q)) return st;
    FnArgs F;
    if (fem_status st = make_fn_args(f, m->dim, params, n_params, &F)) return st;
    if (F.n_comp != 1) return fail(FEM_EINVAL, "fem_majorant_terms: f must be scalar");
    if (fem_status st = ensure_int_partials(m)) return st;
    DofSet& ds = m->dim == 3 ? m->faces : m->edges;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    const unsigned grid = int_grid(m->T);
    if (m->dim == 3)
        hipLaunchKernelGGL(k_majorant_terms<3>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, ds.elems2dofs, v,
                           y, m->T, q, F, m->int_partials, (int64_t)grid);
    else
        hipLaunchKernelGGL(k_majorant_terms<2>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, ds.elems2dofs, v,
                           y, m->T, q, F, m->int_partials, (int64_t)grid);
    FEM_HIP(hipGetLastError());
    if (fem_status st = launch_sum_partials(m->int_partials, grid, terms, s)) return st;
    return launch_sum_partials(m->int_partials + grid, grid, terms + 1, s);
}

}  // extern "C"
