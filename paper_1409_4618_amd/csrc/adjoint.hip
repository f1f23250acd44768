// Adjoint of the assembly (backward): dL/da, dL/db and dL/dnodes for upstream
// weights gK, gM on the CSR pattern, or for the quadratic form
// L = u^T (K(a) + M(b)) u.
//
// Built with floating-point contraction (unlike the forward kernels, whose
// entries must come out bitwise symmetric): the sums of products below fuse
// into FMAs, which is about 30 % fewer FP64 instructions and one rounding per
// fused pair instead of two.
#include "element.h"
#include "fem_internal.h"

namespace fem {

// ===========================================================================
// Backward: element-major adjoint.
// For each element: gather the upstream weights of its n_local^2 entries through
// the scatter map, contract them with the local matrices (dL/da, dL/db) and with
// their derivatives with respect to the element's vertices (hand-derived from
// the closed forms of element.h; d|J| = |J| tr(B^-1 dB)). The per-element
// vertex derivatives are then summed per node in ascending element order.
// ===========================================================================
struct BwdArgs {
    const int32_t* elems;
    const double* nodes;
    const double* a;
    const double* b;
    const double* gK;
    const double* gM;
    const int32_t* slot_base;  // [T*nloc] row start of each slot's dof
    const uint64_t* slot_cp;   // [T*nloc] column offsets of each slot's row
    const double* u;           // quadratic form: [n_dofs] vector, weights u_I u_J
    const int32_t* elems2dofs; // quadratic form: [T*nloc] global dof of each slot
    double* ga;
    double* gb;
    double* lpart;             // quadratic form: [workgroups] partials of L (NULL: no value)
    double* partials;          // [pairs][dim] vertex-derivative partial per (node, workgroup)
    const int32_t* bptr;       // [workgroups+1] pairs of each workgroup (workgroup-major)
    const uint16_t* pst;       // [pairs] first incidence of each pair, workgroup-local
    const uint16_t* inc;       // workgroup-local incidences by workgroup, node, element
    int64_t T;
    int* err_word;
    // sizes, for the checked build's bounds checks
    int64_t V;        // nodes
    int64_t n_dofs;   // rows of the pattern (entries of u)
    int64_t nnz;      // entries of gK, gM
    int64_t n_pairs;  // (node, workgroup) pairs of the node map
};

// Checked build: node ids of an element within [0, V) (an id out of range is
// flagged and replaced by 0, so the gathers stay in bounds).
template <int NV>
__device__ __forceinline__ void check_gids(const BwdArgs& A, int gid[NV]) {
#if FEM_CHECK
#pragma unroll
    for (int v = 0; v < NV; ++v)
        if (!fem_in_range(gid[v], A.V, A.err_word)) gid[v] = 0;
#else
    (void)A;
    (void)gid;
#endif
}

// Weight modes of the adjoint: separate gK and gM arrays, one array for both
// (L = u^T (K + M) u with its weights materialised), or the quadratic form
// itself, whose weight at (I, J) is u_I u_J: its contractions are sums of
// squares of per-element sums of u, and no nnz-sized array is read.
enum BwdMode { BWD_SEPARATE = 0, BWD_SAME = 1, BWD_QUADRATIC = 2 };

// This lane's slot records (row start, column offsets): staged in LDS by the
// workgroup at kernel start (3D Nedelec), or read in place.
struct SlotView {
    const int32_t* base;
    const uint64_t* cp;
};

// Upstream weights of row k of the lane's element (materialised modes): the
// slot's row start and column offsets give the positions of its n_local
// entries. A missing weight array reads the other one and is zeroed by a
// select (not a branch, which would split the gathers into separate blocks);
// the launcher handles both missing.
template <int NLOC, int MODE>
__device__ __forceinline__ void gather_row(const BwdArgs& A, const SlotView& sv, int k, double wk[NLOC],
                                           double wm[NLOC]) {
    static_assert(MODE != BWD_QUADRATIC, "the quadratic form reads no weights");
    const int64_t base = sv.base[k];
    const uint64_t cp = sv.cp[k];
    const double* pK = A.gK ? A.gK : A.gM;
    const double* pM = A.gM ? A.gM : A.gK;
#pragma unroll
    for (int l = 0; l < NLOC; ++l) {
        int64_t pos = base + (int64_t)((cp >> (8 * l)) & 0xFFu);
        if (!fem_in_range(pos, A.nnz, A.err_word)) pos = 0;
        if constexpr (MODE == BWD_SAME) {
            wk[l] = wm[l] = pK[pos];
        } else {
            const double vk = pK[pos];
            const double vm = pM[pos];
            wk[l] = A.gK ? vk : 0.0;
            wm[l] = A.gM ? vm : 0.0;
        }
    }
}

// The element's coefficients (a NULL array reads the constant 1), loaded
// without a branch and at the start of the element's work: a conditional load
// sits in a block of its own, and the wait for it comes at the end of that
// block, a memory round trip of its own.
__device__ const double kUnitCoefficient = 1.0;
__device__ __forceinline__ double2 load_coeffs(const BwdArgs& A, int64_t e) {
    const double* pa = A.a ? A.a + e : &kUnitCoefficient;
    const double* pb = A.b ? A.b + e : &kUnitCoefficient;
    return make_double2(*pa, *pb);
}

// u at the element's dofs (quadratic mode only)
template <int NLOC, int MODE>
__device__ __forceinline__ void load_u(const BwdArgs& A, int64_t e, double ue[NLOC]) {
#pragma unroll
    for (int l = 0; l < NLOC; ++l) ue[l] = 0.0;
    if constexpr (MODE == BWD_QUADRATIC) {
#pragma unroll
        for (int l = 0; l < NLOC; ++l) {
            int64_t d = A.elems2dofs[e * NLOC + l];
            if (!fem_in_range(d, A.n_dofs, A.err_word)) d = 0;
            ue[l] = A.u[d];
        }
    }
}

// Vertex derivative of local vertex v of the lane's element, into the
// workgroup's LDS slot of that incidence (summed per vertex afterwards).
// Component-major layout, sh[(v * DIM + c) * BWD_BLOCK + lane]: the lanes of a
// store write consecutive words (no bank conflicts).
__device__ __forceinline__ int lds_at(int lane, int v, int dim) { return v * dim * BWD_BLOCK + lane; }
constexpr int LDS_CS = BWD_BLOCK;  // stride between the components of one incidence
__device__ __forceinline__ void store_vertex3(double* sh, int v, V3 d) {
    double* p = sh + lds_at((int)threadIdx.x, v, 3);
    p[0] = d.x;
    p[LDS_CS] = d.y;
    p[2 * LDS_CS] = d.z;
}
__device__ __forceinline__ void store_vertex2(double* sh, int v, double dx, double dy) {
    double* p = sh + lds_at((int)threadIdx.x, v, 2);
    p[0] = dx;
    p[LDS_CS] = dy;
}

// 3D Nedelec. With weights w_kl = s_k s_l gK_kl (gM likewise):
//   dL/da = 2/(3|J|) Phi,  Phi = sum w_kl o_k . o_l,
//   dL/db = Psi/(120|J|),  Psi = sum_ab P_ab G_ab (P: the Whitney weights of
//   the Gram entries, symmetric part accumulated once per pair),
// and the vertex derivatives from dPhi (through the edge vectors), dPsi (through
// the cofactor vectors) and d|J| = |J| tr(B^-1 dB).
template <int MODE>
__device__ double2 bwd_ned3(const BwdArgs& A, int64_t e, const SlotView& sv, double* sh) {
    const double2 cab = load_coeffs(A, e);
    int gid[4];
    V3 x[4];
    const int4 q4 = reinterpret_cast<const int4*>(A.elems)[e];
    gid[0] = q4.x; gid[1] = q4.y; gid[2] = q4.z; gid[3] = q4.w;
    check_gids<4>(A, gid);
#pragma unroll
    for (int v = 0; v < 4; ++v)
        x[v] = {A.nodes[(int64_t)gid[v] * 3], A.nodes[(int64_t)gid[v] * 3 + 1], A.nodes[(int64_t)gid[v] * 3 + 2]};
    const V3 b1 = sub(x[1], x[0]), b2 = sub(x[2], x[0]), b3 = sub(x[3], x[0]);
    double s[6];
    ned3_signs(gid, s);
    double ue[6];
    load_u<6, MODE>(A, e, ue);
    double Phi = 0.0, Psi = 0.0;
    V3 dPhi[3], c[4], w[4];  // w_a = dPsi/dc_a
    if constexpr (MODE == BWD_QUADRATIC) {
        // Weights w_kl = v_k v_l with v_k = s_k u_k: both contractions are sums
        // of squares.
        //   Phi = |z|^2, z = sum_k v_k o_k = beta_1 b1 + beta_2 b2 + beta_3 b3,
        //     so dPhi/db_t = 2 beta_t z;
        //   with alpha the antisymmetric vertex matrix of v (alpha_ij = v_k for
        //   edge k = i -> j), the Whitney field is sum_a lambda_a sum_b alpha_ab
        //   grad lambda_b, and the mass contraction is
        //     Psi = sum_bd G_bd sum_ac (1 + delta_ac) alpha_ab alpha_cd
        //         = |S|^2 + sum_a |R_a|^2,
        //     sigma_b = sum_a alpha_ab, S = sum_b sigma_b c_b, R_a = sum_b alpha_ab c_b,
        //     dPsi/dc_b = 2 (sigma_b S + sum_a alpha_ab R_a).
        double v[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = s[k] * ue[k];
        const double beta[3] = {(v[1] - v[2]) + v[4], (v[2] - v[0]) + v[5], (v[0] - v[1]) + v[3]};
        const V3 z = add(add(scale(b1, beta[0]), scale(b2, beta[1])), scale(b3, beta[2]));
        Phi = dot(z, z);
#pragma unroll
        for (int t = 0; t < 3; ++t) dPhi[t] = scale(z, 2.0 * beta[t]);
        c[1] = cross(b2, b3);
        c[2] = cross(b3, b1);
        c[3] = cross(b1, b2);
        c[0] = neg(add(add(c[1], c[2]), c[3]));
        double al[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) al[a][bb] = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            al[nib(NED3_START, k)][nib(NED3_END, k)] = v[k];
            al[nib(NED3_END, k)][nib(NED3_START, k)] = -v[k];
        }
        double sig[4];
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) sig[bb] = (al[0][bb] + al[1][bb]) + (al[2][bb] + al[3][bb]);
        V3 S = {0.0, 0.0, 0.0};
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) S = add(S, scale(c[bb], sig[bb]));
        Psi = dot(S, S);
        V3 Ra[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            Ra[a] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int bb = 0; bb < 4; ++bb)
                if (bb != a) Ra[a] = add(Ra[a], scale(c[bb], al[a][bb]));
            Psi += dot(Ra[a], Ra[a]);
        }
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            V3 t = scale(S, sig[bb]);
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (a != bb) t = add(t, scale(Ra[a], al[a][bb]));
            w[bb] = scale(t, 2.0);
        }
    } else {
        // dPhi_j (derivative of Phi with respect to b_j) is accumulated directly:
        // with q_k = sum_l (w_kl + w_lk) o_l,
        //   dPhi_1 = q_1 - q_2 + q_4, dPhi_2 = q_2 - q_0 + q_5, dPhi_3 = q_0 - q_1 + q_3
        // (o_0 = b3 - b2, o_1 = b1 - b3, o_2 = b2 - b1, o_3 = b3, o_4 = b1, o_5 = b2).
        double P[10];
#pragma unroll
        for (int t = 0; t < 3; ++t) dPhi[t] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 10; ++t) P[t] = 0.0;
        const V3 o[6] = {sub(b3, b2), sub(b1, b3), sub(b2, b1), b3, b1, b2};
        // sign pattern of q_k in dPhi_1..3
        constexpr int QSGN[6][3] = {{0, -1, 1}, {1, 0, -1}, {-1, 1, 0}, {0, 0, 1}, {1, 0, 0}, {0, 1, 0}};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            // one row of weights at a time: the scheduler would otherwise issue all
            // 72 gathers up front and hold them, at one wavefront per SIMD
            __builtin_amdgcn_sched_barrier(0);
            double gk[6], gm[6];
            gather_row<6, MODE>(A, sv, k, gk, gm);
            const int i = nib(NED3_START, k), j = nib(NED3_END, k);
#pragma unroll
            for (int l = 0; l < 6; ++l) {
                const int m = nib(NED3_START, l), n = nib(NED3_END, l);
                const double ss = s[k] * s[l];
                const double wk = gk[l] * ss;
                const double wm = gm[l] * ss;
                Phi += wk * dot(o[k], o[l]);
                // q_k += wk o_l and q_l += wk o_k, folded into dPhi
                const V3 ol = scale(o[l], wk), ok = scale(o[k], wk);
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    if (QSGN[k][t] > 0) dPhi[t] = add(dPhi[t], ol);
                    if (QSGN[k][t] < 0) dPhi[t] = sub(dPhi[t], ol);
                    if (QSGN[l][t] > 0) dPhi[t] = add(dPhi[t], ok);
                    if (QSGN[l][t] < 0) dPhi[t] = sub(dPhi[t], ok);
                }
                P[tri_index(j, n)] += wm * (1.0 + (i == m));
                P[tri_index(j, m)] -= wm * (1.0 + (i == n));
                P[tri_index(i, n)] -= wm * (1.0 + (j == m));
                P[tri_index(i, m)] += wm * (1.0 + (j == n));
            }
            // fold this row in now (the sums would otherwise be sunk into the
            // conditional output blocks with all 72 weights live until there)
            pin(Phi);
#pragma unroll
            for (int t = 0; t < 3; ++t) pin(dPhi[t]);
#pragma unroll
            for (int t = 0; t < 10; ++t) pin(P[t]);
        }
        // cofactor vectors after the weight loop (not live during it)
        c[1] = cross(b2, b3);
        c[2] = cross(b3, b1);
        c[3] = cross(b1, b2);
        c[0] = neg(add(add(c[1], c[2]), c[3]));
#pragma unroll
        for (int a = 0; a < 4; ++a) w[a] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int bb = a; bb < 4; ++bb) {
                const double p = P[tri_index(a, bb)];
                Psi += p * dot(c[a], c[bb]);
                if (a == bb) {
                    w[a] = add(w[a], scale(c[a], 2.0 * p));
                } else {
                    w[a] = add(w[a], scale(c[bb], p));
                    w[bb] = add(w[bb], scale(c[a], p));
                }
            }
        }
    }
    const double J = dot(b1, c[1]);
    const double aJ = fabs(J);
    const double rJ = 1.0 / J, arJ = fabs(rJ);  // the one division; |1/J| = 1/|J| exactly
    const double ca = cab.x;
    const double cb = cab.y;
    const double2 gab = make_double2((2.0 / 3.0) * Phi * arJ, (1.0 / 120.0) * Psi * arJ);
    if (A.ga) A.ga[e] = gab.x;
    if (A.gb) A.gb[e] = gab.y;
    if (A.partials) {
        const V3 w1 = sub(w[1], w[0]), w2 = sub(w[2], w[0]), w3 = sub(w[3], w[0]);
        const V3 dPsi[3] = {add(cross(w2, b3), cross(b2, w3)), add(cross(b3, w1), cross(w3, b1)),
                            add(cross(w1, b2), cross(b1, w2))};
        const double fk = ca * (2.0 / 3.0) * arJ;
        const double fm = cb * (1.0 / 120.0) * arJ;
        V3 d0 = {0.0, 0.0, 0.0};
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            const V3 cj = c[jj + 1];
            const V3 dj = add(scale(sub(dPhi[jj], scale(cj, Phi * rJ)), fk),
                              scale(sub(dPsi[jj], scale(cj, Psi * rJ)), fm));
            store_vertex3(sh, jj + 1, dj);
            d0 = sub(d0, dj);
        }
        store_vertex3(sh, 0, d0);
    }
    if (!(aJ > 0.0) || !isfinite(J)) atomicOr(A.err_word, ERR_DEGENERATE);
    return gab;
}

// 3D Raviart-Thomas
template <int MODE>
__device__ double2 bwd_rt3(const BwdArgs& A, int64_t e, const SlotView& sv, double* sh) {
    const double2 cab = load_coeffs(A, e);
    int gid[4];
    V3 x[4];
    const int4 q4 = reinterpret_cast<const int4*>(A.elems)[e];
    gid[0] = q4.x; gid[1] = q4.y; gid[2] = q4.z; gid[3] = q4.w;
    check_gids<4>(A, gid);
#pragma unroll
    for (int v = 0; v < 4; ++v)
        x[v] = {A.nodes[(int64_t)gid[v] * 3], A.nodes[(int64_t)gid[v] * 3 + 1], A.nodes[(int64_t)gid[v] * 3 + 2]};
    double ue[4];
    load_u<4, MODE>(A, e, ue);
    const GeoRT3 g = geo_rt3(x);
    double s[4];
    rt3_signs(gid, s);
    const double aJ = fabs(g.J);
    double hK = 0.0, hM = 0.0, cross_term = 0.0;
    double rho[4] = {0.0, 0.0, 0.0, 0.0};
    V3 z[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) z[p] = {0.0, 0.0, 0.0};
    if constexpr (MODE == BWD_QUADRATIC) {
        // Weights v_k v_l with v_k = s_k u_k (face k opposite vertex 3 - k): the
        // sums below are squares, with Vs = sum_k v_k and Y = sum_k v_k y_(3-k):
        //   hK = hM = Vs^2, rho_p = 2 v_(3-p) Vs, cross = |Y|^2, z_p = 2 v_(3-p) Y.
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = s[k] * ue[k];
        const double Vs = (v[0] + v[1]) + (v[2] + v[3]);
        const V3 Y = add(add(scale(g.y[3], v[0]), scale(g.y[2], v[1])), scale(g.y[1], v[2]));
        hK = Vs * Vs;
        hM = hK;
        cross_term = dot(Y, Y);
#pragma unroll
        for (int p = 1; p < 4; ++p) {
            rho[p] = 2.0 * v[3 - p] * Vs;
            z[p] = scale(Y, 2.0 * v[3 - p]);
        }
    } else {
        double GK[4][4], GM[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) gather_row<4, MODE>(A, sv, k, GK[k], GM[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int pk = 3 - k;
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const int pl = 3 - l;
                const double ss = s[k] * s[l];
                const double hk = GK[k][l] * ss;
                const double hm = GM[k][l] * ss;
                hK += hk;
                hM += hm;
                rho[pk] += hm;
                rho[pl] += hm;
                cross_term += hm * dot(g.y[pk], g.y[pl]);
                z[pk] = add(z[pk], scale(g.y[pl], hm));
                z[pl] = add(z[pl], scale(g.y[pk], hm));
            }
        }
    }
    double ru = 0.0;
#pragma unroll
    for (int p = 1; p < 4; ++p) ru += rho[p] * g.u[p];
    const double Omega = hM * g.base - 5.0 * ru + 20.0 * cross_term;
    const double ca = cab.x;
    const double cb = cab.y;
    const double rJ = 1.0 / g.J, arJ = fabs(rJ);  // the one division; |1/J| = 1/|J| exactly
    const double2 gab = make_double2(1.5 * hK * arJ, (1.0 / 120.0) * Omega * arJ);
    if (A.ga) A.ga[e] = gab.x;
    if (A.gb) A.gb[e] = gab.y;
    if (A.partials) {
        const V3 S = add(add(g.y[1], g.y[2]), g.y[3]);
        V3 rp = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 1; p < 4; ++p) rp = add(rp, scale(g.y[p], rho[p]));
        const V3 c[3] = {cross(g.y[2], g.y[3]), cross(g.y[3], g.y[1]), cross(g.y[1], g.y[2])};
        const double fk = -ca * 1.5 * hK * arJ * rJ;
        const double fm = cb * (1.0 / 120.0) * arJ;
        const double OmJ = Omega * rJ;
        V3 d0 = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 1; a < 4; ++a) {
            const V3 dOm = add(sub(scale(add(S, g.y[a]), 2.0 * hM), scale(add(scale(S, rho[a]), rp), 5.0)),
                               scale(z[a], 20.0));
            const V3 ck = c[a - 1];
            const V3 dK = scale(ck, fk);
            const V3 dM = scale(sub(dOm, scale(ck, OmJ)), fm);
            const V3 da = add(dK, dM);
            store_vertex3(sh, a, da);
            d0 = sub(d0, da);
        }
        store_vertex3(sh, 0, d0);
    }
    if (!(aJ > 0.0) || !isfinite(g.J)) atomicOr(A.err_word, ERR_DEGENERATE);
    return gab;
}

// 2D (both kinds)
template <int MODE>
__device__ double2 bwd_tri(const BwdArgs& A, int64_t e, const SlotView& sv, double* sh) {
    const double2 cab = load_coeffs(A, e);
    int gid[3];
    V2 x[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) gid[v] = A.elems[e * 3 + v];
    check_gids<3>(A, gid);
#pragma unroll
    for (int v = 0; v < 3; ++v) x[v] = {A.nodes[(int64_t)gid[v] * 2], A.nodes[(int64_t)gid[v] * 2 + 1]};
    double ue[3];
    load_u<3, MODE>(A, e, ue);
    const Geo2 g = geo2(x);
    double s[3];
    tri_signs(gid, s);
    const double aJ = fabs(g.J);
    double hK = 0.0;
    double Psi = 0.0;
    V2 w[3];
    if constexpr (MODE == BWD_QUADRATIC) {
        // Weights v_k v_l with v_k = s_k u_k: hK = (sum_k v_k)^2, and with alpha
        // the antisymmetric vertex matrix of v, sigma_b = sum_a alpha_ab,
        // S = sum_b sigma_b c_b, R_a = sum_b alpha_ab c_b:
        //   Psi = |S|^2 + sum_a |R_a|^2, dPsi/dc_b = 2 (sigma_b S + sum_a alpha_ab R_a).
        double v[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = s[k] * ue[k];
        const double Vs = (v[0] + v[1]) + v[2];
        hK = Vs * Vs;
        double al[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) al[a][bb] = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            al[nib(TRI_START, k)][nib(TRI_END, k)] = v[k];
            al[nib(TRI_END, k)][nib(TRI_START, k)] = -v[k];
        }
        double sig[3];
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) sig[bb] = (al[0][bb] + al[1][bb]) + al[2][bb];
        V2 S = {0.0, 0.0};
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) S = {S.x + sig[bb] * g.c[bb].x, S.y + sig[bb] * g.c[bb].y};
        Psi = dot2(S, S);
        V2 Ra[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Ra[a] = {0.0, 0.0};
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
                if (bb != a) Ra[a] = {Ra[a].x + al[a][bb] * g.c[bb].x, Ra[a].y + al[a][bb] * g.c[bb].y};
            Psi += dot2(Ra[a], Ra[a]);
        }
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
            V2 t = {sig[bb] * S.x, sig[bb] * S.y};
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a != bb) t = {t.x + al[a][bb] * Ra[a].x, t.y + al[a][bb] * Ra[a].y};
            w[bb] = {2.0 * t.x, 2.0 * t.y};
        }
    } else {
        double GK[3][3], GM[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) gather_row<3, MODE>(A, sv, k, GK[k], GM[k]);
        double Q[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Q[i][j] = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int i = nib(TRI_START, k), j = nib(TRI_END, k);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int m = nib(TRI_START, l), n = nib(TRI_END, l);
                const double ss = s[k] * s[l];
                hK += GK[k][l] * ss;
                const double gm = GM[k][l] * ss;
                Q[j][n] += gm * (1.0 + (i == m));
                Q[j][m] -= gm * (1.0 + (i == n));
                Q[i][n] -= gm * (1.0 + (j == m));
                Q[i][m] += gm * (1.0 + (j == n));
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            w[a] = {0.0, 0.0};
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                Psi += Q[a][bb] * dot2(g.c[a], g.c[bb]);
                const double f = Q[a][bb] + Q[bb][a];
                w[a] = {w[a].x + f * g.c[bb].x, w[a].y + f * g.c[bb].y};
            }
        }
    }
    const double ca = cab.x;
    const double cb = cab.y;
    const double rJ = 1.0 / g.J, arJ = fabs(rJ);  // the one division; |1/J| = 1/|J| exactly
    const double2 gab = make_double2(2.0 * hK * arJ, (1.0 / 24.0) * Psi * arJ);
    if (A.ga) A.ga[e] = gab.x;
    if (A.gb) A.gb[e] = gab.y;
    if (A.partials) {
        const V2 w1 = {w[1].x - w[0].x, w[1].y - w[0].y};
        const V2 w2 = {w[2].x - w[0].x, w[2].y - w[0].y};
        const V2 dPsi[2] = {{w2.y, -w2.x}, {-w1.y, w1.x}};
        const double fk = -ca * 2.0 * hK * arJ * rJ;
        const double fm = cb * (1.0 / 24.0) * arJ;
        const double PsiJ = Psi * rJ;
        double d0x = 0.0, d0y = 0.0;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const V2 cj = g.c[jj + 1];
            const double dx = fk * cj.x + fm * (dPsi[jj].x - cj.x * PsiJ);
            const double dy = fk * cj.y + fm * (dPsi[jj].y - cj.y * PsiJ);
            store_vertex2(sh, jj + 1, dx, dy);
            d0x -= dx;
            d0y -= dy;
        }
        store_vertex2(sh, 0, d0x, d0y);
    }
    if (!(aJ > 0.0) || !isfinite(g.J)) atomicOr(A.err_word, ERR_DEGENERATE);
    return gab;
}

// L_e = a_e dL/da_e + b_e dL/db_e (L is linear in the coefficients), and the
// workgroup's sum of it by a fixed tree in LDS (red: BWD_BLOCK doubles), the
// same in k_backward and k_quadratic_value.
__device__ __forceinline__ double elem_value(const BwdArgs& A, int64_t e, double2 g) {
    const double2 cab = load_coeffs(A, e);
    return cab.x * g.x + cab.y * g.y;
}
__device__ __forceinline__ double wg_tree_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = BWD_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

template <int KC, int MODE>
__global__ __launch_bounds__(BWD_BLOCK) void k_backward(const BwdArgs A) {
    constexpr int NV = KT<KC>::NV, DIM = KT<KC>::DIM, NLOC = KT<KC>::NLOC;
    constexpr int NINC = BWD_BLOCK * NV;
    // 3D Nedelec with weights read through the slot map: the slot records are
    // staged in LDS (24 KB; the workgroups per CU are bounded by registers
    // anyway). For the other kinds the extra LDS would cost occupancy.
    constexpr bool SLOTS = MODE != BWD_QUADRATIC && KC == 2;
    __shared__ double sh[NINC * DIM];
    __shared__ uint32_t s_inc_w[NINC / 2];          // incidences, two u16 per word
    __shared__ uint32_t s_pst_w[NINC / 2 + 64];     // pair starts, from the even index at or below the first
    __shared__ int32_t s_base[SLOTS ? BWD_BLOCK * NLOC : 1];
    __shared__ uint64_t s_cp[SLOTS ? BWD_BLOCK * NLOC : 1];
    // XCD-aware element order: workgroup b runs on XCD b % 8, so give each XCD
    // a contiguous range of elements; neighbouring elements share rows of the
    // upstream weights, and that reuse then stays in one L2.
    const int64_t per = gridDim.x / 8;
    const int64_t blk = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    const int64_t e0 = blk * BWD_BLOCK;
    if (e0 >= A.T) return;  // whole workgroup
    const int64_t e = e0 + threadIdx.x;
    const bool live = e < A.T;
    const int n_inc = (int)((A.T - e0 < BWD_BLOCK ? A.T - e0 : BWD_BLOCK) * NV);
    const int lane = (int)threadIdx.x & 63;
    const int wave0 = (int)threadIdx.x & ~63;  // first lane of the wavefront (uniform)
    int pb0 = 0, np = 0;
    const uint16_t* s_inc = reinterpret_cast<const uint16_t*>(s_inc_w);
    const uint16_t* s_pst = reinterpret_cast<const uint16_t*>(s_pst_w);
    if (A.partials) {
        // The workgroup's part of the node map goes straight from memory into
        // LDS (global_load_lds: no registers, no wait before the barrier that
        // precedes its use), so its loads are in flight while the elements
        // are computed. Words past the list's end read the last word again.
        pb0 = A.bptr[blk];
        np = A.bptr[blk + 1] - pb0;
        const uint32_t* w = reinterpret_cast<const uint32_t*>(A.inc + e0 * NV);  // 4-byte aligned: e0 * NV is even
        const int n_w = (n_inc + 1) / 2;
        for (int j = wave0; j < n_w; j += BWD_BLOCK)
            __builtin_amdgcn_global_load_lds(w + min(j + lane, n_w - 1),
                                             (__attribute__((address_space(3))) void*)(s_inc_w + j), 4, 0, 0);
        // pair starts from the even u16 index at or below pb0 (the list has
        // one u16 of padding, so the last word read is in bounds)
        const uint32_t* wp = reinterpret_cast<const uint32_t*>(A.pst + (pb0 & ~1));
        const int n_pw = (np + (pb0 & 1) + 1) / 2;
        for (int j = wave0; j < n_pw; j += BWD_BLOCK)
            __builtin_amdgcn_global_load_lds(wp + min(j + lane, n_pw - 1),
                                             (__attribute__((address_space(3))) void*)(s_pst_w + j), 4, 0, 0);
        s_pst += pb0 & 1;
    }
    if constexpr (SLOTS) {
        // the workgroup's slot records are contiguous (element-major): one
        // pass into LDS (as above) instead of a dependent load per row
        const int n_sl = n_inc / NV * NLOC;
        const uint32_t* wb = reinterpret_cast<const uint32_t*>(A.slot_base + e0 * NLOC);
        const uint32_t* wc = reinterpret_cast<const uint32_t*>(A.slot_cp + e0 * NLOC);
        uint32_t* lb = reinterpret_cast<uint32_t*>(s_base);
        uint32_t* lc = reinterpret_cast<uint32_t*>(s_cp);
        for (int j = wave0; j < n_sl; j += BWD_BLOCK)
            __builtin_amdgcn_global_load_lds(wb + min(j + lane, n_sl - 1),
                                             (__attribute__((address_space(3))) void*)(lb + j), 4, 0, 0);
        for (int j = wave0; j < 2 * n_sl; j += BWD_BLOCK)
            __builtin_amdgcn_global_load_lds(wc + min(j + lane, 2 * n_sl - 1),
                                             (__attribute__((address_space(3))) void*)(lc + j), 4, 0, 0);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
    const SlotView sv = SLOTS ? SlotView{s_base + (int)threadIdx.x * NLOC, s_cp + (int)threadIdx.x * NLOC}
                              : SlotView{A.slot_base + e * NLOC, A.slot_cp + e * NLOC};
    double2 gab = make_double2(0.0, 0.0);
    if (live) {
        if constexpr (KC == 2) gab = bwd_ned3<MODE>(A, e, sv, sh);
        else if constexpr (KC == 1) gab = bwd_rt3<MODE>(A, e, sv, sh);
        else gab = bwd_tri<MODE>(A, e, sv, sh);
    }
    if constexpr (MODE == BWD_QUADRATIC) {
        if (A.lpart) {  // uniform: the value of L as well (partials in element order)
            __shared__ double red[BWD_BLOCK];
            const double s = wg_tree_sum(live ? elem_value(A, e, gab) : 0.0, red);
            if (threadIdx.x == 0) A.lpart[blk] = s;
        }
    }
    if (!A.partials) return;  // uniform
    // the node map's loads into LDS are complete in every wavefront
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    // one partial per (vertex, workgroup): the workgroup's incidences of that
    // vertex, in ascending element order; incidence (lane, v) sits at
    // sh[(v * DIM + c) * BWD_BLOCK + lane]
    for (int j = (int)threadIdx.x; j < np; j += BWD_BLOCK) {
        int i0 = s_pst[j];
        int i1 = j + 1 < np ? s_pst[j + 1] : n_inc;
#if FEM_CHECK
        if (!fem_in_range(i0, n_inc + 1, A.err_word) || !fem_in_range(i1, n_inc + 1, A.err_word) ||
            !fem_in_range(pb0 + j, A.n_pairs, A.err_word))
            continue;
#endif
        double acc[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
        for (int i = i0; i < i1; ++i) {
            const int slot = s_inc[i];
            if (!fem_in_range(slot, n_inc, A.err_word)) continue;
            const int lane = slot / NV;
            const double* q = sh + lds_at(lane, slot - lane * NV, DIM);
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[c] += q[c * LDS_CS];
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) A.partials[(int64_t)(pb0 + j) * DIM + c] = acc[c];
    }
}

// gnodes[v] = sum of the node's (node, workgroup) partials, in ascending
// workgroup order (npair lists them by node).
template <int DIM>
__global__ __launch_bounds__(256) void k_node_reduce(const int32_t* node_ptr, const int32_t* npair,
                                                      const double* partials, int64_t V, double* gnodes,
                                                      int64_t n_pairs, int* err) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    double acc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
    const int64_t j1 = node_ptr[v + 1];
#pragma unroll 4
    for (int64_t j = node_ptr[v]; j < j1; ++j) {
        if (!fem_in_range(j, n_pairs, err)) break;
        const int64_t q = npair[j];
        if (!fem_in_range(q, n_pairs, err)) continue;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += partials[q * DIM + c];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) gnodes[v * DIM + c] = acc[c];
}

// Value of the quadratic form L = u^T (K(a) + M(b)) u. It is linear in the
// coefficients, so L = sum_e (a_e dL/da_e + b_e dL/db_e), with dL/da_e, dL/db_e
// the element sums of squares of the adjoint (no assembled matrix is read).
// Each workgroup adds its elements' terms in a fixed tree order into one
// partial; k_sum_partials then adds the partials in a fixed order, so the value
// is deterministic.
template <int KC>
__global__ __launch_bounds__(BWD_BLOCK) void k_quadratic_value(const BwdArgs A, double* partials) {
    __shared__ double red[BWD_BLOCK];
    const int64_t e = (int64_t)blockIdx.x * BWD_BLOCK + threadIdx.x;
    double v = 0.0;
    if (e < A.T) {
        const SlotView sv{nullptr, nullptr};
        double2 g;
        if constexpr (KC == 2) g = bwd_ned3<BWD_QUADRATIC>(A, e, sv, nullptr);
        else if constexpr (KC == 1) g = bwd_rt3<BWD_QUADRATIC>(A, e, sv, nullptr);
        else g = bwd_tri<BWD_QUADRATIC>(A, e, sv, nullptr);
        v = elem_value(A, e, g);
    }
    const double s = wg_tree_sum(v, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[0] = sum of n partials: lane t adds t, t + 256, ... in order, then a
// fixed tree over the lanes (one workgroup of 256).
__global__ __launch_bounds__(256) void k_sum_partials(const double* partials, int64_t n, double* out) {
    __shared__ double red[256];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) v += partials[i];
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

int64_t quadratic_value_partials(int64_t n_elems) { return (n_elems + BWD_BLOCK - 1) / BWD_BLOCK; }

fem_status launch_quadratic_value(fem_mesh m, DofSet& ds, fem_kind kind, const double* nodes,
                                  const double* a, const double* b, const double* u, double* out,
                                  double* partials, hipStream_t s) {
    const int kc = kind_code(m->dim, kind);
    BwdArgs A = {};
    A.u = u;
    A.elems2dofs = ds.elems2dofs;
    A.elems = m->elems;
    A.nodes = nodes;
    A.a = a;
    A.b = b;
    A.T = m->T;
    A.err_word = m->err_word;
    A.V = m->V;
    A.n_dofs = ds.pat.n_rows;
    A.nnz = ds.pat.nnz;
    A.n_pairs = m->bwd_pairs;
    const int64_t nb = quadratic_value_partials(m->T);
    if (nb > 0) {
        if (kc == 2) hipLaunchKernelGGL(k_quadratic_value<2>, dim3((unsigned)nb), dim3(BWD_BLOCK), 0, s, A, partials);
        else if (kc == 1) hipLaunchKernelGGL(k_quadratic_value<1>, dim3((unsigned)nb), dim3(BWD_BLOCK), 0, s, A, partials);
        else hipLaunchKernelGGL(k_quadratic_value<0>, dim3((unsigned)nb), dim3(BWD_BLOCK), 0, s, A, partials);
        FEM_HIP(hipGetLastError());
    }
    return launch_sum_partials(partials, nb, out, s);
}

fem_status launch_sum_partials(const double* partials, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, n, out);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static fem_status zero_f64(double* p, int64_t n, hipStream_t s) {
    if (!p || n <= 0) return FEM_OK;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, 0.0);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

template <int KC, int MODE>
static void launch_bwd_t(const BwdArgs& A, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_backward<KC, MODE>), dim3(grid), dim3(BWD_BLOCK), 0, s, A);
}

template <int MODE>
static void launch_bwd_mode(int kc, const BwdArgs& A, unsigned grid, hipStream_t s) {
    if (kc == 2) launch_bwd_t<2, MODE>(A, grid, s);
    else if (kc == 1) launch_bwd_t<1, MODE>(A, grid, s);
    else launch_bwd_t<0, MODE>(A, grid, s);
}

fem_status launch_backward(fem_mesh m, DofSet& ds, fem_kind kind, const double* nodes,
                           const double* a, const double* b, const double* gK, const double* gM,
                           const double* u, double* ga, double* gb, double* gnodes, double* L,
                           hipStream_t s) {
    const int kc = kind_code(m->dim, kind);
    if (L && !u) return fail(FEM_EINVAL, "the value of L comes with the quadratic-form adjoint only");
    if (L && !m->qv_partials)
        FEM_HIP(dmalloc(m, &m->qv_partials, std::max<int64_t>(1, quadratic_value_partials(m->T))));
    if (!u && !gK && !gM) {  // L = 0: every derivative is zero
        if (fem_status st = zero_f64(ga, m->T, s)) return st;
        if (fem_status st = zero_f64(gb, m->T, s)) return st;
        return zero_f64(gnodes, m->V * m->dim, s);
    }
    if (!u)
        if (fem_status st = build_slot_map(m, ds, s)) return st;
    if (gnodes) {
        if (fem_status st = build_node_map(m, s)) return st;
        if (!m->elem_partials) FEM_HIP(dmalloc(m, &m->elem_partials, std::max<int64_t>(m->bwd_pairs, 1) * m->dim));
    }
    BwdArgs A;
    A.u = u;
    A.elems2dofs = ds.elems2dofs;
    A.elems = m->elems;
    A.nodes = nodes;
    A.a = a;
    A.b = b;
    A.gK = gK;
    A.gM = gM;
    A.slot_base = ds.slot_base;
    A.slot_cp = ds.slot_cp;
    A.ga = ga;
    A.gb = gb;
    A.lpart = L ? m->qv_partials : nullptr;
    A.partials = gnodes ? m->elem_partials : nullptr;
    A.bptr = m->bwd_bptr;
    A.pst = m->bwd_pst;
    A.inc = m->bwd_inc;
    A.T = m->T;
    A.err_word = m->err_word;
    A.V = m->V;
    A.n_dofs = ds.pat.n_rows;
    A.nnz = ds.pat.nnz;
    A.n_pairs = m->bwd_pairs;
    const unsigned grid = (unsigned)(((m->T + BWD_BLOCK - 1) / BWD_BLOCK + 7) / 8 * 8);
    if (m->T > 0) {
        if (u) launch_bwd_mode<BWD_QUADRATIC>(kc, A, grid, s);
        else if (gK == gM) launch_bwd_mode<BWD_SAME>(kc, A, grid, s);
        else launch_bwd_mode<BWD_SEPARATE>(kc, A, grid, s);
        FEM_HIP(hipGetLastError());
    }
    if (L)
        if (fem_status st = launch_sum_partials(m->qv_partials, quadratic_value_partials(m->T), L, s)) return st;
    if (gnodes && m->V > 0) {
        const unsigned gv = (unsigned)((m->V + 255) / 256);
        if (m->dim == 3)
            hipLaunchKernelGGL(k_node_reduce<3>, dim3(gv), dim3(256), 0, s, m->node_ptr, m->bwd_npair,
                               m->elem_partials, m->V, gnodes, m->bwd_pairs, m->err_word);
        else
            hipLaunchKernelGGL(k_node_reduce<2>, dim3(gv), dim3(256), 0, s, m->node_ptr, m->bwd_npair,
                               m->elem_partials, m->V, gnodes, m->bwd_pairs, m->err_word);
        FEM_HIP(hipGetLastError());
    }
    return FEM_OK;
}

}  // namespace fem
