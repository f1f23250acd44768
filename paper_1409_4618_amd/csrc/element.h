// Per-element geometry and exact local matrices of the lowest-order edge
// elements, in FP64 registers.
//
// The local matrices of Section 2.4 (Anjam & Valdman) are integrals over the
// reference element of Piola-mapped (Sections 2.1, 2.2), sign-adjusted
// (Section 2.3) reference basis functions. All integrands are polynomials of
// degree <= 2, so the integrals have closed forms; the forms used here are:
//
//  Notation: local nodes x0..xd, b_j = x_j - x0 (columns of B_K), J = det B_K,
//  c_a = J grad(lambda_a) (cofactor vectors, c_0 = -(c_1 + ... + c_d)),
//  G_ab = c_a . c_b, s = sign data.
//
//  Nedelec 3D, local edge k = (i -> j) of Figure 1, l = (m -> n):
//    the reference basis is the Whitney form lambda_i grad lambda_j -
//    lambda_j grad lambda_i, so with int lambda_p lambda_q = |K|(1+d_pq)/20:
//      M_kl = s_k s_l [G_jn(1+d_im) - G_jm(1+d_in) - G_in(1+d_jm) + G_im(1+d_jn)]
//             / (120 |J|)
//    B_K times the reference curl of edge k is twice the vector of the opposite
//    edge, o_k, so  K_kl = s_k s_l (2 / (3|J|)) o_k . o_l
//    (edge vectors, no inverse: accurate also on flat elements).
//  Nedelec 2D (and 2D Raviart-Thomas, whose matrices are identical):
//      M_kl as above with 24 in place of 120, K_kl = s_k s_l 2 / |J|.
//  Raviart-Thomas 3D, face k opposite node p_k = 3 - k, basis x - p_k mapped by
//  B_K (flux 1/2 per face, as printed): with y_a = x_a - x0, S = y1 + y2 + y3,
//  u_p = S . y_p, Y_pq = y_p . y_q (y_0 = 0):
//      M_kl = s_k s_l [|S|^2 + tr Y - 5 (u_pk + u_pl) + 20 Y_pk,pl] / (120 |J|)
//      K_kl = s_k s_l 3 / (2 |J|).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fem {

// Local edge tables, packed 4 bits per edge (edge k in bits 4k..4k+3).
// 3D (Figure 1): 1->2, 1->3, 1->4, 2->3, 3->4, 4->2 (0-based 0->1 ... 3->1).
constexpr uint32_t NED3_START = 0x321000u;
constexpr uint32_t NED3_END = 0x132321u;
// 2D: edge k runs from node k+1 to node k+2 (cyclic), Section 3.
constexpr uint32_t TRI_START = 0x021u;
constexpr uint32_t TRI_END = 0x102u;

__host__ __device__ constexpr int nib(uint32_t packed, int k) { return (packed >> (4 * k)) & 0xF; }

struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
// Dot products with fused multiply-adds: one rounding less per term than
// separate products and sums, and fma(a, b, c) == fma(b, a, c) exactly, so
// dot(a, b) == dot(b, a) bitwise (symmetric Gram entries and local matrices).
__device__ __forceinline__ double dot(V3 a, V3 b) { return fma(a.x, b.x, fma(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 neg(V3 a) { return {-a.x, -a.y, -a.z}; }

// Per-lane selection v[k] with a runtime k, written as a one-hot weighted sum:
// exact for finite values (x * 1 + 0 = x) and, unlike a chain of selects, never
// turned by the compiler into a dynamically indexed stack array (scratch).
__device__ __forceinline__ double onehot(int k, int q) { return k == q ? 1.0 : 0.0; }
__device__ __forceinline__ double pick4d(const double v[4], int k) {
    double r = onehot(k, 0) * v[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) r = fma(onehot(k, q), v[q], r);
    return r;
}
__device__ __forceinline__ V3 pick4(const V3 v[4], int k) {
    const double w0 = onehot(k, 0);
    V3 r = {w0 * v[0].x, w0 * v[0].y, w0 * v[0].z};
#pragma unroll
    for (int q = 1; q < 4; ++q) {
        const double w = onehot(k, q);
        r = {fma(w, v[q].x, r.x), fma(w, v[q].y, r.y), fma(w, v[q].z, r.z)};
    }
    return r;
}
__device__ __forceinline__ V3 pick6(const V3 v[6], int k) {
    const double w0 = onehot(k, 0);
    V3 r = {w0 * v[0].x, w0 * v[0].y, w0 * v[0].z};
#pragma unroll
    for (int q = 1; q < 6; ++q) {
        const double w = onehot(k, q);
        r = {fma(w, v[q].x, r.x), fma(w, v[q].y, r.y), fma(w, v[q].z, r.z)};
    }
    return r;
}
__device__ __forceinline__ double pick6d(const double v[6], int k) {
    double r = onehot(k, 0) * v[0];
#pragma unroll
    for (int q = 1; q < 6; ++q) r = fma(onehot(k, q), v[q], r);
    return r;
}

// Materialise a value in a register: an empty asm statement the compiler cannot
// look through, so a product passed through it is rounded on its own and never
// fused into a following add.
__device__ __forceinline__ double rounded(double x) {
    asm("" : "+v"(x));
    return x;
}

// (T1 + T4) - (T2 + T3) of the Whitney mass term with every product rounded
// on its own (no FMA contraction): swapping k and l swaps T2 and T3 only, so
// the local mass matrix is bitwise symmetric.
__device__ __forceinline__ double whitney_term(double t1, double t4, double t2, double t3) {
    return (rounded(t1) + rounded(t4)) - (rounded(t2) + rounded(t3));
}

// ---------------------------------------------------------------------------
// 3D geometry: b_j, cofactor vectors c_a = J grad(lambda_a), J.
struct Geo3 {
    V3 b1, b2, b3;
    V3 c[4];
    double J;
};

__device__ __forceinline__ Geo3 geo3(const V3 x[4]) {
    Geo3 g;
    g.b1 = sub(x[1], x[0]);
    g.b2 = sub(x[2], x[0]);
    g.b3 = sub(x[3], x[0]);
    g.c[1] = cross(g.b2, g.b3);
    g.c[2] = cross(g.b3, g.b1);
    g.c[3] = cross(g.b1, g.b2);
    g.c[0] = neg(add(add(g.c[1], g.c[2]), g.c[3]));
    g.J = dot(g.b1, g.c[1]);
    return g;
}

// Opposite-edge vectors o_k of the 3D Nedelec curls (B_K curl_ref eta_k = 2 o_k).
__device__ __forceinline__ void ned3_o(const Geo3& g, V3 o[6]) {
    o[0] = sub(g.b3, g.b2);
    o[1] = sub(g.b1, g.b3);
    o[2] = sub(g.b2, g.b1);
    o[3] = g.b3;
    o[4] = g.b1;
    o[5] = g.b2;
}

// Sign data of the 6 local edges from the global node ids.
__device__ __forceinline__ void ned3_signs(const int gid[4], double s[6]) {
#pragma unroll
    for (int l = 0; l < 6; ++l) s[l] = gid[nib(NED3_START, l)] > gid[nib(NED3_END, l)] ? 1.0 : -1.0;
}

// Row k (runtime) of the 3D Nedelec local a K and b M, in the canonical
// rounding described at the end of this file.
__device__ __forceinline__ void ned3_row(const Geo3& g, const double s[6], int k, double ca,
                                         double cb, double Kr[6], double Mr[6]) {
    V3 o[6];
    ned3_o(g, o);
    const double inv = 1.0 / fabs(g.J);
    const double sk = pick6d(s, k);
    const V3 ok = pick6(o, k);
    const int i = nib(NED3_START, k);
    const int j = nib(NED3_END, k);
    // Gram matrix of the cofactor vectors, each entry computed once (so that
    // G_ab and G_ba are the same value), then rows i and j picked exactly.
    double G[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) G[a][b] = G[b][a] = dot(g.c[a], g.c[b]);
    double Gi[4], Gj[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double col[4] = {G[0][a], G[1][a], G[2][a], G[3][a]};
        Gi[a] = pick4d(col, i);
        Gj[a] = pick4d(col, j);
    }
    const double kr = sk * (ca * ((2.0 / 3.0) * inv));
    const double mr = sk * (cb * ((1.0 / 120.0) * inv));
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const int m = nib(NED3_START, l);
        const int n = nib(NED3_END, l);
        Kr[l] = (s[l] * kr) * dot(ok, o[l]);
        const double t = whitney_term(Gj[n] * (1.0 + (i == m)), Gi[m] * (1.0 + (j == n)),
                                      Gj[m] * (1.0 + (i == n)), Gi[n] * (1.0 + (j == m)));
        Mr[l] = (s[l] * mr) * t;
    }
}

// ---------------------------------------------------------------------------
// 3D Raviart-Thomas: face signs = -(parity of local order -> (sorted face, opposite)).
__device__ __forceinline__ void rt3_signs(const int gid[4], double s[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int p = 3 - k;  // opposite node of face k
        // face nodes in increasing local order: {0,1,2,3} \ {p}
        const int u = (p == 0) ? 1 : 0;
        const int v = (p <= 1) ? 2 : 1;
        const int w = (p <= 2) ? 3 : 2;
        const int inv = (gid[u] > gid[v]) + (gid[u] > gid[w]) + (gid[v] > gid[w]) + (3 - p);
        s[k] = (inv & 1) ? 1.0 : -1.0;  // odd permutation -> parity -1 -> sign +1
    }
}

struct GeoRT3 {
    V3 y[4];       // y_a = x_a - x0 (y_0 = 0)
    double J;
    double base;   // |S|^2 + tr Y
    double u[4];   // S . y_p
};

__device__ __forceinline__ GeoRT3 geo_rt3(const V3 x[4]) {
    GeoRT3 g;
    g.y[0] = {0.0, 0.0, 0.0};
    g.y[1] = sub(x[1], x[0]);
    g.y[2] = sub(x[2], x[0]);
    g.y[3] = sub(x[3], x[0]);
    g.J = dot(g.y[1], cross(g.y[2], g.y[3]));
    const V3 S = add(add(g.y[1], g.y[2]), g.y[3]);
    g.base = dot(S, S) + dot(g.y[1], g.y[1]) + dot(g.y[2], g.y[2]) + dot(g.y[3], g.y[3]);
    g.u[0] = 0.0;
#pragma unroll
    for (int a = 1; a < 4; ++a) g.u[a] = dot(S, g.y[a]);
    return g;
}

__device__ __forceinline__ void rt3_row(const GeoRT3& g, const double s[4], int k, double ca,
                                        double cb, double Kr[4], double Mr[4]) {
    const double inv = 1.0 / fabs(g.J);
    const double sk = pick4d(s, k);
    const int pk = 3 - k;
    const V3 ypk = pick4(g.y, pk);
    const double upk = pick4d(g.u, pk);
    const double kr = sk * (ca * (1.5 * inv));
    const double mr = sk * (cb * ((1.0 / 120.0) * inv));
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int pl = 3 - l;
        Kr[l] = s[l] * kr;
        const double t = g.base - 5.0 * (upk + g.u[pl]) + 20.0 * dot(ypk, g.y[pl]);
        Mr[l] = (s[l] * mr) * t;
    }
}

// ---------------------------------------------------------------------------
// 2D (Nedelec; the 2D Raviart-Thomas matrices are the same).
struct V2 {
    double x, y;
};
struct Geo2 {
    V2 b1, b2;
    V2 c[3];
    double J;
};

__device__ __forceinline__ Geo2 geo2(const V2 x[3]) {
    Geo2 g;
    g.b1 = {x[1].x - x[0].x, x[1].y - x[0].y};
    g.b2 = {x[2].x - x[0].x, x[2].y - x[0].y};
    g.J = g.b1.x * g.b2.y - g.b1.y * g.b2.x;
    g.c[1] = {g.b2.y, -g.b2.x};
    g.c[2] = {-g.b1.y, g.b1.x};
    g.c[0] = {-(g.c[1].x + g.c[2].x), -(g.c[1].y + g.c[2].y)};
    return g;
}

__device__ __forceinline__ void tri_signs(const int gid[3], double s[3]) {
#pragma unroll
    for (int l = 0; l < 3; ++l) s[l] = gid[nib(TRI_START, l)] > gid[nib(TRI_END, l)] ? 1.0 : -1.0;
}

__device__ __forceinline__ double dot2(V2 a, V2 b) { return fma(a.x, b.x, a.y * b.y); }

__device__ __forceinline__ void tri_row(const Geo2& g, const double s[3], int k, double ca,
                                        double cb, double Kr[3], double Mr[3]) {
    const double inv = 1.0 / fabs(g.J);
    const double sk = onehot(k, 0) * s[0] + onehot(k, 1) * s[1] + onehot(k, 2) * s[2];
    const int i = nib(TRI_START, k);
    const int j = nib(TRI_END, k);
    // Gram matrix of the cofactor vectors, each entry computed once, rows i and
    // j picked exactly (G_ab and G_ba are the same value).
    double G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) G[a][b] = G[b][a] = dot2(g.c[a], g.c[b]);
    double Gi[3], Gj[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Gi[a] = onehot(i, 0) * G[0][a] + onehot(i, 1) * G[1][a] + onehot(i, 2) * G[2][a];
        Gj[a] = onehot(j, 0) * G[0][a] + onehot(j, 1) * G[1][a] + onehot(j, 2) * G[2][a];
    }
    const double kr = sk * (ca * (2.0 * inv));
    const double mr = sk * (cb * ((1.0 / 24.0) * inv));
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int m = nib(TRI_START, l);
        const int n = nib(TRI_END, l);
        Kr[l] = s[l] * kr;
        const double t = whitney_term(Gj[n] * (1.0 + (i == m)), Gi[m] * (1.0 + (j == n)),
                                      Gj[m] * (1.0 + (i == n)), Gi[n] * (1.0 + (j == m)));
        Mr[l] = (s[l] * mr) * t;
    }
}

}  // namespace fem

namespace fem {

// ---------------------------------------------------------------------------
// Canonical rounding of the scaled local entries (shared by the row functions
// above and the element states below, so every kernel produces bitwise the
// same values):
//   a K_kl = (s_l * (s_k * (a * kf))) * q_kl,   b M_kl = (s_l * (s_k * (b * mf))) * t_kl
// with kf, mf the kind's factors times 1/|J| (rounded once), q_kl the
// curl/div term (o_k . o_l for 3D Nedelec, 1 otherwise) and t_kl the mass
// term. Sign factors are +-1, so multiplying by them is exact and (k, l),
// (l, k) give bitwise equal values; q and t are symmetric by construction.
//
// Element state for the element-major kernel: the geometric quantities the
// rows are formed from, kept in registers while the kernel makes one pass for
// K and one for M. Entries are produced one at a time with compile-time
// (k, l).
__host__ __device__ constexpr int tri_index(int a, int b) {  // packed upper triangle of a 4x4
    return a <= b ? a * 4 - a * (a + 1) / 2 + b : b * 4 - b * (b + 1) / 2 + a;
}

__device__ __forceinline__ double sgn_bit(uint32_t bits, int l) {
    return ((bits >> l) & 1u) ? 1.0 : -1.0;
}

// s_l * x as a flip of the sign bit (neg = 0x80000000 iff s_l = -1): bitwise
// the product with +-1.0, without a floating-point multiply.
// x with its sign flipped where neg has the sign bit set. Round-to-nearest is
// symmetric under negation, so with_sign(r * t, neg) == with_sign(r, neg) * t
// bitwise; entries flip the sign of the product, which leaves the low word in
// place.
__device__ __forceinline__ double with_sign(double x, uint32_t neg) {
    return __hiloint2double(__double2hiint(x) ^ (int)neg, __double2loint(x));
}
__device__ __forceinline__ uint32_t neg_mask(uint32_t sbits, int l) {
    return ((~sbits) << (31 - l)) & 0x80000000u;
}

struct Ned3Elem {
    V3 b1, b2, b3;  // x_j - x_0
    double ka, mb;  // a * 2/(3|J|), b * 1/(120|J|)
    double J;
    uint32_t sbits;  // bit l set iff s_l = +1
    uint32_t nm[6];  // sign-bit masks of the s_l
};

// What the mass rows need: the Gram matrix of the cofactor vectors. It is
// formed from b_1..b_3 only when the mass pass starts, so the registers of the
// stiffness pass and of the mass pass are not live at the same time.
struct Ned3Mass {
    double G[10];  // G_ab = c_a . c_b, packed upper triangle
    double mb;
    uint32_t sbits;
    uint32_t nm[6];
};

__device__ __forceinline__ Ned3Elem ned3_elem(const V3 x[4], const int gid[4], double ca,
                                              double cb) {
    Ned3Elem e;
    e.b1 = sub(x[1], x[0]);
    e.b2 = sub(x[2], x[0]);
    e.b3 = sub(x[3], x[0]);
    e.J = dot(e.b1, cross(e.b2, e.b3));
    const double inv = 1.0 / fabs(e.J);
    e.ka = ca * ((2.0 / 3.0) * inv);
    e.mb = cb * ((1.0 / 120.0) * inv);
    e.sbits = 0;
#pragma unroll
    for (int l = 0; l < 6; ++l)
        e.sbits |= (gid[nib(NED3_START, l)] > gid[nib(NED3_END, l)] ? 1u : 0u) << l;
#pragma unroll
    for (int l = 0; l < 6; ++l) e.nm[l] = neg_mask(e.sbits, l);
    return e;
}

// Same cofactor vectors and Gram entries as geo3 / ned3_row.
__device__ __forceinline__ Ned3Mass ned3_mass(const Ned3Elem& e) {
    V3 c[4];
    c[1] = cross(e.b2, e.b3);
    c[2] = cross(e.b3, e.b1);
    c[3] = cross(e.b1, e.b2);
    c[0] = neg(add(add(c[1], c[2]), c[3]));
    Ned3Mass m;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) m.G[tri_index(a, b)] = dot(c[a], c[b]);
    m.mb = e.mb;
    m.sbits = e.sbits;
#pragma unroll
    for (int l = 0; l < 6; ++l) m.nm[l] = e.nm[l];
    return m;
}

template <int k>
__device__ __forceinline__ V3 ned3_o_of(const Ned3Elem& e) {
    if constexpr (k == 0) return sub(e.b3, e.b2);
    else if constexpr (k == 1) return sub(e.b1, e.b3);
    else if constexpr (k == 2) return sub(e.b2, e.b1);
    else if constexpr (k == 3) return e.b3;
    else if constexpr (k == 4) return e.b1;
    else return e.b2;
}

// row scale s_k * (a kf) of the stiffness pass, s_k * (b mf) of the mass pass
template <int k>
__device__ __forceinline__ double ned3_krow(const Ned3Elem& e) {
    return with_sign(e.ka, e.nm[k]);
}
template <int k>
__device__ __forceinline__ double ned3_mrow(const Ned3Mass& e) {
    return with_sign(e.mb, e.nm[k]);
}

template <int k, int l>
__device__ __forceinline__ double ned3_K(const Ned3Elem& e, double kr) {
    return with_sign(kr * dot(ned3_o_of<k>(e), ned3_o_of<l>(e)), e.nm[l]);
}

template <int k, int l>
__device__ __forceinline__ double ned3_M(const Ned3Mass& e, double mr) {
    constexpr int i = nib(NED3_START, k), j = nib(NED3_END, k);
    constexpr int m = nib(NED3_START, l), n = nib(NED3_END, l);
    const double t = whitney_term(e.G[tri_index(j, n)] * (1.0 + (i == m)),
                                  e.G[tri_index(i, m)] * (1.0 + (j == n)),
                                  e.G[tri_index(j, m)] * (1.0 + (i == n)),
                                  e.G[tri_index(i, n)] * (1.0 + (j == m)));
    return with_sign(mr * t, e.nm[l]);
}

struct Rt3Elem {
    V3 y1, y2, y3;  // x_a - x_0
    double base;    // |S|^2 + tr Y
    double u1, u2, u3;
    double ka, mb;  // a * 3/(2|J|), b * 1/(120|J|)
    double J;
    uint32_t sbits;
    uint32_t nm[4];
};

__device__ __forceinline__ Rt3Elem rt3_elem(const V3 x[4], const int gid[4], double ca,
                                            double cb) {
    const GeoRT3 g = geo_rt3(x);
    Rt3Elem e;
    e.y1 = g.y[1];
    e.y2 = g.y[2];
    e.y3 = g.y[3];
    e.base = g.base;
    e.u1 = g.u[1];
    e.u2 = g.u[2];
    e.u3 = g.u[3];
    const double inv = 1.0 / fabs(g.J);
    e.ka = ca * (1.5 * inv);
    e.mb = cb * ((1.0 / 120.0) * inv);
    e.J = g.J;
    double s[4];
    rt3_signs(gid, s);
    e.sbits = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) e.sbits |= (s[l] > 0.0 ? 1u : 0u) << l;
#pragma unroll
    for (int l = 0; l < 4; ++l) e.nm[l] = neg_mask(e.sbits, l);
    return e;
}

template <int p>
__device__ __forceinline__ V3 rt3_y(const Rt3Elem& e) {
    if constexpr (p == 0) return {0.0, 0.0, 0.0};
    else if constexpr (p == 1) return e.y1;
    else if constexpr (p == 2) return e.y2;
    else return e.y3;
}
template <int p>
__device__ __forceinline__ double rt3_u(const Rt3Elem& e) {
    if constexpr (p == 0) return 0.0;
    else if constexpr (p == 1) return e.u1;
    else if constexpr (p == 2) return e.u2;
    else return e.u3;
}

template <int k>
__device__ __forceinline__ double rt3_krow(const Rt3Elem& e) {
    return with_sign(e.ka, e.nm[k]);
}
template <int k>
__device__ __forceinline__ double rt3_mrow(const Rt3Elem& e) {
    return with_sign(e.mb, e.nm[k]);
}

template <int k, int l>
__device__ __forceinline__ double rt3_K(const Rt3Elem& e, double kr) {
    return with_sign(kr, e.nm[l]);
}

template <int k, int l>
__device__ __forceinline__ double rt3_M(const Rt3Elem& e, double mr) {
    constexpr int pk = 3 - k, pl = 3 - l;
    const double t = e.base - 5.0 * (rt3_u<pk>(e) + rt3_u<pl>(e)) + 20.0 * dot(rt3_y<pk>(e), rt3_y<pl>(e));
    return with_sign(mr * t, e.nm[l]);
}

struct TriElem {
    double G[6];  // packed upper triangle of the 3x3 Gram of the cofactor vectors
    double ka, mb;  // a * 2/|J|, b * 1/(24|J|)
    double J;
    uint32_t sbits;
    uint32_t nm[3];
};

__host__ __device__ constexpr int tri3_index(int a, int b) {
    return a <= b ? a * 3 - a * (a + 1) / 2 + b : b * 3 - b * (b + 1) / 2 + a;
}

__device__ __forceinline__ TriElem tri_elem(const V2 x[3], const int gid[3], double ca, double cb) {
    const Geo2 g = geo2(x);
    TriElem e;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) e.G[tri3_index(a, b)] = dot2(g.c[a], g.c[b]);
    const double inv = 1.0 / fabs(g.J);
    e.ka = ca * (2.0 * inv);
    e.mb = cb * ((1.0 / 24.0) * inv);
    e.J = g.J;
    e.sbits = 0;
#pragma unroll
    for (int l = 0; l < 3; ++l)
        e.sbits |= (gid[nib(TRI_START, l)] > gid[nib(TRI_END, l)] ? 1u : 0u) << l;
#pragma unroll
    for (int l = 0; l < 3; ++l) e.nm[l] = neg_mask(e.sbits, l);
    return e;
}

template <int k>
__device__ __forceinline__ double tri_krow(const TriElem& e) {
    return with_sign(e.ka, e.nm[k]);
}
template <int k>
__device__ __forceinline__ double tri_mrow(const TriElem& e) {
    return with_sign(e.mb, e.nm[k]);
}

template <int k, int l>
__device__ __forceinline__ double tri_K(const TriElem& e, double kr) {
    return with_sign(kr, e.nm[l]);
}

template <int k, int l>
__device__ __forceinline__ double tri_M(const TriElem& e, double mr) {
    constexpr int i = nib(TRI_START, k), j = nib(TRI_END, k);
    constexpr int m = nib(TRI_START, l), n = nib(TRI_END, l);
    const double t = whitney_term(e.G[tri3_index(j, n)] * (1.0 + (i == m)),
                                  e.G[tri3_index(i, m)] * (1.0 + (j == n)),
                                  e.G[tri3_index(j, m)] * (1.0 + (i == n)),
                                  e.G[tri3_index(i, n)] * (1.0 + (j == m)));
    return with_sign(mr * t, e.nm[l]);
}

}  // namespace fem

namespace fem {

// Re-materialisation barrier: a value passed through this is, to the compiler,
// a new value in each place it is called. The element-major kernel pins its
// element state at the top of each local row, so the compiler forms that row's
// entries there instead of hoisting the entries shared by two rows (the same
// (k, l) pair) above both rows and holding all of them in registers.
__device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(V3& v) {
    pin(v.x);
    pin(v.y);
    pin(v.z);
}

template <bool MASS>
__device__ __forceinline__ void pin_state(Ned3Elem& e) {
    pin(e.b1);
    pin(e.b2);
    pin(e.b3);
    pin(e.ka);
}
template <bool MASS>
__device__ __forceinline__ void pin_state(Ned3Mass& e) {
#pragma unroll
    for (int q = 0; q < 10; ++q) pin(e.G[q]);
    pin(e.mb);
}
template <bool MASS>
__device__ __forceinline__ void pin_state(Rt3Elem& e) {
    if constexpr (MASS) {
        pin(e.y1);
        pin(e.y2);
        pin(e.y3);
        pin(e.base);
        pin(e.u1);
        pin(e.u2);
        pin(e.u3);
        pin(e.mb);
    } else {
        pin(e.ka);
    }
}
template <bool MASS>
__device__ __forceinline__ void pin_state(TriElem& e) {
    if constexpr (MASS) {
#pragma unroll
        for (int q = 0; q < 6; ++q) pin(e.G[q]);
        pin(e.mb);
    } else {
        pin(e.ka);
    }
}

}  // namespace fem
