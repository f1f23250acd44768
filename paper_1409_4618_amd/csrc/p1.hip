// Linear nodal (P1) elements: the approximation v of the Poisson problem that
// the majorant of Section 4.1 estimates (the paper computes it with linear
// nodal elements). The nodal CSR pattern, the stiffness matrix
// K_ij = sum_K a_K int_K grad(lambda_i) . grad(lambda_j), the load vector
// F_i = int f lambda_i, the elimination of boundary nodes (u = 0 on the
// boundary) and the energy error ||grad(u - v)||.
//
// Pattern: row i holds node i and its edge neighbours, columns ascending; it is
// built once from the edge list (a sort of the (row, column) keys).
// Stiffness: with c_a the cofactor vectors (c_a = J grad lambda_a) an element
// adds (c_a . c_b) / (d! |J|) to entry (a, b). An off-diagonal entry (i, j) is
// summed over the elements of edge {i, j} (the edge's slot list, ascending
// element order); a diagonal entry over the elements of node i (the node's
// incidence list, ascending element order): deterministic, no atomics.
#include <algorithm>

#include "element.h"
#include "fem_internal.h"
#include "quad.h"

namespace fem {

constexpr int P1_TB = 256;
static inline unsigned p1_blocks(int64_t n) { return (unsigned)((n + P1_TB - 1) / P1_TB); }

// ------------------------------------------------------------------ pattern
__global__ void k_p1_entry_keys(const int32_t* edges2nodes, int64_t E, int64_t V, uint64_t* keys, uint32_t* vals,
                                uint32_t* counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < E) {
        const uint64_t lo = (uint32_t)edges2nodes[2 * i], hi = (uint32_t)edges2nodes[2 * i + 1];
        keys[2 * i] = lo * (uint64_t)V + hi;
        keys[2 * i + 1] = hi * (uint64_t)V + lo;
        vals[2 * i] = vals[2 * i + 1] = 0u;
        atomicAdd(&counts[lo], 1u);
        atomicAdd(&counts[hi], 1u);
    } else if (i < E + V) {
        const uint64_t n = (uint64_t)(i - E);
        keys[E + i] = n * (uint64_t)V + n;  // positions 2E .. 2E + V - 1
        vals[E + i] = 0u;
        atomicAdd(&counts[n], 1u);
    }
}

__global__ void k_p1_colind(const uint64_t* keys, int64_t nnz, int64_t V, int32_t* colind) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) colind[p] = (int32_t)(keys[p] % (uint64_t)V);
}

__global__ void k_u32_to_i64(const uint32_t* a, int64_t n, int64_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i];
}

// incidence (slot = e * nv + v) keys: the node
__global__ void k_vertex_keys(const int32_t* elems, int64_t n, uint64_t* keys, uint32_t* vals, uint32_t* counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t node = (uint32_t)elems[i];
    keys[i] = node;
    vals[i] = (uint32_t)i;
    atomicAdd(&counts[node], 1u);
}

// boundary nodes: the nodes of facets that belong to one element
__global__ void k_boundary_nodes(const int32_t* rs_ptr, const int32_t* facet_nodes, int64_t n_facets, int npf,
                                 uint8_t* bnd) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_facets) return;
    if (rs_ptr[f + 1] - rs_ptr[f] == 1)
        for (int k = 0; k < npf; ++k) bnd[facet_nodes[f * npf + k]] = 1;
}

struct P1Build {
    uint64_t* keys = nullptr;
    uint64_t* keys_tmp = nullptr;
    uint32_t* vals = nullptr;
    uint32_t* vals_tmp = nullptr;
    uint32_t* counts = nullptr;
    hipError_t alloc(int64_t n, int64_t V) {
        hipError_t e;
        if ((e = hipMalloc((void**)&keys, std::max<int64_t>(n, 1) * sizeof(uint64_t))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&keys_tmp, std::max<int64_t>(n, 1) * sizeof(uint64_t))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&vals, std::max<int64_t>(n, 1) * sizeof(uint32_t))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&vals_tmp, std::max<int64_t>(n, 1) * sizeof(uint32_t))) != hipSuccess) return e;
        return hipMalloc((void**)&counts, (V + 1) * sizeof(uint32_t));
    }
    ~P1Build() {
        if (keys) (void)hipFree(keys);
        if (keys_tmp) (void)hipFree(keys_tmp);
        if (vals) (void)hipFree(vals);
        if (vals_tmp) (void)hipFree(vals_tmp);
        if (counts) (void)hipFree(counts);
    }
};

// The nodal pattern, the nodes' incidence lists and the boundary flags, built
// once; the handle keeps them only when every step has succeeded.
static fem_status build_p1(fem_mesh m, hipStream_t s) {
    if (m->p1_built) return FEM_OK;
    const int64_t V = m->V, E = m->edges.n, T = m->T;
    const int nv = m->dim + 1;
    const int64_t nnz = 2 * E + V;
    if (nnz >= (int64_t(1) << 31)) return fail(FEM_EOVERFLOW, "fem_p1_pattern: 2 n_edges + n_nodes >= 2^31");
    int64_t* rowptr = nullptr;
    int32_t *colind = nullptr, *vs_ptr = nullptr, *vs_slot = nullptr;
    uint8_t* bnd = nullptr;
    struct Keep {
        std::vector<void*> p;
        bool keep = false;
        ~Keep() {
            if (!keep)
                for (void* q : p) (void)hipFree(q);
        }
    } kp;
    auto dev = [&](void** ptr, size_t bytes) {
        hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
        if (e == hipSuccess) kp.p.push_back(*ptr);
        return e;
    };
    FEM_HIP(dev((void**)&rowptr, (V + 1) * sizeof(int64_t)));
    FEM_HIP(dev((void**)&colind, nnz * sizeof(int32_t)));
    FEM_HIP(dev((void**)&vs_ptr, (V + 1) * sizeof(int32_t)));
    FEM_HIP(dev((void**)&vs_slot, T * nv * sizeof(int32_t)));
    FEM_HIP(dev((void**)&bnd, V * sizeof(uint8_t)));
    const int64_t nmax = std::max<int64_t>(nnz, T * nv);
    P1Build b;
    FEM_HIP(b.alloc(nmax, V));
    // pattern
    FEM_HIP(hipMemsetAsync(b.counts, 0, (V + 1) * sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_p1_entry_keys, dim3(p1_blocks(E + V)), dim3(P1_TB), 0, s, m->edges2nodes, E, V, b.keys,
                       b.vals, b.counts);
    FEM_HIP(hipGetLastError());
    FEM_HIP(radix_sort_pairs(b.keys, b.vals, b.keys_tmp, b.vals_tmp, nnz, bit_length((uint64_t)V * (uint64_t)V - 1),
                             s));
    hipLaunchKernelGGL(k_p1_colind, dim3(p1_blocks(nnz)), dim3(P1_TB), 0, s, b.keys, nnz, V, colind);
    FEM_HIP(hipGetLastError());
    FEM_HIP(scan_exclusive_u32(b.counts, V + 1, s));
    hipLaunchKernelGGL(k_u32_to_i64, dim3(p1_blocks(V + 1)), dim3(P1_TB), 0, s, b.counts, V + 1, rowptr);
    FEM_HIP(hipGetLastError());
    // node incidence lists, ascending element order (stable sort by node)
    FEM_HIP(hipMemsetAsync(b.counts, 0, (V + 1) * sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_vertex_keys, dim3(p1_blocks(T * nv)), dim3(P1_TB), 0, s, m->elems, T * nv, b.keys, b.vals,
                       b.counts);
    FEM_HIP(hipGetLastError());
    FEM_HIP(radix_sort_pairs(b.keys, b.vals, b.keys_tmp, b.vals_tmp, T * nv, bit_length((uint64_t)V - 1), s));
    FEM_HIP(hipMemcpyAsync(vs_slot, b.vals, T * nv * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    FEM_HIP(scan_exclusive_u32(b.counts, V + 1, s));
    FEM_HIP(hipMemcpyAsync(vs_ptr, b.counts, (V + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    // boundary nodes
    FEM_HIP(hipMemsetAsync(bnd, 0, V * sizeof(uint8_t), s));
    if (m->dim == 3)
        hipLaunchKernelGGL(k_boundary_nodes, dim3(p1_blocks(m->faces.n)), dim3(P1_TB), 0, s, m->faces.rs_ptr,
                           m->faces2nodes, m->faces.n, 3, bnd);
    else
        hipLaunchKernelGGL(k_boundary_nodes, dim3(p1_blocks(E)), dim3(P1_TB), 0, s, m->edges.rs_ptr, m->edges2nodes,
                           E, 2, bnd);
    FEM_HIP(hipGetLastError());
    FEM_HIP(hipStreamSynchronize(s));
    for (void* q : kp.p) m->allocs.push_back(q);
    kp.keep = true;
    m->p1_rowptr = rowptr;
    m->p1_colind = colind;
    m->p1_nnz = nnz;
    m->vs_ptr = vs_ptr;
    m->vs_slot = vs_slot;
    m->bnd_nodes = bnd;
    m->p1_built = true;
    return FEM_OK;
}

// ------------------------------------------------------------------ stiffness
__device__ __forceinline__ int64_t find_col(const int64_t* rowptr, const int32_t* colind, int64_t row, int32_t col) {
    int64_t lo = rowptr[row], hi = rowptr[row + 1] - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (colind[mid] < col) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Sizes for the checked build: slots of the element lists, nonzeros, error word.
struct P1Bounds {
    int64_t n_slots, nnz;
    int* err;
};

// Checked build: position pos holds column col (else flagged, and the caller
// skips the store).
__device__ __forceinline__ bool p1_pos_ok(const int32_t* colind, int64_t pos, int32_t col, const P1Bounds& b) {
#if FEM_CHECK
    if (!fem_in_range(pos, b.nnz, b.err)) return false;
    if (colind[pos] != col) {
        atomicOr(b.err, ERR_BOUNDS);
        return false;
    }
#else
    (void)colind;
    (void)pos;
    (void)col;
    (void)b;
#endif
    return true;
}

// (c_a . c_b) / (d! |J|) of element e, times its coefficient
template <int DIM>
__device__ __forceinline__ double p1_entry(const int32_t* elems, const double* nodes, const double* a, int64_t e,
                                           int va, int vb) {
    int gid[DIM + 1];
    load_gid<DIM>(elems, e, gid);
    const QElem<DIM> g = q_elem<DIM>(nodes, gid);
    // rows va, vb of the cofactors, selected with compile-time indices (a
    // runtime index into the array would put it in scratch memory)
    double ca[DIM], cb[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) ca[c] = cb[c] = 0.0;
#pragma unroll
    for (int r = 0; r <= DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            ca[c] = r == va ? g.c[r][c] : ca[c];
            cb[c] = r == vb ? g.c[r][c] : cb[c];
        }
    double d = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) d += ca[c] * cb[c];
    const double fact = DIM == 2 ? 2.0 : 6.0;
    return (a ? a[e] : 1.0) * d / (fact * fabs(g.J));
}

// off-diagonal entries (lo, hi) and (hi, lo) of every edge
template <int DIM>
__global__ __launch_bounds__(P1_TB) void k_p1_offdiag(const int32_t* elems, const double* nodes, const double* a,
                                                      const int32_t* edges2nodes, const int32_t* rs_ptr,
                                                      const int32_t* rs_slot, int64_t E, const int64_t* rowptr,
                                                      const int32_t* colind, double* K, const P1Bounds bd) {
    constexpr int NE = DIM == 2 ? 3 : 6;
    const int64_t ed = (int64_t)blockIdx.x * P1_TB + threadIdx.x;
    if (ed >= E) return;
    double acc = 0.0;
    for (int j = rs_ptr[ed]; j < rs_ptr[ed + 1]; ++j) {
        if (!fem_in_range(j, bd.n_slots, bd.err)) break;
        const int64_t slot = rs_slot[j];
        if (!fem_in_range(slot, bd.n_slots, bd.err)) continue;
        const int64_t e = slot / NE;
        const int k = (int)(slot - e * NE);
        const int va = DIM == 2 ? nib(TRI_START, k) : nib(NED3_START, k);
        const int vb = DIM == 2 ? nib(TRI_END, k) : nib(NED3_END, k);
        acc += p1_entry<DIM>(elems, nodes, a, e, va, vb);
    }
    const int32_t lo = edges2nodes[2 * ed], hi = edges2nodes[2 * ed + 1];
    const int64_t p_lh = find_col(rowptr, colind, lo, hi), p_hl = find_col(rowptr, colind, hi, lo);
    if (p1_pos_ok(colind, p_lh, hi, bd)) K[p_lh] = acc;
    if (p1_pos_ok(colind, p_hl, lo, bd)) K[p_hl] = acc;
}

// diagonal entries: over the elements of each node
template <int DIM>
__global__ __launch_bounds__(P1_TB) void k_p1_diag(const int32_t* elems, const double* nodes, const double* a,
                                                   const int32_t* vs_ptr, const int32_t* vs_slot, int64_t V,
                                                   const int64_t* rowptr, const int32_t* colind, double* K,
                                                   const P1Bounds bd) {
    const int64_t i = (int64_t)blockIdx.x * P1_TB + threadIdx.x;
    if (i >= V) return;
    double acc = 0.0;
    for (int j = vs_ptr[i]; j < vs_ptr[i + 1]; ++j) {
        if (!fem_in_range(j, bd.n_slots, bd.err)) break;
        const int64_t slot = vs_slot[j];
        if (!fem_in_range(slot, bd.n_slots, bd.err)) continue;
        const int64_t e = slot / (DIM + 1);
        const int v = (int)(slot - e * (DIM + 1));
        acc += p1_entry<DIM>(elems, nodes, a, e, v, v);
    }
    const int64_t p = find_col(rowptr, colind, i, (int32_t)i);
    if (p1_pos_ok(colind, p, (int32_t)i, bd)) K[p] = acc;
}

// ------------------------------------------------------------------ load
template <int DIM>
__global__ __launch_bounds__(INT_BLOCK) void k_p1_load_local(const int32_t* elems, const double* nodes, int64_t T,
                                                             const QuadRule q, const FnArgs F, double* loc) {
    const int64_t e = (int64_t)blockIdx.x * INT_BLOCK + threadIdx.x;
    if (e >= T) return;
    int gid[DIM + 1];
    load_gid<DIM>(elems, e, gid);
    const QElem<DIM> g = q_elem<DIM>(nodes, gid);
    double acc[DIM + 1];
#pragma unroll
    for (int v = 0; v <= DIM; ++v) acc[v] = 0.0;
    for_points<DIM>(q, [&](const double* xh, double w) {
        double x[DIM], fv[3] = {0.0, 0.0, 0.0};
        phys_point<DIM>(g, xh, x);
        eval_fn<DIM>(F, x, fv);
        double l0 = 1.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            acc[d + 1] += w * fv[0] * xh[d];
            l0 -= xh[d];
        }
        acc[0] += w * fv[0] * l0;
    });
    const double aJ = fabs(g.J);
#pragma unroll
    for (int v = 0; v <= DIM; ++v) loc[e * (DIM + 1) + v] = acc[v] * aJ;
}

// (n_slots, err: the checked build's bounds of the list entries and slots)
__global__ __launch_bounds__(P1_TB) void k_list_sum(const int32_t* ptr, const int32_t* slot, const double* loc,
                                                    int64_t n, double* out, int64_t n_slots, int* err) {
    const int64_t i = (int64_t)blockIdx.x * P1_TB + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = ptr[i]; j < ptr[i + 1]; ++j) {
        if (!fem_in_range(j, n_slots, err)) break;
        const int q = slot[j];
        if (fem_in_range(q, n_slots, err)) acc += loc[q];
    }
    out[i] = acc;
}

// ------------------------------------------------------------------ boundary
__global__ __launch_bounds__(P1_TB) void k_p1_dirichlet(const int64_t* rowptr, const int32_t* colind,
                                                        const uint8_t* bnd, int64_t V, double* K, double* rhs) {
    const int64_t i = (int64_t)blockIdx.x * P1_TB + threadIdx.x;
    if (i >= V) return;
    const bool bi = bnd[i] != 0;
    if (K)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const int32_t j = colind[p];
            if (bi) K[p] = (j == (int32_t)i) ? 1.0 : 0.0;
            else if (bnd[j]) K[p] = 0.0;
        }
    if (rhs && bi) rhs[i] = 0.0;
}

// ------------------------------------------------------------------ error
template <int DIM>
__global__ __launch_bounds__(INT_BLOCK) void k_p1_grad_error(const int32_t* elems, const double* nodes,
                                                             const double* v, int64_t T, const QuadRule q,
                                                             const FnArgs F, double* per_elem, double* partials) {
    const int64_t e = (int64_t)blockIdx.x * INT_BLOCK + threadIdx.x;
    double acc = 0.0;
    if (e < T) {
        int gid[DIM + 1];
        load_gid<DIM>(elems, e, gid);
        const QElem<DIM> g = q_elem<DIM>(nodes, gid);
        const double rJ = 1.0 / g.J;
        double gv[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a <= DIM; ++a) t += v[gid[a]] * g.c[a][d];
            gv[d] = t * rJ;
        }
        for_points<DIM>(q, [&](const double* xh, double w) {
            double x[DIM], fv[3] = {0.0, 0.0, 0.0};
            phys_point<DIM>(g, xh, x);
            eval_fn<DIM>(F, x, fv);
            double t = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) t += (fv[d] - gv[d]) * (fv[d] - gv[d]);
            acc += w * t;
        });
        acc *= fabs(g.J);
        if (per_elem) per_elem[e] = acc;
    }
    block_sum(acc, partials);
}

}  // namespace fem

using namespace fem;

extern "C" {

fem_status fem_p1_pattern(fem_mesh m, void* stream, int64_t* n_rows, int64_t* nnz, const int64_t** rowptr,
                          const int32_t** colind) {
    if (!m) return fail(FEM_EINVAL, "fem_p1_pattern: mesh is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    if (fem_status st = build_p1(m, s)) return st;
    if (n_rows) *n_rows = m->V;
    if (nnz) *nnz = m->p1_nnz;
    if (rowptr) *rowptr = m->p1_rowptr;
    if (colind) *colind = m->p1_colind;
    return FEM_OK;
}

fem_status fem_p1_assemble(fem_mesh m, const double* nodes, const double* a, double* K, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_p1_assemble: mesh is NULL");
    if (!nodes || !K) return fail(FEM_EINVAL, "fem_p1_assemble: nodes or K is NULL");
    if (!m->p1_built) return fail(FEM_ENOTREADY, "nodal pattern not built: call fem_p1_pattern first");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    const int64_t E = m->edges.n, V = m->V;
    const P1Bounds be{m->T * m->edges.nloc, m->p1_nnz, m->err_word};
    const P1Bounds bv{m->T * (m->dim + 1), m->p1_nnz, m->err_word};
    if (m->dim == 3) {
        hipLaunchKernelGGL(k_p1_offdiag<3>, dim3(p1_blocks(E)), dim3(P1_TB), 0, s, m->elems, nodes, a, m->edges2nodes,
                           m->edges.rs_ptr, m->edges.rs_slot, E, m->p1_rowptr, m->p1_colind, K, be);
        hipLaunchKernelGGL(k_p1_diag<3>, dim3(p1_blocks(V)), dim3(P1_TB), 0, s, m->elems, nodes, a, m->vs_ptr,
                           m->vs_slot, V, m->p1_rowptr, m->p1_colind, K, bv);
    } else {
        hipLaunchKernelGGL(k_p1_offdiag<2>, dim3(p1_blocks(E)), dim3(P1_TB), 0, s, m->elems, nodes, a, m->edges2nodes,
                           m->edges.rs_ptr, m->edges.rs_slot, E, m->p1_rowptr, m->p1_colind, K, be);
        hipLaunchKernelGGL(k_p1_diag<2>, dim3(p1_blocks(V)), dim3(P1_TB), 0, s, m->elems, nodes, a, m->vs_ptr,
                           m->vs_slot, V, m->p1_rowptr, m->p1_colind, K, bv);
    }
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status fem_p1_load(fem_mesh m, const double* nodes, fem_function fn, const double* params, int n_params,
                       int quad_m, double* F, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_p1_load: mesh is NULL");
    if (!nodes || !F) return fail(FEM_EINVAL, "fem_p1_load: nodes or F is NULL");
    if (!m->p1_built) return fail(FEM_ENOTREADY, "nodal pattern not built: call fem_p1_pattern first");
    QuadRule q;
    if (fem_status st = gauss_legendre01(quad_m, &q)) return st;
    FnArgs Fa;
    if (fem_status st = make_fn_args(fn, m->dim, params, n_params, &Fa)) return st;
    if (Fa.n_comp != 1) return fail(FEM_EINVAL, "fem_p1_load: the function must be scalar");
    if (!m->slot_vals) FEM_HIP(dmalloc(m, &m->slot_vals, (size_t)m->T * m->edges.nloc));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    const unsigned grid = (unsigned)((m->T + INT_BLOCK - 1) / INT_BLOCK);
    if (m->dim == 3)
        hipLaunchKernelGGL(k_p1_load_local<3>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, m->T, q, Fa,
                           m->slot_vals);
    else
        hipLaunchKernelGGL(k_p1_load_local<2>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, m->T, q, Fa,
                           m->slot_vals);
    hipLaunchKernelGGL(k_list_sum, dim3(p1_blocks(m->V)), dim3(P1_TB), 0, s, m->vs_ptr, m->vs_slot, m->slot_vals,
                       m->V, F, m->T * (m->dim + 1), m->err_word);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status fem_p1_dirichlet(fem_mesh m, double* K, double* rhs, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_p1_dirichlet: mesh is NULL");
    if (!m->p1_built) return fail(FEM_ENOTREADY, "nodal pattern not built: call fem_p1_pattern first");
    if (!K && !rhs) return FEM_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    hipLaunchKernelGGL(k_p1_dirichlet, dim3(p1_blocks(m->V)), dim3(P1_TB), 0, s, m->p1_rowptr, m->p1_colind,
                       m->bnd_nodes, m->V, K, rhs);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status fem_p1_grad_error(fem_mesh m, const double* nodes, const double* v, fem_function grad_u,
                             const double* params, int n_params, int quad_m, double* per_elem, double* total,
                             void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_p1_grad_error: mesh is NULL");
    if (!nodes || !v || !total) return fail(FEM_EINVAL, "fem_p1_grad_error: nodes, v or total is NULL");
    QuadRule q;
    if (fem_status st = gauss_legendre01(quad_m, &q)) return st;
    FnArgs Fa;
    if (fem_status st = make_fn_args(grad_u, m->dim, params, n_params, &Fa)) return st;
    if (Fa.n_comp > m->dim) return fail(FEM_EINVAL, "fem_p1_grad_error: the gradient has too many components");
    if (fem_status st = ensure_int_partials(m)) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    const unsigned grid = (unsigned)((m->T + INT_BLOCK - 1) / INT_BLOCK);
    if (m->dim == 3)
        hipLaunchKernelGGL(k_p1_grad_error<3>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, v, m->T, q, Fa,
                           per_elem, m->int_partials);
    else
        hipLaunchKernelGGL(k_p1_grad_error<2>, dim3(grid), dim3(INT_BLOCK), 0, s, m->elems, nodes, v, m->T, q, Fa,
                           per_elem, m->int_partials);
    FEM_HIP(hipGetLastError());
    return launch_sum_partials(m->int_partials, grid, total, s);
}

}  // extern "C"
