// Mesh topology (global edge / face numbering, element -> dof maps, sign data)
// and the one-time CSR pattern with its scatter map.
//
// Section 3 (Anjam & Valdman): the rows of edges2nodes / faces2nodes are the
// global degrees of freedom, elems2edges / elems2faces the local -> global
// maps. Here an edge is the sorted node pair (lo, hi) with key lo*V + hi, a face
// the sorted triple (a, b, c) with key eid(a,b)*V + c (eid = global id of the
// edge (a, b), which preserves lexicographic order and keeps keys below 2^64
// for any mesh with int32 ids). A stable radix sort of (key, slot) pairs, slot =
// element*n_local + local index, followed by unique gives the lexicographic
// numbering, the element -> dof map, and for each dof the run of slots that
// reference it in ascending element order (used by the assembly kernels).
//
// Pattern: every local pair (k, l) of every element gives the key
// dof_k * N + dof_l; sort + unique gives colind and rowptr, and each element's
// pairs get their CSR position (the scatter map). The map is stored compactly
// as, for each slot in row-sorted order, the byte offsets of its n_local
// columns inside the row.
#include <algorithm>
#include <vector>

#include "element.h"
#include "fem_internal.h"

namespace fem {

constexpr int TB = 256;

// Workgroups for one thread per item. A dispatch counts its work-items in 32
// bits, so n must stay below 2^32 - t: every launch here is over at most
// T * (edges or faces per element), n_nodes * dim, the rows, the tiles or one
// pair chunk, all below 2^31 by the limits fem_topology and fem_pattern check.
static inline unsigned nblk(int64_t n, int t = TB) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- validation
__global__ void k_validate_range(const int32_t* elems, int64_t n, int64_t V, int* err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = elems[i];
    if (v < 0 || v >= V) atomicOr(err, ERR_RANGE);
}

__global__ void k_validate_nodes(const double* nodes, int64_t n, int* err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!isfinite(nodes[i])) atomicOr(err, ERR_NONFINITE);
}

template <int DIM>
__global__ void k_validate_det(const double* nodes, const int32_t* elems, int64_t T, int* err) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= T) return;
    double J;
    if (DIM == 3) {
        V3 x[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t n = elems[e * 4 + v];
            x[v] = {nodes[n * 3], nodes[n * 3 + 1], nodes[n * 3 + 2]};
        }
        J = geo3(x).J;
    } else {
        V2 x[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const int64_t n = elems[e * 3 + v];
            x[v] = {nodes[n * 2], nodes[n * 2 + 1]};
        }
        J = geo2(x).J;
    }
    if (J == 0.0) atomicOr(err, ERR_DEGENERATE);
    if (!isfinite(J)) atomicOr(err, ERR_NONFINITE);
}

// ---------------------------------------------------------------- edges / faces
template <int DIM>
__global__ void k_edge_keys(const int32_t* elems, int64_t T, int64_t V, uint64_t* keys,
                            uint32_t* vals) {
    constexpr int NE = DIM == 3 ? 6 : 3;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T * NE) return;
    const int64_t e = q / NE;
    const int k = (int)(q - e * NE);
    const int s = DIM == 3 ? nib(NED3_START, k) : nib(TRI_START, k);
    const int t = DIM == 3 ? nib(NED3_END, k) : nib(TRI_END, k);
    const uint64_t gs = (uint32_t)elems[e * (DIM + 1) + s];
    const uint64_t gt = (uint32_t)elems[e * (DIM + 1) + t];
    const uint64_t lo = gs < gt ? gs : gt;
    const uint64_t hi = gs < gt ? gt : gs;
    keys[q] = lo * (uint64_t)V + hi;
    vals[q] = (uint32_t)q;
}

__global__ void k_flags(const uint64_t* keys, int64_t n, uint32_t* flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// After the exclusive scan of the flags: id = scan + flag - 1.
__global__ void k_edge_unique(const uint64_t* keys, const uint32_t* sorted_slots,
                              const uint32_t* scan, int64_t n, int64_t V, int32_t* elems2dofs,
                              int32_t* edges2nodes, int32_t* rs_ptr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool head = (i == 0 || keys[i] != keys[i - 1]);
    const int32_t id = (int32_t)(scan[i] + (head ? 1u : 0u) - 1u);
    elems2dofs[sorted_slots[i]] = id;
    if (head) {
        const uint64_t k = keys[i];
        edges2nodes[2 * (int64_t)id] = (int32_t)(k / (uint64_t)V);
        edges2nodes[2 * (int64_t)id + 1] = (int32_t)(k % (uint64_t)V);
        rs_ptr[id] = (int32_t)i;
    }
}

// 3D local edge index of the local node pair {p, q}.
__device__ __forceinline__ int tet_edge_index(int p, int q) {
    const int a = p < q ? p : q;
    const int b = p < q ? q : p;
    // (0,1)->0 (0,2)->1 (0,3)->2 (1,2)->3 (2,3)->4 (1,3)->5
    if (a == 0) return b - 1;
    if (a == 1) return b == 2 ? 3 : 5;
    return 4;
}

// Sorted (by global id) local node numbers of 3D face k (face k is opposite node 3-k).
__device__ __forceinline__ void face_sorted_local(const int gid[4], int k, int out[3]) {
    const int p = 3 - k;
    int u = (p == 0) ? 1 : 0;
    int v = (p <= 1) ? 2 : 1;
    int w = (p <= 2) ? 3 : 2;
    // sort three local numbers by their global ids
    if (gid[u] > gid[v]) { const int t = u; u = v; v = t; }
    if (gid[v] > gid[w]) { const int t = v; v = w; w = t; }
    if (gid[u] > gid[v]) { const int t = u; u = v; v = t; }
    out[0] = u;
    out[1] = v;
    out[2] = w;
}

__global__ void k_face_keys(const int32_t* elems, const int32_t* elems2edges, int64_t T, int64_t V,
                            uint64_t* keys, uint32_t* vals) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T * 4) return;
    const int64_t e = q / 4;
    const int k = (int)(q - e * 4);
    int gid[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) gid[v] = elems[e * 4 + v];
    int loc[3];
    face_sorted_local(gid, k, loc);
    const uint64_t eid = (uint32_t)elems2edges[e * 6 + tet_edge_index(loc[0], loc[1])];
    keys[q] = eid * (uint64_t)V + (uint64_t)(uint32_t)gid[loc[2]];
    vals[q] = (uint32_t)q;
}

__global__ void k_face_unique(const int32_t* elems, const uint64_t* keys,
                              const uint32_t* sorted_slots, const uint32_t* scan, int64_t n,
                              int32_t* elems2dofs, int32_t* faces2nodes, int32_t* rs_ptr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool head = (i == 0 || keys[i] != keys[i - 1]);
    const int32_t id = (int32_t)(scan[i] + (head ? 1u : 0u) - 1u);
    const uint32_t slot = sorted_slots[i];
    elems2dofs[slot] = id;
    if (head) {
        const int64_t e = slot / 4;
        const int k = (int)(slot - e * 4);
        int gid[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) gid[v] = elems[e * 4 + v];
        int loc[3];
        face_sorted_local(gid, k, loc);
        faces2nodes[3 * (int64_t)id] = gid[loc[0]];
        faces2nodes[3 * (int64_t)id + 1] = gid[loc[1]];
        faces2nodes[3 * (int64_t)id + 2] = gid[loc[2]];
        rs_ptr[id] = (int32_t)i;
    }
}

template <int DIM>
__global__ void k_edge_signs(const int32_t* elems, int64_t T, int8_t* signs) {
    constexpr int NE = DIM == 3 ? 6 : 3;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T * NE) return;
    const int64_t e = q / NE;
    const int k = (int)(q - e * NE);
    const int s = DIM == 3 ? nib(NED3_START, k) : nib(TRI_START, k);
    const int t = DIM == 3 ? nib(NED3_END, k) : nib(TRI_END, k);
    signs[q] = elems[e * (DIM + 1) + s] > elems[e * (DIM + 1) + t] ? 1 : -1;
}

__global__ void k_face_signs(const int32_t* elems, int64_t T, int8_t* signs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= T) return;
    int gid[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) gid[v] = elems[e * 4 + v];
    double s[4];
    rt3_signs(gid, s);
#pragma unroll
    for (int k = 0; k < 4; ++k) signs[e * 4 + k] = s[k] > 0 ? 1 : -1;
}

__global__ void k_set_i32(int32_t* p, int32_t v) { *p = v; }

// Conformity, for the element-major assembly (whose entries with one or two
// contributions are summed without a fixed order): a facet (3D face, 2D edge)
// with more than two elements, or with two elements whose vertices opposite it
// coincide (a duplicated element), makes the mesh non-conforming.
// 3D: face slot s = element * 4 + k, face k opposite local vertex 3 - k.
__global__ void k_face_conformity(const int32_t* rs_ptr, const int32_t* rs_slot, const int32_t* elems,
                                  int64_t F, int* flag) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int32_t j0 = rs_ptr[f];
    const int32_t n = rs_ptr[f + 1] - j0;
    if (n > 2) {
        atomicOr(flag, 1);
    } else if (n == 2) {
        const int64_t s1 = rs_slot[j0], s2 = rs_slot[j0 + 1];
        const int32_t o1 = elems[(s1 / 4) * 4 + 3 - s1 % 4];
        const int32_t o2 = elems[(s2 / 4) * 4 + 3 - s2 % 4];
        if (o1 == o2) atomicOr(flag, 1);
    }
}

// 2D: edge slot s = element * 3 + k, edge k = (start, end) opposite the third
// local vertex 3 - start - end.
__global__ void k_edge_conformity_2d(const int32_t* rs_ptr, const int32_t* rs_slot, const int32_t* elems,
                                     int64_t E, int* flag) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= E) return;
    const int32_t j0 = rs_ptr[q];
    const int32_t n = rs_ptr[q + 1] - j0;
    if (n > 2) {
        atomicOr(flag, 1);
    } else if (n == 2) {
        const int64_t s1 = rs_slot[j0], s2 = rs_slot[j0 + 1];
        const int k1 = (int)(s1 % 3), k2 = (int)(s2 % 3);
        const int32_t o1 = elems[(s1 / 3) * 3 + 3 - nib(TRI_START, k1) - nib(TRI_END, k1)];
        const int32_t o2 = elems[(s2 / 3) * 3 + 3 - nib(TRI_START, k2) - nib(TRI_END, k2)];
        if (o1 == o2) atomicOr(flag, 1);
    }
}
__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

// ---------------------------------------------------------------- helpers
static fem_status read_count(const uint32_t* scan, const uint64_t* keys, int64_t n, hipStream_t s,
                             int64_t* count) {
    uint32_t last_scan = 0;
    uint64_t k[2] = {0, 0};
    FEM_HIP(hipMemcpyAsync(&last_scan, scan + n - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    if (n >= 2) {
        FEM_HIP(hipMemcpyAsync(k, keys + n - 2, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    }
    FEM_HIP(hipStreamSynchronize(s));
    const bool head = (n == 1) || (k[1] != k[0]);
    *count = (int64_t)last_scan + (head ? 1 : 0);
    return FEM_OK;
}

static fem_status read_err(fem_mesh m, hipStream_t s, int* out) {
    FEM_HIP(hipMemcpyAsync(out, m->err_word, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    return FEM_OK;
}

struct TmpBufs {
    uint64_t* keys = nullptr;
    uint64_t* keys_tmp = nullptr;
    uint32_t* vals = nullptr;
    uint32_t* vals_tmp = nullptr;
    uint32_t* scan = nullptr;
    hipError_t alloc(int64_t n) {
        hipError_t e;
        if ((e = hipMalloc((void**)&keys, n * sizeof(uint64_t))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&keys_tmp, n * sizeof(uint64_t))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&vals, n * sizeof(uint32_t))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&vals_tmp, n * sizeof(uint32_t))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&scan, n * sizeof(uint32_t))) != hipSuccess) return e;
        return hipSuccess;
    }
    // (callers synchronise the stream that used the buffers first)
    void release() {
        for (void** q : {(void**)&keys, (void**)&keys_tmp, (void**)&vals, (void**)&vals_tmp, (void**)&scan}) {
            if (*q) (void)hipFree(*q);
            *q = nullptr;
        }
    }
    ~TmpBufs() { release(); }
};

// ---------------------------------------------------------------- topology
fem_status build_topology(fem_mesh m, const double* nodes, const int32_t* elems_in,
                          hipStream_t s) {
    const int dim = m->dim;
    const int64_t T = m->T, V = m->V;
    const int nv = dim + 1;
    const int ne = dim == 3 ? 6 : 3;
    FEM_HIP(dmalloc(m, &m->err_word, 1));
    FEM_HIP(hipMemsetAsync(m->err_word, 0, sizeof(int), s));
    FEM_HIP(dmalloc(m, &m->elems, T * nv));
    FEM_HIP(hipMemcpyAsync(m->elems, elems_in, T * nv * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    // 1. node ids in range, coordinates finite
    hipLaunchKernelGGL(k_validate_range, dim3(nblk(T * nv)), dim3(TB), 0, s, m->elems, T * nv, V,
                       m->err_word);
    hipLaunchKernelGGL(k_validate_nodes, dim3(nblk(V * dim)), dim3(TB), 0, s, nodes, V * dim,
                       m->err_word);
    FEM_HIP(hipGetLastError());
    int err = 0;
    if (fem_status st = read_err(m, s, &err)) return st;
    if (err & ERR_RANGE) return fail(FEM_ERANGE, "fem_topology: an element references a node id outside [0, n_nodes)");
    if (err & ERR_NONFINITE) return fail(FEM_ENONFINITE, "fem_topology: a node coordinate is not finite");
    // 2. non-degenerate elements
    if (dim == 3)
        hipLaunchKernelGGL(k_validate_det<3>, dim3(nblk(T)), dim3(TB), 0, s, nodes, m->elems, T, m->err_word);
    else
        hipLaunchKernelGGL(k_validate_det<2>, dim3(nblk(T)), dim3(TB), 0, s, nodes, m->elems, T, m->err_word);
    FEM_HIP(hipGetLastError());
    if (fem_status st = read_err(m, s, &err)) return st;
    if (err & ERR_DEGENERATE) return fail(FEM_EDEGENERATE, "fem_topology: an element has a zero Jacobian determinant");
    if (err & ERR_NONFINITE) return fail(FEM_ENONFINITE, "fem_topology: an element has a non-finite Jacobian determinant");

    // 3. edges
    const int64_t ns = T * ne;
    TmpBufs tb;
    FEM_HIP(tb.alloc(ns > T * 4 ? ns : T * 4));
    if (dim == 3)
        hipLaunchKernelGGL(k_edge_keys<3>, dim3(nblk(ns)), dim3(TB), 0, s, m->elems, T, V, tb.keys, tb.vals);
    else
        hipLaunchKernelGGL(k_edge_keys<2>, dim3(nblk(ns)), dim3(TB), 0, s, m->elems, T, V, tb.keys, tb.vals);
    FEM_HIP(hipGetLastError());
    const int edge_bits = bit_length((uint64_t)V * (uint64_t)V - 1);
    FEM_HIP(radix_sort_pairs(tb.keys, tb.vals, tb.keys_tmp, tb.vals_tmp, ns, edge_bits, s));
    hipLaunchKernelGGL(k_flags, dim3(nblk(ns)), dim3(TB), 0, s, tb.keys, ns, tb.scan);
    FEM_HIP(hipGetLastError());
    FEM_HIP(scan_exclusive_u32(tb.scan, ns, s));
    int64_t E = 0;
    if (fem_status st = read_count(tb.scan, tb.keys, ns, s, &E)) return st;
    DofSet& ed = m->edges;
    ed.nloc = ne;
    ed.n = E;
    FEM_HIP(dmalloc(m, &ed.elems2dofs, ns));
    FEM_HIP(dmalloc(m, &m->edges2nodes, 2 * E));
    FEM_HIP(dmalloc(m, &ed.rs_ptr, E + 1));
    FEM_HIP(dmalloc(m, &ed.rs_slot, ns));
    hipLaunchKernelGGL(k_edge_unique, dim3(nblk(ns)), dim3(TB), 0, s, tb.keys, tb.vals, tb.scan, ns,
                       V, ed.elems2dofs, m->edges2nodes, ed.rs_ptr);
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, ed.rs_ptr + E, (int32_t)ns);
    FEM_HIP(hipGetLastError());
    FEM_HIP(hipMemcpyAsync(ed.rs_slot, tb.vals, ns * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    FEM_HIP(dmalloc(m, &m->signs_e, ns));
    if (dim == 3)
        hipLaunchKernelGGL(k_edge_signs<3>, dim3(nblk(ns)), dim3(TB), 0, s, m->elems, T, m->signs_e);
    else
        hipLaunchKernelGGL(k_edge_signs<2>, dim3(nblk(ns)), dim3(TB), 0, s, m->elems, T, m->signs_e);
    FEM_HIP(hipGetLastError());
    if (dim == 2) {
        int* flag = reinterpret_cast<int*>(tb.scan);   // free again after the edge numbering
        FEM_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
        if (E > 0)
            hipLaunchKernelGGL(k_edge_conformity_2d, dim3(nblk(E)), dim3(TB), 0, s, ed.rs_ptr, ed.rs_slot, m->elems,
                               E, flag);
        FEM_HIP(hipGetLastError());
        int h = 0;
        FEM_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FEM_HIP(hipStreamSynchronize(s));
        m->nonconforming = h != 0;
    }

    // 4. faces (3D)
    if (dim == 3) {
        const int64_t nf = T * 4;
        hipLaunchKernelGGL(k_face_keys, dim3(nblk(nf)), dim3(TB), 0, s, m->elems, ed.elems2dofs, T, V,
                           tb.keys, tb.vals);
        FEM_HIP(hipGetLastError());
        const int face_bits = bit_length((uint64_t)E * (uint64_t)V - 1);
        FEM_HIP(radix_sort_pairs(tb.keys, tb.vals, tb.keys_tmp, tb.vals_tmp, nf, face_bits, s));
        hipLaunchKernelGGL(k_flags, dim3(nblk(nf)), dim3(TB), 0, s, tb.keys, nf, tb.scan);
        FEM_HIP(hipGetLastError());
        FEM_HIP(scan_exclusive_u32(tb.scan, nf, s));
        int64_t F = 0;
        if (fem_status st = read_count(tb.scan, tb.keys, nf, s, &F)) return st;
        DofSet& fd = m->faces;
        fd.nloc = 4;
        fd.n = F;
        FEM_HIP(dmalloc(m, &fd.elems2dofs, nf));
        FEM_HIP(dmalloc(m, &m->faces2nodes, 3 * F));
        FEM_HIP(dmalloc(m, &fd.rs_ptr, F + 1));
        FEM_HIP(dmalloc(m, &fd.rs_slot, nf));
        hipLaunchKernelGGL(k_face_unique, dim3(nblk(nf)), dim3(TB), 0, s, m->elems, tb.keys, tb.vals,
                           tb.scan, nf, fd.elems2dofs, m->faces2nodes, fd.rs_ptr);
        hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, fd.rs_ptr + F, (int32_t)nf);
        FEM_HIP(hipGetLastError());
        FEM_HIP(hipMemcpyAsync(fd.rs_slot, tb.vals, nf * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        FEM_HIP(dmalloc(m, &m->signs_f, nf));
        hipLaunchKernelGGL(k_face_signs, dim3(nblk(T)), dim3(TB), 0, s, m->elems, T, m->signs_f);
        FEM_HIP(hipGetLastError());
        int* flag = reinterpret_cast<int*>(tb.scan);   // the scan space is free again
        FEM_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
        if (F > 0)
            hipLaunchKernelGGL(k_face_conformity, dim3(nblk(F)), dim3(TB), 0, s, fd.rs_ptr, fd.rs_slot, m->elems, F,
                               flag);
        FEM_HIP(hipGetLastError());
        int h = 0;
        FEM_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FEM_HIP(hipStreamSynchronize(s));
        m->nonconforming = h != 0;
    }
    FEM_HIP(hipStreamSynchronize(s));
    return FEM_OK;
}

// ---------------------------------------------------------------- pattern
// Pairs of the slots j0 .. j0+n of the row-sorted slot list (a range of whole
// rows): pair q = j * nloc + l couples slot j's dof (the row) with the dof of
// local index l of the same element (the column). Key = row * N + column; the
// payload is the chunk-local pair index.
__global__ void k_pair_keys(const int32_t* rs_slot, int64_t n, const int32_t* elems2dofs, int nloc,
                            int64_t N, uint64_t* keys, uint32_t* vals) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n * nloc) return;
    const int64_t j = q / nloc;
    const int l = (int)(q - j * nloc);
    const int64_t sl = rs_slot[j];
    const int64_t e = sl / nloc;
    const uint64_t I = (uint32_t)elems2dofs[sl];
    const uint64_t J = (uint32_t)elems2dofs[e * nloc + l];
    keys[q] = I * (uint64_t)N + J;
    vals[q] = (uint32_t)q;
}

// After the exclusive scan of the head flags: the CSR position of each sorted
// pair is base + (its unique rank within the chunk); heads write the column
// at that rank in the chunk's column buffer and, at a row's first entry, the
// row start. map[pair] = the unique rank (chunk-local pairs; below 2^31
// because a chunk has fewer pairs), so the total number of nonzeros is not
// bounded by the map's width.
__global__ void k_pair_unique(const uint64_t* keys, const uint32_t* sorted_pairs,
                              const uint32_t* scan, int64_t n, int64_t N, int64_t base,
                              int32_t* cols, int64_t* rowptr, uint32_t* map) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    const bool head = (i == 0 || k != keys[i - 1]);
    const uint32_t local = scan[i] + (head ? 1u : 0u) - 1u;
    const int64_t id = base + (int64_t)local;
    map[sorted_pairs[i]] = local;
    if (head) {
        const uint64_t row = k / (uint64_t)N;
        cols[local] = (int32_t)(k - row * (uint64_t)N);
        if (i == 0 || keys[i - 1] / (uint64_t)N != row) rowptr[row] = id;
    }
}

__global__ void k_slot_rank(const int32_t* rs_slot, int64_t n, int32_t* rank) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    rank[rs_slot[i]] = (int32_t)i;
}

// Column offsets of the slots j0 .. j0+n of the row-sorted list (the same
// chunk as the pairs in map, whose first nonzero is chunk_base): byte l = CSR
// position of (row, dof l) minus the row start.
__global__ void k_colpos(const int32_t* rs_slot, int64_t n, const int32_t* elems2dofs, const uint32_t* map,
                         int64_t chunk_base, const int64_t* rowptr, int nloc, int cp, uint8_t* colpos,
                         int* err) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t base = rowptr[elems2dofs[rs_slot[j]]];
    uint8_t out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int l = 0; l < nloc; ++l) {
        const int64_t off = chunk_base + (int64_t)map[j * nloc + l] - base;
        if (off < 0 || off > 255) atomicOr(err, ERR_OVERFLOW);
        out[l] = (uint8_t)off;
    }
    for (int l = 0; l < cp; ++l) colpos[j * cp + l] = out[l];
}

// Longest row and, for R = 32, 64, 128, 256, the most values of a tile of R
// rows: block-wide maxima, one atomic per block and statistic.
__global__ __launch_bounds__(256) void k_row_stats(const int64_t* rowptr, int64_t N, int* max_len,
                                                   int* tile_pmax) {
    __shared__ int red[5][256];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v[5] = {0, 0, 0, 0, 0};
    if (r < N) {
        const int64_t len = rowptr[r + 1] - rowptr[r];
        v[0] = (int)(len > 0x7fffffff ? 0x7fffffff : len);
        const int R[4] = {32, 64, 128, 256};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (r % R[q] == 0) {
                const int64_t r1 = (r + R[q] < N) ? r + R[q] : N;
                const int64_t nn = rowptr[r1] - rowptr[r];
                v[1 + q] = (int)(nn > 0x7fffffff ? 0x7fffffff : nn);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = max(red[q][threadIdx.x], red[q][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(max_len, red[0][0]);
#pragma unroll
        for (int q = 0; q < 4; ++q) atomicMax(&tile_pmax[q], red[1 + q][0]);
    }
}

// Frees a temporary device buffer when the builder returns, on any path.
template <class T>
struct FreeOnExit {
    T** p;
    ~FreeOnExit() { (void)hipFree(*p); }
};

fem_status build_pattern(fem_mesh m, DofSet& ds, hipStream_t s) {
    Pattern& p = ds.pat;
    if (p.built) return FEM_OK;
    const int64_t T = m->T;
    const int nloc = ds.nloc;
    const int64_t N = ds.n;
    const int64_t n_slots = T * nloc;
    const int64_t n_pairs = n_slots * nloc;
    p.nloc = nloc;
    p.cp_stride = nloc <= 4 ? 4 : 8;
    p.n_rows = N;
    // The (row, column) pairs of every element are sorted and made unique in
    // chunks of whole rows (ranges of the row-sorted slot list), each at most
    // FEM_PAIR_CHUNK pairs (default 2^29) unless a single row is larger. The
    // keys are unique per (row, column) and rows do not straddle chunks, so
    // the result does not depend on the chunking.
    int64_t chunk_max = int64_t(1) << 29;
    if (const char* sc = std::getenv("FEM_PAIR_CHUNK")) chunk_max = std::max<int64_t>(std::atoll(sc), 1);
    std::vector<int64_t> rb{0}, sb{0};  // row and slot boundaries of the chunks
    if (n_pairs <= chunk_max) {
        rb.push_back(N);
        sb.push_back(n_slots);
    } else {
        std::vector<int32_t> h((size_t)N + 1);
        FEM_HIP(hipMemcpyAsync(h.data(), ds.rs_ptr, (size_t)(N + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FEM_HIP(hipStreamSynchronize(s));
        for (int64_t r0 = 0; r0 < N;) {
            // the last row boundary r1 with (h[r1] - h[r0]) * nloc <= chunk_max
            const int64_t lim = (int64_t)h[r0] + chunk_max / nloc;
            int64_t r1 = (int64_t)(std::upper_bound(h.begin() + r0 + 1, h.end(), lim) - h.begin()) - 1;
            if (r1 <= r0) r1 = r0 + 1;  // one row larger than a chunk: alone
            rb.push_back(r1);
            sb.push_back(h[r1]);
            r0 = r1;
        }
    }
    const size_t n_chunks = rb.size() - 1;
    int64_t max_pairs = 1;
    for (size_t c = 0; c < n_chunks; ++c) max_pairs = std::max(max_pairs, (sb[c + 1] - sb[c]) * nloc);
    if (max_pairs >= (int64_t(1) << 31))
        return fail(FEM_EOVERFLOW, "fem_pattern: the element pairs of one row range exceed 2^31");
    // The pattern's arrays join the handle only when the build succeeds: a
    // refused build (too many nonzeros, a row too long) leaves nothing behind.
    struct Owned {
        Pattern* p;
        std::vector<void*> v;
        bool keep = false;
        ~Owned() {
            if (keep) return;
            for (void* q : v) (void)hipFree(q);
            p->rowptr = nullptr;
            p->colind = nullptr;
            p->colpos = nullptr;
            p->slot_rank = nullptr;
        }
    } own{&p, {}};
    auto alloc = [&](auto** ptr, int64_t count) {
        *ptr = nullptr;
        const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(**ptr);
        hipError_t e = hipMalloc((void**)ptr, bytes);
        if (e == hipSuccess) own.v.push_back((void*)*ptr);
        return e;
    };
    TmpBufs tb;
    FEM_HIP(tb.alloc(std::max<int64_t>(max_pairs, 8)));
    const int bits = bit_length((uint64_t)N * (uint64_t)N - 1);
    FEM_HIP(alloc(&p.rowptr, N + 1));
    uint32_t* map = nullptr;  // chunk-local CSR position of every pair of the current chunk
    FreeOnExit<uint32_t> free_map{&map};
    // several chunks: each chunk's columns in a buffer of its own until the
    // total is known (nnz words in all, not one per element pair)
    struct Staged {
        std::vector<std::pair<int32_t*, int64_t>> v;
        ~Staged() {
            for (auto& q : v) (void)hipFree(q.first);
        }
    } staged;
    FEM_HIP(hipMalloc((void**)&map, (size_t)max_pairs * sizeof(uint32_t)));
    int* stats = nullptr;  // row statistics: longest row, most values of a tile of 32 .. 256 rows
    FreeOnExit<int> free_stats{&stats};
    FEM_HIP(hipMalloc((void**)&stats, 5 * sizeof(int)));
    FEM_HIP(alloc(&p.colpos, n_slots * p.cp_stride));
    FEM_HIP(hipMemsetAsync(m->err_word, 0, sizeof(int), s));
    int64_t nnz = 0;
    for (size_t c = 0; c < n_chunks; ++c) {
        const int64_t j0 = sb[c], ns = sb[c + 1] - sb[c], np = ns * nloc;
        if (np == 0) continue;
        hipLaunchKernelGGL(k_pair_keys, dim3(nblk(np)), dim3(TB), 0, s, ds.rs_slot + j0, ns, ds.elems2dofs,
                           nloc, N, tb.keys, tb.vals);
        FEM_HIP(hipGetLastError());
        FEM_HIP(radix_sort_pairs(tb.keys, tb.vals, tb.keys_tmp, tb.vals_tmp, np, bits, s));
        hipLaunchKernelGGL(k_flags, dim3(nblk(np)), dim3(TB), 0, s, tb.keys, np, tb.scan);
        FEM_HIP(hipGetLastError());
        FEM_HIP(scan_exclusive_u32(tb.scan, np, s));
        int64_t nc = 0;
        if (fem_status st = read_count(tb.scan, tb.keys, np, s, &nc)) return st;
        int32_t* cols = nullptr;
        if (n_chunks == 1) {
            FEM_HIP(alloc(&p.colind, nc));
            cols = p.colind;
        } else {
            FEM_HIP(hipMalloc((void**)&cols, (size_t)std::max<int64_t>(nc, 1) * sizeof(int32_t)));
            staged.v.push_back({cols, nc});
        }
        hipLaunchKernelGGL(k_pair_unique, dim3(nblk(np)), dim3(TB), 0, s, tb.keys, tb.vals, tb.scan, np, N,
                           nnz, cols, p.rowptr, map);
        hipLaunchKernelGGL(k_colpos, dim3(nblk(ns)), dim3(TB), 0, s, ds.rs_slot + j0, ns, ds.elems2dofs, map,
                           nnz, p.rowptr, nloc, p.cp_stride, p.colpos + j0 * p.cp_stride, m->err_word);
        FEM_HIP(hipGetLastError());
        nnz += nc;
    }
    p.nnz = nnz;
    if (n_chunks > 1) {
        // the sort buffers and the map are done with: free them before the
        // final column array, and each chunk's buffer once it is copied
        FEM_HIP(hipStreamSynchronize(s));
        tb.release();
        (void)hipFree(map);
        map = nullptr;
        FEM_HIP(alloc(&p.colind, nnz));
        int64_t at = 0;
        for (auto& q : staged.v) {
            FEM_HIP(hipMemcpyAsync(p.colind + at, q.first, (size_t)q.second * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s));
            FEM_HIP(hipStreamSynchronize(s));
            (void)hipFree(q.first);
            q.first = nullptr;
            at += q.second;
        }
        staged.v.clear();
    }
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, p.rowptr + N, nnz);
    FEM_HIP(hipGetLastError());
    FEM_HIP(alloc(&p.slot_rank, n_slots));
    hipLaunchKernelGGL(k_slot_rank, dim3(nblk(n_slots)), dim3(TB), 0, s, ds.rs_slot, n_slots, p.slot_rank);
    FEM_HIP(hipGetLastError());
    FEM_HIP(hipMemsetAsync(stats, 0, 5 * sizeof(int), s));
    hipLaunchKernelGGL(k_row_stats, dim3(nblk(N)), dim3(TB), 0, s, p.rowptr, N, stats, stats + 1);
    FEM_HIP(hipGetLastError());
    int host_stats[5];
    int err = 0;
    FEM_HIP(hipMemcpyAsync(host_stats, stats, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipMemcpyAsync(&err, m->err_word, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    p.max_row_len = host_stats[0];
    for (int q = 0; q < 4; ++q) p.tile_pmax[q] = host_stats[1 + q];
    if ((err & ERR_OVERFLOW) || p.max_row_len > 255)
        return fail(FEM_EOVERFLOW, "fem_pattern: a row has more than 255 entries");
    for (void* q : own.v) m->allocs.push_back(q);
    own.keep = true;
    p.built = true;
    return FEM_OK;
}

// Adjoint gather map: per slot (element-major order) the row start of the
// slot's dof and the slot's column-offset record, so the adjoint reaches the
// n_local^2 positions of an element with one level of indirection.
__global__ void k_slot_map(const int32_t* elems2dofs, const int64_t* rowptr, const int32_t* slot_rank,
                           const uint8_t* colpos, int cp_stride, int64_t n, int32_t* base,
                           uint64_t* cp) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    base[s] = (int32_t)rowptr[elems2dofs[s]];
    const int64_t j = slot_rank[s];
    cp[s] = cp_stride == 8 ? reinterpret_cast<const uint64_t*>(colpos)[j]
                           : (uint64_t)reinterpret_cast<const uint32_t*>(colpos)[j];
}

// Arrays of a map that is built on first use. They join the handle, and the
// map counts as built, only when every step of the build has succeeded; on any
// failure they are freed and their pointers cleared, so the next call builds
// the map again instead of using a half-built one.
struct Staged {
    fem_mesh m;
    std::vector<std::pair<void**, void*>> v;
    bool keep = false;
    template <class T>
    hipError_t alloc(T** ptr, int64_t count) {
        *ptr = nullptr;
        const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
        hipError_t e = hipMalloc((void**)ptr, bytes);
        if (e == hipSuccess) v.push_back({reinterpret_cast<void**>(ptr), (void*)*ptr});
        return e;
    }
    ~Staged() {
        for (auto& q : v) {
            if (keep) {
                m->allocs.push_back(q.second);
            } else {
                (void)hipFree(q.second);
                *q.first = nullptr;
            }
        }
    }
};

fem_status build_slot_map(fem_mesh m, DofSet& ds, hipStream_t s) {
    if (ds.slot_map_built) return FEM_OK;
    if (ds.pat.nnz >= (int64_t(1) << 31))
        return fail(FEM_EOVERFLOW, "fem_assemble_backward: weights per nonzero need nnz < 2^31 "
                                   "(the quadratic form has no such limit)");
    Staged st{m, {}};
    const int64_t n = m->T * ds.nloc;
    FEM_HIP(st.alloc(&ds.slot_base, n));
    FEM_HIP(st.alloc(&ds.slot_cp, n));
    if (n > 0) {
        hipLaunchKernelGGL(k_slot_map, dim3(nblk(n)), dim3(TB), 0, s, ds.elems2dofs, ds.pat.rowptr,
                           ds.pat.slot_rank, ds.pat.colpos, ds.pat.cp_stride, n, ds.slot_base,
                           ds.slot_cp);
        FEM_HIP(hipGetLastError());
    }
    st.keep = true;
    ds.slot_map_built = true;
    return FEM_OK;
}

// ---------------------------------------------------------------- adjoint node map
// The adjoint runs one element per lane in workgroups of BWD_BLOCK consecutive
// elements. A workgroup first sums, per vertex it touches, the vertex
// derivatives of its own elements (in ascending element order, in LDS), and
// writes one partial per (vertex, workgroup) pair; the node sum then adds the
// pairs of a node in ascending workgroup order. Both orders are fixed, so the
// result is deterministic, and the partials are far fewer than the incidences.
// Layout, workgroup-major so a workgroup reads its part contiguously:
//   bwd_inc [T*(dim+1)] u16: workgroup b's incidences occupy positions
//       b*BWD_BLOCK*(dim+1) onwards, each as its workgroup-local index
//       (e - b*BWD_BLOCK)*(dim+1) + v, sorted by (node, element);
//   bwd_bptr [workgroups+1]: the pairs of workgroup b are bptr[b] .. bptr[b+1],
//       in ascending node order; pair q's partial is partials[q];
//   bwd_pst [pairs + 1] u16: the workgroup-local position in bwd_inc of the
//       first incidence of each pair (the pair ends where the next one starts,
//       or at the end of the workgroup's incidences); one u16 of padding;
//   node_ptr [V+1], bwd_npair [pairs]: the pairs of each node, ascending
//       workgroup.
__global__ void k_inc_wg_keys(const int32_t* elems, int64_t n, int nv, int64_t V, uint64_t* keys,
                              uint32_t* vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t blk = (i / nv) / BWD_BLOCK;
    keys[i] = (uint64_t)blk * (uint64_t)V + (uint64_t)elems[i];
    vals[i] = (uint32_t)i;
}

// After the stable sort by (workgroup, node): local incidence index and pair
// head flags.
__global__ void k_inc_wg_local(const uint64_t* keys, const uint32_t* vals, int64_t n, int nv,
                               uint16_t* inc, uint32_t* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t wg_first = ((int64_t)vals[i] / (nv * BWD_BLOCK)) * (nv * BWD_BLOCK);
    inc[i] = (uint16_t)((int64_t)vals[i] - wg_first);
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// After the exclusive scan of the head flags: pair starts, and the pair counts
// of each node and of each workgroup; node keys for the node-major pair list.
__global__ void k_inc_wg_pairs(const uint64_t* keys, const uint32_t* scan, int64_t n, int nv, int64_t V,
                               uint16_t* pst, int32_t* node_cnt, int32_t* blk_cnt, uint64_t* nkey,
                               uint32_t* nval) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i != 0 && keys[i] == keys[i - 1]) return;
    const int64_t q = scan[i];
    const uint64_t blk = keys[i] / (uint64_t)V;
    const uint64_t node = keys[i] - blk * (uint64_t)V;
    pst[q] = (uint16_t)(i - (int64_t)blk * nv * BWD_BLOCK);
    atomicAdd(&node_cnt[node], 1);
    atomicAdd(&blk_cnt[blk], 1);
    nkey[q] = node;
    nval[q] = (uint32_t)q;
}

fem_status build_node_map(fem_mesh m, hipStream_t s) {
    if (m->node_map_built) return FEM_OK;
    Staged st{m, {}};
    const int nv = m->dim + 1;
    const int64_t n = m->T * nv;
    const int64_t n_blocks = (m->T + BWD_BLOCK - 1) / BWD_BLOCK;
    static_assert(BWD_BLOCK * 4 <= 65536, "workgroup-local incidence indices are 16-bit");
    FEM_HIP(st.alloc(&m->node_ptr, m->V + 1));
    FEM_HIP(st.alloc(&m->bwd_bptr, n_blocks + 1));
    FEM_HIP(st.alloc(&m->bwd_inc, (n > 0 ? n : 1) + 1));   // +1: read as 32-bit words
    FEM_HIP(hipMemsetAsync(m->node_ptr, 0, (m->V + 1) * sizeof(int32_t), s));
    FEM_HIP(hipMemsetAsync(m->bwd_bptr, 0, (n_blocks + 1) * sizeof(int32_t), s));
    FEM_HIP(hipMemsetAsync(m->bwd_inc, 0, ((n > 0 ? n : 1) + 1) * sizeof(uint16_t), s));
    if (n == 0) {
        FEM_HIP(st.alloc(&m->bwd_pst, 1));
        FEM_HIP(st.alloc(&m->bwd_npair, 1));
        m->bwd_pairs = 0;
        st.keep = true;
        m->node_map_built = true;
        return FEM_OK;
    }
    TmpBufs tb;
    FEM_HIP(tb.alloc(n));
    hipLaunchKernelGGL(k_inc_wg_keys, dim3(nblk(n)), dim3(TB), 0, s, m->elems, n, nv, m->V, tb.keys, tb.vals);
    FEM_HIP(hipGetLastError());
    FEM_HIP(radix_sort_pairs(tb.keys, tb.vals, tb.keys_tmp, tb.vals_tmp, n,
                             bit_length((uint64_t)m->V * (uint64_t)n_blocks - 1), s));
    hipLaunchKernelGGL(k_inc_wg_local, dim3(nblk(n)), dim3(TB), 0, s, tb.keys, tb.vals, n, nv, m->bwd_inc,
                       tb.scan);
    FEM_HIP(hipGetLastError());
    FEM_HIP(scan_exclusive_u32(tb.scan, n, s));
    int64_t P = 0;
    if (fem_status st = read_count(tb.scan, tb.keys, n, s, &P)) return st;
    m->bwd_pairs = P;
    FEM_HIP(st.alloc(&m->bwd_pst, P + 1));  // +1: read as 32-bit words
    FEM_HIP(st.alloc(&m->bwd_npair, P));
    // node keys of the pairs, in the (now free) tmp key/value space after the
    // incidence keys: P <= n entries each
    uint64_t* nkey = tb.keys_tmp;
    uint32_t* nval = tb.vals_tmp;
    hipLaunchKernelGGL(k_inc_wg_pairs, dim3(nblk(n)), dim3(TB), 0, s, tb.keys, tb.scan, n, nv, m->V, m->bwd_pst,
                       m->node_ptr, m->bwd_bptr, nkey, nval);
    FEM_HIP(hipGetLastError());
    FEM_HIP(scan_exclusive_u32(reinterpret_cast<uint32_t*>(m->node_ptr), m->V + 1, s));
    FEM_HIP(scan_exclusive_u32(reinterpret_cast<uint32_t*>(m->bwd_bptr), n_blocks + 1, s));
    // pairs of each node, ascending workgroup (stable sort of the workgroup-major
    // pair list by node)
    FEM_HIP(radix_sort_pairs(nkey, nval, tb.keys, tb.vals, P, bit_length((uint64_t)m->V - 1), s));
    FEM_HIP(hipMemcpyAsync(m->bwd_npair, nval, P * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    FEM_HIP(hipStreamSynchronize(s));
    st.keep = true;
    m->node_map_built = true;
    return FEM_OK;
}

}  // namespace fem

// ---------------------------------------------------------------- row-tile element lists
namespace fem {

__global__ void k_tile_keys(const int32_t* rs_slot, const int32_t* elems2dofs, int64_t n_slots,
                            int nloc, int R, int64_t T, uint64_t* keys, uint32_t* vals) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_slots) return;
    const int64_t s = rs_slot[j];
    const int64_t tile = elems2dofs[s] / R;
    keys[j] = (uint64_t)tile * (uint64_t)T + (uint64_t)(s / nloc);
    vals[j] = (uint32_t)j;
}

// unique (tile, element) pairs: element list entries and tile starts
__global__ void k_tile_unique(const uint64_t* keys, const uint32_t* scan, int64_t n, int64_t T,
                              int32_t* tile_elems, int32_t* eptr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    const bool head = (i == 0 || k != keys[i - 1]);
    if (!head) return;
    const int32_t id = (int32_t)scan[i];  // exclusive scan of the head flags
    const uint64_t tile = k / (uint64_t)T;
    tile_elems[id] = (int32_t)(k - tile * (uint64_t)T);
    if (i == 0 || keys[i - 1] / (uint64_t)T != tile) eptr[tile] = id;
}


}  // namespace fem

// ---------------------------------------------------------------- element-major tiles
namespace fem {

int ema_index(int nt) { return nt <= 128 ? 0 : 1; }

// For each sorted (tile, element) pair: the tile-local slot index of the slot.
__global__ void k_ema_joff(const uint64_t* keys, const uint32_t* sorted_slots, const uint32_t* scan,
                           const int32_t* rs_slot, const int32_t* rs_ptr, const int32_t* eptr,
                           int64_t n, int64_t T, int nloc, int R, uint16_t* joff, int* max_elems,
                           int* overflow) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    const bool head = (i == 0 || k != keys[i - 1]);
    const int64_t id = (int64_t)scan[i] + (head ? 1 : 0) - 1;
    const int64_t tile = (int64_t)(k / (uint64_t)T);
    const uint32_t j = sorted_slots[i];
    const int64_t rel = (int64_t)j - rs_ptr[tile * R];
    if (rel < 0 || rel >= 0xFFFF) atomicOr(overflow, 1);
    joff[id * 8 + rs_slot[j] % nloc] = (uint16_t)rel;
    if (i + 1 == n || keys[i + 1] / (uint64_t)T != (uint64_t)tile)
        atomicMax(max_elems, (int)(id - eptr[tile] + 1));
}

__global__ void k_ema_stats(const int64_t* rowptr, const int32_t* rs_ptr, int64_t N, int R,
                            int64_t n_tiles, int* pmax, int* max_slots) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const int64_t r0 = t * R;
    const int64_t r1 = (r0 + R < N) ? r0 + R : N;
    atomicMax(pmax, (int)(rowptr[r1] - rowptr[r0]));
    atomicMax(max_slots, rs_ptr[r1] - rs_ptr[r0]);
}

// Every entry's eight in-tile slot words set to 0xFFFF (none in the tile),
// one 16-byte entry per thread.
__global__ void k_clear_joff(uint4* joff, int64_t n_ent) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_ent) joff[i] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
}

// One attempt at tiles of R rows; allocations are plain (freed by the caller
// unless adopted into the mesh).
static fem_status ema_attempt(fem_mesh m, DofSet& ds, int R, hipStream_t s, Pattern::Ema& out) {
    const int64_t T = m->T;
    const int64_t n_slots = T * ds.nloc;
    const int64_t n_tiles = (ds.pat.n_rows + R - 1) / R;
    TmpBufs tb;
    FEM_HIP(tb.alloc(n_slots));
    hipLaunchKernelGGL(k_tile_keys, dim3(nblk(n_slots)), dim3(TB), 0, s, ds.rs_slot, ds.elems2dofs,
                       n_slots, ds.nloc, R, T, tb.keys, tb.vals);
    FEM_HIP(hipGetLastError());
    FEM_HIP(radix_sort_pairs(tb.keys, tb.vals, tb.keys_tmp, tb.vals_tmp, n_slots,
                             bit_length((uint64_t)n_tiles * (uint64_t)T - 1), s));
    hipLaunchKernelGGL(k_flags, dim3(nblk(n_slots)), dim3(TB), 0, s, tb.keys, n_slots, tb.scan);
    FEM_HIP(hipGetLastError());
    FEM_HIP(scan_exclusive_u32(tb.scan, n_slots, s));
    int64_t n_ent = 0;
    if (fem_status st = read_count(tb.scan, tb.keys, n_slots, s, &n_ent)) return st;
    out.R = R;
    out.n_tiles = n_tiles;
    FEM_HIP(hipMalloc((void**)&out.eptr, (n_tiles + 1) * sizeof(int32_t)));
    FEM_HIP(hipMalloc((void**)&out.elems, n_ent * sizeof(int32_t)));
    FEM_HIP(hipMalloc((void**)&out.joff, n_ent * 8 * sizeof(uint16_t)));
    hipLaunchKernelGGL(k_tile_unique, dim3(nblk(n_slots)), dim3(TB), 0, s, tb.keys, tb.scan, n_slots,
                       T, out.elems, out.eptr);
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, out.eptr + n_tiles, (int32_t)n_ent);
    hipLaunchKernelGGL(k_clear_joff, dim3(nblk(n_ent)), dim3(TB), 0, s, reinterpret_cast<uint4*>(out.joff),
                       n_ent);
    FEM_HIP(hipGetLastError());
    int* stats = reinterpret_cast<int*>(tb.keys_tmp);  // [4]: max_elems, overflow, pmax, max_slots
    FEM_HIP(hipMemsetAsync(stats, 0, 4 * sizeof(int), s));
    hipLaunchKernelGGL(k_ema_joff, dim3(nblk(n_slots)), dim3(TB), 0, s, tb.keys, tb.vals, tb.scan,
                       ds.rs_slot, ds.rs_ptr, out.eptr, n_slots, T, ds.nloc, R, out.joff, stats,
                       stats + 1);
    hipLaunchKernelGGL(k_ema_stats, dim3(nblk(n_tiles)), dim3(TB), 0, s, ds.pat.rowptr, ds.rs_ptr,
                       ds.pat.n_rows, R, n_tiles, stats + 2, stats + 3);
    FEM_HIP(hipGetLastError());
    int h[4];
    FEM_HIP(hipMemcpyAsync(h, stats, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    out.max_elems = h[0];
    out.pmax = h[2];
    out.max_slots = h[3];
    if (h[1]) return fail(FEM_EOVERFLOW, "fem_pattern: a row tile has more than 65534 slots");
    return FEM_OK;
}

// Order key of an entry within its tile: the lowest local dof the entry has in
// the tile, then the set of those dofs (6 bits), then (stable sort) the
// element. Entries with the same rows in the tile become neighbours, so the
// lanes of a wavefront mostly form the same local rows.
__global__ void k_ema_order_keys(const int32_t* eptr, int64_t n_tiles, const uint16_t* joff,
                                 int nloc, uint64_t* keys, uint32_t* vals) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    for (int32_t i = eptr[t]; i < eptr[t + 1]; ++i) {
        uint32_t mask = 0;
        for (int k = 0; k < nloc; ++k)
            if (joff[(int64_t)i * 8 + k] != 0xFFFFu) mask |= 1u << k;
        const uint32_t low = mask ? (uint32_t)(__ffs(mask) - 1) : 7u;
        keys[i] = ((uint64_t)t << 9) | (low << 6) | mask;
        vals[i] = (uint32_t)i;
    }
}

__global__ void k_ema_permute(const uint32_t* perm, int64_t n, const int32_t* elems_in,
                              const uint4* joff_in, int32_t* elems_out, uint4* joff_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
    elems_out[i] = elems_in[j];
    joff_out[i] = joff_in[j];
}

static fem_status ema_order(Pattern::Ema& E, int nloc, hipStream_t s) {
    int32_t n_ent = 0;
    FEM_HIP(hipMemcpyAsync(&n_ent, E.eptr + E.n_tiles, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    if (n_ent <= 1) return FEM_OK;
    TmpBufs tb;
    FEM_HIP(tb.alloc(n_ent));
    hipLaunchKernelGGL(k_ema_order_keys, dim3(nblk(E.n_tiles)), dim3(TB), 0, s, E.eptr, E.n_tiles,
                       E.joff, nloc, tb.keys, tb.vals);
    FEM_HIP(hipGetLastError());
    FEM_HIP(radix_sort_pairs(tb.keys, tb.vals, tb.keys_tmp, tb.vals_tmp, n_ent,
                             bit_length((((uint64_t)E.n_tiles - 1) << 9) | 511u), s));
    int32_t* elems = nullptr;
    uint16_t* joff = nullptr;
    FEM_HIP(hipMalloc((void**)&elems, (size_t)n_ent * sizeof(int32_t)));
    if (hipMalloc((void**)&joff, (size_t)n_ent * 8 * sizeof(uint16_t)) != hipSuccess) {
        (void)hipFree(elems);
        return fail(FEM_ENOMEM, "fem_pattern: out of device memory");
    }
    hipLaunchKernelGGL(k_ema_permute, dim3(nblk(n_ent)), dim3(TB), 0, s, tb.vals, (int64_t)n_ent,
                       E.elems, reinterpret_cast<const uint4*>(E.joff), elems,
                       reinterpret_cast<uint4*>(joff));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(elems);
        (void)hipFree(joff);
        FEM_HIP(e);
    }
    (void)hipFree(E.elems);
    (void)hipFree(E.joff);
    E.elems = elems;
    E.joff = joff;
    return FEM_OK;
}

static void ema_free(Pattern::Ema& e) {
    if (e.eptr) (void)hipFree(e.eptr);
    if (e.elems) (void)hipFree(e.elems);
    if (e.joff) (void)hipFree(e.joff);
    if (e.ent) (void)hipFree(e.ent);
    if (e.egid) (void)hipFree(e.egid);
    e.egid = nullptr;
    if (e.rec) (void)hipFree(e.rec);
    if (e.hdr) (void)hipFree(e.hdr);
    if (e.rtab) (void)hipFree(e.rtab);
    e.hdr = nullptr;
    e.rtab = nullptr;
    e.eptr = nullptr;
    e.elems = nullptr;
    e.joff = nullptr;
    e.ent = nullptr;
    e.rec = nullptr;
}

// Row of every slot in row-sorted order.
__global__ void k_slot_rows(const int32_t* rs_ptr, int64_t n_rows, int32_t* slot_row) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    for (int32_t j = rs_ptr[r]; j < rs_ptr[r + 1]; ++j) slot_row[j] = (int32_t)r;
}

// Entries and slot records of the element-major tiles (one thread per tile,
// entries in their final order).
__global__ void k_ema_records(const int32_t* eptr, int64_t n_tiles, const int32_t* elems,
                              const uint16_t* joff, const int32_t* rs_ptr, const int32_t* slot_row,
                              const uint8_t* colpos, int cp_stride, int nloc, int R,
                              const int32_t* elem_nodes, int nv, int stride, int32_t* ent, int4* egid,
                              void* rec, int32_t* hdr, int* overflow) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const int32_t js0 = rs_ptr[t * R];
    uint32_t off = 0;
    for (int32_t i = eptr[t]; i < eptr[t + 1]; ++i) {
        uint32_t mask = 0, cnt = 0;
        for (int k = 0; k < nloc; ++k) {
            const uint32_t jk = joff[(int64_t)i * 8 + k];
            if (jk == 0xFFFFu) continue;
            const int32_t j = js0 + (int32_t)jk;
            const int32_t r = slot_row[j];
            const uint64_t lr = (uint64_t)(r - t * R);
            const uint64_t rank = (uint64_t)(j - rs_ptr[r]);
            if (lr > 255u || rank > 255u) atomicOr(overflow, 1);
            const uint64_t cp = cp_stride == 8 ? reinterpret_cast<const uint64_t*>(colpos)[j]
                                               : (uint64_t)reinterpret_cast<const uint32_t*>(colpos)[j];
            if (nloc == 6) {
                reinterpret_cast<uint64_t*>(rec)[js0 + off + cnt] = (cp & 0xFFFFFFFFFFFFull) | (lr << 48) | (rank << 56);
            } else {
                // four 6-bit column offsets and the 8-bit tile-local row
                uint32_t r32 = (uint32_t)lr << 24;
                for (int l = 0; l < nloc; ++l) {
                    const uint32_t o = (uint32_t)(cp >> (8 * l)) & 0xFFu;
                    if (o > 63u) atomicOr(overflow, 1);
                    r32 |= (o & 63u) << (6 * l);
                }
                reinterpret_cast<uint32_t*>(rec)[js0 + off + cnt] = r32;
            }
            mask |= 1u << k;
            ++cnt;
        }
        const int64_t e = elems[i];
        const int64_t li = i - eptr[t];
        const int64_t pi = t * stride + li;  // fixed stride per tile
        // record base of wavefronts 1-3 (header words 8-10)
        if (li > 0 && li % 64 == 0 && li / 64 <= 3) hdr[t * 12 + 7 + li / 64] = (int32_t)off;
        ent[pi] = (int32_t)e;
        const int32_t* q = elem_nodes + e * nv;
        // the dof mask in spare bits of the node ids (3D: ids < 2^30, checked
        // when the tiles are built)
        egid[pi] = nv == 4 ? make_int4((int)((uint32_t)q[0] | ((mask & 3u) << 30)),
                                       (int)((uint32_t)q[1] | (((mask >> 2) & 3u) << 30)),
                                       (int)((uint32_t)q[2] | (((mask >> 4) & 3u) << 30)), q[3])
                           : make_int4(q[0], q[1], q[2], (int)mask);
        off += cnt;
    }
}

// Per-tile headers (8 ints: r0, rows, p0 lo/hi, values, first slot, first
// entry, entries), so a workgroup reads its tile's bounds with one load.
__global__ void k_tile_headers(int64_t n_tiles, int R, int64_t n_rows, const int64_t* rowptr,
                               const int32_t* rs_ptr, const int32_t* eptr, int32_t* hdr) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const int64_t r0 = t * R;
    const int64_t r1 = (r0 + R < n_rows) ? r0 + R : n_rows;
    const int64_t p0 = rowptr[r0];
    int32_t* h = hdr + t * 12;
    h[0] = rs_ptr[r1] - rs_ptr[r0];
    h[1] = (int32_t)(r1 - r0);
    h[2] = (int32_t)(uint32_t)(uint64_t)p0;
    h[3] = (int32_t)((uint64_t)p0 >> 32);
    h[4] = (int32_t)(rowptr[r1] - p0);
    h[5] = rs_ptr[r0];
    h[6] = eptr[t];  // first entry in the compact order (the entry arrays are strided)
    h[7] = eptr[t + 1] - eptr[t];
}

// Row table: each row's value offset and first slot within its tile. Both fit
// 16 bits because a tile's values and diagonal slots fit in LDS (checked when
// the tiles are built); the kernel raises the overflow flag otherwise.
__global__ void k_tile_rows(int64_t n_rows, int R, const int64_t* rowptr, const int32_t* rs_ptr,
                            uint32_t* rtab, int* overflow) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int64_t r0 = (r / R) * R;
    const int64_t pv = rowptr[r] - rowptr[r0];
    const int64_t ps = (int64_t)rs_ptr[r] - rs_ptr[r0];
    if (pv > 0xFFFF || ps > 0xFFFF) atomicOr(overflow, 1);
    rtab[r] = (uint32_t)(pv & 0xFFFF) | ((uint32_t)(ps & 0xFFFF) << 16);
}

// Header words 0-7 here; words 8-10 (the wavefronts' record bases) come from
// the record kernel, which runs first on the same stream.
static fem_status ema_headers(DofSet& ds, Pattern::Ema& E, int* overflow, hipStream_t s) {
    if (ds.pat.n_rows >= (int64_t(1) << 31))
        return fail(FEM_EOVERFLOW, "fem_pattern: more than 2^31 rows");
    FEM_HIP(hipMalloc((void**)&E.rtab, (size_t)std::max<int64_t>(ds.pat.n_rows, 1) * sizeof(uint32_t)));
    if (E.n_tiles == 0) return FEM_OK;
    hipLaunchKernelGGL(k_tile_headers, dim3(nblk(E.n_tiles)), dim3(TB), 0, s, E.n_tiles, E.R,
                       ds.pat.n_rows, ds.pat.rowptr, ds.rs_ptr, E.eptr, E.hdr);
    hipLaunchKernelGGL(k_tile_rows, dim3(nblk(ds.pat.n_rows)), dim3(TB), 0, s, ds.pat.n_rows, E.R,
                       ds.pat.rowptr, ds.rs_ptr, E.rtab, overflow);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

// Tile t's entries sit at t * stride onwards (stride = nt whenever the tiles
// fit their workgroup, the only case in which a kernel reads them), so a
// workgroup can load its entries together with its header. Unused positions
// are zero.
static fem_status ema_records(fem_mesh m, DofSet& ds, Pattern::Ema& E, int nt, hipStream_t s) {
    const int64_t n_slots = m->T * ds.nloc;
    const int stride = std::max(nt, E.max_elems);
    const int64_t n_pad = std::max<int64_t>(E.n_tiles * stride, 1);
    if (E.n_tiles * stride >= (int64_t(1) << 31))
        return fail(FEM_EOVERFLOW, "fem_pattern: more than 2^31 tile entries");
    FEM_HIP(hipMalloc((void**)&E.ent, (size_t)n_pad * sizeof(int32_t)));
    FEM_HIP(hipMalloc((void**)&E.egid, (size_t)n_pad * sizeof(int4)));
    FEM_HIP(hipMemsetAsync(E.ent, 0, (size_t)n_pad * sizeof(int32_t), s));
    FEM_HIP(hipMalloc((void**)&E.hdr, (size_t)std::max<int64_t>(E.n_tiles, 1) * 12 * sizeof(int32_t)));
    FEM_HIP(hipMemsetAsync(E.hdr, 0, (size_t)std::max<int64_t>(E.n_tiles, 1) * 12 * sizeof(int32_t), s));
    FEM_HIP(hipMemsetAsync(E.egid, 0, (size_t)n_pad * sizeof(int4), s));
    FEM_HIP(hipMalloc((void**)&E.rec, (size_t)std::max<int64_t>(n_slots, 1) * (ds.nloc == 6 ? 8 : 4)));
    TmpBufs tb;
    FEM_HIP(tb.alloc(std::max<int64_t>(n_slots, 1)));
    int32_t* slot_row = reinterpret_cast<int32_t*>(tb.vals);
    int* overflow = reinterpret_cast<int*>(tb.scan);
    FEM_HIP(hipMemsetAsync(overflow, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_slot_rows, dim3(nblk(ds.pat.n_rows)), dim3(TB), 0, s, ds.rs_ptr, ds.pat.n_rows,
                       slot_row);
    hipLaunchKernelGGL(k_ema_records, dim3(nblk(E.n_tiles)), dim3(TB), 0, s, E.eptr, E.n_tiles, E.elems,
                       E.joff, ds.rs_ptr, slot_row, ds.pat.colpos, ds.pat.cp_stride, ds.nloc, E.R,
                       m->elems, m->dim + 1, stride, E.ent, reinterpret_cast<int4*>(E.egid), E.rec, E.hdr,
                       overflow);
    FEM_HIP(hipGetLastError());
    if (fem_status st = ema_headers(ds, E, overflow, s)) return st;
    int h = 0;
    FEM_HIP(hipMemcpyAsync(&h, overflow, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP(hipStreamSynchronize(s));
    if (h) return fail(FEM_EOVERFLOW, "fem_pattern: a tile row or slot index exceeds its record field");
    // the build-only arrays
    (void)hipFree(E.elems);
    (void)hipFree(E.joff);
    E.elems = nullptr;
    E.joff = nullptr;
    return FEM_OK;
}

// Build the element-major tiles for workgroups of nt threads: pick the number of
// rows per tile so that the largest tile element list fits in nt lanes (one
// element per lane), within the LDS budget.
fem_status build_ema(fem_mesh m, DofSet& ds, int nt, hipStream_t s) {
    Pattern::Ema& E = ds.pat.ema[ema_index(nt)];
    if (E.built) return FEM_OK;
    const int kc = ds.nloc == 6 ? 2 : (ds.nloc == 4 ? 1 : 0);
    // Raviart-Thomas and 2D records hold 6-bit column offsets: rows of a
    // conforming mesh have at most 7 entries. A mesh with a longer row is not
    // conforming and is assembled by the row kernels anyway.
    if (kc != 2 && ds.pat.max_row_len > 64) {
        E.NT = nt;
        E.built = true;
        E.usable = false;
        return FEM_OK;
    }
    // elements per row: about 2 (3D Nedelec), 0.9 (3D RT), 0.7 (2D)
    int R = kc == 2 ? nt / 2 : nt;
    if (R > 255) R = 255;
    for (int attempt = 0; attempt < 6; ++attempt) {
        Pattern::Ema cand;
        fem_status st = ema_attempt(m, ds, R, s, cand);
        if (st != FEM_OK) {
            ema_free(cand);
            return st;
        }
        const bool fits = cand.max_elems <= nt &&
                          ema_lds_bytes(kc, R, cand.pmax, cand.max_slots) <= lds_limit_bytes() / 2;
        if (fits || R <= 4 || attempt == 5) {
            if (ema_lds_bytes(kc, R, cand.pmax, cand.max_slots) > lds_limit_bytes()) {
                ema_free(cand);
                return fail(FEM_EOVERFLOW, "fem_pattern: a row tile needs more LDS than the device has");
            }
            fem_status so = ema_order(cand, ds.nloc, s);
            if (so == FEM_OK) so = ema_records(m, ds, cand, nt, s);
            if (so != FEM_OK) {
                ema_free(cand);
                return so;
            }
            m->allocs.push_back(cand.eptr);
            m->allocs.push_back(cand.ent);
            m->allocs.push_back(cand.egid);
            m->allocs.push_back(cand.rec);
            m->allocs.push_back(cand.hdr);
            m->allocs.push_back(cand.rtab);
            cand.NT = nt;
            cand.built = true;
            // 3D tiles carry the dof mask in bits 30-31 of the node ids
            cand.usable = cand.max_elems <= nt && (m->dim == 2 || m->V <= (int64_t(1) << 30));
            E = cand;
            return FEM_OK;
        }
        // shrink the tile in proportion to the overshoot: exactly at first (the
        // largest tile that fits keeps the grid's last round of workgroups as
        // full as possible), with a margin once that has not converged
        const double f = cand.max_elems > nt ? (double)nt / cand.max_elems : 0.5;
        int R2 = (int)(R * f * (attempt < 2 ? 1.0 : 0.97));
        if (R2 >= R) R2 = R - 1;
        R = R2 < 4 ? 4 : R2;
        ema_free(cand);
    }
    return fail(FEM_EOVERFLOW, "fem_pattern: could not size the row tiles");
}

}  // namespace fem
