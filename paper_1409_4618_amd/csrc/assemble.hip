// Numeric assembly of K(a), M(b) (forward) and the batched persistent launch
// (the adjoint is in adjoint.hip).
//
// Both forward kernels cut the CSR rows into tiles of R consecutive rows; a
// tile owns the contiguous value range rowptr[r0] .. rowptr[r0+R], accumulates
// it in LDS and writes it to HBM once with coalesced stores.
//   * Element-major tiles (k_forward_ema, the production path, further below):
//     one lane per element that has a dof among the tile's rows.
//   * Row tiles (k_forward, the fallback when a tile's element list does not
//     fit a workgroup, and a batch tiling): R*G threads, G lanes per row. A lane
//     walks its row's slots (element, local dof) in ascending element order,
//     recomputes that element's geometry in registers, forms row k of the
//     element's K and M (Section 2.4; closed forms in element.h) and adds it
//     into the row's segment of the LDS copy, at the byte offsets of the
//     scatter map: a segmented reduction in a fixed order (deterministic, no
//     atomics).
//
// Workgroups are mapped to tiles XCD by XCD (workgroup b runs on XCD b mod 8),
// so each XCD walks a contiguous range of rows and its L2 sees the reuse of
// element data between neighbouring rows.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "element.h"
#include "fem_internal.h"

namespace fem {

// The output values are written once and never read back by the kernel:
// streaming (non-temporal) stores keep them from evicting the gathered inputs
// (node coordinates, element records, scatter map) from L2 and the MALL.
__device__ __forceinline__ void store_stream(double* p, double v) {
    __builtin_nontemporal_store(v, p);
}

int kind_code(int dim, fem_kind kind) {
    if (dim == 2) return 0;
    return kind == FEM_RAVIART_THOMAS ? 1 : 2;
}

int rows_index(int rows_per_tile) {
    return rows_per_tile == 32 ? 0 : rows_per_tile == 64 ? 1 : rows_per_tile == 128 ? 2 : 3;
}

// Element data of one slot: global node ids and coordinates.
template <int KC>
struct SlotData {
    int gid[KT<KC>::NV];
    double x[KT<KC>::NV][KT<KC>::DIM];
};

// Row k of the element's a K and b M (sign-adjusted, canonical rounding of
// element.h). Returns the Jacobian determinant (for the error check).
template <int KC>
__device__ __forceinline__ double slot_row(const SlotData<KC>& d, int k, double ca, double cb,
                                           double* Kr, double* Mr) {
    if constexpr (KC == 2) {
        V3 x[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = {d.x[v][0], d.x[v][1], d.x[v][2]};
        const Geo3 g = geo3(x);
        double s[6];
        ned3_signs(d.gid, s);
        ned3_row(g, s, k, ca, cb, Kr, Mr);
        return g.J;
    } else if constexpr (KC == 1) {
        V3 x[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = {d.x[v][0], d.x[v][1], d.x[v][2]};
        const GeoRT3 g = geo_rt3(x);
        double s[4];
        rt3_signs(d.gid, s);
        rt3_row(g, s, k, ca, cb, Kr, Mr);
        return g.J;
    } else {
        V2 x[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) x[v] = {d.x[v][0], d.x[v][1]};
        const Geo2 g = geo2(x);
        double s[3];
        tri_signs(d.gid, s);
        tri_row(g, s, k, ca, cb, Kr, Mr);
        return g.J;
    }
}

template <int NLOC>
__device__ __forceinline__ uint64_t load_colpos(const uint8_t* colpos, int64_t j) {
    if constexpr (NLOC > 4) {
        return reinterpret_cast<const uint64_t*>(colpos)[j];
    } else {
        return reinterpret_cast<const uint32_t*>(colpos)[j];
    }
}

// One tile of R rows, G lanes per row: the body shared by the single-mesh and
// the batched kernels (workgroup of R*G threads).
//
// Lane g of a row handles the row's slots g, g+G, g+2G, ... in batches of U
// (all loads of a batch are issued first). The G lanes of a row add their
// element rows into the row's LDS segment in G ordered sub-rounds, so every
// matrix entry is summed in ascending slot (= element) order: deterministic,
// and bitwise symmetric because the local matrices are.
template <int KC, int R, int G, int U>
__device__ __forceinline__ void fwd_tile(const MeshDev& md, int64_t tile, double2* sKM) {
    using Tr = KT<KC>;
    constexpr int NLOC = Tr::NLOC, NV = Tr::NV, DIM = Tr::DIM;
    constexpr int NT = R * G;
    const int tid = threadIdx.x;
    const int lrow = tid / G;
    const int g = tid - lrow * G;
    const int64_t r0 = tile * R;
    const int64_t r1 = (r0 + R < md.n_rows) ? r0 + R : md.n_rows;
    const int64_t p0 = md.rowptr[r0];
    int nt = (int)(md.rowptr[r1] - p0);
#if FEM_CHECK
    if (p0 < 0 || nt < 0 || p0 + nt > md.nnz) {
        atomicOr(md.err_word, ERR_BOUNDS);
        nt = 0;
    }
#endif
    for (int i = tid; i < nt; i += NT) sKM[i] = make_double2(0.0, 0.0);
    __syncthreads();
    const int64_t r = r0 + lrow;
    bool bad = false;
    if (r < r1) {
        const int rb = (int)(md.rowptr[r] - p0);
        const int j0 = md.rs_ptr[r];
        const int j1 = md.rs_ptr[r + 1];
        for (int jb = j0; jb < j1; jb += G * U) {
            int slot[U];
            uint64_t cp[U];
            bool live[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = jb + g + G * u;
                live[u] = j < j1;
                int jj = live[u] ? j : j1 - 1;
#if FEM_CHECK
                if (!fem_in_range(jj, md.T * NLOC, md.err_word)) {
                    live[u] = false;
                    jj = 0;
                }
#endif
                slot[u] = md.rs_slot[jj];
                cp[u] = load_colpos<NLOC>(md.colpos, jj);
#if FEM_CHECK
                if (!fem_in_range(slot[u], md.T * NLOC, md.err_word)) {
                    live[u] = false;
                    slot[u] = 0;
                }
#endif
            }
            SlotData<KC> sd[U];
            double ca[U], cb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t e = slot[u] / NLOC;
                if constexpr (NV == 4) {
                    const int4 q = reinterpret_cast<const int4*>(md.elems)[e];
                    sd[u].gid[0] = q.x;
                    sd[u].gid[1] = q.y;
                    sd[u].gid[2] = q.z;
                    sd[u].gid[3] = q.w;
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v) sd[u].gid[v] = md.elems[e * NV + v];
                }
#if FEM_CHECK
                for (int v = 0; v < NV; ++v)
                    if (!fem_in_range(sd[u].gid[v], md.V, md.err_word)) {
                        live[u] = false;
                        sd[u].gid[v] = 0;
                    }
#endif
                ca[u] = md.a ? md.a[e] : 1.0;
                cb[u] = md.b ? md.b[e] : 1.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
#pragma unroll
                    for (int c = 0; c < DIM; ++c)
                        sd[u].x[v][c] = md.nodes[(int64_t)sd[u].gid[v] * DIM + c];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = slot[u] - (slot[u] / NLOC) * NLOC;
                double Kr[NLOC], Mr[NLOC];
                const double J = slot_row<KC>(sd[u], k, ca[u], cb[u], Kr, Mr);
                bad |= live[u] && (!(fabs(J) > 0.0) || !isfinite(J));
                // slot jb + g + G*u: sub-round g of step u, i.e. ascending slot order
#pragma unroll
                for (int gg = 0; gg < G; ++gg) {
                    if (g == gg && live[u]) {
#pragma unroll
                        for (int l = 0; l < NLOC; ++l) {
                            const int pos = rb + (int)((cp[u] >> (8 * l)) & 0xFFu);
                            if (!fem_in_range(pos, nt, md.err_word)) continue;
                            const double2 o = sKM[pos];
                            sKM[pos] = make_double2(o.x + Kr[l], o.y + Mr[l]);
                        }
                    }
                }
            }
        }
    }
    if (bad) atomicOr(md.err_word, ERR_DEGENERATE);
    __syncthreads();
    double* K = md.K;
    double* M = md.M;
    for (int i = tid; i < nt; i += NT) {
        const double2 v = sKM[i];
        if (K) store_stream(K + p0 + i, v.x);
        if (M) store_stream(M + p0 + i, v.y);
    }
}

// Row kernel of the single-mesh forward path (used when a mesh's element-major
// tiles do not fit a workgroup): 128 rows per tile, 2 lanes per row.
constexpr int ROW_R = 128, ROW_G = 2, ROW_U = 1;

template <int KC, int R, int G, int U>
__global__ __launch_bounds__(R * G) void k_forward(const MeshDev md) {
    extern __shared__ __align__(16) char smem_raw[];
    // XCD-aware tile order: workgroup b runs on XCD b % 8; give each XCD a
    // contiguous range of tiles.
    const int64_t per = gridDim.x / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= md.n_tiles) return;
    fwd_tile<KC, R, G, U>(md, tile, reinterpret_cast<double2*>(smem_raw));
}

// Batched persistent kernel: every workgroup pulls (mesh, tile) work items.
// schedule 0: static stride over the work list; 1 and 2: a device counter
// (2 = the host sorted the work list by decreasing cost first). The last
// workgroup to finish resets the counters, so no memset is needed between
// launches (graph replays included).
template <int R, int G, int U>
__global__ __launch_bounds__(R * G) void k_batch(const MeshDev* __restrict__ table,
                                                 const int2* __restrict__ work, int64_t n_work,
                                                 int schedule, unsigned* counters) {
    extern __shared__ __align__(16) char smem_raw[];
    __shared__ int64_t s_w;
    int64_t w = blockIdx.x;
    for (;;) {
        if (schedule != 0) {
            if (threadIdx.x == 0) s_w = (int64_t)atomicAdd(&counters[0], 1u);
            __syncthreads();
            w = s_w;
            __syncthreads();
        }
        if (w >= n_work) break;
        const int2 item = work[w];
        const MeshDev md = table[item.x];
        const int64_t tile = item.y;
        switch (md.kind_code) {
            case 0: fwd_tile<0, R, G, U>(md, tile, reinterpret_cast<double2*>(smem_raw)); break;
            case 1: fwd_tile<1, R, G, U>(md, tile, reinterpret_cast<double2*>(smem_raw)); break;
            default: fwd_tile<2, R, G, U>(md, tile, reinterpret_cast<double2*>(smem_raw)); break;
        }
        __syncthreads();
        if (schedule == 0) w += gridDim.x;
    }
    if (schedule != 0 && threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&counters[1], 1u) == gridDim.x - 1) {
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
        }
    }
}

int lds_limit_bytes() {
    static int lim = 0;
    if (!lim) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        lim = v;
    }
    return lim;
}

int cu_count() {
    static int n = 0;
    if (!n) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        n = v;
    }
    return n;
}

int default_rows_per_tile(int kc) {
    (void)kc;
    return ROW_R;
}

template <class K>
static hipError_t set_lds(K kernel, int bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int KC>
static fem_status launch_fwd_kc(const MeshDev& md, int pmax, hipStream_t s) {
    const int bytes = pmax * 16;
    if (bytes > lds_limit_bytes())
        return fail(FEM_EOVERFLOW, "fem_assemble: a row tile needs more LDS than the device has");
    FEM_HIP(set_lds(k_forward<KC, ROW_R, ROW_G, ROW_U>, bytes));
    const int64_t grid = ((md.n_tiles + 7) / 8) * 8;
    hipLaunchKernelGGL((k_forward<KC, ROW_R, ROW_G, ROW_U>), dim3((unsigned)grid), dim3(ROW_R * ROW_G),
                       bytes, s, md);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status launch_forward(const MeshDev& md, int R, int pmax, hipStream_t s) {
    if (md.n_tiles == 0) return FEM_OK;
    if (R != ROW_R) return fail(FEM_EINVAL, "fem_assemble: rows per tile does not match the row kernel");
    switch (md.kind_code) {
        case 0: return launch_fwd_kc<0>(md, pmax, s);
        case 1: return launch_fwd_kc<1>(md, pmax, s);
        default: return launch_fwd_kc<2>(md, pmax, s);
    }
}

// Batched kernel: lanes per row and slots per lane for each rows-per-tile choice.
template <int R>
struct BatchShape;
template <>
struct BatchShape<64> {
    static constexpr int G = 4, U = 2;
};
template <>
struct BatchShape<128> {
    static constexpr int G = 2, U = 1;
};
template <>
struct BatchShape<256> {
    static constexpr int G = 1, U = 4;
};

template <int R>
static fem_status launch_batch_t(const MeshDev* table, const int2* work, int64_t n_work,
                                 int schedule, int grid, int pmax, unsigned* counters,
                                 hipStream_t s) {
    constexpr int G = BatchShape<R>::G, U = BatchShape<R>::U;
    const int bytes = pmax * 16;
    FEM_HIP(set_lds(k_batch<R, G, U>, bytes));
    hipLaunchKernelGGL((k_batch<R, G, U>), dim3((unsigned)grid), dim3(R * G), bytes, s, table, work,
                       n_work, schedule, counters);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status launch_batch(const MeshDev* table, const int2* work, int64_t n_work, int R,
                        int schedule, int grid, int pmax, unsigned* counters, hipStream_t s) {
    if (n_work == 0) return FEM_OK;
    if (pmax * 16 > lds_limit_bytes())
        return fail(FEM_EOVERFLOW, "fem_batch: a row tile needs more LDS than the device has");
    switch (R) {
        case 64: return launch_batch_t<64>(table, work, n_work, schedule, grid, pmax, counters, s);
        case 128: return launch_batch_t<128>(table, work, n_work, schedule, grid, pmax, counters, s);
        default: return launch_batch_t<256>(table, work, n_work, schedule, grid, pmax, counters, s);
    }
}

int batch_blocks_per_cu(int R, int bytes) {
    int n = 0;
    hipError_t e;
    switch (R) {
        case 64:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<64, 4, 2>, 256, bytes);
            break;
        case 128:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<128, 2, 1>, 256, bytes);
            break;
        default:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<256, 1, 4>, 256, bytes);
            break;
    }
    if (e != hipSuccess || n <= 0) n = 1;
    return n;
}

// ===========================================================================
// Element-major tile ("ema"): the production forward path.
//
// A tile is R consecutive CSR rows (a contiguous value range) and the sorted
// list of the elements that have a local dof among those rows; the tile's
// element list fits in one workgroup, one lane per element. A lane gathers its
// element once and keeps the element's geometry in registers (Ned3Elem,
// Rt3Elem, TriElem); the workgroup then makes two passes over an LDS copy of
// the tile's values, one for K and one for M. In a pass every lane forms the
// entries of the rows of its element that belong to the tile (compile-time
// indices) and adds them into the LDS copy:
//   * off-diagonal entries with LDS fp64 atomic adds. In a conforming mesh an
//     off-diagonal entry has at most two contributions (the elements sharing
//     the face through both dofs), and x + y == y + x bitwise, so the result
//     does not depend on the order of the atomics;
//   * diagonal entries: with at most two contributions likewise (Raviart-
//     Thomas, 2D); in 3D Nedelec (one contribution per element around the
//     edge) into a per-slot buffer, summed by one lane per row in slot order.
// The pass ends with the tile written to HBM once, coalesced, while the LDS
// copy is cleared for the next pass; the stores of the K pass drain while the
// M pass computes. One value array in LDS instead of interleaved K and M
// halves the LDS of a tile, and the element state instead of full local
// matrices keeps the register count low: both set how many workgroups share a
// compute unit, which is what hides the gather latency.
// ===========================================================================
// LDS of a tile: values (and 3D Nedelec diagonal slots), row bases, row slot
// starts (R + 1), row diagonal offsets.
int ema_lds_bytes(int kc, int R, int pmax, int max_slots) {
    const int sd = kc == 2 ? max_slots : 0;
    return 8 * (pmax + sd) + 4 * (3 * R + 1) + 16;
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int KC>
struct EmaElem;
template <>
struct EmaElem<0> {
    using T = TriElem;
};
template <>
struct EmaElem<1> {
    using T = Rt3Elem;
};
template <>
struct EmaElem<2> {
    using T = Ned3Elem;
};

template <int KC>
__device__ __forceinline__ typename EmaElem<KC>::T ema_elem(const int gid[KT<KC>::NV],
                                                            const double x[KT<KC>::NV][KT<KC>::DIM],
                                                            double ca, double cb) {
    if constexpr (KC == 0) {
        V2 v[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] = {x[q][0], x[q][1]};
        return tri_elem(v, gid, ca, cb);
    } else {
        V3 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = {x[q][0], x[q][1], x[q][2]};
        if constexpr (KC == 1) return rt3_elem(v, gid, ca, cb);
        else return ned3_elem(v, gid, ca, cb);
    }
}

// State of one pass: the element state, except for the 3D Nedelec mass pass
// (the Gram matrix, formed when that pass starts).
template <int KC, bool MASS>
struct EmaPass {
    using T = typename EmaElem<KC>::T;
};
template <>
struct EmaPass<2, true> {
    using T = Ned3Mass;
};

template <int KC, bool MASS>
__device__ __forceinline__ typename EmaPass<KC, MASS>::T ema_pass_state(
    const typename EmaElem<KC>::T& st) {
    if constexpr (KC == 2 && MASS) return ned3_mass(st);
    else return st;
}

// Row scale s_k * (coefficient * factor) of row k, then entry (k, l).
template <int KC, bool MASS, int k>
__device__ __forceinline__ double ema_row(const typename EmaPass<KC, MASS>::T& st) {
    if constexpr (KC == 2) {
        if constexpr (MASS) return ned3_mrow<k>(st);
        else return ned3_krow<k>(st);
    } else if constexpr (KC == 1) {
        if constexpr (MASS) return rt3_mrow<k>(st);
        else return rt3_krow<k>(st);
    } else {
        if constexpr (MASS) return tri_mrow<k>(st);
        else return tri_krow<k>(st);
    }
}

template <int KC, bool MASS, int k, int l>
__device__ __forceinline__ double ema_entry(const typename EmaPass<KC, MASS>::T& st, double r) {
    if constexpr (KC == 2) {
        if constexpr (MASS) return ned3_M<k, l>(st, r);
        else return ned3_K<k, l>(st, r);
    } else if constexpr (KC == 1) {
        if constexpr (MASS) return rt3_M<k, l>(st, r);
        else return rt3_K<k, l>(st, r);
    } else {
        if constexpr (MASS) return tri_M<k, l>(st, r);
        else return tri_K<k, l>(st, r);
    }
}

// Slot record fields. 3D Nedelec (u64): column offsets 8 bits each (bits
// 0-47), tile-local row (48-55), rank in the row's slot list (56-63). Raviart-
// Thomas and 2D (u32; rows of a conforming mesh have at most 7 entries):
// column offsets 6 bits each (0-23), tile-local row (24-31).
template <int KC>
__device__ __forceinline__ int rec_row(uint64_t c) {
    return KC == 2 ? (int)((c >> 48) & 0xFFu) : (int)((c >> 24) & 0xFFu);
}
template <int KC>
__device__ __forceinline__ int rec_col(uint64_t c, int l) {
    return KC == 2 ? (int)((c >> (8 * l)) & 0xFFu) : (int)((c >> (6 * l)) & 0x3Fu);
}

// Local edges k and l of a tetrahedron share no vertex (3D Nedelec numbering).
__host__ __device__ constexpr bool ned3_opposite(int k, int l) {
    return nib(NED3_START, k) != nib(NED3_START, l) && nib(NED3_START, k) != nib(NED3_END, l) &&
           nib(NED3_END, k) != nib(NED3_START, l) && nib(NED3_END, k) != nib(NED3_END, l);
}

// One pass (K or M) of a lane's element: rows k that belong to the tile
// (bit k of mask). The slot record cp[k] gives the row's column offsets, its
// tile-local row (LDS base of the row's values) and, for the 3D Nedelec
// diagonal, the slot's rank in the row (index in the tile's diagonal buffer).
// TB: the tile's sizes for the checked build (rows, values, diagonal slots).
struct TileBounds {
    int nrows, nvals, nslots;
    int* err;
};

template <int KC, bool MASS>
__device__ __forceinline__ void ema_scatter(typename EmaPass<KC, MASS>::T& st, uint32_t mask,
                                            const uint64_t cp[KT<KC>::NLOC], const int* rowbase,
                                            const int* rowslot, double* out, double* sdiag,
                                            const TileBounds& tb) {
    constexpr int NLOC = KT<KC>::NLOC;
    static_for<0, NLOC>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        if ((mask >> k) & 1u) {
            pin_state<MASS>(st);
            const typename EmaPass<KC, MASS>::T& sk = st;
            const uint64_t c = cp[k];
            const int lr = rec_row<KC>(c);
#if FEM_CHECK
            if (!fem_in_range(lr, tb.nrows, tb.err)) return;
#endif
            const int base = rowbase[lr];
            const double r = ema_row<KC, MASS, k>(sk);
            const double d = ema_entry<KC, MASS, k, k>(sk, r);
            if constexpr (KC == 2) {
#if FEM_CHECK
                if (fem_in_range(rowslot[lr] + (int)(c >> 56), tb.nslots, tb.err))
#endif
                    sdiag[rowslot[lr] + (int)(c >> 56)] = d;
            } else {
#if FEM_CHECK
                if (fem_in_range(base + rec_col<KC>(c, k), tb.nvals, tb.err))
#endif
                    atomicAdd(&out[base + rec_col<KC>(c, k)], d);
            }
            static_for<0, NLOC>([&](auto ll) {
                constexpr int l = decltype(ll)::value;
                if constexpr (l != k) {
#if FEM_CHECK
                    if (!fem_in_range(base + rec_col<KC>(c, l), tb.nvals, tb.err)) return;
#endif
                    double* o = &out[base + rec_col<KC>(c, l)];
                    const double v = ema_entry<KC, MASS, k, l>(sk, r);
                    // Entries whose two dofs determine the element (3D
                    // Nedelec opposite edges span all four vertices; two faces
                    // of a tetrahedron or two edges of a triangle span all its
                    // vertices) have this element as their only contribution
                    // in a conforming mesh, the only kind these tiles are used
                    // for: a store onto the zeroed copy equals the atomic add
                    // bitwise.
                    if constexpr (KC != 2 || ned3_opposite(k, l)) *o = v;
                    else atomicAdd(o, v);
                }
            });
        }
    });
}

template <int KC, int NT>
__device__ __forceinline__ void tile_ema(const MeshDev& md, int64_t tile, char* smem) {
    using Tr = KT<KC>;
    constexpr int NLOC = Tr::NLOC, NV = Tr::NV, DIM = Tr::DIM;
    const int tid = threadIdx.x;
    const int R = md.ema_R;
    // header of the tile: words 0-7 here; words 8-10, the record bases of
    // wavefronts 1-3, are read by the wavefront that needs one (below)
    const int4 h0 = reinterpret_cast<const int4*>(md.ema_hdr)[3 * tile];
    const int4 h1 = reinterpret_cast<const int4*>(md.ema_hdr)[3 * tile + 1];
    const int64_t r0 = tile * R;
    const int nslots = h0.x;
    const int nrows = h0.y;
    const int64_t p0 = (int64_t)(((uint64_t)(uint32_t)h0.w << 32) | (uint64_t)(uint32_t)h0.z);
    const int nt = h1.x;
    const int js0 = h1.y;
    const int ne = h1.w;  // <= NT (checked when the tiles are built)
    // LDS layout
    double* out = reinterpret_cast<double*>(smem);
    double* sdiag = out + md.ema_pmax;
    int* rowbase = reinterpret_cast<int*>(sdiag + (KC == 2 ? md.ema_max_slots : 0));
    int* rowslot = rowbase + R;
    int* rowdiag = rowslot + R + 1;

    // this lane's element: entry and node ids first, so their latency
    // overlaps the LDS set-up below. A tile's entries sit at a fixed stride,
    // so they load together with the header. The entry's in-tile dofs (mask)
    // ride in spare bits of the node ids; its records start at the sum of the
    // preceding entries' dof counts (padding entries have none).
    const int en = md.ema_ent[tile * NT + tid];
    const int4 q = md.ema_gid[tile * NT + tid];  // the element's node ids, streamed with the entry
    const bool have = tid < ne;
    int64_t e = 0;
    uint32_t mask = 0;
    int gid[NV];
    uint64_t cp[NLOC];
#pragma unroll
    for (int v = 0; v < NV; ++v) gid[v] = 0;
#pragma unroll
    for (int k = 0; k < NLOC; ++k) cp[k] = 0;
    if constexpr (NV == 4) {
        mask = (((uint32_t)q.x >> 30) & 3u) | ((((uint32_t)q.y >> 30) & 3u) << 2) |
               ((((uint32_t)q.z >> 30) & 3u) << 4);
    } else {
        mask = (uint32_t)q.w;
    }
    if (have) {
        e = en;
        if constexpr (NV == 4) {
            gid[0] = q.x & 0x3FFFFFFF;
            gid[1] = q.y & 0x3FFFFFFF;
            gid[2] = q.z & 0x3FFFFFFF;
            gid[3] = q.w;
        } else {
            gid[0] = q.x;
            gid[1] = q.y;
            gid[2] = q.z;
        }
    }
#if FEM_CHECK
    if (have) {
        bool ok = fem_in_range(e, md.T, md.err_word);
        for (int v = 0; v < NV; ++v) ok = ok && fem_in_range(gid[v], md.V, md.err_word);
        if (!ok) {
            e = 0;
            for (int v = 0; v < NV; ++v) gid[v] = 0;
        }
    }
#endif
    // record offset: the wavefront's base (tile header word 7 + wavefront)
    // plus the exclusive prefix of the dof counts within the wavefront (one
    // ballot per bit of a count <= 6, each counted below the lane at once)
    const uint32_t cnt = __popc(mask);
    int in_wave = 0;
#pragma unroll
    for (int bit = 0; bit < 3; ++bit) {
        const uint64_t bb = __ballot(cnt & (1u << bit));
        in_wave += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u)) << bit;
    }
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);  // uniform in the wavefront: a scalar load
    const int wbase = wave == 0 ? 0 : md.ema_hdr[tile * 12 + 7 + wave];
    if (have) {
        const int64_t roff = (int64_t)js0 + wbase + in_wave;
#pragma unroll
        for (int k = 0; k < NLOC; ++k)
            if ((mask >> k) & 1u) {
                const int64_t j = roff + __popc(mask & ((1u << k) - 1u));
#if FEM_CHECK
                if (!fem_in_range(j, md.T * NLOC, md.err_word)) continue;
#endif
                if constexpr (KC == 2) cp[k] = reinterpret_cast<const uint64_t*>(md.ema_rec)[j];
                else cp[k] = reinterpret_cast<const uint32_t*>(md.ema_rec)[j];
            }
    }
#if FEM_CHECK
    // a tile's rows, values and slots within the pattern
    const bool tile_ok = fem_in_range(r0 + nrows - 1, md.n_rows, md.err_word) &&
                         fem_in_range(p0 + nt - 1, md.nnz, md.err_word) && nt <= md.ema_pmax && nrows <= R &&
                         (KC != 2 || nslots <= md.ema_max_slots);
    if (!tile_ok) {
        atomicOr(md.err_word, ERR_BOUNDS);
        return;  // uniform: the whole workgroup leaves before its first barrier
    }
#endif
    const TileBounds tb{nrows, nt, nslots, md.err_word};
    // phase 0: clear the values, row bases (and row slot starts)
    for (int i = tid; i < nt; i += NT) out[i] = 0.0;
    for (int lr = tid; lr < nrows; lr += NT) {
        const uint32_t rt = md.ema_rtab[r0 + lr];
        rowbase[lr] = (int)(rt & 0xFFFFu);
        if constexpr (KC == 2) rowslot[lr] = (int)(rt >> 16);
    }
    if (KC == 2 && tid == 0) rowslot[nrows] = nslots;
    __syncthreads();

    // gather (coordinates, coefficients), then the element state
    typename EmaElem<KC>::T st;
    double ca = 1.0, cb = 1.0;
    bool bad = false;
    if (have) {
        double x[NV][DIM];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int c = 0; c < DIM; ++c) x[v][c] = md.nodes[(int64_t)gid[v] * DIM + c];
        if (md.a) ca = md.a[e];
        if (md.b) cb = md.b[e];
        if constexpr (KC == 2) {
#pragma unroll
            for (int k = 0; k < NLOC; ++k)
#if FEM_CHECK
                if (((mask >> k) & 1u) && fem_in_range(rec_row<KC>(cp[k]), nrows, md.err_word))
#else
                if ((mask >> k) & 1u)
#endif
                    rowdiag[rec_row<KC>(cp[k])] = rec_col<KC>(cp[k], k);
        }
        st = ema_elem<KC>(gid, x, ca, cb);
        bad = !(fabs(st.J) > 0.0) || !isfinite(st.J);
    }
    if (bad) atomicOr(md.err_word, ERR_DEGENERATE);

    // two passes: K (coefficient a), then M (coefficient b)
    static_for<0, 2>([&](auto pp) {
        constexpr bool MASS = decltype(pp)::value == 1;
        double* dst = MASS ? md.M : md.K;
        if (dst) {
            if (have) {
                typename EmaPass<KC, MASS>::T ps = ema_pass_state<KC, MASS>(st);
                ema_scatter<KC, MASS>(ps, mask, cp, rowbase, rowslot, out, sdiag, tb);
            }
            __syncthreads();
            if constexpr (KC == 2) {
                // diagonal entries, summed in slot order
                for (int lr = tid; lr < nrows; lr += NT) {
                    double acc = 0.0;
                    const int j1 = rowslot[lr + 1];
                    for (int j = rowslot[lr]; j < j1; ++j) {
#if FEM_CHECK
                        if (!fem_in_range(j, nslots, md.err_word)) break;
#endif
                        acc += sdiag[j];
                    }
#if FEM_CHECK
                    if (fem_in_range(rowbase[lr] + rowdiag[lr], nt, md.err_word))
#endif
                        out[rowbase[lr] + rowdiag[lr]] = acc;
                }
                __syncthreads();
            }
            // write the tile once; clear the LDS copy for the next pass.
            // Raviart-Thomas and 2D start the loop at the 128-byte line at or
            // below p0, so each wavefront's 512-byte store covers whole lines
            // (128^3 Raviart-Thomas: 7 % faster). 3D Nedelec, whose stiffness
            // stores drain while the mass pass computes, measured 2 % slower
            // that way and keeps the plain loop.
            const int shift = KC == 2 ? 0 : (int)(p0 & 15);
            for (int i = tid - shift; i < nt; i += NT) {
                if (i >= 0) {
                    const double v = out[i];
                    out[i] = 0.0;
                    store_stream(dst + p0 + i, v);
                }
            }
            if (!MASS) __syncthreads();
        }
    });
}

template <int KC, int NT>
__global__ __launch_bounds__(NT) void k_forward_ema(const MeshDev md) {
    extern __shared__ __align__(16) char smem_raw[];
    const int64_t per = gridDim.x / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= md.n_tiles) return;
    tile_ema<KC, NT>(md, tile, smem_raw);
}

int default_ema_threads() {
    static int v = 0;
    if (!v) {
        v = 256;
        const char* s = std::getenv("FEM_EMA_THREADS");
        if (s && std::atoi(s) == 128) v = 128;
    }
    return v;
}

template <int KC, int NT>
static fem_status launch_ema_t(const MeshDev& md, hipStream_t s) {
    const int bytes = ema_lds_bytes(KC, md.ema_R, md.ema_pmax, md.ema_max_slots);
    if (bytes > lds_limit_bytes())
        return fail(FEM_EOVERFLOW, "fem_assemble: a row tile needs more LDS than the device has");
    FEM_HIP(set_lds(k_forward_ema<KC, NT>, bytes));
    const int64_t grid = ((md.n_tiles + 7) / 8) * 8;
    hipLaunchKernelGGL((k_forward_ema<KC, NT>), dim3((unsigned)grid), dim3(NT), bytes, s, md);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status launch_forward_ema(const MeshDev& md, int nt, hipStream_t s) {
    if (md.n_tiles == 0) return FEM_OK;
    if (nt == 128) {
        switch (md.kind_code) {
            case 0: return launch_ema_t<0, 128>(md, s);
            case 1: return launch_ema_t<1, 128>(md, s);
            default: return launch_ema_t<2, 128>(md, s);
        }
    }
    switch (md.kind_code) {
        case 0: return launch_ema_t<0, 256>(md, s);
        case 1: return launch_ema_t<1, 256>(md, s);
        default: return launch_ema_t<2, 256>(md, s);
    }
}

// Batched persistent kernels over element-major tiles: as k_batch, with the
// work items (mesh, element-major tile) and the tile body of the forward path.
// Each mesh keeps its own rows per tile and LDS layout; the dynamic LDS is the
// largest over the meshes. The work loop: a static stride over the items, or
// items taken from a device counter that resets itself when the last
// workgroup leaves (no memset, so graph replays are valid).
template <int NT, class Body>
__device__ __forceinline__ void batch_work_loop(const int2* __restrict__ work, int64_t n_work, int schedule,
                                                unsigned* counters, Body&& body) {
    __shared__ int64_t s_w;
    int64_t w = blockIdx.x;
    for (;;) {
        if (schedule != 0) {
            if (threadIdx.x == 0) s_w = (int64_t)atomicAdd(&counters[0], 1u);
            __syncthreads();
            w = s_w;
            __syncthreads();
        }
        if (w >= n_work) break;
        body(work[w]);
        __syncthreads();
        if (schedule == 0) w += gridDim.x;
    }
    if (schedule != 0 && threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&counters[1], 1u) == gridDim.x - 1) {
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
        }
    }
}

// Every kind in one kernel (a wave-uniform branch per tile). Five wavefronts
// per SIMD: the kernel holds every kind's tile body, and the register count of
// the widest one (3D Nedelec) otherwise lands just above the five-wavefront
// limit.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5))) void k_batch_ema(const MeshDev* __restrict__ table,
                                                  const int2* __restrict__ work, int64_t n_work,
                                                  int schedule, unsigned* counters) {
    extern __shared__ __align__(16) char smem_raw[];
    batch_work_loop<NT>(work, n_work, schedule, counters, [&](int2 item) {
        const MeshDev md = table[item.x];
        switch (md.kind_code) {
            case 0: tile_ema<0, NT>(md, item.y, smem_raw); break;
            case 1: tile_ema<1, NT>(md, item.y, smem_raw); break;
            default: tile_ema<2, NT>(md, item.y, smem_raw); break;
        }
    });
}

template <int NT>
static fem_status launch_batch_ema_t(const MeshDev* table, const int2* work, int64_t n_work, int schedule,
                                     int grid, int lds_bytes, unsigned* counters, hipStream_t s) {
    FEM_HIP(set_lds(k_batch_ema<NT>, lds_bytes));
    hipLaunchKernelGGL((k_batch_ema<NT>), dim3((unsigned)grid), dim3(NT), lds_bytes, s, table, work, n_work,
                       schedule, counters);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

// The items of one element kind as a plain grid, one workgroup per item,
// scheduled by the hardware dispatcher in item order: no work loop, so the
// kernel holds one kind's tile body with the registers (and occupancy) of the
// single-mesh kernel of that kind. One such launch per kind present.
template <int KC, int NT>
__global__ __launch_bounds__(NT) void k_batch_ema_grid(const MeshDev* __restrict__ table,
                                                       const int2* __restrict__ work) {
    extern __shared__ __align__(16) char smem_raw[];
    const int2 item = work[blockIdx.x];
    tile_ema<KC, NT>(table[item.x], item.y, smem_raw);
}

template <int KC, int NT>
static fem_status launch_batch_ema_grid_t(const MeshDev* table, const int2* work, int64_t n_work, int lds_bytes,
                                          hipStream_t s) {
    FEM_HIP(set_lds(k_batch_ema_grid<KC, NT>, lds_bytes));
    hipLaunchKernelGGL((k_batch_ema_grid<KC, NT>), dim3((unsigned)n_work), dim3(NT), lds_bytes, s, table, work);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

fem_status launch_batch_ema(const MeshDev* table, const int2* work, int64_t n_work, int schedule,
                            int grid, int lds_bytes, int nt, int kc, unsigned* counters, hipStream_t s) {
    if (n_work == 0) return FEM_OK;
    if (lds_bytes > lds_limit_bytes())
        return fail(FEM_EOVERFLOW, "fem_batch: a tile needs more LDS than the device has");
    if (kc < 0) {
        if (nt == 128)
            return launch_batch_ema_t<128>(table, work, n_work, schedule, grid, lds_bytes, counters, s);
        return launch_batch_ema_t<256>(table, work, n_work, schedule, grid, lds_bytes, counters, s);
    }
    if (n_work >= (int64_t(1) << 31)) return fail(FEM_EOVERFLOW, "fem_batch: more than 2^31 - 1 tiles of one kind");
    if (nt == 128) {
        if (kc == 0) return launch_batch_ema_grid_t<0, 128>(table, work, n_work, lds_bytes, s);
        if (kc == 1) return launch_batch_ema_grid_t<1, 128>(table, work, n_work, lds_bytes, s);
        return launch_batch_ema_grid_t<2, 128>(table, work, n_work, lds_bytes, s);
    }
    if (kc == 0) return launch_batch_ema_grid_t<0, 256>(table, work, n_work, lds_bytes, s);
    if (kc == 1) return launch_batch_ema_grid_t<1, 256>(table, work, n_work, lds_bytes, s);
    return launch_batch_ema_grid_t<2, 256>(table, work, n_work, lds_bytes, s);
}

int batch_ema_blocks_per_cu(int lds_bytes, int nt) {
    int n = 0;
    const hipError_t e =
        nt == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_ema<128>, 128, lds_bytes)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_ema<256>, 256, lds_bytes);
    if (e != hipSuccess || n <= 0) n = 1;
    return n;
}

}  // namespace fem
