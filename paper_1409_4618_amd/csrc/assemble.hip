// Numeric assembly of K(a), M(b) (forward), its adjoint (backward) and the
// batched persistent launch.
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

template <int KC>
struct KT;
template <>
struct KT<0> {  // 2D (Nedelec / Raviart-Thomas)
    static constexpr int DIM = 2, NLOC = 3, NV = 3;
};
template <>
struct KT<1> {  // 3D Raviart-Thomas
    static constexpr int DIM = 3, NLOC = 4, NV = 4;
};
template <>
struct KT<2> {  // 3D Nedelec
    static constexpr int DIM = 3, NLOC = 6, NV = 4;
};

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
    const int nt = (int)(md.rowptr[r1] - p0);
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
                const int jj = live[u] ? j : j1 - 1;
                slot[u] = md.rs_slot[jj];
                cp[u] = load_colpos<NLOC>(md.colpos, jj);
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
template <int KC, bool MASS>
__device__ __forceinline__ void ema_scatter(typename EmaPass<KC, MASS>::T& st, uint32_t mask,
                                            const uint64_t cp[KT<KC>::NLOC], const int* rowbase,
                                            const int* rowslot, double* out, double* sdiag) {
    constexpr int NLOC = KT<KC>::NLOC;
    static_for<0, NLOC>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        if ((mask >> k) & 1u) {
            pin_state<MASS>(st);
            const typename EmaPass<KC, MASS>::T& sk = st;
            const uint64_t c = cp[k];
            const int lr = rec_row<KC>(c);
            const int base = rowbase[lr];
            const double r = ema_row<KC, MASS, k>(sk);
            const double d = ema_entry<KC, MASS, k, k>(sk, r);
            if constexpr (KC == 2) {
                sdiag[rowslot[lr] + (int)(c >> 56)] = d;
            } else {
                atomicAdd(&out[base + rec_col<KC>(c, k)], d);
            }
            static_for<0, NLOC>([&](auto ll) {
                constexpr int l = decltype(ll)::value;
                if constexpr (l != k) {
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
                if constexpr (KC == 2) cp[k] = reinterpret_cast<const uint64_t*>(md.ema_rec)[j];
                else cp[k] = reinterpret_cast<const uint32_t*>(md.ema_rec)[j];
            }
    }
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
                if ((mask >> k) & 1u)
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
                ema_scatter<KC, MASS>(ps, mask, cp, rowbase, rowslot, out, sdiag);
            }
            __syncthreads();
            if constexpr (KC == 2) {
                // diagonal entries, summed in slot order
                for (int lr = tid; lr < nrows; lr += NT) {
                    double acc = 0.0;
                    const int j1 = rowslot[lr + 1];
                    for (int j = rowslot[lr]; j < j1; ++j) acc += sdiag[j];
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

// Batched persistent kernel over element-major tiles: as k_batch, with the
// work items (mesh, element-major tile) and the tile body of the forward path.
// Each mesh keeps its own rows per tile and LDS layout; the dynamic LDS is the
// largest over the meshes.
template <int NT>
// Five wavefronts per SIMD: the kernel holds every kind's tile body, and the
// register count of the widest one (3D Nedelec) otherwise lands just above
// the five-wavefront limit.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5))) void k_batch_ema(const MeshDev* __restrict__ table,
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
            case 0: tile_ema<0, NT>(md, tile, smem_raw); break;
            case 1: tile_ema<1, NT>(md, tile, smem_raw); break;
            default: tile_ema<2, NT>(md, tile, smem_raw); break;
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

fem_status launch_batch_ema(const MeshDev* table, const int2* work, int64_t n_work, int schedule,
                            int grid, int lds_bytes, unsigned* counters, hipStream_t s) {
    if (n_work == 0) return FEM_OK;
    if (lds_bytes > lds_limit_bytes())
        return fail(FEM_EOVERFLOW, "fem_batch: a tile needs more LDS than the device has");
    FEM_HIP(set_lds(k_batch_ema<256>, lds_bytes));
    hipLaunchKernelGGL((k_batch_ema<256>), dim3((unsigned)grid), dim3(256), lds_bytes, s, table, work,
                       n_work, schedule, counters);
    FEM_HIP(hipGetLastError());
    return FEM_OK;
}

int batch_ema_blocks_per_cu(int lds_bytes) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_ema<256>, 256, lds_bytes) != hipSuccess ||
        n <= 0)
        n = 1;
    return n;
}

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
    double* partials;          // [pairs][dim] vertex-derivative partial per (node, workgroup)
    const int32_t* bptr;       // [workgroups+1] pairs of each workgroup (workgroup-major)
    const uint16_t* pst;       // [pairs] first incidence of each pair, workgroup-local
    const uint16_t* inc;       // workgroup-local incidences by workgroup, node, element
    int64_t T;
    int* err_word;
};

// Upstream weights of row k of an element (the slot's row start and column
// offsets give the positions of its n_local entries).
// Weight modes of the adjoint: separate gK and gM arrays, one array for both
// (L = u^T (K + M) u with its weights materialised), or the quadratic form
// itself, whose weight at (I, J) is u_I u_J and is formed from u without
// reading an nnz-sized array.
enum BwdMode { BWD_SEPARATE = 0, BWD_SAME = 1, BWD_QUADRATIC = 2 };

// Upstream weights of row k of element e. A missing weight array reads the
// other one and is zeroed by a select (not a branch, which would split the
// gathers into separate blocks); the launcher handles both missing. In the
// quadratic mode, uk = u[dof k] and ue[] = u[dofs of the element]: u_I u_J is
// the same product, bitwise, that the materialised weights hold.
// This lane's slot records (row start, column offsets): staged in LDS by the
// workgroup at kernel start (3D Nedelec), or read in place.
struct SlotView {
    const int32_t* base;
    const uint64_t* cp;
};

template <int NLOC, int MODE>
__device__ __forceinline__ void gather_row(const BwdArgs& A, const SlotView& sv, int k, const double ue[NLOC],
                                           double wk[NLOC], double wm[NLOC]) {
    if constexpr (MODE == BWD_QUADRATIC) {
#pragma unroll
        for (int l = 0; l < NLOC; ++l) wk[l] = wm[l] = ue[k] * ue[l];
    } else {
        const int64_t base = sv.base[k];
        const uint64_t cp = sv.cp[k];
        const double* pK = A.gK ? A.gK : A.gM;
        const double* pM = A.gM ? A.gM : A.gK;
#pragma unroll
        for (int l = 0; l < NLOC; ++l) {
            const int64_t pos = base + (int64_t)((cp >> (8 * l)) & 0xFFu);
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
}

// u at the element's dofs (quadratic mode only)
template <int NLOC, int MODE>
__device__ __forceinline__ void load_u(const BwdArgs& A, int64_t e, double ue[NLOC]) {
#pragma unroll
    for (int l = 0; l < NLOC; ++l) ue[l] = 0.0;
    if constexpr (MODE == BWD_QUADRATIC) {
#pragma unroll
        for (int l = 0; l < NLOC; ++l) ue[l] = A.u[A.elems2dofs[e * NLOC + l]];
    }
}

// Vertex derivative of local vertex v of the lane's element, into the
// workgroup's LDS slot of that incidence (summed per vertex afterwards).
__device__ __forceinline__ void store_vertex3(double* sh, int v, V3 d) {
    double* p = sh + ((int)threadIdx.x * 4 + v) * 3;
    p[0] = d.x;
    p[1] = d.y;
    p[2] = d.z;
}
__device__ __forceinline__ void store_vertex2(double* sh, int v, double dx, double dy) {
    double* p = sh + ((int)threadIdx.x * 3 + v) * 2;
    p[0] = dx;
    p[1] = dy;
}

// 3D Nedelec. With weights w_kl = s_k s_l gK_kl (gM likewise):
//   dL/da = 2/(3|J|) Phi,  Phi = sum w_kl o_k . o_l,
//   dL/db = Psi/(120|J|),  Psi = sum_ab P_ab G_ab (P: the Whitney weights of
//   the Gram entries, symmetric part accumulated once per pair),
// and the vertex derivatives from dPhi (through the edge vectors), dPsi (through
// the cofactor vectors) and d|J| = |J| tr(B^-1 dB).
template <int MODE>
__device__ void bwd_ned3(const BwdArgs& A, int64_t e, const SlotView& sv, double* sh) {
    int gid[4];
    V3 x[4];
    const int4 q4 = reinterpret_cast<const int4*>(A.elems)[e];
    gid[0] = q4.x; gid[1] = q4.y; gid[2] = q4.z; gid[3] = q4.w;
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
            gather_row<6, MODE>(A, sv, k, ue, gk, gm);
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
    const double ca = A.a ? A.a[e] : 1.0;
    const double cb = A.b ? A.b[e] : 1.0;
    if (A.ga) A.ga[e] = (2.0 / 3.0) * Phi / aJ;
    if (A.gb) A.gb[e] = Psi / (120.0 * aJ);
    if (A.partials) {
        const V3 w1 = sub(w[1], w[0]), w2 = sub(w[2], w[0]), w3 = sub(w[3], w[0]);
        const V3 dPsi[3] = {add(cross(w2, b3), cross(b2, w3)), add(cross(b3, w1), cross(w3, b1)),
                            add(cross(w1, b2), cross(b1, w2))};
        const double fk = ca * (2.0 / 3.0) / aJ;
        const double fm = cb * (1.0 / 120.0) / aJ;
        V3 d0 = {0.0, 0.0, 0.0};
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            const V3 cj = c[jj + 1];
            const V3 dj = add(scale(sub(dPhi[jj], scale(cj, Phi / J)), fk),
                              scale(sub(dPsi[jj], scale(cj, Psi / J)), fm));
            store_vertex3(sh, jj + 1, dj);
            d0 = sub(d0, dj);
        }
        store_vertex3(sh, 0, d0);
    }
    if (!(aJ > 0.0) || !isfinite(J)) atomicOr(A.err_word, ERR_DEGENERATE);
}

// 3D Raviart-Thomas
template <int MODE>
__device__ void bwd_rt3(const BwdArgs& A, int64_t e, const SlotView& sv, double* sh) {
    int gid[4];
    V3 x[4];
    const int4 q4 = reinterpret_cast<const int4*>(A.elems)[e];
    gid[0] = q4.x; gid[1] = q4.y; gid[2] = q4.z; gid[3] = q4.w;
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
        for (int k = 0; k < 4; ++k) gather_row<4, MODE>(A, sv, k, ue, GK[k], GM[k]);
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
    const double ca = A.a ? A.a[e] : 1.0;
    const double cb = A.b ? A.b[e] : 1.0;
    if (A.ga) A.ga[e] = 1.5 * hK / aJ;
    if (A.gb) A.gb[e] = Omega / (120.0 * aJ);
    if (A.partials) {
        const V3 S = add(add(g.y[1], g.y[2]), g.y[3]);
        V3 rp = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 1; p < 4; ++p) rp = add(rp, scale(g.y[p], rho[p]));
        const V3 c[3] = {cross(g.y[2], g.y[3]), cross(g.y[3], g.y[1]), cross(g.y[1], g.y[2])};
        V3 d0 = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 1; a < 4; ++a) {
            const V3 dOm = add(sub(scale(add(S, g.y[a]), 2.0 * hM), scale(add(scale(S, rho[a]), rp), 5.0)),
                               scale(z[a], 20.0));
            const V3 ck = c[a - 1];
            const V3 dK = scale(ck, -ca * 1.5 * hK / (aJ * g.J));
            const V3 dM = scale(sub(dOm, scale(ck, Omega / g.J)), cb / (120.0 * aJ));
            const V3 da = add(dK, dM);
            store_vertex3(sh, a, da);
            d0 = sub(d0, da);
        }
        store_vertex3(sh, 0, d0);
    }
    if (!(aJ > 0.0) || !isfinite(g.J)) atomicOr(A.err_word, ERR_DEGENERATE);
}

// 2D (both kinds)
template <int MODE>
__device__ void bwd_tri(const BwdArgs& A, int64_t e, const SlotView& sv, double* sh) {
    int gid[3];
    V2 x[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        gid[v] = A.elems[e * 3 + v];
        x[v] = {A.nodes[(int64_t)gid[v] * 2], A.nodes[(int64_t)gid[v] * 2 + 1]};
    }
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
        for (int k = 0; k < 3; ++k) gather_row<3, MODE>(A, sv, k, ue, GK[k], GM[k]);
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
    const double ca = A.a ? A.a[e] : 1.0;
    const double cb = A.b ? A.b[e] : 1.0;
    if (A.ga) A.ga[e] = 2.0 * hK / aJ;
    if (A.gb) A.gb[e] = Psi / (24.0 * aJ);
    if (A.partials) {
        const V2 w1 = {w[1].x - w[0].x, w[1].y - w[0].y};
        const V2 w2 = {w[2].x - w[0].x, w[2].y - w[0].y};
        const V2 dPsi[2] = {{w2.y, -w2.x}, {-w1.y, w1.x}};
        const double fk = -ca * 2.0 * hK / (aJ * g.J);
        const double fm = cb / (24.0 * aJ);
        double d0x = 0.0, d0y = 0.0;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const V2 cj = g.c[jj + 1];
            const double dx = fk * cj.x + fm * (dPsi[jj].x - cj.x * Psi / g.J);
            const double dy = fk * cj.y + fm * (dPsi[jj].y - cj.y * Psi / g.J);
            store_vertex2(sh, jj + 1, dx, dy);
            d0x -= dx;
            d0y -= dy;
        }
        store_vertex2(sh, 0, d0x, d0y);
    }
    if (!(aJ > 0.0) || !isfinite(g.J)) atomicOr(A.err_word, ERR_DEGENERATE);
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
    __shared__ uint16_t s_inc[NINC];
    __shared__ uint16_t s_pst[NINC];
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
    const int n_inc = (int)((A.T - e0 < BWD_BLOCK ? A.T - e0 : BWD_BLOCK) * NV);
    int pb0 = 0, np = 0;
    if (A.partials) {
        // the workgroup's part of the node map, into LDS first: its loads are
        // in flight while the elements are computed
        pb0 = A.bptr[blk];
        np = A.bptr[blk + 1] - pb0;
        const uint32_t* w = reinterpret_cast<const uint32_t*>(A.inc + e0 * NV);  // 4-byte aligned: e0 * NV is even
        for (int i = (int)threadIdx.x; 2 * i < n_inc; i += BWD_BLOCK)
            reinterpret_cast<uint32_t*>(s_inc)[i] = w[i];
        for (int j = (int)threadIdx.x; j < np; j += BWD_BLOCK) s_pst[j] = A.pst[pb0 + j];
    }
    if constexpr (SLOTS) {
        // the workgroup's slot records are contiguous (element-major): one
        // coalesced pass into LDS instead of a dependent load per row
        const int n_sl = n_inc / NV * NLOC;
        for (int i = (int)threadIdx.x; i < n_sl; i += BWD_BLOCK) {
            s_base[i] = A.slot_base[e0 * NLOC + i];
            s_cp[i] = A.slot_cp[e0 * NLOC + i];
        }
        __syncthreads();
    }
    const SlotView sv = SLOTS ? SlotView{s_base + (int)threadIdx.x * NLOC, s_cp + (int)threadIdx.x * NLOC}
                              : SlotView{A.slot_base + e * NLOC, A.slot_cp + e * NLOC};
    if (e < A.T) {
        if constexpr (KC == 2) bwd_ned3<MODE>(A, e, sv, sh);
        else if constexpr (KC == 1) bwd_rt3<MODE>(A, e, sv, sh);
        else bwd_tri<MODE>(A, e, sv, sh);
    }
    if (!A.partials) return;  // uniform
    __syncthreads();
    // one partial per (vertex, workgroup): the workgroup's incidences of that
    // vertex, in ascending element order
    for (int j = (int)threadIdx.x; j < np; j += BWD_BLOCK) {
        const int i0 = s_pst[j];
        const int i1 = j + 1 < np ? s_pst[j + 1] : n_inc;
        double acc[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
        for (int i = i0; i < i1; ++i) {
            const int slot = s_inc[i];
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[c] += sh[slot * DIM + c];
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) A.partials[(int64_t)(pb0 + j) * DIM + c] = acc[c];
    }
}

// gnodes[v] = sum of the node's (node, workgroup) partials, in ascending
// workgroup order (npair lists them by node).
template <int DIM>
__global__ __launch_bounds__(256) void k_node_reduce(const int32_t* node_ptr, const int32_t* npair,
                                                      const double* partials, int64_t V, double* gnodes) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    double acc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
    const int64_t j1 = node_ptr[v + 1];
#pragma unroll 4
    for (int64_t j = node_ptr[v]; j < j1; ++j) {
        const int64_t q = npair[j];
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += partials[q * DIM + c];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) gnodes[v * DIM + c] = acc[c];
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
                           const double* u, double* ga, double* gb, double* gnodes, hipStream_t s) {
    const int kc = kind_code(m->dim, kind);
    if (!u && !gK && !gM) {  // L = 0: every derivative is zero
        if (fem_status st = zero_f64(ga, m->T, s)) return st;
        if (fem_status st = zero_f64(gb, m->T, s)) return st;
        return zero_f64(gnodes, m->V * m->dim, s);
    }
    if (gnodes) {
        if (fem_status st = build_node_map(m, s)) return st;
        if (!m->elem_partials) FEM_HIP(dmalloc(m, &m->elem_partials, std::max<int64_t>(m->bwd_pairs, 1) * m->dim));
    }
    if (!u)
        if (fem_status st = build_slot_map(m, ds, s)) return st;
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
    A.partials = gnodes ? m->elem_partials : nullptr;
    A.bptr = m->bwd_bptr;
    A.pst = m->bwd_pst;
    A.inc = m->bwd_inc;
    A.T = m->T;
    A.err_word = m->err_word;
    const unsigned grid = (unsigned)(((m->T + BWD_BLOCK - 1) / BWD_BLOCK + 7) / 8 * 8);
    if (m->T > 0) {
        if (u) launch_bwd_mode<BWD_QUADRATIC>(kc, A, grid, s);
        else if (gK == gM) launch_bwd_mode<BWD_SAME>(kc, A, grid, s);
        else launch_bwd_mode<BWD_SEPARATE>(kc, A, grid, s);
        FEM_HIP(hipGetLastError());
    }
    if (gnodes && m->V > 0) {
        const unsigned gv = (unsigned)((m->V + 255) / 256);
        if (m->dim == 3)
            hipLaunchKernelGGL(k_node_reduce<3>, dim3(gv), dim3(256), 0, s, m->node_ptr, m->bwd_npair,
                               m->elem_partials, m->V, gnodes);
        else
            hipLaunchKernelGGL(k_node_reduce<2>, dim3(gv), dim3(256), 0, s, m->node_ptr, m->bwd_npair,
                               m->elem_partials, m->V, gnodes);
        FEM_HIP(hipGetLastError());
    }
    return FEM_OK;
}

}  // namespace fem
