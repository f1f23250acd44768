// Internal declarations of libfem (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fem.h"

namespace fem {

// ---------------------------------------------------------------------------
// error reporting
void set_error(const std::string& msg);
fem_status fail(fem_status st, const std::string& msg);
fem_status hip_fail(hipError_t e, const char* what);

#define FEM_HIP(call)                                              \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return ::fem::hip_fail(_e, #call);   \
    } while (0)

// device error word bits
enum : int { ERR_DEGENERATE = 1, ERR_NONFINITE = 2, ERR_RANGE = 4, ERR_OVERFLOW = 8, ERR_BOUNDS = 16 };

// Checked build (compiled with -DFEM_CHECK=1 into libfem_check.so): before a
// kernel reads or writes through an index taken from a map (element and node
// ids, slot records, row tables, dof lists, CSR positions, tile-local LDS
// offsets), it compares the index with the size of what it indexes. An index
// out of range sets ERR_BOUNDS in the error word (fem_status_query reports
// FEM_ERANGE) and the access is skipped, so the kernel still runs to its end.
// In the default build the check is the constant true and compiles away.
#ifndef FEM_CHECK
#define FEM_CHECK 0
#endif
#if defined(__HIPCC__)
__device__ __forceinline__ bool fem_in_range(int64_t i, int64_t n, int* err) {
#if FEM_CHECK
    if (i < 0 || i >= n) {
        atomicOr(err, ERR_BOUNDS);
        return false;
    }
#else
    (void)i;
    (void)n;
    (void)err;
#endif
    return true;
}
#endif

// ---------------------------------------------------------------------------
// device buffers owned by a handle
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Pattern + maps for one dof type (edges or faces) of a mesh.
struct Pattern {
    bool built = false;
    int nloc = 0;             // local dofs per element (3, 4 or 6)
    int cp_stride = 0;        // bytes per colpos record (4 or 8)
    int64_t n_rows = 0;
    int64_t nnz = 0;
    int64_t* rowptr = nullptr;    // [n_rows+1]
    int32_t* colind = nullptr;    // [nnz]
    uint8_t* colpos = nullptr;    // [n_slots][cp_stride], in row-sorted slot order
    int32_t* slot_rank = nullptr; // [n_slots] position of slot s in the row-sorted order
    int max_row_len = 0;
    // max nnz of a tile of R consecutive rows, for R = 32, 64, 128, 256
    int tile_pmax[4] = {0, 0, 0, 0};
    // Element-major tiles (one per workgroup size NT = 128, 256): R consecutive
    // rows per tile with R chosen so a tile's element list fits NT lanes; per
    // tile element entry, the tile-local slot index of each local dof whose row
    // is in the tile (0xFFFF otherwise).
    struct Ema {
        bool built = false;
        bool usable = false;        // every tile's element list fits in NT lanes
        int NT = 0;
        int R = 0;
        int64_t n_tiles = 0;
        int32_t* eptr = nullptr;    // [n_tiles+1]
        int32_t* elems = nullptr;   // [n_entries] (build only)
        uint16_t* joff = nullptr;   // [n_entries][8] (build only)
        // entry i of tile t, at t * NT + i: the element, and its node ids with
        // the entry's in-tile local dofs (6 bits) in spare bits: 3D, bits 30-31
        // of the first three ids (2 bits each); 2D, the fourth word. Records
        // of an entry start at the sum of the preceding entries' dof counts.
        int32_t* ent = nullptr;     // [n_tiles * NT]
        int32_t* egid = nullptr;    // [n_tiles * NT][4]
        // record of an in-tile slot, grouped by entry, ascending local dof:
        // column offsets (bits 0..47), tile-local row (48..55), rank of the
        // slot in its row's slot list (56..63)
        void* rec = nullptr;        // [n_slots] u64 (3D Nedelec) or u32 (the other kinds)
        // per-tile header, 12 ints: slots, rows, p0 (lo, hi), values, first
        // slot, first entry, entries, the record bases of wavefronts 1-3, 0
        // (the first row is tile * R)
        int32_t* hdr = nullptr;     // [n_tiles][12]
        // per row: its value offset in its tile (bits 0..15) and its first
        // slot in the tile's slot list (16..31)
        uint32_t* rtab = nullptr;   // [n_rows]
        int max_elems = 0;          // largest tile element list
        int max_slots = 0;          // most slots of one tile
        int pmax = 0;               // most matrix entries of one tile
    } ema[2];
};

// Dof structure of a mesh shared by the kinds that use the same dofs.
struct DofSet {
    int nloc = 0;
    int64_t n = 0;                 // number of dofs (edges or faces)
    int32_t* elems2dofs = nullptr; // [T][nloc]
    int32_t* rs_ptr = nullptr;     // [n+1] start of each dof's run of slots
    int32_t* rs_slot = nullptr;    // [T*nloc] slots (e*nloc + k) sorted by (dof, slot)
    Pattern pat;
    // adjoint gather map, element-major: for slot e*nloc + k, the CSR position
    // of its row's first entry and its column-offset record (built on first use)
    int32_t* slot_base = nullptr;  // [T*nloc] (built only for nnz < 2^31)
    uint64_t* slot_cp = nullptr;   // [T*nloc]
    bool slot_map_built = false;   // set once every step of the build has succeeded
};

}  // namespace fem

struct fem_mesh_s {
    int device = 0;
    int dim = 0;
    int64_t V = 0, T = 0;
    int32_t* elems = nullptr;        // library copy [T][dim+1]
    int32_t* edges2nodes = nullptr;  // [E][2]
    int8_t* signs_e = nullptr;       // [T][ne]
    int32_t* faces2nodes = nullptr;  // [F][3]
    int8_t* signs_f = nullptr;       // [T][4]
    fem::DofSet edges;
    fem::DofSet faces;
    // backward scratch
    // adjoint node map (built on first use): (node, workgroup) pairs in node-major
    // order; see build_node_map
    double* elem_partials = nullptr; // [pairs][dim] vertex-derivative partial of each pair
    double* qv_partials = nullptr;   // [ceil(T / 256)] workgroup sums of the quadratic-form value
    double* int_partials = nullptr;  // [ceil(T / 256)] workgroup sums of the integration routines
    double* slot_vals = nullptr;     // [T][nloc] element-local load-vector values
    // linear nodal (P1) elements (built on first use by fem_p1_pattern)
    bool p1_built = false;
    int64_t p1_nnz = 0;
    int64_t* p1_rowptr = nullptr;    // [V+1] nodal CSR pattern
    int32_t* p1_colind = nullptr;    // [p1_nnz]
    int32_t* vs_ptr = nullptr;       // [V+1] incidences (e * (dim+1) + v) of each node,
    int32_t* vs_slot = nullptr;      // [T*(dim+1)] ascending element order
    uint8_t* bnd_nodes = nullptr;    // [V] 1 for the nodes of boundary facets
    int32_t* node_ptr = nullptr;     // [V+1] pairs of each node (into bwd_npair)
    int32_t* bwd_npair = nullptr;    // [pairs] pair indices by node, ascending workgroup
    int32_t* bwd_bptr = nullptr;     // [workgroups+1] pairs of each workgroup (pairs are workgroup-major)
    uint16_t* bwd_pst = nullptr;     // [pairs] first incidence of each pair, workgroup-local
    uint16_t* bwd_inc = nullptr;     // [T*(dim+1)+1] workgroup-local incidences, by workgroup, node, element
    int64_t bwd_pairs = 0;
    bool node_map_built = false;     // set once every step of the build has succeeded
    int* err_word = nullptr;         // device error word
    // Some facet (3D face, 2D edge) has more than two elements, or two elements
    // with the same vertices. Such meshes take the row kernels, which sum every
    // entry in element order; the element-major tiles assume at most two
    // contributions per atomically summed entry.
    bool nonconforming = false;
    hipStream_t last_stream = nullptr;
    std::vector<void*> allocs;       // everything to free
};

namespace fem {

// Per-kind sizes: kind code 0 = 2D (Nedelec or Raviart-Thomas, the same
// element), 1 = 3D Raviart-Thomas, 2 = 3D Nedelec.
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

// elements per adjoint workgroup (one per lane)
constexpr int BWD_BLOCK = 256;

// memory helpers (record the allocation in the mesh)
hipError_t dmalloc(fem_mesh m, void** p, size_t bytes);
template <class T>
hipError_t dmalloc(fem_mesh m, T** p, size_t count) {
    return dmalloc(m, reinterpret_cast<void**>(p), count * sizeof(T));
}

// ---------------------------------------------------------------------------
// primitives (radix_sort.hip)
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of key.
// keys/vals hold the input; tmp buffers of the same size are needed. The sorted
// result ends up in keys/vals. `scratch` is managed internally (hipMalloc).
hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp,
                            uint32_t* vals_tmp, int64_t n, int bits, hipStream_t s);
// Exclusive prefix sum of a u32 array in place (total < 2^32).
hipError_t scan_exclusive_u32(uint32_t* data, int64_t n, hipStream_t s);
int bit_length(uint64_t v);

// ---------------------------------------------------------------------------
// topology / pattern (topology.hip)
fem_status build_topology(fem_mesh m, const double* nodes, const int32_t* elems,
                          hipStream_t s);
fem_status build_pattern(fem_mesh m, DofSet& ds, hipStream_t s);
fem_status build_node_map(fem_mesh m, hipStream_t s);
fem_status build_slot_map(fem_mesh m, DofSet& ds, hipStream_t s);
fem_status build_ema(fem_mesh m, DofSet& ds, int nt, hipStream_t s);
int ema_index(int nt);  // 128 -> 0, 256 -> 1
int ema_lds_bytes(int kind_code, int R, int pmax, int max_slots);
int default_ema_threads();

// ---------------------------------------------------------------------------
// per-tile kernels (assemble.hip)
struct MeshDev {
    // geometry / topology
    const int32_t* elems;
    const double* nodes;
    const double* a;
    const double* b;
    double* K;
    double* M;
    // pattern
    const int64_t* rowptr;
    const int32_t* rs_ptr;
    const int32_t* rs_slot;
    const uint8_t* colpos;
    int64_t n_rows;
    int64_t n_tiles;        // for the chosen rows-per-tile
    int32_t kind_code;      // 0: 2D (both kinds), 1: 3D Raviart-Thomas, 2: 3D Nedelec
    int32_t pad0;
    int* err_word;
    // element-major tiles: headers, entries, slot records
    const int32_t* ema_hdr;
    const int32_t* ema_ent;
    const int4* ema_gid;
    const void* ema_rec;        // u64 records (3D Nedelec) or u32 (the other kinds)
    const uint32_t* ema_rtab;
    int32_t ema_R;
    int32_t ema_pmax;
    int32_t ema_max_slots;
    int32_t ema_pad;
    // sizes, for the checked build's bounds checks
    int64_t T;      // elements
    int64_t V;      // nodes
    int64_t nnz;    // values of K and M
};

int kind_code(int dim, fem_kind kind);
int rows_index(int rows_per_tile);  // 32 -> 0, 64 -> 1, 128 -> 2, 256 -> 3
fem_status launch_forward(const MeshDev& md, int rows_per_tile, int pmax, hipStream_t s);
// Adjoint. Weights: gK, gM (either may be NULL = 0), or, when u is not NULL,
// the quadratic form L = u^T (K(a) + M(b)) u (weights u_I u_J, gK/gM unused).
// L (device, may be NULL; quadratic form only): the value of L as well, from
// the same pass.
fem_status launch_backward(fem_mesh m, DofSet& ds, fem_kind kind, const double* nodes,
                           const double* a, const double* b, const double* gK,
                           const double* gM, const double* u, double* ga, double* gb,
                           double* gnodes, double* L, hipStream_t s);
// Value of L = u^T (K(a) + M(b)) u into out[0] (device), through
// quadratic_value_partials(T) device doubles of scratch.
int64_t quadratic_value_partials(int64_t n_elems);
fem_status launch_quadratic_value(fem_mesh m, DofSet& ds, fem_kind kind, const double* nodes,
                                  const double* a, const double* b, const double* u, double* out,
                                  double* partials, hipStream_t s);
// out[0] = sum of n partials in a fixed order (one workgroup).
fem_status launch_sum_partials(const double* partials, int64_t n, double* out, hipStream_t s);

// ---------------------------------------------------------------------------
// integration (integrate.hip)
constexpr int FEM_QUAD_MAX = 8;          // Gauss-Legendre points per direction
constexpr int FEM_POLY_MAX_TERMS = 32;   // terms of a polynomial function
// one-dimensional Gauss-Legendre rule on [0, 1] of the conical-product rule
struct QuadRule {
    int m;
    double x[FEM_QUAD_MAX];
    double w[FEM_QUAD_MAX];
};
// a function of the catalogue (fem_function) with its parameters
struct FnArgs {
    int fn;
    int n_terms;
    int n_comp;
    // polynomial terms: coefficient, component and exponents, the integers
    // stored as such so that a kernel reads and loops on them in scalar
    // registers (they are the same for every lane); 32 bytes a term, one
    // scalar load each
    struct alignas(32) Term {
        double coef;
        int comp;
        int expo[3];
        int pad[2];
    } term[FEM_POLY_MAX_TERMS];
};
fem_status gauss_legendre01(int m, QuadRule* q);
// the handle's scratch for fixed-order element sums (2 ceil(T / 256) doubles)
fem_status ensure_int_partials(fem_mesh m);
fem_status make_fn_args(fem_function fn, int dim, const double* params, int n_params, FnArgs* F);

fem_status launch_batch(const MeshDev* table_dev, const int2* work_dev, int64_t n_work,
                        int rows_per_tile, int schedule, int grid, int pmax,
                        unsigned* counters, hipStream_t s);
int lds_limit_bytes();
int batch_blocks_per_cu(int rows_per_tile, int lds_bytes);
int cu_count();
int default_rows_per_tile(int kind_code);
fem_status launch_forward_ema(const MeshDev& md, int nt, hipStream_t s);
// batched element-major tiles (workgroups of 256 lanes)
// nt: workgroup size of the element-major tiles (128 or 256)
// kc < 0: the persistent kernel over every kind (grid workgroups, schedule
// 0..2); kc = 0..2: a plain grid over the items of that kind (one workgroup
// per item)
fem_status launch_batch_ema(const MeshDev* table_dev, const int2* work_dev, int64_t n_work,
                            int schedule, int grid, int lds_bytes, int nt, int kc, unsigned* counters,
                            hipStream_t s);
int batch_ema_blocks_per_cu(int lds_bytes, int nt);

}  // namespace fem
