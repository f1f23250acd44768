// C ABI of libfem (declared in include/fem.h): argument checking, handle
// lifetime, the batched launch with its autotuner and HIP-graph replay.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "fem_internal.h"
#include "tune_cache.h"

namespace fem {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

fem_status fail(fem_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

fem_status hip_fail(hipError_t e, const char* what) {
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    set_error(msg);
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? FEM_ENOMEM : FEM_EHIP;
}

hipError_t dmalloc(fem_mesh m, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) m->allocs.push_back(*p);
    return e;
}

static DofSet& dofset(fem_mesh m, fem_kind kind) {
    return (m->dim == 3 && kind == FEM_RAVIART_THOMAS) ? m->faces : m->edges;
}

static int env_rows_per_tile(int kc) { return default_rows_per_tile(kc); }

// The element-major tile kernel is the forward path; FEM_FWD_PATH=rows selects
// the row-lane kernels instead (kept for comparison measurements).
static bool use_row_path() {
    static int v = -1;
    if (v < 0) {
        const char* s = std::getenv("FEM_FWD_PATH");
        v = (s && std::strcmp(s, "rows") == 0) ? 1 : 0;
    }
    return v == 1;
}

static void fill_ema(const DofSet& ds, int nt, MeshDev* md) {
    const Pattern::Ema& E = ds.pat.ema[ema_index(nt)];
    md->n_tiles = E.n_tiles;
    md->ema_hdr = E.hdr;

    md->ema_ent = E.ent;
    md->ema_gid = reinterpret_cast<const int4*>(E.egid);
    md->ema_rec = E.rec;
    md->ema_rtab = E.rtab;
    md->ema_R = E.R;
    md->ema_pmax = E.pmax;
    md->ema_max_slots = E.max_slots;
}

}  // namespace fem

using namespace fem;

extern "C" {

const char* fem_last_error(void) { return g_last_error.c_str(); }

const char* fem_version(void) { return "libfem 1.0 (gfx950, fp64)"; }

void fem_mesh_destroy(fem_mesh m) {
    if (!m) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    for (void* p : m->allocs) (void)hipFree(p);
    (void)hipSetDevice(cur);
    delete m;
}

fem_status fem_topology(const double* nodes, int64_t n_nodes, int dim, const int32_t* elems,
                        int64_t n_elems, void* stream, fem_mesh* out) {
    g_last_error.clear();
    if (!out) return fail(FEM_EINVAL, "fem_topology: out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(FEM_EINVAL, "fem_topology: dim must be 2 or 3");
    if (n_nodes <= 0 || n_elems <= 0) return fail(FEM_EINVAL, "fem_topology: empty mesh");
    if (!nodes || !elems) return fail(FEM_EINVAL, "fem_topology: nodes or elems is NULL");
    const int ne = dim == 3 ? 6 : 3;
    if (n_nodes * dim >= (int64_t(1) << 31) || n_elems * ne >= (int64_t(1) << 31) ||
        n_elems * (dim + 1) >= (int64_t(1) << 31))
        return fail(FEM_EOVERFLOW, "fem_topology: mesh exceeds the int32 index limits");
    fem_mesh m = new fem_mesh_s();
    (void)hipGetDevice(&m->device);
    m->dim = dim;
    m->V = n_nodes;
    m->T = n_elems;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    fem_status st = build_topology(m, nodes, elems, s);
    if (st != FEM_OK) {
        std::string msg = g_last_error;
        fem_mesh_destroy(m);
        g_last_error = msg;
        return st;
    }
    *out = m;
    return FEM_OK;
}

fem_status fem_mesh_counts(fem_mesh m, int64_t* n_nodes, int64_t* n_elems, int64_t* n_edges,
                           int64_t* n_faces, int* dim) {
    if (!m) return fail(FEM_EINVAL, "fem_mesh_counts: mesh is NULL");
    if (n_nodes) *n_nodes = m->V;
    if (n_elems) *n_elems = m->T;
    if (n_edges) *n_edges = m->edges.n;
    if (n_faces) *n_faces = m->dim == 3 ? m->faces.n : 0;
    if (dim) *dim = m->dim;
    return FEM_OK;
}

fem_status fem_mesh_topology(fem_mesh m, const int32_t** edges2nodes, const int32_t** elems2edges,
                             const int8_t** signs_e, const int32_t** faces2nodes,
                             const int32_t** elems2faces, const int8_t** signs_f) {
    if (!m) return fail(FEM_EINVAL, "fem_mesh_topology: mesh is NULL");
    if (edges2nodes) *edges2nodes = m->edges2nodes;
    if (elems2edges) *elems2edges = m->edges.elems2dofs;
    if (signs_e) *signs_e = m->signs_e;
    if (faces2nodes) *faces2nodes = m->dim == 3 ? m->faces2nodes : nullptr;
    if (elems2faces) *elems2faces = m->dim == 3 ? m->faces.elems2dofs : nullptr;
    if (signs_f) *signs_f = m->dim == 3 ? m->signs_f : nullptr;
    return FEM_OK;
}

fem_status fem_pattern(fem_mesh m, fem_kind kind, void* stream, int64_t* n_rows, int64_t* nnz,
                       const int64_t** rowptr, const int32_t** colind) {
    g_last_error.clear();
    if (!m) return fail(FEM_EINVAL, "fem_pattern: mesh is NULL");
    if (kind != FEM_NEDELEC && kind != FEM_RAVIART_THOMAS) return fail(FEM_EINVAL, "fem_pattern: bad kind");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    DofSet& ds = dofset(m, kind);
    if (fem_status st = build_pattern(m, ds, s)) return st;
    // (a mesh with an edge or face shared by very many elements can leave a
    // tile whose element list does not fit one workgroup: the row kernel then
    // takes the mesh, see fem_assemble)
    if (!use_row_path())
        if (fem_status st = build_ema(m, ds, default_ema_threads(), s)) return st;
    if (n_rows) *n_rows = ds.pat.n_rows;
    if (nnz) *nnz = ds.pat.nnz;
    if (rowptr) *rowptr = ds.pat.rowptr;
    if (colind) *colind = ds.pat.colind;
    return FEM_OK;
}

static fem_status fill_meshdev(fem_mesh m, fem_kind kind, const double* nodes, const double* a,
                               const double* b, double* K, double* M, int R, MeshDev* md) {
    DofSet& ds = dofset(m, kind);
    if (!ds.pat.built) return fail(FEM_ENOTREADY, "pattern not built: call fem_pattern first");
    md->elems = m->elems;
    md->nodes = nodes;
    md->a = a;
    md->b = b;
    md->K = K;
    md->M = M;
    md->rowptr = ds.pat.rowptr;
    md->rs_ptr = ds.rs_ptr;
    md->rs_slot = ds.rs_slot;
    md->colpos = ds.pat.colpos;
    md->n_rows = ds.pat.n_rows;
    md->n_tiles = (ds.pat.n_rows + R - 1) / R;
    md->kind_code = kind_code(m->dim, kind);
    md->err_word = m->err_word;
    md->T = m->T;
    md->V = m->V;
    md->nnz = ds.pat.nnz;
    return FEM_OK;
}

fem_status fem_assemble(fem_mesh m, fem_kind kind, const double* nodes, const double* a,
                        const double* b, double* K_vals, double* M_vals, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_assemble: mesh is NULL");
    if (kind != FEM_NEDELEC && kind != FEM_RAVIART_THOMAS) return fail(FEM_EINVAL, "fem_assemble: bad kind");
    if (!nodes) return fail(FEM_EINVAL, "fem_assemble: nodes is NULL");
    if (!K_vals && !M_vals) return FEM_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    const int kc = kind_code(m->dim, kind);
    if (!use_row_path()) {
        const int nt = default_ema_threads();
        const Pattern::Ema& E = dofset(m, kind).pat.ema[ema_index(nt)];
        if (!E.built) return fail(FEM_ENOTREADY, "pattern not built: call fem_pattern first");
        if (E.usable && !m->nonconforming) {
            MeshDev md;
            if (fem_status st = fill_meshdev(m, kind, nodes, a, b, K_vals, M_vals, 128, &md))
                return st;
            fill_ema(dofset(m, kind), nt, &md);
            return launch_forward_ema(md, nt, s);
        }
    }
    const int R = env_rows_per_tile(kc);
    MeshDev md;
    if (fem_status st = fill_meshdev(m, kind, nodes, a, b, K_vals, M_vals, R, &md)) return st;
    const int pmax = dofset(m, kind).pat.tile_pmax[rows_index(R)];
    return launch_forward(md, R, pmax, s);
}

fem_status fem_assemble_backward(fem_mesh m, fem_kind kind, const double* nodes, const double* a,
                                 const double* b, const double* gK, const double* gM, double* ga,
                                 double* gb, double* gnodes, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_assemble_backward: mesh is NULL");
    if (kind != FEM_NEDELEC && kind != FEM_RAVIART_THOMAS)
        return fail(FEM_EINVAL, "fem_assemble_backward: bad kind");
    if (!nodes) return fail(FEM_EINVAL, "fem_assemble_backward: nodes is NULL");
    DofSet& ds = dofset(m, kind);
    if (!ds.pat.built) return fail(FEM_ENOTREADY, "pattern not built: call fem_pattern first");
    if (!ga && !gb && !gnodes) return FEM_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    return launch_backward(m, ds, kind, nodes, a, b, gK, gM, nullptr, ga, gb, gnodes, nullptr, s);
}

fem_status fem_assemble_backward_quadratic(fem_mesh m, fem_kind kind, const double* nodes,
                                           const double* a, const double* b, const double* u,
                                           double* ga, double* gb, double* gnodes, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_assemble_backward_quadratic: mesh is NULL");
    if (kind != FEM_NEDELEC && kind != FEM_RAVIART_THOMAS)
        return fail(FEM_EINVAL, "fem_assemble_backward_quadratic: bad kind");
    if (!nodes || !u) return fail(FEM_EINVAL, "fem_assemble_backward_quadratic: nodes or u is NULL");
    DofSet& ds = dofset(m, kind);
    if (!ds.pat.built) return fail(FEM_ENOTREADY, "pattern not built: call fem_pattern first");
    if (!ga && !gb && !gnodes) return FEM_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    return launch_backward(m, ds, kind, nodes, a, b, nullptr, nullptr, u, ga, gb, gnodes, nullptr, s);
}

fem_status fem_quadratic_value_adjoint(fem_mesh m, fem_kind kind, const double* nodes, const double* a,
                                       const double* b, const double* u, double* L, double* ga, double* gb,
                                       double* gnodes, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_quadratic_value_adjoint: mesh is NULL");
    if (kind != FEM_NEDELEC && kind != FEM_RAVIART_THOMAS)
        return fail(FEM_EINVAL, "fem_quadratic_value_adjoint: bad kind");
    if (!nodes || !u || !L) return fail(FEM_EINVAL, "fem_quadratic_value_adjoint: nodes, u or L is NULL");
    DofSet& ds = dofset(m, kind);
    if (!ds.pat.built) return fail(FEM_ENOTREADY, "pattern not built: call fem_pattern first");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    if (!ga && !gb && !gnodes) return fem_quadratic_value(m, kind, nodes, a, b, u, L, stream);
    return launch_backward(m, ds, kind, nodes, a, b, nullptr, nullptr, u, ga, gb, gnodes, L, s);
}

fem_status fem_quadratic_value(fem_mesh m, fem_kind kind, const double* nodes, const double* a,
                               const double* b, const double* u, double* L, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_quadratic_value: mesh is NULL");
    if (kind != FEM_NEDELEC && kind != FEM_RAVIART_THOMAS)
        return fail(FEM_EINVAL, "fem_quadratic_value: bad kind");
    if (!nodes || !u || !L) return fail(FEM_EINVAL, "fem_quadratic_value: nodes, u or L is NULL");
    DofSet& ds = dofset(m, kind);
    if (!ds.pat.built) return fail(FEM_ENOTREADY, "pattern not built: call fem_pattern first");
    if (!m->qv_partials) FEM_HIP(dmalloc(m, &m->qv_partials, std::max<int64_t>(1, quadratic_value_partials(m->T))));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    return launch_quadratic_value(m, ds, kind, nodes, a, b, u, L, m->qv_partials, s);
}

fem_status fem_status_query(fem_mesh m) {
    if (!m) return fail(FEM_EINVAL, "fem_status_query: mesh is NULL");
    int err = 0;
    FEM_HIP(hipStreamSynchronize(m->last_stream));
    FEM_HIP(hipMemcpy(&err, m->err_word, sizeof(int), hipMemcpyDeviceToHost));
    FEM_HIP(hipMemset(m->err_word, 0, sizeof(int)));
    if (err & ERR_BOUNDS)
        return fail(FEM_ERANGE, "checked build: a kernel met a map index outside the array it indexes");
    if (err & ERR_NONFINITE) return fail(FEM_ENONFINITE, "a Jacobian determinant was not finite");
    if (err & ERR_DEGENERATE) return fail(FEM_EDEGENERATE, "an element had a zero or non-finite Jacobian determinant");
    return FEM_OK;
}

}  // extern "C"

// ===========================================================================
// batched assembly
// ===========================================================================
struct fem_batch_s {
    int device = 0;
    std::vector<fem_mesh> meshes;
    std::vector<fem_kind> kinds;
    std::vector<MeshDev> host_table;
    bool bound = false;
    MeshDev* table_dev = nullptr;
    int2* work_dev = nullptr;
    int64_t work_cap = 0;
    int64_t n_work = 0;
    unsigned* counters = nullptr;
    int R = 128;            // rows per row tile (64/128/256), 0 = element-major tiles
    int schedule = 1;
    int grid = 0;
    int pmax = 0;
    int lds_bytes = 0;      // element-major tiles: largest tile LDS over the meshes
    bool ema_ok = false;    // every mesh has usable element-major tiles (256 lanes)
    int nt = 256;           // element-major tiles: workgroup size, 128 or 256
    int ema128 = -1;        // 128-lane tiles: -1 not built yet, 0 unusable, 1 usable
    // element-major tiles, schedules 3-4: the work items grouped by element
    // kind, one plain-grid launch per kind present (its own kernel and LDS
    // size, one workgroup per item)
    struct Seg {
        int kc;
        int64_t off, n;
        int lds_bytes;
    };
    std::vector<Seg> segs;
    bool work_valid = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_valid = false;
};

namespace fem {

static void drop_graph(fem_batch B) {
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->graph_valid = false;
}

// Element-major tiles of 128-lane workgroups for every mesh (built on first
// use, by the tuner or a configuration that asks for them).
static fem_status ensure_ema128(fem_batch B) {
    if (B->ema128 >= 0) return FEM_OK;
    bool ok = true;
    for (size_t i = 0; i < B->meshes.size(); ++i) {
        DofSet& ds = dofset(B->meshes[i], B->kinds[i]);
        if (fem_status st = build_ema(B->meshes[i], ds, 128, nullptr)) return st;
        ok = ok && ds.pat.ema[ema_index(128)].usable && !B->meshes[i]->nonconforming;
    }
    B->ema128 = ok ? 1 : 0;
    return FEM_OK;
}

static fem_status build_work(fem_batch B) {
    const bool ema = B->R == 0;
    if (ema && !B->ema_ok) return fail(FEM_EINVAL, "fem_batch: element-major tiles unavailable for this batch");
    if (ema && B->nt == 128) {
        if (fem_status st = ensure_ema128(B)) return st;
        if (B->ema128 != 1) return fail(FEM_EINVAL, "fem_batch: 128-lane element-major tiles unavailable for this batch");
    }
    // an earlier launch of this batch, on any stream, may still be reading the
    // work list and the mesh table that are rewritten below
    FEM_HIP(hipDeviceSynchronize());
    // invalid until the rebuild below completes: a failed rebuild leaves no
    // mix of old and new tiling behind (the next launch retries it)
    B->work_valid = false;
    drop_graph(B);
    std::vector<int2> work;
    std::vector<double> cost;
    std::vector<int> kcs;  // element kind of each item
    B->pmax = 0;
    B->lds_bytes = 0;
    for (size_t i = 0; i < B->meshes.size(); ++i) {
        fem_mesh m = B->meshes[i];
        DofSet& ds = dofset(m, B->kinds[i]);
        const Pattern::Ema& E = ds.pat.ema[ema_index(B->nt)];
        const int R = ema ? E.R : B->R;
        const int64_t nt = ema ? E.n_tiles : (ds.pat.n_rows + R - 1) / R;
        if (ema)
            B->lds_bytes = std::max(B->lds_bytes, ema_lds_bytes(kind_code(m->dim, B->kinds[i]), E.R, E.pmax,
                                                                E.max_slots));
        else
            B->pmax = std::max(B->pmax, ds.pat.tile_pmax[rows_index(R)]);
        const double per_row = ds.pat.n_rows ? (double)ds.pat.nnz / (double)ds.pat.n_rows : 0.0;
        const int kc = kind_code(m->dim, B->kinds[i]);
        for (int64_t t = 0; t < nt; ++t) {
            work.push_back(make_int2((int)i, (int)t));
            const int64_t rows = std::min<int64_t>(R, ds.pat.n_rows - t * R);
            cost.push_back(per_row * (double)rows * ds.nloc);
            kcs.push_back(kc);
        }
    }
    // Schedules 3-4 (element-major tiles): grouped by kind (stable), one
    // segment per kind. The decreasing-cost order of schedules 2 and 4 applies
    // within a segment (or to the whole list).
    const bool split = ema && B->schedule >= 3;
    const bool by_cost = B->schedule == 2 || B->schedule == 4;
    {
        std::vector<size_t> idx(work.size());
        for (size_t q = 0; q < idx.size(); ++q) idx[q] = q;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
            if (split && kcs[x] != kcs[y]) return kcs[x] < kcs[y];
            return by_cost && cost[x] > cost[y];
        });
        std::vector<int2> w2(work.size());
        std::vector<int> k2(work.size());
        for (size_t q = 0; q < idx.size(); ++q) {
            w2[q] = work[idx[q]];
            k2[q] = kcs[idx[q]];
        }
        work.swap(w2);
        kcs.swap(k2);
    }
    B->n_work = (int64_t)work.size();
    if (B->n_work > B->work_cap) {
        if (B->work_dev) FEM_HIP(hipFree(B->work_dev));
        B->work_dev = nullptr;
        FEM_HIP(hipMalloc((void**)&B->work_dev, std::max<int64_t>(1, B->n_work) * sizeof(int2)));
        B->work_cap = B->n_work;
    }
    if (B->n_work)
        FEM_HIP(hipMemcpy(B->work_dev, work.data(), B->n_work * sizeof(int2), hipMemcpyHostToDevice));
    // persistent grid: as many workgroups as can be resident
    int per_cu = 1;
    B->segs.clear();
    if (ema) {
        if (B->lds_bytes > lds_limit_bytes())
            return fail(FEM_EOVERFLOW, "fem_batch: a tile needs more LDS than the device has");
        if (split) {
            for (int64_t q = 0; q < B->n_work;) {
                int64_t q1 = q;
                int lds = 0;
                while (q1 < B->n_work && kcs[q1] == kcs[q]) {
                    const int i = work[q1].x;
                    const Pattern::Ema& E = dofset(B->meshes[i], B->kinds[i]).pat.ema[ema_index(B->nt)];
                    lds = std::max(lds, ema_lds_bytes(kcs[q], E.R, E.pmax, E.max_slots));
                    ++q1;
                }
                B->segs.push_back({kcs[q], q, q1 - q, lds});
                q = q1;
            }
        }
        per_cu = batch_ema_blocks_per_cu(B->lds_bytes, B->nt);
    } else {
        const int bytes = B->pmax * 16;
        if (bytes > lds_limit_bytes())
            return fail(FEM_EOVERFLOW, "fem_batch: a row tile needs more LDS than the device has");
        per_cu = batch_blocks_per_cu(B->R, bytes);
    }
    B->grid = (int)std::min<int64_t>((int64_t)cu_count() * per_cu, std::max<int64_t>(1, B->n_work));
    if (split) {  // workgroups launched: one per item
        B->grid = (int)std::min<int64_t>(B->n_work, 0x7FFFFFFF);
    }
    // rebuild the device table with the tiling of this configuration
    for (size_t i = 0; i < B->host_table.size(); ++i) {
        MeshDev& md = B->host_table[i];
        if (ema) fill_ema(dofset(B->meshes[i], B->kinds[i]), B->nt, &md);
        else md.n_tiles = (md.n_rows + B->R - 1) / B->R;
    }
    if (B->bound)
        FEM_HIP(hipMemcpy(B->table_dev, B->host_table.data(), B->host_table.size() * sizeof(MeshDev),
                          hipMemcpyHostToDevice));
    B->work_valid = true;
    return FEM_OK;
}

// What the tuned configuration depends on: per mesh its element count,
// dimension and kind, its row count and nonzeros (the row structure), and
// whether element-major tiles are usable for the whole batch, with their rows
// per tile and LDS size. Batches that differ in any of these get their own
// cache entries.
static std::string batch_signature(fem_batch B) {
    std::ostringstream os;
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t x) {
        h ^= x;
        h *= 1099511628211ull;
    };
    mix(B->ema_ok ? 1u : 0u);
    for (size_t i = 0; i < B->meshes.size(); ++i) {
        DofSet& ds = dofset(B->meshes[i], B->kinds[i]);
        const Pattern::Ema& em = ds.pat.ema[ema_index(256)];
        const uint64_t v[8] = {(uint64_t)B->meshes[i]->T, (uint64_t)B->meshes[i]->dim, (uint64_t)B->kinds[i],
                               (uint64_t)ds.pat.n_rows, (uint64_t)ds.pat.nnz, (uint64_t)em.R,
                               (uint64_t)em.pmax, (uint64_t)B->meshes[i]->nonconforming};
        for (uint64_t x : v) mix(x);
    }
    os << B->meshes.size() << "-" << std::hex << h;
    return os.str();
}

static std::string device_name() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string n = p.gcnArchName;
    for (char& c : n)
        if (c == '"' || c == '\n') c = '_';
    return n + "-cu" + std::to_string(p.multiProcessorCount);
}

}  // namespace fem

extern "C" {

fem_status fem_batch_create(const fem_mesh* meshes, const fem_kind* kinds, int n, fem_batch* out) {
    g_last_error.clear();
    if (!out) return fail(FEM_EINVAL, "fem_batch_create: out is NULL");
    *out = nullptr;
    if (n <= 0 || !meshes || !kinds) return fail(FEM_EINVAL, "fem_batch_create: empty batch");
    fem_batch B = new fem_batch_s();
    (void)hipGetDevice(&B->device);
    for (int i = 0; i < n; ++i) {
        if (!meshes[i] || (kinds[i] != FEM_NEDELEC && kinds[i] != FEM_RAVIART_THOMAS)) {
            delete B;
            return fail(FEM_EINVAL, "fem_batch_create: NULL mesh or bad kind");
        }
        if (!dofset(meshes[i], kinds[i]).pat.built) {
            delete B;
            return fail(FEM_ENOTREADY, "fem_batch_create: pattern not built for a mesh");
        }
        B->meshes.push_back(meshes[i]);
        B->kinds.push_back(kinds[i]);
    }
    // element-major tiles (256 lanes) for every mesh, if they fit
    B->ema_ok = true;
    for (int i = 0; i < n; ++i) {
        DofSet& ds = dofset(meshes[i], kinds[i]);
        if (fem_status st = build_ema(meshes[i], ds, 256, nullptr)) {
            delete B;
            return st;
        }
        B->ema_ok = B->ema_ok && ds.pat.ema[ema_index(256)].usable && !meshes[i]->nonconforming;
    }
    B->host_table.resize(n);
    hipError_t e = hipMalloc((void**)&B->table_dev, n * sizeof(MeshDev));
    if (e == hipSuccess) e = hipMalloc((void**)&B->counters, 2 * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(B->counters, 0, 2 * sizeof(unsigned));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        fem_status st = hip_fail(e, "fem_batch_create");
        fem_batch_destroy(B);
        return st;
    }
    B->R = B->ema_ok ? 0 : 128;
    B->schedule = B->ema_ok ? 4 : 1;
    *out = B;
    return FEM_OK;
}

fem_status fem_batch_bind(fem_batch B, const double* const* nodes, const double* const* a,
                          const double* const* b, double* const* K_vals, double* const* M_vals) {
    if (!B || !nodes) return fail(FEM_EINVAL, "fem_batch_bind: NULL argument");
    for (size_t i = 0; i < B->meshes.size(); ++i) {
        if (!nodes[i]) return fail(FEM_EINVAL, "fem_batch_bind: nodes[i] is NULL");
        MeshDev md;
        fem_status st = fill_meshdev(B->meshes[i], B->kinds[i], nodes[i], a ? a[i] : nullptr,
                                     b ? b[i] : nullptr, K_vals ? K_vals[i] : nullptr,
                                     M_vals ? M_vals[i] : nullptr, B->R > 0 ? B->R : 128, &md);
        if (st) return st;
        B->host_table[i] = md;
    }
    B->bound = true;
    drop_graph(B);
    return build_work(B);  // sets the tiling fields of the table and uploads it
}

fem_status fem_batch_set_config(fem_batch B, int R, int schedule, int threads) {
    if (!B) return fail(FEM_EINVAL, "fem_batch_set_config: batch is NULL");
    if ((R != 0 && R != 64 && R != 128 && R != 256) || schedule < 0 || schedule > (R == 0 ? 4 : 2))
        return fail(FEM_EINVAL, "fem_batch_set_config: rows_per_tile must be 0/64/128/256, schedule 0..4 for "
                                "element-major tiles and 0..2 for row tiles");
    if (R == 0 ? (threads != 128 && threads != 256) : (threads != 0 && threads != 256))
        return fail(FEM_EINVAL, "fem_batch_set_config: threads must be 128 or 256 for element-major tiles, "
                                "0 or 256 for row tiles");
    if (R == 0 && !B->ema_ok)
        return fail(FEM_EINVAL, "fem_batch_set_config: element-major tiles unavailable for this batch");
    B->R = R;
    B->schedule = schedule;
    B->nt = R == 0 ? threads : 256;
    return build_work(B);
}

fem_status fem_batch_config(fem_batch B, int* R, int* schedule, int* threads, int64_t* n_work, int* grid) {
    if (!B) return fail(FEM_EINVAL, "fem_batch_config: batch is NULL");
    if (R) *R = B->R;
    if (schedule) *schedule = B->schedule;
    if (threads) *threads = B->nt;
    if (n_work) *n_work = B->n_work;
    if (grid) *grid = B->grid;
    return FEM_OK;
}

fem_status fem_batch_assemble(fem_batch B, void* stream) {
    if (!B) return fail(FEM_EINVAL, "fem_batch_assemble: batch is NULL");
    if (!B->bound) return fail(FEM_ENOTREADY, "fem_batch_assemble: call fem_batch_bind first");
    if (!B->work_valid)
        if (fem_status st = build_work(B)) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (B->R == 0 && !B->segs.empty()) {
        for (const auto& g : B->segs)
            if (fem_status st = launch_batch_ema(B->table_dev, B->work_dev + g.off, g.n, B->schedule, 0,
                                                 g.lds_bytes, B->nt, g.kc, nullptr, s))
                return st;
        return FEM_OK;
    }
    if (B->R == 0)
        return launch_batch_ema(B->table_dev, B->work_dev, B->n_work, B->schedule, B->grid, B->lds_bytes, B->nt, -1,
                                B->counters, s);
    return launch_batch(B->table_dev, B->work_dev, B->n_work, B->R, B->schedule, B->grid, B->pmax,
                        B->counters, s);
}

fem_status fem_batch_tune(fem_batch B, const char* cache_path, void* stream) {
    if (!B) return fail(FEM_EINVAL, "fem_batch_tune: batch is NULL");
    if (!B->bound) return fail(FEM_ENOTREADY, "fem_batch_tune: call fem_batch_bind first");
    const std::string dev = device_name();
    const std::string sig = batch_signature(B);
    int R = 0, sc = 0, nt = 256;
    // A cached configuration that this batch cannot use (element-major tiles
    // unavailable, a tile too large for LDS) is ignored: the search below runs.
    if (cache_lookup(cache_path, dev, sig, &R, &sc, &nt) && (R != 0 || B->ema_ok) &&
        fem_batch_set_config(B, R, sc, R == 0 ? nt : 256) == FEM_OK)
        return FEM_OK;
    g_last_error.clear();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    struct Events {  // destroyed on every return path
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    FEM_HIP(hipEventCreate(&ev.e0));
    FEM_HIP(hipEventCreate(&ev.e1));
    const hipEvent_t e0 = ev.e0, e1 = ev.e1;
    double best = 1e30;
    int bestR = B->ema_ok ? 0 : 128, bestS = 1, bestT = 256;
    // tilings: element-major tiles of 256 and of 128 lanes (the elements per
    // tile and the wavefronts per workgroup; schedules 0-4), then row tiles of
    // 64/128/256 rows (schedules 0-2)
    const int Rs[5] = {0, 0, 64, 128, 256};
    const int Ts[5] = {256, 128, 256, 256, 256};
    for (int ri = B->ema_ok ? 0 : 2; ri < 5; ++ri) {
        for (int sched = 0; sched < (Rs[ri] == 0 ? 5 : 3); ++sched) {
            B->R = Rs[ri];
            B->nt = Ts[ri];
            B->schedule = sched;
            if (build_work(B) != FEM_OK) continue;  // e.g. tile too large for LDS
            bool ok = true;
            for (int w = 0; w < 2 && ok; ++w) ok = fem_batch_assemble(B, stream) == FEM_OK;
            if (!ok) continue;
            FEM_HIP(hipEventRecord(e0, s));
            const int reps = 5;
            for (int w = 0; w < reps && ok; ++w) ok = fem_batch_assemble(B, stream) == FEM_OK;
            FEM_HIP(hipEventRecord(e1, s));
            FEM_HIP(hipEventSynchronize(e1));
            if (!ok) continue;
            float ms = 0.f;
            FEM_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double t = ms / reps;
            if (t < best) {
                best = t;
                bestR = Rs[ri];
                bestS = sched;
                bestT = Ts[ri];
            }
        }
    }
    g_last_error.clear();
    fem_status st = fem_batch_set_config(B, bestR, bestS, bestT);
    if (st == FEM_OK) cache_store(cache_path, dev, sig, bestR, bestS, bestT, best);
    return st;
}

fem_status fem_batch_graph_launch(fem_batch B, void* stream) {
    if (!B) return fail(FEM_EINVAL, "fem_batch_graph_launch: batch is NULL");
    if (!B->bound) return fail(FEM_ENOTREADY, "fem_batch_graph_launch: call fem_batch_bind first");
    if (!B->work_valid)
        if (fem_status st = build_work(B)) return st;
    if (!B->graph_valid) {
        drop_graph(B);
        // One plain launch first, so that the kernel attributes are set outside
        // the capture. It runs on the capture stream after the work already
        // queued on `stream` (which may still read K and M, or run an earlier
        // launch of this batch that shares its work-queue counters), and has
        // finished before the replay below is queued.
        hipEvent_t ev = nullptr;
        FEM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        hipError_t e0 = hipEventRecord(ev, reinterpret_cast<hipStream_t>(stream));
        if (e0 == hipSuccess) e0 = hipStreamWaitEvent(B->cap_stream, ev, 0);
        fem_status st0 = e0 == hipSuccess ? fem_batch_assemble(B, B->cap_stream) : hip_fail(e0, "fem_batch_graph_launch");
        if (st0 == FEM_OK) {
            e0 = hipStreamSynchronize(B->cap_stream);
            if (e0 != hipSuccess) st0 = hip_fail(e0, "fem_batch_graph_launch");
        }
        (void)hipEventDestroy(ev);
        if (st0 != FEM_OK) return st0;
        FEM_HIP(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeRelaxed));
        fem_status st = fem_batch_assemble(B, B->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
        if (st != FEM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        B->graph = g;
        e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(B);
            return hip_fail(e, "hipGraphInstantiate");
        }
        B->graph_valid = true;
    }
    FEM_HIP(hipGraphLaunch(B->exec, reinterpret_cast<hipStream_t>(stream)));
    return FEM_OK;
}

void fem_batch_destroy(fem_batch B) {
    if (!B) return;
    (void)hipDeviceSynchronize();
    drop_graph(B);
    if (B->table_dev) (void)hipFree(B->table_dev);
    if (B->work_dev) (void)hipFree(B->work_dev);
    if (B->counters) (void)hipFree(B->counters);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    delete B;
}

}  // extern "C"
