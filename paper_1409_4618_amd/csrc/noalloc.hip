// Allocation-free value of the quadratic form L = u^T (K(a) + M(b)) u, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// fem_quadratic_value keeps its workgroup partials in the mesh handle and
// allocates them on its first call. This variant keeps them in `scratch`, a
// file-scope device array of fixed size that the code object brings with it
// (each GPU the library runs on holds its own copy until the process ends).
// The kernels are those of fem_quadratic_value.
//
// On the host, `scratch` names a host-side stand-in, not the device array: its
// device address is looked up once per device with hipGetSymbolAddress and
// only that address is handed to kernels.
#include <mutex>

#include "fem_internal.h"

namespace fem {

// Partials of one call: one double per workgroup of BWD_BLOCK elements, so the
// array serves meshes of up to NOALLOC_PARTIALS * BWD_BLOCK = 2^27 elements.
constexpr int64_t NOALLOC_PARTIALS = int64_t(1) << 19;  // 4 MiB
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) double scratch[NOALLOC_PARTIALS];

static std::mutex g_scratch_mu;
static double* g_scratch_dev[NOALLOC_MAX_DEVICES];  // device address of `scratch`, per device

// Device address of `scratch` on device `dev` (the current device), found on
// the first call for that device.
static fem_status scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(FEM_EINVAL, "fem_quadratic_value_noalloc: device ordinal beyond the supported range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FEM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return FEM_OK;
}

}  // namespace fem

using namespace fem;

extern "C" {

fem_status fem_quadratic_value_noalloc(fem_mesh m, fem_kind kind, const double* nodes,
                                       const double* a, const double* b, const double* u,
                                       double* L, void* stream) {
    if (!m) return fail(FEM_EINVAL, "fem_quadratic_value_noalloc: mesh is NULL");
    if (kind != FEM_NEDELEC && kind != FEM_RAVIART_THOMAS)
        return fail(FEM_EINVAL, "fem_quadratic_value_noalloc: bad kind");
    if (!nodes || !u || !L) return fail(FEM_EINVAL, "fem_quadratic_value_noalloc: nodes, u or L is NULL");
    const int64_t np = quadratic_value_partials(m->T);
    if (np > NOALLOC_PARTIALS)
        return fail(FEM_EOVERFLOW, "fem_quadratic_value_noalloc: the mesh has more than 2^27 elements, "
                                   "beyond its fixed scratch (use fem_quadratic_value)");
    DofSet& ds = (m->dim == 3 && kind == FEM_RAVIART_THOMAS) ? m->faces : m->edges;
    if (!ds.pat.built) return fail(FEM_ENOTREADY, "pattern not built: call fem_pattern first");
    int dev = -1;
    FEM_HIP(hipGetDevice(&dev));
    if (dev != m->device)
        return fail(FEM_EINVAL, "fem_quadratic_value_noalloc: the mesh lives on device " +
                                    std::to_string(m->device) + ", not on the current device " +
                                    std::to_string(dev));
    double* partials = nullptr;
    if (fem_status st = scratch_address(dev, &partials)) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->last_stream = s;
    // every partial the sum reads is written by this call's first kernel, so
    // nothing needs clearing
    return launch_quadratic_value(m, ds, kind, nodes, a, b, u, L, partials, s);
}

}  // extern "C"
