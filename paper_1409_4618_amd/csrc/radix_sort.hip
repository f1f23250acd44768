// Device primitives: exclusive prefix sum and a stable LSD radix sort of
// (u64 key, u32 value) pairs, written for 64-wide CDNA wavefronts.
//
// Radix sort: 8-bit digits, one pass per digit over the key's significant bits.
// Each pass = per-tile digit histograms (digit-major table) -> exclusive scan of
// the table -> stable scatter. Inside a tile the scatter ranks keys with equal
// digits by wave ballots (8 ballots give each lane the mask of lanes holding its
// digit) and a per-wave prefix over LDS counters, so the order of equal keys
// is the input order: the sort is stable and deterministic.
#include "fem_internal.h"

namespace fem {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;
constexpr int SORT_WAVES = SORT_THREADS / 64;

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

int bit_length(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// ---------------------------------------------------------------- scan
// Block-level exclusive scan of a tile; writes the tile total to block_sums.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(uint32_t* data, int64_t n,
                                                             uint32_t* block_sums) {
    __shared__ uint32_t s_part[SCAN_THREADS];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < n ? data[idx] : 0u;
        sum += v[i];
    }
    s_part[threadIdx.x] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan over thread partials
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        uint32_t t = threadIdx.x >= off ? s_part[threadIdx.x - off] : 0u;
        __syncthreads();
        s_part[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = s_part[threadIdx.x] - sum;  // exclusive prefix of this thread
    if (threadIdx.x == SCAN_THREADS - 1 && block_sums) block_sums[blockIdx.x] = s_part[threadIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t idx = base + i;
        if (idx < n) data[idx] = run;
        run += v[i];
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(uint32_t* data, int64_t n,
                                                           const uint32_t* block_offsets) {
    const uint32_t off = block_offsets[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_THREADS) {
        const int64_t idx = base + i;
        if (idx < n) data[idx] += off;
    }
}

hipError_t scan_exclusive_u32(uint32_t* data, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(SCAN_THREADS), 0, s, data, n, nullptr);
        return hipGetLastError();
    }
    uint32_t* sums = nullptr;
    hipError_t e = hipMallocAsync((void**)&sums, nb * sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, data, n, sums);
    e = hipGetLastError();
    if (e == hipSuccess) e = scan_exclusive_u32(sums, nb, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, data, n, sums);
        e = hipGetLastError();
    }
    hipError_t e2 = hipFreeAsync(sums, s);
    return e != hipSuccess ? e : e2;
}

// ---------------------------------------------------------------- radix sort
__global__ __launch_bounds__(SORT_THREADS) void k_digit_hist(const uint64_t* keys, int64_t n,
                                                             int shift, uint32_t* table,
                                                             int64_t n_tiles) {
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
#pragma unroll 4
    for (int i = 0; i < SORT_ITEMS; ++i) {
        const int64_t idx = base + (int64_t)i * SORT_THREADS + threadIdx.x;
        if (idx < n) atomicAdd(&hist[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    table[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(SORT_THREADS) void k_digit_scatter(
    const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* keys_out, uint32_t* vals_out,
    int64_t n, int shift, const uint32_t* table, int64_t n_tiles) {
    __shared__ uint32_t digit_base[256];
    __shared__ uint32_t wave_cnt[SORT_WAVES][256];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    digit_base[tid] = table[(int64_t)tid * n_tiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
#pragma unroll
        for (int w = 0; w < SORT_WAVES; ++w) wave_cnt[w][tid] = 0;
        __syncthreads();
        const int64_t idx = base + (int64_t)r * SORT_THREADS + tid;
        const bool valid = idx < n;
        uint64_t key = 0;
        uint32_t val = 0;
        if (valid) {
            key = keys_in[idx];
            val = vals_in[idx];
        }
        const uint32_t digit = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bal = __ballot((digit >> bit) & 1u);
            peers &= ((digit >> bit) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wave_cnt[wave][digit] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t run = digit_base[tid];
#pragma unroll
            for (int w = 0; w < SORT_WAVES; ++w) {
                const uint32_t c = wave_cnt[w][tid];
                wave_cnt[w][tid] = run;
                run += c;
            }
            digit_base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = wave_cnt[wave][digit] + rank;
            keys_out[dst] = key;
            vals_out[dst] = val;
        }
        __syncthreads();
    }
}

__global__ void k_copy_pairs(const uint64_t* ks, const uint32_t* vs, uint64_t* kd, uint32_t* vd,
                             int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    kd[i] = ks[i];
    vd[i] = vs[i];
}

hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp,
                            uint32_t* vals_tmp, int64_t n, int bits, hipStream_t s) {
    if (n <= 1 || bits <= 0) return hipSuccess;
    if (n >= (int64_t(1) << 32)) return hipErrorInvalidValue;
    const int64_t n_tiles = (n + SORT_TILE - 1) / SORT_TILE;
    uint32_t* table = nullptr;
    hipError_t e = hipMallocAsync((void**)&table, (size_t)n_tiles * 256 * sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
    uint64_t* kin = keys;
    uint32_t* vin = vals;
    uint64_t* kout = keys_tmp;
    uint32_t* vout = vals_tmp;
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes && e == hipSuccess; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)n_tiles), dim3(SORT_THREADS), 0, s, kin, n,
                           shift, table, n_tiles);
        e = hipGetLastError();
        if (e == hipSuccess) e = scan_exclusive_u32(table, n_tiles * 256, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)n_tiles), dim3(SORT_THREADS), 0, s,
                               kin, vin, kout, vout, n, shift, table, n_tiles);
            e = hipGetLastError();
        }
        uint64_t* tk = kin;
        kin = kout;
        kout = tk;
        uint32_t* tv = vin;
        vin = vout;
        vout = tv;
    }
    if (e == hipSuccess && kin != keys) {
        // odd number of passes: move the result back with a kernel on the same stream
        hipLaunchKernelGGL(k_copy_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, kin, vin,
                           keys, vals, n);
        e = hipGetLastError();
    }
    hipError_t e2 = hipFreeAsync(table, s);
    return e != hipSuccess ? e : e2;
}

}  // namespace fem
