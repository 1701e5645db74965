// Device primitives: scan, stable radix sort, fills and gathers.
#include "prim.h"

namespace hspmm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Exclusive scan of 256 per-thread values inside a workgroup; returns the
// prefix for this thread, *total receives the workgroup sum.
__device__ int32_t block_exclusive_scan(int32_t v, int32_t* total) {
    __shared__ int32_t s_wave[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
        int32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[w] = x;
    __syncthreads();
    int32_t base = 0, all = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
        if (i < w) base += s_wave[i];
        all += s_wave[i];
    }
    __syncthreads();
    *total = all;
    return base + x - v;
}

__global__ void k_scan_reduce(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ part) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    int32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single workgroup: exclusive scan of the tile sums, in chunks of 256
__global__ void k_scan_partials(int32_t* part, int64_t nparts, int32_t* total) {
    int32_t carry = 0;
    for (int64_t c = 0; c < nparts; c += kScanThreads) {
        const int64_t i = c + threadIdx.x;
        int32_t v = i < nparts ? part[i] : 0;
        int32_t tot;
        int32_t ex = block_exclusive_scan(v, &tot);
        if (i < nparts) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_scan_down(const int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t n,
                            const int32_t* __restrict__ part) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    int32_t tot;
    int32_t run = block_exclusive_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// ---------------------------------------------------------------------------
// radix sort: 8-bit digits, tiles of 2048 items
// ---------------------------------------------------------------------------
constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 8;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;
constexpr int kRadixBins = 256;

__global__ void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n, int shift, uint32_t mask,
                             int32_t* __restrict__ hist, int64_t ntiles) {
    __shared__ int32_t s_h[kRadixBins];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t i = base + r * kRadixThreads + threadIdx.x;
        if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & mask], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = s_h[threadIdx.x];
}

// Stable scatter: items of a tile keep their order inside each digit.
__global__ void k_radix_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                uint32_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t n,
                                int shift, int nbits, const int32_t* __restrict__ offs, int64_t ntiles) {
    __shared__ int32_t s_run[kRadixBins];
    __shared__ int32_t s_w[kRadixThreads / 64][kRadixBins];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t mask = (1u << nbits) - 1u;
    s_run[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kRadixRounds; ++r) {
        for (int j = tid; j < (kRadixThreads / 64) * kRadixBins; j += kRadixThreads)
            (&s_w[0][0])[j] = 0;
        __syncthreads();
        const int64_t i = base + r * kRadixThreads + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const int32_t val = valid ? vin[i] : 0;
        const uint32_t d = (key >> shift) & mask;
        uint64_t match = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const int rank = __popcll(match & lt);
        if (valid && rank == 0) s_w[w][d] = __popcll(match);
        __syncthreads();
        if (valid) {
            int32_t off = s_run[d] + rank;
            for (int w2 = 0; w2 < w; ++w2) off += s_w[w2][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        int32_t add = 0;
        for (int w2 = 0; w2 < kRadixThreads / 64; ++w2) add += s_w[w2][tid];
        s_run[tid] += add;
        __syncthreads();
    }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_iota_i32(int32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}
__global__ void k_gather_u32(uint32_t* dst, const uint32_t* src, const int32_t* idx, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}
__global__ void k_gather_key_shift(uint32_t* dst, const int32_t* src, const int32_t* idx, int shift,
                                   int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = ((uint32_t)src[idx[i]]) >> shift;
}

inline unsigned grid_for(int64_t n, int threads = 256) {
    int64_t g = ceil_div(n, threads);
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

int scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total, Allocator& al,
                       hipStream_t s) {
    if (n <= 0) {
        if (total) HIP_TRY(hipMemsetAsync(total, 0, sizeof(int32_t), s));
        return HSPMM_OK;
    }
    const int64_t tiles = ceil_div(n, kScanTile);
    DevBuf part;
    HSPMM_TRY(al.alloc(part, tiles * sizeof(int32_t)));
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, n,
                       part.as<int32_t>());
    HIP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s, part.as<int32_t>(), tiles,
                       total);
    HIP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n,
                       part.as<int32_t>());
    HIP_LAUNCH_CHECK();
    // `part` is released when this returns (after the stream's work on it)
    HSPMM_TRY(sync_for_release(al, s));
    al.free(part);
    return HSPMM_OK;
}

int radix_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_tmp, int32_t* vals_tmp, int64_t n,
                     int nbits, Allocator& al, hipStream_t s) {
    if (n <= 1 || nbits <= 0) return HSPMM_OK;
    const int64_t ntiles = ceil_div(n, kRadixTile);
    if (ntiles * kRadixBins >= (int64_t(1) << 31)) return fail(HSPMM_ERR_OVERFLOW, "radix sort too large");
    DevBuf hist;
    HSPMM_TRY(al.alloc(hist, (size_t)ntiles * kRadixBins * sizeof(int32_t)));
    uint32_t *ka = keys, *kb = keys_tmp;
    int32_t *va = vals, *vb = vals_tmp;
    int passes = 0;
    for (int shift = 0; shift < nbits; shift += 8, ++passes) {
        const int nb = (nbits - shift) < 8 ? (nbits - shift) : 8;
        const uint32_t mask = (1u << nb) - 1u;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kRadixThreads), 0, s, ka, n, shift,
                           mask, hist.as<int32_t>(), ntiles);
        HIP_LAUNCH_CHECK();
        HSPMM_TRY(scan_exclusive_i32(hist.as<int32_t>(), hist.as<int32_t>(), ntiles * kRadixBins, nullptr,
                                     al, s));
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kRadixThreads), 0, s, ka, va, kb,
                           vb, n, shift, nb, hist.as<int32_t>(), ntiles);
        HIP_LAUNCH_CHECK();
        uint32_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        HIP_TRY(hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    HSPMM_TRY(sync_for_release(al, s));
    al.free(hist);
    return HSPMM_OK;
}

int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return HSPMM_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}
int iota_i32(int32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return HSPMM_OK;
    hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}
int gather_u32(uint32_t* dst, const uint32_t* src, const int32_t* idx, int64_t n, hipStream_t s) {
    if (n <= 0) return HSPMM_OK;
    hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(n)), dim3(256), 0, s, dst, src, idx, n);
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}
int gather_key_shift(uint32_t* dst, const int32_t* src, const int32_t* idx, int shift, int64_t n,
                     hipStream_t s) {
    if (n <= 0) return HSPMM_OK;
    hipLaunchKernelGGL(k_gather_key_shift, dim3(grid_for(n)), dim3(256), 0, s, dst, src, idx, shift, n);
    HIP_LAUNCH_CHECK();
    return HSPMM_OK;
}

}  // namespace hspmm
