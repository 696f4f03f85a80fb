// Generic device utilities: fills and a single-workgroup exclusive scan used for every
// order-preserving compaction (tile lists, live-ray lists, PO tiles).
#include "pe_device.h"

namespace pe {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t v, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

static inline int fill_blocks(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b ? b : 1) : 4096);
}

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, st, p, v, n);
}

void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_blocks(n)), dim3(256), 0, st, p, v, n);
}

// Exclusive scans.  A workgroup of 1024 threads scans 16 Ki items per round (16 per thread,
// contiguous: a wave-level shuffle scan and a 16-entry scan of the wave totals).  launch_scan
// runs one workgroup over all items; launch_scan_wide gives each 16 Ki tile a workgroup that
// scans it and stores its total, then adds to each tile the sum of the earlier tiles' totals
// (integer sums: both give the same result).
constexpr int kScanT = 1024;
constexpr int kScanItems = 16;
constexpr uint32_t kScanTile = (uint32_t)kScanT * kScanItems;

__device__ inline uint32_t scan_count(uint32_t n_static, const uint32_t* n_dev, uint32_t div) {
    if (!n_dev) return n_static;
    const uint32_t n = (uint32_t)(((uint64_t)*n_dev + div - 1) / div);
    return n < n_static ? n : n_static;
}

// Exclusive scan of one tile [base, base + kScanTile) of in into out, offset by carry; returns
// the tile's total (to every thread).
__device__ inline uint32_t scan_tile(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                     uint64_t base, uint32_t n, uint32_t carry,
                                     uint32_t* wsum) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    const uint64_t i0 = base + (uint64_t)t * kScanItems;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        const uint64_t i = i0 + j;
        v[j] = i < n ? in[i] : 0u;
        s += v[j];
    }
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
        uint32_t a = lane < kScanT / 64 ? wsum[lane] : 0u;
        uint32_t b = a;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            uint32_t y = __shfl_up(b, o);
            if (lane >= o) b += y;
        }
        if (lane < kScanT / 64) wsum[lane] = b - a;
        if (lane == kScanT / 64 - 1) wsum[kScanT / 64] = b;
    }
    __syncthreads();
    uint32_t pre = carry + wsum[w] + (x - s);
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        const uint64_t i = i0 + j;
        if (i < n) out[i] = pre;
        pre += v[j];
    }
    const uint32_t tot = wsum[kScanT / 64];
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(kScanT) void k_scan(const uint32_t* __restrict__ in,
                                                 uint32_t* __restrict__ out, uint32_t n_static,
                                                 const uint32_t* __restrict__ n_dev,
                                                 uint32_t div, uint32_t* __restrict__ total) {
    __shared__ uint32_t wsum[kScanT / 64 + 1];
    const uint32_t n = n_dev ? (uint32_t)(((uint64_t)*n_dev + div - 1) / div) : n_static;
    uint32_t carry = 0;
    for (uint64_t base = 0; base < n; base += kScanTile)
        carry += scan_tile(in, out, base, n, carry, wsum);
    if (threadIdx.x == 0 && total) *total = carry;
}

void launch_scan(const uint32_t* in, uint32_t* out, uint32_t n_static, const uint32_t* n_dev,
                 uint32_t div, uint32_t* total, hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanT), 0, st, in, out, n_static, n_dev,
                       div ? div : 1u, total);
}

__global__ __launch_bounds__(kScanT) void k_scan_local(const uint32_t* __restrict__ in,
                                                       uint32_t* __restrict__ out,
                                                       uint32_t n_max,
                                                       const uint32_t* __restrict__ n_dev,
                                                       uint32_t div,
                                                       uint32_t* __restrict__ tile_total) {
    __shared__ uint32_t wsum[kScanT / 64 + 1];
    const uint32_t n = scan_count(n_max, n_dev, div);
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    if (base >= n) return;
    const uint32_t tot = scan_tile(in, out, base, n, 0u, wsum);
    if (threadIdx.x == 0) tile_total[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanT) void k_scan_carry(uint32_t* __restrict__ out, uint32_t n_max,
                                                       const uint32_t* __restrict__ n_dev,
                                                       uint32_t div,
                                                       const uint32_t* __restrict__ tile_total,
                                                       uint32_t* __restrict__ total) {
    __shared__ uint32_t part[kScanT / 64];
    __shared__ uint32_t s_carry;
    const uint32_t n = scan_count(n_max, n_dev, div);
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    if (n == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && total) *total = 0u;
        return;
    }
    if (base >= n) return;
    uint32_t c = 0;
    for (uint32_t j = threadIdx.x; j < blockIdx.x; j += kScanT) c += tile_total[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int q = 0; q < kScanT / 64; q++) a += part[q];
        s_carry = a;
    }
    __syncthreads();
    const uint32_t carry = s_carry;
    const uint64_t end = base + kScanTile < n ? base + kScanTile : (uint64_t)n;
    if (carry != 0)
        for (uint64_t i = base + threadIdx.x; i < end; i += kScanT) out[i] += carry;
    if (end == n && threadIdx.x == 0 && total) *total = carry + tile_total[blockIdx.x];
}

uint32_t scan_wide_scratch(uint32_t n_max) {
    return (uint32_t)(((uint64_t)n_max + kScanTile - 1) / kScanTile) + 1;
}

void launch_scan_wide(const uint32_t* in, uint32_t* out, uint32_t n_max, const uint32_t* n_dev,
                      uint32_t div, uint32_t* total, uint32_t* scratch, hipStream_t st) {
    div = div ? div : 1u;
    const uint32_t blocks = (uint32_t)(((uint64_t)n_max + kScanTile - 1) / kScanTile);
    if (blocks <= 1) {
        launch_scan(in, out, n_max, n_dev, div, total, st);
        return;
    }
    hipLaunchKernelGGL(k_scan_local, dim3(blocks), dim3(kScanT), 0, st, in, out, n_max, n_dev,
                       div, scratch);
    hipLaunchKernelGGL(k_scan_carry, dim3(blocks), dim3(kScanT), 0, st, out, n_max, n_dev, div,
                       (const uint32_t*)scratch, total);
}

}  // namespace pe
