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

// Exclusive scan by one workgroup of 1024 threads; each round covers 16 Ki items (16 per
// thread, contiguous), a wave-level shuffle scan and a 16-entry scan of the wave totals.
constexpr int kScanT = 1024;
constexpr int kScanItems = 16;

__global__ __launch_bounds__(kScanT) void k_scan(const uint32_t* __restrict__ in,
                                                 uint32_t* __restrict__ out, uint32_t n_static,
                                                 const uint32_t* __restrict__ n_dev,
                                                 uint32_t div, uint32_t* __restrict__ total) {
    __shared__ uint32_t wsum[kScanT / 64];
    __shared__ uint32_t s_carry;
    const uint32_t n = n_dev ? (uint32_t)(((uint64_t)*n_dev + div - 1) / div) : n_static;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t carry = 0;
    for (uint64_t base = 0; base < n; base += (uint64_t)kScanT * kScanItems) {
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
        }
        __syncthreads();
        uint32_t pre = carry + wsum[w] + (x - s);
#pragma unroll
        for (int j = 0; j < kScanItems; j++) {
            const uint64_t i = i0 + j;
            if (i < n) out[i] = pre;
            pre += v[j];
        }
        if (t == kScanT - 1) s_carry = pre;
        __syncthreads();
        carry = s_carry;
        __syncthreads();
    }
    if (t == 0 && total) *total = carry;
}

void launch_scan(const uint32_t* in, uint32_t* out, uint32_t n_static, const uint32_t* n_dev,
                 uint32_t div, uint32_t* total, hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanT), 0, st, in, out, n_static, n_dev,
                       div ? div : 1u, total);
}

}  // namespace pe
