// Spatial order of a scene's points (input P of Alg. 1): a stable radix sort of their 30-bit
// Morton codes on a 1024^3 grid over the bounding box.  Consecutive points of the sorted
// arrays are then close in space at every scale, so each 64-point chunk covers a compact
// patch: its screen rectangles, and the tiles the raster visits for it, stay small.
//
// The sort is least-significant-digit first over 8-bit digits (four passes for 30 bits).  A
// pass splits the keys into tiles of kSortTile, one workgroup each: a histogram pass counts
// each tile's digits into a digit-major table, an exclusive scan of that table gives every
// (digit, tile) its first output position, and a scatter pass places each key at that position
// plus its rank among the equal digits before it in the tile.  The rank comes from 64-lane
// ballots (the lanes holding the same digit) and per-wavefront digit counts in LDS, taken in
// index order, so each pass is stable and the result is the unique stable order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "pe_device.h"

namespace pe {

__device__ inline uint32_t spread10(uint32_t v) {  // 10 bits -> every third bit of 30
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton_key(const float4* __restrict__ pa, uint64_t n, float lx, float ly,
                             float lz, float inv, uint32_t* __restrict__ key,
                             uint32_t* __restrict__ idx) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float4 a = pa[i];
        const int cx = min(max((int)((a.x - lx) * inv), 0), 1023);
        const int cy = min(max((int)((a.y - ly) * inv), 0), 1023);
        const int cz = min(max((int)((a.z - lz) * inv), 0), 1023);
        key[i] = spread10(cx) | (spread10(cy) << 1) | (spread10(cz) << 2);
        idx[i] = (uint32_t)i;
    }
}

// Sorted position i takes point idx[i]; its original index travels in pb_s.w.
__global__ void k_morton_gather(const float4* __restrict__ pa, const float4* __restrict__ pb,
                                uint64_t n, const uint32_t* __restrict__ idx,
                                float4* __restrict__ pa_s, float4* __restrict__ pb_s) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t j = idx[i];
        const float4 b = pb[j];
        pa_s[i] = pa[j];
        pb_s[i] = make_float4(b.x, b.y, b.z, __uint_as_float(j));
    }
}

constexpr int kSortThreads = 256;  // four wavefronts
constexpr int kSortRounds = 16;    // items per thread per tile
constexpr uint32_t kSortTile = kSortThreads * kSortRounds;
constexpr int kSortPasses = 4;     // 8-bit digits over the 30-bit code

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* __restrict__ key,
                                                             uint32_t n, int shift,
                                                             uint32_t n_tiles,
                                                             uint32_t* __restrict__ count) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; r++) {
        const uint32_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    count[threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* __restrict__ key_in, const uint32_t* __restrict__ val_in, uint32_t n,
    int shift, uint32_t n_tiles, const uint32_t* __restrict__ offset,
    uint32_t* __restrict__ key_out, uint32_t* __restrict__ val_out) {
    __shared__ uint32_t next[256];     // next output position of each digit in this tile
    __shared__ uint32_t wcnt[4][256];  // this round's count of each digit per wavefront
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    next[threadIdx.x] = offset[threadIdx.x * n_tiles + blockIdx.x];
    for (int v = 0; v < 4; v++) wcnt[v][threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortTile;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortRounds; r++) {
        const uint32_t i = base + r * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        const uint32_t k = valid ? key_in[i] : 0u, v = valid ? val_in[i] : 0u;
        const uint32_t dg = (k >> shift) & 0xFFu;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            const uint64_t bal = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) wcnt[w][dg] = (uint32_t)__popcll(peers);
        __syncthreads();
        uint32_t pos = 0;
        if (valid) {
            pos = next[dg] + rank;
            for (int u = 0; u < w; u++) pos += wcnt[u][dg];
        }
        __syncthreads();
        next[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                             wcnt[3][threadIdx.x];
        for (int u = 0; u < 4; u++) wcnt[u][threadIdx.x] = 0;
        if (valid) {
            key_out[pos] = k;
            val_out[pos] = v;
        }
        __syncthreads();
    }
}

static uint32_t sort_tiles(uint64_t n) { return (uint32_t)((n + kSortTile - 1) / kSortTile); }

size_t morton_sort_temp_bytes(uint64_t n) {
    const uint32_t m = 256u * std::max(1u, sort_tiles(n));
    return 4ull * (2ull * m + 1 + scan_wide_scratch(m));
}

hipError_t launch_morton_sort(const float4* pa, const float4* pb, uint64_t n, float lo_x,
                              float lo_y, float lo_z, float inv_cell, uint32_t* keys,
                              void* temp, size_t temp_bytes, float4* pa_s, float4* pb_s,
                              hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (n > 0xFFFFFFFFull - kSortTile || temp_bytes < morton_sort_temp_bytes(n))
        return hipErrorInvalidValue;
    // codes start in the second quarter so that an even number of passes ends there too
    uint32_t* kb[2] = {keys + n, keys};
    uint32_t* vb[2] = {keys + 3 * n, keys + 2 * n};
    const uint32_t tiles = sort_tiles(n), m = 256u * tiles;
    uint32_t* count = (uint32_t*)temp;
    uint32_t* offset = count + m;
    uint32_t* scratch = offset + m + 1;
    const int b = (int)std::min<uint64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_morton_key, dim3(b), dim3(256), 0, st, pa, n, lo_x, lo_y, lo_z, inv_cell,
                       kb[0], vb[0]);
    for (int p = 0; p < kSortPasses; p++) {
        const int in = p & 1;
        hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(kSortThreads), 0, st, kb[in],
                           (uint32_t)n, 8 * p, tiles, count);
        launch_scan_wide(count, offset, m, nullptr, 1, offset + m, scratch, st);
        hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(kSortThreads), 0, st, kb[in],
                           vb[in], (uint32_t)n, 8 * p, tiles, offset, kb[in ^ 1], vb[in ^ 1]);
    }
    hipLaunchKernelGGL(k_morton_gather, dim3(b), dim3(256), 0, st, pa, pb, n,
                       (const uint32_t*)vb[0], pa_s, pb_s);
    return hipGetLastError();
}

}  // namespace pe
