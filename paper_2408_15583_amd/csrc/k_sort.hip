// Spatial order of a scene's points (input P of Alg. 1): a stable radix sort of their 30-bit
// Morton codes on a 1024^3 grid over the bounding box.  Consecutive points of the sorted
// arrays are then close in space at every scale, so each 64-point chunk covers a compact
// patch: its screen rectangles, and the tiles the raster visits for it, stay small.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <rocprim/device/device_radix_sort.hpp>

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

size_t morton_sort_temp_bytes(uint64_t n) {
    size_t bytes = 0;
    const hipError_t e = rocprim::radix_sort_pairs(
        nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr, (const uint32_t*)nullptr,
        (uint32_t*)nullptr, (size_t)n, 0u, 30u);
    return e == hipSuccess ? bytes : 0;
}

hipError_t launch_morton_sort(const float4* pa, const float4* pb, uint64_t n, float lo_x,
                              float lo_y, float lo_z, float inv_cell, uint32_t* keys,
                              void* temp, size_t temp_bytes, float4* pa_s, float4* pb_s,
                              hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint32_t *key_in = keys, *key_out = keys + n, *idx_in = keys + 2 * n, *idx_out = keys + 3 * n;
    const int b = (int)std::min<uint64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_morton_key, dim3(b), dim3(256), 0, st, pa, n, lo_x, lo_y, lo_z, inv_cell,
                       key_in, idx_in);
    size_t bytes = temp_bytes;
    const hipError_t e = rocprim::radix_sort_pairs(temp, bytes, (const uint32_t*)key_in, key_out,
                                                   (const uint32_t*)idx_in, idx_out, (size_t)n,
                                                   0u, 30u, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_morton_gather, dim3(b), dim3(256), 0, st, pa, pb, n,
                       (const uint32_t*)idx_out, pa_s, pb_s);
    return hipGetLastError();
}

}  // namespace pe
