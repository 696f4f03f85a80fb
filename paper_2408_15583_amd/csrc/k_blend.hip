// Overlap refinement and normal blending of ray-splat hits (Sec. III-B, Eq. (23), Fig. 4(a)).
//
// After a ray's nearest hit P' is known, every splat whose disk the ray crosses within
// distance r beyond P' is a candidate; the hit moves to the candidate whose crossing lies
// relatively closest to its centre (smallest |p_i - c_i| / R_i; ties: lowest index), and the
// record's normal becomes the Eq. (23) blend of the candidates' normals (each turned against
// the ray) with weights 1 - |p_i - c_i| / R_i.  Candidates come from a uniform grid over the
// splat centres whose cell edge is at least r + r_max, so the cells overlapping the cube of
// half-side r + r_max about P' (at most 2 per axis) hold every candidate.  The weighted
// normal sums are 64-bit fixed point, so the result does not depend on the visiting order.
#include <float.h>

#include "pe_device.h"

namespace pe {

namespace {

struct v3f {
    float x, y, z;
};
__device__ inline v3f mkv(float x, float y, float z) { return {x, y, z}; }
__device__ inline v3f add(v3f a, v3f b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline v3f sub(v3f a, v3f b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline v3f scl(v3f a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline float vdot(v3f a, v3f b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

__device__ inline int blend_cell(float x, float R, float h, int G) {
    const int q = (int)floorf((x + R) / h);
    return min(max(q, 0), G - 1);
}

}  // namespace

__global__ void k_blend_count(const float4* __restrict__ pa, uint64_t n, float R, float h, int G,
                              uint32_t* __restrict__ cell_of, uint32_t* __restrict__ counts) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float4 a = pa[i];
        const uint32_t c = ((uint32_t)blend_cell(a.z, R, h, G) * G + blend_cell(a.y, R, h, G)) * G +
                           blend_cell(a.x, R, h, G);
        cell_of[i] = c;
        atomicAdd(&counts[c], 1u);
    }
}

__global__ void k_blend_scatter(uint64_t n, const uint32_t* __restrict__ cell_of,
                                const uint32_t* __restrict__ start, uint32_t* __restrict__ cursor,
                                uint32_t* __restrict__ items) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cell_of[i];
        items[start[c] + atomicAdd(&cursor[c], 1u)] = (uint32_t)i;
    }
}

void launch_blend_grid(const float4* pa, uint64_t n, float R, float h, int G, uint32_t* cell_of,
                       uint32_t* counts, uint32_t* start, uint32_t* cursor, uint32_t* items,
                       hipStream_t st) {
    const uint64_t nc = (uint64_t)G * G * G;
    int b = (int)std::min<uint64_t>(8192, (n + 255) / 256);
    launch_fill_u32(counts, 0u, nc, st);
    launch_fill_u32(cursor, 0u, nc, st);
    hipLaunchKernelGGL(k_blend_count, dim3(b), dim3(256), 0, st, pa, n, R, h, G, cell_of, counts);
    launch_scan(counts, start, (uint32_t)nc, nullptr, 1u, start + nc, st);
    hipLaunchKernelGGL(k_blend_scatter, dim3(b), dim3(256), 0, st, n, cell_of, start, cursor,
                       items);
}

// One thread per live ray of the list whose record was written by the current pass.
__global__ __launch_bounds__(256) void k_blend(const SlotDesc* __restrict__ ds,
                                               const uint32_t* __restrict__ list,
                                               const uint32_t* __restrict__ n_live, RayState rs,
                                               int primary) {
    const uint32_t n = *n_live;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const uint32_t entry = list[e];
        const SlotDesc& d = ds[entry_slot(entry)];
        if (!(d.blend_r > 0.f)) continue;
        const uint64_t g = d.pix_base + entry_pix(entry);
        const v3f x = mkv(rs.f[RX][g], rs.f[RX + 1][g], rs.f[RX + 2][g]);
        // a primary record does not store its direction (the slot's)
        const v3f k = primary ? mkv(d.k[0], d.k[1], d.k[2])
                              : mkv(rs.f[RKX][g], rs.f[RKX + 1][g], rs.f[RKX + 2][g]);
        const float r = d.blend_r, reach = d.blend_r + d.r_max;
        const float tol = 1e-6f * d.R;  // the nearest hit itself lies on P' up to rounding
        int lo[3], hi[3];
        const float xs[3] = {x.x, x.y, x.z};
        for (int a = 0; a < 3; a++) {
            lo[a] = blend_cell(xs[a] - reach, d.R, d.bl_h, d.bl_G);
            hi[a] = blend_cell(xs[a] + reach, d.R, d.bl_h, d.bl_G);
        }
        uint64_t best = ~0ull;
        float best_s = 0.f;
        long long acc[3] = {0, 0, 0};
        long long accw = 0;
        const double q = 1099511627776.0;  // 2^40
        for (int cz = lo[2]; cz <= hi[2]; cz++)
            for (int cy = lo[1]; cy <= hi[1]; cy++)
                for (int cx = lo[0]; cx <= hi[0]; cx++) {
                    const uint32_t c = ((uint32_t)cz * d.bl_G + cy) * d.bl_G + cx;
                    for (uint32_t j = d.bl_start[c]; j < d.bl_start[c + 1]; j++) {
                        const uint32_t i = d.bl_items[j];
                        const float4 a = gld(d.pa + i), b = gld(d.pb + i);
                        if (b.w != 0.f) continue;  // absorbers neither move nor shade a hit
                        const v3f ci = mkv(a.x, a.y, a.z), ni = mkv(b.x, b.y, b.z);
                        const v3f w = sub(ci, x);
                        if (vdot(w, w) > (r + a.w) * (r + a.w)) continue;
                        const float nk = vdot(ni, k);
                        if (fabsf(nk) < kGraze) continue;
                        const float s = vdot(w, ni) / nk;
                        if (s < -tol || s > r) continue;
                        const v3f dp = sub(scl(k, s), w);  // p_i - c_i
                        const float dd = sqrtf(vdot(dp, dp));
                        if (!(dd <= a.w)) continue;
                        const float ratio = dd / a.w;
                        const uint64_t key = ((uint64_t)__float_as_uint(ratio) << 32) | i;
                        if (key < best) {
                            best = key;
                            best_s = s;
                        }
                        const double wt = 1.0 - (double)ratio;
                        const double sg = nk > 0.f ? -1.0 : 1.0;  // normal against the ray
                        acc[0] += llrint(wt * sg * ni.x * q);
                        acc[1] += llrint(wt * sg * ni.y * q);
                        acc[2] += llrint(wt * sg * ni.z * q);
                        accw += llrint(wt * q);
                    }
                }
        if (best == ~0ull) continue;  // no candidate (the hit's own disk lost to rounding)
        const uint32_t bi = (uint32_t)(best & 0xFFFFFFFFu);
        const v3f xn = add(x, scl(k, best_s));
        v3f nn;
        const double sx = (double)acc[0], sy = (double)acc[1], sz = (double)acc[2];
        const double l = sqrt(sx * sx + sy * sy + sz * sz);
        if (accw > 0 && l > 0) {
            nn = mkv((float)(sx / l), (float)(sy / l), (float)(sz / l));
        } else {
            const float4 b = gld(d.pb + bi);
            nn = mkv(b.x, b.y, b.z);
            if (vdot(nn, k) > 0.f) nn = scl(nn, -1.f);
        }
        rs.f[RX][g] = xn.x;
        rs.f[RX + 1][g] = xn.y;
        rs.f[RX + 2][g] = xn.z;
        rs.f[RNX][g] = nn.x;
        rs.f[RNX + 1][g] = nn.y;
        rs.f[RNX + 2][g] = nn.z;
        rs.d[g] += (double)best_s;
        rs.hit[g] = bi;
    }
}

void launch_blend(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live, RayState rs,
                  int primary, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_blend, dim3(n_blocks), dim3(256), 0, st, d, list, n_live, rs, primary);
}

}  // namespace pe
