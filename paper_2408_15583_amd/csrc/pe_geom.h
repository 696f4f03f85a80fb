// Device geometry shared by the bounce march, the object-space traversal and the facet records:
// fp32 3-vectors in the scene frame and the exact ray-disk test every intersection uses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pe_device.h"

namespace pe {

struct f3 {
    float x, y, z;
};
__device__ inline f3 mk3(float x, float y, float z) { return {x, y, z}; }
__device__ inline f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline f3 mirror(f3 a, f3 n) { return a - n * (2.f * dot(n, a)); }
__device__ inline f3 ld3(const RayState& rs, int c, uint64_t g) {
    return {rs.f[c][g], rs.f[c + 1][g], rs.f[c + 2][g]};
}
__device__ inline void st3(const RayState& rs, int c, uint64_t g, f3 v) {
    rs.f[c][g] = v.x;
    rs.f[c + 1][g] = v.y;
    rs.f[c + 2][g] = v.z;
}

// Direction of the ray leaving a facet: Eq. (4) reflection of the incoming direction about the
// oriented normal, renormalised (every pass that needs it computes it this one way).
__device__ inline f3 leave_dir(f3 kin, f3 nn) {
    f3 k = mirror(kin, nn);
    return k * rsqrtf(dot(k, k));
}

// Exact ray-disk test in the scene frame (two-sided; grazing |n.k| < 1e-6 misses; t > tmin;
// inclusive boundary).
__device__ inline bool disk_test(float4 a, float4 b, f3 o, f3 k, float tmin, float& t) {
    const float den = b.x * k.x + b.y * k.y + b.z * k.z;
    if (fabsf(den) < kGraze) return false;
    const f3 w = mk3(a.x - o.x, a.y - o.y, a.z - o.z);
    const float tt = (b.x * w.x + b.y * w.y + b.z * w.z) / den;
    if (!(tt > tmin)) return false;
    const f3 q = k * tt - w;
    if (dot(q, q) <= a.w * a.w) {
        t = tt;
        return true;
    }
    return false;
}

// Hit key: fp32 bits of t > 0 (monotone) above the point index, so the 64-bit minimum is the
// nearest hit with ties going to the lowest index.
__device__ inline uint64_t pack_hit(float t, uint32_t i) {
    return ((uint64_t)__float_as_uint(t) << 32) | i;
}

}  // namespace pe
