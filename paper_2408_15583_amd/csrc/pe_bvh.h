// Traversal of the object-space hierarchy over a scene's splats (Algorithm 3's TraverseSplatAS
// applied to every splat of the scene): nearest hit beyond tmin, or any hit, of one ray per
// lane.  Every point of the scene is reachable, so the result is the exact first hit of the
// fp32 disk test over all disks (ties: lowest index), independent of traversal order.
//
// The hierarchy is an octree of the points' Morton codes (node records at kBvhLeaf in
// pe_device.h).  Expanding a node tests its children's boxes and pushes ONE stack entry: the
// first child's index, the octant mask and the mask of children still to visit, so the stack
// holds at most one entry per level.  Children are visited front to back for the ray's
// direction signs (octant order XOR the sign mask); once a hit is known, a popped child's box
// is tested again against it.  Each lane's stack lives in LDS, laid out [depth][thread].
#pragma once
#include <float.h>

#include "pe_device.h"
#include "pe_geom.h"

namespace pe {

struct BvhRay {
    f3 o, inv;  // origin and reciprocal direction (components kept away from 0)
    float tmin;
};

__device__ inline float safe_inv(float k) {
    return 1.f / (fabsf(k) > 1e-20f ? k : copysignf(1e-20f, k));
}

__device__ inline BvhRay bvh_ray(f3 o, f3 k, float tmin) {
    return {o, mk3(safe_inv(k.x), safe_inv(k.y), safe_inv(k.z)), tmin};
}

// Slab test: near and far planes picked by the direction's sign.  Returns the entry parameter,
// or FLT_MAX when the box misses [tmin, tmax].
__device__ inline float box_enter(const BvhRay& r, float4 lo, float4 hi, float tmax) {
    const float ax = ((r.inv.x >= 0.f ? lo.x : hi.x) - r.o.x) * r.inv.x;
    const float bx = ((r.inv.x >= 0.f ? hi.x : lo.x) - r.o.x) * r.inv.x;
    const float ay = ((r.inv.y >= 0.f ? lo.y : hi.y) - r.o.y) * r.inv.y;
    const float by = ((r.inv.y >= 0.f ? hi.y : lo.y) - r.o.y) * r.inv.y;
    const float az = ((r.inv.z >= 0.f ? lo.z : hi.z) - r.o.z) * r.inv.z;
    const float bz = ((r.inv.z >= 0.f ? hi.z : lo.z) - r.o.z) * r.inv.z;
    const float tn = fmaxf(fmaxf(ax, ay), az);
    const float tf = fminf(fminf(bx, by), bz);
    return (tn <= tf && tf >= r.tmin && tn <= tmax) ? tn : FLT_MAX;
}

__device__ inline float key_t(uint64_t key) {
    return key == kEmptyKey ? FLT_MAX : __uint_as_float((uint32_t)(key >> 32));
}

// Nearest hit (any = false: packed key, kEmptyKey when none) or any hit (any = true: 0 when
// something is hit, kEmptyKey otherwise) of the ray (o, k) beyond tmin.  stk: this thread's
// stack base (kBvhMaxStack entries, stride apart).
template <bool any>
__device__ inline uint64_t bvh_trace(const SlotDesc& d, f3 o, f3 k, float tmin, uint64_t* stk,
                                     int stride) {
    const BvhRay r = bvh_ray(o, k, tmin);
    const uint32_t dmask = (k.x < 0.f ? 1u : 0u) | (k.y < 0.f ? 2u : 0u) | (k.z < 0.f ? 4u : 0u);
    uint64_t key = kEmptyKey;
    if (box_enter(r, gld(d.bvh), gld(d.bvh + 1), FLT_MAX) == FLT_MAX) return key;
    int sp = 0;
    uint32_t cur = 0;
    for (;;) {
        const float4 lo = gld(d.bvh + 2 * (uint64_t)cur), hi = gld(d.bvh + 2 * (uint64_t)cur + 1);
        const uint32_t first = __float_as_uint(lo.w), info = __float_as_uint(hi.w);
        if (info & kBvhLeafBit) {
            const uint32_t p1 = first + (info & 0xFFFFFFu);
            for (uint32_t p = first; p < p1; p++) {
                const float4 a = gld(d.pa_s + p), b = gld(d.pb_s + p);
                float t;
                if (disk_test(a, b, o, k, tmin, t)) {
                    if (any) return 0;
                    const uint64_t c = pack_hit(t, __float_as_uint(b.w));
                    key = c < key ? c : key;
                }
            }
        } else {
            const uint32_t occ = info & 0xFFu;
            const float tmax = any ? FLT_MAX : key_t(key);
            uint32_t pending = 0, m = occ;
#pragma unroll
            for (int c = 0; c < 8; c++) {
                if (m == 0) break;
                const uint32_t oct = __builtin_ctz(m);
                m &= m - 1u;
                const float4* cn = d.bvh + 2 * ((uint64_t)first + c);
                if (box_enter(r, gld(cn), gld(cn + 1), tmax) != FLT_MAX)
                    pending |= 1u << (oct ^ dmask);
            }
            if (pending) {
                stk[sp * stride] = (uint64_t)first | ((uint64_t)occ << 32) | ((uint64_t)pending << 40);
                sp++;
            }
        }
        // next node: front-most pending child of the deepest entry
        bool found = false;
        while (sp > 0) {
            const uint64_t e = stk[(sp - 1) * stride];
            uint32_t pend = (uint32_t)(e >> 40) & 0xFFu;
            const uint32_t j = __builtin_ctz(pend);
            pend &= pend - 1u;
            if (pend)
                stk[(sp - 1) * stride] = (e & 0xFFFFFFFFFFull) | ((uint64_t)pend << 40);
            else
                sp--;
            const uint32_t occ = (uint32_t)(e >> 32) & 0xFFu, oct = j ^ dmask;
            const uint32_t child = (uint32_t)e + __popc(occ & ((1u << oct) - 1u));
            if (!any && key != kEmptyKey) {
                const float4* cn = d.bvh + 2 * (uint64_t)child;
                if (box_enter(r, gld(cn), gld(cn + 1), key_t(key)) == FLT_MAX) continue;
            }
            cur = child;
            found = true;
            break;
        }
        if (!found) break;
    }
    return key;
}

}  // namespace pe
