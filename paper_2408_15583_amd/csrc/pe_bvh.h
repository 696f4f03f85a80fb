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

// Traversal state of one ray (one lane), advanced one node expansion per step so that a
// wavefront can give finished lanes new rays while the others go on.
struct BvhState {
    BvhRay r;
    f3 o, k;
    uint32_t dmask;        // octant bits of the negative direction components
    uint64_t key;          // best hit so far (packed t, index); any-hit: 0 once hit
    int sp;                // stack entries in use
    uint32_t first, info;  // record fields of the node to expand next
};

// Starts a ray; false when it misses the root's box (nothing to trace).
__device__ inline bool bvh_begin(const SlotDesc& d, f3 o, f3 k, float tmin, BvhState& s) {
    s.r = bvh_ray(o, k, tmin);
    s.o = o;
    s.k = k;
    s.dmask = (k.x < 0.f ? 1u : 0u) | (k.y < 0.f ? 2u : 0u) | (k.z < 0.f ? 4u : 0u);
    s.key = kEmptyKey;
    s.sp = 0;
    const float4 lo = gld(d.bvh), hi = gld(d.bvh + 1);
    s.first = __float_as_uint(lo.w);
    s.info = __float_as_uint(hi.w);
    return box_enter(s.r, lo, hi, FLT_MAX) != FLT_MAX;
}

// One step: expands the current node (a leaf's points, or an internal node's children boxes),
// then picks the next node: the front-most hit child (its record came with its box), else the
// front-most waiting child of the deepest stack entry.  Returns true when the ray is done
// (any-hit: at the first hit, with key = 0).  stk: this lane's stack base, entries stride apart.
template <bool any>
__device__ inline bool bvh_step(const SlotDesc& d, BvhState& s, uint64_t* stk, int stride) {
    if (s.info & kBvhLeafBit) {
        const uint32_t p1 = s.first + (s.info & 0xFFFFFFu);
        for (uint32_t p = s.first; p < p1; p++) {
            const float4 a = gld(d.pa_s + p), b = gld(d.pb_s + p);
            float t;
            if (disk_test(a, b, s.o, s.k, s.r.tmin, t)) {
                if (any) {
                    s.key = 0;
                    return true;
                }
                const uint64_t c = pack_hit(t, __float_as_uint(b.w));
                s.key = c < s.key ? c : s.key;
            }
        }
    } else {
        const uint32_t occ = s.info & 0xFFu;
        const float tmax = any ? FLT_MAX : key_t(s.key);
        uint32_t pending = 0, m = occ, bj = 8u, bf = 0u, bi = 0u;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            if (m == 0) break;
            const uint32_t oct = __builtin_ctz(m);
            m &= m - 1u;
            const float4* cn = d.bvh + 2 * ((uint64_t)s.first + c);
            const float4 lo = gld(cn), hi = gld(cn + 1);
            if (box_enter(s.r, lo, hi, tmax) != FLT_MAX) {
                const uint32_t rank = oct ^ s.dmask;
                pending |= 1u << rank;
                if (rank < bj) {
                    bj = rank;
                    bf = __float_as_uint(lo.w);
                    bi = __float_as_uint(hi.w);
                }
            }
        }
        if (pending) {
            pending &= ~(1u << bj);
            if (pending) {
                stk[s.sp * stride] =
                    (uint64_t)s.first | ((uint64_t)occ << 32) | ((uint64_t)pending << 40);
                s.sp++;
            }
            s.first = bf;
            s.info = bi;
            return false;
        }
    }
    while (s.sp > 0) {
        const uint64_t e = stk[(s.sp - 1) * stride];
        uint32_t pend = (uint32_t)(e >> 40) & 0xFFu;
        const uint32_t j = __builtin_ctz(pend);
        pend &= pend - 1u;
        if (pend)
            stk[(s.sp - 1) * stride] = (e & 0xFFFFFFFFFFull) | ((uint64_t)pend << 40);
        else
            s.sp--;
        const uint32_t occ = (uint32_t)(e >> 32) & 0xFFu, oct = j ^ s.dmask;
        const float4* cn = d.bvh + 2 * ((uint64_t)(uint32_t)e + __popc(occ & ((1u << oct) - 1u)));
        const float4 lo = gld(cn), hi = gld(cn + 1);
        // once a hit is known, a waiting child entered beyond it is skipped
        if (!any && s.key != kEmptyKey && box_enter(s.r, lo, hi, key_t(s.key)) == FLT_MAX)
            continue;
        s.first = __float_as_uint(lo.w);
        s.info = __float_as_uint(hi.w);
        return false;
    }
    return true;
}

// Whole traversal of one ray on one lane: nearest hit (any = false: packed key, kEmptyKey when
// none) or any hit (any = true: 0 when something is hit, kEmptyKey otherwise).
template <bool any>
__device__ inline uint64_t bvh_trace(const SlotDesc& d, f3 o, f3 k, float tmin, uint64_t* stk,
                                     int stride) {
    BvhState s;
    if (!bvh_begin(d, o, k, tmin, s)) return kEmptyKey;
    while (!bvh_step<any>(d, s, stk, stride)) {
    }
    return s.key;
}

}  // namespace pe
