// Traversal of the object-space hierarchy over a scene's splats (Algorithm 3's TraverseSplatAS
// applied to every splat of the scene): nearest hit beyond tmin, or any hit, of one ray per
// lane.  Every point of the scene is reachable, so the result is the exact first hit of the
// fp32 disk test over all disks (ties: lowest index), independent of traversal order.
//
// The hierarchy is the octree of the points' Morton codes (kBvhLeaf in pe_device.h), traversed
// through its wide records (kWideRec): one 80-byte record per internal node holds the boxes of
// all its children, quantised to 8 bits per plane relative to the node's own box and rounded
// outward, so expanding a node is one memory round trip however many children it has.  Leaf
// children are not records: their points sit consecutively in a leaf-ordered copy of the scene
// (wpts), and the points of every hit leaf child of a node form one point group, tested four
// points per round trip before the traversal descends further.
//
// Per lane the traversal keeps a node group (the record base of a node's internal children,
// the mask of hit children still to visit in front-to-back rank order = octant XOR the ray's
// sign mask, the octant mask of internal children) and a point group (base and 64-bit mask).
// Descending into a child pushes the rest of the current node group, so the LDS stack holds at
// most one u64 per level; a popped group is not culled again (its boxes were tested when its
// parent was expanded, and the child's own children are tested against the current hit).
#pragma once
#include <float.h>

#include "pe_device.h"
#include "pe_geom.h"

namespace pe {

__device__ inline float safe_inv(float k) {
    return 1.f / (fabsf(k) > 1e-20f ? k : copysignf(1e-20f, k));
}

__device__ inline float key_t(uint64_t key) {
    return key == kEmptyKey ? FLT_MAX : __uint_as_float((uint32_t)(key >> 32));
}

__device__ inline uint4 gld(const uint4* p) {
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    const v4u r = *(const __attribute__((address_space(1))) v4u*)p;
    return make_uint4(r.x, r.y, r.z, r.w);
}

// Disk test of the traversal, written without early exits so that a batch of points can be
// requested before the first test: the same arithmetic as disk_test (IEEE division, grazing
// |n.k| < kGraze misses, t > tmin, inclusive boundary); FLT_MAX when the disk is missed.
__device__ inline float disk_t(float4 a, float4 b, f3 o, f3 k, float tmin) {
    const float den = b.x * k.x + b.y * k.y + b.z * k.z;
    const f3 w = mk3(a.x - o.x, a.y - o.y, a.z - o.z);
    const float tt = (b.x * w.x + b.y * w.y + b.z * w.z) / den;
    const f3 q = k * tt - w;
    const bool hit = fabsf(den) >= kGraze && tt > tmin && dot(q, q) <= a.w * a.w;
    return hit ? tt : FLT_MAX;
}

// Traversal state of one ray (one lane), advanced one round trip per step so that a wavefront
// can give finished lanes new rays while the others go on.
struct BvhState {
    f3 o, k, inv;          // origin, direction, reciprocal direction (kept away from 0)
    float tmin;
    uint32_t dmask;        // octant bits of the negative direction components
    uint64_t key;          // best hit so far (packed t, index); any-hit: 0 once hit
    int sp;                // stack entries in use
    uint32_t gbase, ghits, giocc;  // node group
    uint32_t pbase;                // point group: wpts index of its first point
    uint64_t pmask;                //   and the points still to test
    const uint4* wrec;             // the ray's scene (kept per lane: a launch may mix scenes)
    const float4* wpts;
    uint64_t out;                  // where the pass writes the ray's result
};

// What a ray needs of its scene to start: the wide records, the leaf-ordered points, the
// point count of a leaf root, and the root's exact box (kept in the slot descriptor so that a
// ray starts without a round trip of its own).
struct BvhScene {
    const uint4* wrec;
    const float4* wpts;
    uint32_t root_pts;
    float lo[3], hi[3];
};

// The scene fields of a slot descriptor (read through the global address space; the caller
// pins them with bvh_pin together with its own fields, so that all are requested in one round).
__device__ inline BvhScene bvh_scene(const SlotDesc* dp) {
    typedef const __attribute__((address_space(1))) SlotDesc& GSlot;
    GSlot sd = (GSlot)*dp;
    BvhScene b;
    b.wrec = sd.wrec;
    b.wpts = sd.wpts;
    b.root_pts = sd.w_root_pts;
    for (int a = 0; a < 3; a++) {
        b.lo[a] = sd.bvh_lo[a];
        b.hi[a] = sd.bvh_hi[a];
    }
    return b;
}

// Keeps the compiler from sinking the loads of these values into their first uses (which
// would make each a round trip of its own): they are all requested before any is waited for.
template <class A, class B, class C>
__device__ inline void bvh_pin(BvhScene& b, A& x, B& y, C& z) {
    asm volatile("" : "+v"(b.wrec), "+v"(b.wpts), "+v"(b.root_pts), "+v"(b.lo[0]), "+v"(b.lo[1]),
                 "+v"(b.lo[2]), "+v"(b.hi[0]), "+v"(b.hi[1]), "+v"(b.hi[2]), "+v"(x), "+v"(y),
                 "+v"(z));
}

// Starts a ray; false when it misses the root's box (nothing to trace).
__device__ inline bool bvh_begin(const BvhScene& sc, f3 o, f3 k, float tmin, BvhState& s) {
    s.o = o;
    s.k = k;
    s.inv = mk3(safe_inv(k.x), safe_inv(k.y), safe_inv(k.z));
    s.tmin = tmin;
    s.dmask = (k.x < 0.f ? 1u : 0u) | (k.y < 0.f ? 2u : 0u) | (k.z < 0.f ? 4u : 0u);
    s.key = kEmptyKey;
    s.sp = 0;
    s.wrec = sc.wrec;
    s.wpts = sc.wpts;
    // the root's exact box (slab test with the near and far planes picked by the signs)
    const float ax = ((s.inv.x >= 0.f ? sc.lo[0] : sc.hi[0]) - o.x) * s.inv.x;
    const float bx = ((s.inv.x >= 0.f ? sc.hi[0] : sc.lo[0]) - o.x) * s.inv.x;
    const float ay = ((s.inv.y >= 0.f ? sc.lo[1] : sc.hi[1]) - o.y) * s.inv.y;
    const float by = ((s.inv.y >= 0.f ? sc.hi[1] : sc.lo[1]) - o.y) * s.inv.y;
    const float az = ((s.inv.z >= 0.f ? sc.lo[2] : sc.hi[2]) - o.z) * s.inv.z;
    const float bz = ((s.inv.z >= 0.f ? sc.hi[2] : sc.lo[2]) - o.z) * s.inv.z;
    const float tn = fmaxf(fmaxf(ax, ay), az), tf = fminf(fminf(bx, by), bz);
    if (!(tn <= tf && tf >= tmin)) return false;
    if (sc.root_pts) {  // the whole scene is one leaf
        s.pbase = 0;
        s.pmask = (1ull << sc.root_pts) - 1ull;
        s.ghits = 0;
    } else {  // a node group holding the root record alone (octant 0, internal)
        s.pmask = 0;
        s.gbase = 0;
        s.giocc = 1u;
        s.ghits = 1u << s.dmask;
    }
    return true;
}

// Points tested per round trip of a point group.
constexpr int kBvhBatch = 4;

// Point step: tests up to kBvhBatch points of the lane's point group.  Returns true when the
// ray is done (any-hit: at the first hit, with key = 0).
template <bool any>
__device__ inline bool bvh_points(BvhState& s) {
    uint64_t mm = s.pmask;
    uint32_t p[kBvhBatch];
    bool ok[kBvhBatch];
#pragma unroll
    for (int i = 0; i < kBvhBatch; i++) {
        ok[i] = mm != 0;
        p[i] = ok[i] ? s.pbase + (uint32_t)__builtin_ctzll(mm) : p[0];
        mm &= mm - 1ull;
    }
    s.pmask = mm;
    // all requests go out before the first test (a slot a lane does not need repeats its
    // first point's address, and its test result is dropped)
    float4 pa[kBvhBatch], pb[kBvhBatch];
#pragma unroll
    for (int i = 0; i < kBvhBatch; i++) {
        pa[i] = gld(s.wpts + 2 * (uint64_t)p[i]);
        pb[i] = gld(s.wpts + 2 * (uint64_t)p[i] + 1);
    }
#pragma unroll
    for (int i = 0; i < kBvhBatch; i++) {
        const float t = disk_t(pa[i], pb[i], s.o, s.k, s.tmin);
        if (ok[i] && t != FLT_MAX) {
            if (any) {
                s.key = 0;
                return true;
            }
            const uint64_t c = pack_hit(t, __float_as_uint(pb[i].w));
            s.key = c < s.key ? c : s.key;
        }
    }
    return s.pmask == 0 && s.ghits == 0 && s.sp == 0;
}

// Node step (for a lane whose point group is empty): expands the front-most child of the node
// group, popping a group when the current one is spent; the child's hit internal children
// become the node group and its hit leaf children's points the point group.  Returns true when
// the ray is done.  stk: this lane's stack base, entries stride apart.
template <bool any>
__device__ inline bool bvh_node(BvhState& s, uint64_t* stk, int stride) {
    if (s.ghits == 0) {
        if (s.sp == 0) return true;
        const uint64_t e = stk[(--s.sp) * stride];
        s.gbase = (uint32_t)e;
        s.ghits = (uint32_t)(e >> 32) & 0xFFu;
        s.giocc = (uint32_t)(e >> 40) & 0xFFu;
    }
    const uint32_t r = __builtin_ctz(s.ghits), oct = r ^ s.dmask;
    s.ghits &= s.ghits - 1u;
    const uint32_t idx = s.gbase + __popc(s.giocc & ((1u << oct) - 1u));
    if (s.ghits) {
        stk[s.sp * stride] =
            (uint64_t)s.gbase | ((uint64_t)s.ghits << 32) | ((uint64_t)s.giocc << 40);
        s.sp++;
    }
    const uint4* rec = s.wrec + (uint64_t)kWideRec * idx;
    const uint4 q0 = gld(rec), q1 = gld(rec + 1), q2 = gld(rec + 2), q3 = gld(rec + 3),
                q4 = gld(rec + 4);
    // plane parameter of quantised coordinate q on axis a: (org + q scale - o) / k, as
    // q (scale / k) + (org - o) / k
    const float sx = __uint_as_float((q0.w & 0xFFu) << 23) * s.inv.x;
    const float sy = __uint_as_float(((q0.w >> 8) & 0xFFu) << 23) * s.inv.y;
    const float sz = __uint_as_float(((q0.w >> 16) & 0xFFu) << 23) * s.inv.z;
    const float ax = (__uint_as_float(q0.x) - s.o.x) * s.inv.x;
    const float ay = (__uint_as_float(q0.y) - s.o.y) * s.inv.y;
    const float az = (__uint_as_float(q0.z) - s.o.z) * s.inv.z;
    const uint32_t occ = q0.w >> 24, iocc = q1.z, counts = q1.w;
    const float tmax = any ? FLT_MAX : key_t(s.key);
    // the near plane of an axis is the low one where the ray runs toward +axis (reciprocal
    // > 0), else the high one: picked once per record.  The plane parameter q (scale / k) +
    // (org - o) / k is monotonic in q (a correctly rounded fma of a monotonic map), so the
    // picked planes give exactly the minimum and maximum of each child's two.
    const bool bx = s.inv.x < 0.f, by = s.inv.y < 0.f, bz = s.inv.z < 0.f;
    const uint32_t nx[2] = {bx ? q3.z : q2.x, bx ? q3.w : q2.y},
                   fx[2] = {bx ? q2.x : q3.z, bx ? q2.y : q3.w},
                   ny[2] = {by ? q4.x : q2.z, by ? q4.y : q2.w},
                   fy[2] = {by ? q2.z : q4.x, by ? q2.w : q4.y},
                   nz[2] = {bz ? q4.z : q3.x, bz ? q4.w : q3.y},
                   fz[2] = {bz ? q3.x : q4.z, bz ? q3.y : q4.w};
    // hit octants, then the internal ones to the node group (rank order) and the leaf ones'
    // points to the point group.  Any-hit skips an octant no lane of the wavefront occupies;
    // nearest-hit tests all eight (fewer instructions than the skip's branches) and keeps the
    // occupied ones.
    uint32_t hits = 0;
#pragma unroll
    for (int o = 0; o < 8; o++) {
        if (any && !((occ >> o) & 1u)) continue;
        const int w = o >> 2, sh = 8 * (o & 3);
        const float tn = fmaxf(fmaxf(fmaf((float)((nx[w] >> sh) & 0xFFu), sx, ax),
                                     fmaf((float)((ny[w] >> sh) & 0xFFu), sy, ay)),
                               fmaf((float)((nz[w] >> sh) & 0xFFu), sz, az));
        const float tf = fminf(fminf(fmaf((float)((fx[w] >> sh) & 0xFFu), sx, ax),
                                     fmaf((float)((fy[w] >> sh) & 0xFFu), sy, ay)),
                               fmaf((float)((fz[w] >> sh) & 0xFFu), sz, az));
        hits |= (tn <= tf && tf >= s.tmin && tn <= tmax) ? 1u << o : 0u;
    }
    hits &= occ;
    // the hit internal octants in rank order (octant XOR sign mask): XOR with each set bit of
    // the sign mask swaps neighbouring bits, pairs of bits or nibbles
    uint32_t nh = hits & iocc;
    if (s.dmask & 1u) nh = ((nh & 0x55u) << 1) | ((nh >> 1) & 0x55u);
    if (s.dmask & 2u) nh = ((nh & 0x33u) << 2) | ((nh >> 2) & 0x33u);
    if (s.dmask & 4u) nh = ((nh & 0x0Fu) << 4) | (nh >> 4);
    // point bits of octant o: cnt_o bits from S_o, the sum of the lower octants' counts (at
    // most 64 in all).  The S_o come as bytes: the counts summed in pairs, each byte then the
    // sum of the pairs below it (a 24-bit multiply by 0x010101, which ignores the top pair,
    // shifted up a byte; no byte carries over) for the even octants' starts, plus the even
    // octant's count for the odd ones'.  Counts of leaf octants not hit are cleared (a nibble
    // mask spread from the hit bits; its last two steps written as shift-or instructions,
    // which the compiler would otherwise fold into a full 32-bit multiply by 15) after the
    // offsets are taken.
    const uint32_t ce = counts & 0x0F0F0F0Fu, co = (counts >> 4) & 0x0F0F0F0Fu;
    const uint32_t pr = ce + co;
    const uint32_t s_even = __umul24(pr, 0x010101u) << 8, s_odd = s_even + ce;
    uint32_t lm = hits & ~iocc;
    lm = (lm | (lm << 12)) & 0x000F000Fu;
    lm = (lm | (lm << 6)) & 0x03030303u;
    lm = (lm | (lm << 3)) & 0x11111111u;
    asm("v_lshl_or_b32 %0, %1, 1, %1" : "=v"(lm) : "v"(lm));
    asm("v_lshl_or_b32 %0, %1, 2, %1" : "=v"(lm) : "v"(lm));
    const uint32_t hc = counts & lm;
    uint64_t pm = 0;
#pragma unroll
    for (int o = 0; o < 8; o++) {
        const uint32_t cnt = (hc >> (4 * o)) & 0xFu;
        const uint32_t st = (((o & 1) ? s_odd : s_even) >> (8 * (o >> 1))) & 63u;
        pm |= (uint64_t)((1u << cnt) - 1u) << st;
    }
    s.gbase = q1.x;
    s.giocc = iocc;
    s.ghits = nh;
    s.pbase = q1.y;
    s.pmask = pm;
    return nh == 0 && pm == 0 && s.sp == 0;
}

// One step of a lane: a point step while its point group holds points, else a node step (the
// persistent loop can instead take one kind of step for the whole wavefront at a time).
template <bool any>
__device__ inline bool bvh_step(const SlotDesc&, BvhState& s, uint64_t* stk, int stride) {
    return s.pmask != 0 ? bvh_points<any>(s) : bvh_node<any>(s, stk, stride);
}

}  // namespace pe
