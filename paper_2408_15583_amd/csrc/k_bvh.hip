// Object-space hierarchy over a scene's splats and the secondary-hit pass that traverses it.
//
// Algorithm 3 builds an acceleration structure over the splats and traverses it for every ray
// and bounce.  Here the splats are the scene's points, already sorted by their 30-bit Morton
// codes, so an octree needs no sorting or splitting search: the points sharing a 3 l-bit code
// prefix form a node of level l, and its children (the occupied octants of the next 3 bits) are
// contiguous runs found by binary search in the sorted codes.  The tree is built one level at a
// time (count, scan, emit), then its boxes bottom-up; a leaf's box is the union of its disks'
// exact boxes (centre +- r sqrt(1 - n_a^2) per axis), widened by a scene-relative slack so that
// any hit the fp32 disk test accepts lies inside it.
#include <float.h>

#include <algorithm>

#include "pe_bvh.h"
#include "pe_device.h"
#include "pe_geom.h"

namespace pe {

// First index i in [a, b) whose octant ((codes[i] >> s) & 7) is >= o (codes of [a, b) share
// their bits above s + 2, so the octants are non-decreasing there).
__device__ inline uint32_t octant_bound(const uint32_t* codes, uint32_t a, uint32_t b, int s,
                                        uint32_t o) {
    while (a < b) {
        const uint32_t mid = a + (b - a) / 2;
        if (((codes[mid] >> s) & 7u) < o)
            a = mid + 1;
        else
            b = mid;
    }
    return a;
}

// Children of node (a, b) at `level`: octant boundaries bnd[0..8] (level < 10), or a count
// split into k chunks (level >= 10, all 30 code bits shared); returns the child count (0 = leaf).
__device__ inline int node_children(const uint32_t* codes, uint32_t a, uint32_t b, int level,
                                    uint32_t bnd[9], uint32_t& split_len) {
    const uint32_t cnt = b - a;
    if (cnt <= (uint32_t)kBvhLeaf) return 0;
    if (level >= 10) {
        const uint32_t k = min(8u, (cnt + kBvhLeaf - 1) / kBvhLeaf);
        split_len = (cnt + k - 1) / k;
        return (int)k;
    }
    const int s = 27 - 3 * level;
    bnd[0] = a;
    bnd[8] = b;
    int nc = 0;
    for (uint32_t o = 1; o < 8; o++) bnd[o] = octant_bound(codes, bnd[o - 1], b, s, o);
    for (int o = 0; o < 8; o++) nc += bnd[o] < bnd[o + 1];
    return nc;
}

__global__ __launch_bounds__(256) void k_bvh_count(const uint2* __restrict__ rng, uint32_t n_nodes,
                                                   int level, const uint32_t* __restrict__ codes,
                                                   uint32_t* __restrict__ ccount) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_nodes;
         j += gridDim.x * blockDim.x) {
        uint32_t bnd[9], len = 0;
        ccount[j] = (uint32_t)node_children(codes, rng[j].x, rng[j].y, level, bnd, len);
    }
}

void launch_bvh_count(const uint2* rng, uint32_t n_nodes, int level, const uint32_t* codes,
                      uint32_t* ccount, hipStream_t st) {
    const uint32_t b = std::min<uint32_t>(65535u, (n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_bvh_count, dim3(b), dim3(256), 0, st, rng, n_nodes, level, codes,
                       ccount);
}

__global__ __launch_bounds__(256) void k_bvh_emit(const uint2* __restrict__ rng, uint32_t n_nodes,
                                                  int level, const uint32_t* __restrict__ codes,
                                                  const uint32_t* __restrict__ coff,
                                                  uint32_t cbase, uint2* __restrict__ rng_next,
                                                  uint2* __restrict__ finfo) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_nodes;
         j += gridDim.x * blockDim.x) {
        const uint32_t a = rng[j].x, b = rng[j].y;
        uint32_t bnd[9], len = 0;
        const int nc = node_children(codes, a, b, level, bnd, len);
        if (nc == 0) {
            finfo[j] = make_uint2(a, kBvhLeafBit | (b - a));
            continue;
        }
        uint2* out = rng_next + coff[j];
        uint32_t occ = 0;
        if (level >= 10) {
            for (int c = 0; c < nc; c++)
                out[c] = make_uint2(a + c * len, min(a + (c + 1) * len, b));
            occ = (1u << nc) - 1u;
        } else {
            int c = 0;
            for (int o = 0; o < 8; o++)
                if (bnd[o] < bnd[o + 1]) {
                    out[c++] = make_uint2(bnd[o], bnd[o + 1]);
                    occ |= 1u << o;
                }
        }
        finfo[j] = make_uint2(cbase + coff[j], occ);
    }
}

void launch_bvh_emit(const uint2* rng, uint32_t n_nodes, int level, const uint32_t* codes,
                     const uint32_t* coff, uint32_t cbase, uint2* rng_next, uint2* finfo,
                     hipStream_t st) {
    const uint32_t b = std::min<uint32_t>(65535u, (n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_bvh_emit, dim3(b), dim3(256), 0, st, rng, n_nodes, level, codes, coff,
                       cbase, rng_next, finfo);
}

__global__ __launch_bounds__(256) void k_bvh_box(const uint2* __restrict__ finfo, uint32_t n_nodes,
                                                 uint32_t base, const float4* __restrict__ pa_s,
                                                 const float4* __restrict__ pb_s, float pad,
                                                 float4* __restrict__ nodes) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_nodes;
         j += gridDim.x * blockDim.x) {
        const uint32_t first = finfo[j].x, info = finfo[j].y;
        float4 lo = make_float4(FLT_MAX, FLT_MAX, FLT_MAX, 0.f);
        float4 hi = make_float4(-FLT_MAX, -FLT_MAX, -FLT_MAX, 0.f);
        if (info & kBvhLeafBit) {
            const uint32_t p1 = first + (info & 0xFFFFFFu);
            for (uint32_t p = first; p < p1; p++) {
                const float4 a = pa_s[p], b = pb_s[p];
                const float ex = a.w * sqrtf(fmaxf(0.f, 1.f - b.x * b.x));
                const float ey = a.w * sqrtf(fmaxf(0.f, 1.f - b.y * b.y));
                const float ez = a.w * sqrtf(fmaxf(0.f, 1.f - b.z * b.z));
                lo.x = fminf(lo.x, a.x - ex);
                lo.y = fminf(lo.y, a.y - ey);
                lo.z = fminf(lo.z, a.z - ez);
                hi.x = fmaxf(hi.x, a.x + ex);
                hi.y = fmaxf(hi.y, a.y + ey);
                hi.z = fmaxf(hi.z, a.z + ez);
            }
            lo.x -= pad;
            lo.y -= pad;
            lo.z -= pad;
            hi.x += pad;
            hi.y += pad;
            hi.z += pad;
        } else {
            const uint32_t nc = __popc(info & 0xFFu);
            for (uint32_t c = 0; c < nc; c++) {
                const float4 a = nodes[2 * ((uint64_t)first + c)];
                const float4 b = nodes[2 * ((uint64_t)first + c) + 1];
                lo.x = fminf(lo.x, a.x);
                lo.y = fminf(lo.y, a.y);
                lo.z = fminf(lo.z, a.z);
                hi.x = fmaxf(hi.x, b.x);
                hi.y = fmaxf(hi.y, b.y);
                hi.z = fmaxf(hi.z, b.z);
            }
        }
        lo.w = __uint_as_float(first);
        hi.w = __uint_as_float(info);
        nodes[2 * ((uint64_t)base + j)] = lo;
        nodes[2 * ((uint64_t)base + j) + 1] = hi;
    }
}

void launch_bvh_box(const uint2* finfo, uint32_t n_nodes, uint32_t base, const float4* pa_s,
                    const float4* pb_s, float pad, float4* nodes, hipStream_t st) {
    const uint32_t b = std::min<uint32_t>(65535u, (n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_bvh_box, dim3(b), dim3(256), 0, st, finfo, n_nodes, base, pa_s, pb_s,
                       pad, nodes);
}

__global__ __launch_bounds__(256) void k_wide_count(const float4* __restrict__ nodes,
                                                    uint32_t n_nodes, uint32_t* __restrict__ is_int,
                                                    uint32_t* __restrict__ leafpts) {
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n_nodes;
         g += gridDim.x * blockDim.x) {
        const uint32_t first = __float_as_uint(nodes[2 * (uint64_t)g].w);
        const uint32_t info = __float_as_uint(nodes[2 * (uint64_t)g + 1].w);
        uint32_t pts = 0;
        if (!(info & kBvhLeafBit)) {
            const uint32_t nc = __popc(info & 0xFFu);
            for (uint32_t c = 0; c < nc; c++) {
                const uint32_t ci = __float_as_uint(nodes[2 * ((uint64_t)first + c) + 1].w);
                if (ci & kBvhLeafBit) pts += ci & 0xFFFFFFu;
            }
        }
        is_int[g] = (info & kBvhLeafBit) ? 0u : 1u;
        leafpts[g] = pts;
    }
}

void launch_wide_count(const float4* nodes, uint32_t n_nodes, uint32_t* is_int,
                       uint32_t* leafpts, hipStream_t st) {
    const uint32_t b = std::min<uint32_t>(65535u, (n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_wide_count, dim3(b), dim3(256), 0, st, nodes, n_nodes, is_int, leafpts);
}

// Outward 8-bit quantisation of one axis of a child box [clo, chi] in the frame (org, scale):
// the planes org + q scale, evaluated in fp32 as the traversal evaluates them, enclose it.
__device__ inline void quantise_axis(float org, float scale, float clo, float chi, uint32_t& qlo,
                                     uint32_t& qhi) {
    int a = (int)floorf((clo - org) / scale), b = (int)ceilf((chi - org) / scale);
    a = min(max(a, 0), 255);
    b = min(max(b, 0), 255);
    while (a > 0 && org + (float)a * scale > clo) a--;
    while (b < 255 && org + (float)b * scale < chi) b++;
    qlo = (uint32_t)a;
    qhi = (uint32_t)b;
}

__device__ inline void copy_points(const float4* __restrict__ pa_s,
                                   const float4* __restrict__ pb_s, uint32_t first, uint32_t cnt,
                                   float4* __restrict__ wpts, uint32_t dst) {
    for (uint32_t i = 0; i < cnt; i++) {
        wpts[2 * ((uint64_t)dst + i)] = pa_s[first + i];
        wpts[2 * ((uint64_t)dst + i) + 1] = pb_s[first + i];
    }
}

__global__ __launch_bounds__(256) void k_wide_emit(const float4* __restrict__ nodes,
                                                   uint32_t n_nodes,
                                                   const uint32_t* __restrict__ rec,
                                                   const uint32_t* __restrict__ lbase,
                                                   const float4* __restrict__ pa_s,
                                                   const float4* __restrict__ pb_s,
                                                   uint4* __restrict__ wrec,
                                                   float4* __restrict__ wpts) {
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n_nodes;
         g += gridDim.x * blockDim.x) {
        const float4 lo = nodes[2 * (uint64_t)g], hi = nodes[2 * (uint64_t)g + 1];
        const uint32_t first = __float_as_uint(lo.w), info = __float_as_uint(hi.w);
        if (info & kBvhLeafBit) {
            if (g == 0) copy_points(pa_s, pb_s, first, info & 0xFFFFFFu, wpts, 0);
            continue;
        }
        // per-axis scale 2^e, the smallest power of two whose 255 steps from the low corner
        // reach the high corner in fp32
        const float org[3] = {lo.x, lo.y, lo.z}, top[3] = {hi.x, hi.y, hi.z};
        float scale[3];
        uint32_t eb[3];
        for (int a = 0; a < 3; a++) {
            const float ext = fmaxf(top[a] - org[a], 0.f);
            int e = -100;
            if (ext > 0.f) {
                frexpf(ext / 255.f, &e);
                e = max(e, -100);
            }
            while (e < 120 && org[a] + 255.f * ldexpf(1.f, e) < top[a]) e++;
            scale[a] = ldexpf(1.f, e);
            eb[a] = (uint32_t)(e + 127);
        }
        const uint32_t occ = info & 0xFFu, nc = __popc(occ);
        uint32_t iocc = 0, counts = 0, off = 0, m = occ;
        uint32_t q[6][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (uint32_t c = 0; c < nc; c++) {
            const uint32_t o = __builtin_ctz(m);
            m &= m - 1u;
            const float4 clo = nodes[2 * ((uint64_t)first + c)];
            const float4 chi = nodes[2 * ((uint64_t)first + c) + 1];
            const uint32_t cinfo = __float_as_uint(chi.w);
            if (cinfo & kBvhLeafBit) {
                const uint32_t cnt = cinfo & 0xFFFFFFu;
                counts |= cnt << (4 * o);
                copy_points(pa_s, pb_s, __float_as_uint(clo.w), cnt, wpts, lbase[g] + off);
                off += cnt;
            } else {
                iocc |= 1u << o;
            }
            const float cl[3] = {clo.x, clo.y, clo.z}, ch[3] = {chi.x, chi.y, chi.z};
            const int w = o >> 2, sh = 8 * (o & 3);
            for (int a = 0; a < 3; a++) {
                uint32_t ql, qh;
                quantise_axis(org[a], scale[a], cl[a], ch[a], ql, qh);
                q[a][w] |= ql << sh;
                q[3 + a][w] |= qh << sh;
            }
        }
        uint4* r = wrec + (uint64_t)kWideRec * rec[g];
        r[0] = make_uint4(__float_as_uint(org[0]), __float_as_uint(org[1]),
                          __float_as_uint(org[2]), eb[0] | (eb[1] << 8) | (eb[2] << 16) | (occ << 24));
        r[1] = make_uint4(rec[first], lbase[g], iocc, counts);
        r[2] = make_uint4(q[0][0], q[0][1], q[1][0], q[1][1]);
        r[3] = make_uint4(q[2][0], q[2][1], q[3][0], q[3][1]);
        r[4] = make_uint4(q[4][0], q[4][1], q[5][0], q[5][1]);
    }
}

void launch_wide_emit(const float4* nodes, uint32_t n_nodes, const uint32_t* rec,
                      const uint32_t* lbase, const float4* pa_s, const float4* pb_s,
                      uint4* wrec, float4* wpts, hipStream_t st) {
    const uint32_t b = std::min<uint32_t>(65535u, (n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_wide_emit, dim3(b), dim3(256), 0, st, nodes, n_nodes, rec, lbase, pa_s,
                       pb_s, wrec, wpts);
}

// Threads per workgroup of the traversal kernels; a lane's stack entries lie this many apart
// in LDS (a constant, so an entry's address is a shift, not a multiply).
constexpr int kBvhBlock = 256;

// Launch parameter of the persistent loop: idle lanes at which a wavefront refills (bits 0-7,
// 1 .. 64) and the quorum of lanes holding points for a point step (bits 8-15, 0 .. 64).
static int pack_refill(int refill) {
    const int r = std::min(64, std::max(1, refill & 0xFF));
    const int q = std::min(64, (refill >> 8) & 0xFF);
    return r | (q << 8);
}

// Persistent traversal loop shared by the two passes: every lane holds one ray; a wavefront
// takes new work items for its idle lanes from a global counter once at least `refill` of its
// lanes are idle (all from one atomic, so the lanes of a batch are neighbouring items), and
// advances its busy lanes one node expansion per iteration.  The loop indices and the exit
// test are wave-uniform (ballots, the shuffled counter value), so every lane leaves together.
// start(j, s): set up item j (returns false when it needs no traversal, after writing its
// result); finish(j, s): write the result of a finished item.
template <bool any, class Start, class Finish>
__device__ inline void bvh_persistent(const SlotDesc* __restrict__ ds, uint64_t n_items,
                                      uint32_t* __restrict__ queue, int refill, int quorum,
                                      Start start, Finish finish) {
    extern __shared__ uint64_t stk[];
    uint64_t* my = stk + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool active = false, exhausted = n_items == 0;
    uint64_t item = 0;
    const SlotDesc* dp = ds;
    BvhState s;
    for (;;) {
        const uint64_t idle = __ballot(!active);
        const int n_idle = __popcll(idle);
        if (!exhausted && n_idle >= refill) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(queue, (uint32_t)n_idle);
            base = __shfl(base, 0);
            if ((uint64_t)base + (uint64_t)n_idle >= n_items) exhausted = true;
            if (!active) {
                const uint64_t j = (uint64_t)base + __popcll(idle & ((1ull << lane) - 1ull));
                if (j < n_items) {
                    item = j;
                    active = start(j, dp, s);
                }
            }
        }
        const uint64_t act = __ballot(active);
        if (act == 0) {
            if (exhausted) break;
            continue;
        }
        // quorum > 0: one kind of step per iteration for the whole wavefront, point tests once
        // `quorum` lanes (or all busy lanes) hold points, else node expansions by the lanes
        // that hold none; quorum 0: each lane takes its own kind of step
        bool done = false;
        if (quorum > 0) {
            const uint64_t want = __ballot(active && s.pmask != 0);
            const bool points = __popcll(want) >= quorum || want == act;
            if (points) {
                if (active && s.pmask != 0) done = bvh_points<any>(s);
            } else {
                if (active && s.pmask == 0) done = bvh_node<any>(s, my, kBvhBlock);
            }
        } else if (active) {
            done = bvh_step<any>(*dp, s, my, kBvhBlock);
        }
        if (done) {
            finish(item, s);
            active = false;
        }
    }
}

// One bounce, pass 1 with every splat as bounce geometry: each live ray leaves its facet along
// the Eq. (4) reflection and takes the nearest disk hit beyond eps over the whole scene; the
// packed (t, index) key goes to hitkey[entry] for the apply pass.
__global__ __launch_bounds__(kBvhBlock) void k_trace_bvh(const SlotDesc* __restrict__ ds,
                                                   const uint32_t* __restrict__ list,
                                                   const uint32_t* __restrict__ n_live,
                                                   RayState rs, uint64_t* __restrict__ hitkey,
                                                   int bounce, uint32_t* __restrict__ queue,
                                                   int refill) {
    bvh_persistent<false>(
        ds, *n_live, queue, refill & 0xFF, refill >> 8,
        [&](uint64_t j, const SlotDesc*& dp, BvhState& s) {
            // three rounds of loads: the entry; the slot's fields; the ray state
            const uint32_t entry = list[j];
            dp = ds + entry_slot(entry);
            typedef const __attribute__((address_space(1))) SlotDesc& GSlot;
            GSlot sd = (GSlot)*dp;
            int max_b = sd.max_b;
            uint64_t pix_base = sd.pix_base;
            float eps = sd.eps;
            BvhScene sc = bvh_scene(dp);
            bvh_pin(sc, max_b, pix_base, eps);
            // the ray state is read whatever the bounce guard says (the entry's pixel is
            // always in range)
            const uint64_t g = pix_base + entry_pix(entry);
            const f3 x = ld3(rs, RX, g), nn = ld3(rs, RNX, g);
            // a primary record (every ray of the second bounce) does not store its direction
            const f3 kin = bounce == 2 ? mk3(sd.k[0], sd.k[1], sd.k[2]) : ld3(rs, RKX, g);
            if (bounce <= max_b && bvh_begin(sc, x, leave_dir(kin, nn), eps, s)) return true;
            hitkey[j] = kEmptyKey;
            return false;
        },
        [&](uint64_t j, const BvhState& s) { hitkey[j] = s.key; });
}

void launch_trace_bvh(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live,
                      RayState rs, uint64_t* hitkey, int bounce, int stack_depth,
                      uint32_t* queue, int refill, int n_blocks, hipStream_t st) {
    launch_fill_u32(queue, 0u, 1, st);
    hipLaunchKernelGGL(k_trace_bvh, dim3(n_blocks), dim3(kBvhBlock),
                       (size_t)stack_depth * kBvhBlock * sizeof(uint64_t), st, d, list, n_live, rs,
                       hitkey, bounce, queue, pack_refill(refill));
}

// Visibility, pass 1: which entries need a traced Psi (every facet of a bistatic slot, the
// later-bounce facets of a monostatic one), with per-chunk survivor counts for the compaction.
__global__ __launch_bounds__(256) void k_psi_mark(const SlotDesc* __restrict__ ds,
                                                  const uint32_t* __restrict__ list,
                                                  const uint32_t* __restrict__ n_list,
                                                  RayState rs, uint8_t* __restrict__ alive,
                                                  uint32_t* __restrict__ chunk_count) {
    const uint32_t n = *n_list;
    const uint32_t n_chunks = (n + kWaveChunk - 1) / kWaveChunk;
    const int lane = threadIdx.x & 63;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const uint32_t nw = gridDim.x * 4;
    for (uint32_t c = wid; c < n_chunks; c += nw) {
        const uint32_t e = c * kWaveChunk + lane;
        bool need = false;
        if (e < n) {
            const uint32_t entry = list[e];
            const SlotDesc& d = ds[entry_slot(entry)];
            need = !d.mono || rs.m[d.pix_base + entry_pix(entry)] >= 2;
            alive[e] = need ? 1 : 0;
        }
        const uint64_t bal = __ballot(need);
        if (lane == 0) chunk_count[c] = (uint32_t)__popcll(bal);
    }
}

void launch_psi_mark(const SlotDesc* d, const uint32_t* list, const uint32_t* n_list,
                     RayState rs, uint8_t* alive, uint32_t* chunk_count, int n_blocks,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_psi_mark, dim3(n_blocks), dim3(256), 0, st, d, list, n_list, rs, alive,
                       chunk_count);
}

// Visibility, pass 2: one lane per (compacted facet, observation direction): any hit toward
// k_s beyond eps.
__global__ __launch_bounds__(kBvhBlock) void k_psi_trace(const SlotDesc* __restrict__ ds,
                                                   const ObsDesc* __restrict__ obs,
                                                   const uint32_t* __restrict__ list,
                                                   const uint32_t* __restrict__ n_list,
                                                   int max_obs, RayState rs,
                                                   uint8_t* __restrict__ vis, uint64_t vis_stride,
                                                   uint32_t* __restrict__ queue, int refill) {
    bvh_persistent<true>(
        ds, (uint64_t)*n_list * (uint32_t)max_obs, queue, refill & 0xFF, refill >> 8,
        [&](uint64_t w, const SlotDesc*& dp, BvhState& s) {
            // three rounds of loads: the entry; the slot's fields; the facet position and the
            // observation direction
            const uint32_t o = (uint32_t)(w % (uint32_t)max_obs);
            const uint32_t entry = list[w / (uint32_t)max_obs];
            dp = ds + entry_slot(entry);
            typedef const __attribute__((address_space(1))) SlotDesc& GSlot;
            GSlot sd = (GSlot)*dp;
            int n_obs = sd.n_obs, obs_base = sd.obs_base;
            uint64_t pix_base = sd.pix_base;
            float eps = sd.eps;
            BvhScene sc = bvh_scene(dp);
            bvh_pin(sc, n_obs, pix_base, eps);
            asm volatile("" : "+v"(obs_base));
            const uint64_t g = pix_base + entry_pix(entry);
            const bool take = (int)o < n_obs;
            const ObsDesc& O = obs[take ? obs_base + (int)o : obs_base];
            const f3 x = ld3(rs, RX, g), ks = mk3(O.ks[0], O.ks[1], O.ks[2]);
            if (!take) return false;
            s.out = o * vis_stride + g;
            if (bvh_begin(sc, x, ks, eps, s)) return true;
            vis[s.out] = 1;
            return false;
        },
        [&](uint64_t, const BvhState& s) { vis[s.out] = s.key == kEmptyKey ? 1 : 0; });
}

void launch_psi_trace(const SlotDesc* d, const ObsDesc* obs, const uint32_t* list,
                      const uint32_t* n_list, int max_obs, RayState rs, uint8_t* vis,
                      uint64_t vis_stride, int stack_depth, uint32_t* queue, int refill,
                      int n_blocks, hipStream_t st) {
    launch_fill_u32(queue, 0u, 1, st);
    hipLaunchKernelGGL(k_psi_trace, dim3(n_blocks), dim3(kBvhBlock),
                       (size_t)stack_depth * kBvhBlock * sizeof(uint64_t), st, d, obs, list, n_list,
                       max_obs, rs, vis, vis_stride, queue, pack_refill(refill));
}

}  // namespace pe
