// Ray generation, screen-space bounce march and live-ray compaction.
//
// Geometric optics of a bounce (Sec. II-A): the direction reflects by Eq. (4), the field by
// Eq. (2)-(3) with Gamma_p = +1 and Gamma_v = -1, which for a PEC plane is E_r = 2 (n.E) n - E;
// the tube vectors mirror the same way; the image-method path length grows by the segment.
// Secondary rays ignore hits closer than eps (Sec. III-B, after Eq. (23)).
//
// The march replaces the paper's acceleration structure over fused splats: a secondary ray is
// projected into each aggregation view and walked through that view's min/max depth pyramid
// (stackless: descend on overlap, ascend after a skipped cell); at level-0 candidate pixels
// the disks stored in the 3x3 neighbourhood are intersected exactly and the nearest hit
// beyond eps over all views wins (ties: lowest index).  Live rays are kept in an ordered list
// of (slot, pixel) entries that is compacted after every bounce with wavefront ballots and an
// exclusive scan, so the order (and every downstream sum) is deterministic.
#include <float.h>

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

// ------------------------------------------------------------------------------------------
// Ray generation from the first-hit buffer
// ------------------------------------------------------------------------------------------

__device__ inline bool primary_live(const SlotDesc& d, const uint64_t* keys, int p) {
    if (p >= d.W * d.H) return false;
    const uint64_t key = keys[d.pix_base + p];
    if (key == kEmptyKey) return false;
    const uint32_t i = (uint32_t)(key & 0xFFFFFFFFu);
    return d.pb[i].w == 0.f;  // absorbers end the ray before its first record
}

__global__ __launch_bounds__(256) void k_raygen_count(const SlotDesc* __restrict__ ds,
                                                      const uint64_t* __restrict__ keys,
                                                      uint32_t* __restrict__ wg_count) {
    const SlotDesc& d = ds[blockIdx.y];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool live = primary_live(d, keys, p);
    __shared__ uint32_t wc[4];
    const uint64_t bal = __ballot(live);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0)
        wg_count[(uint64_t)blockIdx.y * gridDim.x + blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

void launch_raygen_count(const SlotDesc* d, int n_slots, int max_pix, const uint64_t* keys,
                         uint32_t* wg_count, hipStream_t st) {
    hipLaunchKernelGGL(k_raygen_count, dim3((max_pix + 255) / 256, n_slots), dim3(256), 0, st, d,
                       keys, wg_count);
}

__global__ __launch_bounds__(256) void k_raygen_write(const SlotDesc* __restrict__ ds,
                                                      const uint64_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ wg_off,
                                                      uint32_t* __restrict__ list, RayState rs,
                                                      uint64_t* __restrict__ hitkey) {
    const uint32_t slot = blockIdx.y;
    const SlotDesc& d = ds[slot];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool live = primary_live(d, keys, p);
    __shared__ uint32_t wc[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t bal = __ballot(live);
    if (lane == 0) wc[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (p >= d.W * d.H) return;
    const uint64_t g = d.pix_base + p;
    if (!live) {
        rs.m[g] = 0;
        return;
    }
    uint32_t off = wg_off[(uint64_t)slot * gridDim.x + blockIdx.x];
    for (int w = 0; w < wave; w++) off += wc[w];
    off += (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
    list[off] = make_entry(slot, (uint32_t)p);
    hitkey[off] = kEmptyKey;

    const uint64_t key = keys[g];
    const float t = __uint_as_float((uint32_t)(key >> 32));
    const uint32_t i = (uint32_t)(key & 0xFFFFFFFFu);
    const int px = p % d.W, py = p / d.W;
    const f3 U = mk3(d.u[0], d.u[1], d.u[2]), V = mk3(d.v[0], d.v[1], d.v[2]);
    const f3 K = mk3(d.k[0], d.k[1], d.k[2]);
    const float ou = (px + 0.5f - 0.5f * d.W) * d.pitch, ov = (py + 0.5f - 0.5f * d.H) * d.pitch;
    const f3 x = U * ou + V * ov + K * (t - d.R);
    const float4 b = d.pb[i];
    f3 n = mk3(b.x, b.y, b.z);
    if (dot(n, K) > 0.f) n = n * -1.f;
    st3(rs, RX, g, x);
    st3(rs, RNX, g, n);
    st3(rs, RKX, g, K);
    st3(rs, RETX, g, mk3(d.eth[0], d.eth[1], d.eth[2]));
    st3(rs, REPX, g, mk3(d.eph[0], d.eph[1], d.eph[2]));
    st3(rs, RUX, g, U * d.pitch);
    st3(rs, RVX, g, V * d.pitch);
    rs.d[g] = (double)t - (double)d.R;
    rs.m[g] = 1;
    rs.hit[g] = i;
}

void launch_raygen_write(const SlotDesc* d, int n_slots, int max_pix, const uint64_t* keys,
                         const uint32_t* wg_off, uint32_t* list, RayState rs, uint64_t* hitkey,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_raygen_write, dim3((max_pix + 255) / 256, n_slots), dim3(256), 0, st, d,
                       keys, wg_off, list, rs, hitkey);
}

// ------------------------------------------------------------------------------------------
// March through one aggregation view
// ------------------------------------------------------------------------------------------

// Clips s to where a0 + s*da stays in [lo, hi].
__device__ inline void slab(float a0, float da, float lo, float hi, float& s0, float& s1) {
    if (da == 0.f) {
        if (a0 < lo || a0 > hi) { s0 = 1.f; s1 = 0.f; }
        return;
    }
    const float inv = 1.f / da;
    float ta = (lo - a0) * inv, tb = (hi - a0) * inv;
    if (ta > tb) { const float q = ta; ta = tb; tb = q; }
    s0 = fmaxf(s0, ta);
    s1 = fminf(s1, tb);
}

// March of one ray through one aggregation view's pyramid.  A level-0 texel is a candidate
// when the ray's depth over the pixel, widened by one pixel of travel (the 3x3 refinement
// reaches one pixel around), meets the texel's [min, max] of stored disk extents; the disks of
// the 3x3 block are then intersected exactly, skipping those already tested in the previous
// block.  A hit counts only when its point projects within one pixel of the pixel that stores
// the disk: the set of hits the views retain, whatever path pixel the test came from.
__device__ void march_view(const ViewDesc& V, f3 x, f3 k, float tmin, float smax, float tol,
                           float& best_t, uint32_t& best_i, uint32_t* cap_hits) {
    const float ip = 1.f / V.pitch;
    const f3 vu = mk3(V.u[0], V.u[1], V.u[2]), vv = mk3(V.v[0], V.v[1], V.v[2]);
    const f3 vk = mk3(V.k[0], V.k[1], V.k[2]);
    const int W = V.W, H = V.H, P = V.P;
    const float2* __restrict__ hiz = V.hiz;
    const float4* __restrict__ pix = V.pix;
    const float a0 = dot(x, vu) * ip + 0.5f * W, b0 = dot(x, vv) * ip + 0.5f * H;
    const float z0 = dot(x, vk) + V.R;
    const float da = dot(k, vu) * ip, db = dot(k, vv) * ip, dz = dot(k, vk);
    float s_lo = tmin, s_hi = fminf(smax, best_t);
    slab(a0, da, 0.f, (float)W, s_lo, s_hi);
    slab(b0, db, 0.f, (float)H, s_lo, s_hi);
    if (!(s_lo <= s_hi)) return;
    const float ida = da != 0.f ? 1.f / da : 0.f, idb = db != 0.f ? 1.f / db : 0.f;
    const float lat = fmaxf(fabsf(da), fabsf(db));
    const float zpad = (lat > 0.f ? fabsf(dz) / lat : 0.f) + tol;  // depth change per pixel
    float s = s_lo;
    int ix = min(max((int)floorf(a0 + s * da), 0), W - 1);
    int iy = min(max((int)floorf(b0 + s * db), 0), H - 1);
    int px_prev = -1000, py_prev = -1000;
    int level = 0;
    const int lmax = V.lp;
    const int cap = 4 * (W + H) * (lmax + 1) + 64;
    for (int it = 0;; it++) {
        if (it > cap) {
            atomicAdd(cap_hits, 1u);
            break;
        }
        const int cx = ix >> level, cy = iy >> level;
        const int xl = cx << level, xh = min((cx + 1) << level, W);
        const int yl = cy << level, yh = min((cy + 1) << level, H);
        const float sx = da > 0.f ? (xh - a0) * ida : (da < 0.f ? (xl - a0) * ida : FLT_MAX);
        const float sy = db > 0.f ? (yh - b0) * idb : (db < 0.f ? (yl - b0) * idb : FLT_MAX);
        const float se = fminf(fminf(sx, sy), s_hi);
        const float za = z0 + s * dz, zb = z0 + se * dz;
        const float2 h = hiz[hiz_offset(P, level) + hiz_texel(P >> level, cx, cy)];
        const bool ov = fmaxf(za, zb) + zpad >= h.x && fminf(za, zb) - zpad <= h.y;
        if (ov && level > 0) {
            level--;
            continue;
        }
        if (ov) {
            for (int dy = -1; dy <= 1; dy++) {
                const int py = iy + dy;
                if (py < 0 || py >= H) continue;
                for (int dx = -1; dx <= 1; dx++) {
                    const int px = ix + dx;
                    if (px < 0 || px >= W) continue;
                    if (abs(px - px_prev) <= 1 && abs(py - py_prev) <= 1) continue;
                    const float4 pb = pix[2 * (py * W + px) + 1];
                    const uint32_t i = __float_as_uint(pb.w);
                    if (i == kNone) continue;
                    float t;
                    if (disk_test(pix[2 * (py * W + px)], pb, x, k, tmin, t) &&
                        (t < best_t || (t == best_t && i < best_i))) {
                        // the view retains this disk for hit points within one pixel of where
                        // it is stored (the hit point's own pixel is always on the walk)
                        const int ha = (int)floorf(a0 + t * da), hb = (int)floorf(b0 + t * db);
                        if (abs(ha - px) <= 1 && abs(hb - py) <= 1) {
                            best_t = t;
                            best_i = i;
                        }
                    }
                }
            }
            px_prev = ix;
            py_prev = iy;
            s_hi = fminf(s_hi, best_t);
        }
        if (se >= s_hi) break;
        if (sx <= sy) {
            ix = da > 0.f ? xh : xl - 1;
            iy = min(max((int)floorf(b0 + se * db), yl), yh - 1);
        } else {
            iy = db > 0.f ? yh : yl - 1;
            ix = min(max((int)floorf(a0 + se * da), xl), xh - 1);
        }
        if (ix < 0 || ix >= W || iy < 0 || iy >= H) break;
        s = se;
        if (level < lmax) level++;
    }
}

// Distance along k from x (inside the bounding sphere of radius R) to the sphere.
__device__ inline float sphere_exit(f3 x, f3 k, float R) {
    const float b = dot(x, k), c = dot(x, x) - R * R;
    return -b + sqrtf(fmaxf(b * b - c, 0.f));
}

// fp32 tolerance of depth comparisons in the march (scene-size relative).
__device__ inline float march_tol(const SlotDesc& d) { return 4e-6f * d.R; }
__device__ inline float march_smax(const SlotDesc& d, f3 x, f3 k) {
    return sphere_exit(x, k, d.R * 1.0001f) + 2.f * d.r_max;
}

// Nearest hit of the ray (x, k) beyond tmin over all aggregation views, one lane (used for the
// visibility of bistatic facets).
__device__ inline void march_all(const SlotDesc& d, f3 x, f3 k, float tmin, float& best_t,
                                 uint32_t& best_i, uint32_t* cap_hits) {
    const float tol = march_tol(d);
    const float smax = march_smax(d, x, k);
    for (int v = 0; v < d.n_views; v++)
        march_view(d.views[v], x, k, tmin, smax, tol, best_t, best_i, cap_hits);
}

__device__ inline uint64_t pack_hit(float t, uint32_t i) {
    return ((uint64_t)__float_as_uint(t) << 32) | i;
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// Applies the bounce found for one live ray: on a PEC hit the record advances to the new facet
// (Eq. (2)-(4) at the old facet's normal, path += t), otherwise the ray stops and keeps its
// last record, which is what radiates under Eq. (14).
__device__ bool apply_bounce(const SlotDesc& d, uint64_t g, const RayState& rs, f3 x, f3 n, f3 k,
                             uint64_t key, int bounce) {
    const uint32_t best_i = (uint32_t)(key & 0xFFFFFFFFu);
    if (best_i == kNone) return false;
    const float best_t = __uint_as_float((uint32_t)(key >> 32));
    const float4 b = d.pb[best_i];
    if (b.w != 0.f) return false;
    f3 nn = mk3(b.x, b.y, b.z);
    if (dot(nn, k) > 0.f) nn = nn * -1.f;
    st3(rs, RX, g, x + k * best_t);
    st3(rs, RNX, g, nn);
    st3(rs, RKX, g, k);
    const f3 Et = ld3(rs, RETX, g), Ep = ld3(rs, REPX, g);
    st3(rs, RETX, g, n * (2.f * dot(n, Et)) - Et);
    st3(rs, REPX, g, n * (2.f * dot(n, Ep)) - Ep);
    st3(rs, RUX, g, mirror(ld3(rs, RUX, g), n));
    st3(rs, RVX, g, mirror(ld3(rs, RVX, g), n));
    rs.d[g] += (double)best_t;
    rs.m[g] = (uint8_t)bounce;
    rs.hit[g] = best_i;
    return true;
}

// One bounce, pass 1: every wavefront marches ONE aggregation view for 64 consecutive live
// rays (adjacent pixels of one incidence, so the lanes walk similar paths through the same
// view data).  Work items are (view, chunk) pairs in view-major order; the nearest hit of each
// (ray, view) is folded into the ray's packed t|index key with a 64-bit atomic minimum, so the
// result is the same minimum over views whatever the order (ties: lowest index).
__global__ __launch_bounds__(256, 6) void k_march(const SlotDesc* __restrict__ ds,
                                                  const uint32_t* __restrict__ list,
                                                  const uint32_t* __restrict__ n_live,
                                                  RayState rs, uint64_t* __restrict__ hitkey,
                                                  int bounce, int max_views,
                                                  uint32_t* __restrict__ cap_hits) {
    const uint32_t n = *n_live;
    const uint32_t n_chunks = (n + kWaveChunk - 1) / kWaveChunk;
    const uint32_t total = n_chunks * (uint32_t)max_views;
    const int lane = threadIdx.x & 63;
    // Each XCD takes a contiguous eighth of the (view, chunk) items so that its L2 serves one
    // region of one view; within an XCD the wavefronts stride over that range.
    const uint32_t xcd = blockIdx.x % kNumXcd;
    const uint32_t per_xcd_waves = (gridDim.x / kNumXcd) * 4;
    const uint32_t wx = __builtin_amdgcn_readfirstlane((blockIdx.x / kNumXcd) * 4 + (threadIdx.x >> 6));
    const uint32_t q0 = (uint32_t)(((uint64_t)total * xcd) / kNumXcd);
    const uint32_t q1 = (uint32_t)(((uint64_t)total * (xcd + 1)) / kNumXcd);
    for (uint32_t q = q0 + wx; q < q1; q += per_xcd_waves) {
        const uint32_t v = q / n_chunks, c = q - v * n_chunks;
        const uint32_t e = c * kWaveChunk + lane;
        if (e >= n) continue;
        const uint32_t entry = list[e];
        const SlotDesc& d = ds[entry_slot(entry)];
        if (bounce > d.max_b || (int)v >= d.n_views) continue;
        const uint64_t g = d.pix_base + entry_pix(entry);
        const f3 x = ld3(rs, RX, g), nn = ld3(rs, RNX, g), kin = ld3(rs, RKX, g);
        f3 k = mirror(kin, nn);
        k = k * rsqrtf(dot(k, k));
        // Start from the best hit other views have already published for this ray: the walk
        // then stops at that depth, and only strictly better (t, index) hits are kept, so the
        // final minimum over views is the same whatever the order in which views finish.
        const uint64_t known =
            __hip_atomic_load(&hitkey[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        float bt = FLT_MAX;
        uint32_t bi = kNone;
        if (known != kEmptyKey) {
            bt = __uint_as_float((uint32_t)(known >> 32));
            bi = (uint32_t)(known & 0xFFFFFFFFu);
        }
        march_view(d.views[v], x, k, d.eps, march_smax(d, x, k), march_tol(d), bt, bi, cap_hits);
        if (bi != kNone && pack_hit(bt, bi) < known)
            atomicMin((unsigned long long*)&hitkey[e], (unsigned long long)pack_hit(bt, bi));
    }
}

void launch_march(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live, RayState rs,
                  uint64_t* hitkey, int bounce, int max_views, uint32_t* cap_hits, int n_blocks,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_march, dim3(n_blocks), dim3(256), 0, st, d, list, n_live, rs, hitkey,
                       bounce, max_views, cap_hits);
}

// One bounce, pass 2: apply each ray's nearest hit (or stop it), reset its key for the next
// bounce, and count the survivors of each 64-entry chunk for the order-preserving compaction.
__global__ __launch_bounds__(256) void k_bounce_apply(const SlotDesc* __restrict__ ds,
                                                      const uint32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ n_live,
                                                      RayState rs, uint64_t* __restrict__ hitkey,
                                                      uint8_t* __restrict__ alive,
                                                      uint32_t* __restrict__ chunk_count,
                                                      int bounce) {
    const uint32_t n = *n_live;
    const uint32_t n_chunks = (n + kWaveChunk - 1) / kWaveChunk;
    const int lane = threadIdx.x & 63;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const uint32_t nw = gridDim.x * 4;
    for (uint32_t c = wid; c < n_chunks; c += nw) {
        const uint32_t e = c * kWaveChunk + lane;
        bool live = false;
        if (e < n) {
            const uint32_t entry = list[e];
            const SlotDesc& d = ds[entry_slot(entry)];
            const uint64_t key = hitkey[e];
            hitkey[e] = kEmptyKey;
            if (bounce <= d.max_b) {
                const uint64_t g = d.pix_base + entry_pix(entry);
                const f3 x = ld3(rs, RX, g), nn = ld3(rs, RNX, g), kin = ld3(rs, RKX, g);
                f3 k = mirror(kin, nn);
                k = k * rsqrtf(dot(k, k));
                live = apply_bounce(d, g, rs, x, nn, k, key, bounce);
            }
            alive[e] = live ? 1 : 0;
        }
        const uint64_t bal = __ballot(live);
        if (lane == 0) chunk_count[c] = (uint32_t)__popcll(bal);
    }
}

void launch_bounce_apply(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live,
                         RayState rs, uint64_t* hitkey, uint8_t* alive, uint32_t* chunk_count,
                         int bounce, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_bounce_apply, dim3(n_blocks), dim3(256), 0, st, d, list, n_live, rs,
                       hitkey, alive, chunk_count, bounce);
}

// Order-preserving compaction of 64-entry chunks, one wavefront per chunk (grid-stride over
// wavefronts, no barriers): survivors go to chunk_off[chunk] + rank among the chunk's survivors.
__global__ __launch_bounds__(256) void k_compact(const uint32_t* __restrict__ list_in,
                                                 const uint32_t* __restrict__ n_in,
                                                 const uint8_t* __restrict__ alive,
                                                 const uint32_t* __restrict__ chunk_off,
                                                 uint32_t* __restrict__ list_out) {
    const uint32_t n = *n_in;
    const uint32_t n_chunks = (n + kWaveChunk - 1) / kWaveChunk;
    const int lane = threadIdx.x & 63;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const uint32_t nw = gridDim.x * 4;
    for (uint32_t c = wid; c < n_chunks; c += nw) {
        const uint32_t e = c * kWaveChunk + lane;
        const bool live = e < n && alive[e];
        const uint64_t bal = __ballot(live);
        if (live)
            list_out[chunk_off[c] + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = list_in[e];
    }
}

void launch_compact(const uint32_t* list_in, const uint32_t* n_in, const uint8_t* alive,
                    const uint32_t* chunk_off, uint32_t* list_out, int n_blocks,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_compact, dim3(n_blocks), dim3(256), 0, st, list_in, n_in, alive,
                       chunk_off, list_out);
}

// Inspection: per-pixel last records of slot 0 (pixels without a first hit report 0 bounces).
__global__ void k_trace_out(const SlotDesc* __restrict__ ds, RayState rs,
                            int32_t* __restrict__ n_bounce, float* __restrict__ last_x,
                            float* __restrict__ last_n, double* __restrict__ path,
                            uint32_t* __restrict__ last_idx) {
    const SlotDesc& d = ds[0];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.W * d.H) return;
    const uint64_t g = d.pix_base + p;
    const int m = rs.m[g];
    if (n_bounce) n_bounce[p] = m;
    const bool h = m > 0;
    for (int c = 0; c < 3; c++) {
        if (last_x) last_x[3 * p + c] = h ? rs.f[RX + c][g] : 0.f;
        if (last_n) last_n[3 * p + c] = h ? rs.f[RNX + c][g] : 0.f;
    }
    if (path) path[p] = h ? rs.d[g] : 0.0;
    if (last_idx) last_idx[p] = h ? rs.hit[g] : kNone;
}

void launch_trace_out(const SlotDesc* d, const uint32_t* list, const uint32_t* n_list,
                      RayState rs, int32_t* n_bounce, float* last_x, float* last_n,
                      double* path, uint32_t* last_idx, int n_blocks, hipStream_t st) {
    (void)list;
    (void)n_list;
    hipLaunchKernelGGL(k_trace_out, dim3(n_blocks), dim3(256), 0, st, d, rs, n_bounce, last_x,
                       last_n, path, last_idx);
}

// Visibility (Eq. (14) Psi) of a point x toward ks through the aggregation views: blocked when
// any stored disk is hit beyond eps.  Used for bistatic observation directions.
__device__ bool visible_views(const SlotDesc& d, f3 x, f3 ks, uint32_t* cap_hits) {
    float best_t = FLT_MAX;
    uint32_t best_i = kNone;
    march_all(d, x, ks, d.eps, best_t, best_i, cap_hits);
    return best_i == kNone;
}

}  // namespace pe

namespace pe {

// Monostatic visibility of a later-bounce facet point x toward ks = -k_i: the ray leaves x back
// toward the incidence screen; it is blocked when a disk stored in the first-hit buffer around
// x's projection is hit beyond eps.  (A first-bounce facet is visible by construction: it is
// the nearest hit along its own central ray.)
__device__ bool visible_primary(const SlotDesc& d, const uint64_t* __restrict__ keys, f3 x,
                                f3 ks) {
    const float ip = 1.f / d.pitch;
    const int ix = (int)floorf((x.x * d.u[0] + x.y * d.u[1] + x.z * d.u[2]) * ip + 0.5f * d.W);
    const int iy = (int)floorf((x.x * d.v[0] + x.y * d.v[1] + x.z * d.v[2]) * ip + 0.5f * d.H);
    for (int dy = -1; dy <= 1; dy++) {
        const int py = iy + dy;
        if (py < 0 || py >= d.H) continue;
        for (int dx = -1; dx <= 1; dx++) {
            const int px = ix + dx;
            if (px < 0 || px >= d.W) continue;
            const uint64_t key = keys[d.pix_base + (uint64_t)py * d.W + px];
            if (key == kEmptyKey) continue;
            const uint32_t i = (uint32_t)(key & 0xFFFFFFFFu);
            float t;
            if (disk_test(d.pa[i], d.pb[i], x, ks, d.eps, t)) return false;
        }
    }
    return true;
}

__device__ inline f3 cross(f3 a, f3 b) {
    return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Frequency-independent part of each radiating facet of Eq. (14), per observation direction:
//   u', v' from Eq. (12)-(13); area = |u' x v'|; alpha, beta = (k_in - k_s).(u', v') / 2;
//   D = d - k_s.x (fp64); A_pq = psi * area * ([(n x h) x k_s] x k_s) . e_p, h = k_in x E_q.
__global__ __launch_bounds__(256) void k_po_prep(const SlotDesc* __restrict__ ds,
                                                 const ObsDesc* __restrict__ obs,
                                                 const uint32_t* __restrict__ list,
                                                 const uint32_t* __restrict__ n_list,
                                                 RayState rs, const uint64_t* __restrict__ keys,
                                                 ExitRecs er, uint32_t rec_stride, int seg,
                                                 int n_seg, uint32_t* cap_hits) {
    const uint32_t n = *n_list;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const uint32_t entry = list[e];
        const SlotDesc& d = ds[entry_slot(entry)];
        const uint64_t g = d.pix_base + entry_pix(entry);
        const f3 x = ld3(rs, RX, g), nn = ld3(rs, RNX, g), kin = ld3(rs, RKX, g);
        const f3 Et = ld3(rs, RETX, g), Ep = ld3(rs, REPX, g);
        const f3 u = ld3(rs, RUX, g), v = ld3(rs, RVX, g);
        const double dd = rs.d[g];
        const int m = rs.m[g];
        const float ink = 1.f / dot(nn, kin);
        const f3 up = u - kin * (dot(nn, u) * ink);
        const f3 vp = v - kin * (dot(nn, v) * ink);
        const f3 cr = cross(up, vp);
        const float area = sqrtf(dot(cr, cr));
        const f3 ht = cross(kin, Et), hp = cross(kin, Ep);
        const f3 jt = cross(nn, ht), jp = cross(nn, hp);
        for (int o = 0; o < d.n_obs; o++) {
            const ObsDesc& O = obs[d.obs_base + o];
            const f3 ks = mk3(O.ks[0], O.ks[1], O.ks[2]);
            bool vis = true;
            if (d.mono) {
                if (m >= 2) vis = visible_primary(d, keys, x, ks);
            } else {
                vis = visible_views(d, x, ks, cap_hits);
            }
            const float w = vis ? area : 0.f;
            const f3 q = kin - ks;
            const f3 Vt = cross(cross(jt, ks), ks), Vp = cross(cross(jp, ks), ks);
            const f3 rt = mk3(O.eth[0], O.eth[1], O.eth[2]), rp = mk3(O.eph[0], O.eph[1], O.eph[2]);
            const uint64_t r = ((uint64_t)o * n_seg + seg) * rec_stride + e;
            er.D[r] = dd - ((double)ks.x * x.x + (double)ks.y * x.y + (double)ks.z * x.z);
            er.al[r] = 0.5f * dot(q, up);
            er.be[r] = 0.5f * dot(q, vp);
            er.A[0][r] = w * dot(Vt, rt);
            er.A[1][r] = w * dot(Vp, rt);
            er.A[2][r] = w * dot(Vt, rp);
            er.A[3][r] = w * dot(Vp, rp);
        }
    }
}

void launch_po_prep(const SlotDesc* d, const ObsDesc* obs, const uint32_t* list,
                    const uint32_t* n_list, RayState rs, const uint64_t* keys, ExitRecs er,
                    uint32_t rec_stride, int seg, int n_seg, uint32_t* cap_hits, int n_blocks,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_po_prep, dim3(n_blocks), dim3(256), 0, st, d, obs, list, n_list, rs,
                       keys, er, rec_stride, seg, n_seg, cap_hits);
}

}  // namespace pe
