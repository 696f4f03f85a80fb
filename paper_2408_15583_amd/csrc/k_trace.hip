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
#include "pe_geom.h"

namespace pe {

// ------------------------------------------------------------------------------------------
// Ray generation from the first-hit buffer
// ------------------------------------------------------------------------------------------

// Incoming direction, fields and tube vectors of a primary record, which ray generation does
// not store (they are the same for every pixel of the slot).
__device__ inline f3 primary_dir(const SlotDesc& d) { return mk3(d.k[0], d.k[1], d.k[2]); }
__device__ inline void primary_fields(const SlotDesc& d, f3& Et, f3& Ep, f3& U, f3& V) {
    Et = mk3(d.eth[0], d.eth[1], d.eth[2]);
    Ep = mk3(d.eph[0], d.eph[1], d.eph[2]);
    U = mk3(d.u[0], d.u[1], d.u[2]) * d.pitch;
    V = mk3(d.v[0], d.v[1], d.v[2]) * d.pitch;
}

__device__ inline bool primary_live(const SlotDesc& d, const uint64_t* keys, int p) {
    if (p >= d.W * d.H) return false;
    const uint64_t key = keys[d.pix_base + p];
    if (key == kEmptyKey) return false;
    const uint32_t i = (uint32_t)(key & 0xFFFFFFFFu);
    return gld(d.pb + i).w == 0.f;  // absorbers end the ray before its first record
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
    if (hitkey) hitkey[off] = kEmptyKey;  // null: the bounce pass writes every key itself

    const uint64_t key = keys[g];
    const float t = __uint_as_float((uint32_t)(key >> 32));
    const uint32_t i = (uint32_t)(key & 0xFFFFFFFFu);
    const int px = p % d.W, py = p / d.W;
    const f3 U = mk3(d.u[0], d.u[1], d.u[2]), V = mk3(d.v[0], d.v[1], d.v[2]);
    const f3 K = mk3(d.k[0], d.k[1], d.k[2]);
    const float ou = (px + 0.5f - 0.5f * d.W) * d.pitch, ov = (py + 0.5f - 0.5f * d.H) * d.pitch;
    const f3 x = U * ou + V * ov + K * (t - d.R);
    const float4 b = gld(d.pb + i);
    f3 n = mk3(b.x, b.y, b.z);
    if (dot(n, K) > 0.f) n = n * -1.f;
    st3(rs, RX, g, x);
    st3(rs, RNX, g, n);
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
//
// The walk is a small state machine (walk_init, then walk_step until it returns false) so
// that a lane can finish one walk and start the next without waiting for its wavefront.
struct Walk {
    const float2* hiz;  // the view's pyramid and pixel records, held in registers
    const float4* pix;
    int W, H, P, lp;
    float tmin;
    float a0, b0, z0, da, db, dz, ida, idb, zpad;
    float s, s_hi;
    int ix, iy, px_prev, py_prev, level, it, cap;
};

// The fields of a view descriptor a walk starts from, read in one round of loads.
struct ViewFields {
    f3 u, v, k;
    float pitch, R;
    int W, H, P, lp;
    const float2* hiz;
    const float4* pix;
};

__device__ inline ViewFields view_fields(const ViewDesc& Vr) {
    typedef const __attribute__((address_space(1))) ViewDesc& GView;
    GView V = (GView)Vr;  // the view table lives in global memory
    ViewFields f;
    f.u = mk3(V.u[0], V.u[1], V.u[2]);
    f.v = mk3(V.v[0], V.v[1], V.v[2]);
    f.k = mk3(V.k[0], V.k[1], V.k[2]);
    f.pitch = V.pitch;
    f.R = V.R;
    f.W = V.W;
    f.H = V.H;
    f.P = V.P;
    f.lp = V.lp;
    f.hiz = V.hiz;
    f.pix = V.pix;
    return f;
}

__device__ inline bool walk_init(const ViewFields& V, f3 x, f3 k, float tmin, float smax,
                                 float tol, float best_t, Walk& w) {
    const float ip = 1.f / V.pitch;
    const f3 vu = V.u, vv = V.v, vk = V.k;
    const int W = V.W, H = V.H;
    w.hiz = V.hiz;
    w.pix = V.pix;
    w.W = W;
    w.H = H;
    w.P = V.P;
    w.lp = V.lp;
    w.tmin = tmin;
    w.a0 = dot(x, vu) * ip + 0.5f * W;
    w.b0 = dot(x, vv) * ip + 0.5f * H;
    w.z0 = dot(x, vk) + V.R;
    w.da = dot(k, vu) * ip;
    w.db = dot(k, vv) * ip;
    w.dz = dot(k, vk);
    float s_lo = tmin;
    w.s_hi = fminf(smax, best_t);
    slab(w.a0, w.da, 0.f, (float)W, s_lo, w.s_hi);
    slab(w.b0, w.db, 0.f, (float)H, s_lo, w.s_hi);
    if (!(s_lo <= w.s_hi)) return false;
    w.ida = w.da != 0.f ? 1.f / w.da : 0.f;
    w.idb = w.db != 0.f ? 1.f / w.db : 0.f;
    const float lat = fmaxf(fabsf(w.da), fabsf(w.db));
    w.zpad = (lat > 0.f ? fabsf(w.dz) / lat : 0.f) + tol;  // depth change per pixel
    w.s = s_lo;
    w.ix = min(max((int)floorf(w.a0 + s_lo * w.da), 0), W - 1);
    w.iy = min(max((int)floorf(w.b0 + s_lo * w.db), 0), H - 1);
    w.px_prev = -1000;
    w.py_prev = -1000;
    w.level = 0;
    w.it = 0;
    w.cap = 4 * (W + H) * (V.lp + 1) + 64;
    return true;
}

// The cell after [xl, xh) x [yl, yh) whose exit is at se (sx, sy: exits through the x and y
// sides); false when the walk ends there.  Written with selects, not branches: lanes of a
// wavefront take both sides at once.
__device__ inline bool cell_next(const Walk& w, float sx, float sy, float se, int xl, int xh,
                                 int yl, int yh, int& nix, int& niy) {
    const bool along_x = sx <= sy;
    const int cxn = min(max((int)floorf(w.a0 + se * w.da), xl), xh - 1);
    const int cyn = min(max((int)floorf(w.b0 + se * w.db), yl), yh - 1);
    nix = along_x ? (w.da > 0.f ? xh : xl - 1) : cxn;
    niy = along_x ? cyn : (w.db > 0.f ? yh : yl - 1);
    return (se < w.s_hi) & (nix >= 0) & (nix < w.W) & (niy >= 0) & (niy < w.H);
}

// Moves the walk past its current cell (see cell_next); false once the walk is over.
__device__ inline bool walk_advance(Walk& w, float sx, float sy, float se, int xl, int xh, int yl,
                                    int yh) {
    int nix, niy;
    if (!cell_next(w, sx, sy, se, xl, xh, yl, yh, nix, niy)) return false;
    w.ix = nix;
    w.iy = niy;
    w.s = se;
    w.level = min(w.level + 1, w.lp);
    return true;
}

__device__ inline void cell_exits(const Walk& w, int xl, int xh, int yl, int yh, float& sx,
                                  float& sy, float& se) {
    const float bx = (float)(w.da > 0.f ? xh : xl), by = (float)(w.db > 0.f ? yh : yl);
    sx = w.da != 0.f ? (bx - w.a0) * w.ida : FLT_MAX;
    sy = w.db != 0.f ? (by - w.b0) * w.idb : FLT_MAX;
    se = fminf(fminf(sx, sy), w.s_hi);
}

enum { kWalkOver = 0, kWalkMoved = 1, kWalkRefine = 2 };

// Probe of the walk's current cell against the pyramid: the walk descends on overlap above
// level 0, moves on past a cell it misses, and at an overlapping level-0 cell reports that the
// exact 3x3 refinement (walk_refine) is due before it moves on.  The texel of the child cell
// (one level down, holding the walk's pixel) is fetched in the same round trip, so a descent
// and the step that follows it take one probe: the walk visits the same cells as one level per
// probe would.  The outcome is applied with selects.
__device__ inline int walk_probe(Walk& w, uint32_t* cap_hits) {
    if (w.it++ > w.cap) {
        atomicAdd(cap_hits, 1u);
        return kWalkOver;
    }
    const int W = w.W, H = w.H, P = w.P, lv = w.level, lc = max(lv - 1, 0);
    const int cx = w.ix >> lv, cy = w.iy >> lv, cx2 = w.ix >> lc, cy2 = w.iy >> lc;
    const float2 h = gld(w.hiz + hiz_offset(P, lv) + hiz_texel(P >> lv, cx, cy));
    const float2 h2 = gld(w.hiz + hiz_offset(P, lc) + hiz_texel(P >> lc, cx2, cy2));
    const int xl = cx << lv, xh = min((cx + 1) << lv, W);
    const int yl = cy << lv, yh = min((cy + 1) << lv, H);
    const int xl2 = cx2 << lc, xh2 = min((cx2 + 1) << lc, W);
    const int yl2 = cy2 << lc, yh2 = min((cy2 + 1) << lc, H);
    float sx, sy, se, sx2, sy2, se2;
    cell_exits(w, xl, xh, yl, yh, sx, sy, se);
    cell_exits(w, xl2, xh2, yl2, yh2, sx2, sy2, se2);
    const float za = w.z0 + w.s * w.dz, zb = w.z0 + se * w.dz, zb2 = w.z0 + se2 * w.dz;
    const bool ov = (fmaxf(za, zb) + w.zpad >= h.x) & (fminf(za, zb) - w.zpad <= h.y);
    const bool ov2 = (fmaxf(za, zb2) + w.zpad >= h2.x) & (fminf(za, zb2) - w.zpad <= h2.y);
    // an overlap above level 0 hands the decision to the child cell
    const bool child = ov & (lv > 0);
    const int ls = child ? lc : lv;
    const bool ovs = child ? ov2 : ov;
    int nix, niy;
    const float Se = child ? se2 : se;
    const bool ok = cell_next(w, child ? sx2 : sx, child ? sy2 : sy, Se, child ? xl2 : xl,
                              child ? xh2 : xh, child ? yl2 : yl, child ? yh2 : yh, nix, niy);
    const bool down = ovs & (ls > 0), move = !ovs & ok;
    w.level = down ? ls - 1 : (move ? min(ls + 1, w.lp) : ls);
    w.ix = move ? nix : w.ix;
    w.iy = move ? niy : w.iy;
    w.s = move ? Se : w.s;
    return (down | move) ? kWalkMoved : (ovs ? kWalkRefine : kWalkOver);
}

// The exact test of the 3x3 block around the walk's level-0 cell, then the move past the cell;
// false once the walk is over.
__device__ inline bool walk_refine(f3 x, f3 k, Walk& w, float& best_t, uint32_t& best_i) {
    const int W = w.W, H = w.H;
    const int xl = w.ix, xh = min(w.ix + 1, W), yl = w.iy, yh = min(w.iy + 1, H);
    float sx, sy, se;
    cell_exits(w, xl, xh, yl, yh, sx, sy, se);
    // The pixels of the 3x3 block not tested in the previous block, one line of three at a
    // time with all of a line's records requested before any is used (one memory round trip
    // per line).  Lines are columns when the walk moved along x, since the new pixels then
    // form one column, and rows otherwise.  The kept hit is the minimum of (t, index) over
    // retained hits, so the visiting order does not change it.
    const float4* __restrict__ pix = w.pix;
    const bool cols = w.iy == w.py_prev;
    for (int l = -1; l <= 1; l++) {
        float4 ra[3], rb[3];
        bool use[3];
        int qx[3], qy[3];
        bool any = false;
#pragma unroll
        for (int m = 0; m < 3; m++) {
            qx[m] = w.ix + (cols ? l : m - 1);
            qy[m] = w.iy + (cols ? m - 1 : l);
            use[m] = qx[m] >= 0 && qx[m] < W && qy[m] >= 0 && qy[m] < H &&
                     !(abs(qx[m] - w.px_prev) <= 1 && abs(qy[m] - w.py_prev) <= 1);
            any |= use[m];
        }
        if (!any) continue;
#pragma unroll
        for (int m = 0; m < 3; m++) {
            // unused slots read the walk's own pixel, which is in bounds
            const int q = use[m] ? qy[m] * W + qx[m] : w.iy * W + w.ix;
            ra[m] = gld(pix + 2 * q);
            rb[m] = gld(pix + 2 * q + 1);
        }
#pragma unroll
        for (int m = 0; m < 3; m++) {
            const uint32_t i = __float_as_uint(rb[m].w);
            if (!use[m] || i == kNone) continue;
            float t;
            if (disk_test(ra[m], rb[m], x, k, w.tmin, t) &&
                (t < best_t || (t == best_t && i < best_i))) {
                // the view retains this disk for hit points within one pixel of where it is
                // stored (the hit point's own pixel is always on the walk)
                const int ha = (int)floorf(w.a0 + t * w.da), hb = (int)floorf(w.b0 + t * w.db);
                if (abs(ha - qx[m]) <= 1 && abs(hb - qy[m]) <= 1) {
                    best_t = t;
                    best_i = i;
                }
            }
        }
    }
    w.px_prev = w.ix;
    w.py_prev = w.iy;
    w.s_hi = fminf(w.s_hi, best_t);
    return walk_advance(w, sx, sy, se, xl, xh, yl, yh);
}

// One cell of the walk; false once the walk is over.
__device__ inline bool walk_step(f3 x, f3 k, Walk& w, float& best_t, uint32_t& best_i,
                                 uint32_t* cap_hits) {
    const int r = walk_probe(w, cap_hits);
    if (r == kWalkRefine) return walk_refine(x, k, w, best_t, best_i);
    return r == kWalkMoved;
}

__device__ void march_view(const ViewDesc& V, f3 x, f3 k, float tmin, float smax, float tol,
                           float& best_t, uint32_t& best_i, uint32_t* cap_hits) {
    Walk w;
    if (!walk_init(view_fields(V), x, k, tmin, smax, tol, best_t, w)) return;
    while (walk_step(x, k, w, best_t, best_i, cap_hits)) {
    }
}

// Distance along k from x (inside the bounding sphere of radius R) to the sphere.
__device__ inline float sphere_exit(f3 x, f3 k, float R) {
    const float b = dot(x, k), c = dot(x, x) - R * R;
    return -b + sqrtf(fmaxf(b * b - c, 0.f));
}

// fp32 tolerance of depth comparisons in the march (scene-size relative).
__device__ inline float march_tol(float R) { return 4e-6f * R; }
__device__ inline float march_tol(const SlotDesc& d) { return march_tol(d.R); }
__device__ inline float march_smax(float R, float r_max, f3 x, f3 k) {
    return sphere_exit(x, k, R * 1.0001f) + 2.f * r_max;
}
__device__ inline float march_smax(const SlotDesc& d, f3 x, f3 k) {
    return march_smax(d.R, d.r_max, x, k);
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
    const float4 b = gld(d.pb + best_i);
    if (b.w != 0.f) return false;
    f3 nn = mk3(b.x, b.y, b.z);
    if (dot(nn, k) > 0.f) nn = nn * -1.f;
    st3(rs, RX, g, x + k * best_t);
    st3(rs, RNX, g, nn);
    st3(rs, RKX, g, k);
    f3 Et, Ep, U, V;
    if (bounce == 2) {
        primary_fields(d, Et, Ep, U, V);
    } else {
        Et = ld3(rs, RETX, g);
        Ep = ld3(rs, REPX, g);
        U = ld3(rs, RUX, g);
        V = ld3(rs, RVX, g);
    }
    st3(rs, RETX, g, n * (2.f * dot(n, Et)) - Et);
    st3(rs, REPX, g, n * (2.f * dot(n, Ep)) - Ep);
    st3(rs, RUX, g, mirror(U, n));
    st3(rs, RVX, g, mirror(V, n));
    rs.d[g] += (double)best_t;
    rs.m[g] = (uint8_t)bounce;
    rs.hit[g] = best_i;
    return true;
}

// Lane-parallel refinement of a wavefront's pending walks: every pending lane publishes its
// ray, its level-0 cell and the new pixels of its 3x3 block (those outside the previous block)
// in LDS; then all 64 lanes take the (walk, pixel) candidates in turn, test them exactly and
// fold retained hits into the owner's packed (t, index) key with an LDS 64-bit minimum (t > 0,
// so the key order is the order of t, then of the index: the same choice as the serial test).
struct RefineWave {
    float prm[64][12];             // x, k, tmin, a0, b0, da, db, bits(ix | iy << 16) (owner)
    uint32_t width[64];            // W of the owner's view
    const float4* pix[64];         // the owner's view pixel records
    unsigned long long key[64];    // the owner's best (t, index) so far
    uint16_t cand[64 * 9];         // owner lane | (3x3 position << 6)
};

// The 3x3 positions (bit (dy + 1) * 3 + dx + 1) of the walk's block that are inside the view
// and outside the previous block.
__device__ inline uint32_t refine_mask(const Walk& w) {
    uint32_t m = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) {
            const int px = w.ix + dx, py = w.iy + dy;
            const bool use = (px >= 0) & (px < w.W) & (py >= 0) & (py < w.H) &
                             !((abs(px - w.px_prev) <= 1) & (abs(py - w.py_prev) <= 1));
            m |= use ? 1u << ((dy + 1) * 3 + dx + 1) : 0u;
        }
    return m;
}

// A wavefront runs its pending refinements once kRefineBatch lanes wait for one, or once the
// waiting lanes are at least 1 / kRefineRatio of its busy lanes.
constexpr int kRefillIdleFirst = 56;  // idle lanes before a refill, second bounce
constexpr int kRefillIdle = 48;       // the same for later bounces
constexpr int kRefineBatch = 8;
constexpr int kRefineRatio = 4;

// One bounce, pass 1: the (view, ray) walks of the live list, view-major, each XCD taking a
// contiguous eighth so that its L2 serves few views at a time (and then helping the other
// XCDs once its own eighth is drained).  Lanes run walks independently: a lane that finishes
// publishes its hit and, once most of its wavefront is idle (kRefillIdleFirst / kRefillIdle
// lanes), the wavefront takes the next walks with one atomic (consecutive rays of one view, so
// the new lanes are coherent with each other; refilling earlier trades that coherence for
// fewer idle lanes and was measured slower).  Each walk starts from the best hit already published
// for its ray and keeps only strictly better (t, index) hits, and the hits fold into the
// ray's packed t|index key with a 64-bit atomic minimum: the result is the minimum over views
// whatever the order in which walks run.
__global__ __launch_bounds__(256, 4) void k_march(const SlotDesc* __restrict__ ds,
                                                  const uint32_t* __restrict__ list,
                                                  const uint32_t* __restrict__ n_live,
                                                  RayState rs, uint64_t* __restrict__ hitkey,
                                                  int bounce, int max_views,
                                                  uint32_t* __restrict__ cap_hits,
                                                  uint32_t* __restrict__ queue) {
    const uint32_t n = *n_live;
    const uint64_t total = (uint64_t)n * (uint32_t)max_views;
    const int lane = threadIdx.x & 63;
    // Walks right after the primary hits are coherent (neighbouring pixels of one screen): a
    // wavefront keeps them together by refilling only once most of its lanes are idle.  Later
    // bounces have scattered directions and gain more from busier lanes than from coherence.
    const int refill_idle = bounce <= 2 ? kRefillIdleFirst : kRefillIdle;
    // the XCD's own eighth first, then the other eighths in turn (work left at the end)
    uint32_t src = blockIdx.x % kNumXcd;
    int tried = 1;
    uint64_t q0 = (total * src) / kNumXcd, q1 = (total * (src + 1)) / kNumXcd;
    bool active = false, exhausted = total == 0;
    uint32_t e = 0;
    f3 x = mk3(0.f, 0.f, 0.f), k = x;
    float bt = FLT_MAX;
    uint32_t bi = kNone;
    uint32_t known_i = kNone;  // index of the published hit the walk started from
    bool pend = false;         // the walk waits for its level-0 refinement
    Walk w;
    __shared__ RefineWave rwave[4];
    RefineWave& rw = rwave[threadIdx.x >> 6];
    for (;;) {
        const uint64_t idle = __ballot(!active);
        const int n_idle = __popcll(idle);
        if (!exhausted && n_idle >= refill_idle) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(queue + src, (uint32_t)n_idle);
            base = __shfl(base, 0);
            if (!active) {
                const uint64_t j = q0 + base + (uint64_t)__popcll(idle & ((1ull << lane) - 1ull));
                if (j < q1) {
                    const uint32_t v = (uint32_t)(j / n);
                    e = (uint32_t)(j - (uint64_t)v * n);
                    // three rounds of dependent loads: the entry and the best hit other views
                    // have already published for the ray; the slot's fields; the ray state and
                    // the view's descriptor
                    const uint32_t entry = list[e];
                    const uint64_t known = __hip_atomic_load(&hitkey[e], __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                    typedef const __attribute__((address_space(1))) SlotDesc& GSlot;
                    GSlot sd = (GSlot)ds[entry_slot(entry)];
                    int max_b = sd.max_b, n_views = sd.n_views;
                    uint64_t pix_base = sd.pix_base;
                    const ViewDesc* views = sd.views;
                    float eps = sd.eps, R = sd.R, r_max = sd.r_max;
                    // keep the compiler from sinking these loads into their later uses (which
                    // would make them rounds of their own)
                    asm volatile("" : "+v"(max_b), "+v"(n_views), "+v"(pix_base), "+v"(views),
                                 "+v"(eps), "+v"(R), "+v"(r_max));
                    // the ray state is read whatever the guard says (the entry's pixel is
                    // always in range), so that it shares a round with the view's descriptor
                    const bool take = (bounce <= max_b) & ((int)v < n_views);
                    const uint64_t g = pix_base + entry_pix(entry);
                    const f3 xs = ld3(rs, RX, g), nn = ld3(rs, RNX, g);
                    const f3 kin = bounce == 2 ? mk3(sd.k[0], sd.k[1], sd.k[2]) : ld3(rs, RKX, g);
                    bt = FLT_MAX;
                    bi = kNone;
                    if (known != kEmptyKey) {
                        bt = __uint_as_float((uint32_t)(known >> 32));
                        bi = (uint32_t)(known & 0xFFFFFFFFu);
                    }
                    known_i = bi;
                    if (take) {
                        const ViewFields vf = view_fields(views[v]);
                        __builtin_amdgcn_sched_barrier(0);  // issue these before waiting above
                        x = xs;
                        k = leave_dir(kin, nn);
                        active = walk_init(vf, x, k, eps, march_smax(R, r_max, x, k),
                                           march_tol(R), bt, w);
                    }
                }
            }
            if (q0 + base + (uint64_t)n_idle >= q1) {
                if (tried == kNumXcd) {
                    exhausted = true;
                } else {
                    src = (src + 1) % kNumXcd;
                    tried++;
                    q0 = (total * src) / kNumXcd;
                    q1 = (total * (src + 1)) / kNumXcd;
                }
            }
        }
        if (exhausted && __ballot(active) == 0ull) break;
        bool over = false;
        if (active && !pend) {
            const int r = walk_probe(w, cap_hits);
            pend = r == kWalkRefine;
            over = r == kWalkOver;
        }
        // Refinements wait until enough lanes of the wavefront need one, so that the long
        // refinement path runs for many lanes at once instead of stalling the traversal of
        // all the others at nearly every step.
        const int n_pend = __popcll(__ballot(pend));
        if (n_pend > 0) {
            const int n_busy = __popcll(__ballot(active));
            if (n_pend >= kRefineBatch || kRefineRatio * n_pend >= n_busy) {
                uint32_t m = 0;
                if (pend) {
                    m = refine_mask(w);
                    float* pr = rw.prm[lane];
                    pr[0] = x.x; pr[1] = x.y; pr[2] = x.z;
                    pr[3] = k.x; pr[4] = k.y; pr[5] = k.z;
                    pr[6] = w.tmin; pr[7] = w.a0; pr[8] = w.b0; pr[9] = w.da; pr[10] = w.db;
                    pr[11] = __uint_as_float((uint32_t)w.ix | ((uint32_t)w.iy << 16));
                    rw.width[lane] = (uint32_t)w.W;
                    rw.pix[lane] = w.pix;
                    rw.key[lane] = pack_hit(bt, bi);
                }
                // exclusive scan of the candidate counts over the wavefront
                const int cnt = __popc(m);
                int incl = cnt;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int v = __shfl_up(incl, o);
                    if (lane >= o) incl += v;
                }
                const int n_cand = __shfl(incl, 63);
                int off = incl - cnt;
                while (m) {
                    const int b = __ffs(m) - 1;
                    m &= m - 1;
                    rw.cand[off++] = (uint16_t)(lane | (b << 6));
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int j = lane; j < n_cand; j += 64) {
                    const uint32_t c = rw.cand[j];
                    const int o = (int)(c & 63u), b = (int)(c >> 6);
                    const float* pr = rw.prm[o];
                    const uint32_t cell = __float_as_uint(pr[11]);
                    const int qx = (int)(cell & 0xFFFFu) + b % 3 - 1;
                    const int qy = (int)(cell >> 16) + b / 3 - 1;
                    const int q = qy * (int)rw.width[o] + qx;
                    const float4* pix = rw.pix[o];
                    const float4 ra = gld(pix + 2 * q), rb = gld(pix + 2 * q + 1);
                    const uint32_t i = __float_as_uint(rb.w);
                    float t;
                    if (i != kNone &&
                        disk_test(ra, rb, mk3(pr[0], pr[1], pr[2]), mk3(pr[3], pr[4], pr[5]),
                                  pr[6], t)) {
                        // retained by the view for hit points within one pixel of where it is
                        // stored
                        const int ha = (int)floorf(pr[7] + t * pr[9]);
                        const int hb = (int)floorf(pr[8] + t * pr[10]);
                        if (abs(ha - qx) <= 1 && abs(hb - qy) <= 1)
                            atomicMin(&rw.key[o], (unsigned long long)pack_hit(t, i));
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (pend) {
                    pend = false;
                    const unsigned long long kk = rw.key[lane];
                    bt = __uint_as_float((uint32_t)(kk >> 32));
                    bi = (uint32_t)(kk & 0xFFFFFFFFu);
                    const int xl = w.ix, xh = min(w.ix + 1, w.W), yl = w.iy,
                              yh = min(w.iy + 1, w.H);
                    float sx, sy, se;
                    cell_exits(w, xl, xh, yl, yh, sx, sy, se);
                    w.px_prev = w.ix;
                    w.py_prev = w.iy;
                    w.s_hi = fminf(w.s_hi, bt);
                    over = !walk_advance(w, sx, sy, se, xl, xh, yl, yh);
                }
            }
        }
        if (over) {
            active = false;
            // a walk keeps only strictly better hits than the one it started from, and one
            // disk always gives one t, so a changed index is an improvement
            if (bi != known_i)
                atomicMin((unsigned long long*)&hitkey[e], (unsigned long long)pack_hit(bt, bi));
        }
    }
}

void launch_march(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live, RayState rs,
                  uint64_t* hitkey, int bounce, int max_views, uint32_t* cap_hits, uint32_t* queue,
                  int n_blocks, hipStream_t st) {
    launch_fill_u32(queue, 0u, kNumXcd, st);
    hipLaunchKernelGGL(k_march, dim3(n_blocks), dim3(256), 0, st, d, list, n_live, rs, hitkey,
                       bounce, max_views, cap_hits, queue);
}

// One bounce, pass 2: apply each ray's nearest hit (or stop it), reset its key for the next
// bounce when reset_keys (the views' march min-updates keys; the splat traversal writes every
// key itself), and count the survivors of each 64-entry chunk for the order-preserving
// compaction.
__global__ __launch_bounds__(256) void k_bounce_apply(const SlotDesc* __restrict__ ds,
                                                      const uint32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ n_live,
                                                      RayState rs, uint64_t* __restrict__ hitkey,
                                                      uint8_t* __restrict__ alive,
                                                      uint32_t* __restrict__ chunk_count,
                                                      int bounce, int reset_keys) {
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
            if (reset_keys) hitkey[e] = kEmptyKey;
            // a ray without a hit stops: its state is not read (most second-bounce rays)
            if (bounce <= d.max_b && (uint32_t)(key & 0xFFFFFFFFu) != kNone) {
                const uint64_t g = d.pix_base + entry_pix(entry);
                const f3 x = ld3(rs, RX, g), nn = ld3(rs, RNX, g);
                const f3 kin = bounce == 2 ? primary_dir(d) : ld3(rs, RKX, g);
                const f3 k = leave_dir(kin, nn);
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
                         int bounce, int reset_keys, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_bounce_apply, dim3(n_blocks), dim3(256), 0, st, d, list, n_live, rs,
                       hitkey, alive, chunk_count, bounce, reset_keys);
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
            if (disk_test(gld(d.pa + i), gld(d.pb + i), x, ks, d.eps, t)) return false;
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
                                                 int n_seg, uint32_t* cap_hits, int splats,
                                                 const uint8_t* __restrict__ vis_splats,
                                                 uint64_t vis_stride) {
    const uint32_t n = *n_list;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const uint32_t entry = list[e];
        const SlotDesc& d = ds[entry_slot(entry)];
        const uint64_t g = d.pix_base + entry_pix(entry);
        const f3 x = ld3(rs, RX, g), nn = ld3(rs, RNX, g);
        const double dd = rs.d[g];
        const int m = rs.m[g];
        f3 kin, Et, Ep, u, v;
        if (m == 1) {
            kin = primary_dir(d);
            primary_fields(d, Et, Ep, u, v);
        } else {
            kin = ld3(rs, RKX, g);
            Et = ld3(rs, RETX, g);
            Ep = ld3(rs, REPX, g);
            u = ld3(rs, RUX, g);
            v = ld3(rs, RVX, g);
        }
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
            if (splats) {
                // every splat can hide the facet (traced by the visibility pass); a monostatic
                // first-bounce facet is the nearest hit along its own reversed ray: visible
                if (!d.mono || m >= 2) vis = vis_splats[(uint64_t)o * vis_stride + g] != 0;
            } else if (d.mono) {
                if (m >= 2) vis = visible_primary(d, keys, x, ks);
            } else {
                vis = visible_views(d, x, ks, cap_hits);
            }
            const float w = vis ? area : 0.f;
            const f3 q = kin - ks;
            const f3 Vt = cross(cross(jt, ks), ks), Vp = cross(cross(jp, ks), ks);
            const f3 rt = mk3(O.eth[0], O.eth[1], O.eth[2]), rp = mk3(O.eph[0], O.eph[1], O.eph[2]);
            const uint64_t r = ((uint64_t)o * n_seg + seg) * rec_stride + e;
            const double D = dd - ((double)ks.x * x.x + (double)ks.y * x.y + (double)ks.z * x.z);
            const uint64_t Db = (uint64_t)__double_as_longlong(D);
            uint4* out = reinterpret_cast<uint4*>(er.rec + r);
            out[0] = make_uint4((uint32_t)Db, (uint32_t)(Db >> 32),
                                __float_as_uint(0.5f * dot(q, up)), __float_as_uint(0.5f * dot(q, vp)));
            out[1] = make_uint4(__float_as_uint(w * dot(Vt, rt)), __float_as_uint(w * dot(Vp, rt)),
                                __float_as_uint(w * dot(Vt, rp)), __float_as_uint(w * dot(Vp, rp)));
        }
    }
}

void launch_po_prep(const SlotDesc* d, const ObsDesc* obs, const uint32_t* list,
                    const uint32_t* n_list, RayState rs, const uint64_t* keys, ExitRecs er,
                    uint32_t rec_stride, int seg, int n_seg, uint32_t* cap_hits, int splats,
                    const uint8_t* vis, uint64_t vis_stride, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_po_prep, dim3(n_blocks), dim3(256), 0, st, d, obs, list, n_list, rs,
                       keys, er, rec_stride, seg, n_seg, cap_hits, splats, vis, vis_stride);
}

}  // namespace pe
