// Host runtime of the SBR library: contexts with an HBM budget, resident scenes, the batched
// solve pipeline and the C ABI declared in include/pointemray.h.
//
// A solve is cut into batches of incidences ("slots"); every kernel of the pipeline processes all
// slots of a batch in one launch (2-D grids over slot x work for host-known extents, persistent
// grids over device-side lists otherwise).  Slots are independent, so a result does not depend
// on which other slots share its batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pe_bvh.h"
#include "pe_device.h"
#include "pe_gfb.h"
#include "pe_runtime.h"
#include "pointemray.h"

using namespace pe;

namespace pe {

thread_local std::string g_err;

pe_status set_error(pe_status s, const std::string& m) {
    g_err = m;
    return s;
}

void hip_check(hipError_t e, const char* what, int line) {
    if (e != hipSuccess) {
        char buf[512];
        snprintf(buf, sizeof buf, "HIP error %d (%s) in %s (runtime.cpp:%d)", (int)e,
                 hipGetErrorString(e), what, line);
        throw Error{PE_EDEVICE, buf};
    }
}

// ------------------------------------------------------------------------------------------
// Budgeted device memory
// ------------------------------------------------------------------------------------------

// Largest total of released blocks a context keeps for reuse.
constexpr uint64_t kCacheCap = 32ull << 30;

// Returns every cached block to HIP (after the device has finished with them).
void ctx_release_cache(pe_ctx ctx) {
    std::lock_guard<std::mutex> lk(ctx->alloc_mu);
    if (ctx->cache.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->cache) (void)hipFree(kv.second.p);
    ctx->cache.clear();
    ctx->cached = 0;
    ctx->idle_gen++;
}

// Drops cached blocks, largest first, until used + cached <= limit.  Caller holds alloc_mu.
static void trim_cache_locked(pe_ctx ctx, uint64_t limit) {
    while (!ctx->cache.empty() && ctx->used.load() + ctx->cached > limit) {
        auto it = std::prev(ctx->cache.end());
        (void)hipFree(it->second.p);
        ctx->cached -= it->first;
        ctx->cache.erase(it);
    }
}

void* ctx_alloc(pe_ctx ctx, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    uint64_t cur = ctx->used.load();
    do {
        if (cur + bytes > ctx->budget)
            throw Error{PE_ENOMEM, "HBM budget exceeded: need " + std::to_string(bytes) +
                                       " more bytes, " + std::to_string(ctx->budget - cur) +
                                       " left"};
    } while (!ctx->used.compare_exchange_weak(cur, cur + bytes));
    {
        std::lock_guard<std::mutex> lk(ctx->alloc_mu);
        auto it = ctx->cache.find(bytes);
        if (it != ctx->cache.end()) {
            if (it->second.gen >= ctx->idle_gen) {
                (void)hipDeviceSynchronize();
                ctx->idle_gen++;
            }
            void* p = it->second.p;
            ctx->cached -= bytes;
            ctx->cache.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        // the device may be short only because of cached blocks: return them and retry once
        (void)hipGetLastError();
        ctx_release_cache(ctx);
        e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) {
        ctx->used -= bytes;
        (void)hipGetLastError();
        throw Error{PE_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    }
    {
        std::lock_guard<std::mutex> lk(ctx->alloc_mu);
        trim_cache_locked(ctx, ctx->budget);
    }
    return p;
}

void ctx_free(pe_ctx ctx, void* p, size_t bytes) {
    if (!p) return;
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    ctx->used -= bytes;
    std::lock_guard<std::mutex> lk(ctx->alloc_mu);
    if (ctx->cached + bytes > kCacheCap || ctx->used.load() + ctx->cached + bytes > ctx->budget) {
        (void)hipFree(p);
        return;
    }
    ctx->cache.insert({bytes, pe_ctx_s::CachedBlock{p, ctx->idle_gen}});
    ctx->cached += bytes;
}

void* Workspace::raw(int id, size_t bytes) {
    Buf& b = bufs[id];
    if (bytes == 0) bytes = 16;
    if (arena) {
        if (b.cap >= bytes) return b.p;
        const size_t want = (bytes + 255) & ~(size_t)255;
        if (want > arena_cap - arena_used)
            throw Error{PE_ENOMEM, "solve needs more than the fixed scratch of " +
                                       std::to_string(arena_cap) + " bytes (" +
                                       std::to_string(arena_used + want) + " requested)"};
        b.p = arena + arena_used;
        b.cap = want;
        arena_used += want;
        return b.p;
    }
    if (b.cap < bytes) {
        if (b.p) ctx_free(ctx, b.p, b.cap);
        b.p = nullptr;
        b.cap = 0;
        size_t want = bytes + bytes / 8;
        want = (want + 255) & ~(size_t)255;
        b.p = ctx_alloc(ctx, want);
        b.cap = want;
    }
    return b.p;
}

void Workspace::release() {
    for (auto& b : bufs) {
        if (b.p && !arena) ctx_free(ctx, b.p, b.cap);
        b.p = nullptr;
        b.cap = 0;
    }
    arena_used = 0;
}

void Workspace::begin_batch() {
    if (arena) release();
}

uint64_t Workspace::bytes() const {
    uint64_t s = 0;
    for (const auto& b : bufs) s += b.cap;
    return s;
}

// ------------------------------------------------------------------------------------------
// Geometry helpers (host, fp64)
// ------------------------------------------------------------------------------------------

static void normalize3(double v[3]) {
    const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= l;
    v[1] /= l;
    v[2] /= l;
}

static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Screen basis of a propagation direction: u = normalise(z x k) (x when k is within 1e-9 of
// +-z), v = k x u; the screen is 2R wide, centred on the scene, R before the centre along k.
void screen_basis(const double kin[3], double u[3], double v[3], double k[3]) {
    k[0] = kin[0];
    k[1] = kin[1];
    k[2] = kin[2];
    normalize3(k);
    if (std::fabs(k[2]) > 1.0 - 1e-9) {
        u[0] = 1;
        u[1] = 0;
        u[2] = 0;
    } else {
        const double z[3] = {0, 0, 1};
        cross3(z, k, u);
        normalize3(u);
    }
    cross3(k, u, v);
}

// theta-hat and phi-hat of the spherical angles of direction s.
void pol_basis(const double s_in[3], double th[3], double ph[3]) {
    double s[3] = {s_in[0], s_in[1], s_in[2]};
    normalize3(s);
    const double theta = std::acos(std::max(-1.0, std::min(1.0, s[2])));
    const double phi = std::atan2(s[1], s[0]);
    th[0] = std::cos(theta) * std::cos(phi);
    th[1] = std::cos(theta) * std::sin(phi);
    th[2] = -std::sin(theta);
    ph[0] = -std::sin(phi);
    ph[1] = std::cos(phi);
    ph[2] = 0;
}

// ------------------------------------------------------------------------------------------
// Batch pipeline
// ------------------------------------------------------------------------------------------

enum BufId {
    B_SLOTS, B_OBS, B_FREQ, B_AABB, B_TCOUNT, B_TCURSOR, B_TOFF, B_TLIST, B_KEYS, B_RSF,
    B_RSD, B_RSM, B_RSH, B_LIST0, B_LIST1, B_LIST2, B_ALIVE, B_CCOUNT, B_COFF, B_WGC, B_WGO,
    B_RECD, B_RECF, B_SEGB, B_SEGC, B_TPRE, B_TTMP, B_PART, B_EOUT, B_ROUT, B_CNT, B_HITKEY,
    B_MQUEUE, B_SCAN, B_NUMBUF
};
static_assert(B_NUMBUF <= 34, "workspace ids 34..39 belong to the densified solve");
constexpr int B_PSILIST = 40, B_VIS = 41;  // monostatic visibility pass (secondary = splats)

enum Counter : int {
    C_TILES = 0, C_OVERFLOW, C_N0, C_N1, C_N2, C_WORK, C_CAP, C_BOUNCE0, C_NCOUNT = C_BOUNCE0 + 64
};
constexpr int C_PSI = C_BOUNCE0 + 63;  // facets of the monostatic visibility pass

static int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

Batch::Batch(Workspace& w, hipStream_t s) : ws(w), st(s) {}

void Batch::setup(const std::vector<SlotSpec>& slots, int contrib_, int precision_) {
    spec = slots;
    n = (int)slots.size();
    if (n < 1 || n > kMaxSlots) throw Error{PE_EINVAL, "batch must hold 1..1024 slots"};
    contrib = contrib_;
    precision = precision_;
    hd.assign(n, SlotDesc{});
    blend = false;
    ho.clear();
    hf.clear();
    max_chunks = max_tiles = max_pix = 0;
    tot_pix = 0;
    tot_tiles = tot_chunks = 0;
    max_obs = max_freq = 1;
    tot_out = 0;
    max_b = 1;
    max_views = 0;
    bvh_depth = 1;
    for (int i = 0; i < n; i++) {
        const SlotSpec& sp = slots[i];
        const pe_scene sc = sp.sc;
        SlotDesc& d = hd[i];
        if ((uint64_t)sp.W * sp.H > (1u << kPixBits) || sp.W < 1 || sp.H < 1)
            throw Error{PE_EINVAL, "screen must hold 1 .. 2^22 pixels"};
        d.pa_s = sc->pa_s;
        d.pb_s = sc->pb_s;
        d.cbox = sc->cbox;
        d.pa = sc->pa;
        d.pb = sc->pb;
        d.blend_r = sc->blend_r;
        d.bl_h = sc->bl_h;
        d.bl_G = sc->bl_G;
        d.bl_start = sc->bl_start;
        d.bl_items = sc->bl_items;
        d.bvh = sc->bvh;
        d.wrec = sc->wrec;
        d.wpts = sc->wpts;
        d.w_root_pts = sc->w_root_pts;
        for (int a = 0; a < 3; a++) {
            d.bvh_lo[a] = sc->bvh_root[a];
            d.bvh_hi[a] = sc->bvh_root[3 + a];
        }
        bvh_depth = std::max(bvh_depth, sc->bvh_levels);
        if (sc->blend_r > 0.f) blend = true;
        d.views = sc->views_dev;
        d.n_views = (int)sc->views.size();
        max_views = std::max(max_views, d.n_views);
        d.n_pts = (uint32_t)sc->n;
        d.n_chunks = (uint32_t)((sc->n + kChunk - 1) / kChunk);
        d.R = (float)sc->R;
        d.r_max = (float)sc->r_max;
        double u[3], v[3], k[3];
        screen_basis(sp.k, u, v, k);
        for (int a = 0; a < 3; a++) {
            d.u[a] = (float)u[a];
            d.v[a] = (float)v[a];
            d.k[a] = (float)k[a];
        }
        d.pitch = (float)(2.0 * sc->R / std::max(sp.W, sp.H));
        d.W = sp.W;
        d.H = sp.H;
        // the K-point heap keeps one pixel per thread (16 x 16 tiles); the nearest-hit raster
        // takes 32 x 32 tiles, so each chunk of points overlaps fewer tiles
        d.tile = topk > 0 ? kTile : kTileWide;
        d.tiles_x = (sp.W + d.tile - 1) / d.tile;
        d.tiles_y = (sp.H + d.tile - 1) / d.tile;
        d.mode = sp.mode;
        d.tube_r = (float)sp.tube_r;
        d.pix_base = tot_pix;
        d.tile_base = tot_tiles;
        d.chunk_base = tot_chunks;
        tot_pix += (uint64_t)sp.W * sp.H;
        tot_tiles += (uint32_t)(d.tiles_x * d.tiles_y);
        tot_chunks += d.n_chunks;
        max_chunks = std::max(max_chunks, (int)d.n_chunks);
        max_tiles = std::max(max_tiles, d.tiles_x * d.tiles_y);
        max_pix = std::max(max_pix, sp.W * sp.H);
        double src[3] = {-k[0], -k[1], -k[2]}, th[3], ph[3];
        pol_basis(src, th, ph);
        for (int a = 0; a < 3; a++) {
            d.eth[a] = (float)th[a];
            d.eph[a] = (float)ph[a];
        }
        d.eps = (float)sp.eps;
        d.max_b = sp.max_b;
        max_b = std::max(max_b, sp.max_b);
        d.mono = sp.obs == nullptr;
        d.n_obs = d.mono ? 1 : sp.n_obs;
        d.obs_base = (int)ho.size();
        for (int o = 0; o < d.n_obs; o++) {
            ObsDesc O{};
            double ks[3];
            if (d.mono) {
                ks[0] = -k[0]; ks[1] = -k[1]; ks[2] = -k[2];
            } else {
                ks[0] = sp.obs[3 * o]; ks[1] = sp.obs[3 * o + 1]; ks[2] = sp.obs[3 * o + 2];
                normalize3(ks);
            }
            double rt[3], rp[3];
            pol_basis(ks, rt, rp);
            for (int a = 0; a < 3; a++) {
                O.ks[a] = (float)ks[a];
                O.eth[a] = (float)rt[a];
                O.eph[a] = (float)rp[a];
            }
            O.dc = (k[0] - ks[0]) * sc->c[0] + (k[1] - ks[1]) * sc->c[1] + (k[2] - ks[2]) * sc->c[2];
            ho.push_back(O);
        }
        d.n_freq = sp.n_freq;
        d.freq_base = (int)hf.size();
        for (int f = 0; f < sp.n_freq; f++) hf.push_back(sp.freq ? sp.freq[f] : 1.0);
        d.out_base = tot_out;
        tot_out += d.n_obs * d.n_freq;
        max_obs = std::max(max_obs, d.n_obs);
        max_freq = std::max(max_freq, d.n_freq);
    }
    if (tot_pix >= 0xFFFFFFF0ull) throw Error{PE_EINVAL, "batch too large"};
    n_seg = contrib == PE_CONTRIB_EVERY ? max_b : 1;
    ft = std::min(64, pow2_at_least(max_freq));
    dd = ws.get<SlotDesc>(B_SLOTS, n);
    dobs = ws.get<ObsDesc>(B_OBS, ho.size());
    dfreq = ws.get<double>(B_FREQ, hf.size());
    cnt = ws.get<uint32_t>(B_CNT, C_NCOUNT);
    scan_ws = ws.get<uint32_t>(B_SCAN, scan_wide_scratch(0xFFFFFFFFu));  // 1 MiB, any scan size
    HIPCHK(hipMemcpyAsync(dd, hd.data(), sizeof(SlotDesc) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dobs, ho.data(), sizeof(ObsDesc) * ho.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dfreq, hf.data(), sizeof(double) * hf.size(), hipMemcpyHostToDevice, st));
    launch_fill_u32(cnt, 0u, C_NCOUNT, st);
}

void Batch::splat() {
    if (tlist_cap == 0) tlist_cap = (uint32_t)std::min<uint64_t>(0xFFFFFF00ull, (uint64_t)tot_chunks * 4 + tot_tiles + 1024);
    int4* aabb = ws.get<int4>(B_AABB, tot_chunks);
    uint32_t* tcount = ws.get<uint32_t>(B_TCOUNT, tot_tiles);
    uint32_t* tcursor = ws.get<uint32_t>(B_TCURSOR, tot_tiles);
    uint32_t* toff = ws.get<uint32_t>(B_TOFF, tot_tiles + 1);
    uint32_t* tlist = ws.get<uint32_t>(B_TLIST, tlist_cap);
    keys = ws.get<uint64_t>(B_KEYS, tot_pix);
    launch_fill_u32(tcount, 0u, tot_tiles, st);
    launch_fill_u32(tcursor, 0u, tot_tiles, st);
    prof_begin();
    launch_chunk_bounds(dd, n, max_chunks, aabb, tcount, st);
    prof_end("chunk_bounds");
    prof_begin();
    launch_scan_wide(tcount, toff, tot_tiles, nullptr, 1, cnt + C_TILES,
                     scan_ws, st);
    prof_end("tile_scan");
    prof_begin();
    launch_tile_scatter(dd, n, max_chunks, aabb, toff, tcursor, tlist, tlist_cap,
                        cnt + C_OVERFLOW, st);
    prof_end("tile_scatter");
    // the nearest-hit raster also counts, per 256-pixel block, the pixels that start rays (the
    // ray generation's count) when every slot's tile rows lie in single blocks
    live_counted = topk == 0;
    for (int s = 0; s < n && live_counted; s++) live_counted = hd[s].W % hd[0].tile == 0;
    const int gx = (max_pix + 255) / 256;
    uint32_t* wgc = nullptr;
    if (live_counted) {
        wgc = ws.get<uint32_t>(B_WGC, (uint64_t)gx * n + 1);
        launch_fill_u32(wgc, 0u, (uint64_t)gx * n, st);
    }
    prof_begin();
    if (topk > 0)
        launch_raster_topk(dd, n, max_tiles, toff, tcount, tlist, tlist_cap, topk, keys, st);
    else
        launch_raster(dd, n, max_tiles, toff, tcount, tlist, tlist_cap, keys, hd[0].tile, wgc,
                      (uint32_t)gx, st);
    prof_end("raster");
    HIPCHK(hipGetLastError());
}

void Batch::alloc_rays() {
    float* f = ws.get<float>(B_RSF, tot_pix * RNCOMP);
    for (int c = 0; c < RNCOMP; c++) rs.f[c] = f + (uint64_t)c * tot_pix;
    rs.d = ws.get<double>(B_RSD, tot_pix);
    rs.m = ws.get<uint8_t>(B_RSM, tot_pix);
    rs.hit = ws.get<uint32_t>(B_RSH, tot_pix);
    lists[0] = ws.get<uint32_t>(B_LIST0, tot_pix);
    lists[1] = ws.get<uint32_t>(B_LIST1, tot_pix);
    lists[2] = ws.get<uint32_t>(B_LIST2, tot_pix);
    alive = ws.get<uint8_t>(B_ALIVE, tot_pix);
    hitkey = ws.get<uint64_t>(B_HITKEY, tot_pix);
    ccount = ws.get<uint32_t>(B_CCOUNT, tot_pix / kWaveChunk + 2);
    coff = ws.get<uint32_t>(B_COFF, tot_pix / kWaveChunk + 2);
}

// Workgroups of the persistent passes (traversal, apply, compaction, facet records); the
// traversal holds 6 wavefronts per SIMD, 1536 workgroups of 4 on 256 CUs.  Measured on the
// composite bench (ms per step): 1024 70.3, 1536 67.1, 2048 66.0, 3072 66.8, 4096 66.2.
// PE_PERSIST_BLOCKS overrides.
static int persistent_blocks() {
    static const int v = [] {
        const char* e = std::getenv("PE_PERSIST_BLOCKS");
        return e ? std::max(1, std::atoi(e)) : 2048;
    }();
    return v;
}

// Idle lanes at which a traversal wavefront takes new rays (bits 0-7) and the quorum of lanes
// holding points at which it runs a point step for the whole wavefront (bits 8-15, 0 = each
// lane its own kind of step).  Measured on the composite bench (ms per step, second bounce /
// visibility), refill alone at 8: 83.4 / 13.8, 16: 46.0 / 8.5, 24: 32.0 / 7.0, 32: 26.1 / 7.2,
// 40: 25.8 / 7.6, 48: 25.8 / 7.7, 64: 32.1 / 10.0; with refill 40, quorum 8: 22.9 / 6.6,
// 12: 22.4 / 7.0, 16: 22.7 / 7.1.  Visibility alone, later (ms per step): refill 24 6.85, 40
// 7.10; refill 40 with quorum 8 6.63, 10 6.75, 12 6.80; refill 24 with quorum 8 6.75.  Once
// node steps took fewer instructions (near and far planes picked per record), the second
// bounce at quorum 12 moved to refill 32: 25.4, 40: 21.4-21.5, 44: 20.4, 48: 20.1-20.2, 52:
// 20.9, 56: 23.8 ms (48 with quorum 8: 20.4, 16: 21.0); visibility at refill 32, 40 and 48:
// 5.9-6.1 ms.  With every child slot tested in nearest-hit: second bounce at refill 48 and
// quorum 10 20.1, 12 19.9-20.1, 14 20.3 ms; visibility at refill 24 6.41, 32 5.92-5.98, 40
// 5.93-6.10 ms (quorum 8).  PE_BVH_REFILL, PE_BVH_QUORUM, PE_PSI_REFILL and PE_PSI_QUORUM
// override.
static int bvh_refill(bool psi) {
    auto env = [](const char* name, int dflt) {
        const char* e = std::getenv(name);
        return e ? std::atoi(e) : dflt;
    };
    static const int v[2] = {env("PE_BVH_REFILL", 48) | (env("PE_BVH_QUORUM", 12) << 8),
                             env("PE_PSI_REFILL", 40) | (env("PE_PSI_QUORUM", 8) << 8)};
    return v[psi ? 1 : 0];
}

void Batch::raygen() {
    alloc_rays();
    const int gx = (max_pix + 255) / 256;
    uint32_t* wgc = ws.get<uint32_t>(B_WGC, (uint64_t)gx * n + 1);
    uint32_t* wgo = ws.get<uint32_t>(B_WGO, (uint64_t)gx * n + 1);
    if (!live_counted) {
        prof_begin();
        launch_raygen_count(dd, n, max_pix, keys, wgc, st);
        prof_end("raygen_count");
    }
    prof_begin();
    launch_scan_wide(wgc, wgo, (uint32_t)(gx * n), nullptr, 1, cnt + C_N0,
                     scan_ws, st);
    prof_end("raygen_scan");
    prof_begin();
    // the splat traversal writes every ray's key; the views' march needs them cleared
    launch_raygen_write(dd, n, max_pix, keys, wgo, lists[0], rs,
                        secondary == PE_SECONDARY_SPLATS ? nullptr : hitkey, st);
    prof_end("raygen_write");
    if (blend) {
        prof_begin();
        launch_blend(dd, lists[0], cnt + C_N0, rs, 1, persistent_blocks(), st);
        prof_end("blend");
    }
    HIPCHK(hipGetLastError());
}

void Batch::raygen_gfb(const float* depth, const float* nrm, const float* prob,
                       const uint8_t* use, float thresh) {
    alloc_rays();
    const int gx = (max_pix + 255) / 256;
    uint32_t* wgc = ws.get<uint32_t>(B_WGC, (uint64_t)gx * n + 1);
    uint32_t* wgo = ws.get<uint32_t>(B_WGO, (uint64_t)gx * n + 1);
    prof_begin();
    launch_gfb_raygen(dd, n, max_pix, depth, nrm, prob, use, thresh, wgc, wgo, lists[0], rs,
                      hitkey, cnt + C_N0, scan_ws, st);
    prof_end("gfb_raygen");
    HIPCHK(hipGetLastError());
}

void Batch::alloc_records() {
    rec_stride = (uint32_t)tot_pix;
    const uint64_t nrec = (uint64_t)max_obs * n_seg * rec_stride;
    er.rec = ws.get<ExitRec>(B_RECD, nrec);
    seg_beg = ws.get<uint32_t>(B_SEGB, (uint64_t)n_seg * n + 1);
    seg_cnt = ws.get<uint32_t>(B_SEGC, (uint64_t)n_seg * n + 1);
}

void Batch::records(int seg, const uint32_t* list, const uint32_t* n_list) {
    const bool splats = secondary == PE_SECONDARY_SPLATS;
    uint8_t* vis = nullptr;
    if (splats) {
        // dense any-hit pass over the facets that need a traced Psi (monostatic first bounces
        // are visible and are most facets, so tracing inside po_prep would idle most lanes)
        uint32_t* plist = ws.get<uint32_t>(B_PSILIST, tot_pix);
        vis = ws.get<uint8_t>(B_VIS, (uint64_t)max_obs * tot_pix);
        const uint32_t max_chunks = (uint32_t)((tot_pix + kWaveChunk - 1) / kWaveChunk);
        prof_begin();
        launch_psi_mark(dd, list, n_list, rs, alive, ccount, persistent_blocks(), st);
        launch_scan_wide(ccount, coff, max_chunks, n_list, kWaveChunk, cnt + C_PSI, scan_ws, st);
        launch_compact(list, n_list, alive, coff, plist, persistent_blocks(), st);
        prof_end("psi_compact");
        prof_begin();
        launch_psi_trace(dd, dobs, plist, cnt + C_PSI, max_obs, rs, vis, tot_pix, bvh_depth,
                         ws.get<uint32_t>(B_MQUEUE, kNumXcd), bvh_refill(true), persistent_blocks(),
                         st);
        prof_end("psi_bvh");
    }
    prof_begin();
    launch_po_prep(dd, dobs, list, n_list, rs, keys, er, rec_stride, seg, n_seg, cnt + C_CAP,
                   splats, vis, tot_pix, persistent_blocks(), st);
    prof_end("po_prep");
    prof_begin();
    launch_slot_ranges(list, n_list, n, seg_beg + (uint64_t)seg * n, seg_cnt + (uint64_t)seg * n,
                       st);
    prof_end("slot_ranges");
}

// Bounces 2..max_b.  For LAST the first-hit list is kept intact: every ray's state ends as its
// last record, so the radiating set is exactly the first-hit list.
void Batch::trace(bool with_records) {
    if (with_records) alloc_records();
    if (with_records && contrib == PE_CONTRIB_EVERY) records(0, lists[0], cnt + C_N0);
    const uint32_t* cur = lists[0];
    const uint32_t* ncur = cnt + C_N0;
    for (int b = 2; b <= max_b; b++) {
        uint32_t* out = lists[b % 2 == 0 ? 1 : 2];
        uint32_t* nout = cnt + (b % 2 == 0 ? C_N1 : C_N2);
        prof_begin();
        if (secondary == PE_SECONDARY_SPLATS) {
            launch_trace_bvh(dd, cur, ncur, rs, hitkey, b, bvh_depth,
                             ws.get<uint32_t>(B_MQUEUE, kNumXcd), bvh_refill(false),
                             persistent_blocks(),
                             st);
            static const char* names[] = {"bvh_b2", "bvh_b3", "bvh_b4", "bvh_b5", "bvh_b6",
                                          "bvh_b7", "bvh_b8", "bvh_b9+"};
            prof_end(names[std::min(b - 2, 7)]);
        } else {
            launch_march(dd, cur, ncur, rs, hitkey, b, max_views, cnt + C_CAP,
                         ws.get<uint32_t>(B_MQUEUE, kNumXcd), persistent_blocks(), st);
            static const char* names[] = {"march_b2", "march_b3", "march_b4", "march_b5",
                                          "march_b6", "march_b7", "march_b8", "march_b9+"};
            prof_end(names[std::min(b - 2, 7)]);
        }
        prof_begin();
        launch_bounce_apply(dd, cur, ncur, rs, hitkey, alive, ccount, b,
                            secondary != PE_SECONDARY_SPLATS, persistent_blocks(), st);
        prof_end("bounce_apply");
        prof_begin();
        const uint32_t max_chunks = (uint32_t)((tot_pix + kWaveChunk - 1) / kWaveChunk);
        launch_scan_wide(ccount, coff, max_chunks, ncur, kWaveChunk, nout,
                         scan_ws, st);
        prof_end("compact_scan");
        prof_begin();
        launch_compact(cur, ncur, alive, coff, out, persistent_blocks(), st);
        prof_end("compact");
        if (blend) {
            prof_begin();
            launch_blend(dd, out, nout, rs, 0, persistent_blocks(), st);
            prof_end("blend");
        }
        HIPCHK(hipMemcpyAsync(cnt + C_BOUNCE0 + b, ncur, sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(cnt + C_BOUNCE0 + 32 + b, nout, sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
        if (with_records && contrib == PE_CONTRIB_EVERY) records(b - 1, out, nout);
        cur = out;
        ncur = nout;
        HIPCHK(hipGetLastError());
    }
    if (with_records && contrib != PE_CONTRIB_EVERY) records(0, lists[0], cnt + C_N0);
}

void Batch::field(double* E_host, double* rcs_host) {
    uint32_t* tpre = ws.get<uint32_t>(B_TPRE, (uint64_t)n_seg * n + 1);
    uint32_t* ttmp = ws.get<uint32_t>(B_TTMP, (uint64_t)n_seg * n + 1);
    const uint64_t nft = (uint64_t)(max_freq + ft - 1) / ft;
    const uint64_t max_tiles_po = (uint64_t)n_seg * (tot_pix / kRT + n + 1) * max_obs * nft;
    double* part = ws.get<double>(B_PART, max_tiles_po * ft * 8);
    double* Eo = ws.get<double>(B_EOUT, (uint64_t)tot_out * 8);
    double* Ro = ws.get<double>(B_ROUT, (uint64_t)tot_out * 4);
    prof_begin();
    launch_po_tiles(dd, seg_cnt, n_seg, n, ft, ttmp, tpre, st);
    prof_end("po_tiles");
    prof_begin();
    // PO accumulation mode of k_po_sum / k_po_reduce: 0 fp64 phase with fp32 groups of four,
    // 1 all fp32, 2 fp64 phase with every term accumulated in fp64
    const int po_mode = precision == PE_PREC_FP32 ? 1 : precision == PE_PREC_FP64ACC ? 2 : 0;
    launch_po_sum(dd, seg_beg, seg_cnt, n_seg, n, dfreq, er, rec_stride, tpre,
                  po_mode, ft, part, persistent_blocks(), st);
    prof_end("po_sum");
    prof_begin();
    launch_po_reduce(dd, dobs, n, max_obs, max_freq, n_seg, dfreq, seg_cnt, tpre, ft, part,
                     po_mode, Eo, Ro, st);
    prof_end("po_reduce");
    HIPCHK(hipGetLastError());
    if (E_host) HIPCHK(hipMemcpyAsync(E_host, Eo, sizeof(double) * 8 * tot_out, hipMemcpyDeviceToHost, st));
    if (rcs_host) HIPCHK(hipMemcpyAsync(rcs_host, Ro, sizeof(double) * 4 * tot_out, hipMemcpyDeviceToHost, st));
}

void Batch::read_counters(uint32_t* host) {
    HIPCHK(hipMemcpyAsync(host, cnt, sizeof(uint32_t) * C_NCOUNT, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    prof_flush();
}

// Per-kernel HIP-event timers on the launch stream (enabled per context).
void Batch::prof_begin() {
    if (!ws.ctx->profile || ws.arena) return;  // the no-allocation path records no events
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(e, st));
    pend_begin = e;
}

void Batch::prof_end(const char* name) {
    if (!ws.ctx->profile || ws.arena) return;
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(e, st));
    pend.push_back({name, pend_begin, e});
}

void Batch::prof_flush() {
    if (pend.empty()) return;
    std::lock_guard<std::mutex> lk(ws.ctx->prof_mu);
    for (auto& p : pend) {
        float ms = 0;
        HIPCHK(hipEventSynchronize(p.e1));
        HIPCHK(hipEventElapsedTime(&ms, p.e0, p.e1));
        auto& slot = ws.ctx->ktab[p.name];
        slot.first += ms;
        slot.second += 1;
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    pend.clear();
}

double Batch::queries(const uint32_t* c) const {
    double q = (double)tot_pix;
    for (int b = 2; b <= max_b; b++) q += c[C_BOUNCE0 + b];
    return q;
}

double Batch::march_rays(const uint32_t* c) const {
    double r = 0;
    for (int b = 2; b <= max_b; b++) r += c[C_BOUNCE0 + b];
    return r;
}

double Batch::march_hits(const uint32_t* c) const {
    double r = 0;
    for (int b = 2; b <= max_b; b++) r += c[C_BOUNCE0 + 32 + b];
    return r;
}

double Batch::records_made(const uint32_t* c) const {
    double r = c[C_N0];
    if (contrib == PE_CONTRIB_EVERY)
        for (int b = 2; b <= max_b; b++) r += c[C_BOUNCE0 + 32 + b];
    return r;
}

bool Batch::overflowed(const uint32_t* c) {
    if (c[C_OVERFLOW] == 0) return false;
    tlist_cap = (uint32_t)std::min<uint64_t>(0xFFFFFF00ull, (uint64_t)c[C_TILES] + c[C_TILES] / 4 + 1024);
    return true;
}

}  // namespace pe
