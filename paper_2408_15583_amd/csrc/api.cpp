// C ABI entry points of the SBR library (include/pointemray.h): contexts, scenes, synchronous
// solves and the inspection hooks.  No C++ exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pe_bvh.h"
#include "pe_device.h"
#include "pe_runtime.h"
#include "pointemray.h"

using namespace pe;



namespace pe {

void scene_release_server(pe_ctx ctx);  // server.cpp
void server_shutdown(pe_ctx ctx);       // server.cpp

static bool finite3(const double* v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]) &&
           (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) > 0;
}

// Shared by pe_solve and pe_submit.
void validate_solve(pe_scene sc, const pe_solve_desc* d, bool need_scene) {
    if ((need_scene && !sc) || !d) throw Error{PE_EINVAL, "null scene or descriptor"};
    if (d->n_inc < 1 || !d->inc_dir) throw Error{PE_EINVAL, "need n_inc >= 1 incidence directions"};
    for (int i = 0; i < d->n_inc; i++)
        if (!finite3(d->inc_dir + 3 * i)) throw Error{PE_EINVAL, "non-finite or zero incidence direction"};
    if (d->obs_dir) {
        if (d->n_obs < 1) throw Error{PE_EINVAL, "n_obs must be >= 1 with obs_dir"};
        for (int i = 0; i < d->n_obs; i++)
            if (!finite3(d->obs_dir + 3 * i)) throw Error{PE_EINVAL, "non-finite or zero observation direction"};
    }
    if (d->n_freq < 1 || !d->freq_hz) throw Error{PE_EINVAL, "need n_freq >= 1 frequencies"};
    for (int f = 0; f < d->n_freq; f++)
        if (!(d->freq_hz[f] > 0) || !std::isfinite(d->freq_hz[f])) throw Error{PE_EINVAL, "frequencies must be finite and > 0"};
    if (d->screen_w < 1 || d->screen_h < 1 || (uint64_t)d->screen_w * d->screen_h > (1u << kPixBits))
        throw Error{PE_EINVAL, "screen must hold 1 .. 2^22 pixels"};
    if (d->max_bounces < 1 || d->max_bounces > kMaxBounces) throw Error{PE_EINVAL, "max_bounces must be 1..16"};
    if (!(d->eps >= 0) || !std::isfinite(d->eps)) throw Error{PE_EINVAL, "eps must be finite and >= 0"};
    if (d->contrib != PE_CONTRIB_LAST && d->contrib != PE_CONTRIB_EVERY) throw Error{PE_EINVAL, "bad contrib flag"};
    if (d->precision != PE_PREC_FP64PHASE && d->precision != PE_PREC_FP32 &&
        d->precision != PE_PREC_FP64ACC)
        throw Error{PE_EINVAL, "bad precision flag"};
    if (d->secondary != PE_SECONDARY_VIEWS && d->secondary != PE_SECONDARY_SPLATS)
        throw Error{PE_EINVAL, "bad secondary flag"};
    if (d->geometry != PE_GEOM_PLAIN && d->geometry != PE_GEOM_DENSIFIED && d->geometry != PE_GEOM_COARSE)
        throw Error{PE_EINVAL, "bad geometry flag"};
    if (d->geometry != PE_GEOM_PLAIN) {
        if (d->geometry == PE_GEOM_DENSIFIED && !d->densifier) throw Error{PE_EINVAL, "densified geometry needs a densifier"};
        if (d->max_bounces != 1) throw Error{PE_EUNSUPPORTED, "densified/coarse geometry supports max_bounces == 1"};
        if (d->screen_w != d->screen_h || d->screen_w % 16 != 0)
            throw Error{PE_EINVAL, "densified/coarse geometry needs a square screen, multiple of 16"};
        if (!(d->tube_px >= 0) || !std::isfinite(d->tube_px)) throw Error{PE_EINVAL, "tube_px must be finite and >= 0"};
        if (!(d->max_uncertain >= 0) || !(d->max_uncertain <= 1)) throw Error{PE_EINVAL, "max_uncertain must be in [0, 1]"};
        if (d->tube_k < 0 || d->tube_k > 1024) throw Error{PE_EINVAL, "tube_k must be 0..1024"};
    }
}

uint64_t batch_bytes_per_pixel(const pe_solve_desc* d) {
    const uint64_t n_obs = d->obs_dir ? d->n_obs : 1;
    const uint64_t seg = d->contrib == PE_CONTRIB_EVERY ? d->max_bounces : 1;
    // ray state, depth, bounce count, hit index, three lists, alive flag, hit key, first-hit key,
    // compaction counts, exit records; against every splat also the visibility pass's facet
    // list and its per-observation flags
    const uint64_t vis = d->secondary == PE_SECONDARY_SPLATS ? 4 + n_obs : 0;
    return RNCOMP * 4 + 8 + 1 + 4 + 12 + 1 + 8 + 8 + 8 + seg * n_obs * 40 + vis;
}

int slots_per_batch(pe_ctx ctx, const pe_solve_desc* d) {
    static const uint64_t env = [] {
        const char* e = std::getenv("PE_BATCH_PIXELS");
        return e ? std::strtoull(e, nullptr, 10) : (uint64_t)0;
    }();
    uint64_t target = env;
    if (target == 0) {
        // As many pixels as half of the HBM budget left to this call holds (the default
        // workspace's own buffers are reused), between 2^22 and 2^29: large batches keep the
        // later bounces' launches full and amortise each launch's drain.
        const uint64_t used = ctx->used.load(), held = ctx->ws->bytes();
        const uint64_t avail = (ctx->budget > used ? ctx->budget - used : 0) + held;
        target = avail / 2 / (batch_bytes_per_pixel(d) * 9 / 8);
        target = std::min<uint64_t>(std::max<uint64_t>(target, (uint64_t)1 << 22),
                                    (uint64_t)1 << 29);
    }
    const uint64_t px = (uint64_t)d->screen_w * d->screen_h;
    uint64_t s = std::max<uint64_t>(1, target / px);
    s = std::min<uint64_t>(s, (uint64_t)kMaxSlots);
    s = std::min<uint64_t>(s, (uint64_t)d->n_inc);
    return (int)s;
}

std::vector<SlotSpec> make_slots(pe_scene sc, const pe_solve_desc* d, int i0, int count) {
    std::vector<SlotSpec> v(count);
    for (int i = 0; i < count; i++) {
        SlotSpec& s = v[i];
        s.sc = sc;
        for (int a = 0; a < 3; a++) s.k[a] = d->inc_dir[3 * (i0 + i) + a];
        s.W = d->screen_w;
        s.H = d->screen_h;
        s.mode = PE_SPLAT_DISK;
        s.max_b = d->max_bounces;
        s.eps = d->eps;
        s.obs = d->obs_dir;
        s.n_obs = d->obs_dir ? d->n_obs : 1;
        s.n_freq = d->n_freq;
        s.freq = d->freq_hz;
    }
    return v;
}

// Runs one batch to completion (re-running with a larger tile list if it overflowed).
void run_field_batch(Workspace& ws, hipStream_t st, const std::vector<SlotSpec>& slots,
                     int contrib, int precision, double* E_host, double* rcs_host,
                     pe_stats* acc, int secondary) {
    Batch b(ws, st);
    b.secondary = secondary;
    ws.begin_batch();
    b.setup(slots, contrib, precision);
    uint32_t c[kNumCounters];
    for (int attempt = 0;; attempt++) {
        b.splat();
        b.raygen();
        b.trace(true);
        b.field(E_host, rcs_host);
        b.read_counters(c);
        if (!b.overflowed(c)) break;
        if (attempt > 3) throw Error{PE_EDEVICE, "tile list overflow persists"};
        ws.begin_batch();
        b.setup(slots, contrib, precision);
    }
    if (acc) {
        acc->ray_queries += b.queries(c);
        const double recs = b.records_made(c) * b.max_obs;
        acc->exit_records += recs;
        acc->po_terms += recs * b.max_freq;
        acc->march_cap_hits += c[kCounterCap];
        acc->march_rays += b.march_rays(c);
        acc->march_hits += b.march_hits(c);
    }
}

solve_fn g_densified_solve = nullptr;  // set by the densifier module

}  // namespace pe

extern "C" {

const char* pe_last_error(void) { return g_err.c_str(); }

pe_status pe_ctx_create(int32_t device, uint64_t hbm_budget, pe_ctx* out) {
    API_BEGIN
    if (!out) return set_error(PE_EINVAL, "null output handle");
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return set_error(PE_EINVAL, "no such HIP device");
    HIPCHK(hipSetDevice(device));
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    auto ctx = std::make_unique<pe_ctx_s>();
    ctx->device = device;
    ctx->budget = hbm_budget ? hbm_budget : (uint64_t)(0.9 * (double)free_b);
    ctx->ws = new Workspace(ctx.get());
    scratch_init(device);
    *out = ctx.release();
    return PE_OK;
    API_END
}

pe_status pe_ctx_destroy(pe_ctx ctx) {
    API_BEGIN
    if (!ctx) return PE_OK;
    (void)hipSetDevice(ctx->device);
    server_shutdown(ctx);
    (void)hipDeviceSynchronize();
    delete ctx->ws;
    pe::ctx_release_cache(ctx);
    delete ctx;
    return PE_OK;
    API_END
}

pe_status pe_ctx_footprint(pe_ctx ctx, uint64_t* bytes, uint64_t* budget) {
    if (!ctx) return set_error(PE_EINVAL, "null context");
    if (bytes) *bytes = ctx->used.load();
    if (budget) *budget = ctx->budget;
    return PE_OK;
}

pe_status pe_ctx_set_profiling(pe_ctx ctx, int32_t enable) {
    if (!ctx) return set_error(PE_EINVAL, "null context");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->profile = enable != 0;
    return PE_OK;
}

pe_status pe_ctx_kernel_stats(pe_ctx ctx, int32_t cap, const char** names, double* total_ms,
                              uint64_t* launches, int32_t* n, int32_t reset) {
    if (!ctx || !n) return set_error(PE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    static std::map<std::string, const char*> interned;
    int32_t i = 0;
    for (const auto& kv : ctx->ktab) {
        if (i < cap) {
            auto it = interned.find(kv.first);
            if (it == interned.end()) it = interned.emplace(kv.first, strdup(kv.first.c_str())).first;
            if (names) names[i] = it->second;
            if (total_ms) total_ms[i] = kv.second.first;
            if (launches) launches[i] = kv.second.second;
        }
        i++;
    }
    *n = i;
    if (reset) ctx->ktab.clear();
    return PE_OK;
}

pe_status pe_scene_create(pe_ctx ctx, const pe_scene_desc* desc, void* hip_stream,
                          pe_scene* out) {
    API_BEGIN
    if (!ctx || !desc || !out) return set_error(PE_EINVAL, "null argument");
    const pe_scene_desc& d = *desc;
    if (d.n < 1 || d.n >= (1ull << 31)) return set_error(PE_EINVAL, "n must be 1 .. 2^31-1");
    if (!d.xyz || !d.nrm) return set_error(PE_EINVAL, "xyz and nrm are required");
    if (d.xyz_type != PE_F32 && d.xyz_type != PE_F64) return set_error(PE_EINVAL, "bad xyz_type");
    if (d.mem_kind != PE_MEM_HOST && d.mem_kind != PE_MEM_DEVICE) return set_error(PE_EINVAL, "bad mem_kind");
    if (!d.radius && !(d.radius_scalar > 0 && std::isfinite(d.radius_scalar)))
        return set_error(PE_EINVAL, "radius_scalar must be finite and > 0");
    if (d.view_res < 16 || d.view_res > 4096) return set_error(PE_EINVAL, "view_res must be 16..4096");
    if (d.n_views < 0 || d.n_views > 64 || (d.n_views > 0 && !d.view_dirs))
        return set_error(PE_EINVAL, "n_views must be 0..64 with view_dirs");
    for (int v = 0; v < d.n_views; v++)
        if (!finite3(d.view_dirs + 3 * v)) return set_error(PE_EINVAL, "non-finite or zero view direction");
    if (!(d.blend_radius >= 0) || !std::isfinite(d.blend_radius))
        return set_error(PE_EINVAL, "blend_radius must be finite and >= 0");
    HIPCHK(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    const uint64_t n = d.n;
    auto sc = std::make_unique<pe_scene_s>();
    sc->ctx = ctx;
    sc->n = n;

    struct Tmp {
        pe_ctx ctx;
        std::vector<std::pair<void*, size_t>> v;
        void* get(size_t b) {
            void* p = ctx_alloc(ctx, b);
            v.push_back({p, b});
            return p;
        }
        ~Tmp() {
            (void)hipDeviceSynchronize();
            for (auto& a : v) ctx_free(ctx, a.first, a.second);
        }
    } tmp{ctx, {}};

    const size_t xyz_b = n * 3 * (d.xyz_type == PE_F64 ? 8 : 4);
    const void* xyz = d.xyz;
    const float* nrm = d.nrm;
    const uint8_t* mat = d.material;
    const float* rad = d.radius;
    if (d.mem_kind == PE_MEM_HOST) {
        void* p = tmp.get(xyz_b);
        HIPCHK(hipMemcpyAsync(p, d.xyz, xyz_b, hipMemcpyHostToDevice, st));
        xyz = p;
        p = tmp.get(n * 12);
        HIPCHK(hipMemcpyAsync(p, d.nrm, n * 12, hipMemcpyHostToDevice, st));
        nrm = (const float*)p;
        if (d.material) {
            p = tmp.get(n);
            HIPCHK(hipMemcpyAsync(p, d.material, n, hipMemcpyHostToDevice, st));
            mat = (const uint8_t*)p;
        }
        if (d.radius) {
            p = tmp.get(n * 4);
            HIPCHK(hipMemcpyAsync(p, d.radius, n * 4, hipMemcpyHostToDevice, st));
            rad = (const float*)p;
        }
    }
    const int nb = (int)std::min<uint64_t>(1024, (n + 255) / 256);
    double* part = (double*)tmp.get(sizeof(double) * 8 * nb);
    std::vector<double> hp(8 * nb);
    launch_ingest_stats(xyz, d.xyz_type == PE_F64, nrm, mat, rad, d.radius_scalar, n, part, nb, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * 8 * nb, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, bad = 0;
    for (int b = 0; b < nb; b++) {
        for (int a = 0; a < 3; a++) {
            lo[a] = std::min(lo[a], hp[8 * b + a]);
            hi[a] = std::max(hi[a], hp[8 * b + 3 + a]);
        }
        bad += hp[8 * b + 6];
    }
    if (bad > 0)
        return set_error(PE_EINVAL, std::to_string((uint64_t)bad) +
                                        " points with non-finite position, zero normal, bad radius or material");
    for (int a = 0; a < 3; a++) sc->c[a] = 0.5 * (lo[a] + hi[a]);

    sc->pa = (float4*)sc->alloc(n * 16);
    sc->pb = (float4*)sc->alloc(n * 16);
    sc->pa_s = (float4*)sc->alloc(n * 16);
    sc->pb_s = (float4*)sc->alloc(n * 16);
    launch_ingest_pack(xyz, d.xyz_type == PE_F64, nrm, mat, rad, d.radius_scalar, n, sc->c[0],
                       sc->c[1], sc->c[2], sc->pa, sc->pb, part, nb, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int b = 0; b < nb; b++) {
        sc->R = std::max(sc->R, hp[2 * b]);
        sc->r_max = std::max(sc->r_max, hp[2 * b + 1]);
    }

    // spatial order: stable radix sort by the Morton code of a 1024^3 grid over the bounding box
    double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    if (!(ext > 0)) ext = 1.0;
    const size_t sort_bytes = morton_sort_temp_bytes(n);
    if (sort_bytes == 0) return set_error(PE_EDEVICE, "radix sort size query failed");
    uint32_t* sort_keys = (uint32_t*)tmp.get(n * 16);
    void* sort_tmp = tmp.get(sort_bytes);
    HIPCHK(launch_morton_sort(sc->pa, sc->pb, n, (float)(lo[0] - sc->c[0]),
                              (float)(lo[1] - sc->c[1]), (float)(lo[2] - sc->c[2]),
                              (float)(1024.0 / (ext * (1 + 1e-6))), sort_keys, sort_tmp, sort_bytes,
                              sc->pa_s, sc->pb_s, st));
    sc->cbox = (float4*)sc->alloc(((n + kChunk - 1) / kChunk) * 32);
    launch_chunk_box(sc->pa_s, n, sc->cbox, st);
    HIPCHK(hipGetLastError());

    // object-space hierarchy over the ordered points: an octree of their sorted Morton codes,
    // built top-down one level at a time (each level's node count comes back to the host to
    // size the next), then its boxes bottom-up into one node array
    {
        const uint32_t* codes = sort_keys + n;  // sorted keys of launch_morton_sort
        std::vector<uint2*> rng{(uint2*)tmp.get(8)}, finfo;
        std::vector<uint32_t> cnt{1u}, base{0u};
        launch_fill_u32((uint32_t*)rng[0], 0u, 1, st);
        launch_fill_u32((uint32_t*)rng[0] + 1, (uint32_t)n, 1, st);
        uint32_t* d_total = (uint32_t*)tmp.get(4);
        for (int level = 0;; level++) {
            const uint32_t m = cnt[level];
            uint32_t* ccount = (uint32_t*)tmp.get(4ull * m);
            uint32_t* coff = (uint32_t*)tmp.get(4ull * m + 4);
            uint32_t* scr = (uint32_t*)tmp.get(4ull * scan_wide_scratch(m));
            finfo.push_back((uint2*)tmp.get(8ull * m));
            launch_bvh_count(rng[level], m, level, codes, ccount, st);
            launch_scan_wide(ccount, coff, m, nullptr, 1, d_total, scr, st);
            uint32_t next = 0;
            HIPCHK(hipMemcpyAsync(&next, d_total, 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            uint2* rng_next = next ? (uint2*)tmp.get(8ull * next) : nullptr;
            launch_bvh_emit(rng[level], m, level, codes, coff, base[level] + m, rng_next,
                            finfo[level], st);
            if (next == 0) break;
            if (level + 1 >= kBvhMaxLevels)
                return set_error(PE_EINVAL, "point cloud too dense for the hierarchy");
            rng.push_back(rng_next);
            cnt.push_back(next);
            base.push_back(base[level] + m);
        }
        const int L = (int)cnt.size();
        sc->bvh_levels = L;
        sc->bvh_nodes = (uint64_t)base[L - 1] + cnt[L - 1];
        sc->bvh = (float4*)sc->alloc(sc->bvh_nodes * 32);
        // slack: fp32 rounding of the disk test's hit point at scene scale (a few ulps of R)
        const float pad = (float)(4e-6 * sc->R);
        for (int l = L - 1; l >= 0; l--)
            launch_bvh_box(finfo[l], cnt[l], base[l], sc->pa_s, sc->pb_s, pad, sc->bvh, st);
        HIPCHK(hipGetLastError());
        // wide records: internal nodes numbered in node order, leaf points in record order
        const uint32_t nn = (uint32_t)sc->bvh_nodes;
        uint32_t* is_int = (uint32_t*)tmp.get(4ull * nn);
        uint32_t* leafpts = (uint32_t*)tmp.get(4ull * nn);
        uint32_t* rec = (uint32_t*)tmp.get(4ull * nn + 4);
        uint32_t* lbase = (uint32_t*)tmp.get(4ull * nn + 4);
        uint32_t* scr = (uint32_t*)tmp.get(4ull * scan_wide_scratch(nn));
        launch_wide_count(sc->bvh, nn, is_int, leafpts, st);
        launch_scan_wide(is_int, rec, nn, nullptr, 1, rec + nn, scr, st);
        launch_scan_wide(leafpts, lbase, nn, nullptr, 1, lbase + nn, scr, st);
        uint32_t n_rec = 0;
        HIPCHK(hipMemcpyAsync(&n_rec, rec + nn, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        sc->w_root_pts = n_rec == 0 ? (uint32_t)n : 0u;  // no internal node: the root is a leaf
        sc->wrec = (uint4*)sc->alloc(std::max<uint64_t>(n_rec, 1) * kWideRec * 16);
        sc->wpts = (float4*)sc->alloc(n * 32);
        launch_wide_emit(sc->bvh, nn, rec, lbase, sc->pa_s, sc->pb_s, sc->wrec, sc->wpts, st);
        HIPCHK(hipGetLastError());
        float4 root[2];
        HIPCHK(hipMemcpyAsync(root, sc->bvh, sizeof(root), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const float rb[6] = {root[0].x, root[0].y, root[0].z, root[1].x, root[1].y, root[1].z};
        std::copy(rb, rb + 6, sc->bvh_root);
    }

    // aggregation views
    std::vector<double> dirs;
    if (d.n_views > 0) {
        dirs.assign(d.view_dirs, d.view_dirs + 3 * d.n_views);
    } else {
        const double ax[18] = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
        dirs.assign(ax, ax + 18);
    }
    const int V = (int)dirs.size() / 3;
    std::vector<SlotSpec> vs(V);
    for (int v = 0; v < V; v++) {
        vs[v].sc = sc.get();
        for (int a = 0; a < 3; a++) vs[v].k[a] = dirs[3 * v + a];
        vs[v].W = vs[v].H = d.view_res;
        vs[v].mode = PE_SPLAT_DISK;
    }
    Batch b(*ctx->ws, st);
    b.setup(vs, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
    uint32_t c[kNumCounters];
    for (int attempt = 0;; attempt++) {
        b.splat();
        b.read_counters(c);
        if (!b.overflowed(c)) break;
        if (attempt > 3) return set_error(PE_EDEVICE, "tile list overflow persists");
        b.setup(vs, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
    }
    sc->views.resize(V);
    for (int v = 0; v < V; v++) {
        ViewDesc& vd = sc->views[v];
        const SlotDesc& sd = b.hd[v];
        std::memset(&vd, 0, sizeof vd);
        for (int a = 0; a < 3; a++) {
            vd.u[a] = sd.u[a];
            vd.v[a] = sd.v[a];
            vd.k[a] = sd.k[a];
        }
        vd.pitch = sd.pitch;
        vd.R = sd.R;
        vd.W = sd.W;
        vd.H = sd.H;
        int P = 1, lp = 0;
        while (P < std::max(sd.W, sd.H)) {
            P <<= 1;
            lp++;
        }
        vd.P = P;
        vd.lp = lp;
        vd.levels = lp + 1;
        const uint64_t total = hiz_offset(P, lp) + 1;
        float4* pix = (float4*)sc->alloc((uint64_t)sd.W * sd.H * 32);
        float2* hiz = (float2*)sc->alloc(total * 8);
        float2* ext = (float2*)tmp.get((uint64_t)sd.W * sd.H * 8);
        vd.pix = pix;
        vd.hiz = hiz;
        launch_view_level0(b.dd, v, b.keys, sd.W, sd.H, P, pix, ext, hiz, st);
        for (int l = 1; l <= lp; l++)
            launch_hiz_down(hiz + hiz_offset(P, l - 1), P >> (l - 1), hiz + hiz_offset(P, l), st);
    }
    sc->views_dev = (ViewDesc*)sc->alloc(sizeof(ViewDesc) * V);
    HIPCHK(hipMemcpyAsync(sc->views_dev, sc->views.data(), sizeof(ViewDesc) * V,
                          hipMemcpyHostToDevice, st));
    if (d.blend_radius > 0) {
        // Eq. (23) candidates: grid over the splat centres, cell edge >= r + r_max, <= 256^3
        const double h0 = d.blend_radius + sc->r_max;
        const int G = (int)std::max(1.0, std::min(256.0, std::floor(2.0 * sc->R / h0)));
        sc->blend_r = (float)d.blend_radius;
        sc->bl_G = G;
        sc->bl_h = (float)(2.0 * sc->R / G * (1 + 1e-6));
        const uint64_t nc = (uint64_t)G * G * G;
        sc->bl_start = (uint32_t*)sc->alloc(4 * (nc + 1));
        sc->bl_items = (uint32_t*)sc->alloc(4 * n);
        uint32_t* cell_of2 = (uint32_t*)tmp.get(4 * n);
        uint32_t* cnt2 = (uint32_t*)tmp.get(4 * nc);
        uint32_t* cur2 = (uint32_t*)tmp.get(4 * nc);
        launch_blend_grid(sc->pa, n, (float)sc->R, sc->bl_h, G, cell_of2, cnt2, sc->bl_start, cur2,
                          sc->bl_items, st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    *out = sc.release();
    return PE_OK;
    API_END
}

pe_status pe_scene_destroy(pe_scene scene) {
    API_BEGIN
    if (!scene) return PE_OK;
    pe_ctx ctx = scene->ctx;
    // A scene still held by a submitted request is refused at once (before waiting for the
    // device lock, which the server may hold for many batches in a row); the check is repeated
    // under the lock, which also serialises the free with the synchronous calls that launch
    // with this scene.
    auto busy = [&]() -> pe_status {
        const int held = scene->refs.load();
        if (held <= 0) return PE_OK;
        return set_error(PE_EBUSY, "scene is held by " + std::to_string(held) +
                                       " unfinished server request(s); wait or cancel them first");
    };
    if (busy() != PE_OK) return PE_EBUSY;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (busy() != PE_OK) return PE_EBUSY;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    delete scene;
    return PE_OK;
    API_END
}

pe_status pe_scene_info(pe_scene scene, double centre[3], double* R, double* r_max,
                        uint64_t* bytes) {
    if (!scene) return set_error(PE_EINVAL, "null scene");
    if (centre)
        for (int a = 0; a < 3; a++) centre[a] = scene->c[a];
    if (R) *R = scene->R;
    if (r_max) *r_max = scene->r_max;
    if (bytes) *bytes = scene->bytes;
    return PE_OK;
}

pe_status pe_solve(pe_ctx ctx, pe_scene scene, const pe_solve_desc* desc, pe_result* res,
                   void* hip_stream) {
    API_BEGIN
    if (!ctx || !res || !res->E) return set_error(PE_EINVAL, "null context or result buffer");
    validate_solve(scene, desc);
    if (scene->ctx != ctx) return set_error(PE_EINVAL, "scene belongs to another context");
    HIPCHK(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    pe_stats acc{};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    if (desc->geometry != PE_GEOM_PLAIN) {
        if (!g_densified_solve) return set_error(PE_EUNSUPPORTED, "densifier module unavailable");
        g_densified_solve(*ctx->ws, st, scene, desc, res->E, res->rcs_dbsm, &acc);
    } else {
        const int per = slots_per_batch(ctx, desc);
        const int n_obs = desc->obs_dir ? desc->n_obs : 1;
        const uint64_t per_inc = (uint64_t)n_obs * desc->n_freq * 4;
        for (int i0 = 0; i0 < desc->n_inc; i0 += per) {
            const int cnt = std::min(per, desc->n_inc - i0);
            run_field_batch(*ctx->ws, st, make_slots(scene, desc, i0, cnt), desc->contrib,
                            desc->precision, res->E + i0 * per_inc * 2,
                            res->rcs_dbsm ? res->rcs_dbsm + i0 * per_inc : nullptr, &acc,
                            desc->secondary);
        }
    }
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    acc.time_ms = ms;
    if (res->stats) *res->stats = acc;
    return PE_OK;
    API_END
}

}  // extern "C"

namespace pe {
static pe_status render_gfb(pe_ctx ctx, pe_scene scene, const double dir[3], int32_t w, int32_t h,
                           int32_t mode, double tube_radius, int32_t topk, float* depth,
                           float* nrm, uint32_t* idx, uint8_t* mask, void* hip_stream);
}  // namespace pe

extern "C" {

pe_status pe_render_gfb(pe_ctx ctx, pe_scene scene, const double dir[3], int32_t w, int32_t h,
                        int32_t mode, double tube_radius, float* depth, float* nrm,
                        uint32_t* idx, uint8_t* mask, void* hip_stream) {
    return render_gfb(ctx, scene, dir, w, h, mode, tube_radius, 0, depth, nrm, idx, mask,
                      hip_stream);
}

pe_status pe_render_tube_topk(pe_ctx ctx, pe_scene scene, const double dir[3], int32_t w,
                              int32_t h, double tube_radius, int32_t K, float* depth, float* nrm,
                              uint32_t* idx, uint8_t* mask, void* hip_stream) {
    if (K < 1 || K > 1024) return set_error(PE_EINVAL, "K must be 1..1024");
    return render_gfb(ctx, scene, dir, w, h, PE_SPLAT_TUBE, tube_radius, K, depth, nrm, idx, mask,
                      hip_stream);
}

}  // extern "C"

namespace pe {
static pe_status render_gfb(pe_ctx ctx, pe_scene scene, const double dir[3], int32_t w, int32_t h,
                           int32_t mode, double tube_radius, int32_t topk, float* depth,
                           float* nrm, uint32_t* idx, uint8_t* mask, void* hip_stream) {
    API_BEGIN
    if (!ctx || !scene || !dir) return set_error(PE_EINVAL, "null argument");
    if (!finite3(dir)) return set_error(PE_EINVAL, "non-finite or zero direction");
    if (w < 1 || h < 1 || (uint64_t)w * h > (1u << kPixBits)) return set_error(PE_EINVAL, "bad screen size");
    if (mode != PE_SPLAT_DISK && mode != PE_SPLAT_TUBE) return set_error(PE_EINVAL, "bad mode");
    if (mode == PE_SPLAT_TUBE && !(tube_radius > 0 && std::isfinite(tube_radius)))
        return set_error(PE_EINVAL, "tube_radius must be > 0");
    HIPCHK(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<SlotSpec> s(1);
    s[0].sc = scene;
    for (int a = 0; a < 3; a++) s[0].k[a] = dir[a];
    s[0].W = w;
    s[0].H = h;
    s[0].mode = mode;
    s[0].tube_r = tube_radius;
    Batch b(*ctx->ws, st);
    b.topk = topk;
    b.setup(s, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
    uint32_t c[kNumCounters];
    for (int attempt = 0;; attempt++) {
        b.splat();
        b.read_counters(c);
        if (!b.overflowed(c)) break;
        if (attempt > 3) return set_error(PE_EDEVICE, "tile list overflow persists");
        b.setup(s, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
    }
    launch_resolve(b.dd, b.keys, depth, nrm, idx, mask, w * h, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return PE_OK;
    API_END
}
}  // namespace pe

extern "C" {

pe_status pe_trace_pixels(pe_ctx ctx, pe_scene scene, const double inc_dir[3], int32_t w,
                          int32_t h, int32_t max_bounces, double eps, int32_t secondary,
                          int32_t* n_bounce,
                          float* last_x, float* last_n, double* path, uint32_t* last_idx,
                          void* hip_stream) {
    API_BEGIN
    if (!ctx || !scene || !inc_dir) return set_error(PE_EINVAL, "null argument");
    if (!finite3(inc_dir)) return set_error(PE_EINVAL, "non-finite or zero direction");
    if (w < 1 || h < 1 || (uint64_t)w * h > (1u << kPixBits)) return set_error(PE_EINVAL, "bad screen size");
    if (max_bounces < 1 || max_bounces > kMaxBounces) return set_error(PE_EINVAL, "max_bounces must be 1..16");
    if (!(eps >= 0) || !std::isfinite(eps)) return set_error(PE_EINVAL, "eps must be >= 0");
    if (secondary != PE_SECONDARY_VIEWS && secondary != PE_SECONDARY_SPLATS)
        return set_error(PE_EINVAL, "bad secondary flag");
    HIPCHK(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<SlotSpec> s(1);
    s[0].sc = scene;
    for (int a = 0; a < 3; a++) s[0].k[a] = inc_dir[a];
    s[0].W = w;
    s[0].H = h;
    s[0].max_b = max_bounces;
    s[0].eps = eps;
    Batch b(*ctx->ws, st);
    b.secondary = secondary;
    b.setup(s, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
    uint32_t c[kNumCounters];
    for (int attempt = 0;; attempt++) {
        b.splat();
        b.raygen();
        b.trace(false);
        b.read_counters(c);
        if (!b.overflowed(c)) break;
        if (attempt > 3) return set_error(PE_EDEVICE, "tile list overflow persists");
        b.setup(s, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
    }
    launch_trace_out(b.dd, nullptr, nullptr, b.rs, n_bounce, last_x, last_n, path, last_idx,
                     (w * h + 255) / 256, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return PE_OK;
    API_END
}

}  // extern "C"
