// Edge filtering and fusion of geometric frame buffers into splats (Sec. III-B, Algorithm 3,
// Eq. (22)): host side of pe_fuse_gfbs.
#include <cmath>
#include <cstring>
#include <vector>

#include "pe_fuse.h"
#include "pe_runtime.h"

namespace pe {

namespace {

// Device temporaries of one call, freed (after the stream drains) when the call returns.
struct Scratch {
    pe_ctx ctx;
    hipStream_t st;
    std::vector<std::pair<void*, size_t>> v;
    void* get(size_t b) {
        void* p = ctx_alloc(ctx, b);
        v.push_back({p, b});
        return p;
    }
    ~Scratch() {
        (void)hipStreamSynchronize(st);
        for (auto& a : v) ctx_free(ctx, a.first, a.second);
    }
};

bool finite_dir(const double* v) {
    const double l = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    return std::isfinite(l) && l > 0;
}

}  // namespace

}  // namespace pe

using namespace pe;

extern "C" {

pe_status pe_fuse_gfbs(pe_ctx ctx, const pe_gfb_set* g, const pe_fuse_desc* f, double* xyz,
                       float* nrm, float* radius, uint32_t* count, uint8_t* edge, uint64_t cap,
                       uint64_t* n_out, void* hip_stream) {
    API_BEGIN
    if (!ctx || !g || !f || !n_out) return set_error(PE_EINVAL, "null argument");
    if (g->n_views < 1 || g->n_views > kFuseMaxViews || !g->view_dirs)
        return set_error(PE_EINVAL, "n_views must be 1..64 with view_dirs");
    for (int v = 0; v < g->n_views; v++)
        if (!finite_dir(g->view_dirs + 3 * v))
            return set_error(PE_EINVAL, "non-finite or zero view direction");
    if (g->w < 8 || g->w != g->h || g->w > 8192)
        return set_error(PE_EINVAL, "buffers must be square, 8..8192 pixels");
    if (!g->depth || !g->nrm || !g->hit) return set_error(PE_EINVAL, "depth, nrm and hit are required");
    if (!(g->R > 0) || !std::isfinite(g->R) || !std::isfinite(g->centre[0]) ||
        !std::isfinite(g->centre[1]) || !std::isfinite(g->centre[2]))
        return set_error(PE_EINVAL, "bad frame (R > 0 and a finite centre required)");
    const int G = f->grid ? f->grid : 256;
    if (G < 8 || G > 512) return set_error(PE_EINVAL, "grid must be 8..512");
    const double side = f->grid_side > 0 ? f->grid_side : 2.0 * g->R;
    if (!std::isfinite(side)) return set_error(PE_EINVAL, "grid_side must be finite");
    const double lo = f->edge_lo > 0 ? f->edge_lo : 2.0, hi = f->edge_hi > 0 ? f->edge_hi : 4.0;
    if (!(lo <= hi) || !std::isfinite(hi)) return set_error(PE_EINVAL, "need 0 < edge_lo <= edge_hi");
    const int dil = f->edge_dilate < 0 ? 1 : f->edge_dilate;
    if (dil > 8) return set_error(PE_EINVAL, "edge_dilate must be 0..8 (negative = 1)");
    if (cap > 0 && !(xyz && nrm && radius)) return set_error(PE_EINVAL, "cap > 0 needs xyz, nrm, radius");

    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const int w = g->w, h = g->h, nv = g->n_views;
    const size_t npix = (size_t)nv * w * h;
    const size_t ncell = (size_t)G * G * G;

    FuseArgs a{};
    a.n_views = nv;
    a.w = w;
    a.h = h;
    a.depth = g->depth;
    a.nrm = g->nrm;
    a.hit = g->hit;
    a.R = (float)g->R;
    // Gaussian of sigma = 1 pixel: exp(-d^2 / 2) at d = 0, 1, 2, normalised over the 5 taps
    const double e1 = std::exp(-0.5), e2 = std::exp(-2.0), gs = 1.0 + 2.0 * (e1 + e2);
    a.g[0] = (float)(1.0 / gs);
    a.g[1] = (float)(e1 / gs);
    a.g[2] = (float)(e2 / gs);
    // Sobel sums are 8 x the depth change per pixel; a slope s (depth change per pitch
    // 2R / w) is a Sobel sum of s * 16 R / w.
    const double tl = lo * 16.0 * g->R / w, th = hi * 16.0 * g->R / w;
    a.thr2_lo = (float)(tl * tl);
    a.thr2_hi = (float)(th * th);
    a.tan22 = (float)(std::sqrt(2.0) - 1.0);
    a.dilate = dil;
    a.half = (float)(0.5 * side);
    a.L = (float)(side / G);
    a.G = G;
    a.qpos = side / 68719476736.0;  // 2^-36 of the grid side
    for (int k = 0; k < 3; k++) a.c[k] = g->centre[k];

    Scratch s{ctx, st, {}};
    std::vector<float> hb(9 * (size_t)nv);
    for (int v = 0; v < nv; v++) {
        double u[3], vv[3], k[3];
        screen_basis(g->view_dirs + 3 * v, u, vv, k);
        for (int c = 0; c < 3; c++) {
            hb[9 * v + c] = (float)u[c];
            hb[9 * v + 3 + c] = (float)vv[c];
            hb[9 * v + 6 + c] = (float)k[c];
        }
    }
    float* basis = (float*)s.get(hb.size() * sizeof(float));
    HIPCHK(hipMemcpyAsync(basis, hb.data(), hb.size() * sizeof(float), hipMemcpyHostToDevice, st));
    a.basis = basis;

    float* blur = (float*)s.get(npix * sizeof(float));
    uint8_t* cls = (uint8_t*)s.get(npix);
    uint8_t* drop = (uint8_t*)s.get(npix);
    constexpr int kPasses = 8;
    uint32_t* changed = (uint32_t*)s.get(kPasses * sizeof(uint32_t));
    launch_fuse_blur(a, blur, st);
    launch_fuse_classify(a, blur, cls, st);
    // hysteresis to its fixed point, checked every kPasses passes
    for (;;) {
        launch_fill_u32(changed, 0u, kPasses, st);
        for (int p = 0; p < kPasses; p++) launch_fuse_hysteresis(a, cls, changed + p, st);
        uint32_t hc[kPasses];
        HIPCHK(hipMemcpyAsync(hc, changed, sizeof(hc), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hc[kPasses - 1] == 0) break;
    }
    launch_fuse_drop(a, cls, drop, edge, st);

    unsigned long long* acc = (unsigned long long*)s.get(ncell * kFuseWords * 8);
    launch_fill_u64((uint64_t*)acc, 0ull, (uint64_t)ncell * kFuseWords, st);
    launch_fuse_accum(a, drop, acc, st);
    uint32_t* flag = (uint32_t*)s.get(ncell * sizeof(uint32_t));
    uint32_t* off = (uint32_t*)s.get(ncell * sizeof(uint32_t));
    uint32_t* total = (uint32_t*)s.get(sizeof(uint32_t));
    uint32_t* scan_ws = (uint32_t*)s.get(scan_wide_scratch((uint32_t)ncell) * sizeof(uint32_t));
    launch_fuse_flag(acc, ncell, flag, st);
    launch_scan_wide(flag, off, (uint32_t)ncell, nullptr, 1u, total, scan_ws, st);
    uint32_t nt = 0;
    HIPCHK(hipMemcpyAsync(&nt, total, sizeof(nt), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *n_out = nt;
    if (cap > 0 && nt > 0)
        launch_fuse_emit(a, acc, flag, off, ncell, xyz, nrm, radius, count, cap, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return PE_OK;
    API_END
}

}  // extern "C"
