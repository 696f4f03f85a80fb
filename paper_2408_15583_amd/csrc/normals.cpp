// PCA normal estimation for point clouds without normals: host side of pe_estimate_normals.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pe_runtime.h"

namespace pe {
namespace {

struct NrmScratch {
    pe_ctx ctx;
    hipStream_t st;
    std::vector<std::pair<void*, size_t>> v;
    void* get(size_t b) {
        void* p = ctx_alloc(ctx, b);
        v.push_back({p, b});
        return p;
    }
    ~NrmScratch() {
        (void)hipStreamSynchronize(st);
        for (auto& a : v) ctx_free(ctx, a.first, a.second);
    }
};

}  // namespace
}  // namespace pe

using namespace pe;

extern "C" {

pe_status pe_estimate_normals(pe_ctx ctx, uint64_t n, const void* xyz, int32_t xyz_type,
                              int32_t mem_kind, int32_t k, float* nrm, void* hip_stream) {
    API_BEGIN
    if (!ctx || !xyz || !nrm) return set_error(PE_EINVAL, "null argument");
    if (n < 1 || n >= (1ull << 31)) return set_error(PE_EINVAL, "n must be 1 .. 2^31-1");
    if (xyz_type != PE_F32 && xyz_type != PE_F64) return set_error(PE_EINVAL, "bad xyz_type");
    if (mem_kind != PE_MEM_HOST && mem_kind != PE_MEM_DEVICE) return set_error(PE_EINVAL, "bad mem_kind");
    if (k < 3 || k > kMaxNormalK) return set_error(PE_EINVAL, "k must be 3..64");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    NrmScratch s{ctx, st, {}};
    const size_t xb = (size_t)n * 3 * (xyz_type == PE_F64 ? 8 : 4);
    const void* dx = xyz;
    float* dn = nrm;
    if (mem_kind == PE_MEM_HOST) {
        void* p = s.get(xb);
        HIPCHK(hipMemcpyAsync(p, xyz, xb, hipMemcpyHostToDevice, st));
        dx = p;
        dn = (float*)s.get((size_t)n * 12);
    }
    const int is64 = xyz_type == PE_F64;
    const int nb = (int)std::min<uint64_t>(1024, (n + 255) / 256);
    double* part = (double*)s.get(sizeof(double) * 7 * nb);
    launch_nrm_bbox(dx, is64, n, part, nb, st);
    std::vector<double> hp(7 * (size_t)nb);
    HIPCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, bad = 0;
    for (int b = 0; b < nb; b++) {
        for (int a = 0; a < 3; a++) {
            lo[a] = std::min(lo[a], hp[7 * b + a]);
            hi[a] = std::max(hi[a], hp[7 * b + 3 + a]);
        }
        bad += hp[7 * b + 6];
    }
    if (bad > 0) return set_error(PE_EINVAL, "non-finite positions");
    double c[3], ext = 0;
    for (int a = 0; a < 3; a++) {
        c[a] = 0.5 * (lo[a] + hi[a]);
        ext = std::max(ext, hi[a] - lo[a]);
    }
    const double half = ext > 0 ? 0.5 * ext * (1 + 1e-5) : 1.0;
    // cells of about sqrt(k) point spacings, spacing estimated for points on surfaces
    const double spacing = 2 * half * std::sqrt(6.0 / (double)n);
    const double ht = spacing * std::sqrt((double)k);
    const int G = (int)std::max(1.0, std::min(256.0, std::round(2 * half / ht)));
    const float h = (float)(2 * half / G), flo = (float)(-half);
    const uint64_t nc = (uint64_t)G * G * G;
    float4* p = (float4*)s.get((size_t)n * 16);
    float4* ps = (float4*)s.get((size_t)n * 16);
    uint32_t* cell_of = (uint32_t*)s.get((size_t)n * 4);
    uint32_t* counts = (uint32_t*)s.get(4 * nc);
    uint32_t* cursor = (uint32_t*)s.get(4 * nc);
    uint32_t* start = (uint32_t*)s.get(4 * (nc + 1));
    launch_nrm_grid(dx, is64, n, c, flo, h, G, p, ps, cell_of, counts, start, cursor, st);
    launch_nrm_pca(p, n, ps, start, flo, h, G, k, dn, st);
    HIPCHK(hipGetLastError());
    if (mem_kind == PE_MEM_HOST)
        HIPCHK(hipMemcpyAsync(nrm, dn, (size_t)n * 12, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PE_OK;
    API_END
}

}  // extern "C"
