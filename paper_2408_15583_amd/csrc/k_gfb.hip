// Geometric frame buffers as network data and as a ray source (Sec. III-A / III-B):
//   * coarse network input from a TUBE first-hit buffer (Algorithm 1 output before U),
//   * training targets from a DISK first-hit buffer (depth, view-frame normal, hit mask),
//   * normals from depth gradients (Eq. (15)-(16)),
//   * primary rays generated from a GFB (depth, normal, hit probability) instead of the
//     splat keys, so that Eq. (14) can be summed over a densified buffer.
#include "pe_device.h"
#include "pe_gfb.h"

namespace pe {
namespace {

struct f3 {
    float x, y, z;
};
__device__ inline f3 mk3(float x, float y, float z) { return {x, y, z}; }
__device__ inline f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline void st3(const RayState& rs, int c, uint64_t g, f3 v) {
    rs.f[c][g] = v.x;
    rs.f[c + 1][g] = v.y;
    rs.f[c + 2][g] = v.z;
}

}  // namespace

__device__ inline f3 slot_u(const SlotDesc& d) { return mk3(d.u[0], d.u[1], d.u[2]); }
__device__ inline f3 slot_v(const SlotDesc& d) { return mk3(d.v[0], d.v[1], d.v[2]); }
__device__ inline f3 slot_k(const SlotDesc& d) { return mk3(d.k[0], d.k[1], d.k[2]); }

// coarse[pix] = 1 - t / D on hits, 0 elsewhere (D = 2R, t measured from the screen plane).
__global__ void k_coarse_encode(const SlotDesc* __restrict__ ds, const uint64_t* __restrict__ keys,
                                float* __restrict__ out) {
    const SlotDesc& d = ds[blockIdx.y];
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= d.W * d.H) return;
    const uint64_t g = d.pix_base + p;
    const uint64_t key = keys[g];
    out[g] = key == kEmptyKey ? 0.f
                              : 1.f - __uint_as_float((uint32_t)(key >> 32)) / (2.f * d.R);
}

void launch_coarse_encode(const SlotDesc* d, int n_slots, int max_pix, const uint64_t* keys,
                          float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse_encode, dim3((max_pix + 255) / 256, n_slots), dim3(256), 0, st, d,
                       keys, out);
}

// Targets: depth t / D (0 where empty), unit normal oriented against the ray in the view frame
// (u, v, w = -k), mask 1 on hits.
__global__ void k_target_encode(const SlotDesc* __restrict__ ds, const uint64_t* __restrict__ keys,
                                float* __restrict__ depth, float* __restrict__ nrm,
                                float* __restrict__ mask) {
    const SlotDesc& d = ds[blockIdx.y];
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= d.W * d.H) return;
    const uint64_t g = d.pix_base + p;
    const uint64_t key = keys[g];
    if (key == kEmptyKey) {
        depth[g] = 0.f;
        nrm[3 * g] = nrm[3 * g + 1] = nrm[3 * g + 2] = 0.f;
        mask[g] = 0.f;
        return;
    }
    const float4 b = d.pb[(uint32_t)(key & 0xFFFFFFFFu)];
    f3 n = mk3(b.x, b.y, b.z);
    const f3 K = slot_k(d);
    if (dot(n, K) > 0.f) n = n * -1.f;
    depth[g] = __uint_as_float((uint32_t)(key >> 32)) / (2.f * d.R);
    nrm[3 * g] = dot(n, slot_u(d));
    nrm[3 * g + 1] = dot(n, slot_v(d));
    nrm[3 * g + 2] = -dot(n, K);
    mask[g] = 1.f;
}

void launch_target_encode(const SlotDesc* d, int n_slots, int max_pix, const uint64_t* keys,
                          float* depth, float* nrm, float* mask, hipStream_t st) {
    hipLaunchKernelGGL(k_target_encode, dim3((max_pix + 255) / 256, n_slots), dim3(256), 0, st, d,
                       keys, depth, nrm, mask);
}

// Eq. (16) in the view frame: on the surface w(a, b) = -t(a, b) seen from the screen, the
// outward normal is proportional to (t_a, t_b, 1) with t_a = dt/da in metres per metre.
// depth holds t / D, so t_a = (depth difference per pixel) * D / pitch = difference * W.
// Central differences where both neighbours are hits, one-sided where one is, else flat.
__global__ void k_depth_normals(const float* __restrict__ depth, const float* __restrict__ hit,
                                int W, int H, int n_img, float scale, float* __restrict__ nrm) {
    const uint64_t n = (uint64_t)W * H * n_img;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % W), y = (int)((i / W) % H);
        float ta = 0.f, tb = 0.f;
        if (hit[i] > 0.5f) {
            const bool l = x > 0 && hit[i - 1] > 0.5f, r = x + 1 < W && hit[i + 1] > 0.5f;
            const bool u = y > 0 && hit[i - W] > 0.5f, dn = y + 1 < H && hit[i + W] > 0.5f;
            if (l && r) ta = 0.5f * (depth[i + 1] - depth[i - 1]);
            else if (r) ta = depth[i + 1] - depth[i];
            else if (l) ta = depth[i] - depth[i - 1];
            if (u && dn) tb = 0.5f * (depth[i + W] - depth[i - W]);
            else if (dn) tb = depth[i + W] - depth[i];
            else if (u) tb = depth[i] - depth[i - W];
        }
        ta *= scale;
        tb *= scale;
        const float inv = rsqrtf(ta * ta + tb * tb + 1.f);
        nrm[3 * i] = ta * inv;
        nrm[3 * i + 1] = tb * inv;
        nrm[3 * i + 2] = inv;
    }
}

void launch_depth_normals(const float* depth, const float* hit, int W, int H, int n_img,
                          float scale, float* nrm, hipStream_t st) {
    const uint64_t n = (uint64_t)W * H * n_img;
    int b = (int)((n + 255) / 256);
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_depth_normals, dim3(b), dim3(256), 0, st, depth, hit, W, H, n_img, scale,
                       nrm);
}

// Per slot: counts[2s] = pixels with prob > lo, counts[2s+1] = pixels with lo < prob < hi.
__global__ void k_gfb_uncertain(const SlotDesc* __restrict__ ds, const float* __restrict__ prob,
                                float lo, float hi, uint32_t* __restrict__ counts) {
    const int s = blockIdx.y;
    const SlotDesc& d = ds[s];
    const int p = blockIdx.x * 256 + threadIdx.x;
    bool a = false, u = false;
    if (p < d.W * d.H) {
        const float q = prob[d.pix_base + p];
        a = q > lo;
        u = q > lo && q < hi;
    }
    const uint64_t ba = __ballot(a), bu = __ballot(u);
    if ((threadIdx.x & 63) == 0) {
        if (ba) atomicAdd(&counts[2 * s], (uint32_t)__popcll(ba));
        if (bu) atomicAdd(&counts[2 * s + 1], (uint32_t)__popcll(bu));
    }
}

void launch_gfb_uncertain(const SlotDesc* d, int n_slots, int max_pix, const float* prob, float lo,
                          float hi, uint32_t* counts, hipStream_t st) {
    hipLaunchKernelGGL(k_gfb_uncertain, dim3((max_pix + 255) / 256, n_slots), dim3(256), 0, st, d,
                       prob, lo, hi, counts);
}

// A GFB pixel carries a ray when its hit probability reaches thresh and its normal is not
// within kGfbGraze of grazing (the facet area of Eq. (12)-(13) grows as 1 / |n . k|).
constexpr float kGfbGraze = 1e-3f;

__device__ inline bool gfb_live(const SlotDesc& d, const float* prob, const float* nrm,
                                const uint8_t* use, int slot, int p, float thresh) {
    if (p >= d.W * d.H || !use[slot]) return false;
    const uint64_t g = d.pix_base + p;
    if (!(prob[g] >= thresh)) return false;
    const float a = nrm[3 * g], b = nrm[3 * g + 1], c = nrm[3 * g + 2];
    const float l2 = a * a + b * b + c * c;
    return c * c > kGfbGraze * kGfbGraze * l2;
}

__global__ __launch_bounds__(256) void k_gfb_count(const SlotDesc* __restrict__ ds,
                                                   const float* __restrict__ prob,
                                                   const float* __restrict__ nrm,
                                                   const uint8_t* __restrict__ use, float thresh,
                                                   uint32_t* __restrict__ wg_count) {
    const SlotDesc& d = ds[blockIdx.y];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool live = gfb_live(d, prob, nrm, use, blockIdx.y, p, thresh);
    __shared__ uint32_t wc[4];
    const uint64_t bal = __ballot(live);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0)
        wg_count[(uint64_t)blockIdx.y * gridDim.x + blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// Writes the first-bounce state of every live GFB pixel in the same layout as the splat ray
// generation: position from the depth, facet normal from the normal map (view frame, oriented
// against the ray), incident direction and both incident polarisations, tube vectors, path.
__global__ __launch_bounds__(256) void k_gfb_write(const SlotDesc* __restrict__ ds,
                                                   const float* __restrict__ depth,
                                                   const float* __restrict__ nrm,
                                                   const float* __restrict__ prob,
                                                   const uint8_t* __restrict__ use, float thresh,
                                                   const uint32_t* __restrict__ wg_off,
                                                   uint32_t* __restrict__ list, RayState rs,
                                                   uint64_t* __restrict__ hitkey) {
    const uint32_t slot = blockIdx.y;
    const SlotDesc& d = ds[slot];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool live = gfb_live(d, prob, nrm, use, slot, p, thresh);
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
    const f3 U = slot_u(d), V = slot_v(d), K = slot_k(d);
    const float t = depth[g] * 2.f * d.R;
    const int px = p % d.W, py = p / d.W;
    const float ou = (px + 0.5f - 0.5f * d.W) * d.pitch, ov = (py + 0.5f - 0.5f * d.H) * d.pitch;
    f3 n = U * nrm[3 * g] + V * nrm[3 * g + 1] - K * nrm[3 * g + 2];
    const float nl = sqrtf(dot(n, n));
    n = nl > 0.f ? n * (1.f / nl) : K * -1.f;
    if (dot(n, K) > 0.f) n = n * -1.f;
    st3(rs, RX, g, U * ou + V * ov + K * (t - d.R));
    st3(rs, RNX, g, n);
    // a primary record: incoming direction, fields and tube vectors not stored
    rs.d[g] = (double)t - (double)d.R;
    rs.m[g] = 1;
    rs.hit[g] = (uint32_t)p;
}

void launch_gfb_raygen(const SlotDesc* d, int n_slots, int max_pix, const float* depth,
                       const float* nrm, const float* prob, const uint8_t* use, float thresh,
                       uint32_t* wg_count, uint32_t* wg_off, uint32_t* list, RayState rs,
                       uint64_t* hitkey, uint32_t* n_out, uint32_t* scan_ws, hipStream_t st) {
    const int gx = (max_pix + 255) / 256;
    hipLaunchKernelGGL(k_gfb_count, dim3(gx, n_slots), dim3(256), 0, st, d, prob, nrm, use,
                       thresh, wg_count);
    launch_scan_wide(wg_count, wg_off, (uint32_t)(gx * n_slots), nullptr, 1, n_out, scan_ws, st);
    hipLaunchKernelGGL(k_gfb_write, dim3(gx, n_slots), dim3(256), 0, st, d, depth, nrm, prob, use,
                       thresh, wg_off, list, rs, hitkey);
}

// Network outputs -> probabilities and unit normals.
__global__ void k_head_post(const float* __restrict__ logit, const float* __restrict__ nrm_raw,
                            size_t n, float* __restrict__ prob, float* __restrict__ nrm) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (prob) prob[i] = 1.f / (1.f + __expf(-logit[i]));
        if (nrm) {
            const float a = nrm_raw[3 * i], b = nrm_raw[3 * i + 1], c = nrm_raw[3 * i + 2];
            const float l = sqrtf(a * a + b * b + c * c);
            if (l > 0.f) {
                nrm[3 * i] = a / l;
                nrm[3 * i + 1] = b / l;
                nrm[3 * i + 2] = c / l;
            } else {
                nrm[3 * i] = 0.f;
                nrm[3 * i + 1] = 0.f;
                nrm[3 * i + 2] = 1.f;
            }
        }
    }
}

void launch_head_post(const float* logit, const float* nrm_raw, size_t n, float* prob, float* nrm,
                      hipStream_t st) {
    int b = (int)((n + 255) / 256);
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_head_post, dim3(b > 0 ? b : 1), dim3(256), 0, st, logit, nrm_raw, n, prob,
                       nrm);
}

}  // namespace pe
