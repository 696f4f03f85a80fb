// Geometry for GFB-assisted bounces (Sec. III-B, Algorithm 3): edge filtering of geometric
// frame buffers with a Canny operator, fusion into a cubic grid, and one splat per occupied
// cell with the radius of Eq. (22).
//
// Buffers: n_views x h x w, depth t/D (D = 2R, t from the view's screen plane), normals in the
// view frame (u, v, -k), hit where hit >= 0.5.  The edge decisions are made in fp32 with every
// operation rounded on its own (no fused multiply-add), so they are reproducible off the GPU;
// fusion sums are fixed-point 64-bit integers, so their order does not matter either.
#include <float.h>

#include "pe_device.h"
#include "pe_fuse.h"

namespace pe {

// Depth in metres with empty pixels pushed to the far side of the scene (2R): silhouettes are
// then the strongest edges.
__device__ inline float fuse_depth(const FuseArgs& a, size_t i) {
#pragma clang fp contract(off)
    const float D = 2.f * a.R;
    return a.hit[i] >= 0.5f ? a.depth[i] * D : D;
}

// 5 x 5 Gaussian of the depth, separable weights g[|d|] multiplied per tap, clamp-to-edge;
// the 25 taps are summed row by row.
__global__ void k_fuse_blur(FuseArgs a, float* __restrict__ blur) {
#pragma clang fp contract(off)
    const size_t n = (size_t)a.n_views * a.h * a.w;
    const float g[5] = {a.g[2], a.g[1], a.g[0], a.g[1], a.g[2]};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % a.w), y = (int)((i / a.w) % a.h);
        const size_t base = i - (size_t)y * a.w - x;
        float s = 0.f;
        for (int dy = -2; dy <= 2; dy++) {
            const int yy = min(max(y + dy, 0), a.h - 1);
            for (int dx = -2; dx <= 2; dx++) {
                const int xx = min(max(x + dx, 0), a.w - 1);
                const float wgt = g[dy + 2] * g[dx + 2];
                s = s + wgt * fuse_depth(a, base + (size_t)yy * a.w + xx);
            }
        }
        blur[i] = s;
    }
}

// Sobel sums (gx, gy) of the blurred depth at (x, y), clamp-to-edge.
__device__ inline float2 fuse_sobel(const float* __restrict__ blur, size_t base, int w, int h,
                                    int x, int y) {
#pragma clang fp contract(off)
    auto B = [&](int xx, int yy) {
        xx = min(max(xx, 0), w - 1);
        yy = min(max(yy, 0), h - 1);
        return blur[base + (size_t)yy * w + xx];
    };
    const float gx = ((B(x + 1, y - 1) + 2.f * B(x + 1, y)) + B(x + 1, y + 1)) -
                     ((B(x - 1, y - 1) + 2.f * B(x - 1, y)) + B(x - 1, y + 1));
    const float gy = ((B(x - 1, y + 1) + 2.f * B(x, y + 1)) + B(x + 1, y + 1)) -
                     ((B(x - 1, y - 1) + 2.f * B(x, y - 1)) + B(x + 1, y - 1));
    return make_float2(gx, gy);
}

__device__ inline float fuse_mag2(float2 g) {
#pragma clang fp contract(off)
    return g.x * g.x + g.y * g.y;
}

// Non-maximum suppression along the gradient (direction quantised to 0, 45, 90, 135 degrees;
// neighbours outside the buffer are clamped) and the double threshold on the squared Sobel
// magnitude: cls = 2 strong, 1 weak, 0 none.
__global__ void k_fuse_classify(FuseArgs a, const float* __restrict__ blur,
                                uint8_t* __restrict__ cls) {
#pragma clang fp contract(off)
    const size_t n = (size_t)a.n_views * a.h * a.w;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % a.w), y = (int)((i / a.w) % a.h);
        const size_t base = i - (size_t)y * a.w - x;
        const float2 gc = fuse_sobel(blur, base, a.w, a.h, x, y);
        const float m = fuse_mag2(gc);
        uint8_t c = 0;
        if (m >= a.thr2_lo) {
            const float ax = fabsf(gc.x), ay = fabsf(gc.y);
            int dx, dy;
            if (ay <= a.tan22 * ax) { dx = 1; dy = 0; }
            else if (ax <= a.tan22 * ay) { dx = 0; dy = 1; }
            else if ((gc.x > 0.f) == (gc.y > 0.f)) { dx = 1; dy = 1; }
            else { dx = 1; dy = -1; }
            const float m1 = fuse_mag2(fuse_sobel(blur, base, a.w, a.h, x + dx, y + dy));
            const float m2 = fuse_mag2(fuse_sobel(blur, base, a.w, a.h, x - dx, y - dy));
            if (m >= m1 && m >= m2) c = m >= a.thr2_hi ? 2 : 1;
        }
        cls[i] = c;
    }
}

// One hysteresis pass: a weak pixel with an edge among its 8 neighbours becomes an edge.
// Passes repeat until none changes; the fixed point is every weak pixel 8-connected through
// weak pixels to a strong one, whatever order the pass visits them in.
__global__ void k_fuse_hysteresis(FuseArgs a, uint8_t* __restrict__ cls,
                                  uint32_t* __restrict__ changed) {
    const size_t n = (size_t)a.n_views * a.h * a.w;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (cls[i] != 1) continue;
        const int x = (int)(i % a.w), y = (int)((i / a.w) % a.h);
        const size_t base = i - (size_t)y * a.w - x;
        bool e = false;
        for (int dy = -1; dy <= 1 && !e; dy++) {
            const int yy = y + dy;
            if (yy < 0 || yy >= a.h) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int xx = x + dx;
                if (xx < 0 || xx >= a.w) continue;
                if (cls[base + (size_t)yy * a.w + xx] == 2) { e = true; break; }
            }
        }
        if (e) {
            cls[i] = 2;
            atomicAdd(changed, 1u);
        }
    }
}

// Pixels dropped from fusion: within `dilate` pixels (Chebyshev) of an edge.  edge (optional)
// receives the Canny edge map itself.
__global__ void k_fuse_drop(FuseArgs a, const uint8_t* __restrict__ cls,
                            uint8_t* __restrict__ drop, uint8_t* __restrict__ edge) {
    const size_t n = (size_t)a.n_views * a.h * a.w;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % a.w), y = (int)((i / a.w) % a.h);
        const size_t base = i - (size_t)y * a.w - x;
        bool d = false;
        for (int yy = max(y - a.dilate, 0); yy <= min(y + a.dilate, a.h - 1) && !d; yy++)
            for (int xx = max(x - a.dilate, 0); xx <= min(x + a.dilate, a.w - 1); xx++)
                if (cls[base + (size_t)yy * a.w + xx] == 2) { d = true; break; }
        drop[i] = d ? 1 : 0;
        if (edge) edge[i] = cls[i] == 2 ? 1 : 0;
    }
}

// Fusion: every kept hit pixel adds its point (fixed point, quantum qpos, from the grid
// corner), its unit normal turned to a canonical side (largest component positive: splats are
// two-sided; quantum 2^-30), a count and its view's bit to its grid cell.  Points up to one
// cell outside the grid go to the boundary cell; points further out are ignored.  The point,
// the cell index and the side of the normal are computed in fp32 with every operation rounded
// on its own, like the edge decisions.
__global__ void k_fuse_accum(FuseArgs a, const uint8_t* __restrict__ drop,
                             unsigned long long* __restrict__ acc) {
#pragma clang fp contract(off)
    const size_t n = (size_t)a.n_views * a.h * a.w;
    const float D = 2.f * a.R;
    const float pitch = D / (float)a.w;
    const float hw = 0.5f * (float)a.w, hh = 0.5f * (float)a.h;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (!(a.hit[i] >= 0.5f) || drop[i]) continue;
        const int x = (int)(i % a.w), y = (int)((i / a.w) % a.h), v = (int)(i / ((size_t)a.w * a.h));
        const float* b = a.basis + 9 * v;  // u, v, k of the view
        const float ou = (((float)x + 0.5f) - hw) * pitch, ov = (((float)y + 0.5f) - hh) * pitch;
        const float t = a.depth[i] * D - a.R;
        float P[3], N[3];
        for (int c = 0; c < 3; c++) P[c] = (b[c] * ou + b[3 + c] * ov) + b[6 + c] * t;
        const float nu = a.nrm[3 * i], nv = a.nrm[3 * i + 1], nw = a.nrm[3 * i + 2];
        for (int c = 0; c < 3; c++) N[c] = (b[c] * nu + b[3 + c] * nv) - b[6 + c] * nw;
        const float nl = sqrtf((N[0] * N[0] + N[1] * N[1]) + N[2] * N[2]);
        if (!(nl > 0.f)) continue;
        int ci[3];
        bool in = true;
        for (int c = 0; c < 3; c++) {
            int q = (int)floorf((P[c] + a.half) / a.L);
            if (q == -1) q = 0;
            if (q == a.G) q = a.G - 1;
            ci[c] = q;
            in = in && q >= 0 && q < a.G;
        }
        if (!in) continue;
        int am = 0;
        if (fabsf(N[1]) > fabsf(N[am])) am = 1;
        if (fabsf(N[2]) > fabsf(N[am])) am = 2;
        const double s = (N[am] < 0.f ? -1.0 : 1.0) / (double)nl;
        const size_t cell = ((size_t)ci[2] * a.G + ci[1]) * a.G + ci[0];
        unsigned long long* A = acc + cell * kFuseWords;
        for (int c = 0; c < 3; c++)
            atomicAdd(&A[c], (unsigned long long)llrint(((double)P[c] + (double)a.half) / a.qpos));
        for (int c = 0; c < 3; c++)
            atomicAdd(&A[3 + c], (unsigned long long)llrint(s * (double)N[c] * 1073741824.0));
        atomicAdd(&A[6], 1ull);
        atomicOr(&A[7], 1ull << v);
    }
}

// Occupied cells: flag for the scan.
__global__ void k_fuse_flag(const unsigned long long* __restrict__ acc, size_t n_cells,
                            uint32_t* __restrict__ flag) {
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += (size_t)gridDim.x * blockDim.x)
        flag[c] = acc[c * kFuseWords + 6] > 0 ? 1u : 0u;
}

// One splat per occupied cell, in cell order (x fastest): mean position (world), normalised
// mean normal, and the Eq. (22) radius of that normal for the contributing view that sees it
// most squarely (the radius grows with 1/|n.p|, so this is the minimum over the views).
__global__ void k_fuse_emit(FuseArgs a, const unsigned long long* __restrict__ acc,
                            const uint32_t* __restrict__ flag, const uint32_t* __restrict__ off,
                            size_t n_cells, double* __restrict__ xyz, float* __restrict__ nrm,
                            float* __restrict__ radius, uint32_t* __restrict__ count,
                            uint64_t cap) {
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += (size_t)gridDim.x * blockDim.x) {
        if (!flag[c]) continue;
        const uint32_t o = off[c];
        if (o >= cap) continue;
        const unsigned long long* A = acc + c * kFuseWords;
        const double cnt = (double)A[6];
        for (int k = 0; k < 3; k++)
            xyz[3 * (size_t)o + k] = (double)(long long)A[k] / cnt * a.qpos - (double)a.half + a.c[k];
        double N[3], l = 0;
        for (int k = 0; k < 3; k++) {
            N[k] = (double)(long long)A[3 + k];
            l += N[k] * N[k];
        }
        l = sqrt(l);
        for (int k = 0; k < 3; k++) N[k] = l > 0 ? N[k] / l : (k == 2 ? 1.0 : 0.0);
        for (int k = 0; k < 3; k++) nrm[3 * (size_t)o + k] = (float)N[k];
        double best = 0;
        unsigned long long m = A[7];
        while (m) {
            const int v = __ffsll((long long)m) - 1;
            m &= m - 1;
            const float* b = a.basis + 9 * v + 6;
            best = fmax(best, fabs(N[0] * b[0] + N[1] * b[1] + N[2] * b[2]));
        }
        const double f = best > 0 ? sqrt(1.0 / best) : 1e30;
        radius[o] = (float)(f < 2.5 ? 1.4142135623730951 * a.L * f : 3.535 * a.L);
        if (count) count[o] = (uint32_t)A[6];
    }
}

static int grid_blocks(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (int)(b > 0 ? b : 1);
}

static size_t n_pix(const FuseArgs& a) { return (size_t)a.n_views * a.h * a.w; }

void launch_fuse_blur(const FuseArgs& a, float* blur, hipStream_t st) {
    hipLaunchKernelGGL(k_fuse_blur, dim3(grid_blocks(n_pix(a))), dim3(256), 0, st, a, blur);
}
void launch_fuse_classify(const FuseArgs& a, const float* blur, uint8_t* cls, hipStream_t st) {
    hipLaunchKernelGGL(k_fuse_classify, dim3(grid_blocks(n_pix(a))), dim3(256), 0, st, a, blur,
                       cls);
}
void launch_fuse_hysteresis(const FuseArgs& a, uint8_t* cls, uint32_t* changed, hipStream_t st) {
    hipLaunchKernelGGL(k_fuse_hysteresis, dim3(grid_blocks(n_pix(a))), dim3(256), 0, st, a, cls,
                       changed);
}
void launch_fuse_drop(const FuseArgs& a, const uint8_t* cls, uint8_t* drop, uint8_t* edge,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_fuse_drop, dim3(grid_blocks(n_pix(a))), dim3(256), 0, st, a, cls, drop,
                       edge);
}
void launch_fuse_accum(const FuseArgs& a, const uint8_t* drop, unsigned long long* acc,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_fuse_accum, dim3(grid_blocks(n_pix(a))), dim3(256), 0, st, a, drop, acc);
}
void launch_fuse_flag(const unsigned long long* acc, size_t n_cells, uint32_t* flag,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_fuse_flag, dim3(grid_blocks(n_cells)), dim3(256), 0, st, acc, n_cells,
                       flag);
}
void launch_fuse_emit(const FuseArgs& a, const unsigned long long* acc, const uint32_t* flag,
                      const uint32_t* off, size_t n_cells, double* xyz, float* nrm,
                      float* radius, uint32_t* count, uint64_t cap, hipStream_t st) {
    hipLaunchKernelGGL(k_fuse_emit, dim3(grid_blocks(n_cells)), dim3(256), 0, st, a, acc, flag,
                       off, n_cells, xyz, nrm, radius, count, cap);
}

}  // namespace pe
