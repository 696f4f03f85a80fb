// Point-cloud normals by principal component analysis of the k nearest neighbours (the normals
// a raw point cloud is given when it carries none, as in the paper's point-cloud baseline,
// Sec. IV).  Exact k nearest neighbours through a uniform grid searched in growing shells of
// cells; the normal is the eigenvector of the neighbourhood covariance with the smallest
// eigenvalue (closed-form eigenvalues of a symmetric 3x3 matrix by the trigonometric method of
// O. K. Smith, Comm. ACM 4(4), 1961; eigenvector from cross products of rows of C - lambda I),
// turned so that its largest component is positive (splats are two-sided).
#include <float.h>

#include "pe_device.h"

namespace pe {

namespace {

__device__ inline void nrm_load(const void* xyz, int is_f64, uint64_t i, double& x, double& y,
                                double& z) {
    if (is_f64) {
        const double* p = (const double*)xyz + 3 * i;
        x = p[0]; y = p[1]; z = p[2];
    } else {
        const float* p = (const float*)xyz + 3 * i;
        x = p[0]; y = p[1]; z = p[2];
    }
}

__device__ inline int nrm_cell1(float v, float lo, float inv_h, int G) {
    const int q = (int)floorf((v - lo) * inv_h);
    return min(max(q, 0), G - 1);
}

}  // namespace

// Per-block min/max of the coordinates (fp64) for the grid's bounding box.
__global__ __launch_bounds__(256) void k_nrm_bbox(const void* __restrict__ xyz, int is_f64,
                                                  uint64_t n, double* __restrict__ partial) {
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    double bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double v[3];
        nrm_load(xyz, is_f64, i, v[0], v[1], v[2]);
        if (!(isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]))) {
            bad += 1;
            continue;
        }
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], v[a]);
            hi[a] = fmax(hi[a], v[a]);
        }
    }
    __shared__ double red[7][256];
    for (int a = 0; a < 3; a++) {
        red[a][threadIdx.x] = lo[a];
        red[3 + a][threadIdx.x] = hi[a];
    }
    red[6][threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int a = 0; a < 3; a++) {
                red[a][threadIdx.x] = fmin(red[a][threadIdx.x], red[a][threadIdx.x + s]);
                red[3 + a][threadIdx.x] = fmax(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
            }
            red[6][threadIdx.x] += red[6][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) partial[7 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Points relative to the box centre (fp32) and their grid cells; counts per cell.
__global__ void k_nrm_cells(const void* __restrict__ xyz, int is_f64, uint64_t n, double cx,
                            double cy, double cz, float lo, float inv_h, int G,
                            float4* __restrict__ p, uint32_t* __restrict__ cell_of,
                            uint32_t* __restrict__ counts) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double x, y, z;
        nrm_load(xyz, is_f64, i, x, y, z);
        const float4 q = make_float4((float)(x - cx), (float)(y - cy), (float)(z - cz), 0.f);
        p[i] = q;
        const uint32_t c = ((uint32_t)nrm_cell1(q.z, lo, inv_h, G) * G +
                            nrm_cell1(q.y, lo, inv_h, G)) * G + nrm_cell1(q.x, lo, inv_h, G);
        cell_of[i] = c;
        atomicAdd(&counts[c], 1u);
    }
}

__global__ void k_nrm_scatter(const float4* __restrict__ p, uint64_t n,
                              const uint32_t* __restrict__ cell_of,
                              const uint32_t* __restrict__ start, uint32_t* __restrict__ cursor,
                              float4* __restrict__ ps) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cell_of[i];
        const float4 q = p[i];
        ps[start[c] + atomicAdd(&cursor[c], 1u)] = make_float4(q.x, q.y, q.z, __uint_as_float((uint32_t)i));
    }
}

// Smallest-eigenvalue eigenvector of the symmetric matrix (a00 a01 a02; a11 a12; a22).
__device__ inline void smallest_eigvec(double a00, double a01, double a02, double a11, double a12,
                                       double a22, double v[3]) {
    const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
    const double q = (a00 + a11 + a22) / 3.0;
    double lam;
    if (p1 <= 1e-300) {
        // diagonal: the axis of the smallest diagonal entry
        int m = 0;
        if (a11 < a00) m = 1;
        if (a22 < (m == 0 ? a00 : a11)) m = 2;
        v[0] = m == 0; v[1] = m == 1; v[2] = m == 2;
        return;
    }
    const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
    const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
    const double p = sqrt(p2 / 6.0);
    const double ip = 1.0 / p;
    const double c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip;
    const double c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
    double r = 0.5 * (c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) +
                      c02 * (c01 * c12 - c11 * c02));
    r = fmin(1.0, fmax(-1.0, r));
    const double phi = acos(r) / 3.0;
    lam = q + 2.0 * p * cos(phi + 2.0943951023931957);  // smallest (phi + 2 pi / 3)
    const double r0[3] = {a00 - lam, a01, a02};
    const double r1[3] = {a01, a11 - lam, a12};
    const double r2[3] = {a02, a12, a22 - lam};
    auto cross = [](const double* x, const double* y, double* o) {
        o[0] = x[1] * y[2] - x[2] * y[1];
        o[1] = x[2] * y[0] - x[0] * y[2];
        o[2] = x[0] * y[1] - x[1] * y[0];
    };
    double e0[3], e1[3], e2[3];
    cross(r0, r1, e0);
    cross(r0, r2, e1);
    cross(r1, r2, e2);
    const double d0 = e0[0] * e0[0] + e0[1] * e0[1] + e0[2] * e0[2];
    const double d1 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const double d2 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const double* e = e0;
    double dm = d0;
    if (d1 > dm) { e = e1; dm = d1; }
    if (d2 > dm) { e = e2; dm = d2; }
    if (!(dm > 0)) {
        v[0] = 0; v[1] = 0; v[2] = 1;
        return;
    }
    const double il = 1.0 / sqrt(dm);
    v[0] = e[0] * il; v[1] = e[1] * il; v[2] = e[2] * il;
}

// One thread per point: k nearest (keys d^2 | index, ties lowest index) by shells of cells
// until the k-th distance is within the searched radius, then the PCA normal.
__global__ __launch_bounds__(256) void k_nrm_pca(const float4* __restrict__ p, uint64_t n,
                                                 const float4* __restrict__ ps,
                                                 const uint32_t* __restrict__ start, float lo,
                                                 float h, int G, int k, float* __restrict__ nrm) {
    uint64_t best[kMaxNormalK];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float4 q = p[i];
        const float inv_h = 1.f / h;
        const int cx = nrm_cell1(q.x, lo, inv_h, G), cy = nrm_cell1(q.y, lo, inv_h, G),
                  cz = nrm_cell1(q.z, lo, inv_h, G);
        int cnt = 0;
        for (int j = 0; j < k; j++) best[j] = ~0ull;
        for (int m = 0; m <= G; m++) {
            for (int z = max(cz - m, 0); z <= min(cz + m, G - 1); z++)
                for (int y = max(cy - m, 0); y <= min(cy + m, G - 1); y++)
                    for (int x = max(cx - m, 0); x <= min(cx + m, G - 1); x++) {
                        if (max(max(abs(x - cx), abs(y - cy)), abs(z - cz)) != m) continue;
                        const uint32_t c = ((uint32_t)z * G + y) * G + x;
                        for (uint32_t t = start[c]; t < start[c + 1]; t++) {
                            const float4 o = ps[t];
                            const float dx = o.x - q.x, dy = o.y - q.y, dz = o.z - q.z;
                            const float d2 = dx * dx + dy * dy + dz * dz;
                            const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) |
                                                 __float_as_uint(o.w);
                            if (key >= best[k - 1]) continue;
                            int j = k - 1;
                            while (j > 0 && best[j - 1] > key) {
                                best[j] = best[j - 1];
                                j--;
                            }
                            best[j] = key;
                            cnt++;
                        }
                    }
            // every point within m * h of q lies in the cells searched so far
            if (cnt >= k) {
                const float dk = __uint_as_float((uint32_t)(best[k - 1] >> 32));
                const float rm = (float)m * h;
                if (dk <= rm * rm) break;
            }
        }
        const int kk = min(cnt, k);
        double mu[3] = {0, 0, 0};
        for (int j = 0; j < kk; j++) {
            const float4 o = p[(uint32_t)(best[j] & 0xFFFFFFFFu)];
            mu[0] += o.x; mu[1] += o.y; mu[2] += o.z;
        }
        for (int a = 0; a < 3; a++) mu[a] /= kk;
        double c00 = 0, c01 = 0, c02 = 0, c11 = 0, c12 = 0, c22 = 0;
        for (int j = 0; j < kk; j++) {
            const float4 o = p[(uint32_t)(best[j] & 0xFFFFFFFFu)];
            const double ux = o.x - mu[0], uy = o.y - mu[1], uz = o.z - mu[2];
            c00 += ux * ux; c01 += ux * uy; c02 += ux * uz;
            c11 += uy * uy; c12 += uy * uz; c22 += uz * uz;
        }
        double v[3];
        smallest_eigvec(c00, c01, c02, c11, c12, c22, v);
        int am = 0;
        if (fabs(v[1]) > fabs(v[am])) am = 1;
        if (fabs(v[2]) > fabs(v[am])) am = 2;
        const double sg = v[am] < 0 ? -1.0 : 1.0;
        for (int a = 0; a < 3; a++) nrm[3 * i + a] = (float)(sg * v[a]);
    }
}

void launch_nrm_bbox(const void* xyz, int is_f64, uint64_t n, double* partial, int nb,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_nrm_bbox, dim3(nb), dim3(256), 0, st, xyz, is_f64, n, partial);
}

void launch_nrm_grid(const void* xyz, int is_f64, uint64_t n, const double c[3], float lo,
                     float h, int G, float4* p, float4* ps, uint32_t* cell_of, uint32_t* counts,
                     uint32_t* start, uint32_t* cursor, hipStream_t st) {
    const uint64_t nc = (uint64_t)G * G * G;
    const int b = (int)std::min<uint64_t>(8192, (n + 255) / 256);
    launch_fill_u32(counts, 0u, nc, st);
    launch_fill_u32(cursor, 0u, nc, st);
    hipLaunchKernelGGL(k_nrm_cells, dim3(b), dim3(256), 0, st, xyz, is_f64, n, c[0], c[1], c[2],
                       lo, 1.f / h, G, p, cell_of, counts);
    launch_scan(counts, start, (uint32_t)nc, nullptr, 1u, start + nc, st);
    hipLaunchKernelGGL(k_nrm_scatter, dim3(b), dim3(256), 0, st, p, n, cell_of, start, cursor, ps);
}

void launch_nrm_pca(const float4* p, uint64_t n, const float4* ps, const uint32_t* start,
                    float lo, float h, int G, int k, float* nrm, hipStream_t st) {
    const int b = (int)std::min<uint64_t>(16384, (n + 255) / 256);
    hipLaunchKernelGGL(k_nrm_pca, dim3(b), dim3(256), 0, st, p, n, ps, start, lo, h, G, k, nrm);
}

}  // namespace pe
