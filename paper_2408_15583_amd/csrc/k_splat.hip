// Scene ingest and the splat raster: points carrying normals become oriented disks; every
// pixel's central ray keeps the nearest disk it crosses (DISK mode) or the nearest point within
// the tube radius of the central ray (TUBE mode, Algorithm 1 with an unbounded Top-K).
//
// MI355X design: points are sorted once per scene in Morton order of a 1024^3 grid
// (k_sort.hip) so that a wavefront of 64 consecutive points is a compact surface patch; per
// view, each patch's screen rectangle (from its 3D box) is binned into 32x32-pixel tiles
// (16x16 for the K-point heap); one workgroup per tile rasterises its patches
// into an LDS tile of packed 64-bit keys (fp32 depth bits << 32 | point index) with ds_min_u64,
// then writes the tile once.  The minimum key is the nearest hit with ties going to the lowest
// index, independent of the order in which patches arrive.
#include <float.h>
#include <limits.h>

#include "pe_device.h"
#include "pe_gfb.h"

namespace pe {

// ------------------------------------------------------------------------------------------
// Ingest
// ------------------------------------------------------------------------------------------

__device__ inline void load_xyz(const void* xyz, int is_f64, uint64_t i, double& x, double& y,
                                double& z) {
    if (is_f64) {
        const double* p = (const double*)xyz + 3 * i;
        x = p[0]; y = p[1]; z = p[2];
    } else {
        const float* p = (const float*)xyz + 3 * i;
        x = p[0]; y = p[1]; z = p[2];
    }
}

// Per-block partials: [lo x, lo y, lo z, hi x, hi y, hi z, bad count, 0].
__global__ __launch_bounds__(256) void k_ingest_stats(const void* __restrict__ xyz, int is_f64,
                                                      const float* __restrict__ nrm,
                                                      const uint8_t* __restrict__ mat,
                                                      const float* __restrict__ rad,
                                                      float rad_s, uint64_t n,
                                                      double* __restrict__ partial) {
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    double bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double x, y, z;
        load_xyz(xyz, is_f64, i, x, y, z);
        const float nx = nrm[3 * i], ny = nrm[3 * i + 1], nz = nrm[3 * i + 2];
        const float nl = nx * nx + ny * ny + nz * nz;
        const float r = rad ? rad[i] : rad_s;
        const uint8_t m = mat ? mat[i] : 0;
        const bool fin = isfinite(x) && isfinite(y) && isfinite(z);
        const bool ok = fin && nl > 0.f && isfinite(nl) && r > 0.f && isfinite(r) && m <= 1;
        if (!ok) bad += 1;
        if (fin) {
            lo[0] = fmin(lo[0], x); lo[1] = fmin(lo[1], y); lo[2] = fmin(lo[2], z);
            hi[0] = fmax(hi[0], x); hi[1] = fmax(hi[1], y); hi[2] = fmax(hi[2], z);
        }
    }
    __shared__ double red[7][256];
    for (int a = 0; a < 3; a++) { red[a][threadIdx.x] = lo[a]; red[3 + a][threadIdx.x] = hi[a]; }
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
    if (threadIdx.x == 0) {
        for (int a = 0; a < 7; a++) partial[blockIdx.x * 8 + a] = red[a][0];
        partial[blockIdx.x * 8 + 7] = 0;
    }
}

void launch_ingest_stats(const void* xyz, int is_f64, const float* nrm, const uint8_t* mat,
                         const float* rad, float rad_scalar, uint64_t n, double* partial,
                         int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_ingest_stats, dim3(n_blocks), dim3(256), 0, st, xyz, is_f64, nrm, mat,
                       rad, rad_scalar, n, partial);
}

// Recentre on c (in fp64, then round), normalise normals, pack (x,y,z,r) and (n, material).
// Per-block partial: max over points of |x - c| + r (fp64), the scene radius R.
__global__ __launch_bounds__(256) void k_ingest_pack(const void* __restrict__ xyz, int is_f64,
                                                     const float* __restrict__ nrm,
                                                     const uint8_t* __restrict__ mat,
                                                     const float* __restrict__ rad, float rad_s,
                                                     uint64_t n, double cx, double cy, double cz,
                                                     float4* __restrict__ pa,
                                                     float4* __restrict__ pb,
                                                     double* __restrict__ partial) {
    double rmax = 0, radmax = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double x, y, z;
        load_xyz(xyz, is_f64, i, x, y, z);
        const double dx = x - cx, dy = y - cy, dz = z - cz;
        const float r = rad ? rad[i] : rad_s;
        const double nx = nrm[3 * i], ny = nrm[3 * i + 1], nz = nrm[3 * i + 2];
        const double il = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
        pa[i] = make_float4((float)dx, (float)dy, (float)dz, r);
        pb[i] = make_float4((float)(nx * il), (float)(ny * il), (float)(nz * il),
                            (float)(mat ? mat[i] : 0));
        rmax = fmax(rmax, sqrt(dx * dx + dy * dy + dz * dz) + (double)r);
        radmax = fmax(radmax, (double)r);
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = rmax;
    red[1][threadIdx.x] = radmax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x * 2] = red[0][0];
        partial[blockIdx.x * 2 + 1] = red[1][0];
    }
}

void launch_ingest_pack(const void* xyz, int is_f64, const float* nrm, const uint8_t* mat,
                        const float* rad, float rad_scalar, uint64_t n, double cx, double cy,
                        double cz, float4* pa, float4* pb, double* partial, int n_blocks,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_ingest_pack, dim3(n_blocks), dim3(256), 0, st, xyz, is_f64, nrm, mat,
                       rad, rad_scalar, n, cx, cy, cz, pa, pb, partial);
}

// ------------------------------------------------------------------------------------------
// Splat raster
// ------------------------------------------------------------------------------------------

struct Screen {
    float u0, u1, u2, v0, v1, v2, k0, k1, k2;
    float pitch, ipitch, R, hw, hh, tube_r;
    int W, H, mode;
};

__device__ inline Screen screen_of(const SlotDesc& d) {
    Screen s;
    s.u0 = d.u[0]; s.u1 = d.u[1]; s.u2 = d.u[2];
    s.v0 = d.v[0]; s.v1 = d.v[1]; s.v2 = d.v[2];
    s.k0 = d.k[0]; s.k1 = d.k[1]; s.k2 = d.k[2];
    s.pitch = d.pitch; s.ipitch = 1.0f / d.pitch; s.R = d.R;
    s.W = d.W; s.H = d.H; s.hw = 0.5f * d.W; s.hh = 0.5f * d.H;
    s.mode = d.mode; s.tube_r = d.tube_r;
    return s;
}

// A point projected on the screen: coordinates along u, v, k; normal components along u, v, k.
struct Proj {
    float xa, xb, xk, na, nb, nk, r;
};

__device__ inline Proj project(const Screen& s, float4 a, float4 b) {
    Proj p;
    p.xa = a.x * s.u0 + a.y * s.u1 + a.z * s.u2;
    p.xb = a.x * s.v0 + a.y * s.v1 + a.z * s.v2;
    p.xk = a.x * s.k0 + a.y * s.k1 + a.z * s.k2;
    p.na = b.x * s.u0 + b.y * s.u1 + b.z * s.u2;
    p.nb = b.x * s.v0 + b.y * s.v1 + b.z * s.v2;
    p.nk = b.x * s.k0 + b.y * s.k1 + b.z * s.k2;
    p.r = a.w;
    return p;
}

// Inclusive pixel range whose centres can pass the exact test (empty: x0 > x1).  The disk's
// extent along a screen axis e is r * sqrt(1 - (n.e)^2); a tube's is its radius.
__device__ inline void footprint(const Screen& s, const Proj& p, int& x0, int& y0, int& x1,
                                 int& y1) {
    float ea, eb;
    if (s.mode == 0) {
        if (fabsf(p.nk) < kGraze) { x0 = y0 = INT_MAX; x1 = y1 = INT_MIN; return; }
        ea = p.r * sqrtf(fmaxf(0.f, 1.f - p.na * p.na));
        eb = p.r * sqrtf(fmaxf(0.f, 1.f - p.nb * p.nb));
    } else {
        ea = eb = s.tube_r;
    }
    const float ac = p.xa * s.ipitch + s.hw - 0.5f, bc = p.xb * s.ipitch + s.hh - 0.5f;
    const float ex = ea * s.ipitch + 1e-3f, ey = eb * s.ipitch + 1e-3f;
    x0 = max(0, (int)ceilf(ac - ex));
    x1 = min(s.W - 1, (int)floorf(ac + ex));
    y0 = max(0, (int)ceilf(bc - ey));
    y1 = min(s.H - 1, (int)floorf(bc + ey));
}

// XCD-aware order of a (unit, slot) grid: workgroup b runs on XCD b % kNumXcd, and each XCD
// takes a contiguous share of the unit-major, slot-minor order.  Consecutive workgroups of one
// XCD then project the same chunks for neighbouring incidences of the batch, reading those
// points from that XCD's L2.
__host__ __device__ inline uint32_t xcd_grid(uint32_t n_units, uint32_t n_slots) {
    return (n_units * n_slots + kNumXcd - 1) / kNumXcd * kNumXcd;
}
__device__ inline bool xcd_unit_slot(uint32_t b, uint32_t n_units, uint32_t n_slots,
                                     uint32_t& unit, uint32_t& slot) {
    const uint32_t total = n_units * n_slots, per = (total + kNumXcd - 1) / kNumXcd;
    const uint32_t pos = (b % kNumXcd) * per + b / kNumXcd;
    if (pos >= total) return false;
    unit = pos / n_slots;
    slot = pos % n_slots;
    return true;
}

// The raster's order: XCD x takes the tiles t = x (mod kNumXcd), each for every incidence in
// turn, so one XCD's L2 serves a tile's points to neighbouring incidences while the XCDs share
// every region of the screen (whose point counts differ widely) evenly.
__host__ __device__ inline uint32_t xcd_tile_grid(uint32_t n_tiles, uint32_t n_slots) {
    return (n_tiles + kNumXcd - 1) / kNumXcd * kNumXcd * n_slots;
}
__device__ inline bool xcd_tile_slot(uint32_t b, uint32_t n_tiles, uint32_t n_slots,
                                     uint32_t& tile, uint32_t& slot) {
    const uint32_t x = b % kNumXcd, q = b / kNumXcd;
    tile = (q / n_slots) * kNumXcd + x;
    slot = q % n_slots;
    return tile < n_tiles;
}

// One wavefront per chunk: the box of the chunk's disk centres and its largest radius.
__global__ __launch_bounds__(256) void k_chunk_box(const float4* __restrict__ pa_s, uint64_t n,
                                                   float4* __restrict__ cbox) {
    const uint64_t chunk = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (chunk >= (n + kChunk - 1) / kChunk) return;
    const uint64_t i = chunk * kChunk + lane;
    float lx = FLT_MAX, ly = FLT_MAX, lz = FLT_MAX, hx = -FLT_MAX, hy = -FLT_MAX, hz = -FLT_MAX;
    float r = 0.f;
    if (i < n) {
        const float4 a = gld(pa_s + i);
        lx = hx = a.x;
        ly = hy = a.y;
        lz = hz = a.z;
        r = a.w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lx = fminf(lx, __shfl_xor(lx, o));
        ly = fminf(ly, __shfl_xor(ly, o));
        lz = fminf(lz, __shfl_xor(lz, o));
        hx = fmaxf(hx, __shfl_xor(hx, o));
        hy = fmaxf(hy, __shfl_xor(hy, o));
        hz = fmaxf(hz, __shfl_xor(hz, o));
        r = fmaxf(r, __shfl_xor(r, o));
    }
    if (lane == 0) {
        cbox[2 * chunk] = make_float4(lx, ly, lz, r);
        cbox[2 * chunk + 1] = make_float4(hx, hy, hz, 0.f);
    }
}

void launch_chunk_box(const float4* pa_s, uint64_t n, float4* cbox, hipStream_t st) {
    const uint64_t n_chunks = (n + kChunk - 1) / kChunk;
    if (n_chunks == 0) return;
    hipLaunchKernelGGL(k_chunk_box, dim3((uint32_t)((n_chunks + 3) / 4)), dim3(256), 0, st, pa_s,
                       n, cbox);
}

// Pixel range of a chunk on one screen, from its box: the box's orthographic shadow widened by
// the largest disk (or the tube) radius.  It contains the footprint of every point of the
// chunk (the slack covers the rounding of the per-point projection), so the tiles it
// reaches hold every pixel the chunk can cover; the raster tests each point exactly.  One
// thread per (chunk, slot) reads 32 bytes, where projecting the chunk's points read 2 KiB.
constexpr float kBoxSlack = 1e-2f;  // pixels

__device__ inline void box_span(float4 lo, float4 hi, float e0, float e1, float e2, float& a,
                                float& b) {
    a = fminf(lo.x * e0, hi.x * e0) + fminf(lo.y * e1, hi.y * e1) + fminf(lo.z * e2, hi.z * e2);
    b = fmaxf(lo.x * e0, hi.x * e0) + fmaxf(lo.y * e1, hi.y * e1) + fmaxf(lo.z * e2, hi.z * e2);
}

__device__ inline int pix_floor(float x) { return (int)floorf(fminf(fmaxf(x, -1e8f), 1e8f)); }
__device__ inline int pix_ceil(float x) { return (int)ceilf(fminf(fmaxf(x, -1e8f), 1e8f)); }

__global__ __launch_bounds__(256) void k_chunk_bounds(const SlotDesc* __restrict__ ds,
                                                      int4* __restrict__ aabb,
                                                      uint32_t* __restrict__ tile_count,
                                                      uint32_t n_groups, uint32_t n_slots) {
    uint32_t group, slot;
    if (!xcd_unit_slot(blockIdx.x, n_groups, n_slots, group, slot)) return;
    const SlotDesc& d = ds[slot];
    const uint32_t chunk = group * 256 + threadIdx.x;
    if (chunk >= d.n_chunks) return;
    const Screen s = screen_of(d);
    const float4 lo = gld(d.cbox + 2 * (uint64_t)chunk), hi = gld(d.cbox + 2 * (uint64_t)chunk + 1);
    float ua, ub, va, vb;
    box_span(lo, hi, s.u0, s.u1, s.u2, ua, ub);
    box_span(lo, hi, s.v0, s.v1, s.v2, va, vb);
    const float e = (s.mode == 0 ? lo.w : s.tube_r) * s.ipitch + 1e-3f + kBoxSlack;
    int x0 = max(0, pix_ceil(ua * s.ipitch + s.hw - 0.5f - e));
    int x1 = min(s.W - 1, pix_floor(ub * s.ipitch + s.hw - 0.5f + e));
    int y0 = max(0, pix_ceil(va * s.ipitch + s.hh - 0.5f - e));
    int y1 = min(s.H - 1, pix_floor(vb * s.ipitch + s.hh - 0.5f + e));
    if (x0 > x1 || y0 > y1) { x0 = y0 = INT_MAX; x1 = y1 = INT_MIN; }
    aabb[d.chunk_base + chunk] = make_int4(x0, y0, x1, y1);
    if (x0 > x1) return;
    const int tx0 = x0 / d.tile, tx1 = x1 / d.tile, ty0 = y0 / d.tile, ty1 = y1 / d.tile;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++)
            atomicAdd(&tile_count[d.tile_base + ty * d.tiles_x + tx], 1u);
}

void launch_chunk_bounds(const SlotDesc* d, int n_slots, int max_chunks, int4* aabb,
                         uint32_t* tile_count, hipStream_t st) {
    const uint32_t groups = (uint32_t)(max_chunks + 255) / 256;
    hipLaunchKernelGGL(k_chunk_bounds, dim3(xcd_grid(groups, (uint32_t)n_slots)), dim3(256), 0, st,
                       d, aabb, tile_count, groups, (uint32_t)n_slots);
}

__global__ __launch_bounds__(256) void k_tile_scatter(const SlotDesc* __restrict__ ds,
                                                      const int4* __restrict__ aabb,
                                                      const uint32_t* __restrict__ tile_off,
                                                      uint32_t* __restrict__ cursor,
                                                      uint32_t* __restrict__ list,
                                                      uint32_t capacity,
                                                      uint32_t* __restrict__ overflow) {
    const SlotDesc& d = ds[blockIdx.y];
    const uint32_t chunk = blockIdx.x * 256 + threadIdx.x;
    if (chunk >= d.n_chunks) return;
    const int4 bb = aabb[d.chunk_base + chunk];
    if (bb.x > bb.z) return;
    const int tx0 = bb.x / d.tile, tx1 = bb.z / d.tile, ty0 = bb.y / d.tile, ty1 = bb.w / d.tile;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) {
            const uint32_t t = d.tile_base + ty * d.tiles_x + tx;
            const uint32_t pos = tile_off[t] + atomicAdd(&cursor[t], 1u);
            if (pos < capacity) list[pos] = chunk;
            else atomicOr(overflow, 1u);
        }
}

void launch_tile_scatter(const SlotDesc* d, int n_slots, int max_chunks, const int4* aabb,
                         const uint32_t* tile_off, uint32_t* tile_cursor, uint32_t* list,
                         uint32_t capacity, uint32_t* overflow, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_scatter, dim3((max_chunks + 255) / 256, n_slots), dim3(256), 0, st,
                       d, aabb, tile_off, tile_cursor, list, capacity, overflow);
}

template <int TILE>
__global__ __launch_bounds__(256) void k_raster(const SlotDesc* __restrict__ ds,
                                                const uint32_t* __restrict__ tile_off,
                                                const uint32_t* __restrict__ tile_count,
                                                const uint32_t* __restrict__ list,
                                                uint32_t capacity,
                                                uint64_t* __restrict__ keys, uint32_t n_tiles,
                                                uint32_t n_slots, uint32_t* __restrict__ live_count,
                                                uint32_t live_stride) {
    uint32_t utile, slot;
    if (!xcd_tile_slot(blockIdx.x, n_tiles, n_slots, utile, slot)) return;
    const SlotDesc& d = ds[slot];
    const int tile = (int)utile;
    if (tile >= d.tiles_x * d.tiles_y) return;
    __shared__ unsigned long long lk[TILE * TILE];
    for (int q = threadIdx.x; q < TILE * TILE; q += 256) lk[q] = kEmptyKey;
    __syncthreads();
    const Screen s = screen_of(d);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int px0 = tx * TILE, py0 = ty * TILE;
    const int px1 = min(px0 + TILE, s.W) - 1, py1 = min(py0 + TILE, s.H) - 1;
    const uint32_t beg = tile_off[d.tile_base + tile];
    const uint32_t cnt = tile_count[d.tile_base + tile];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float zoff = s.R;
    for (uint32_t e = wave; e < cnt; e += 4) {
        if (beg + e >= capacity) break;
        const uint32_t chunk = list[beg + e];
        const uint32_t i = chunk * kChunk + lane;
        if (i >= d.n_pts) continue;
        const float4 a = gld(d.pa_s + i), b = gld(d.pb_s + i);
        const Proj p = project(s, a, b);
        int x0, y0, x1, y1;
        footprint(s, p, x0, y0, x1, y1);
        x0 = max(x0, px0); x1 = min(x1, px1); y0 = max(y0, py0); y1 = min(y1, py1);
        if (x0 > x1 || y0 > y1) continue;
        const uint64_t idx = __float_as_uint(b.w);
        const float r2 = p.r * p.r;
        if (s.mode == 0) {
            const float ink = 1.0f / p.nk;
            const float tbase = p.xk + zoff;
            for (int y = y0; y <= y1; y++) {
                const float dv = (y + 0.5f - s.hh) * s.pitch - p.xb;
                for (int x = x0; x <= x1; x++) {
                    const float du = (x + 0.5f - s.hw) * s.pitch - p.xa;
                    const float dz = -(p.na * du + p.nb * dv) * ink;
                    if (du * du + dv * dv + dz * dz <= r2) {
                        const float t = tbase + dz;
                        if (t > 0.f) {
                            const uint64_t key = ((uint64_t)__float_as_uint(t) << 32) | idx;
                            atomicMin(&lk[(y - py0) * TILE + (x - px0)],
                                      (unsigned long long)key);
                        }
                    }
                }
            }
        } else {
            const float tc = p.xk + zoff;
            const float d2 = s.tube_r * s.tube_r;
            if (tc > 0.f) {
                const uint64_t key = ((uint64_t)__float_as_uint(tc) << 32) | idx;
                for (int y = y0; y <= y1; y++) {
                    const float dv = (y + 0.5f - s.hh) * s.pitch - p.xb;
                    for (int x = x0; x <= x1; x++) {
                        const float du = (x + 0.5f - s.hw) * s.pitch - p.xa;
                        if (du * du + dv * dv < d2)
                            atomicMin(&lk[(y - py0) * TILE + (x - px0)], (unsigned long long)key);
                    }
                }
            }
        }
    }
    __syncthreads();
    // 256 threads over TILE x TILE pixels: a wavefront's lanes cover 64 / TILE whole tile rows
    static_assert(256 % (TILE * TILE) == 0 || (TILE * TILE) % 256 == 0, "whole iterations");
    static_assert(64 % TILE == 0, "whole tile rows per wavefront");
    for (int q = threadIdx.x; q < TILE * TILE; q += 256) {
        const int x = px0 + q % TILE, y = py0 + q / TILE;
        const bool in = x < s.W && y < s.H;
        const uint64_t key = lk[q];
        if (in) keys[d.pix_base + (uint64_t)y * s.W + x] = key;
        if (live_count) {
            // a ray starts where the first hit is not an absorber (as the ray generation tests)
            const bool live = in && key != kEmptyKey &&
                              gld(d.pb + (uint32_t)(key & 0xFFFFFFFFu)).w == 0.f;
            const uint64_t bal = __ballot(live);
            const int lane = threadIdx.x & 63;
            if (lane % TILE == 0 && y < s.H) {
                const uint64_t run = (bal >> lane) & ((TILE == 64) ? ~0ull : ((1ull << TILE) - 1ull));
                const uint32_t c = (uint32_t)__popcll(run);
                if (c) {
                    const uint32_t blk = (uint32_t)(((uint64_t)y * s.W + px0) / 256);
                    atomicAdd(&live_count[(uint64_t)slot * live_stride + blk], c);
                }
            }
        }
    }
}

void launch_raster(const SlotDesc* d, int n_slots, int max_tiles, const uint32_t* tile_off,
                   const uint32_t* tile_count, const uint32_t* list, uint32_t capacity,
                   uint64_t* keys, int tile, uint32_t* live_count, uint32_t live_stride,
                   hipStream_t st) {
    const dim3 grid(xcd_tile_grid((uint32_t)max_tiles, (uint32_t)n_slots));
    if (tile == kTileWide)
        hipLaunchKernelGGL(k_raster<kTileWide>, grid, dim3(256), 0, st, d, tile_off, tile_count,
                           list, capacity, keys, (uint32_t)max_tiles, (uint32_t)n_slots,
                           live_count, live_stride);
    else
        hipLaunchKernelGGL(k_raster<kTile>, grid, dim3(256), 0, st, d, tile_off, tile_count, list,
                           capacity, keys, (uint32_t)max_tiles, (uint32_t)n_slots, live_count,
                           live_stride);
}

// Algorithm 1 with a K-point heap (TUBE slots): per pixel, the K candidates nearest the central
// ray (keys axis distance^2 | index) are found in K rounds of an LDS atomic minimum, each round
// taking the smallest key above the previous round's; the pixel's own thread keeps, among
// them, the point nearest the tube origin (|p - o|^2 = axis^2 + t_c^2; ties: lowest index) and
// writes the key (|p - o| | index).  Rounds stop early once no pixel of the tile has more.
__global__ __launch_bounds__(256) void k_raster_topk(const SlotDesc* __restrict__ ds,
                                                     const uint32_t* __restrict__ tile_off,
                                                     const uint32_t* __restrict__ tile_count,
                                                     const uint32_t* __restrict__ list,
                                                     uint32_t capacity, int K,
                                                     uint64_t* __restrict__ keys) {
    const SlotDesc& d = ds[blockIdx.y];
    const int tile = blockIdx.x;
    if (tile >= d.tiles_x * d.tiles_y) return;
    __shared__ unsigned long long cur[kTile * kTile];
    __shared__ unsigned long long thr[kTile * kTile];
    const Screen s = screen_of(d);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int px0 = tx * kTile, py0 = ty * kTile;
    const int px1 = min(px0 + kTile, s.W) - 1, py1 = min(py0 + kTile, s.H) - 1;
    const uint32_t beg = tile_off[d.tile_base + tile];
    const uint32_t cnt = tile_count[d.tile_base + tile];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float zoff = s.R, d2 = s.tube_r * s.tube_r;
    thr[threadIdx.x] = 0ull;
    float best_d = FLT_MAX;
    uint32_t best_i = kNone;
    for (int round = 0; round < K; round++) {
        cur[threadIdx.x] = kEmptyKey;
        __syncthreads();
        for (uint32_t e = wave; e < cnt; e += 4) {
            if (beg + e >= capacity) break;
            const uint32_t chunk = list[beg + e];
            const uint32_t i = chunk * kChunk + lane;
            if (i >= d.n_pts) continue;
            const float4 a = gld(d.pa_s + i), b = gld(d.pb_s + i);
            const Proj p = project(s, a, b);
            if (!(p.xk + zoff > 0.f)) continue;
            int x0, y0, x1, y1;
            footprint(s, p, x0, y0, x1, y1);
            x0 = max(x0, px0); x1 = min(x1, px1); y0 = max(y0, py0); y1 = min(y1, py1);
            const uint64_t idx = __float_as_uint(b.w);
            for (int y = y0; y <= y1; y++) {
                const float dv = (y + 0.5f - s.hh) * s.pitch - p.xb;
                for (int x = x0; x <= x1; x++) {
                    const float du = (x + 0.5f - s.hw) * s.pitch - p.xa;
                    const float a2 = du * du + dv * dv;
                    if (a2 < d2) {
                        const int q = (y - py0) * kTile + (x - px0);
                        const uint64_t key = ((uint64_t)__float_as_uint(a2) << 32) | idx;
                        if (key >= thr[q]) atomicMin(&cur[q], (unsigned long long)key);
                    }
                }
            }
        }
        __syncthreads();
        const uint64_t c = cur[threadIdx.x];
        if (c != kEmptyKey) {
            const uint32_t i = (uint32_t)(c & 0xFFFFFFFFu);
            const float a2 = __uint_as_float((uint32_t)(c >> 32));
            const float4 a = d.pa[i];
            const float tc = a.x * s.k0 + a.y * s.k1 + a.z * s.k2 + zoff;
            const float dist = sqrtf(a2 + tc * tc);
            if (dist < best_d || (dist == best_d && i < best_i)) {
                best_d = dist;
                best_i = i;
            }
            thr[threadIdx.x] = c + 1;
        } else {
            thr[threadIdx.x] = kEmptyKey;
        }
        if (!__syncthreads_or(c != kEmptyKey)) break;
    }
    const int lx = threadIdx.x & (kTile - 1), ly = threadIdx.x / kTile;
    const int x = px0 + lx, y = py0 + ly;
    if (x < s.W && y < s.H)
        keys[d.pix_base + (uint64_t)y * s.W + x] =
            best_i == kNone ? kEmptyKey : (((uint64_t)__float_as_uint(best_d) << 32) | best_i);
}

void launch_raster_topk(const SlotDesc* d, int n_slots, int max_tiles, const uint32_t* tile_off,
                        const uint32_t* tile_count, const uint32_t* list, uint32_t capacity, int K,
                        uint64_t* keys, hipStream_t st) {
    hipLaunchKernelGGL(k_raster_topk, dim3(max_tiles, n_slots), dim3(256), 0, st, d, tile_off,
                       tile_count, list, capacity, K, keys);
}

// Geometric frame buffer of slot 0: depth, oriented normal, index, mask.
__global__ void k_resolve(const SlotDesc* __restrict__ ds, const uint64_t* __restrict__ keys,
                          float* __restrict__ depth, float* __restrict__ nrm,
                          uint32_t* __restrict__ idx, uint8_t* __restrict__ mask, int npix) {
    const SlotDesc& d = ds[0];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const uint64_t key = keys[d.pix_base + p];
    if (key == kEmptyKey) {
        if (depth) depth[p] = __int_as_float(0x7f800000);
        if (idx) idx[p] = kNone;
        if (mask) mask[p] = 0;
        if (nrm) { nrm[3 * p] = 0.f; nrm[3 * p + 1] = 0.f; nrm[3 * p + 2] = 0.f; }
        return;
    }
    const uint32_t i = (uint32_t)(key & 0xFFFFFFFFu);
    if (depth) depth[p] = __uint_as_float((uint32_t)(key >> 32));
    if (idx) idx[p] = i;
    if (mask) mask[p] = 1;
    if (nrm) {
        const float4 b = d.pb[i];
        const float s = (b.x * d.k[0] + b.y * d.k[1] + b.z * d.k[2]) > 0.f ? -1.f : 1.f;
        nrm[3 * p] = s * b.x; nrm[3 * p + 1] = s * b.y; nrm[3 * p + 2] = s * b.z;
    }
}

void launch_resolve(const SlotDesc* d, const uint64_t* keys, float* depth, float* nrm,
                    uint32_t* idx, uint8_t* mask, int npix, hipStream_t st) {
    hipLaunchKernelGGL(k_resolve, dim3((npix + 255) / 256), dim3(256), 0, st, d, keys, depth, nrm,
                       idx, mask, npix);
}

// Aggregation view, level 0.  Pass 1: each pixel stores its front-most disk inline (so the
// march's 3x3 refinement reads contiguous rows) and that disk's depth extent along the view,
// centre depth +- r sqrt(1 - (n.k)^2).  Pass 2: the pyramid base (P x P) holds the min/max of
// those extents over each pixel's 3x3 neighbourhood; texels outside the screen are empty
// (min = +max float, max = -max float).
__global__ void k_view_pix(const SlotDesc* __restrict__ ds, int slot,
                           const uint64_t* __restrict__ keys, float4* __restrict__ pix,
                           float2* __restrict__ ext) {
    const SlotDesc& d = ds[slot];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.W * d.H) return;
    const uint64_t key = keys[d.pix_base + p];
    if (key == kEmptyKey) {
        pix[2 * p] = make_float4(0.f, 0.f, 0.f, 0.f);
        pix[2 * p + 1] = make_float4(0.f, 0.f, 0.f, __uint_as_float(kNone));
        ext[p] = make_float2(FLT_MAX, -FLT_MAX);
        return;
    }
    const uint32_t i = (uint32_t)(key & 0xFFFFFFFFu);
    const float4 a = d.pa[i], b = d.pb[i];
    pix[2 * p] = a;
    pix[2 * p + 1] = make_float4(b.x, b.y, b.z, __uint_as_float(i));
    const float tc = a.x * d.k[0] + a.y * d.k[1] + a.z * d.k[2] + d.R;
    const float nk = b.x * d.k[0] + b.y * d.k[1] + b.z * d.k[2];
    const float e = a.w * sqrtf(fmaxf(0.f, 1.f - nk * nk));
    ext[p] = make_float2(tc - e, tc + e);
}

__global__ void k_view_dilate(const float2* __restrict__ ext, int W, int H, int P,
                              float2* __restrict__ hiz0) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P * P) return;
    const int x = p % P, y = p / P;
    float mn = FLT_MAX, mx = -FLT_MAX;
    if (x < W && y < H) {
        for (int dy = -1; dy <= 1; dy++) {
            const int yy = y + dy;
            if (yy < 0 || yy >= H) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int xx = x + dx;
                if (xx < 0 || xx >= W) continue;
                const float2 v = ext[yy * W + xx];
                mn = fminf(mn, v.x);
                mx = fmaxf(mx, v.y);
            }
        }
    }
    hiz0[hiz_texel(P, x, y)] = make_float2(mn, mx);
}

void launch_view_level0(const SlotDesc* d, int slot, const uint64_t* keys, int W, int H, int P,
                        float4* pix, float2* ext, float2* hiz0, hipStream_t st) {
    hipLaunchKernelGGL(k_view_pix, dim3((W * H + 255) / 256), dim3(256), 0, st, d, slot, keys,
                       pix, ext);
    hipLaunchKernelGGL(k_view_dilate, dim3((P * P + 255) / 256), dim3(256), 0, st,
                       (const float2*)ext, W, H, P, hiz0);
}

__global__ void k_hiz_down(const float2* __restrict__ src, int sp, float2* __restrict__ dst) {
    const int dp = sp >> 1;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= dp * dp) return;
    const int x = p % dp, y = p / dp;
    const float2 a = src[hiz_texel(sp, 2 * x, 2 * y)], b = src[hiz_texel(sp, 2 * x + 1, 2 * y)];
    const float2 c = src[hiz_texel(sp, 2 * x, 2 * y + 1)];
    const float2 d = src[hiz_texel(sp, 2 * x + 1, 2 * y + 1)];
    dst[hiz_texel(dp, x, y)] = make_float2(fminf(fminf(a.x, b.x), fminf(c.x, d.x)),
                                           fmaxf(fmaxf(a.y, b.y), fmaxf(c.y, d.y)));
}

void launch_hiz_down(const float2* src, int sp, float2* dst, hipStream_t st) {
    const int dp = sp >> 1;
    hipLaunchKernelGGL(k_hiz_down, dim3((dp * dp + 255) / 256), dim3(256), 0, st, src, sp, dst);
}

}  // namespace pe
