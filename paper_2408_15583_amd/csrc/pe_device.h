// Internal structures shared by the HIP kernels and the host runtime of the SBR library.
// Geometry lives in the scene frame: positions relative to the bounding-box centre c, in fp32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe {

constexpr int kChunk = 64;          // points per spatial chunk (one wavefront)
constexpr int kTile = 16;           // screen tile edge (pixels) of the K-point-heap raster
constexpr int kTileWide = 32;       // screen tile edge of the nearest-hit raster
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kEmptyKey = ~0ull;
constexpr float kGraze = 1e-6f;     // |n.k| below this is a miss (grazing)
constexpr int kSlotBits = 10;       // list entry = slot << 22 | pixel
constexpr int kPixBits = 22;
constexpr int kMaxLevels = 14;
constexpr int kMaxSlots = 1 << kSlotBits;
constexpr int kMaxNormalK = 64;   // largest neighbourhood of the PCA normal estimate
constexpr int kWaveChunk = 64;    // live-list entries per compaction chunk (one wavefront)

// One aggregation view of a scene: a disk first-hit buffer with its min/max depth pyramid.
// The min/max pyramid is stored square and power-of-two: level l is (P >> l)^2 texels at
// offset 4 (P^2 - (P >> l)^2) / 3, so a march step needs no table lookup before its fetch.
struct ViewDesc {
    float u[3], v[3], k[3];   // screen basis: u, v span the screen, k = propagation
    float pitch, R;
    int W, H, levels;         // levels = log2(P) + 1
    int P, lp;                // pyramid side (power of two >= max(W, H)) and log2(P)
    const float4* pix;        // W*H x 2: the pixel's front-most disk (x, y, z, r),
                              // (nx, ny, nz, bits(point index)); index kNone = empty pixel
    const float2* hiz;        // all levels; level 0 (P x P): min/max over the pixel's 3x3
                              // neighbourhood of each stored disk's depth extent
};

// Loads through the global address space.  Pointers read from descriptors or kept in per-lane
// state are generic to the compiler, which would otherwise emit flat loads (slower, and counted
// on two waitcnt queues); the load goes through a native clang vector because HIP's float2 and
// float4 copy through a generic reference.
__device__ inline float4 gld(const float4* p) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 r = *(const __attribute__((address_space(1))) v4*)p;
    return make_float4(r.x, r.y, r.z, r.w);
}
__device__ inline float2 gld(const float2* p) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 r = *(const __attribute__((address_space(1))) v2*)p;
    return make_float2(r.x, r.y);
}

__host__ __device__ inline uint32_t hiz_offset(int P, int l) {
    const uint32_t a = (uint32_t)P * (uint32_t)P, b = (uint32_t)(P >> l) * (uint32_t)(P >> l);
    return 4u * ((a - b) / 3u);
}

// Texel (x, y) of a level of side w: levels of side >= 4 are stored in 4x4 tiles (16 texels,
// 128 B, one cache line) so a ray crossing a tile in any direction stays in one line.
__host__ __device__ inline uint32_t hiz_texel(int w, int x, int y) {
    if (w < 4) return (uint32_t)(y * w + x);
    return (uint32_t)((((y >> 2) * (w >> 2) + (x >> 2)) << 4) | ((y & 3) << 2) | (x & 3));
}

constexpr int kNumXcd = 8;  // MI355X: workgroups are dealt round-robin to 8 XCDs, each with its L2

// Object-space hierarchy over a scene's points in Morton order (an octree of their 30-bit codes):
// node = the points sharing a code prefix of 3 l bits at level l; a node of at most kBvhLeaf
// points is a leaf; past the 30 bits (level 10) a node of more points is split by count into
// up to 8 chunks, again and again.  Node record: 2 float4, (lo xyz, bits(first)), (hi xyz,
// bits(info)); info bit 31 = leaf with (info & 0xFFFFFF) points from pa_s[first]; else children
// nodes first .. first + popc(occ) - 1 for the occupied octants occ = info & 0xFF (octant = the
// 3 code bits below the prefix, x in bit 0; chunk number past the code), stored in increasing
// octant order.  The root is node 0.
//
// Wide records (what the traversal reads): one record of kWideRec uint4 per internal node, in
// node order (so the internal children of a node have consecutive record indices):
//   [0] origin x, y, z (the node's box low corner, fp32 bits); w = e_x | e_y << 8 | e_z << 16 |
//       occ << 24, with the per-axis scale 2^(e - 127) (biased fp32 exponent) and occ the
//       octant mask of the children;
//   [1] x = record index of the first internal child, y = wpts index of the first point of the
//       leaf children, z = octant mask of the internal children, w = 4-bit point count of the
//       leaf child in each octant (0 for internal or empty octants);
//   [2..4] child boxes by octant, 8-bit coordinates q (plane = origin + q scale, rounded
//       outward so each contains the child's exact box): low x[8], low y[8], low z[8], high
//       x[8], high y[8], high z[8] bytes.
// wpts holds every point once (2 float4 as pa_s / pb_s), the leaf children of each node
// consecutively in octant order; when the root is itself a leaf its points come first and
// there is no record.
constexpr int kBvhLeaf = 8;
constexpr uint32_t kBvhLeafBit = 0x80000000u;
constexpr int kWideRec = 5;
constexpr int kBvhMaxLevels = 20;  // 10 code levels + count splits of up to 2^31 points
constexpr int kBvhMaxStack = kBvhMaxLevels;  // one stack entry per level

// One work item of a batched launch: one screen (one incidence) on one scene.
struct SlotDesc {
    // scene
    const float4* pa_s;       // spatially ordered (x, y, z, r)
    const float4* pb_s;       // spatially ordered (nx, ny, nz, bits(original index))
    const float4* cbox;       // per chunk of pa_s: (lo x, y, z, max r), (hi x, y, z, 0)
    const float4* pa;         // original order (x, y, z, r)
    const float4* pb;         // original order (nx, ny, nz, material)
    const ViewDesc* views;
    uint32_t n_pts, n_chunks;
    int n_views;
    float R, r_max;
    // screen
    float u[3], v[3], k[3];
    float pitch;
    int W, H, tiles_x, tiles_y;
    int tile;                 // screen tile edge (kTile or kTileWide), one workgroup per tile
    int mode;                 // 0 disk, 1 tube
    float tube_r;
    // buffers
    uint64_t pix_base;        // into per-pixel arrays of the batch
    uint32_t tile_base;       // into per-tile arrays of the batch
    uint32_t chunk_base;      // into per-chunk arrays of the batch
    // field
    float eth[3], eph[3];     // transmit polarisations (theta, phi of -k)
    float eps;
    int max_b;
    int n_obs, obs_base;      // observation descriptors [obs_base, obs_base + n_obs)
    int mono;
    int n_freq, freq_base;
    int out_base;             // output index of (slot, obs 0, freq 0)
    // Eq. (23) overlap refinement (blend_r > 0): uniform grid of G^3 cells of edge bl_h over
    // [-R, R]^3, CSR lists of splat indices by centre
    float blend_r, bl_h;
    int bl_G;
    const uint32_t* bl_start;
    const uint32_t* bl_items;
    // object-space hierarchy over pa_s (secondary hits and visibility against every splat),
    // node records and wide records as described at kBvhLeaf
    const float4* bvh;
    const uint4* wrec;
    const float4* wpts;
    uint32_t w_root_pts;  // points of the root when it is a leaf, else 0
    float bvh_lo[3], bvh_hi[3];  // the root's box (as in its node record)
};

struct ObsDesc {
    float ks[3];              // scattered propagation direction
    float eth[3], eph[3];     // receive polarisations (theta, phi of ks)
    double dc;                // (k_i - k_s) . c: phase offset of the scene frame (m)
};

// Ray state, structure of arrays indexed by batch pixel.  The state of a live ray is the
// record of its last bounce: hit point, oriented normal, incoming direction, incoming fields
// for both transmit polarisations, incoming tube vectors, image-method path length to x.  A
// primary record (bounce count 1) does not store the incoming direction, fields and tube
// vectors: they are its slot's direction, transmit polarisations and screen axes times the
// pixel pitch.
enum RayComp { RX = 0, RNX = 3, RKX = 6, RETX = 9, REPX = 12, RUX = 15, RVX = 18, RNCOMP = 21 };
struct RayState {
    float* f[RNCOMP];
    double* d;
    uint8_t* m;               // bounce count of the record
    uint32_t* hit;            // point index of the record's facet
};

// Exit (facet) record: frequency-independent part of one term of Eq. (14), 32 bytes (written
// and read as two 16-byte halves).
struct __attribute__((aligned(16))) ExitRec {
    double D;                 // d - k_s . x (scene frame)
    float al;                 // (k_in - k_s) . u' / 2
    float be;                 // (k_in - k_s) . v' / 2
    float A[4];               // psi * area * V . e_rx for (rx, tx) = (t,t), (t,p), (p,t), (p,p)
};
struct ExitRecs {
    ExitRec* rec;
};

__host__ __device__ inline uint32_t entry_slot(uint32_t e) { return e >> kPixBits; }
__host__ __device__ inline uint32_t entry_pix(uint32_t e) { return e & ((1u << kPixBits) - 1); }
__host__ __device__ inline uint32_t make_entry(uint32_t s, uint32_t p) {
    return (s << kPixBits) | p;
}

}  // namespace pe

// ----------------------------------------------------------------------------------------------
// Kernel launchers (defined next to their kernels).  All are asynchronous on `st`.
// ----------------------------------------------------------------------------------------------
namespace pe {

// generic
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st);
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t st);
// exclusive scan of n items (n = n_static, or ceil(*n_dev / div) if n_dev); writes total.
void launch_scan(const uint32_t* in, uint32_t* out, uint32_t n_static, const uint32_t* n_dev,
                 uint32_t div, uint32_t* total, hipStream_t st);
// The same scan by one workgroup per 16 Ki items, for large n: n = n_max, or
// min(n_max, ceil(*n_dev / div)) if n_dev (n_max sizes the grid).  scratch holds
// scan_wide_scratch(n_max) u32 (per-tile totals).
uint32_t scan_wide_scratch(uint32_t n_max);
void launch_scan_wide(const uint32_t* in, uint32_t* out, uint32_t n_max, const uint32_t* n_dev,
                      uint32_t div, uint32_t* total, uint32_t* scratch, hipStream_t st);

// ingest
void launch_ingest_stats(const void* xyz, int is_f64, const float* nrm, const uint8_t* mat,
                         const float* rad, float rad_scalar, uint64_t n, double* partial,
                         int n_blocks, hipStream_t st);
void launch_ingest_pack(const void* xyz, int is_f64, const float* nrm, const uint8_t* mat,
                        const float* rad, float rad_scalar, uint64_t n, double cx, double cy,
                        double cz, float4* pa, float4* pb, double* partial, int n_blocks,
                        hipStream_t st);
// Spatial order of a scene (k_sort.hip): sorts the points by the Morton code of a 1024^3 grid
// whose cells have edge 1 / inv_cell from (lo_x, lo_y, lo_z), writing pa_s / pb_s (original
// index in pb_s.w).  keys: 4 n u32 of scratch, the sorted codes end in keys[n .. 2n); temp:
// morton_sort_temp_bytes(n) bytes (digit counts, their offsets and the scan's tile totals).
size_t morton_sort_temp_bytes(uint64_t n);
hipError_t launch_morton_sort(const float4* pa, const float4* pb, uint64_t n, float lo_x,
                              float lo_y, float lo_z, float inv_cell, uint32_t* keys,
                              void* temp, size_t temp_bytes, float4* pa_s, float4* pb_s,
                              hipStream_t st);

// Bounding box of each kChunk-point chunk of pa_s (2 float4 per chunk, see SlotDesc::cbox).
void launch_chunk_box(const float4* pa_s, uint64_t n, float4* cbox, hipStream_t st);

// splat pipeline for a batch of slots
void launch_chunk_bounds(const SlotDesc* d, int n_slots, int max_chunks, int4* aabb,
                         uint32_t* tile_count, hipStream_t st);
void launch_tile_scatter(const SlotDesc* d, int n_slots, int max_chunks, const int4* aabb,
                         const uint32_t* tile_off, uint32_t* tile_cursor, uint32_t* list,
                         uint32_t capacity, uint32_t* overflow, hipStream_t st);
// tile: the batch's screen tile edge (every slot's SlotDesc::tile; kTile or kTileWide).
// live_count (or null): per slot and 256-pixel block of its row-major pixels, the number of
// pixels whose first hit starts a ray (a hit on a non-absorber), added as the tiles finish
// (zeroed by the caller; every slot's W a multiple of the tile edge, so a tile row lies in one
// block); the ray generation's count, at live_stride blocks per slot.
void launch_raster(const SlotDesc* d, int n_slots, int max_tiles, const uint32_t* tile_off,
                   const uint32_t* tile_count, const uint32_t* list, uint32_t capacity,
                   uint64_t* keys, int tile, uint32_t* live_count, uint32_t live_stride,
                   hipStream_t st);
void launch_resolve(const SlotDesc* d, const uint64_t* keys, float* depth, float* nrm,
                    uint32_t* idx, uint8_t* mask, int npix, hipStream_t st);
void launch_view_level0(const SlotDesc* d, int slot, const uint64_t* keys, int W, int H, int P,
                        float4* pix, float2* ext, float2* hiz0, hipStream_t st);
void launch_hiz_down(const float2* src, int sp, float2* dst, hipStream_t st);

// trace
void launch_raygen_count(const SlotDesc* d, int n_slots, int max_pix, const uint64_t* keys,
                         uint32_t* wg_count, hipStream_t st);
void launch_raygen_write(const SlotDesc* d, int n_slots, int max_pix, const uint64_t* keys,
                         const uint32_t* wg_off, uint32_t* list, RayState rs, uint64_t* hitkey,
                         hipStream_t st);
// queue: kNumXcd u32 work counters (cleared by the launcher).
// Object-space hierarchy, built one level at a time from the sorted codes.  A level's nodes are
// point ranges rng[j] = (a, b); count pass: child count and octant mask (or count split) of each
// node; emit pass (after an exclusive scan of the counts, cbase = global index of the next
// level's first node): the next level's ranges and each node's (first, info); box pass (deepest
// level first): each node's box into its record (pad widens leaf boxes: fp32 slack of the
// ray-box test).
void launch_bvh_count(const uint2* rng, uint32_t n_nodes, int level, const uint32_t* codes,
                      uint32_t* ccount, hipStream_t st);
void launch_bvh_emit(const uint2* rng, uint32_t n_nodes, int level, const uint32_t* codes,
                     const uint32_t* coff, uint32_t cbase, uint2* rng_next, uint2* finfo,
                     hipStream_t st);
void launch_bvh_box(const uint2* finfo, uint32_t n_nodes, uint32_t base, const float4* pa_s,
                    const float4* pb_s, float pad, float4* nodes, hipStream_t st);
// Wide records from the finished node records: count pass (is_int[g] = node g is internal,
// leafpts[g] = points of its leaf children), then, after exclusive scans of both into rec and
// lbase, the emit pass writes each internal node's record at rec[g] and copies its leaf
// children's points to wpts from lbase[g] (a leaf root copies its points to wpts[0..]).
void launch_wide_count(const float4* nodes, uint32_t n_nodes, uint32_t* is_int,
                       uint32_t* leafpts, hipStream_t st);
void launch_wide_emit(const float4* nodes, uint32_t n_nodes, const uint32_t* rec,
                      const uint32_t* lbase, const float4* pa_s, const float4* pb_s,
                      uint4* wrec, float4* wpts, hipStream_t st);

// Visibility of facets against every splat, as a dense pass: mark the entries of list whose
// facet needs a traced Psi (every facet of a bistatic slot, the later-bounce facets of a
// monostatic one; alive[e], and per-64-entry chunk counts for the order-preserving compaction);
// then, over the compacted list x the slot's observation directions, vis[o * vis_stride +
// pixel] = 1 iff no disk is hit from the facet toward k_s(o) beyond eps.
void launch_psi_mark(const SlotDesc* d, const uint32_t* list, const uint32_t* n_list,
                     RayState rs, uint8_t* alive, uint32_t* chunk_count, int n_blocks,
                     hipStream_t st);
void launch_psi_trace(const SlotDesc* d, const ObsDesc* obs, const uint32_t* list,
                      const uint32_t* n_list, int max_obs, RayState rs, uint8_t* vis,
                      uint64_t vis_stride, int stack_depth, uint32_t* queue, int refill,
                      int n_blocks, hipStream_t st);
// Nearest hit beyond eps of every live ray against all of its scene's splats (the hierarchy
// above), written to hitkey[entry] (kEmptyKey when none).  stack_depth: the batch's largest
// octree level count (<= kBvhMaxStack), u64 LDS entries per thread.  Both traversal passes are
// persistent: queue is one u32 work counter (cleared by the launcher), and a wavefront refills
// its idle lanes once `refill & 0xFF` (1 .. 64) of them are idle; with a quorum q = refill >> 8
// above 0 it takes one kind of step per iteration (point tests once q lanes hold points, else
// node expansions), with 0 each lane its own.
void launch_trace_bvh(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live,
                      RayState rs, uint64_t* hitkey, int bounce, int stack_depth,
                      uint32_t* queue, int refill, int n_blocks, hipStream_t st);
void launch_march(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live, RayState rs,
                  uint64_t* hitkey, int bounce, int max_views, uint32_t* cap_hits, uint32_t* queue,
                  int n_blocks, hipStream_t st);
// Eq. (23): centre grid of a scene's splats, and the refinement/blend pass over a live list.
void launch_blend_grid(const float4* pa, uint64_t n, float R, float h, int G, uint32_t* cell_of,
                       uint32_t* counts, uint32_t* start, uint32_t* cursor, uint32_t* items,
                       hipStream_t st);
void launch_blend(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live, RayState rs,
                  int primary, int n_blocks, hipStream_t st);
// PCA normals: bounding box partials (7 doubles per block: lo xyz, hi xyz, non-finite count),
// grid of G^3 cells of edge h from lo (box-centred frame), k-nearest PCA.
void launch_nrm_bbox(const void* xyz, int is_f64, uint64_t n, double* partial, int nb,
                     hipStream_t st);
void launch_nrm_grid(const void* xyz, int is_f64, uint64_t n, const double c[3], float lo,
                     float h, int G, float4* p, float4* ps, uint32_t* cell_of, uint32_t* counts,
                     uint32_t* start, uint32_t* cursor, hipStream_t st);
void launch_nrm_pca(const float4* p, uint64_t n, const float4* ps, const uint32_t* start,
                    float lo, float h, int G, int k, float* nrm, hipStream_t st);
void launch_bounce_apply(const SlotDesc* d, const uint32_t* list, const uint32_t* n_live,
                         RayState rs, uint64_t* hitkey, uint8_t* alive, uint32_t* chunk_count,
                         int bounce, int reset_keys, int n_blocks, hipStream_t st);
void launch_compact(const uint32_t* list_in, const uint32_t* n_in, const uint8_t* alive,
                    const uint32_t* chunk_off, uint32_t* list_out, int n_blocks,
                    hipStream_t st);
void launch_trace_out(const SlotDesc* d, const uint32_t* list, const uint32_t* n_list,
                      RayState rs, int32_t* n_bounce, float* last_x, float* last_n,
                      double* path, uint32_t* last_idx, int n_blocks, hipStream_t st);

// physical optics
constexpr int kRT = 1024;  // facet records per PO tile
// splats != 0: visibility against every splat from the visibility pass (vis, see
// launch_psi_trace); else through the aggregation views / incidence first-hit buffer.
void launch_po_prep(const SlotDesc* d, const ObsDesc* obs, const uint32_t* list,
                    const uint32_t* n_list, RayState rs, const uint64_t* keys, ExitRecs er,
                    uint32_t rec_stride, int seg, int n_seg, uint32_t* cap_hits, int splats,
                    const uint8_t* vis, uint64_t vis_stride, int n_blocks, hipStream_t st);
void launch_slot_ranges(const uint32_t* list, const uint32_t* n_list, int n_slots,
                        uint32_t* beg, uint32_t* cnt, hipStream_t st);
// tile_prefix gets n_seg*n_slots+1 entries (exclusive prefix, total last); tmp same size.
void launch_po_tiles(const SlotDesc* d, const uint32_t* seg_cnt, int n_seg, int n_slots, int ft,
                     uint32_t* tmp, uint32_t* tile_prefix, hipStream_t st);
void launch_po_sum(const SlotDesc* d, const uint32_t* seg_beg, const uint32_t* seg_cnt,
                   int n_seg, int n_slots, const double* freq, ExitRecs er, uint32_t rec_stride,
                   const uint32_t* tile_prefix, int fp32, int ft, double* partial, int n_blocks,
                   hipStream_t st);
void launch_po_reduce(const SlotDesc* d, const ObsDesc* obs, int n_slots, int max_obs,
                      int max_freq, int n_seg, const double* freq, const uint32_t* seg_cnt,
                      const uint32_t* tile_prefix, int ft, const double* partial, int fp32,
                      double* E_out, double* rcs_out, hipStream_t st);

}  // namespace pe
