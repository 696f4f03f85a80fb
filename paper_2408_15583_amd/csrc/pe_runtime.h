// Host-side runtime structures of the SBR library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pe_device.h"
#include "pointemray.h"

namespace pe {

struct Error {
    pe_status status;
    std::string msg;
};

extern thread_local std::string g_err;
pe_status set_error(pe_status s, const std::string& m);
void hip_check(hipError_t e, const char* what, int line);
#define HIPCHK(x) ::pe::hip_check((x), #x, __LINE__)

void screen_basis(const double kin[3], double u[3], double v[3], double k[3]);
void pol_basis(const double s[3], double th[3], double ph[3]);

void* ctx_alloc(pe_ctx ctx, size_t bytes);
void ctx_free(pe_ctx ctx, void* p, size_t bytes);
void ctx_release_cache(pe_ctx ctx);

// Growable set of device buffers charged to a context's budget.  In arena mode (arena !=
// nullptr) nothing is allocated: buffers are carved in request order from a fixed device
// region owned by someone else, and running past its end throws PE_ENOMEM.
struct Workspace {
    struct Buf {
        void* p = nullptr;
        size_t cap = 0;
    };
    pe_ctx ctx = nullptr;
    Buf bufs[44];
    uint8_t* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    explicit Workspace(pe_ctx c) : ctx(c) {}
    Workspace(pe_ctx c, void* region, size_t cap)
        : ctx(c), arena((uint8_t*)region), arena_cap(cap) {}
    ~Workspace() { release(); }
    void* raw(int id, size_t bytes);
    template <class T>
    T* get(int id, uint64_t count) {
        return (T*)raw(id, (size_t)count * sizeof(T));
    }
    void release();
    // Arena mode: forgets every buffer so that the next batch carves its own from the start
    // (no-op for allocated workspaces, whose buffers are kept and grown).
    void begin_batch();
    uint64_t bytes() const;
};

// One screen of one incidence on one scene.
struct SlotSpec {
    pe_scene sc = nullptr;
    double k[3] = {0, 0, -1};
    int W = 0, H = 0;
    int mode = PE_SPLAT_DISK;
    double tube_r = 0;
    int max_b = 1;
    double eps = 0;
    int n_obs = 1;
    const double* obs = nullptr;  // null: monostatic
    int n_freq = 1;
    const double* freq = nullptr;
};

struct Batch {
    Workspace& ws;
    hipStream_t st;
    std::vector<SlotSpec> spec;
    std::vector<SlotDesc> hd;
    std::vector<ObsDesc> ho;
    std::vector<double> hf;
    SlotDesc* dd = nullptr;
    ObsDesc* dobs = nullptr;
    double* dfreq = nullptr;
    uint32_t* cnt = nullptr;
    uint32_t* scan_ws = nullptr;  // per-tile totals of the wide scans
    int n = 0, contrib = 0, precision = 0, n_seg = 1, ft = 1, max_b = 1;
    int topk = 0;  // > 0: TUBE slots keep a K-point heap (Algorithm 1) instead of K unbounded
    // PE_SECONDARY_SPLATS: bounces and visibility against every splat through the scene's
    // object-space hierarchy; PE_SECONDARY_VIEWS: through the aggregation views
    int secondary = 0;
    int bvh_depth = 1;  // LDS stack entries per lane of the hierarchy traversals
    bool blend = false;  // some slot's scene refines hits by Eq. (23)
    bool live_counted = false;  // the raster counted each block's ray-starting pixels
    int max_chunks = 0, max_tiles = 0, max_pix = 0, max_obs = 1, max_freq = 1, tot_out = 0;
    uint64_t tot_pix = 0;
    uint32_t tot_tiles = 0, tot_chunks = 0, tlist_cap = 0, rec_stride = 0;
    uint64_t* keys = nullptr;
    RayState rs{};
    uint32_t* lists[3] = {nullptr, nullptr, nullptr};
    uint8_t* alive = nullptr;
    uint64_t* hitkey = nullptr;
    int max_views = 0;
    uint32_t *ccount = nullptr, *coff = nullptr, *seg_beg = nullptr, *seg_cnt = nullptr;
    ExitRecs er{};

    Batch(Workspace& w, hipStream_t s);
    void setup(const std::vector<SlotSpec>& slots, int contrib, int precision);
    void splat();
    void alloc_rays();
    void raygen();
    // Primary rays from a GFB on every slot's screen (depth t/D, view-frame normals, hit
    // probability >= thresh) instead of the splat keys; slots with use[s] == 0 get none.
    void raygen_gfb(const float* depth, const float* nrm, const float* prob, const uint8_t* use,
                    float thresh);
    void alloc_records();
    void records(int seg, const uint32_t* list, const uint32_t* n_list);
    void trace(bool with_records);
    void field(double* E_host, double* rcs_host);
    void read_counters(uint32_t* host);
    double queries(const uint32_t* c) const;
    double records_made(const uint32_t* c) const;
    double march_rays(const uint32_t* c) const;
    double march_hits(const uint32_t* c) const;
    bool overflowed(const uint32_t* c);
    struct Pending {
        const char* name;
        hipEvent_t e0, e1;
    };
    std::vector<Pending> pend;
    hipEvent_t pend_begin = nullptr;
    void prof_begin();
    void prof_end(const char* name);
    void prof_flush();
    ~Batch() {
        try {
            prof_flush();
        } catch (...) {
        }
    }
};

constexpr int kNumCounters = 7 + 64;
constexpr int kCounterCap = 6;
constexpr int kMaxBounces = 16;

struct Server;
struct Densifier;

}  // namespace pe

namespace pe {
// Fixed per-device scratch of the no-allocation solve (noalloc.hip): looked up once per device
// by pe_ctx_create with the device current.
void scratch_init(int device);
}  // namespace pe

struct pe_ctx_s {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    // Device blocks released by ctx_free, kept for reuse by an allocation of the same rounded
    // size (scenes and their build buffers come and go with the same sizes in steady serving).
    // `used` counts live blocks only; used + cached stays within the budget and cached within
    // kCacheCap.  A block freed at generation g is handed out again only after a device
    // synchronisation (idle_gen > g): its last kernels may still run on any stream.
    struct CachedBlock {
        void* p;
        uint64_t gen;
    };
    std::mutex alloc_mu;
    std::multimap<size_t, CachedBlock> cache;
    uint64_t cached = 0;
    uint64_t idle_gen = 0;
    std::mutex mu;  // serialises synchronous calls that use the default workspace
    pe::Workspace* ws = nullptr;
    pe::Server* server = nullptr;
    std::mutex server_mu;
    bool profile = false;
    std::mutex prof_mu;
    std::map<std::string, std::pair<double, uint64_t>> ktab;  // kernel -> (total ms, launches)
};

struct pe_scene_s {
    pe_ctx ctx = nullptr;
    std::atomic<int> refs{0};  // server requests holding this scene until they finish
    uint64_t n = 0;
    double c[3] = {0, 0, 0};
    double R = 0, r_max = 0;
    float4 *pa = nullptr, *pb = nullptr, *pa_s = nullptr, *pb_s = nullptr;
    float4* cbox = nullptr;  // per-chunk bounding boxes of pa_s
    std::vector<pe::ViewDesc> views;
    pe::ViewDesc* views_dev = nullptr;
    float4* bvh = nullptr;  // object-space hierarchy over pa_s (node records at pe::kBvhLeaf)
    uint64_t bvh_nodes = 0;
    int bvh_levels = 1;  // octree levels: the traversal's stack holds at most one entry each
    uint4* wrec = nullptr;     // wide records of the internal nodes (pe::kWideRec)
    float4* wpts = nullptr;    // the points in leaf order, 2 float4 each
    uint32_t w_root_pts = 0;   // points of the root when it is a leaf
    float bvh_root[6] = {0, 0, 0, 0, 0, 0};  // the root's box: low x, y, z, high x, y, z
    float blend_r = 0.f, bl_h = 0.f;  // Eq. (23) refinement radius and centre-grid cell edge
    int bl_G = 0;
    uint32_t *bl_start = nullptr, *bl_items = nullptr;
    std::vector<std::pair<void*, size_t>> allocs;
    uint64_t bytes = 0;
    void* alloc(size_t b) {
        void* p = pe::ctx_alloc(ctx, b);
        allocs.push_back({p, b});
        bytes += (b + 255) & ~(size_t)255;
        return p;
    }
    ~pe_scene_s() {
        for (auto& a : allocs) pe::ctx_free(ctx, a.first, a.second);
    }
};

// Exception barrier of every C entry point: no C++ exception crosses the ABI.
#define API_BEGIN try {
#define API_END                                                              \
    }                                                                        \
    catch (const ::pe::Error& e) {                                                 \
        return ::pe::set_error(e.status, e.msg);                                   \
    }                                                                        \
    catch (const std::bad_alloc&) {                                          \
        return ::pe::set_error(PE_ENOMEM, "host allocation failed");               \
    }                                                                        \
    catch (const std::exception& e) {                                        \
        return ::pe::set_error(PE_EDEVICE, std::string("internal error: ") + e.what()); \
    }                                                                        \
    catch (...) {                                                            \
        return ::pe::set_error(PE_EDEVICE, "internal error");                      \
    }

namespace pe {
typedef void (*solve_fn)(Workspace& ws, hipStream_t st, pe_scene sc, const pe_solve_desc* d,
                         double* E, double* rcs, pe_stats* acc);
extern solve_fn g_densified_solve;
void validate_solve(pe_scene sc, const pe_solve_desc* d, bool need_scene = true);
// Device bytes per pixel of a plain batch (before headroom), and the incidences per batch of a
// synchronous solve.
uint64_t batch_bytes_per_pixel(const pe_solve_desc* d);
int slots_per_batch(pe_ctx ctx, const pe_solve_desc* d);
std::vector<SlotSpec> make_slots(pe_scene sc, const pe_solve_desc* d, int i0, int count);
void run_field_batch(Workspace& ws, hipStream_t st, const std::vector<SlotSpec>& slots,
                     int contrib, int precision, double* E_host, double* rcs_host,
                     pe_stats* acc, int secondary = PE_SECONDARY_VIEWS);
}  // namespace pe
