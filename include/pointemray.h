/*
 * pointemray.h -- C ABI of the MI355X point-cloud shooting-and-bouncing-ray (SBR) library.
 *
 * The problem statement follows the paper: a point cloud carrying normals (PEC targets,
 * plane-wave excitation, far field, no diffraction -- Sec. I and Sec. II) is intersected by a
 * screen of central rays (Sec. III-A, Algorithm 1), rays bounce across the geometry recovered
 * from several views (Sec. III-B, Algorithm 3), and the scattered field is the sum of
 * physical-optics facet integrals of each ray's last facet (Sec. II-B/C, Eq. (11)-(14)).
 *
 * Conventions (all entry points):
 *   - Units are SI.  Directions are unit 3-vectors in double precision.  An incidence
 *     direction is the PROPAGATION direction k_i of the incident plane wave; the monostatic
 *     observation direction is k_s = -k_i.  |E_i| = 1; fields have the far-field factor
 *     exp(-jkr)/r removed; time convention exp(+jwt).
 *   - Polarisation basis of a direction s: theta-hat, phi-hat of the spherical angles of s.
 *     Transmit polarisations use s = -k_i, receive polarisations use s = k_s.
 *   - Every call returns pe_status: PE_OK (0) or a negative error.  On error no output is
 *     written and pe_last_error() describes the failure.  No C++ exception crosses the ABI.
 *   - Device pointers are accessed on the given HIP stream (a hipStream_t passed as void*,
 *     NULL = the null stream).  Host pointers are read/written before the call returns.
 *   - The caller owns every buffer it passes.  Handles own their device memory.
 *   - A pe_ctx binds one HIP device; calls on one context may come from several threads
 *     (internally serialised); pe_submit/pe_wait/pe_cancel are designed for concurrent use.
 */
#ifndef POINTEMRAY_H
#define POINTEMRAY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pe_status;
#define PE_OK 0
#define PE_EINVAL (-1)       /* bad argument: NaN/inf position, zero normal, bad flag, zero size */
#define PE_ENOMEM (-2)       /* footprint above the context's HBM budget (nothing allocated) */
#define PE_EDEVICE (-3)      /* HIP runtime error; the context stays usable */
#define PE_EUNSUPPORTED (-4) /* valid but not implemented combination */
#define PE_EBUSY (-5)        /* resource still in use (a scene held by unfinished requests) */
#define PE_ECANCELED (-6)    /* request cancelled before completion */
#define PE_ETIMEOUT (-7)     /* pe_wait timed out; the request is still pending */

typedef struct pe_ctx_s* pe_ctx;
typedef struct pe_scene_s* pe_scene;
typedef struct pe_densifier_s* pe_densifier;
typedef uint64_t pe_ticket;

enum { PE_MEM_HOST = 0, PE_MEM_DEVICE = 1 };
enum { PE_F32 = 0, PE_F64 = 1 };
enum { PE_MAT_PEC = 0, PE_MAT_ABSORBER = 1 };
enum { PE_CONTRIB_LAST = 0, PE_CONTRIB_EVERY = 1 };
enum { PE_PREC_FP64PHASE = 0, PE_PREC_FP32 = 1, PE_PREC_FP64ACC = 2 };
enum { PE_GEOM_PLAIN = 0, PE_GEOM_DENSIFIED = 1, PE_GEOM_COARSE = 2 };
enum { PE_SPLAT_DISK = 0, PE_SPLAT_TUBE = 1 };
enum { PE_SECONDARY_VIEWS = 0, PE_SECONDARY_SPLATS = 1 };

/* Scene description (input P of Algorithm 1, with normals and a material flag per point). */
typedef struct {
    uint64_t n;              /* number of points, >= 1 */
    const void* xyz;         /* n x 3 positions, row-major, float or double (xyz_type) */
    int32_t xyz_type;        /* PE_F32 or PE_F64 */
    const float* nrm;        /* n x 3 normals (any non-zero length; normalised on ingest) */
    const uint8_t* material; /* n flags: 0 = PEC, 1 = absorber (occludes, never reflects,
                                contributes nothing); NULL = all PEC; other values: PE_EINVAL */
    const float* radius;     /* n splat radii (m), or NULL to use radius_scalar */
    float radius_scalar;     /* splat radius when radius == NULL; must be > 0 */
    int32_t mem_kind;        /* PE_MEM_HOST or PE_MEM_DEVICE for xyz/nrm/material/radius */
    int32_t n_views;         /* aggregation views for the bounce march; 0 = six axis views */
    const double* view_dirs; /* n_views x 3 propagation directions (host), NULL with n_views=0 */
    int32_t view_res;        /* square resolution of each aggregation view (16 .. 4096) */
    double blend_radius;     /* > 0: every hit (primary and secondary) is refined by Eq. (23):
                                of the splats the ray crosses within this distance (m) beyond
                                the nearest hit, the one crossed relatively closest to its
                                centre gives the hit point, and the normal is the blend of
                                their normals with weights 1 - |p_i - c_i| / R_i (Sec. III-B,
                                Fig. 4(a)); 0 = off */
} pe_scene_desc;

/* Solve description (inputs tx, rx, mb and E_i of Algorithm 3, plus frequencies). */
typedef struct {
    int32_t n_inc;           /* number of incidence directions, >= 1 */
    const double* inc_dir;   /* n_inc x 3 propagation directions (host) */
    int32_t n_obs;           /* number of observation directions; ignored when obs_dir==NULL */
    const double* obs_dir;   /* n_obs x 3 scattered propagation directions k_s (host), shared
                                by every incidence (bistatic); NULL = monostatic k_s = -k_i */
    int32_t n_freq;          /* >= 1 */
    const double* freq_hz;   /* n_freq frequencies (host), > 0 */
    int32_t screen_w;        /* ray screen, pixels; pitch = 2R / max(w, h); w*h <= 2^22 */
    int32_t screen_h;
    int32_t max_bounces;     /* >= 1 (1 = physical optics from the first-hit buffer only) */
    double eps;              /* minimum travel distance of secondary rays (m), >= 0 */
    int32_t contrib;         /* PE_CONTRIB_LAST (Eq. (14)) or PE_CONTRIB_EVERY */
    int32_t precision;       /* PO sum of Eq. (14): PE_PREC_FP64PHASE (phase k D reduced in fp64,
                                fp32 sin/cos and sinc, each aligned group of four facet terms
                                summed in fp32 and the group sums accumulated in fp64),
                                PE_PREC_FP64ACC (the same with every term accumulated in fp64),
                                PE_PREC_FP32 (phase, sums and accumulation in fp32) */
    int32_t geometry;        /* PE_GEOM_PLAIN: first hits from the disk splat (Algorithm 3).
                                PE_GEOM_DENSIFIED: coarse TUBE buffer at half resolution
                                (Algorithm 1) -> network -> GFB at the screen resolution ->
                                Eq. (14) at the first bounce (Sec. III-A); incidences whose
                                network output is uncertain fall back to PLAIN.
                                PE_GEOM_COARSE: the same without the network, PO straight from
                                the half-resolution TUBE buffer with normals from its depth
                                gradients (Eq. (16)).  DENSIFIED and COARSE need
                                max_bounces == 1 and a square screen, multiple of 16. */
    pe_densifier densifier;  /* network used when geometry == PE_GEOM_DENSIFIED */
    uint64_t seed;           /* reserved for stochastic variants; results do not depend on it */
    double tube_px;          /* DENSIFIED/COARSE: tube radius delta of Algorithm 1 in coarse
                                pixels (0 = 2.0) */
    double max_uncertain;    /* DENSIFIED: fall back to PLAIN for an incidence when more than
                                this fraction of its pixels with hit probability > 0.1 lie in
                                (0.1, 0.9) (0 = 0.25) */
    int32_t tube_k;          /* DENSIFIED/COARSE: heap size K of Algorithm 1 for the coarse
                                buffer, 1 .. 1024 (see pe_render_tube_topk); 0 = unbounded K
                                (the front-most point in the tube, depth along the ray) */
    int32_t secondary;       /* geometry the bounces and the visibility Psi of Eq. (14) see:
                                PE_SECONDARY_VIEWS (0): what the scene's aggregation views
                                retain (Sec. III-B): a secondary hit on disk i at p counts iff a
                                view stores i within one pixel of p's projection; monostatic
                                Psi from the incidence first-hit buffer, bistatic Psi by a march
                                through the views.
                                PE_SECONDARY_SPLATS (1): every splat of the scene, through an
                                object-space hierarchy over them (Algorithm 3's acceleration
                                structure over splats): the nearest disk hit beyond eps, and Psi
                                = 0 iff any disk is hit from the facet toward k_s beyond eps
                                (monostatic first-bounce facets are visible). */
} pe_solve_desc;

/* Counters of one solve. */
typedef struct {
    double ray_queries;      /* live-ray intersection queries, primary rays included */
    double exit_records;     /* radiating facet records (per observation direction) */
    double po_terms;         /* facet x frequency x observation terms summed */
    double time_ms;          /* wall time of the solve measured on the stream (HIP events) */
    double march_cap_hits;   /* rays whose march reached the iteration cap (should be 0) */
    double densifier_fallbacks; /* incidences that fell back to the plain first-hit buffer */
    double march_rays;       /* live rays processed by the bounce march (all bounces) */
    double march_hits;       /* of which found a PEC facet and continued */
} pe_stats;

/* Caller-allocated host outputs of a solve.
 * E:        n_inc x n_obs' x n_freq x 2 (rx: theta, phi) x 2 (tx: theta, phi) x 2 (re, im)
 *           doubles, n_obs' = 1 when monostatic.
 * rcs_dbsm: same shape without the last axis; 10 log10(4 pi |E|^2) (may be NULL).
 * stats:    may be NULL. */
typedef struct {
    double* E;
    double* rcs_dbsm;
    pe_stats* stats;
} pe_result;

/* ---- context ---------------------------------------------------------------------------- */

/* Binds HIP device `device`.  hbm_budget = bytes the context may hold (scenes + workspaces);
 * 0 = 90 % of the device's free memory at creation. */
pe_status pe_ctx_create(int32_t device, uint64_t hbm_budget, pe_ctx* out);
pe_status pe_ctx_destroy(pe_ctx ctx);
/* Bytes currently charged to the context's budget. */
pe_status pe_ctx_footprint(pe_ctx ctx, uint64_t* bytes, uint64_t* budget);

/* Per-kernel timing: while enabled, every kernel the pipeline launches is bracketed by HIP
 * events recorded on its own launch stream; elapsed times accumulate per kernel name. */
pe_status pe_ctx_set_profiling(pe_ctx ctx, int32_t enable);
/* Copies up to `cap` entries (kernel name, total ms, launch count) into the caller's arrays
 * (names point to library-owned strings valid for the process lifetime); *n = number of
 * kernels recorded (may exceed cap).  reset != 0 clears the table afterwards. */
pe_status pe_ctx_kernel_stats(pe_ctx ctx, int32_t cap, const char** names, double* total_ms,
                              uint64_t* launches, int32_t* n, int32_t reset);

/* ---- scenes ------------------------------------------------------------------------------ */

/* Ingests the points (validates, recentres on the bounding-box centre, normalises normals,
 * orders them spatially) and renders the aggregation views with their min/max depth
 * pyramids; the scene is immutable afterwards and may be shared by concurrent solves.
 * Errors: PE_EINVAL (bad desc or bad point data), PE_ENOMEM (footprint above budget). */
pe_status pe_scene_create(pe_ctx ctx, const pe_scene_desc* desc, void* hip_stream, pe_scene* out);
/* Frees the scene's device memory.  Every request submitted with the scene (pe_submit) holds it
 * until the request finishes (completed, failed or cancelled); while any does, the call returns
 * PE_EBUSY and frees nothing.  Serialised with the context's other calls, so a synchronous
 * solve on another thread never sees the scene disappear mid-launch. */
pe_status pe_scene_destroy(pe_scene scene);
/* Scene frame: centre c (bounding-box centre, m), radius R = max |x_i - c| + r_i, r_max, and
 * the device bytes the scene holds. */
pe_status pe_scene_info(pe_scene scene, double centre[3], double* R, double* r_max,
                        uint64_t* bytes);

/* ---- solving ---------------------------------------------------------------------------- */

/* Synchronous solve: traces every incidence direction on a screen of central rays, bounces
 * up to max_bounces times and sums the PO field of Eq. (14) for every observation direction
 * and frequency.  Returns after the results are in the host buffers.  Incidences run in
 * batches sized to half of the context's unused HBM budget (2^22 .. 2^29 pixels; the
 * PE_BATCH_PIXELS environment variable overrides); the context keeps the batch workspace for
 * later calls, and results do not depend on the batching. */
pe_status pe_solve(pe_ctx ctx, pe_scene scene, const pe_solve_desc* desc, pe_result* res,
                   void* hip_stream);

/* Size of the fixed per-device array behind pe_solve_noalloc (128 MiB). */
#define PE_NOALLOC_SCRATCH_BYTES (128ull << 20)

/* pe_solve for callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, semantics, results (bitwise)
 * and errors as pe_solve with geometry PE_GEOM_PLAIN, but no device or pinned memory is
 * allocated or freed and no HIP event is created: every transient buffer is carved from one
 * fixed array of PE_NOALLOC_SCRATCH_BYTES bytes that the library's code object holds on each
 * device (for the process lifetime; its address is looked up by pe_ctx_create).  Incidences run
 * in batches that fit the array.  The scene, the desc and the result buffers are the caller's,
 * as for pe_solve.  Limits: one incidence's batch must fit the array (about 180 bytes per screen
 * pixel, 40 more per observation direction and, with PE_CONTRIB_EVERY, per bounce: screens up to
 * 512 x 512 fit, 1024 x 1024 do not); a larger screen returns PE_ENOMEM before anything is
 * launched, and a single incidence that still outgrows the array returns PE_ENOMEM before the
 * kernel that would use the missing bytes.  Other geometries return PE_EUNSUPPORTED.  All calls on one device share the
 * array, so the library runs them one at a time (a second caller blocks until the first
 * returns); stats->time_ms is host wall time. */
pe_status pe_solve_noalloc(pe_ctx ctx, pe_scene scene, const pe_solve_desc* desc,
                           pe_result* res, void* hip_stream);

/* Asynchronous solve through the context's continuous-batching server.  The desc's host
 * arrays are copied during the call; the res buffers (E, rcs_dbsm, stats) are written by the
 * server thread and must stay valid until pe_wait has returned the request's final status
 * (anything but PE_ETIMEOUT): to give them up early, pe_cancel and then pe_wait.  The request
 * holds the scene until it finishes (pe_scene_destroy returns PE_EBUSY meanwhile).  Admission
 * waits until the request's HBM footprint fits the budget.
 * Errors at submit: PE_EINVAL, PE_ENOMEM (request larger than the whole budget). */
pe_status pe_submit(pe_ctx ctx, pe_scene scene, const pe_solve_desc* desc, pe_result* res,
                    pe_ticket* ticket);
/* Waits up to timeout_us (< 0 = forever).  Returns the request's status, or PE_ETIMEOUT. */
pe_status pe_wait(pe_ctx ctx, pe_ticket ticket, int64_t timeout_us);
/* Cancels a pending or running request; pe_wait then returns PE_ECANCELED. */
pe_status pe_cancel(pe_ctx ctx, pe_ticket ticket);
/* HBM bytes the server charges a request for admission (its transient workspace at the
 * largest batch share it can take); pe_submit fails with PE_ENOMEM when this exceeds the
 * context's budget. */
pe_status pe_request_footprint(const pe_solve_desc* desc, uint64_t* bytes);
/* Latency/throughput counters of the server since creation (or the last reset):
 * out[0] completed, out[1] p50 latency ms, out[2] p99 latency ms, out[3] mean ms,
 * out[4] max concurrent requests on the device, out[5] mean requests per shared launch batch. */
pe_status pe_server_stats(pe_ctx ctx, double out[6], int32_t reset);

/* ---- inspection hooks (tests) ----------------------------------------------------------- */

/* Geometric frame buffer of one view (Algorithm 1 output without the network):
 * mode PE_SPLAT_DISK = first disk hit along every pixel's central ray;
 * mode PE_SPLAT_TUBE = nearest point (along the ray) within tube_radius (m) of the central ray.
 * Device outputs (any may be NULL), row-major h x w: depth (m, +inf where empty),
 * nrm (x3, oriented against the ray), idx (input point index, 0xFFFFFFFF where empty),
 * mask (1 = hit). */
pe_status pe_render_gfb(pe_ctx ctx, pe_scene scene, const double dir[3], int32_t w, int32_t h,
                        int32_t mode, double tube_radius, float* depth, float* nrm,
                        uint32_t* idx, uint8_t* mask, void* hip_stream);

/* Coarse buffer of Algorithm 1 with a K-point heap (Sec. III-A): for each pixel's ray tube of
 * radius tube_radius (m), the K points nearest the central ray (in front of the screen; ties:
 * lowest index) are kept and the one nearest the tube origin is chosen (ties: lowest index).
 * Outputs as pe_render_gfb, with depth = Euclidean distance |p - o| from the pixel centre on the
 * screen.  K in 1..1024 (PE_EINVAL otherwise); K at least the candidate count of every tube
 * selects the nearest candidate to the origin. */
pe_status pe_render_tube_topk(pe_ctx ctx, pe_scene scene, const double dir[3], int32_t w,
                              int32_t h, double tube_radius, int32_t K, float* depth, float* nrm,
                              uint32_t* idx, uint8_t* mask, void* hip_stream);

/* Per-pixel bounce records of one incidence (what the PO sum consumes), device outputs,
 * row-major h x w: n_bounce (0 = no hit), last_x (x3, scene frame: add the centre for world),
 * last_n (x3, oriented), path (image-method path length to last_x in the scene frame), last_idx
 * (point index of the last facet).  Any output may be NULL.  secondary: PE_SECONDARY_VIEWS or
 * PE_SECONDARY_SPLATS, as in pe_solve_desc. */
pe_status pe_trace_pixels(pe_ctx ctx, pe_scene scene, const double inc_dir[3], int32_t w,
                          int32_t h, int32_t max_bounces, double eps, int32_t secondary,
                          int32_t* n_bounce,
                          float* last_x, float* last_n, double* path, uint32_t* last_idx,
                          void* hip_stream);

/* ---- learned densifier (Sec. III-A, Eq. (15)-(21)) -------------------------------------- */

/* A U-Net densifier: 4 levels with base_ch channels (base_ch, 2, 4, 8 x), ConvNeXt encoder
 * blocks, max-pool down, sub-pixel-convolution up, one shared encoder and three decoder heads
 * (depth, normal, hit probability).  Input: coarse depth map (h x w); output: 2h x 2w maps.
 * Weights are bf16 with fp32 master copies and AdamW state on the device. */
pe_status pe_densifier_create(pe_ctx ctx, int32_t base_ch, uint64_t seed, pe_densifier* out);
pe_status pe_densifier_destroy(pe_densifier net);
pe_status pe_densifier_save(pe_densifier net, const char* path);
pe_status pe_densifier_load(pe_densifier net, const char* path);
pe_status pe_densifier_num_params(pe_densifier net, uint64_t* n);
/* One AdamW step on a batch (device pointers, batch b, coarse size h x w):
 *   coarse   b x h x w       network input (1 - t/D on hits, 0 elsewhere)
 *   depth_gt b x 2h x 2w     normalised depth target (t/D), valid where mask_gt = 1
 *   nrm_gt   b x 2h x 2w x 3 unit normals in the view frame (u, v, w), valid where mask_gt = 1
 *   mask_gt  b x 2h x 2w     0/1
 * loss_out (host, 5 doubles): total, L1..L4 of Eq. (17)-(20) weighted as in Eq. (21).
 * lr: learning rate of this step; weight_decay: AdamW decoupled decay. */
pe_status pe_densifier_train_step(pe_densifier net, int32_t b, int32_t h, int32_t w,
                                  const float* coarse, const float* depth_gt, const float* nrm_gt,
                                  const float* mask_gt, float lr, float weight_decay,
                                  double* loss_out, void* hip_stream);
/* Inference: outputs (device, may be NULL) depth b x 2h x 2w, nrm b x 2h x 2w x 3 (unit,
 * view frame), prob b x 2h x 2w (hit probability).  h, w: multiples of 8. */
pe_status pe_densifier_infer(pe_densifier net, int32_t b, int32_t h, int32_t w,
                             const float* coarse, float* depth, float* nrm, float* prob,
                             void* hip_stream);
/* Parameter table: *n = number of tensors; for i < cap: names[i] (library-owned, valid while
 * the network lives), offsets[i] into the flat parameter vector, shapes[4 i .. 4 i + 3]
 * (convolutions [Cout][K][K][Cin], depthwise [C][7][7], vectors [C]; unused trailing dims 0).
 * Any of names/offsets/shapes may be NULL. */
pe_status pe_densifier_tensors(pe_densifier net, int32_t cap, const char** names,
                               uint64_t* offsets, int32_t* shapes, int32_t* n);
/* Copies a flat fp32 vector of pe_densifier_num_params values to the host: which = 0 master
 * parameters, 1 gradients of the last train step, 2 / 3 AdamW first / second moments. */
pe_status pe_densifier_get(pe_densifier net, int32_t which, float* host, uint64_t n);
/* Replaces the master parameters (host fp32, n = pe_densifier_num_params) and refreshes the
 * bf16 copies; AdamW state is kept.  PE_EINVAL on a non-finite value. */
pe_status pe_densifier_set(pe_densifier net, const float* host, uint64_t n);
/* Training data from a scene (Sec. IV-A recipe on synthetic scenes): for each of n_dir
 * propagation directions (host, n_dir x 3), the network input and targets on that
 * direction's screen (side 2R, as for pe_solve), device outputs, any group may be NULL:
 *   coarse   n_dir x h x w        TUBE first hits (radius tube_px coarse pixels): 1 - t/D, 0 empty;
 *                                  tube_k = 0: the front-most point in each tube (t along the
 *                                  ray); 1 .. 1024: the K-point heap of pe_render_tube_topk
 *                                  (t = distance from the pixel centre)
 *   depth_gt n_dir x 2h x 2w      DISK first hits: t/D (0 where empty)
 *   nrm_gt   n_dir x 2h x 2w x 3  unit normal against the ray in the view frame (u, v, -k)
 *   mask_gt  n_dir x 2h x 2w      1 on hits
 * (t: distance from the screen plane along the ray, D = 2R.) */
pe_status pe_densifier_make_pair(pe_ctx ctx, pe_scene scene, int32_t n_dir, const double* dirs,
                                 int32_t h, int32_t w, double tube_px, int32_t tube_k,
                                 float* coarse, float* depth_gt, float* nrm_gt, float* mask_gt,
                                 void* hip_stream);

/* ---- point-cloud normals ---------------------------------------------------------------- */

/* Normals of a point cloud that carries none (the point-cloud baseline of Sec. IV estimates them
 * by principal component analysis): for every point, its k nearest points (itself included;
 * ties: lowest index) are found exactly through a uniform grid, and the normal is the
 * eigenvector of their covariance with the smallest eigenvalue, turned so that its largest
 * component is positive (unoriented: splats are two-sided).  xyz: n x 3 (xyz_type) and nrm:
 * n x 3 floats, both in mem_kind memory.  k: 3 .. 64.  Errors: PE_EINVAL (bad arguments,
 * non-finite positions).  Collinear or coincident neighbourhoods give an arbitrary unit vector
 * orthogonal to them (or +z). */
pe_status pe_estimate_normals(pe_ctx ctx, uint64_t n, const void* xyz, int32_t xyz_type,
                              int32_t mem_kind, int32_t k, float* nrm, void* hip_stream);

/* ---- GFB fusion for multi-bounce geometry (Sec. III-B, Algorithm 3, Eq. (22)) ------------- */

/* Geometric frame buffers of n_views screens over one scene frame, in the layout of
 * pe_densifier_make_pair's targets and pe_densifier_infer's outputs. */
typedef struct {
    int32_t n_views;          /* 1 .. 64 */
    const double* view_dirs;  /* host, n_views x 3 propagation directions of the screens */
    int32_t w, h;             /* square buffers (w == h, 8 .. 8192); pitch 2R / w */
    double centre[3];         /* frame of the screens: centre c and radius R (pe_scene_info); */
    double R;                 /* each screen is 2R wide, centred on c, R before c along k */
    const float* depth;       /* device n_views x h x w: t / (2R), t from the screen plane */
    const float* nrm;         /* device n_views x h x w x 3: normals in the view frame (u, v, -k) */
    const float* hit;         /* device n_views x h x w: a hit where >= 0.5 (mask or probability) */
} pe_gfb_set;

typedef struct {
    int32_t grid;             /* cells per axis of the fusion grid, 8 .. 512 (0 = 256) */
    double grid_side;         /* side of the cubic grid about c (m); 0 = 2R.  The pixel side L
                                 of Eq. (22) is grid_side / grid. */
    double edge_lo, edge_hi;  /* Canny thresholds on the depth slope (depth change per pixel
                                 pitch); 0 = 2 and 4 */
    int32_t edge_dilate;      /* pixels within this many pixels of an edge are dropped too;
                                 0 .. 8, negative = 1 */
} pe_fuse_desc;

/* Edge filtering and fusion: the depth of each buffer (empty pixels at 2R) is smoothed by a
 * 5 x 5 Gaussian (sigma 1 pixel), its Sobel gradient thinned by non-maximum suppression and
 * double-thresholded with 8-connected hysteresis; hit pixels away from those edges are placed
 * in the grid, and every occupied cell becomes one splat: mean position, normalised mean of
 * the normals (each turned so that its largest component is positive), and the radius of
 * Eq. (22) for the contributing view that sees the mean normal most squarely.
 * Outputs (device, splats in cell order, x fastest): xyz (n x 3 doubles, world), nrm (n x 3),
 * radius (n), count (n pixels fused per splat; may be NULL), edge (n_views x h x w, 1 on Canny
 * edges; may be NULL).  At most `cap` splats are written; *n_out = number of splats (cap =
 * n_views * w * h always suffices; cap = 0 only counts).  The splats suit pe_scene_create
 * with mem_kind PE_MEM_DEVICE, xyz_type PE_F64 and per-point radii. */
pe_status pe_fuse_gfbs(pe_ctx ctx, const pe_gfb_set* gfbs, const pe_fuse_desc* desc, double* xyz,
                       float* nrm, float* radius, uint32_t* count, uint8_t* edge, uint64_t cap,
                       uint64_t* n_out, void* hip_stream);

/* ---- errors ------------------------------------------------------------------------------ */

/* Thread-local description of the last failure on the calling thread (valid until the next
 * call on that thread). */
const char* pe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* POINTEMRAY_H */
