/*
 * FP64 CPU oracle for point-cloud SBR -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct reference for what the GPU path computes.  Only the test
 * suite, the smoke check and the bench's CPU-baseline leg may load this library; the product
 * path never does.  It shares no code, header or constant with the HIP library.
 *
 * The method being checked: points carrying normals are treated as oriented disks ("splats"),
 * a screen of central rays is shot at them along the incident direction, rays bounce off PEC
 * disks by geometric optics, and the physical-optics aperture integral of each ray's last
 * facet is summed into the far field.  Definitions followed, by section of the paper:
 *   - ray field and PEC reflection: Sec. II-A, Eq. (1)-(4);
 *   - PO facet integral with central rays only: Sec. II-B, Eq. (5)-(13);
 *   - total SBR field over rays, last bounce, image-method path length: Sec. II-C, Eq. (14);
 *   - ray-tube nearest-point depth (Top-K with K unbounded): Sec. III-A, Algorithm 1;
 *   - bounce loop with a minimum travel distance eps for secondary rays: Sec. III-B,
 *     Algorithm 3 and the paragraph after Eq. (23).
 * Readings where the paper is silent (screen placement, tie-breaks, grazing threshold, the
 * parallelogram area, sinc convention) are stated at each function.
 *
 * Everything is double precision; libm sin/cos.  No blocking or reordering beyond what the
 * definitions state, except the optional uniform grid (or_scene_build_grid) which visits a
 * superset of the disks a ray can hit in ray order and returns the bitwise-identical first hit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_C0 299792458.0
#define OR_GRAZE 1e-6
#define OR_PI 3.14159265358979323846

typedef struct { double x, y, z; } v3;

static inline v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static inline v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static inline double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 cross(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline double len(v3 a) { return sqrt(dot(a, a)); }
static inline v3 unit(v3 a) { return scl(a, 1.0 / len(a)); }
static inline v3 ld(const double* p) { return mk(p[0], p[1], p[2]); }
static inline void st(double* p, v3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }

/* ------------------------------------------------------------------------------------------ */
/* Scene: disks (centre, unit normal, radius, material) plus optional uniform grid.            */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    double* xyz;
    double* nrm;
    double* rad;
    uint8_t* mat;
    double c[3];   /* bounding-box centre */
    double R;      /* max over disks of |x_i - c| + r_i */
    /* grid (c.8): CSR lists of disk ids per cell */
    int G;
    double lo[3], h;
    int64_t* cell_start; /* G^3 + 1 */
    int32_t* cell_ids;
    /* aggregation views (see or_scene_set_views): n_views first-hit index maps res x res */
    int n_views, view_res;
    double* view_basis;  /* n_views x 9: u, v, k */
    int64_t* view_idx;   /* n_views x res x res, -1 where empty */
    double blend_r;      /* Eq. (23) refinement radius (0 = off), see blend_hit */
} or_scene;

/* Returns NULL and *err != 0 on invalid input: non-finite position, zero/non-finite normal,
 * non-positive radius or a material other than 0 (PEC) / 1 (absorber). */
void* or_scene_new(int64_t n, const double* xyz, const double* nrm, const double* rad,
                   const uint8_t* mat, int* err) {
    *err = 0;
    if (n <= 0) { *err = 1; return NULL; }
    or_scene* s = (or_scene*)calloc(1, sizeof(or_scene));
    s->n = n;
    s->xyz = (double*)malloc(sizeof(double) * 3 * n);
    s->nrm = (double*)malloc(sizeof(double) * 3 * n);
    s->rad = (double*)malloc(sizeof(double) * n);
    s->mat = (uint8_t*)malloc(n);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; i++) {
        v3 x = ld(xyz + 3 * i), nn = ld(nrm + 3 * i);
        double l = len(nn);
        if (!isfinite(x.x) || !isfinite(x.y) || !isfinite(x.z) || !(l > 0) || !isfinite(l) ||
            !(rad[i] > 0) || !isfinite(rad[i]) || (mat && mat[i] > 1)) {
            *err = 1;
        }
        st(s->xyz + 3 * i, x);
        st(s->nrm + 3 * i, scl(nn, 1.0 / l));
        s->rad[i] = rad[i];
        s->mat[i] = mat ? mat[i] : 0;
        for (int a = 0; a < 3; a++) {
            double v = (&x.x)[a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    }
    if (*err) {
        free(s->xyz); free(s->nrm); free(s->rad); free(s->mat); free(s);
        return NULL;
    }
    for (int a = 0; a < 3; a++) s->c[a] = 0.5 * (lo[a] + hi[a]);
    double R = 0;
    v3 c = ld(s->c);
    for (int64_t i = 0; i < n; i++) {
        double r = len(sub(ld(s->xyz + 3 * i), c)) + s->rad[i];
        if (r > R) R = r;
    }
    s->R = R;
    return s;
}

void or_scene_free(void* p) {
    or_scene* s = (or_scene*)p;
    if (!s) return;
    free(s->xyz); free(s->nrm); free(s->rad); free(s->mat);
    free(s->cell_start); free(s->cell_ids);
    free(s->view_basis); free(s->view_idx);
    free(s);
}

void or_scene_frame(const void* p, double* c, double* R) {
    const or_scene* s = (const or_scene*)p;
    c[0] = s->c[0]; c[1] = s->c[1]; c[2] = s->c[2];
    *R = s->R;
}

/* ------------------------------------------------------------------------------------------ */
/* Screen (Algorithm 1, RayTubeInitialization).  Reading: the screen is a square of side 2R   */
/* centred on the scene, placed R before the centre along the propagation direction k, pixel  */
/* pitch 2R/max(W,H); u = normalise(z x k) (x if k is within 1e-9 of +-z), v = k x u.          */
/* ------------------------------------------------------------------------------------------ */

void or_screen(const void* p, const double* kin, int W, int H, double* o00, double* du,
               double* dv) {
    const or_scene* s = (const or_scene*)p;
    v3 k = unit(ld(kin));
    v3 u = fabs(k.z) > 1.0 - 1e-9 ? mk(1, 0, 0) : unit(cross(mk(0, 0, 1), k));
    v3 v = cross(k, u);
    double pitch = 2.0 * s->R / (double)(W > H ? W : H);
    v3 c = ld(s->c);
    /* centre of pixel (0,0): c - R k + (0.5 - W/2) pitch u + (0.5 - H/2) pitch v */
    v3 o = add(sub(c, scl(k, s->R)),
               add(scl(u, (0.5 - 0.5 * W) * pitch), scl(v, (0.5 - 0.5 * H) * pitch)));
    st(o00, o);
    st(du, scl(u, pitch));
    st(dv, scl(v, pitch));
}

/* ------------------------------------------------------------------------------------------ */
/* Ray-disk test.  Reading: disks are two-sided; |n.k| < 1e-6 is a miss (grazing); the hit     */
/* must satisfy t > tmin; the boundary |q - x|^2 <= r^2 is inclusive.                          */
/* ------------------------------------------------------------------------------------------ */

static inline int disk_hit(const or_scene* s, int64_t i, v3 o, v3 k, double tmin, double* t) {
    v3 n = ld(s->nrm + 3 * i), x = ld(s->xyz + 3 * i);
    double den = dot(n, k);
    if (fabs(den) < OR_GRAZE) return 0;
    double tt = dot(n, sub(x, o)) / den;
    if (!(tt > tmin)) return 0;
    v3 q = sub(add(o, scl(k, tt)), x);
    if (dot(q, q) <= s->rad[i] * s->rad[i]) { *t = tt; return 1; }
    return 0;
}

static int64_t first_hit_brute(const or_scene* s, v3 o, v3 k, double tmin, double* tbest,
                               int64_t* ntests) {
    int64_t best = -1;
    double bt = INFINITY, t;
    for (int64_t i = 0; i < s->n; i++) {
        if (disk_hit(s, i, o, k, tmin, &t) && t < bt) { bt = t; best = i; }
    }
    *ntests += s->n;
    *tbest = bt;
    return best;
}

/* Uniform grid (c.8).  Each disk is listed in every cell its inflated bounding cube touches. */
int or_scene_build_grid(void* p, int G) {
    or_scene* s = (or_scene*)p;
    if (G < 1) G = 1;
    double rmax = 0;
    for (int64_t i = 0; i < s->n; i++) if (s->rad[i] > rmax) rmax = s->rad[i];
    double lo[3], hi[3];
    for (int a = 0; a < 3; a++) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int64_t i = 0; i < s->n; i++)
        for (int a = 0; a < 3; a++) {
            double v = s->xyz[3 * i + a];
            if (v - s->rad[i] < lo[a]) lo[a] = v - s->rad[i];
            if (v + s->rad[i] > hi[a]) hi[a] = v + s->rad[i];
        }
    double ext = 0;
    for (int a = 0; a < 3; a++) if (hi[a] - lo[a] > ext) ext = hi[a] - lo[a];
    double pad = 1e-6 * ext + 1e-12;
    for (int a = 0; a < 3; a++) { s->lo[a] = lo[a] - pad; }
    s->h = (ext + 2 * pad) / G;
    s->G = G;
    int64_t nc = (int64_t)G * G * G;
    free(s->cell_start); free(s->cell_ids);
    s->cell_start = (int64_t*)calloc(nc + 1, sizeof(int64_t));
    double e = 1e-9 * ext;
    for (int pass = 0; pass < 2; pass++) {
        int64_t* cursor = NULL;
        if (pass == 1) {
            for (int64_t c = 0; c < nc; c++) s->cell_start[c + 1] += s->cell_start[c];
            s->cell_ids = (int32_t*)malloc(sizeof(int32_t) * (s->cell_start[nc] + 1));
            cursor = (int64_t*)malloc(sizeof(int64_t) * nc);
            memcpy(cursor, s->cell_start, sizeof(int64_t) * nc);
        }
        for (int64_t i = 0; i < s->n; i++) {
            int c0[3], c1[3];
            for (int a = 0; a < 3; a++) {
                double v = s->xyz[3 * i + a];
                int q0 = (int)floor((v - s->rad[i] - e - s->lo[a]) / s->h);
                int q1 = (int)floor((v + s->rad[i] + e - s->lo[a]) / s->h);
                c0[a] = q0 < 0 ? 0 : (q0 >= G ? G - 1 : q0);
                c1[a] = q1 < 0 ? 0 : (q1 >= G ? G - 1 : q1);
            }
            for (int z = c0[2]; z <= c1[2]; z++)
                for (int y = c0[1]; y <= c1[1]; y++)
                    for (int x = c0[0]; x <= c1[0]; x++) {
                        int64_t c = ((int64_t)z * G + y) * G + x;
                        if (pass == 0) s->cell_start[c + 1]++;
                        else s->cell_ids[cursor[c]++] = (int32_t)i;
                    }
        }
        free(cursor);
    }
    return 0;
}

/* Amanatides-Woo traversal; a candidate is accepted once its t lies within the current cell. */
static int64_t first_hit_grid(const or_scene* s, v3 o, v3 k, double tmin, double* tbest,
                              int64_t* ntests) {
    int G = s->G;
    double t0 = tmin > 0 ? tmin : 0, t1 = INFINITY;
    double oo[3] = {o.x, o.y, o.z}, kk[3] = {k.x, k.y, k.z};
    double hi[3];
    for (int a = 0; a < 3; a++) hi[a] = s->lo[a] + G * s->h;
    for (int a = 0; a < 3; a++) {
        if (kk[a] == 0.0) {
            if (oo[a] < s->lo[a] || oo[a] > hi[a]) { *tbest = INFINITY; return -1; }
        } else {
            double ta = (s->lo[a] - oo[a]) / kk[a], tb = (hi[a] - oo[a]) / kk[a];
            if (ta > tb) { double tt = ta; ta = tb; tb = tt; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        }
    }
    if (t0 > t1) { *tbest = INFINITY; return -1; }
    int cell[3], step[3];
    double tmax[3], tdel[3];
    for (int a = 0; a < 3; a++) {
        double pa = oo[a] + t0 * kk[a];
        int q = (int)floor((pa - s->lo[a]) / s->h);
        cell[a] = q < 0 ? 0 : (q >= G ? G - 1 : q);
        if (kk[a] > 0) {
            step[a] = 1;
            tmax[a] = (s->lo[a] + (cell[a] + 1) * s->h - oo[a]) / kk[a];
            tdel[a] = s->h / kk[a];
        } else if (kk[a] < 0) {
            step[a] = -1;
            tmax[a] = (s->lo[a] + cell[a] * s->h - oo[a]) / kk[a];
            tdel[a] = -s->h / kk[a];
        } else {
            step[a] = 0;
            tmax[a] = INFINITY;
            tdel[a] = INFINITY;
        }
    }
    int64_t best = -1;
    double bt = INFINITY, t;
    for (;;) {
        int64_t c = ((int64_t)cell[2] * G + cell[1]) * G + cell[0];
        for (int64_t j = s->cell_start[c]; j < s->cell_start[c + 1]; j++) {
            int64_t i = s->cell_ids[j];
            (*ntests)++;
            if (disk_hit(s, i, o, k, tmin, &t) && (t < bt || (t == bt && i < best))) {
                bt = t;
                best = i;
            }
        }
        int a = (tmax[0] < tmax[1]) ? (tmax[0] < tmax[2] ? 0 : 2) : (tmax[1] < tmax[2] ? 1 : 2);
        double texit = tmax[a];
        if (best >= 0 && bt <= texit) break;
        cell[a] += step[a];
        if (cell[a] < 0 || cell[a] >= G) break;
        tmax[a] += tdel[a];
    }
    *tbest = bt;
    return best;
}

static int64_t first_hit(const or_scene* s, v3 o, v3 k, double tmin, int use_grid,
                         double* t, int64_t* ntests) {
    if (use_grid && s->cell_start) return first_hit_grid(s, o, k, tmin, t, ntests);
    return first_hit_brute(s, o, k, tmin, t, ntests);
}

int64_t or_first_hit(const void* p, const double* o, const double* k, double tmin, int use_grid,
                     double* t) {
    int64_t nt = 0;
    return first_hit((const or_scene*)p, ld(o), unit(ld(k)), tmin, use_grid, t, &nt);
}

/* ------------------------------------------------------------------------------------------ */
/* The method's secondary-hit rule (Sec. III-B: bounces are traced against the geometry the   */
/* frame buffers of a set of views retain).  Each aggregation view is the first-hit index map */
/* (c.4) of a res x res screen along the view's direction.  A secondary intersection of disk  */
/* i at point p is ADMISSIBLE iff some view stores i at a pixel within one pixel (in both     */
/* screen axes) of p's projection; the restricted first hit is the nearest admissible         */
/* intersection (ties: smallest index).  Exact tracing (first_hit) is the special case where  */
/* every intersection is admissible.                                                          */
/* ------------------------------------------------------------------------------------------ */

void or_render_disk(const void* p, const double* kin, int W, int H, int use_grid, double* depth,
                    int64_t* idx, double* nrm, uint8_t* mask);

int or_scene_set_views(void* p, int n_views, const double* dirs, int res, int use_grid) {
    or_scene* s = (or_scene*)p;
    if (n_views < 1 || res < 1) return 1;
    free(s->view_basis); free(s->view_idx);
    s->n_views = n_views;
    s->view_res = res;
    s->view_basis = (double*)malloc(sizeof(double) * 9 * n_views);
    s->view_idx = (int64_t*)malloc(sizeof(int64_t) * (int64_t)n_views * res * res);
    double* depth = (double*)malloc(sizeof(double) * (int64_t)res * res);
    uint8_t* mask = (uint8_t*)malloc((size_t)res * res);
    for (int v = 0; v < n_views; v++) {
        double o00[3], du[3], dv[3];
        or_screen(p, dirs + 3 * v, res, res, o00, du, dv);
        st(s->view_basis + 9 * v + 0, unit(ld(du)));
        st(s->view_basis + 9 * v + 3, unit(ld(dv)));
        st(s->view_basis + 9 * v + 6, unit(ld(dirs + 3 * v)));
        or_render_disk(p, dirs + 3 * v, res, res, use_grid, depth,
                       s->view_idx + (int64_t)v * res * res, NULL, mask);
    }
    free(depth);
    free(mask);
    return 0;
}

static int admissible(const or_scene* s, int64_t i, v3 pt) {
    const int res = s->view_res;
    const double pitch = 2.0 * s->R / res;
    v3 q = sub(pt, ld(s->c));
    for (int v = 0; v < s->n_views; v++) {
        const double* b = s->view_basis + 9 * v;
        int ia = (int)floor(dot(q, ld(b + 0)) / pitch + 0.5 * res);
        int ib = (int)floor(dot(q, ld(b + 3)) / pitch + 0.5 * res);
        const int64_t* m = s->view_idx + (int64_t)v * res * res;
        for (int dy = -1; dy <= 1; dy++) {
            int y = ib + dy;
            if (y < 0 || y >= res) continue;
            for (int dx = -1; dx <= 1; dx++) {
                int x = ia + dx;
                if (x < 0 || x >= res) continue;
                if (m[(int64_t)y * res + x] == i) return 1;
            }
        }
    }
    return 0;
}

/* Same traversal as first_hit_grid (or all disks without a grid); only admissible
 * intersections compete. */
static int64_t first_hit_views(const or_scene* s, v3 o, v3 k, double tmin, double* tbest,
                               int64_t* ntests) {
    int64_t best = -1;
    double bt = INFINITY, t;
    if (!s->cell_start) {
        for (int64_t i = 0; i < s->n; i++)
            if (disk_hit(s, i, o, k, tmin, &t) && (t < bt || (t == bt && i < best)) &&
                admissible(s, i, add(o, scl(k, t)))) {
                bt = t;
                best = i;
            }
        *ntests += s->n;
        *tbest = bt;
        return best;
    }
    int G = s->G;
    double t0 = tmin > 0 ? tmin : 0, t1 = INFINITY;
    double oo[3] = {o.x, o.y, o.z}, kk[3] = {k.x, k.y, k.z};
    double hi[3];
    for (int a = 0; a < 3; a++) hi[a] = s->lo[a] + G * s->h;
    for (int a = 0; a < 3; a++) {
        if (kk[a] == 0.0) {
            if (oo[a] < s->lo[a] || oo[a] > hi[a]) { *tbest = INFINITY; return -1; }
        } else {
            double ta = (s->lo[a] - oo[a]) / kk[a], tb = (hi[a] - oo[a]) / kk[a];
            if (ta > tb) { double tt = ta; ta = tb; tb = tt; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        }
    }
    if (t0 > t1) { *tbest = INFINITY; return -1; }
    int cell[3], step[3];
    double tmax[3], tdel[3];
    for (int a = 0; a < 3; a++) {
        double pa = oo[a] + t0 * kk[a];
        int q = (int)floor((pa - s->lo[a]) / s->h);
        cell[a] = q < 0 ? 0 : (q >= G ? G - 1 : q);
        if (kk[a] > 0) {
            step[a] = 1;
            tmax[a] = (s->lo[a] + (cell[a] + 1) * s->h - oo[a]) / kk[a];
            tdel[a] = s->h / kk[a];
        } else if (kk[a] < 0) {
            step[a] = -1;
            tmax[a] = (s->lo[a] + cell[a] * s->h - oo[a]) / kk[a];
            tdel[a] = -s->h / kk[a];
        } else {
            step[a] = 0;
            tmax[a] = INFINITY;
            tdel[a] = INFINITY;
        }
    }
    for (;;) {
        int64_t c = ((int64_t)cell[2] * G + cell[1]) * G + cell[0];
        for (int64_t j = s->cell_start[c]; j < s->cell_start[c + 1]; j++) {
            int64_t i = s->cell_ids[j];
            (*ntests)++;
            if (disk_hit(s, i, o, k, tmin, &t) && (t < bt || (t == bt && i < best)) &&
                admissible(s, i, add(o, scl(k, t)))) {
                bt = t;
                best = i;
            }
        }
        int a = (tmax[0] < tmax[1]) ? (tmax[0] < tmax[2] ? 0 : 2) : (tmax[1] < tmax[2] ? 1 : 2);
        double texit = tmax[a];
        if (best >= 0 && bt <= texit) break;
        cell[a] += step[a];
        if (cell[a] < 0 || cell[a] >= G) break;
        tmax[a] += tdel[a];
    }
    *tbest = bt;
    return best;
}

int64_t or_first_hit_views(const void* p, const double* o, const double* k, double tmin,
                           double* t) {
    int64_t nt = 0;
    const or_scene* s = (const or_scene*)p;
    if (!s->view_idx) return -2;
    return first_hit_views(s, ld(o), unit(ld(k)), tmin, t, &nt);
}

int or_admissible(const void* p, int64_t i, const double* pt) {
    const or_scene* s = (const or_scene*)p;
    if (!s->view_idx) return -1;
    return admissible(s, i, ld(pt));
}

/* ------------------------------------------------------------------------------------------ */
/* Primary geometric frame buffer with disks (c.4): first hit with tmin = 0 at every pixel;   */
/* normal oriented against the ray (two-sided splats, "oriented normal map").                 */
/* ------------------------------------------------------------------------------------------ */

void or_render_disk(const void* p, const double* kin, int W, int H, int use_grid, double* depth,
                    int64_t* idx, double* nrm, uint8_t* mask) {
    const or_scene* s = (const or_scene*)p;
    double o00[3], du[3], dv[3];
    or_screen(p, kin, W, H, o00, du, dv);
    v3 k = unit(ld(kin));
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < H; j++) {
        int64_t nt = 0;
        for (int i = 0; i < W; i++) {
            v3 o = add(ld(o00), add(scl(ld(du), i), scl(ld(dv), j)));
            double t;
            int64_t h = first_hit(s, o, k, 0.0, use_grid, &t, &nt);
            int64_t q = (int64_t)j * W + i;
            if (h >= 0) {
                v3 n = ld(s->nrm + 3 * h);
                if (dot(n, k) > 0) n = scl(n, -1.0);
                depth[q] = t; idx[q] = h; mask[q] = 1;
                if (nrm) st(nrm + 3 * q, n);
            } else {
                depth[q] = INFINITY; idx[q] = -1; mask[q] = 0;
                if (nrm) st(nrm + 3 * q, mk(0, 0, 0));
            }
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Coarse depth by ray tubes (Algorithm 1 with K unbounded, c.5): a point is a candidate iff   */
/* its distance to the central ray is below delta and it lies in front of the screen; the     */
/* depth is the along-ray distance of the nearest candidate (ties: smallest index).           */
/* ------------------------------------------------------------------------------------------ */

void or_render_tube(const void* p, const double* kin, int W, int H, double delta, double* depth,
                    int64_t* idx) {
    const or_scene* s = (const or_scene*)p;
    double o00[3], du[3], dv[3];
    or_screen(p, kin, W, H, o00, du, dv);
    v3 k = unit(ld(kin));
    double d2 = delta * delta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < H; j++) {
        for (int i = 0; i < W; i++) {
            v3 o = add(ld(o00), add(scl(ld(du), i), scl(ld(dv), j)));
            double bt = INFINITY;
            int64_t best = -1;
            for (int64_t m = 0; m < s->n; m++) {
                v3 w = sub(ld(s->xyz + 3 * m), o);
                double tc = dot(w, k);
                if (!(tc > 0)) continue;
                v3 c = cross(w, k);
                if (dot(c, c) < d2 && tc < bt) { bt = tc; best = m; }
            }
            int64_t q = (int64_t)j * W + i;
            depth[q] = bt;
            idx[q] = best;
        }
    }
}

/* Algorithm 1 with a bounded heap (Sec. III-A): the candidates of a tube are the points within
 * delta of its central ray and in front of the screen; the K candidates nearest the ray are
 * kept (ties: smallest index), and of those the one nearest the tube origin o is chosen (ties:
 * smallest index); the coarse depth is its Euclidean distance |p - o|.  Brute force. */
void or_render_tube_topk(const void* p, const double* kin, int W, int H, double delta, int K,
                         double* depth, int64_t* idx) {
    const or_scene* s = (const or_scene*)p;
    double o00[3], du[3], dv[3];
    or_screen(p, kin, W, H, o00, du, dv);
    v3 k = unit(ld(kin));
    double d2 = delta * delta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < H; j++) {
        double* hd = (double*)malloc(sizeof(double) * (K + 1));
        int64_t* hi = (int64_t*)malloc(sizeof(int64_t) * (K + 1));
        for (int i = 0; i < W; i++) {
            v3 o = add(ld(o00), add(scl(ld(du), i), scl(ld(dv), j)));
            int n = 0;  /* kept candidates, ascending by (axis distance^2, index) */
            for (int64_t m = 0; m < s->n; m++) {
                v3 w = sub(ld(s->xyz + 3 * m), o);
                double tc = dot(w, k);
                if (!(tc > 0)) continue;
                v3 c = cross(w, k);
                double a2 = dot(c, c);
                if (!(a2 < d2)) continue;
                if (n == K && !(a2 < hd[n - 1])) continue; /* m > kept indices on equal a2 */
                int q = n < K ? n++ : K - 1;
                while (q > 0 && hd[q - 1] > a2) { hd[q] = hd[q - 1]; hi[q] = hi[q - 1]; q--; }
                hd[q] = a2;
                hi[q] = m;
            }
            double bd = INFINITY;
            int64_t best = -1;
            for (int q = 0; q < n; q++) {
                double dist = len(sub(ld(s->xyz + 3 * hi[q]), o));
                if (dist < bd || (dist == bd && hi[q] < best)) { bd = dist; best = hi[q]; }
            }
            int64_t qq = (int64_t)j * W + i;
            depth[qq] = bd;
            idx[qq] = best;
        }
        free(hd);
        free(hi);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Bounce recursion for one central ray (c.6).                                                  */
/* Record per bounce b (22 doubles): x(3) hit point, n(3) oriented normal, kin(3) incoming     */
/* direction, Eth(3) and Eph(3) incoming field for the two incident polarisations, u(3), v(3) */
/* incoming tube vectors, d path length to x by the image method.                              */
/* ------------------------------------------------------------------------------------------ */

#define REC 22

/* ------------------------------------------------------------------------------------------ */
/* Overlap refinement and normal blending of a hit (Sec. III-B, Eq. (23), Fig. 4(a)).          */
/* Reading: the sphere of radius r about the nearest hit P' selects the splats the ray crosses */
/* at or beyond P' within distance r (signed offset s in [-1e-6 R, r] along k, crossing inside */
/* the disk).  The hit moves to the candidate crossed relatively closest to its centre         */
/* (smallest |p_i - c_i| / R_i, ties lowest index), and the normal is Eq. (23): the sum of the */
/* candidates' normals (each turned against the ray) weighted by 1 - |p_i - c_i| / R_i,       */
/* normalised.  Absorbers are not candidates.                                                  */
/* ------------------------------------------------------------------------------------------ */

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void blend_hit(const or_scene* s, v3 xp, v3 k, int64_t h0, v3* x_out, v3* n_out,
                      int64_t* h_out, double* s_out) {
    const double r = s->blend_r, tol = 1e-6 * s->R;
    int64_t* cand = NULL;
    int64_t nc = 0;
    if (s->cell_start) {
        int c0[3], c1[3];
        double xx[3] = {xp.x, xp.y, xp.z};
        for (int a = 0; a < 3; a++) {
            int q0 = (int)floor((xx[a] - r - s->lo[a]) / s->h);
            int q1 = (int)floor((xx[a] + r - s->lo[a]) / s->h);
            c0[a] = q0 < 0 ? 0 : (q0 >= s->G ? s->G - 1 : q0);
            c1[a] = q1 < 0 ? 0 : (q1 >= s->G ? s->G - 1 : q1);
        }
        int64_t cap = 0;
        for (int z = c0[2]; z <= c1[2]; z++)
            for (int y = c0[1]; y <= c1[1]; y++)
                for (int x = c0[0]; x <= c1[0]; x++) {
                    int64_t c = ((int64_t)z * s->G + y) * s->G + x;
                    cap += s->cell_start[c + 1] - s->cell_start[c];
                }
        cand = (int64_t*)malloc(sizeof(int64_t) * (cap + 1));
        for (int z = c0[2]; z <= c1[2]; z++)
            for (int y = c0[1]; y <= c1[1]; y++)
                for (int x = c0[0]; x <= c1[0]; x++) {
                    int64_t c = ((int64_t)z * s->G + y) * s->G + x;
                    for (int64_t j = s->cell_start[c]; j < s->cell_start[c + 1]; j++)
                        cand[nc++] = s->cell_ids[j];
                }
        qsort(cand, (size_t)nc, sizeof(int64_t), cmp_i64);
    } else {
        cand = (int64_t*)malloc(sizeof(int64_t) * (s->n + 1));
        for (int64_t i = 0; i < s->n; i++) cand[nc++] = i;
    }
    int64_t best = -1;
    double best_ratio = INFINITY, best_s = 0;
    v3 acc = mk(0, 0, 0);
    double accw = 0;
    for (int64_t m = 0; m < nc; m++) {
        int64_t i = cand[m];
        if (m > 0 && cand[m - 1] == i) continue; /* a disk listed by several cells */
        if (s->mat[i] != 0) continue;
        v3 c = ld(s->xyz + 3 * i), n = ld(s->nrm + 3 * i);
        double nk = dot(n, k);
        if (fabs(nk) < OR_GRAZE) continue;
        double sv = dot(sub(c, xp), n) / nk;
        if (sv < -tol || sv > r) continue;
        double dd = len(sub(add(xp, scl(k, sv)), c));
        if (!(dd <= s->rad[i])) continue;
        double ratio = dd / s->rad[i];
        if (ratio < best_ratio || (ratio == best_ratio && i < best)) {
            best_ratio = ratio;
            best = i;
            best_s = sv;
        }
        v3 no = nk > 0 ? scl(n, -1.0) : n;
        acc = add(acc, scl(no, 1.0 - ratio));
        accw += 1.0 - ratio;
    }
    free(cand);
    if (best < 0) { /* no candidate: the hit stays as found */
        v3 n = ld(s->nrm + 3 * h0);
        *x_out = xp;
        *n_out = dot(n, k) > 0 ? scl(n, -1.0) : n;
        *h_out = h0;
        *s_out = 0;
        return;
    }
    *x_out = add(xp, scl(k, best_s));
    if (accw > 0 && len(acc) > 0) {
        *n_out = unit(acc);
    } else {
        v3 n = ld(s->nrm + 3 * best);
        *n_out = dot(n, k) > 0 ? scl(n, -1.0) : n;
    }
    *h_out = best;
    *s_out = best_s;
}

void or_scene_set_blend(void* p, double r) { ((or_scene*)p)->blend_r = r > 0 ? r : 0; }

/* Refinement of one hit for the pins: returns the chosen disk, writes the point and normal. */
int64_t or_blend_hit(const void* p, const double* x, const double* k, int64_t h0, double* x_out,
                     double* n_out, double* s_out) {
    v3 xo, no;
    int64_t h;
    blend_hit((const or_scene*)p, ld(x), unit(ld(k)), h0, &xo, &no, &h, s_out);
    st(x_out, xo);
    st(n_out, no);
    return h;
}

/* polarisation basis (theta-hat, phi-hat) of a direction s (spherical angles of s) */
static void pol_basis(v3 s, v3* th, v3* ph) {
    double theta = acos(s.z > 1 ? 1 : (s.z < -1 ? -1 : s.z));
    double phi = atan2(s.y, s.x);
    *th = mk(cos(theta) * cos(phi), cos(theta) * sin(phi), -sin(theta));
    *ph = mk(-sin(phi), cos(phi), 0);
}

static int trace_ray(const or_scene* s, v3 o, v3 k0, v3 u0, v3 v0, int max_b, double eps,
                     int use_grid, int restricted, double* rec, int64_t* hit_idx,
                     int64_t* ntests) {
    v3 th, ph;
    pol_basis(scl(k0, -1.0), &th, &ph);
    v3 k = k0, Et = th, Ep = ph, u = u0, v = v0;
    double d = dot(k0, o);
    int M = 0;
    for (int b = 1; b <= max_b; b++) {
        double t;
        int64_t h = (restricted && b > 1) ? first_hit_views(s, o, k, eps, &t, ntests)
                                          : first_hit(s, o, k, b == 1 ? 0.0 : eps, use_grid, &t,
                                                      ntests);
        if (h < 0) break;
        if (s->mat[h] != 0) break; /* absorber: the ray ends, nothing recorded */
        v3 x = add(o, scl(k, t));
        v3 n = ld(s->nrm + 3 * h);
        if (dot(n, k) > 0) n = scl(n, -1.0);
        if (s->blend_r > 0) {
            double ds;
            blend_hit(s, x, k, h, &x, &n, &h, &ds);
            t += ds;
        }
        double* r = rec + (int64_t)(b - 1) * REC;
        st(r + 0, x); st(r + 3, n); st(r + 6, k); st(r + 9, Et); st(r + 12, Ep);
        st(r + 15, u); st(r + 18, v); r[21] = d + t;
        if (hit_idx) hit_idx[b - 1] = h;
        /* Eq. (4) for k and the tube vectors; Eq. (2)-(3) with Gamma_p = +1, Gamma_v = -1,
         * which for a PEC plane is E_r = 2 (n.E) n - E. */
        k = sub(k, scl(n, 2 * dot(n, k)));
        Et = sub(scl(n, 2 * dot(n, Et)), Et);
        Ep = sub(scl(n, 2 * dot(n, Ep)), Ep);
        u = sub(u, scl(n, 2 * dot(n, u)));
        v = sub(v, scl(n, 2 * dot(n, v)));
        d += t;
        o = x;
        M = b;
    }
    return M;
}

/* Eq. (2)-(3) written as the paper states them: decompose into perpendicular/parallel parts
 * with e_v = k x n / |k x n|, e_p = e_v x k, apply Gamma, recombine. Exposed for the pin that
 * checks it against the vector form used in trace_ray. Requires k not parallel to n. */
void or_reflect_field_decomposed(const double* kin, const double* nin, const double* Ein,
                                 double* Eout, double* kout) {
    v3 k = unit(ld(kin)), n = unit(ld(nin)), E = ld(Ein);
    v3 kr = sub(k, scl(n, 2 * dot(n, k)));
    v3 ev = unit(cross(k, n));
    v3 epi = unit(cross(ev, k));
    v3 epr = unit(cross(ev, kr));
    double Ep = dot(E, epi), Ev = dot(E, ev);
    double Gp = 1.0, Gv = -1.0;
    st(Eout, add(scl(epr, Gp * Ep), scl(ev, Gv * Ev)));
    st(kout, kr);
}

void or_reflect_field_vector(const double* kin, const double* nin, const double* Ein,
                             double* Eout, double* kout) {
    v3 k = unit(ld(kin)), n = unit(ld(nin)), E = ld(Ein);
    st(kout, sub(k, scl(n, 2 * dot(n, k))));
    st(Eout, sub(scl(n, 2 * dot(n, E)), E));
}

void or_pol_basis(const double* s, double* th, double* ph) {
    v3 a, b;
    pol_basis(unit(ld(s)), &a, &b);
    st(th, a);
    st(ph, b);
}

int or_trace_pixels(const void* p, const double* kin, int W, int H, int64_t n_pix,
                    const int64_t* pix, int max_b, double eps, int use_grid, int restricted,
                    int32_t* n_bounce, double* rec, int64_t* hit_idx) {
    const or_scene* s = (const or_scene*)p;
    if (restricted && !s->view_idx) return 1;
    double o00[3], du[3], dv[3];
    or_screen(p, kin, W, H, o00, du, dv);
    v3 k = unit(ld(kin));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t m = 0; m < n_pix; m++) {
        int64_t q = pix[m];
        int i = (int)(q % W), j = (int)(q / W);
        v3 o = add(ld(o00), add(scl(ld(du), i), scl(ld(dv), j)));
        int64_t nt = 0;
        n_bounce[m] = trace_ray(s, o, k, ld(du), ld(dv), max_b, eps, use_grid, restricted,
                                rec + m * (int64_t)max_b * REC,
                                hit_idx ? hit_idx + m * (int64_t)max_b : NULL, &nt);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Field of one facet record toward k_s at wavenumber k (Eq. (11)-(14)).                       */
/* Readings: the parallelogram area is |u' x v'| (the paper's U'V' equals it when u' and v'   */
/* are perpendicular); sinc(x) = sin(x)/x; h = k_in x E_in with |E_i| = 1 so eta_0 cancels;    */
/* time convention exp(+jwt), incident phase exp(-j k.r) about the global origin.              */
/* Adds  -(j k / 2 pi) * psi * area * S * V * exp(-j k (d - k_s . x))  projected on (th, ph)  */
/* of k_s for both transmit polarisations: acc[rx][tx][re,im].                                 */
/* ------------------------------------------------------------------------------------------ */

static inline double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

static void facet_field(const double* r, v3 ks, double kw, v3 rth, v3 rph, double psi,
                        double acc[2][2][2]) {
    v3 x = ld(r + 0), n = ld(r + 3), ki = ld(r + 6), u = ld(r + 15), v = ld(r + 18);
    double d = r[21];
    double nk = dot(n, ki);
    v3 up = sub(u, scl(ki, dot(n, u) / nk));   /* Eq. (12) */
    v3 vp = sub(v, scl(ki, dot(n, v) / nk));   /* Eq. (13) */
    double area = len(cross(up, vp));
    v3 q = scl(sub(ki, ks), kw);
    double S = sinc(0.5 * dot(q, up)) * sinc(0.5 * dot(q, vp));
    double phase = kw * (d - dot(ks, x));
    double a0 = psi * area * S * kw / (2 * OR_PI);
    /* -(j) * exp(-j phase) = -sin(phase) - j cos(phase) */
    double cre = -a0 * sin(phase), cim = -a0 * cos(phase);
    for (int tx = 0; tx < 2; tx++) {
        v3 E = ld(r + (tx == 0 ? 9 : 12));
        v3 hh = cross(ki, E);
        v3 V = cross(cross(cross(n, hh), ks), ks);
        double vp_[2] = {dot(V, rth), dot(V, rph)};
        for (int rx = 0; rx < 2; rx++) {
            acc[rx][tx][0] += vp_[rx] * cre;
            acc[rx][tx][1] += vp_[rx] * cim;
        }
    }
}

/* Visibility Psi of Eq. (14) under the method's rule (restricted solve).  Monostatic: a
 * first-bounce facet is the nearest hit along its own central ray and is visible; a later
 * facet at x is hidden iff a disk stored in the primary first-hit buffer within one pixel of
 * x's projection onto the incidence screen is intersected by the ray from x toward k_s beyond
 * eps.  Bistatic: the restricted first hit from x toward k_s beyond eps is empty. */
static int psi_restricted(const or_scene* s, const int64_t* prim, int W, int H, const double* o00,
                          v3 du, v3 dv, int mono, int bounce, v3 x, v3 ks, double eps,
                          int64_t* nt) {
    double t;
    if (!mono) return first_hit_views(s, x, ks, eps, &t, nt) < 0;
    if (bounce == 1) return 1;
    v3 r = sub(x, ld(o00));
    double pu = len(du), pv = len(dv);
    int ia = (int)floor(dot(r, scl(du, 1.0 / pu)) / pu + 0.5);
    int ib = (int)floor(dot(r, scl(dv, 1.0 / pv)) / pv + 0.5);
    for (int dy = -1; dy <= 1; dy++) {
        int y = ib + dy;
        if (y < 0 || y >= H) continue;
        for (int dx = -1; dx <= 1; dx++) {
            int xx = ia + dx;
            if (xx < 0 || xx >= W) continue;
            int64_t i = prim[(int64_t)y * W + xx];
            if (i < 0) continue;
            (*nt)++;
            if (disk_hit(s, i, x, ks, eps, &t)) return 0;
        }
    }
    return 1;
}

/* Full solve (c.6 + c.7): E[inc][obs][freq][rx][tx][re,im].  obs_dir == NULL means monostatic
 * (k_s = -k_inc).  contrib 0 = last bounce only (Eq. (14)), 1 = every bounce.
 * Visibility psi of a radiating facet: the ray from x toward k_s with tmin = eps hits nothing
 * (exact solve); psi_restricted with restricted != 0, where secondary hits are also restricted
 * to admissible intersections (needs or_scene_set_views).
 * Summation order: pixels row by row; rows summed in order (independent of thread count).
 * stats[0] += ray-disk tests, stats[1] += rays traced (queries), stats[2] += radiating facets. */
int or_solve(const void* p, int n_inc, const double* inc_dir, int n_obs, const double* obs_dir,
             int n_freq, const double* freq, int W, int H, int max_b, double eps, int contrib,
             int use_grid, int restricted, double* E, double* stats) {
    const or_scene* s = (const or_scene*)p;
    if (restricted && !s->view_idx) return 1;
    int mono = obs_dir == NULL;
    int64_t* prim = restricted ? (int64_t*)malloc(sizeof(int64_t) * (int64_t)W * H) : NULL;
    int no = mono ? 1 : n_obs;
    size_t per_row = (size_t)no * n_freq * 8;
    double* rows = (double*)malloc(sizeof(double) * per_row * H);
    int64_t tests = 0, queries = 0, facets = 0;
    for (int ia = 0; ia < n_inc; ia++) {
        double o00[3], du[3], dv[3];
        or_screen(p, inc_dir + 3 * ia, W, H, o00, du, dv);
        v3 k0 = unit(ld(inc_dir + 3 * ia));
        memset(rows, 0, sizeof(double) * per_row * H);
        if (prim) {
#pragma omp parallel for schedule(dynamic, 1)
            for (int j = 0; j < H; j++) {
                int64_t nt = 0;
                for (int i = 0; i < W; i++) {
                    double t;
                    v3 o = add(ld(o00), add(scl(ld(du), i), scl(ld(dv), j)));
                    prim[(int64_t)j * W + i] = first_hit(s, o, k0, 0.0, use_grid, &t, &nt);
                }
            }
        }
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tests, queries, facets)
        for (int j = 0; j < H; j++) {
            double* rec = (double*)malloc(sizeof(double) * REC * max_b);
            double* racc = rows + per_row * j;
            int64_t nt = 0, nq = 0, nf = 0;
            for (int i = 0; i < W; i++) {
                v3 o = add(ld(o00), add(scl(ld(du), i), scl(ld(dv), j)));
                int M = trace_ray(s, o, k0, ld(du), ld(dv), max_b, eps, use_grid, restricted,
                                  rec, NULL, &nt);
                nq += M + (M < max_b ? 1 : 0);
                if (M == 0) continue;
                int b0 = contrib == 1 ? 1 : M;
                for (int io = 0; io < no; io++) {
                    v3 ks = mono ? scl(k0, -1.0) : unit(ld(obs_dir + 3 * io));
                    v3 rth, rph;
                    pol_basis(ks, &rth, &rph);
                    for (int b = b0; b <= M; b++) {
                        const double* r = rec + (int64_t)(b - 1) * REC;
                        double psi;
                        if (restricted) {
                            psi = psi_restricted(s, prim, W, H, o00, ld(du), ld(dv), mono, b,
                                                 ld(r), ks, eps, &nt) ? 1.0 : 0.0;
                        } else {
                            double tv;
                            psi = first_hit(s, ld(r), ks, eps, use_grid, &tv, &nt) >= 0 ? 0.0 : 1.0;
                        }
                        nq++;
                        nf++;
                        if (psi == 0.0) continue;
                        for (int f = 0; f < n_freq; f++) {
                            double kw = 2 * OR_PI * freq[f] / OR_C0;
                            double acc[2][2][2] = {{{0}}};
                            facet_field(r, ks, kw, rth, rph, psi, acc);
                            double* a = racc + ((size_t)io * n_freq + f) * 8;
                            for (int t = 0; t < 8; t++) a[t] += (&acc[0][0][0])[t];
                        }
                    }
                }
            }
            free(rec);
            tests += nt;
            queries += nq;
            facets += nf;
        }
        double* out = E + (size_t)ia * per_row;
        memset(out, 0, sizeof(double) * per_row);
        for (int j = 0; j < H; j++)
            for (size_t t = 0; t < per_row; t++) out[t] += rows[per_row * j + t];
    }
    free(rows);
    free(prim);
    if (stats) {
        stats[0] += (double)tests;
        stats[1] += (double)queries;
        stats[2] += (double)facets;
    }
    return 0;
}

int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_num_threads(int n) { omp_set_num_threads(n); }
