"""GFB edge filtering and fusion into splats -- TEST INFRASTRUCTURE ONLY.

Restates Algorithm 3's EdgeFilteringAndFusion step and Eq. (22) (Sec. III-B) in plain NumPy:
a Canny operator removes the edge portions of each geometric frame buffer (GFB), the kept
pixels are placed in a cubic grid and averaged per cell, and each occupied cell becomes one
splat whose radius follows Eq. (22).

Readings of the paper (it names the operator, the grid and Eq. (22), not their details):
  - Canny runs on the depth map in metres, empty pixels set to the far side of the scene (2R),
    so silhouettes are edges; smoothing is a 5 x 5 Gaussian of sigma 1 pixel (clamp-to-edge),
    the gradient is Sobel, non-maximum suppression quantises the gradient direction to
    0/45/90/135 degrees, the two thresholds are depth slopes (depth change per pixel pitch), and
    hysteresis keeps weak pixels 8-connected through weak pixels to a strong one.
  - Pixels within `dilate` pixels of an edge are dropped with it.
  - The grid is a cube of `side` about the frame centre with G cells per axis; L of Eq. (22)
    is its cell edge.  Points up to one cell outside go to the boundary cell.
  - A splat's normal is the normalised sum of its pixels' unit normals, each first turned so
    that its largest component is positive (splats are two-sided); p of Eq. (22) is the
    projection direction of a contributing view, and the splat takes the smallest radius over
    its contributing views.

Everything is computed in fp64 from the buffers' values.  Decisions that turn floating point
into an integer or a branch (edge classes, the grid cell of a point, the side a normal is
turned to) are reported with an ambiguity flag where their fp64 margin is within reach of fp32
rounding: a fp32 implementation may take those the other way, and the tests bound where such
flips may appear.  The reach is stated with generous factors on the fp32 unit roundoff u:
  - Canny: every gradient component within 256 u D of its fp64 value (25 blur taps of depths up
    to D = 2R, then 8 Sobel terms), so m = gx^2 + gy^2 moves by up to 2 e (|g| + |g'|) + e^2;
  - cells: a point's grid coordinate within 32 u R / L (the point is two products and sums of
    size R on fp32-rounded screen axes, about 17 u R, then shifted by half the side and divided
    by L, about 4 u R / L more in grid units); such a point may land in the neighbouring cell
    across each face within reach, and every cell it may land in is reported;
  - normal side: the largest and second largest |component| of the turned normal within 1e-5.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import ndimage

U32 = 2.0 ** -24  # fp32 unit roundoff


def screen_basis(k):
    """Screen axes of a propagation direction: u = normalise(z x k) (x when k is within 1e-9 of
    +-z), v = k x u, k normalised (the screen frame of every GFB)."""
    k = np.asarray(k, np.float64)
    k = k / np.linalg.norm(k)
    if abs(k[2]) > 1.0 - 1e-9:
        u = np.array([1.0, 0.0, 0.0])
    else:
        u = np.cross([0.0, 0.0, 1.0], k)
        u = u / np.linalg.norm(u)
    return u, np.cross(k, u), k


def gaussian_taps():
    """Weights of the 5-tap Gaussian, sigma = 1 pixel, at offsets 0, 1, 2."""
    e = [math.exp(-0.5 * d * d) for d in range(3)]
    s = e[0] + 2.0 * (e[1] + e[2])
    return [x / s for x in e]


def canny(depth, hit, R, lo, hi, ambiguity=False):
    """Edge map (bool, n x h x w) of depth buffers (t / 2R) per the readings above; with
    ambiguity=True also the map of pixels whose class (strong / weak / none after non-maximum
    suppression, or the suppression direction) is within fp32 reach of changing, and the map of
    candidates (strong or weak, or ambiguous) through which hysteresis can carry a change."""
    depth = np.asarray(depth, np.float64)
    n, h, w = depth.shape
    D = 2.0 * float(R)
    d = np.where(np.asarray(hit, np.float64) >= 0.5, depth * D, D)
    g = gaussian_taps()
    gw = [g[2], g[1], g[0], g[1], g[2]]
    dp = np.pad(d, ((0, 0), (2, 2), (2, 2)), mode="edge")
    blur = np.zeros_like(d)
    for dy in range(5):
        for dx in range(5):
            blur = blur + gw[dy] * gw[dx] * dp[:, dy:dy + h, dx:dx + w]
    # Sobel sums at every pixel and one ring outside (clamped reads = edge padding)
    bp = np.pad(blur, ((0, 0), (2, 2), (2, 2)), mode="edge")

    def B(ox, oy):  # blurred value at (x + ox, y + oy) for x in -1..w, y in -1..h
        return bp[:, 1 + oy:1 + oy + h + 2, 1 + ox:1 + ox + w + 2]

    gx = (B(1, -1) + 2.0 * B(1, 0) + B(1, 1)) - (B(-1, -1) + 2.0 * B(-1, 0) + B(-1, 1))
    gy = (B(-1, 1) + 2.0 * B(0, 1) + B(1, 1)) - (B(-1, -1) + 2.0 * B(0, -1) + B(1, -1))
    m2 = gx * gx + gy * gy  # indexed [v, y + 1, x + 1]
    tl, th = lo * 16.0 * R / w, hi * 16.0 * R / w
    t2lo, t2hi = tl * tl, th * th
    tan22 = math.sqrt(2.0) - 1.0
    m = m2[:, 1:h + 1, 1:w + 1]
    gxc, gyc = gx[:, 1:h + 1, 1:w + 1], gy[:, 1:h + 1, 1:w + 1]
    ax, ay = np.abs(gxc), np.abs(gyc)
    horiz = ay <= tan22 * ax
    vert = ~horiz & (ax <= tan22 * ay)
    diag = ~horiz & ~vert & ((gxc > 0) == (gyc > 0))
    dx = np.where(horiz, 1, np.where(vert, 0, 1))
    dy = np.where(horiz, 0, np.where(vert, 1, np.where(diag, 1, -1)))
    vi, yi, xi = np.meshgrid(np.arange(n), np.arange(h), np.arange(w), indexing="ij")
    m1 = m2[vi, yi + 1 + dy, xi + 1 + dx]
    mm = m2[vi, yi + 1 - dy, xi + 1 - dx]
    keep = (m >= t2lo) & (m >= m1) & (m >= mm)
    strong = keep & (m >= t2hi)
    weak = keep & ~strong
    edges = np.stack([hysteresis(strong[v], weak[v]) for v in range(n)])
    if not ambiguity:
        return edges
    e = 256.0 * U32 * D  # reach of a gradient component

    def near_sq(a, b):  # squared magnitudes a, b within reach of each other
        return np.abs(a - b) <= 2.0 * e * (np.sqrt(a) + np.sqrt(b)) + e * e

    relevant = (m >= t2lo) | near_sq(m, t2lo)  # below it a pixel is no edge either way
    amb = (near_sq(m, t2lo) | near_sq(m, t2hi) |
           (relevant & (near_sq(m, m1) | near_sq(m, mm) |
                        (np.abs(ay - tan22 * ax) <= 2.0 * e) |
                        (np.abs(ax - tan22 * ay) <= 2.0 * e) |
                        (np.minimum(ax, ay) <= e))))
    return edges, amb, keep | amb


def hysteresis(strong, weak):
    """Strong pixels plus every weak pixel 8-connected to one through weak pixels (one 2-D map):
    the 8-connected components of strong | weak that hold a strong pixel."""
    lab, _ = ndimage.label(strong | weak, structure=np.ones((3, 3), bool))
    ids = np.unique(lab[strong])
    return np.isin(lab, ids[ids > 0])


def eq22_radius(cos_np, L):
    """Eq. (22) with unit n and p: sqrt(2) L sqrt(1/|n.p|) below the bound 2.5 on
    sqrt(1/|n.p|), else 3.535 L."""
    c = np.abs(np.asarray(cos_np, np.float64))
    with np.errstate(divide="ignore"):
        f = np.where(c > 0, np.sqrt(1.0 / np.where(c > 0, c, 1.0)), np.inf)
    return np.where(f < 2.5, math.sqrt(2.0) * L * f, 3.535 * L)


def fuse(view_dirs, depth, nrm, hit, centre, R, grid=256, side=0.0, lo=2.0, hi=4.0, dilate=1):
    """Splats from GFBs: dict of xyz (world), nrm, radius, count (pixels per splat), cell (flat
    index, x fastest) and edge (the Canny map), splats in cell order; coherence and best_cos
    (the |n.p| the radius was taken at) describe each splat's conditioning.  Per pixel: edge_amb
    (the Canny decision is ambiguous), edge_cand (see canny), pix_cell (grid cell of each hit
    pixel, -1 elsewhere) and pix_amb (its cell or its normal's side is ambiguous); amb_cells
    lists every cell that a pixel with an ambiguous cell decision may land in."""
    depth = np.asarray(depth, np.float64)
    nrm = np.asarray(nrm, np.float64)
    hit = np.asarray(hit, np.float64)
    n, h, w = depth.shape
    G = int(grid)
    side = float(side) if side > 0 else 2.0 * R
    edge, edge_amb, edge_cand = canny(depth, hit, R, lo, hi, ambiguity=True)
    if dilate > 0:
        st = np.ones((1, 2 * dilate + 1, 2 * dilate + 1), bool)
        drop = ndimage.binary_dilation(edge, structure=st)
    else:
        drop = edge
    is_hit = hit >= 0.5
    keep = is_hit & ~drop
    half, L = 0.5 * side, side / G
    reach_cell = 32.0 * U32 * R / L
    pix_cell = np.full((n, h, w), -1, np.int64)
    pix_amb = np.zeros((n, h, w), bool)
    P_all, N_all, C_all, V_all, A_all = [], [], [], [], []
    for v in range(n):
        u, vv, k = screen_basis(view_dirs[v])
        ys, xs = np.nonzero(is_hit[v])
        dep, nv3 = depth[v, ys, xs], nrm[v, ys, xs]
        tt = dep * 2.0 * R - R
        pu = (xs + 0.5 - 0.5 * w) * (2.0 * R / w)
        pv = (ys + 0.5 - 0.5 * h) * (2.0 * R / w)
        P = pu[:, None] * u + pv[:, None] * vv + tt[:, None] * k
        N = nv3[:, 0:1] * u + nv3[:, 1:2] * vv - nv3[:, 2:3] * k
        g = (P + half) / L
        q = np.floor(g).astype(np.int64)
        q[q == -1] = 0
        q[q == G] = G - 1
        fr = g - np.floor(g)
        amb_cell = np.any(np.minimum(fr, 1 - fr) <= reach_cell, 1)
        qa, fa = np.floor(g[amb_cell]).astype(np.int64), fr[amb_cell]
        for off in np.ndindex(3, 3, 3):  # the cell itself and its neighbours across near faces
            o3 = np.array(off) - 1
            ok_o = np.all(((o3 != -1) | (fa <= reach_cell)) & ((o3 != 1) | (1 - fa <= reach_cell)),
                          1)
            qo = qa + o3
            qo[qo == -1] = 0
            qo[qo == G] = G - 1
            ok_o &= np.all((qo >= 0) & (qo < G), 1)
            A_all.append(((qo[:, 2] * G + qo[:, 1]) * G + qo[:, 0])[ok_o])
        inside = np.all((q >= 0) & (q < G), 1) & np.any(N != 0, 1)
        aN = np.abs(N)
        am = np.argmax(aN, 1)
        top = aN[np.arange(len(am)), am]
        second = np.sort(aN, 1)[:, 1]
        amb_sign = (top - second <= 1e-5) | (top <= 1e-5)
        sgn = np.where(N[np.arange(len(am)), am] < 0, -1.0, 1.0)
        N = N / np.linalg.norm(N, axis=1, keepdims=True).clip(1e-300) * sgn[:, None]
        cell = (q[:, 2] * G + q[:, 1]) * G + q[:, 0]
        pix_cell[v, ys[inside], xs[inside]] = cell[inside]
        pix_amb[v, ys, xs] = amb_cell | amb_sign
        ok = inside & keep[v, ys, xs]
        P_all.append(P[ok]); N_all.append(N[ok]); C_all.append(cell[ok])
        V_all.append(np.full(int(ok.sum()), v))
    P, N, C, V = (np.concatenate(a) for a in (P_all, N_all, C_all, V_all))
    cells, inv, cnt = np.unique(C, return_inverse=True, return_counts=True)
    m = len(cells)
    Ps = np.zeros((m, 3)); Ns = np.zeros((m, 3))
    np.add.at(Ps, inv, P)
    np.add.at(Ns, inv, N)
    xyz = Ps / cnt[:, None] + np.asarray(centre, np.float64)
    nl = np.linalg.norm(Ns, axis=1, keepdims=True)
    nf = np.where(nl > 0, Ns / np.where(nl > 0, nl, 1.0), np.array([0.0, 0.0, 1.0]))
    kv = np.stack([screen_basis(d)[2] for d in view_dirs])
    best = np.zeros(m)
    for v in range(n):
        has = np.zeros(m, bool)
        has[np.unique(inv[V == v])] = True
        best = np.where(has, np.maximum(best, np.abs(nf @ kv[v])), best)
    radius = eq22_radius(best, side / G)
    # conditioning of each splat's normal: |sum of unit normals| / count (near 0 when they
    # nearly cancel, where any rounding in the inputs is amplified by 1 / coherence)
    return dict(xyz=xyz, nrm=nf, radius=radius, count=cnt, cell=cells, edge=edge,
                coherence=nl[:, 0] / cnt, best_cos=best, edge_amb=edge_amb, edge_cand=edge_cand,
                pix_cell=pix_cell, pix_amb=pix_amb, amb_cells=np.unique(np.concatenate(A_all)))
