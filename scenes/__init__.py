"""Seeded synthetic scenes and sweep definitions shared by the oracle, the tests and the bench.

This module only produces *inputs*: point positions, unit normals, splat radii, material flags,
incidence directions, frequencies and the scalar knobs of a run.  It holds none of the method's
arithmetic (no screens, no intersections, no fields), so the oracle and the HIP path can both
consume it without sharing any computation.

The paper's own workloads are meshes from a public model repository sampled into 10k-50k point
clouds, scaled to 20 m and simulated at 500 MHz with a ray spacing of a tenth of a wavelength
(Sec. IV-A).  Those meshes are not available here; the seeded analytic scenes below stand in for
them with the same structure (point-sampled PEC surfaces with exact normals, uniform area
density, optional Gaussian position noise) at electrically larger sizes.

All random numbers come from NumPy's PCG64 with the stated seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C0 = 299_792_458.0  # speed of light in vacuum, m/s

MAT_PEC = 0
MAT_ABSORBER = 1


@dataclass
class Scene:
    """A point-sampled surface: positions (n,3) f64, unit normals (n,3) f64, radius, material."""

    xyz: np.ndarray
    nrm: np.ndarray
    radius: float | np.ndarray
    material: np.ndarray
    name: str = ""
    noise_sigma: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    def radius_array(self) -> np.ndarray:
        if np.isscalar(self.radius):
            return np.full(self.n, float(self.radius))
        return np.asarray(self.radius, dtype=np.float64)


@dataclass
class Sweep:
    """What to solve on a scene: incidence propagation directions, frequencies and knobs."""

    inc_dir: np.ndarray          # (n_inc, 3) unit propagation directions of the incident wave
    freq_hz: np.ndarray          # (n_freq,)
    screen: int                  # square ray screen, pixels per side
    max_bounces: int
    eps: float                   # minimum travel distance of secondary rays (m)
    view_res: int                # resolution of the aggregation views
    view_dirs: np.ndarray | None = None  # None -> the six axis views
    obs_dir: np.ndarray | None = None    # None -> monostatic
    az_deg: np.ndarray | None = None
    el_deg: float = 0.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def azimuth_sweep(az_deg, el_deg: float) -> np.ndarray:
    """Propagation directions of plane waves arriving FROM azimuth az at elevation el."""
    az = np.radians(np.asarray(az_deg, dtype=np.float64))
    el = math.radians(el_deg)
    src = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az),
                    np.full_like(az, np.sin(el))], axis=1)
    return -src


def random_unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


# ---------------------------------------------------------------------------------------------
# Dihedral: two square plates meeting at a right angle (the small case the oracle finishes).
# ---------------------------------------------------------------------------------------------

def dihedral(seed: int = 1, n_side: int = 100, size: float = 0.3, jitter: float = 0.2,
             radius_factor: float = 1.5) -> Scene:
    """Plate A on y=0 (normal +y, x in [0,size]), plate B on x=0 (normal +x, y in [0,size]);
    both span z in [-size/2, size/2].  Each plate is an n_side x n_side cell-centred grid with
    uniform in-plane jitter of +-jitter*spacing.  Splat radius = radius_factor * spacing."""
    rng = _rng(seed)
    s = size / n_side
    g = (np.arange(n_side) + 0.5) * s
    a, b = np.meshgrid(g, g - size / 2, indexing="ij")
    a = a.ravel()
    b = b.ravel()
    n = a.size
    ja = rng.uniform(-jitter * s, jitter * s, n)
    jb = rng.uniform(-jitter * s, jitter * s, n)
    plate_a = np.stack([a + ja, np.zeros(n), b + jb], axis=1)
    ja = rng.uniform(-jitter * s, jitter * s, n)
    jb = rng.uniform(-jitter * s, jitter * s, n)
    plate_b = np.stack([np.zeros(n), a + ja, b + jb], axis=1)
    xyz = np.concatenate([plate_a, plate_b])
    nrm = np.concatenate([np.tile([0.0, 1.0, 0.0], (n, 1)), np.tile([1.0, 0.0, 0.0], (n, 1))])
    return Scene(xyz=xyz, nrm=nrm, radius=radius_factor * s, material=np.zeros(2 * n, np.uint8),
                 name="dihedral", meta=dict(size=size, spacing=s, n_side=n_side))


def plate(seed: int = 1, n_side: int = 100, size: float = 0.3, jitter: float = 0.2,
          radius_factor: float = 1.5) -> Scene:
    """A single square plate on x=0 with normal +x (plate B of the dihedral, alone)."""
    d = dihedral(seed, n_side, size, jitter, radius_factor)
    n = n_side * n_side
    return Scene(xyz=d.xyz[n:].copy(), nrm=d.nrm[n:].copy(), radius=d.radius,
                 material=np.zeros(n, np.uint8), name="plate", meta=d.meta)


def _jittered_plate(rng, u_rng, v_rng, n_u, n_v, jitter):
    """Cell-centred jittered grid over [u0,u1] x [v0,v1]; returns (u, v) arrays and spacing."""
    su = (u_rng[1] - u_rng[0]) / n_u
    sv = (v_rng[1] - v_rng[0]) / n_v
    u, v = np.meshgrid(u_rng[0] + (np.arange(n_u) + 0.5) * su,
                       v_rng[0] + (np.arange(n_v) + 0.5) * sv, indexing="ij")
    u = u.ravel() + rng.uniform(-jitter * su, jitter * su, u.size)
    v = v.ravel() + rng.uniform(-jitter * sv, jitter * sv, v.size)
    return u, v, max(su, sv)


def trihedral(seed: int = 6, n_side: int = 100, size: float = 0.3, jitter: float = 0.2,
              radius_factor: float = 1.5) -> Scene:
    """Square trihedral corner in the first octant: plates on z=0, y=0 and x=0 (normals +z, +y,
    +x), each size x size, sampled like the dihedral's plates."""
    rng = _rng(seed)
    parts, nrms = [], []
    for axis in (2, 1, 0):
        u, v, s = _jittered_plate(rng, (0.0, size), (0.0, size), n_side, n_side, jitter)
        p = np.zeros((u.size, 3))
        others = [a for a in range(3) if a != axis]
        p[:, others[0]] = u
        p[:, others[1]] = v
        nn = np.zeros((u.size, 3))
        nn[:, axis] = 1.0
        parts.append(p)
        nrms.append(nn)
    xyz = np.concatenate(parts)
    return Scene(xyz=xyz, nrm=np.concatenate(nrms), radius=radius_factor * size / n_side,
                 material=np.zeros(len(xyz), np.uint8), name="trihedral",
                 meta=dict(size=size, spacing=size / n_side))


def octar(seed: int = 7, half: float = 1.0, spacing: float = 0.01, jitter: float = 0.2,
          radius_factor: float = 1.5, noise_sigma: float = 0.0) -> Scene:
    """Three mutually orthogonal square plates through the origin, each spanning
    [-half, half]^2: eight square trihedral corners of edge `half` (a synthetic stand-in for the
    OctAR target).  Two-sided disks on a jittered grid of the given spacing; optional Gaussian
    position noise (exact normals kept)."""
    rng = _rng(seed)
    n = int(round(2 * half / spacing))
    parts, nrms = [], []
    for axis in (2, 1, 0):
        u, v, s = _jittered_plate(rng, (-half, half), (-half, half), n, n, jitter)
        p = np.zeros((u.size, 3))
        others = [a for a in range(3) if a != axis]
        p[:, others[0]] = u
        p[:, others[1]] = v
        nn = np.zeros((u.size, 3))
        nn[:, axis] = 1.0
        parts.append(p)
        nrms.append(nn)
    xyz = np.concatenate(parts)
    if noise_sigma > 0:
        xyz = xyz + rng.normal(0.0, noise_sigma, xyz.shape)
    return Scene(xyz=xyz, nrm=np.concatenate(nrms), radius=radius_factor * spacing,
                 material=np.zeros(len(xyz), np.uint8), name="octar", noise_sigma=noise_sigma,
                 meta=dict(half=half, spacing=spacing))


def octar_views() -> np.ndarray:
    """The eight sensor positions of the OctAR experiment (theta in {60, 120} deg, phi in
    {45, 135, 225, 315} deg) as propagation directions (sensor toward the target)."""
    out = []
    for th in (60.0, 120.0):
        for ph in (45.0, 135.0, 225.0, 315.0):
            t, p = math.radians(th), math.radians(ph)
            out.append([-math.sin(t) * math.cos(p), -math.sin(t) * math.sin(p), -math.cos(t)])
    return np.array(out)


def corner_assembly(seed: int, n_points: int = 200_000, size: float = 1.0,
                    jitter: float = 0.2, radius_factor: float = 1.5) -> Scene:
    """Concave corners (training data of the same structure as corner reflectors, never the
    OctAR itself): one to three vertices, each with three edge vectors at pairwise angles in
    [60, 120] deg and lengths in [0.4, 1] x size; the parallelogram spanned by each pair of
    edges is a plate (one of the three is dropped with probability 0.3, leaving a dihedral),
    placed with a random rotation and offset.  Plates are sampled on jittered grids at a common
    spacing so that the assembly holds about n_points points; exact normals."""
    rng = _rng(seed)
    n_vert = int(rng.integers(1, 4))
    plates = []  # (origin, edge a, edge b)
    for _ in range(n_vert):
        while True:
            e = random_unit_vectors(rng, 3)
            c = [abs(float(e[i] @ e[j])) for i, j in ((0, 1), (0, 2), (1, 2))]
            if max(c) <= 0.5 and abs(float(np.linalg.det(e))) > 0.3:
                break
        e = e * rng.uniform(0.4, 1.0, (3, 1)) * size
        o = rng.uniform(-0.5, 0.5, 3) * size * (n_vert > 1)
        pairs = [(0, 1), (0, 2), (1, 2)]
        if rng.uniform() < 0.3:
            pairs.pop(int(rng.integers(3)))
        for i, j in pairs:
            plates.append((o, e[i], e[j]))
    areas = np.array([np.linalg.norm(np.cross(a, b)) for _, a, b in plates])
    spacing = math.sqrt(areas.sum() / n_points)
    parts, nrms = [], []
    for (o, a, b), A in zip(plates, areas):
        na = max(2, int(round(np.linalg.norm(a) / spacing)))
        nb = max(2, int(round(A / np.linalg.norm(a) / spacing)))
        u, v, _ = _jittered_plate(rng, (0.0, 1.0), (0.0, 1.0), na, nb, jitter)
        parts.append(o + u[:, None] * a + v[:, None] * b)
        n = np.cross(a, b)
        nrms.append(np.tile(n / np.linalg.norm(n), (u.size, 1)))
    rot = _random_rotation(rng)
    xyz = np.concatenate(parts) @ rot.T
    nrm = np.concatenate(nrms) @ rot.T
    return Scene(xyz=xyz, nrm=nrm, radius=radius_factor * spacing,
                 material=np.zeros(len(xyz), np.uint8), name="corners",
                 meta=dict(spacing=spacing, plates=len(plates)))


def synthetic_gfbs(seed: int, n_views: int, res: int, n_regions: int = 4,
                   soft_hit: bool = False) -> dict:
    """GFB-shaped input buffers for the fusion step, with the structure of rendered or predicted
    frame buffers: each view holds a few elliptical regions (the hit mask) of smooth depth
    (a tilted ramp plus gentle ripples, t/D in [0.15, 0.85]), regions in front of one another
    with depth steps between them, and a smooth unit normal field per region facing the screen
    (third component, along -k, positive).  soft_hit=True gives probabilities in (0, 1) instead
    of a 0/1 mask.  Returns float32 arrays depth [n,res,res], nrm [n,res,res,3], hit
    [n,res,res] and float64 view_dirs [n,3] (random unit vectors)."""
    rng = _rng(seed)
    yy, xx = np.meshgrid(np.linspace(-1, 1, res), np.linspace(-1, 1, res), indexing="ij")
    depth = np.zeros((n_views, res, res))
    nrm = np.zeros((n_views, res, res, 3))
    hit = np.zeros((n_views, res, res))
    for v in range(n_views):
        zbuf = np.full((res, res), np.inf)
        for _ in range(n_regions):
            cx, cy = rng.uniform(-0.5, 0.5, 2)
            a, b = rng.uniform(0.25, 0.6, 2)
            th = rng.uniform(0, math.pi)
            xr = (xx - cx) * math.cos(th) + (yy - cy) * math.sin(th)
            yr = -(xx - cx) * math.sin(th) + (yy - cy) * math.cos(th)
            inside = (xr / a) ** 2 + (yr / b) ** 2 <= 1.0
            d0 = rng.uniform(0.3, 0.6)
            gx, gy = rng.uniform(-0.15, 0.15, 2)
            amp, fx, fy = rng.uniform(0.0, 0.03), rng.uniform(1, 4), rng.uniform(1, 4)
            d = d0 + gx * xx + gy * yy + amp * np.sin(fx * xx * math.pi) * np.cos(fy * yy * math.pi)
            d = np.clip(d, 0.15, 0.85)
            n0 = rng.normal(0, 0.4, 3)
            n0[2] = abs(n0[2]) + 0.5
            nf = np.stack([n0[0] + 0.2 * np.sin(2 * xx + v), n0[1] + 0.2 * np.cos(3 * yy - v),
                           np.full_like(xx, n0[2])], -1)
            nf /= np.linalg.norm(nf, axis=-1, keepdims=True)
            front = inside & (d < zbuf)
            zbuf[front] = d[front]
            depth[v][front] = d[front]
            nrm[v][front] = nf[front]
            hit[v][front] = 1.0
        if soft_hit:
            p = rng.uniform(0.02, 0.45, hit[v].shape)
            hit[v] = np.where(hit[v] > 0, 1.0 - p, p)
    return dict(depth=depth.astype(np.float32), nrm=nrm.astype(np.float32),
                hit=hit.astype(np.float32), view_dirs=random_unit_vectors(rng, n_views))


# ---------------------------------------------------------------------------------------------
# Analytic primitives for the composite scene.
# ---------------------------------------------------------------------------------------------

def _box_sample(rng, dims, m):
    a, b, c = dims
    areas = np.array([b * c, b * c, a * c, a * c, a * b, a * b])
    face = rng.choice(6, size=m, p=areas / areas.sum())
    u = rng.uniform(-0.5, 0.5, m)
    v = rng.uniform(-0.5, 0.5, m)
    p = np.zeros((m, 3))
    nrm = np.zeros((m, 3))
    for f in range(6):
        sel = face == f
        axis, sign = f // 2, (1.0 if f % 2 == 0 else -1.0)
        o1, o2 = [ax for ax in range(3) if ax != axis]
        p[sel, axis] = sign * dims[axis] / 2
        p[sel, o1] = u[sel] * dims[o1]
        p[sel, o2] = v[sel] * dims[o2]
        nrm[sel, axis] = sign
    return p, nrm, float(areas.sum())


def _cylinder_sample(rng, r, h, m):
    a_lat = 2 * math.pi * r * h
    a_cap = math.pi * r * r
    areas = np.array([a_lat, a_cap, a_cap])
    part = rng.choice(3, size=m, p=areas / areas.sum())
    p = np.zeros((m, 3))
    nrm = np.zeros((m, 3))
    lat = part == 0
    phi = rng.uniform(0, 2 * math.pi, lat.sum())
    p[lat, 0] = r * np.cos(phi)
    p[lat, 1] = r * np.sin(phi)
    p[lat, 2] = rng.uniform(-h / 2, h / 2, lat.sum())
    nrm[lat, 0] = np.cos(phi)
    nrm[lat, 1] = np.sin(phi)
    for k, sign in ((1, 1.0), (2, -1.0)):
        sel = part == k
        rr = r * np.sqrt(rng.uniform(0, 1, sel.sum()))
        ph = rng.uniform(0, 2 * math.pi, sel.sum())
        p[sel, 0] = rr * np.cos(ph)
        p[sel, 1] = rr * np.sin(ph)
        p[sel, 2] = sign * h / 2
        nrm[sel, 2] = sign
    return p, nrm, float(areas.sum())


def _sphere_sample(rng, r, m):
    d = random_unit_vectors(rng, m)
    return r * d, d.copy(), 4 * math.pi * r * r


def _plate_sample(rng, a, b, m):
    p = np.zeros((m, 3))
    p[:, 0] = rng.uniform(-a / 2, a / 2, m)
    p[:, 1] = rng.uniform(-b / 2, b / 2, m)
    nrm = np.zeros((m, 3))
    nrm[:, 2] = 1.0
    return p, nrm, a * b


def _split_counts(n_total: int, areas: np.ndarray) -> np.ndarray:
    share = n_total * areas / areas.sum()
    counts = np.floor(share).astype(np.int64)
    rem = n_total - counts.sum()
    order = np.argsort(-(share - counts), kind="stable")
    counts[order[:rem]] += 1
    return counts


def composite(seed: int = 2, n_points: int = 2_000_000, noise_sigma: float | None = None,
              n_prims: int = 12, slab=(6.0, 6.0, 2.0), radius_factor: float = 1.5) -> Scene:
    """Twelve primitives cycling box / capped cylinder / sphere / two-sided plate, each with a
    random orientation, centres in a slab with bounding-sphere rejection (no overlap; a
    primitive that cannot be placed after 2000 tries is shrunk by 0.85 and tried again).
    Points are split between primitives by area (uniform density); positions get isotropic
    Gaussian noise of sigma (default: a fiftieth of the wavelength at 12 GHz); normals are the
    exact analytic normals at the unperturbed sample.  radius = radius_factor*sqrt(area/N)."""
    rng = _rng(seed)
    if noise_sigma is None:
        noise_sigma = C0 / 12e9 / 50
    kinds = ["box", "cylinder", "sphere", "plate"]
    prims = []
    for i in range(n_prims):
        kind = kinds[i % 4]
        if kind == "box":
            params = rng.uniform(0.2, 2.0, 3)
        elif kind == "cylinder":
            params = np.array([rng.uniform(0.1, 1.0), rng.uniform(0.2, 2.0)])
        elif kind == "sphere":
            params = np.array([rng.uniform(0.1, 1.0)])
        else:
            params = rng.uniform(0.2, 2.0, 2)
        rot = _random_rotation(rng)
        prims.append([kind, params, rot, None])

    def bound(kind, p):
        if kind == "box":
            return 0.5 * float(np.linalg.norm(p))
        if kind == "cylinder":
            return float(math.hypot(p[0], p[1] / 2))
        if kind == "sphere":
            return float(p[0])
        return 0.5 * float(math.hypot(p[0], p[1]))

    placed = []
    half = np.array(slab) / 2
    for pr in prims:
        while True:
            rb = bound(pr[0], pr[1])
            ok = False
            for _ in range(2000):
                c = rng.uniform(-half, half)
                if all(np.linalg.norm(c - c2) > rb + r2 for c2, r2 in placed):
                    ok = True
                    break
            if ok:
                pr[3] = c
                placed.append((c, rb))
                break
            pr[1] = pr[1] * 0.85

    areas = []
    for kind, p, _, _ in prims:
        if kind == "box":
            a, b, c = p
            areas.append(2 * (a * b + b * c + a * c))
        elif kind == "cylinder":
            areas.append(2 * math.pi * p[0] * p[1] + 2 * math.pi * p[0] ** 2)
        elif kind == "sphere":
            areas.append(4 * math.pi * p[0] ** 2)
        else:
            areas.append(p[0] * p[1])
    areas = np.array(areas)
    counts = _split_counts(n_points, areas)
    xs, ns = [], []
    for (kind, p, rot, c), m in zip(prims, counts):
        if kind == "box":
            pts, nr, _ = _box_sample(rng, p, m)
        elif kind == "cylinder":
            pts, nr, _ = _cylinder_sample(rng, p[0], p[1], m)
        elif kind == "sphere":
            pts, nr, _ = _sphere_sample(rng, p[0], m)
        else:
            pts, nr, _ = _plate_sample(rng, p[0], p[1], m)
        xs.append(pts @ rot.T + c)
        ns.append(nr @ rot.T)
    xyz = np.concatenate(xs)
    nrm = np.concatenate(ns)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    if noise_sigma > 0:
        xyz = xyz + rng.normal(0.0, noise_sigma, xyz.shape)
    radius = radius_factor * math.sqrt(areas.sum() / n_points)
    meta = dict(prims=[(k, np.asarray(p).tolist(), np.asarray(c).tolist()) for k, p, _, c in prims],
                area=float(areas.sum()))
    return Scene(xyz=xyz, nrm=nrm, radius=radius, material=np.zeros(n_points, np.uint8),
                 name="composite", noise_sigma=noise_sigma, meta=meta)


def sphere(seed: int = 3, n_points: int = 4_000_000, a: float = 4.0,
           noise_sigma: float | None = None, radius_factor: float = 1.5) -> Scene:
    """Points uniform on a sphere of radius a (normalised Gaussians), radial normals, Gaussian
    position noise (default: a fiftieth of the wavelength at 24 GHz)."""
    rng = _rng(seed)
    if noise_sigma is None:
        noise_sigma = C0 / 24e9 / 50
    d = random_unit_vectors(rng, n_points)
    xyz = a * d
    if noise_sigma > 0:
        xyz = xyz + rng.normal(0.0, noise_sigma, xyz.shape)
    radius = radius_factor * math.sqrt(4 * math.pi * a * a / n_points)
    return Scene(xyz=xyz, nrm=d, radius=radius, material=np.zeros(n_points, np.uint8),
                 name="sphere", noise_sigma=noise_sigma, meta=dict(a=a))


def random_disks(seed: int, n: int, extent: float = 1.0, r_lo: float = 0.05,
                 r_hi: float = 0.2, absorber_frac: float = 0.0) -> Scene:
    """Tiny random clouds for exhaustive tests: centres uniform in a cube, random normals,
    per-point radii, optionally some absorbers."""
    rng = _rng(seed)
    xyz = rng.uniform(-extent / 2, extent / 2, (n, 3))
    nrm = random_unit_vectors(rng, n)
    radius = rng.uniform(r_lo, r_hi, n)
    mat = (rng.uniform(0, 1, n) < absorber_frac).astype(np.uint8)
    return Scene(xyz=xyz, nrm=nrm, radius=radius, material=mat, name="random_disks")


# ---------------------------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------------------------

def workload_dihedral() -> tuple[Scene, Sweep]:
    """Dihedral of two 0.3 m plates, 256^2 screen, 10 GHz, <=2 bounces, azimuth 0..90 deg."""
    sc = dihedral(seed=1)
    az = np.arange(0, 91, dtype=np.float64)
    sw = Sweep(inc_dir=azimuth_sweep(az, 0.0), freq_hz=np.array([10e9]), screen=256,
               max_bounces=2, eps=0.5 * float(sc.radius), view_res=256, az_deg=az, el_deg=0.0)
    return sc, sw


def workload_composite(n_points: int = 2_000_000, n_az: int = 360, screen: int = 1024,
                       n_freq: int = 64, max_bounces: int = 4, seed: int = 2) -> tuple[Scene, Sweep]:
    """Twelve-primitive composite, 1024^2 screen and views, 64 freqs 2-12 GHz, 360 azimuths at
    30 deg elevation, <=4 bounces."""
    sc = composite(seed=seed, n_points=n_points)
    az = np.arange(n_az, dtype=np.float64) * (360.0 / n_az)
    eps = max(0.5 * float(sc.radius), 6.0 * sc.noise_sigma)
    sw = Sweep(inc_dir=azimuth_sweep(az, 30.0), freq_hz=np.linspace(2e9, 12e9, n_freq),
               screen=screen, max_bounces=max_bounces, eps=eps, view_res=screen,
               az_deg=az, el_deg=30.0)
    return sc, sw


def workload_sphere(n_points: int = 4_000_000, n_az: int = 360, screen: int = 1024,
                    n_freq: int = 64) -> tuple[Scene, Sweep]:
    """Sphere r=4 m, 64 freqs 2-24 GHz (ka up to ~2000), 360 azimuths at 0 deg elevation."""
    sc = sphere(seed=3, n_points=n_points)
    az = np.arange(n_az, dtype=np.float64) * (360.0 / n_az)
    eps = max(0.5 * float(sc.radius), 6.0 * sc.noise_sigma)
    sw = Sweep(inc_dir=azimuth_sweep(az, 0.0), freq_hz=np.linspace(2e9, 24e9, n_freq),
               screen=screen, max_bounces=4, eps=eps, view_res=screen, az_deg=az, el_deg=0.0)
    return sc, sw


# ------------------------------------------------------------------------------ serving mix --

SERVING_SCREENS = (256, 512, 1024, 2048)


def serving_pool_sizes(n_scenes: int = 64, seed: int = 5) -> list[int]:
    """Point counts of the serving workload's scene pool, log-uniform in [5e4, 4e6]."""
    rng = _rng(seed)
    return [int(np.exp(rng.uniform(np.log(5e4), np.log(4e6)))) for _ in range(n_scenes)]


def serving_scene(i: int, n_points: int) -> Scene:
    """Scene i of the serving pool: the composite generator at n_points."""
    return composite(seed=1000 + i, n_points=n_points)


def serving_request(rng: np.random.Generator, pool: list, screens=SERVING_SCREENS,
                    max_angles: int = 720, max_freqs: int = 128) -> dict:
    """One request of the serving mix: a scene index into `pool` (a list of Scene), a screen
    uniform over `screens`, an angle count log-uniform in [1, 720] (monostatic azimuths at 30
    deg elevation, evenly spaced from a random start), a frequency count log-uniform in [1, 128]
    (2-12 GHz) and 1-5 bounces.  max_angles / max_freqs cap the counts after they are drawn, so
    the same rng yields the same scenes, screens and bounce limits with or without a cap."""
    i = int(rng.integers(len(pool)))
    sc = pool[i]
    screen = int(rng.choice(screens))
    n_ang = int(np.exp(rng.uniform(0.0, np.log(720.0))))
    n_f = int(np.exp(rng.uniform(0.0, np.log(128.0))))
    az = (rng.uniform(0, 360) + np.arange(min(n_ang, max_angles)) * (360.0 / n_ang)) % 360.0
    return dict(scene=i, inc_dir=azimuth_sweep(az, 30.0),
                freq_hz=np.linspace(2e9, 12e9, min(n_f, max_freqs)), screen=screen,
                max_bounces=int(rng.integers(1, 6)),
                eps=max(0.5 * float(sc.radius), 6.0 * sc.noise_sigma))
