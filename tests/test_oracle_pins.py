"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test is chosen so that a plausible slip in the oracle (a dropped term, a wrong sign, a
transposed operand, a wrong area or sinc convention) fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import scenes

C0 = scenes.C0


def _rect_coverage(nb, W):
    m = (nb >= 1).reshape(W, W)
    rows = np.where(m.any(1))[0]
    cols = np.where(m.any(0))[0]
    ok = (m[rows.min():rows.max() + 1, cols.min():cols.max() + 1].all()
          and m.sum() == len(rows) * len(cols))
    return ok, len(rows), len(cols)


def test_reflection_decomposition_equals_vector_form():
    """Eq. (2)-(3) with Gamma_p = +1, Gamma_v = -1 (PEC, Sec. II-A) equals E_r = 2(n.E)n - E,
    and reflection (Eq. (4)) preserves |k|, |E| and E.k = 0."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        k = rng.standard_normal(3); k /= np.linalg.norm(k)
        n = rng.standard_normal(3); n /= np.linalg.norm(n)
        E = np.cross(k, rng.standard_normal(3))
        E /= np.linalg.norm(E)
        Ed, kd = oracle.reflect_decomposed(k, n, E)
        Ev, kv = oracle.reflect_vector(k, n, E)
        assert np.allclose(Ed, Ev, atol=1e-13)
        assert np.allclose(kd, kv, atol=1e-14)
        assert abs(np.linalg.norm(kv) - 1) < 1e-14
        assert abs(np.linalg.norm(Ev) - 1) < 1e-13
        assert abs(np.dot(Ev, kv)) < 1e-13


def test_pol_basis_is_right_handed():
    rng = np.random.default_rng(3)
    for _ in range(50):
        s = rng.standard_normal(3); s /= np.linalg.norm(s)
        th, ph = oracle.pol_basis(s)
        assert np.allclose(np.cross(th, ph), s, atol=1e-14)


@pytest.mark.parametrize("az", [0.0, 1.0, 2.5, 4.0, 7.0, 13.0, 25.0])
def test_plate_pattern_exact(az):
    """A flat plate tiled by whole pixel facets: the central-ray facet sum (Eq. (11)-(14)) is
    the exact PO integral over the covered rectangle, so
        sigma = 4 pi / lambda^2 (n_r n_c pitch^2)^2 sinc^2(k n_c pitch tan(theta))
    for both polarisations to rounding.  Pins the sinc argument, the footprint vectors of
    Eq. (12)-(13), the area, the prefactor k/2pi and the phase."""
    sc = scenes.plate(jitter=0.0)
    o = oracle.OracleScene(sc)
    f = 10e9
    lam = C0 / f
    k = 2 * math.pi / lam
    W = 40
    _, R = o.frame()
    pitch = 2 * R / W
    kk = scenes.azimuth_sweep([az], 0.0)
    E, _ = o.solve(kk, [f], W, W, 1, 0.5 * sc.radius)
    nb, _, _ = o.trace_pixels(kk[0], W, W, np.arange(W * W), 1, 0.5 * sc.radius)
    rect, nr, nc = _rect_coverage(nb, W)
    assert rect
    x = k * nc * pitch * math.tan(math.radians(az))
    s = 1.0 if x == 0 else math.sin(x) / x
    sig = 4 * math.pi / lam ** 2 * (nr * nc * pitch * pitch) ** 2 * s * s
    got = oracle.rcs_m2(E)[0, 0, 0]
    assert abs(got[0, 0] / sig - 1) < 1e-9
    assert abs(got[1, 1] / sig - 1) < 1e-9
    # single-bounce monostatic PO has no cross-polarisation
    assert abs(E[0, 0, 0, 0, 1]) <= 1e-12 * abs(E[0, 0, 0, 0, 0])
    assert abs(E[0, 0, 0, 1, 0]) <= 1e-12 * abs(E[0, 0, 0, 1, 1])


def test_plate_broadside_nominal():
    """Broadside sigma = 4 pi A^2 / lambda^2: exact with the covered area n_hit pitch^2, and
    within 0.5 dB of the nominal 0.3 x 0.3 m plate (20.54 dBsm at 10 GHz; the disks overhang
    the edges by about r - s/2)."""
    sc = scenes.plate()
    o = oracle.OracleScene(sc)
    f = 10e9
    lam = C0 / f
    W = 128
    _, R = o.frame()
    pitch = 2 * R / W
    kk = scenes.azimuth_sweep([0.0], 0.0)
    E, st = o.solve(kk, [f], W, W, 1, 0.5 * sc.radius)
    nb, _, _ = o.trace_pixels(kk[0], W, W, np.arange(W * W), 1, 0.5 * sc.radius)
    A = (nb == 1).sum() * pitch ** 2
    got = oracle.rcs_dbsm(E)[0, 0, 0]
    assert abs(got[0, 0] - 10 * math.log10(4 * math.pi * A ** 2 / lam ** 2)) < 1e-9
    nominal = 10 * math.log10(4 * math.pi * 0.09 ** 2 / lam ** 2)
    assert abs(nominal - 20.5405) < 1e-3
    assert abs(got[0, 0] - nominal) < 0.5


def test_dihedral_double_bounce_peak():
    """Right-angle dihedral at the bisector: the double-bounce aperture is 2 b sin(45 deg)
    per unit height, so sigma = 8 pi a^2 b^2 / lambda^2 (23.55 dBsm for 0.3 m plates at
    10 GHz); with the aperture measured as n_double * pitch^2 the facet sum matches to
    0.05 dB.  Pins the bounce recursion, the mirrored tube vectors and the image-method path
    length (every double-bounce ray arrives in phase)."""
    sc = scenes.dihedral()
    o = oracle.OracleScene(sc, grid=64)
    f = 10e9
    lam = C0 / f
    W = 160
    _, R = o.frame()
    pitch = 2 * R / W
    kk = scenes.azimuth_sweep([45.0], 0.0)
    E, _ = o.solve(kk, [f], W, W, 2, 0.5 * sc.radius)
    nb, _, _ = o.trace_pixels(kk[0], W, W, np.arange(W * W), 2, 0.5 * sc.radius)
    A = (nb == 2).sum() * pitch ** 2
    expect = 10 * math.log10(4 * math.pi * A ** 2 / lam ** 2)
    got = oracle.rcs_dbsm(E)[0, 0, 0]
    assert abs(got[0, 0] - expect) < 0.05
    assert abs(got[1, 1] - expect) < 0.05
    nominal = 10 * math.log10(8 * math.pi * 0.3 ** 4 / lam ** 2)
    assert abs(nominal - 23.5508) < 1e-3
    assert abs(got[0, 0] - nominal) < 0.5
    # with one bounce only, the bisector return collapses (no retro-reflection)
    E1, _ = o.solve(kk, [f], W, W, 1, 0.5 * sc.radius)
    assert oracle.rcs_dbsm(E1)[0, 0, 0, 0, 0] < expect - 15


def test_dihedral_every_vs_last():
    """At the bisector nearly every ray bounces twice; EVERY adds the first-bounce facets,
    which are far off-specular there, so it changes sigma by well under 1 dB; both modes agree
    exactly when max_bounces = 1."""
    sc = scenes.dihedral()
    o = oracle.OracleScene(sc, grid=64)
    kk = scenes.azimuth_sweep([45.0], 0.0)
    El, _ = o.solve(kk, [10e9], 96, 96, 2, 0.5 * sc.radius, contrib="last")
    Ee, _ = o.solve(kk, [10e9], 96, 96, 2, 0.5 * sc.radius, contrib="every")
    d = oracle.rcs_dbsm(Ee)[0, 0, 0, 0, 0] - oracle.rcs_dbsm(El)[0, 0, 0, 0, 0]
    assert 0 < abs(d) < 1.0
    kk = scenes.azimuth_sweep([10.0], 0.0)
    El, _ = o.solve(kk, [10e9], 64, 64, 1, 0.5 * sc.radius, contrib="last")
    Ee, _ = o.solve(kk, [10e9], 64, 64, 1, 0.5 * sc.radius, contrib="every")
    assert np.array_equal(El, Ee)


def test_sphere_po():
    """Large PEC sphere under PO: sigma = pi a^2 [1 - sin(2ka)/(ka) + sin^2(ka)/(ka)^2].
    The point-sampled sphere carries ~0.1 dB of sampling noise per angle; the mean over angles
    and frequencies must sit within 0.1 dB and every sample within 0.3 dB; sigma does not
    depend on azimuth beyond that noise."""
    a = 0.5
    sc = scenes.sphere(seed=5, n_points=400_000, a=a, noise_sigma=0.0)
    o = oracle.OracleScene(sc, grid=160)
    errs = []
    for f in (10e9, 20e9):
        ka = 2 * math.pi * f / C0 * a
        assert ka > 100
        exact = 10 * math.log10(math.pi * a * a * (1 - math.sin(2 * ka) / ka
                                                  + math.sin(ka) ** 2 / ka ** 2))
        E, _ = o.solve(scenes.azimuth_sweep([0.0, 33.0, 71.0, 200.0], 10.0), [f], 400, 400, 1,
                       0.5 * sc.radius)
        r = oracle.rcs_dbsm(E)[:, 0, 0]
        errs.append(r[:, 0, 0] - exact)
        errs.append(r[:, 1, 1] - exact)
    errs = np.concatenate(errs)
    assert abs(errs.mean()) < 0.1
    assert np.abs(errs).max() < 0.3


def test_reciprocity_rolled_dihedral():
    """Monostatic reciprocity S_theta_phi = S_phi_theta on a dihedral rolled 22.5 deg about
    the line of sight (strong cross-polarised double-bounce return).  PO-SBR is reciprocal to
    the ray sampling; the measured imbalance is required below 1e-3 of the co-pol peak."""
    sc = scenes.dihedral()
    kk = scenes.azimuth_sweep([45.0], 0.0)[0]
    axis = -kk
    ang = math.radians(22.5)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    Rm = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    o = oracle.OracleScene(sc.xyz @ Rm.T, sc.nrm @ Rm.T, sc.radius, sc.material, grid=64)
    E, _ = o.solve(kk[None], [10e9], 128, 128, 2, 0.5 * sc.radius)
    S = E[0, 0, 0]
    peak = np.abs(S).max()
    assert abs(S[0, 1]) > 0.3 * peak
    assert abs(S[0, 1] - S[1, 0]) < 1e-3 * peak


def test_frequency_independence():
    """The GO trace does not depend on frequency: an F-frequency solve equals F one-frequency
    solves bit for bit."""
    sc = scenes.dihedral()
    o = oracle.OracleScene(sc, grid=64)
    kk = scenes.azimuth_sweep([30.0], 0.0)
    fr = [8e9, 10e9, 12.5e9]
    E, _ = o.solve(kk, fr, 64, 64, 2, 0.5 * sc.radius)
    for i, f in enumerate(fr):
        Ei, _ = o.solve(kk, [f], 64, 64, 2, 0.5 * sc.radius)
        assert np.array_equal(E[:, :, i], Ei[:, :, 0])


# ------------------------------- tiny clouds, hand-derived --------------------------------

def _one(xyz, nrm, r, mat=None):
    xyz = np.atleast_2d(np.asarray(xyz, float))
    nrm = np.atleast_2d(np.asarray(nrm, float))
    return oracle.OracleScene(xyz, nrm, np.broadcast_to(np.asarray(r, float), (len(xyz),)).copy(),
                              mat)


def test_single_disk_hits():
    o = _one([0, 0, 0], [0, 0, 1], 1.0)
    down = [0, 0, -1]
    assert o.first_hit([0.5, 0, 5], down) == (0, 5.0)
    assert o.first_hit([1.0, 0, 5], down)[0] == 0          # boundary is inclusive
    assert o.first_hit([1.0 + 1e-9, 0, 5], down)[0] == -1
    assert o.first_hit([0, 0, -5], [0, 0, 1]) == (0, 5.0)  # two-sided
    assert o.first_hit([0.2, 0, 5], down, tmin=5.0)[0] == -1  # t must exceed tmin
    g = np.array([1.0, 0.0, 5e-7]); g /= np.linalg.norm(g)
    assert o.first_hit([-2, 0, 0], g)[0] == -1              # grazing |n.k| < 1e-6
    g = np.array([1.0, 0.0, 2e-6]); g /= np.linalg.norm(g)
    assert o.first_hit([-0.5, 0, -1e-6], g)[0] == 0


def test_overlap_nearest_then_smallest_index():
    o = _one([[0, 0, 0], [0, 0, 1], [0, 0, 1]], [[0, 0, 1]] * 3, 1.0)
    i, t = o.first_hit([0, 0, 5], [0, 0, -1])
    assert (i, t) == (1, 4.0)                              # nearest wins; equal t -> index 1
    i, t = o.first_hit([0, 0, -5], [0, 0, 1])
    assert (i, t) == (0, 5.0)


def test_mirror_pair_bounces():
    """Two facing disks 1 m apart (a large one below, a small one above): a ray arriving from
    above just outside the small disk hits the large one, then bounces straight up into the
    small one if it lies within its radius, and so on; the image-method path grows by exactly
    1 m per bounce and eps prevents self-hits."""
    xyz = [[0, 0, 0], [0, 0, 1.0]]
    nrm = [[0, 0, 1], [0, 0, -1]]
    o = _one(xyz, nrm, [0.5, 0.05])
    # ray arriving from above, slightly off-axis, passes the small upper disk and hits the lower
    k = np.array([0.0, 0.0, -1.0])
    c, R = o.frame()
    W = 33
    pix = np.array([16 * W + 16 + 4])  # a pixel 4 columns right of the centre
    nb, rec, hidx = o.trace_pixels(k, W, W, pix, 4, 1e-3)
    # first hit lower disk (index 0), reflects straight up into the upper disk only if within
    # its radius; 4 pixels * pitch vs 0.05 m radius decides
    o00, du, dv = o.screen(k, W, W)
    off = 4 * np.linalg.norm(du)
    assert hidx[0, 0] == 0
    if off <= 0.05:
        assert nb[0] == 4 and list(hidx[0]) == [0, 1, 0, 1]
        d = rec[0, :, 21]
        assert np.allclose(np.diff(d), 1.0, atol=1e-12)
    else:
        assert nb[0] == 1


def test_absorber_stops_ray():
    o = _one([[0, 0, 0], [0, 0, 1.0]], [[0, 0, 1], [0, 0, 1]], [1.0, 1.0],
             np.array([0, 1], np.uint8))
    W = 9
    nb, rec, hidx = o.trace_pixels([0, 0, -1.0], W, W, np.array([40]), 3, 1e-3)
    assert nb[0] == 0                                       # absorber in front: no record
    c, R = o.frame()
    E, _ = o.solve(np.array([[0, 0, -1.0]]), [1e9], W, W, 3, 1e-3)
    assert np.all(E == 0)


def test_tube_depth_hand():
    """Ray tube (Algorithm 1): a point is a candidate iff its distance to the central ray is
    below delta; the depth is its along-ray distance from the tube origin."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.5]])
    o = oracle.OracleScene(xyz, np.array([[0, 0, 1.0]] * 2), np.array([0.1, 0.1]))
    W = 11
    o00, du, dv = o.screen([0, 0, -1.0], W, W)
    c, R = o.frame()
    depth, idx = o.render_tube([0, 0, -1.0], W, W, 0.3 * np.linalg.norm(du))
    centre = 5 * W + 5
    # the nearer point (index 1, z = 0.5) wins at the centre pixel
    assert idx.ravel()[centre] == 1
    o_c = o00 + 5 * du + 5 * dv
    assert abs(depth.ravel()[centre] - (o_c[2] - 0.5)) < 1e-12
    assert np.isinf(depth.ravel()[0]) and idx.ravel()[0] == -1
    # only the centre pixel is within 0.3 pitch of the two points
    assert (idx >= 0).sum() == 1


def test_grid_equals_brute_force_bitwise():
    """The culled-exact grid returns the same first hit, bit for bit, as brute force, on random
    tiny clouds (with overlaps, absorbers and per-point radii) and on the dihedral."""
    rng = np.random.default_rng(5)
    for seed in range(6):
        sc = scenes.random_disks(seed, 60, extent=1.0, absorber_frac=0.2)
        ob = oracle.OracleScene(sc)
        og = oracle.OracleScene(sc, grid=7 + seed)
        for _ in range(300):
            o = rng.uniform(-1.5, 1.5, 3)
            k = rng.standard_normal(3); k /= np.linalg.norm(k)
            tmin = float(rng.choice([0.0, 1e-3, 0.3]))
            assert ob.first_hit(o, k, tmin) == og.first_hit(o, k, tmin)
        kk = scenes.azimuth_sweep([17.0], 20.0)
        Eb, _ = ob.solve(kk, [3e9], 24, 24, 3, 1e-3)
        Eg, _ = og.solve(kk, [3e9], 24, 24, 3, 1e-3)
        assert np.array_equal(Eb, Eg)
    sc = scenes.dihedral()
    ob = oracle.OracleScene(sc)
    og = oracle.OracleScene(sc, grid=48)
    for az in (3.0, 45.0, 80.0):
        kk = scenes.azimuth_sweep([az], 0.0)
        Eb, _ = ob.solve(kk, [10e9], 48, 48, 2, 0.5 * sc.radius)
        Eg, _ = og.solve(kk, [10e9], 48, 48, 2, 0.5 * sc.radius)
        assert np.array_equal(Eb, Eg)


def test_render_matches_brute_first_hit():
    """The disk GFB is the first hit of every pixel's central ray with tmin = 0."""
    sc = scenes.random_disks(9, 40)
    o = oracle.OracleScene(sc)
    k = np.array([0.3, -0.2, -0.9]); k /= np.linalg.norm(k)
    W = 32
    depth, idx, nrm, mask = o.render_disk(k, W, W)
    o00, du, dv = o.screen(k, W, W)
    for q in range(0, W * W, 7):
        i, j = q % W, q // W
        h, t = o.first_hit(o00 + (i * du + j * dv), k, 0.0)
        assert idx.ravel()[q] == h
        if h >= 0:
            assert depth.ravel()[q] == t
            n = nrm.reshape(-1, 3)[q]
            assert np.dot(n, k) < 0
        else:
            assert mask.ravel()[q] == 0


def test_invalid_scene_rejected():
    with pytest.raises(ValueError):
        _one([np.nan, 0, 0], [0, 0, 1], 1.0)
    with pytest.raises(ValueError):
        _one([0, 0, 0], [0, 0, 0], 1.0)
    with pytest.raises(ValueError):
        _one([0, 0, 0], [0, 0, 1], 1.0, np.array([7], np.uint8))


def test_trihedral_triple_bounce_peak():
    """Square trihedral of edge a viewed along its symmetry axis: the rays entering the
    hexagonal region of projected area sqrt(3) a^2 bounce three times and leave antiparallel,
    all with the same image-method path, so sigma = 4 pi (sqrt(3) a^2)^2 / lambda^2 =
    12 pi a^4 / lambda^2 (25.31 dBsm for a = 0.3 m at 10 GHz).  With the aperture measured as
    n_triple * pitch^2 the facet sum matches to 0.1 dB (single and double bounces leave in other
    directions); the measured aperture is the hexagon to within the splats' overhang."""
    sc = scenes.trihedral()
    o = oracle.OracleScene(sc, grid=64)
    f = 10e9
    lam = C0 / f
    W = 192
    _, R = o.frame()
    pitch = 2 * R / W
    k = -np.ones(3) / math.sqrt(3.0)        # arriving from (1, 1, 1)
    eps = 0.5 * sc.radius
    E, _ = o.solve(k[None], [f], W, W, 3, eps)
    nb, _, _ = o.trace_pixels(k, W, W, np.arange(W * W), 3, eps)
    A = (nb == 3).sum() * pitch ** 2
    expect = 10 * math.log10(4 * math.pi * A ** 2 / lam ** 2)
    got = oracle.rcs_dbsm(E)[0, 0, 0]
    assert abs(got[0, 0] - expect) < 0.1
    assert abs(got[1, 1] - expect) < 0.1
    nominal = 10 * math.log10(12 * math.pi * 0.3 ** 4 / lam ** 2)
    assert abs(nominal - 25.3117) < 1e-3
    assert abs(A / (math.sqrt(3.0) * 0.3 ** 2) - 1.0) < 0.05
    assert abs(got[0, 0] - nominal) < 0.5
    # with two bounces at most there is no retro-reflection along the axis
    E2, _ = o.solve(k[None], [f], W, W, 2, eps)
    assert oracle.rcs_dbsm(E2)[0, 0, 0, 0, 0] < expect - 10


def test_tube_topk_brute_force_tiny_clouds():
    """Algorithm 1 with a K-point heap, checked against an independent all-points loop: keep the
    K candidates (axis distance < delta, in front of the screen) nearest the central ray, pick
    the one nearest the tube origin, depth = |p - o|.  K = 1 is the point nearest the axis; a
    K above the candidate count is the nearest candidate to the origin; the depth always lies
    between the along-ray distance and sqrt(t^2 + delta^2)."""
    rng = np.random.default_rng(5)
    for seed in range(3):
        sc = scenes.random_disks(seed=200 + seed, n=60, r_lo=0.02, r_hi=0.05)
        o = oracle.OracleScene(sc)
        W = H = 12
        for K in (1, 2, 3, 100):
            k = rng.normal(size=3)
            k /= np.linalg.norm(k)
            delta = 0.15
            dep, idx = o.render_tube_topk(k, W, H, delta, K)
            o00, du, dv = o.screen(k, W, H)
            for j in range(H):
                for i in range(W):
                    org = o00 + i * du + j * dv
                    w = o.xyz - org
                    tc = w @ k
                    a2 = np.sum(np.cross(w, k) ** 2, axis=1)
                    cand = np.where((tc > 0) & (a2 < delta ** 2))[0]
                    if cand.size == 0:
                        assert idx[j, i] == -1 and np.isinf(dep[j, i])
                        continue
                    kept = sorted(cand, key=lambda m: (a2[m], m))[:K]
                    dist = np.linalg.norm(w[kept], axis=1)
                    best = min(zip(dist, kept))
                    assert idx[j, i] == best[1]
                    assert abs(dep[j, i] - best[0]) < 1e-12
                    m = best[1]
                    assert tc[m] - 1e-12 <= dep[j, i] <= math.sqrt(tc[m] ** 2 + delta ** 2) + 1e-12
