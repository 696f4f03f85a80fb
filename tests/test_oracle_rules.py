"""Hand-built pins of the oracle's secondary-hit extent, visibility Psi and EVERY mode.

Each scene is a handful of disks placed so that the expected value is worked out by hand from
the definitions (Sec. II-C Eq. (14) and its visibility Psi; Sec. III-B, Algorithm 3):

- extent of the views' retention rule: a disk stored at one view pixel is admissible where a
  secondary ray meets it one pixel away (so a same-pixel rule fails) and not two pixels away
  (so a 5 x 5 rule fails); the restricted first hit follows, worked by hand;
- Psi = 0 decides a result: a dihedral whose double-bounce returns are all hidden from the
  receiver by an absorbing disk radiates nothing, exactly, in the exact and in the restricted
  mode; beside an open dihedral it leaves the open dihedral's field unchanged; moved aside, the
  same disk lets a large return through (what a Psi that is always 1 would give);
- EVERY mode: where every ray bounces exactly twice, radiating every facet equals the sum of the
  first-facet field (one bounce) and the last-facet field (two bounces).
"""
import numpy as np

import oracle

C0 = 299_792_458.0


def _scene(disks):
    xyz = np.array([d[0] for d in disks], float)
    nrm = np.array([d[1] for d in disks], float)
    rad = np.array([d[2] for d in disks], float)
    mat = np.array([d[3] if len(d) > 3 else 0 for d in disks], np.uint8)
    return xyz, nrm, rad, mat


# ---------------------------------------------------------------------------------------------
# extent of the retention rule
# ---------------------------------------------------------------------------------------------

R_EXTENT = np.sqrt(1.25) + 0.001


def _extent_scene():
    """Frame fixed by six tiny absorbing anchors (bounding box [-1, 1]^3, centre 0; the two at
    (0.3, 0.4, +-1) are farthest, so R = sqrt(1.25) + 0.001, and they stay off the view axis).
    With one view along -z at 1001 x 1001 pixels the pitch is h = 2R / 1001, u = +x, v = -y,
    and pixel (i, j) is centred at x = (i - 500) h, y = -(j - 500) h.  Disk D (centre 0, normal
    +z, radius 1.8 h) covers the nine pixel centres of the 3 x 3 block around (500, 500); eight
    small covers (radius 0.4 h, 0.5 mm above D) sit on the eight outer centres, so the view
    stores D at pixel (500, 500) only and a cover at each neighbour."""
    h = 2 * R_EXTENT / 1001
    disks = [((-1.0, 0.0, 0.0), (1.0, 0.0, 0.0), 0.001, 1), ((1.0, 0.0, 0.0), (1.0, 0.0, 0.0),
                                                              0.001, 1),
             ((0.0, -1.0, 0.0), (0.0, 1.0, 0.0), 0.001, 1), ((0.0, 1.0, 0.0), (0.0, 1.0, 0.0),
                                                              0.001, 1),
             ((0.3, 0.4, -1.0), (0.0, 0.0, 1.0), 0.001, 1), ((0.3, 0.4, 1.0), (0.0, 0.0, 1.0),
                                                              0.001, 1)]
    disks.append(((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 1.8 * h))
    D = len(disks) - 1
    covers = {}
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            covers[(di, dj)] = len(disks)
            disks.append(((di * h, -dj * h, 0.0005), (0.0, 0.0, 1.0), 0.4 * h))
    return disks, D, covers, h


def test_retention_extent_is_one_pixel():
    disks, D, covers, h = _extent_scene()
    o = oracle.OracleScene(*_scene(disks))
    c, R = o.frame()
    assert np.allclose(c, 0.0) and abs(R - R_EXTENT) < 1e-15
    o.set_views(1001, np.array([[0.0, 0.0, -1.0]]))
    _, idx, _, _ = o.render_disk([0.0, 0.0, -1.0], 1001, 1001)
    assert idx[500, 500] == D
    assert idx[500, 501] == covers[(1, 0)] and idx[499, 499] == covers[(-1, -1)]
    assert (idx == D).sum() == 1
    # D is stored at pixel (500, 500): admissible on its own pixel and one pixel away, not two
    assert o.admissible(D, [0.3 * h, 0.0, 0.0])
    assert o.admissible(D, [0.7 * h, 0.0, 0.0])       # projects to pixel 501
    assert o.admissible(D, [0.0, -0.7 * h, 0.0])      # pixel row 501
    assert not o.admissible(D, [1.6 * h, 0.0, 0.0])   # projects to pixel 502
    assert not o.admissible(D, [1.55 * h, 0.8 * h, 0.0])  # on D, pixel (502, 499)
    up = np.array([0.0, 0.0, 1.0])
    # a secondary ray from below at x = 0.7 h meets D first (t = 0.1): D one pixel from where it
    # is stored counts; a same-pixel rule would skip D and return the cover above it (t = 0.1005)
    i, t = o.first_hit_views([0.7 * h, 0.0, -0.1], up, 0.01)
    assert i == D and abs(t - 0.1) < 1e-12
    # at x = 1.6 h the ray meets D two pixels from where it is stored and no cover (the nearest
    # is 0.6 h away, radius 0.4 h): nothing admissible (a 5 x 5 rule would return D at t = 0.1)
    i, t = o.first_hit_views([1.6 * h, 0.0, -0.1], up, 0.01)
    assert i == -1 and t == np.inf
    # the exact tracer hits D in both places
    assert o.first_hit([1.6 * h, 0.0, -0.1], up, 0.01)[0] == D
    # at x = 0.95 h the ray meets D (admissible, one pixel) before the cover of pixel 501
    i, t = o.first_hit_views([0.95 * h, 0.0, -0.1], up, 0.01)
    assert i == D


# ---------------------------------------------------------------------------------------------
# visibility Psi
# ---------------------------------------------------------------------------------------------

def _dihedral_pair(y0, rho=0.1037, a=0.1531, rho_b=1.05):
    """Two big disks forming a 90-degree dihedral open toward +z with its crease on the line
    x = z = 0 at y = y0: A on the plane z = -x (normal (1, 0, 1)/sqrt 2), B on z = x (normal
    (-1, 0, 1)/sqrt 2).  A ray coming down (-z) onto A at x1 < 0 turns to +x, meets B at
    x2 = -x1 (the mirror image, inside B since B is slightly larger) and leaves toward +z."""
    s = 1 / np.sqrt(2)
    A = ((-a, y0, a), (s, 0.0, s), rho)
    B = ((a, y0, a), (-s, 0.0, s), rho * rho_b)
    return [A, B]


def _anchors():
    return [((-1.0, -1.0, -1.0), (0.0, 0.0, 1.0), 0.001, 1), ((1.0, 1.0, 1.0), (0.0, 0.0, 1.0),
                                                               0.001, 1)]


def _occluder(y0, a=0.1531, x_shift=0.0):
    # absorbing disk 0.4 m up, centred over B (radius 0.12 covers B's shadow on the ground,
    # semi-axes 0.077 x 0.109, and stays clear of A's, which lies at x < -0.079)
    return ((a + x_shift, y0, 0.4), (0.0, 0.0, 1.0), 0.12, 1)


def _solve(o, restricted=False):
    inc = np.array([[0.0, 0.0, -1.0]])
    E, st = o.solve(inc, [3e9, 5e9], 200, 200, 2, 1e-4, restricted=restricted)
    return E


def test_psi_zero_hides_double_bounce():
    hidden = _anchors() + _dihedral_pair(0.0) + [_occluder(0.0)]
    o = oracle.OracleScene(*_scene(hidden))
    o.set_views(128)
    for restricted in (False, True):
        E = _solve(o, restricted)
        # every facet that would radiate is the second bounce on B, whose return toward +z
        # crosses the absorber: Psi = 0 for all of them, so the field is exactly zero
        assert np.all(E == 0), (restricted, np.abs(E).max())
    # the same disk moved aside (over nothing) hides nothing: the dihedral returns strongly
    aside = _anchors() + _dihedral_pair(0.0) + [_occluder(0.0, x_shift=0.5)]
    o2 = oracle.OracleScene(*_scene(aside))
    o2.set_views(128)
    for restricted in (False, True):
        E = _solve(o2, restricted)
        sigma = 4 * np.pi * np.abs(E[0, 0, :, 0, 0]) ** 2
        assert np.all(sigma > 1e-3), sigma


def test_psi_hidden_pair_leaves_open_pair_unchanged():
    open_only = _anchors() + _dihedral_pair(0.6)
    both = _anchors() + _dihedral_pair(0.6) + _dihedral_pair(0.0) + [_occluder(0.0)]
    o1 = oracle.OracleScene(*_scene(open_only))
    o2 = oracle.OracleScene(*_scene(both))
    assert np.allclose(o1.frame()[0], o2.frame()[0]) and o1.frame()[1] == o2.frame()[1]
    o1.set_views(128)
    o2.set_views(128)
    for restricted in (False, True):
        E1, E2 = _solve(o1, restricted), _solve(o2, restricted)
        assert np.abs(E1).max() > 0
        assert np.abs(E2 - E1).max() <= 1e-12 * np.abs(E1).max(), restricted


# ---------------------------------------------------------------------------------------------
# EVERY mode
# ---------------------------------------------------------------------------------------------

def test_every_equals_first_plus_last_when_all_rays_bounce_twice():
    # equal disks, incidence along the bisector: every ray that meets one plate meets the other
    # at the mirror point, so M = 2 for every hit pixel and both facets face the open sky
    pair = _anchors() + _dihedral_pair(0.0, rho_b=1.0)
    o = oracle.OracleScene(*_scene(pair))
    inc = np.array([[0.0, 0.0, -1.0]])
    f = [2e9, 7e9, 11e9]
    nb, _, _ = o.trace_pixels(inc[0], 200, 200, np.arange(200 * 200), 2, 1e-4)
    assert nb.max() == 2 and np.all(nb[nb > 0] == 2)
    E_every, _ = o.solve(inc, f, 200, 200, 2, 1e-4, contrib="every")
    E_first, _ = o.solve(inc, f, 200, 200, 1, 1e-4)
    E_last, _ = o.solve(inc, f, 200, 200, 2, 1e-4)
    assert np.abs(E_first).max() > 1e-3 * np.abs(E_last).max()  # both terms matter
    assert np.abs(E_every - (E_first + E_last)).max() <= 1e-12 * np.abs(E_last).max()
    # with one bounce only, EVERY and LAST radiate the same single facet per ray
    E1_every, _ = o.solve(inc, f, 200, 200, 1, 1e-4, contrib="every")
    assert np.array_equal(E1_every, E_first)
