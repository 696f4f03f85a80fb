"""Pins of the oracle's GFB edge filtering and fusion (Sec. III-B, Algorithm 3, Eq. (22)).

Each pin is fixed by geometry or by a textbook definition, not by re-running the oracle's own
formulas:
  - a plane seen square-on at 4 x 4 pixels per cell fuses to splats at the exact cell centres,
    on the plane, 16 pixels each, normal +-axis, radius sqrt(2) L (views along -z and along -x,
    so both screen-basis branches are covered);
  - the same plane seen from both sides fuses to one normal, not to a cancelled one;
  - Eq. (22) closed forms on either side of its bound, and the minimum over views;
  - Canny thresholds in slope units: a slope ridge below the high threshold gives no edge (a
    weak one only when joined to a strong edge), above it the crest column; a depth step gives
    an edge beside it in every row;
  - hysteresis == brute-force propagation on random tiny maps;
  - empty pixels count as far depth, so a hit square's border is an edge all round;
  - the fp32-reach flags cover what a few ulps of input rounding actually change.
"""
import math

import numpy as np
import pytest

import scenes
from oracle import fuse


def plane_gfb(n, depth_val, nrm_view=(0.0, 0.0, 1.0)):
    d = np.full((1, n, n), depth_val, np.float32)
    nr = np.zeros((1, n, n, 3), np.float32)
    nr[...] = np.asarray(nrm_view, np.float32)
    return d, nr, np.ones((1, n, n), np.float32)


@pytest.mark.parametrize("k,axis", [((0.0, 0.0, -1.0), 2), ((-1.0, 0.0, 0.0), 0)])
def test_square_on_plane_fuses_to_cell_centres(k, axis):
    R, G = 1.0, 16
    n = 4 * G
    z0 = 0.3  # plane coordinate along the view axis; screen sits at +R on that axis
    d, nr, hit = plane_gfb(n, (R - z0) / (2 * R))
    r = fuse.fuse(np.array([k]), d, nr, hit, np.zeros(3), R, grid=G, dilate=0)
    assert not r["edge"].any()
    L = 2 * R / G
    assert len(r["xyz"]) == G * G
    assert (r["count"] == 16).all()
    np.testing.assert_allclose(r["xyz"][:, axis], z0, atol=1e-12)
    others = [a for a in range(3) if a != axis]
    for a in others:
        frac = (r["xyz"][:, a] + R) / L - 0.5  # cell centres are at (i + 1/2) L - R
        np.testing.assert_allclose(frac, np.round(frac), atol=1e-9)
    expect_n = np.zeros(3)
    expect_n[axis] = 1.0
    np.testing.assert_allclose(r["nrm"], np.broadcast_to(expect_n, r["nrm"].shape), atol=1e-12)
    np.testing.assert_allclose(r["radius"], math.sqrt(2.0) * L, rtol=1e-12)


def test_plane_from_both_sides_keeps_its_normal():
    R, G, n = 1.0, 16, 64
    z0 = 0.0
    d1, nr1, h1 = plane_gfb(n, (R - z0) / (2 * R))  # from +z looking down: normal +z
    d2, nr2, h2 = plane_gfb(n, (R + z0) / (2 * R))  # from -z looking up: normal -z
    d = np.concatenate([d1, d2]); nr = np.concatenate([nr1, nr2]); h = np.concatenate([h1, h2])
    r = fuse.fuse(np.array([[0, 0, -1.0], [0, 0, 1.0]]), d, nr, h, np.zeros(3), R, grid=G,
                  dilate=0)
    assert (r["count"] == 32).all()
    np.testing.assert_allclose(np.abs(r["nrm"][:, 2]), 1.0, atol=1e-12)


def test_eq22_closed_forms_and_bound():
    L = 0.01
    assert fuse.eq22_radius(1.0, L) == pytest.approx(math.sqrt(2) * L, rel=1e-15)
    c = 0.5
    assert fuse.eq22_radius(c, L) == pytest.approx(math.sqrt(2) * L / math.sqrt(c), rel=1e-15)
    # bound: sqrt(1/|cos|) >= 2.5  <=>  |cos| <= 0.16
    assert fuse.eq22_radius(0.17, L) == pytest.approx(math.sqrt(2 / 0.17) * L, rel=1e-15)
    assert fuse.eq22_radius(0.15, L) == pytest.approx(3.535 * L, rel=1e-15)
    assert fuse.eq22_radius(0.0, L) == pytest.approx(3.535 * L, rel=1e-15)
    assert fuse.eq22_radius(-0.5, L) == fuse.eq22_radius(0.5, L)


def test_eq22_radius_takes_the_squarest_view():
    R, G, n = 1.0, 8, 32
    a1, a2 = math.radians(60.0), math.radians(30.0)
    d1, nr1, h1 = plane_gfb(n, 0.35, (math.sin(a1), 0.0, math.cos(a1)))
    d2, nr2, h2 = plane_gfb(n, 0.35, (math.sin(a2), 0.0, math.cos(a2)))
    d = np.concatenate([d1, d2]); nr = np.concatenate([nr1, nr2]); h = np.concatenate([h1, h2])
    r = fuse.fuse(np.array([[0, 0, -1.0], [0, 0, -1.0]]), d, nr, h, np.zeros(3), R, grid=G,
                  dilate=0)
    # fused normal bisects the two, at 45 deg from the (shared) projection direction (fp32 inputs)
    L = 2 * R / G
    np.testing.assert_allclose(r["radius"], math.sqrt(2) * L / math.sqrt(math.cos(math.radians(45))),
                               rtol=1e-6)
    r1 = fuse.fuse(np.array([[0, 0, -1.0]]), d1, nr1, h1, np.zeros(3), R, grid=G, dilate=0)
    np.testing.assert_allclose(r1["radius"], math.sqrt(2) * L / math.sqrt(0.5), rtol=1e-6)


def ridge(n, slope, xc=32.3, wd=6.0, R=1.0):
    """Full-frame depth whose slope (depth change per pixel pitch) along x peaks at `slope` on
    the line x = xc (tanh profile of width wd pixels) and falls off to zero on both sides."""
    pitch = 2 * R / n
    x = np.arange(n, dtype=np.float64)
    t = 0.5 * (2 * R) + slope * pitch * wd * np.tanh((x - xc) / wd)
    d = np.broadcast_to(t / (2 * R), (n, n))[None].astype(np.float32)
    return d, np.ones_like(d)


@pytest.mark.parametrize("slope,edge", [(1.9, False), (3.0, False), (4.5, True)])
def test_canny_thresholds_are_slopes(slope, edge):
    """Thresholds 2 and 4: a slope ridge of 1.9 is below both, 3.0 is weak only (no strong pixel
    to join), 4.5 (about 4.3 after smoothing) is strong and thinned to its crest column."""
    n = 64
    d, h = ridge(n, slope)
    e = fuse.canny(d, h, 1.0, 2.0, 4.0)[0]
    if edge:
        assert np.nonzero(e.any(axis=0))[0].tolist() == [32]
        assert e[:, 32].all()
    else:
        assert not e.any()


def test_canny_weak_line_joins_a_strong_edge():
    """A weak ridge line (slope 3) becomes an edge where it continues a strong one (slope 4.5
    over the lower rows) and stays out when alone."""
    n = 64
    d, h = ridge(n, 3.0)
    ds, _ = ridge(n, 4.5)
    d = d.copy()
    d[0, 48:, :] = ds[0, 48:, :]
    e = fuse.canny(d, h, 1.0, 2.0, 4.0)[0]
    assert e[:, 32].all()
    d2, _ = ridge(n, 3.0)
    assert not fuse.canny(d2, h, 1.0, 2.0, 4.0)[0].any()


def test_canny_step_edge_columns():
    n = 64
    d = np.full((1, n, n), 0.4, np.float32)
    d[0, :, n // 2:] = 0.6
    e = fuse.canny(d, np.ones_like(d), 1.0, 2.0, 4.0)
    cols = np.nonzero(e[0].any(axis=0))[0]
    # the two columns beside the step tie in exact arithmetic; rounding may keep one of them
    assert set(cols.tolist()) <= {n // 2 - 1, n // 2} and len(cols) >= 1
    assert (e[0, :, n // 2 - 1] | e[0, :, n // 2]).all()


def test_silhouette_is_an_edge_all_round():
    n = 64
    d = np.full((1, n, n), 0.4, np.float32)
    h = np.zeros((1, n, n), np.float32)
    h[0, 16:48, 16:48] = 1.0
    e = fuse.canny(d, h, 1.0, 2.0, 4.0)[0]
    assert not e[20:44, 20:44].any()
    ring = np.zeros((n, n), bool)
    ring[15:49, 15:49] = True
    ring[17:47, 17:47] = False
    # every pixel of the square's outline has an edge within one pixel
    from scipy import ndimage
    near = ndimage.binary_dilation(e, structure=np.ones((3, 3), bool))
    assert near[ring].all()


def brute_hysteresis(strong, weak):
    out = strong.copy()
    h, w = out.shape
    changed = True
    while changed:
        changed = False
        for y in range(h):
            for x in range(w):
                if weak[y, x] and not out[y, x]:
                    ys, xs = slice(max(y - 1, 0), y + 2), slice(max(x - 1, 0), x + 2)
                    if out[ys, xs].any():
                        out[y, x] = True
                        changed = True
    return out


def test_hysteresis_matches_brute_force():
    rng = np.random.default_rng(5)
    for _ in range(20):
        u = rng.random((12, 14))
        strong, weak = u > 0.93, (u > 0.55) & (u <= 0.93)
        np.testing.assert_array_equal(fuse.hysteresis(strong, weak),
                                      brute_hysteresis(strong, weak))


def test_ambiguity_flags_cover_ulp_perturbations():
    """The fp32 reach the oracle flags is wide enough: perturbing every depth and normal by up to
    4 fp32 ulps (the size of the GPU kernels' own rounding) changes edge decisions only inside
    candidate components that hold a flagged pixel, and moves only flagged pixels across cell
    faces, into cells the oracle lists as reachable."""
    from scipy import ndimage
    g = scenes.synthetic_gfbs(13, 4, 512, n_regions=6)
    centre, R = np.zeros(3), 10.0
    r0 = fuse.fuse(g["view_dirs"], g["depth"], g["nrm"], g["hit"], centre, R, grid=256)
    rng = np.random.default_rng(5)
    d32 = g["depth"].astype(np.float32)
    dp = d32 + rng.integers(-4, 5, d32.shape) * np.spacing(d32)
    n32 = g["nrm"].astype(np.float32)
    npert = n32 + rng.integers(-4, 5, n32.shape) * np.spacing(n32)
    r1 = fuse.fuse(g["view_dirs"], dp, npert, g["hit"], centre, R, grid=256)
    diff = r0["edge"] ^ r1["edge"]
    allowed = np.zeros_like(diff)
    for v in range(diff.shape[0]):
        lab, _ = ndimage.label(r0["edge_cand"][v] | r1["edge"][v], structure=np.ones((3, 3), bool))
        ids = np.unique(lab[r0["edge_amb"][v]])
        allowed[v] = np.isin(lab, ids[ids > 0])
    assert not (diff & ~allowed).any()
    hit = g["hit"] >= 0.5
    moved = (r0["pix_cell"] != r1["pix_cell"]) & hit
    assert moved.sum() > 0  # the perturbation does move some points across cell faces
    assert not (moved & ~r0["pix_amb"]).any()
    assert np.isin(r1["pix_cell"][moved], r0["amb_cells"]).all()
