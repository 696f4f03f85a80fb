"""Pins of the oracle's Eq. (23) overlap refinement and normal blending (Sec. III-B, Fig. 4(a)).

  - the Fig. 4(a) configuration worked by hand: a ray crosses a tilted disk B near its rim just
    before a flat disk A near A's centre; within r the hit moves to A and the normal is the
    Eq. (23) blend, with weights 1 - |p - c| / R computed from the geometry; with r smaller than
    the gap, nothing moves and the normal is B's;
  - a lone disk is unchanged by the refinement;
  - on a plane of overlapping coplanar disks the chosen disk is, by brute force over all disks,
    the one whose centre is relatively closest to the ray's crossing, and the blended normal is
    the plane's;
  - the dihedral's double-bounce peak 8 pi a^2 b^2 / lambda^2 survives blending (0.5 dB);
  - grid and brute-force candidate searches give identical traces (bitwise).
"""
import math

import numpy as np
import pytest

import oracle
import scenes


def two_disks():
    nB = np.array([0.1, 0.0, 1.0]) / math.sqrt(1.01)
    xyz = np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.01]])
    nrm = np.array([[0.0, 0.0, 1.0], nB])
    return oracle.OracleScene(xyz, nrm, np.array([1.0, 1.2])), nB


def test_fig4a_hand_worked():
    o, nB = two_disks()
    o.set_blend(0.2)
    k = np.array([0.0, 0.0, -1.0])
    # B's plane: 0.1 (x - 1.5) + (z - 0.01) = 0 at x = 0.4 gives z = 0.12
    pB = np.array([0.4, 0.0, 0.12])
    rB = math.hypot(1.1, 0.11) / 1.2
    h, x, n, s = o.blend_hit(pB, k, 1)
    assert h == 0
    np.testing.assert_allclose(x, [0.4, 0.0, 0.0], atol=1e-12)
    assert s == pytest.approx(0.12, abs=1e-12)
    wA, wB = 1.0 - 0.4, 1.0 - rB
    blend = wA * np.array([0.0, 0.0, 1.0]) + wB * nB
    np.testing.assert_allclose(n, blend / np.linalg.norm(blend), atol=1e-12)


def test_fig4a_radius_smaller_than_gap():
    o, nB = two_disks()
    o.set_blend(0.1)
    h, x, n, s = o.blend_hit(np.array([0.4, 0.0, 0.12]), np.array([0.0, 0.0, -1.0]), 1)
    assert h == 1 and s == pytest.approx(0.0, abs=1e-12)
    np.testing.assert_allclose(n, nB, atol=1e-12)


def test_trace_applies_refinement():
    """The bounce recursion uses the refined hit: a pixel ray through the two disks records
    A's point and the blended normal when r covers the gap."""
    o, nB = two_disks()
    o.set_blend(0.2)
    k = np.array([0.0, 0.0, -1.0])
    W = 64
    o00, du, dv = o.screen(k, W, W)  # k = -z: du along +x, dv along -y
    ix = int(round((0.4 - o00[0]) / du[0]))
    iy = int(round((0.0 - o00[1]) / dv[1]))
    px = o00 + du * ix + dv * iy  # the pixel centre nearest (0.4, 0)
    nb, rec, hidx = o.trace_pixels(k, W, W, [iy * W + ix], 1, 0.0)
    assert nb[0] == 1 and hidx[0, 0] in (0, 1)
    h, x, n, s = o.blend_hit(np.array([px[0], px[1], 0.1 * -(px[0] - 1.5) + 0.01]), k, 1)
    assert h == 0 and hidx[0, 0] == h
    np.testing.assert_allclose(rec[0, 0, 0:3], x, atol=1e-9)
    np.testing.assert_allclose(rec[0, 0, 3:6], n, atol=1e-9)


def test_lone_disk_unchanged():
    o = oracle.OracleScene(np.array([[0.0, 0.0, 0.0]]), np.array([[0.3, 0.0, 1.0]]),
                           np.array([0.5]))
    o.set_blend(0.3)
    k = np.array([0.0, 0.0, -1.0])
    x0 = np.array([0.1, 0.2, -0.03])  # on the disk's plane: 0.3 * 0.1 + z = 0
    h, x, n, s = o.blend_hit(x0, k, 0)
    assert h == 0 and s == pytest.approx(0.0, abs=1e-12)
    np.testing.assert_allclose(x, x0, atol=1e-12)
    nn = np.array([0.3, 0.0, 1.0]) / math.hypot(0.3, 1.0)
    np.testing.assert_allclose(n, nn, atol=1e-12)


def test_coplanar_choice_is_brute_force_nearest_relative_centre():
    rng = np.random.default_rng(4)
    n = 400
    xy = rng.uniform(-1, 1, (n, 2))
    xyz = np.column_stack([xy, np.zeros(n)])
    rad = rng.uniform(0.08, 0.2, n)
    o = oracle.OracleScene(xyz, np.tile([0.0, 0.0, 1.0], (n, 1)), rad)
    o.set_blend(0.01)
    k = np.array([0.0, 0.0, -1.0])
    checked = 0
    for _ in range(200):
        p = np.array([*rng.uniform(-0.8, 0.8, 2), 0.0])
        d = np.hypot(xy[:, 0] - p[0], xy[:, 1] - p[1]) / rad
        cover = np.nonzero(d <= 1.0)[0]
        if len(cover) == 0:
            continue
        h, x, nrm, s = o.blend_hit(p, k, int(cover[0]))
        assert h == cover[np.argmin(d[cover])]
        np.testing.assert_allclose(x, p, atol=1e-12)
        np.testing.assert_allclose(nrm, [0.0, 0.0, 1.0], atol=1e-12)
        checked += 1
    assert checked > 150


def test_dihedral_peak_survives_blending():
    sc = scenes.dihedral()
    o = oracle.OracleScene(sc, grid=64)
    o.set_blend(0.5 * sc.radius)
    lam = scenes.C0 / 10e9
    kk = scenes.azimuth_sweep([45.0], 0.0)
    E, _ = o.solve(kk, [10e9], 160, 160, 2, 0.5 * sc.radius)
    nominal = 10 * math.log10(8 * math.pi * 0.3 ** 4 / lam ** 2)
    got = oracle.rcs_dbsm(E)[0, 0, 0]
    assert abs(got[0, 0] - nominal) < 0.5 and abs(got[1, 1] - nominal) < 0.5


def test_grid_and_brute_force_blend_identical():
    sc = scenes.random_disks(3, 300)
    og = oracle.OracleScene(sc, grid=9)
    ob = oracle.OracleScene(sc)
    for o in (og, ob):
        o.set_blend(0.05)
    k = scenes.azimuth_sweep([20.0], 25.0)[0]
    pix = np.arange(0, 48 * 48, 5)
    a = og.trace_pixels(k, 48, 48, pix, 3, 0.01)
    b = ob.trace_pixels(k, 48, 48, pix, 3, 0.01)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
