"""Pins of the oracle's view-restricted tracing (the method's rule that secondary hits and
later-bounce visibility come from the geometry the aggregation views retain, Sec. III-B).

- projection: every view pixel's stored disk is admissible at the point where that pixel's
  own central ray meets it, and a disk no view stores is admissible nowhere;
- brute force on tiny clouds: the restricted first hit equals the nearest admissible
  intersection found by an independent all-disks loop written here;
- special case: the restricted first hit coincides with the exact first hit whenever the exact
  hit is admissible, and is never nearer;
- physics: on the dihedral (both plates fully seen by the axis views) the restricted solve keeps
  the double-bounce RCS of the exact solve.
"""
import numpy as np

import oracle
import scenes


def _screen_rays(o, k, res):
    o00, du, dv = o.screen(k, res, res)
    return o00, du, dv


def test_view_pixels_admit_their_disk():
    sc = scenes.dihedral(n_side=40)
    o = oracle.OracleScene(sc, grid=32)
    res = 48
    o.set_views(res)
    dirs, _ = o.views
    stored = set()
    checked = 0
    for k in dirs:
        o00, du, dv = _screen_rays(o, k, res)
        for j in range(0, res, 3):
            for i in range(0, res, 3):
                p = o00 + i * du + j * dv
                d, t = o.first_hit(p, k, 0.0)
                if d < 0:
                    continue
                stored.add(d)
                assert o.admissible(d, p + t * k / np.linalg.norm(k))
                checked += 1
    assert checked > 100
    # a disk no view stores anywhere is never admissible
    dep = {}
    allstored = set()
    for k in dirs:
        _, idx, _, _ = o.render_disk(k, res, res)
        allstored |= set(idx[idx >= 0].ravel().tolist())
    hidden = [i for i in range(o.n) if i not in allstored][:20]
    for i in hidden:
        assert not o.admissible(i, o.xyz[i])


def _all_hits(o, p, k, tmin):
    """Every disk intersection beyond tmin (independent FP64 loop)."""
    out = []
    for i in range(o.n):
        n = o.nrm[i] / np.linalg.norm(o.nrm[i])
        den = n @ k
        if abs(den) < 1e-6:
            continue
        t = n @ (o.xyz[i] - p) / den
        if not t > tmin:
            continue
        q = p + t * k - o.xyz[i]
        if q @ q <= o.rad[i] ** 2:
            out.append((t, i))
    return sorted(out)


def test_restricted_first_hit_brute_force_tiny_clouds():
    rng = np.random.default_rng(4)
    agree = 0
    for seed in range(4):
        sc = scenes.random_disks(seed=100 + seed, n=40, r_lo=0.05, r_hi=0.15)
        for grid in (0, 8):
            o = oracle.OracleScene(sc, grid=grid or None)
            o.set_views(24)
            for _ in range(150):
                p = rng.uniform(-1.5, 1.5, 3)
                k = o.xyz[rng.integers(o.n)] - p  # aimed at a disk centre
                k /= np.linalg.norm(k)
                tmin = 0.01
                hits = _all_hits(o, p, k, tmin)
                want = next(((t, i) for t, i in hits if o.admissible(i, p + t * k)), (np.inf, -1))
                i_r, t_r = o.first_hit_views(p, k, tmin)
                assert i_r == want[1]
                if i_r >= 0:
                    assert abs(t_r - want[0]) <= 1e-12 * max(1.0, abs(want[0]))
                i_e, t_e = o.first_hit(p, k, tmin)
                if i_e >= 0:
                    assert i_r < 0 or t_r >= t_e
                    if o.admissible(i_e, p + t_e * k):
                        assert (i_r, t_r) == (i_e, t_e)
                        agree += 1
    assert agree > 200


def test_restricted_solve_keeps_dihedral_double_bounce():
    sc = scenes.dihedral()
    o = oracle.OracleScene(sc, grid=64)
    o.set_views(256)
    inc = scenes.azimuth_sweep([30.0, 45.0, 60.0], 0.0)
    eps = 0.5 * sc.radius
    E, _ = o.solve(inc, [10e9], 128, 128, 2, eps)
    Er, _ = o.solve(inc, [10e9], 128, 128, 2, eps, restricted=True)
    r, rr = oracle.rcs_dbsm(E), oracle.rcs_dbsm(Er)
    for p in range(2):
        assert np.abs(r[..., p, p] - rr[..., p, p]).max() < 0.01
