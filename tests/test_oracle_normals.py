"""Pins of the oracle's PCA normals (oracle/normals.py).

  - points on a tilted plane get exactly the plane's normal, turned to the canonical side;
  - points uniform on a sphere get nearly radial normals (the neighbourhood is a small cap);
  - on a dihedral, points away from the crease get their plate's normal exactly;
  - the k nearest neighbours equal a brute-force sort of all distances on a small cloud;
  - the eigenvector step recovers the known smallest axis of constructed covariances.
"""
import numpy as np

import scenes
from oracle import normals as N


def test_plane_exact():
    rng = np.random.default_rng(1)
    nrm = np.array([0.3, -0.5, 0.81])
    nrm /= np.linalg.norm(nrm)
    a = np.cross(nrm, [1.0, 0, 0]); a /= np.linalg.norm(a)
    b = np.cross(nrm, a)
    uv = rng.uniform(-1, 1, (3000, 2))
    xyz = uv[:, :1] * a + uv[:, 1:] * b + 0.2
    got = N.pca_normals(xyz, 12)
    expect = N.canonical(nrm[None])[0]
    assert np.abs(got - expect).max() < 1e-9


def test_sphere_radial():
    rng = np.random.default_rng(2)
    v = rng.normal(size=(20000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    got = N.pca_normals(2.0 * v, 16)
    ang = np.degrees(np.arccos(np.clip(np.abs((got * v).sum(1)), 0, 1)))
    assert ang.max() < 3.0 and ang.mean() < 0.5


def test_dihedral_plates_away_from_crease():
    sc = scenes.dihedral()
    got = N.pca_normals(sc.xyz, 16)
    # one of x, y is 0 on each plate, so x + y is the distance from the crease
    far = (sc.xyz[:, 0] + sc.xyz[:, 1] > 0.02) & (np.abs(sc.xyz[:, 2]) < 0.14)
    dots = np.abs((got * sc.nrm).sum(1))[far]
    assert (dots > 1 - 1e-9).mean() > 0.999


def test_knn_brute_force():
    rng = np.random.default_rng(3)
    xyz = rng.uniform(-1, 1, (300, 3))
    k = 9
    d = ((xyz[:, None, :] - xyz[None, :, :]) ** 2).sum(-1)
    brute = np.argsort(d, axis=1, kind="stable")[:, :k]
    got = N.knn(xyz, k)
    for i in range(len(xyz)):
        assert set(got[i]) == set(brute[i])
        assert got[i][0] == i


def test_eigvec_of_constructed_covariance():
    rng = np.random.default_rng(4)
    q = np.stack([np.linalg.qr(rng.normal(size=(3, 3)))[0] for _ in range(50)])
    lam = np.sort(rng.uniform(0.1, 3.0, (50, 3)), axis=1)
    lam[:, 0] *= 0.05
    C = np.einsum("nij,nj,nkj->nik", q, lam, q)
    got = N.smallest_eigvec(C)
    assert np.abs(np.abs((got * q[:, :, 0]).sum(1)) - 1).max() < 1e-12
