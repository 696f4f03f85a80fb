"""PCA normals of point clouds -- TEST INFRASTRUCTURE ONLY.

The normals a point cloud is given when it carries none, as in the paper's point-cloud baseline
(Sec. IV, normals by principal component analysis): for every point, the k nearest points of
the cloud (the point itself included) are taken, their covariance formed about their mean, and
the eigenvector of its smallest eigenvalue is the normal, turned so that its largest component
is positive (unoriented; splats are two-sided).  FP64.  Library steps: scipy's KD-tree for the
exact k nearest neighbours and numpy.linalg.eigh for the symmetric eigenproblem (both pinned
in tests/test_oracle_normals.py against brute force and closed forms).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def knn(xyz, k):
    """Indices [n, k] of each point's k nearest points (itself first), nearest first."""
    xyz = np.asarray(xyz, np.float64)
    _, idx = cKDTree(xyz).query(xyz, k)
    return np.asarray(idx).reshape(len(xyz), k)


def canonical(v):
    """Turn each row so that its largest-magnitude component is positive."""
    am = np.argmax(np.abs(v), axis=1)
    s = np.where(v[np.arange(len(v)), am] < 0, -1.0, 1.0)
    return v * s[:, None]


def smallest_eigvec(C):
    """Unit eigenvectors [n, 3] of the smallest eigenvalues of symmetric matrices [n, 3, 3]."""
    _, vec = np.linalg.eigh(C)
    return vec[:, :, 0]


def pca_normals(xyz, k=16):
    xyz = np.asarray(xyz, np.float64)
    nb = xyz[knn(xyz, k)]
    u = nb - nb.mean(axis=1, keepdims=True)
    C = np.einsum("nki,nkj->nij", u, u)
    return canonical(smallest_eigvec(C))
