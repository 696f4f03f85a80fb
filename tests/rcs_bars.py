"""RCS comparison helpers shared by the GPU parity tests: the 30 dB window, the per-sample
conditioning of the exact oracle under fp32 rounding of its inputs, and a one-line report."""
import numpy as np

import oracle


def ensemble(sc, seeds=(1, 2)):
    """Oracle scenes on fp32-perturbed inputs: the scene-frame positions and the normals
    rounded to fp32, and seeded jitters of +-2 fp32 ulps of each coordinate."""
    c = 0.5 * (sc.xyz.min(0) + sc.xyz.max(0))
    q = sc.xyz - c
    out = [oracle.OracleScene(q.astype(np.float32).astype(np.float64) + c,
                              sc.nrm.astype(np.float32).astype(np.float64), sc.radius_array(),
                              sc.material, grid=256)]
    for seed in seeds:
        rng = np.random.default_rng(seed)
        ulp = np.spacing(np.abs(q).astype(np.float32)).astype(np.float64)
        xq = q + rng.uniform(-2, 2, q.shape) * ulp
        nq = sc.nrm + rng.uniform(-2, 2, sc.nrm.shape) * 2.0 ** -24
        out.append(oracle.OracleScene(xq + c, nq, sc.radius_array(), sc.material, grid=256))
    return out


def conditioned_errors(r, ro, r_ens, dyn=30.0):
    """Co-polar |r - ro| (dB) where ro is within dyn dB of the curve's peak over angles, with
    each sample's fp32 spread max_j |r_j - ro| over the ensemble."""
    err, spread = [], []
    for p in range(2):
        a, b = r[..., p, p], ro[..., p, p]
        sel = b >= b.max(axis=0, keepdims=True) - dyn
        err.append(np.abs(a - b)[sel])
        spread.append(np.max([np.abs(re[..., p, p] - b)[sel] for re in r_ens], axis=0))
    return np.concatenate(err), np.concatenate(spread)


def report(name, e):
    print(f"{name}: median {np.median(e):.4f} dB, p90 {np.percentile(e, 90):.3f}, p99 "
          f"{np.percentile(e, 99):.3f}, max {e.max():.3f}; within 0.1 dB {(e <= 0.1).mean():.4f} "
          f"of {e.size}")


def db_errors(r, ro, dyn=30.0):
    out = []
    for p in range(2):
        a, b = r[..., p, p], ro[..., p, p]
        sel = b >= b.max(axis=0, keepdims=True) - dyn
        out.append(np.abs(a - b)[sel])
    return np.concatenate(out)
