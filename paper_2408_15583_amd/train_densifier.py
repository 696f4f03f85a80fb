"""Training and evaluation of the learned densifier on seeded synthetic scenes.

Data (a synthetic stand-in for the sampled-mesh dataset of Sec. IV-A): composite scenes of the
twelve-primitive generator with N points drawn from [n_lo, n_hi]; each scene is viewed from
random propagation directions uniform on the sphere; per view the network input is the TUBE
first-hit buffer at h x w (tube radius drawn from U(1, 3) coarse pixels per scene, as the
relative radii of Sec. IV-A) and the targets are the DISK first-hit buffer at 2h x 2w (depth
t/D, view-frame normal, hit mask).  Every pair is made on the GPU by pe_densifier_make_pair.

Training: AdamW (Sec. IV-A), learning rate halved every `decay_every` steps down to lr_min.

Evaluation (single-bounce monostatic PO of Eq. (14)): RCS from the densified GFB and from the
coarse GFB with depth-gradient normals (no network), each compared with the plain first-hit
trace at the full screen, as RMSE in dB over azimuths and frequencies of the co-polarised
channels where the plain curve is within `dyn` dB of its peak.

    python -m paper_2408_15583_amd.train_densifier --steps 3000 --out densifier.ckpt
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def sphere_dirs(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def make_dataset(pe, ctx, n_scenes, views, h, seed, n_lo=100_000, n_hi=500_000, view_res=256,
                 tube_k=0, corner_frac=0.0):
    """Returns device tensors (coarse, depth_gt, nrm_gt, mask_gt) with n_scenes * views pairs;
    tube_k: heap size of Algorithm 1 for the coarse buffers (0 = unbounded); corner_frac: the
    share of scenes drawn as concave plate corners (scenes.corner_assembly) instead of
    composites."""
    import torch
    import scenes
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(n_scenes):
        n = int(rng.integers(n_lo, n_hi + 1))
        sd = int(rng.integers(1 << 30))
        if rng.uniform() < corner_frac:
            sc = scenes.corner_assembly(seed=sd, n_points=n)
        else:
            sc = scenes.composite(seed=sd, n_points=n)
        s = pe.Scene.from_scene(ctx, sc, view_res=view_res)
        dirs = sphere_dirs(rng, views)
        parts.append(pe.make_pair(ctx, s, dirs, h, h, tube_px=float(rng.uniform(1.0, 3.0)),
                                  tube_k=tube_k))
        s.close()
    return tuple(torch.cat([p[j] for p in parts]) for j in range(4))


def train(net, data, steps, batch=8, lr0=1e-3, lr_min=1e-5, decay_every=1000, wd=1e-4,
          seed=0, log=None):
    import torch
    coarse, dg, ng, mg = data
    n = coarse.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(coarse.device)
        lr = max(lr_min, lr0 * 0.5 ** (it // decay_every))
        L = net.train_step(coarse[idx].contiguous(), dg[idx].contiguous(), ng[idx].contiguous(),
                           mg[idx].contiguous(), lr=lr, weight_decay=wd)
        hist.append(L)
        if log and (it % 100 == 0 or it == steps - 1):
            log(f"step {it} lr {lr:.2e} loss {L[0]:.4f} (L1 {L[1]:.2e} L2 {L[2]:.3f} "
                f"L3 {L[3]:.4f} L4 {L[4]:.3f})")
    return hist


def rmse_db(r, ref, dyn=30.0):
    """RMSE in dB over [az, f] of the co-polarised channels where ref is within dyn dB of
    its peak over azimuths."""
    errs = []
    for p in (0, 1):
        a = r[:, 0, :, p, p]
        b = ref[:, 0, :, p, p]
        sel = b >= b.max(axis=0, keepdims=True) - dyn
        errs.append((a - b)[sel])
    e = np.concatenate(errs)
    return float(np.sqrt(np.mean(e ** 2)))


def evaluate(pe, ctx, net, n_scenes, az, el, freqs, screen, seed, n_lo=100_000,
             n_hi=500_000, view_res=256, max_uncertain=0.0, tube_k=0):
    """max_uncertain: fallback threshold of the densified solve (0 = library default,
    1 = never fall back, which measures the network alone)."""
    import scenes
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_scenes):
        n = int(rng.integers(n_lo, n_hi + 1))
        sc = scenes.composite(seed=int(rng.integers(1 << 30)), n_points=n)
        s = pe.Scene.from_scene(ctx, sc, view_res=view_res)
        inc = scenes.azimuth_sweep(az, el)
        _, r_plain, _ = pe.solve(ctx, s, inc, freqs, screen)
        _, r_coarse, _ = pe.solve(ctx, s, inc, freqs, screen, geometry="coarse", tube_k=tube_k)
        _, r_dens, st = pe.solve(ctx, s, inc, freqs, screen, densifier=net,
                                 max_uncertain=max_uncertain, tube_k=tube_k)
        out.append(dict(n=n, coarse=rmse_db(r_coarse, r_plain), densified=rmse_db(r_dens, r_plain),
                        fallbacks=st["densifier_fallbacks"]))
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--coarse", type=int, default=128, help="coarse (input) resolution")
    ap.add_argument("--scenes", type=int, default=32)
    ap.add_argument("--views", type=int, default=32)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--eval-scenes", type=int, default=2)
    ap.add_argument("--tube-k", type=int, default=0, help="heap size K of the coarse buffer "
                    "(0 = unbounded)")
    ap.add_argument("--corner-frac", type=float, default=0.0,
                    help="share of concave plate-corner training scenes")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    import torch
    import paper_2408_15583_amd as pe
    log = lambda m: print(f"[train] {m}", flush=True)
    ctx = pe.Context(0)
    t0 = time.time()
    data = make_dataset(pe, ctx, args.scenes, args.views, args.coarse, args.seed,
                        tube_k=args.tube_k, corner_frac=args.corner_frac)
    torch.cuda.synchronize()
    log(f"{data[0].shape[0]} pairs at {args.coarse}^2 -> {2 * args.coarse}^2 in {time.time() - t0:.1f} s")
    net = pe.Densifier(ctx, base=args.base, seed=args.seed)
    t0 = time.time()
    train(net, data, args.steps, args.batch, args.lr, decay_every=max(1, args.steps // 4),
          seed=args.seed, log=log)
    torch.cuda.synchronize()
    dt = time.time() - t0
    log(f"{args.steps} steps in {dt:.1f} s ({args.steps * args.batch / dt:.1f} pairs/s)")
    if args.out:
        net.save(args.out)
    for mu, what in ((1.0, "network alone"), (0.0, "default fallback")):
        res = evaluate(pe, ctx, net, args.eval_scenes, np.arange(0, 360, 10.0), 30.0,
                       np.linspace(2e9, 12e9, 16), 2 * args.coarse, args.seed + 1000,
                       max_uncertain=mu, tube_k=args.tube_k)
        for r in res:
            log(f"eval ({what}) N={r['n']}: RMSE vs plain: coarse {r['coarse']:.2f} dB, "
                f"densified {r['densified']:.2f} dB, fallbacks {r['fallbacks']:.0f}")
    net.close()
    ctx.close()


if __name__ == "__main__":
    main()
