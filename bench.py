#!/usr/bin/env python3
"""Benchmark of the plain SBR hot path on one MI355X.

Workload (default): the twelve-primitive composite scene sampled to 2,000,000 points, six
1024^2 aggregation views, a 1024^2 ray screen, 360 monostatic azimuths at 30 deg elevation,
64 frequencies from 2 to 12 GHz, up to 4 bounces.  One step = one pass of the whole path on
that input: scene ingest (recentre, normalise, spatial order), the six view buffers with their
min/max pyramids, then for every azimuth the first-hit splat, ray generation, bounce march,
visibility, facet records and the PO sum over all frequencies.  Inputs (points, normals) are
resident in device memory before the timed region.

Bounces and visibility are traced against every splat through the object-space hierarchy by
default (--secondary splats: the result follows the exact oracle); the aggregation views' march
(--secondary views) is timed beside it for a few steps.

Prints one JSON line: value = ray-bounces/s (live-ray intersection queries, primary rays
included, per second of step wall time); extra fields give RCS samples/s, the dominant
kernel's roofline (HIP events on its launch stream, over the timed steps), the FP64 CPU
oracle timed on a bounded sample of the same workload, and the error of each bounce geometry
against that oracle's culled-exact solve of 36 azimuths.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# fp32 vector issue rate of MI355X: 256 CUs x 128 fp32 lanes per clock x 2.4 GHz = 78.6 T
# lane-ops/s (the published 157.3 TFLOP/s counts an FMA as two flops).
FP32_LANE_OPS = 256 * 128 * 2.4e9

# HBM traffic of k_march from two rocprofv3 --pmc passes over one step of the default workload
# (mean KiB per dispatch), each scaled by what the counter reads for a plain 1 GiB device copy
# (FETCH_SIZE reads 524302 KiB for 1 GiB: factor 2.0; WRITE_SIZE 1048576 KiB: factor 1.0).
# Valid only for the sources they were taken on; any edit of those files reports null.
MARCH_TRAFFIC = dict(
    fetch_kib=12002034.8, write_kib=272779.7, fetch_factor=2.0, write_factor=1.0,
    sources={"paper_2408_15583_amd/csrc/k_trace.hip":
             "29d5a3ed46fcc6a9e8e3a31d52ad3cb4dccb09ca086581c56200e5d7259b3adc",
             "paper_2408_15583_amd/csrc/pe_device.h":
             "e8ec339ff11e3ccc787afcff74d5151897879d2a05c2796c91656e2912572470"})


# L2-to-fabric traffic of k_trace_bvh from the same two counter passes over one step (mean KiB
# per dispatch over its three bounces), scaled by the same copy calibration; null once any of
# the traversal's sources changes.
BVH_TRAFFIC = dict(
    fetch_kib=17450870.3, write_kib=842965.5, fetch_factor=2.0, write_factor=1.0,
    sources={"paper_2408_15583_amd/csrc/k_bvh.hip":
             "2f00419cfdb57f5d932923cde7392aa7fade7dd46970408766a0a4a1c5ef215e",
             "paper_2408_15583_amd/csrc/pe_bvh.h":
             "16d20123701aff881396c50d0cef005bd6dc8b60e7ed4c0845356475ff60e2d1",
             "paper_2408_15583_amd/csrc/pe_device.h":
             "0fc49f89a3ef47b0f58a548b553fdaf736d9d75156e0aa2a339a8359f14eab05",
             "paper_2408_15583_amd/csrc/pe_geom.h":
             "c59a832fb993886519791ad8760ae772576bcca31bb44d5e2b6504e5f4058df1"})


def _counter_traffic(t):
    import hashlib
    for rel, digest in t["sources"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"])


def bvh_traffic():
    """Counter-measured bytes per k_trace_bvh launch, or None once its sources changed."""
    return _counter_traffic(BVH_TRAFFIC)


def march_traffic():
    """Counter-measured bytes per k_march launch, or None once the kernel's sources changed."""
    return _counter_traffic(MARCH_TRAFFIC)


def po_slots_per_term():
    """Issue slots (fp32 lane-op equivalents) one PO term needs: fp64 ops count twice (half
    rate), transcendentals four times (quarter rate).  The 8 fp64 conversions and adds of the
    accumulators run once per aligned group of four terms."""
    fp64 = 1 + 1 + 1 + (8 + 8) / 4  # D*rev, fraction, cvt f64->f32, accumulators
    fp32 = 2 + 2 * 10 + 2 + 2 + 8  # k*al, k*be, two sinc (series and full, select),
    #                                S and tail mask, wr/wi, 8 fma
    trans = 4 + 2                          # sin, cos, two sinc sines, two reciprocals
    return 2 * fp64 + fp32 + 4 * trans


def cpu_baseline(sc, sw, n_az, sample_px, gpu_rcs, seed=11):
    """FP64 oracle on the host, timed on a bounded sample of the workload: its culled-exact mode
    (uniform grid, bitwise equal to brute force) solves n_az of the workload's azimuths in full
    (screen, frequencies, bounces), and its brute-force mode traces sample_px seeded pixel rays
    of azimuth 0.  The culled-exact RCS also measures each GPU mode's error on those azimuths
    (gpu_rcs: {mode: rcs of all azimuths}), reported with the per-sample fp32 spread of the
    oracle itself (inputs rounded to fp32 in the scene frame)."""
    import numpy as np
    import oracle
    idx = np.linspace(0, len(sw.inc_dir), n_az, endpoint=False).astype(int)
    inc = sw.inc_dir[idx]
    t0 = time.perf_counter()
    o = oracle.OracleScene(sc, grid=256)
    t_grid = time.perf_counter() - t0
    t0 = time.perf_counter()
    E, st = o.solve(inc, sw.freq_hz, sw.screen, sw.screen, sw.max_bounces, sw.eps)
    dt = time.perf_counter() - t0
    ro = oracle.rcs_dbsm(E)
    c = 0.5 * (sc.xyz.min(0) + sc.xyz.max(0))
    o32 = oracle.OracleScene((sc.xyz - c).astype(np.float32).astype(np.float64) + c,
                             sc.nrm.astype(np.float32).astype(np.float64), sc.radius_array(),
                             sc.material, grid=256)
    r32 = oracle.rcs_dbsm(o32.solve(inc, sw.freq_hz, sw.screen, sw.screen, sw.max_bounces,
                                    sw.eps)[0])

    def errors(r):
        out = []
        for p in range(2):
            a, b = r[..., p, p], ro[..., p, p]
            sel = b >= b.max(axis=0, keepdims=True) - 30.0
            out.append(np.abs(a - b)[sel])
        e = np.concatenate(out)
        return dict(median_db=float(np.median(e)), p90_db=float(np.percentile(e, 90)),
                    p99_db=float(np.percentile(e, 99)), max_db=float(e.max()),
                    within_0p1db=float((e <= 0.1).mean()), samples=int(e.size))

    accuracy = {m: errors(r[idx]) for m, r in gpu_rcs.items()}
    accuracy["oracle_fp32_inputs"] = errors(r32)
    rng = np.random.default_rng(seed)
    pix = rng.choice(sw.screen * sw.screen, size=sample_px, replace=False)
    t0 = time.perf_counter()
    nb, _, _ = o.trace_pixels(sw.inc_dir[0], sw.screen, sw.screen, pix, sw.max_bounces, sw.eps,
                              grid=0)
    dtb = time.perf_counter() - t0
    qb = float(np.sum(nb + (nb < sw.max_bounces)))
    q = float(st["queries"])
    return dict(value=q / dt, unit="ray-bounces/s", cores=oracle.num_threads(), kind="oracle",
                rcs_samples_per_s=len(inc) * len(sw.freq_hz) / dt,
                sample=f"culled-exact oracle (256^3 grid, built in {t_grid:.1f} s, not timed), "
                       f"{len(inc)} of the {len(sw.inc_dir)} azimuths at {sw.screen}^2, "
                       f"{len(sw.freq_hz)} freqs, <= {sw.max_bounces} bounces: {q:.0f} queries "
                       f"in {dt:.1f} s",
                brute_force=dict(value=qb / dtb, unit="ray-bounces/s",
                                 sample=f"{sample_px} seeded pixel rays of azimuth 0, brute force "
                                        f"over all {sc.n} disks ({qb:.0f} queries in "
                                        f"{dtb:.1f} s)"),
                accuracy=accuracy)


def _latency_classes(done):
    """p50 / p99 / count of submit-to-completion latency per screen-size class and overall;
    done: list of (screen, latency ms)."""
    import numpy as np
    out = {}
    for cls in scenes_mod().SERVING_SCREENS + (None,):
        v = np.array([ms for sc, ms in done if cls is None or sc == cls])
        if len(v):
            out["all" if cls is None else f"{cls}^2"] = dict(
                n=int(len(v)), p50_ms=float(np.percentile(v, 50)),
                p99_ms=float(np.percentile(v, 99)))
    return out


def scenes_mod():
    import scenes
    return scenes


def serving(pe, ctx, seconds, n_scenes=64, seed=5, log=None, budget_8gb_seconds=0.0):
    """Continuous-batching server under the serving workload's request mix: a resident pool of
    n_scenes composite scenes (N log-uniform in [5e4, 4e6]), screens uniform in {256, 512, 1024,
    2048}^2, angle counts log-uniform in [1, 720], frequency counts log-uniform in [1, 128]
    (2-12 GHz), 1-5 bounces, every request traced against every splat.  Phase 1 submits a closed
    batch of 64 requests at once (saturation: solves/s and work/s the GPU sustains); phase 2
    offers Poisson arrivals for `seconds` at 70 % of the saturated work rate and reports latency
    percentiles from submit to completion, overall and per screen-size class.  Phase 3 (when
    budget_8gb_seconds > 0) repeats phase 2's offered load in a context limited to 8 GiB with the
    part of the pool that fits in 1.25 GiB, so admission by footprint serialises the large
    requests (a request larger than the budget left by the scenes is refused and counted).  Work per request follows a cost model, pixels x angles x (bounces + frequencies
    / 16), whose mean over the mix is estimated from 20000 draws; the request sizes span five
    orders of magnitude, so a rate set from request counts alone would offer a load that
    depends on which few large requests the saturation sample happened to hold."""
    import numpy as np
    scenes = scenes_mod()
    rng = np.random.default_rng(seed)
    t_pool = time.perf_counter()
    held0 = ctx.footprint()[0]
    sizes = scenes.serving_pool_sizes(n_scenes, seed)
    pool_sc, pool = [], []
    for i, n in enumerate(sizes):
        sc = scenes.serving_scene(i, n)
        pool_sc.append(sc)
        pool.append(pe.Scene.from_scene(ctx, sc, view_res=1024))
    pool_bytes = ctx.footprint()[0] - held0
    t_pool = time.perf_counter() - t_pool
    if log:
        log(f"serving pool: {len(pool)} scenes, {sum(sizes) / 1e6:.1f}M points, "
            f"{pool_bytes / 2**30:.2f} GiB resident ({t_pool:.1f} s)")

    def submit(c, scene_list, r):
        return pe.submit(c, scene_list[r["scene"]], r["inc_dir"], r["freq_hz"], r["screen"],
                         max_bounces=r["max_bounces"], eps=r["eps"], secondary="splats")

    def work(r):
        return float(r["screen"]) ** 2 * len(r["inc_dir"]) * (r["max_bounces"] +
                                                              len(r["freq_hz"]) / 16.0)

    mrng = np.random.default_rng(seed + 1)
    mean_work = float(np.mean([work(scenes.serving_request(mrng, pool_sc))
                               for _ in range(20000)]))

    # phase 1: saturation
    reqs = [scenes.serving_request(rng, pool_sc) for _ in range(64)]
    pe.server_stats(ctx, reset=True)
    t0 = time.perf_counter()
    ts = [submit(ctx, pool, r) for r in reqs]
    samples = 0
    for t, r in zip(ts, reqs):
        t.wait()
        samples += len(r["inc_dir"]) * len(r["freq_hz"])
    dt = time.perf_counter() - t0
    cap = len(reqs) / dt
    work_rate = sum(work(r) for r in reqs) / dt
    sat = pe.server_stats(ctx, reset=True)
    if log:
        log(f"serving saturation: {len(reqs)} requests in {dt:.2f} s ({cap:.2f} solves/s)")

    def poisson(c, scene_list, draw, rate, window, tag):
        arrivals = []
        t = 0.0
        while t < window:
            t += rng.exponential(1.0 / rate)
            arrivals.append(t)
        rs = [draw() for _ in arrivals]
        pe.server_stats(c, reset=True)
        t0 = time.perf_counter()
        ts = []
        next_log = 15.0
        for a, r in zip(arrivals, rs):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            ts.append(submit(c, scene_list, r))
            if log and now > next_log:
                log(f"serving {tag}: {len(ts)} submitted at {now:.0f} s")
                next_log += 15.0
        done = []
        rejected = 0
        for t, r in zip(ts, rs):
            try:
                _, _, st = t.wait()
            except pe.PEError as e:
                # admission by footprint: a request larger than the budget the resident scenes
                # leave is refused at once
                if e.status != pe._native.PE_ENOMEM:
                    raise
                rejected += 1
                continue
            done.append((r["screen"], st["time_ms"]))
        st = pe.server_stats(c, reset=True)
        return dict(offered_rate_per_s=rate, requests=len(ts), completed=st["completed"],
                    rejected_over_budget=rejected,
                    window_s=time.perf_counter() - t0, p50_ms=st["p50_ms"], p99_ms=st["p99_ms"],
                    mean_ms=st["mean_ms"], max_concurrent=st["max_concurrent"],
                    reqs_per_batch=st["reqs_per_batch"], by_screen=_latency_classes(done))

    # phase 2: Poisson arrivals offering 70 % of the saturated work rate
    rate = 0.7 * work_rate / mean_work
    full = poisson(ctx, pool, lambda: scenes.serving_request(rng, pool_sc), rate, seconds,
                   "full HBM")
    if log:
        log(f"serving full HBM: {full['requests']} requests, p50 {full['p50_ms']:.0f} ms, "
            f"p99 {full['p99_ms']:.0f} ms")
    for s in pool:
        s.close()
    out = dict(pool_scenes=len(pool), pool_points=int(sum(sizes)), pool_gib=pool_bytes / 2**30,
               saturation_solves_per_s=cap, saturation_rcs_samples_per_s=samples / dt,
               saturation_reqs_per_batch=sat["reqs_per_batch"],
               capacity_for_mix_per_s=work_rate / mean_work, full_hbm=full)
    # phase 3: the same offered load under an 8 GiB budget
    if budget_8gb_seconds > 0:
        c8 = pe.Context(0, budget=8 << 30)
        sub_sc, sub = [], []
        for sc in pool_sc:
            s = pe.Scene.from_scene(c8, sc, view_res=1024)
            if c8.footprint()[0] > 1.25 * 2**30:
                s.close()
                continue
            sub_sc.append(sc)
            sub.append(s)
        b8 = poisson(c8, sub, lambda: scenes.serving_request(rng, sub_sc), rate,
                     budget_8gb_seconds, "8 GiB")
        b8["pool_scenes"] = len(sub)
        if log:
            log(f"serving 8 GiB: {b8['requests']} requests, p50 {b8['p50_ms']:.0f} ms, "
                f"p99 {b8['p99_ms']:.0f} ms, max concurrent {b8['max_concurrent']:.0f}")
        for s in sub:
            s.close()
        c8.close()
        out["budget_8gib"] = b8
    out["note"] = ("serving request mix (scene pool of %d); Poisson arrivals offering 70%% of the "
                   "saturated work rate (cost model pixels x angles x (bounces + freqs/16)); "
                   "200 req/s of this mix is %.0fx one GPU's capacity"
                   % (len(pool), 200.0 * mean_work / work_rate))
    return out


# Dense MFMA flops of one densifier forward pass at base 32 from a coarse h x w input
def densifier_flops(base, h, w):
    C = [base << l for l in range(4)]
    f = 0.0
    for l in range(4):
        M = (h >> l) * (w >> l)
        f += 2 * M * C[l] * 4 * C[l] * 2           # ConvNeXt 1x1 expand + project
        if l > 0:
            f += 2 * M * C[l - 1] * C[l]           # 1x1 down
    for co in (1, 3, 1):
        for l in (3, 2, 1):
            Ml = (h >> l) * (w >> l)
            f += 2 * Ml * 9 * C[l] * 4 * C[l - 1]          # 3x3 up (before the shuffle)
            f += 2 * (4 * Ml) * 9 * 2 * C[l - 1] * C[l - 1]  # 3x3 fuse
        f += 2 * h * w * 9 * C[0] * 4 * co                 # 3x3 out
    return f


def densifier_bench(pe, ctx, batch=8, h=256, steps=10, log=None):
    """Inference and training throughput of the densifier at the workload size (coarse
    256^2 -> 512^2, base 32), on synthetic inputs; dense-conv flops / wall time."""
    import torch
    net = pe.Densifier(ctx, base=32, seed=1)
    g = torch.Generator(device="cpu").manual_seed(0)
    x = (torch.rand((batch, h, h), generator=g) * (torch.rand((batch, h, h), generator=g) < 0.7)).cuda()
    dg = torch.rand((batch, 2 * h, 2 * h), generator=g).cuda()
    ng = torch.nn.functional.normalize(torch.randn((batch, 2 * h, 2 * h, 3), generator=g), dim=-1).cuda()
    mg = (torch.rand((batch, 2 * h, 2 * h), generator=g) < 0.6).float().cuda()
    net.infer(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.infer(x)
    torch.cuda.synchronize()
    ti = (time.perf_counter() - t0) / steps
    net.train_step(x, dg, ng, mg, lr=1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(x, dg, ng, mg, lr=1e-4)
    torch.cuda.synchronize()
    tt = (time.perf_counter() - t0) / steps
    net.close()
    fl = densifier_flops(32, h, h) * batch
    return dict(batch=batch, coarse=h, infer_ms=ti * 1e3, infer_images_per_s=batch / ti,
                train_step_ms=tt * 1e3, train_pairs_per_s=batch / tt,
                infer_tflops=fl / ti / 1e12, train_tflops=3 * fl / tt / 1e12,
                mfma_bf16_peak_tflops=2500.0, infer_frac=fl / ti / 2.5e15,
                note="dense-conv flops of the network / wall time (whole pass incl. VALU layers)")


def densifier_claim(pe, ctx, train_steps=1500, log=None):
    """Densified against plain solves at the densifier workload (coarse 256^2 -> 512^2,
    composite scenes of 1e5-5e5 points): a network trained here for a short schedule on
    8 x 48 GPU-made pairs, then, on two held-out scenes (18 azimuths at 30 deg x 16 frequencies,
    single bounce), the RCS error of each solve form against the plain 512^2 first-hit trace
    (RMSE in dB of the co-polar channels within 30 dB of each curve's peak) and its solves/s.
    Forms: densified (network alone, no fallback), plain at 512^2 in fp32 phase and sum (the
    mixed-precision form), and plain at 256^2 and 128^2 (cheaper plain solves whose error
    brackets the densified one)."""
    import numpy as np
    import torch
    import scenes
    from paper_2408_15583_amd import train_densifier as T
    t0 = time.perf_counter()
    data = T.make_dataset(pe, ctx, n_scenes=8, views=48, h=256, seed=11, n_lo=100_000,
                          n_hi=500_000)
    net = pe.Densifier(ctx, base=32, seed=5)
    hist = T.train(net, data, steps=train_steps, batch=8, lr0=1e-3, decay_every=500, seed=5)
    del data
    t_train = time.perf_counter() - t0
    if log:
        log(f"densifier claim: trained {train_steps} steps in {t_train:.1f} s, loss "
            f"{np.mean([h[0] for h in hist[:50]]):.3f} -> {np.mean([h[0] for h in hist[-50:]]):.3f}")
    rng = np.random.default_rng(1234)
    az = np.arange(0, 360, 20.0)
    freqs = np.linspace(2e9, 12e9, 16)
    forms = {"densified_512": dict(screen=512, densifier=net, max_uncertain=1.0),
             "plain_512_fp32": dict(screen=512, precision="fp32"),
             "plain_256": dict(screen=256), "plain_128": dict(screen=128)}
    err = {k: [] for k in forms}
    ms = {k: [] for k in list(forms) + ["plain_512"]}

    def timed(s, inc, kw):
        kw = dict(kw)
        screen = kw.pop("screen")
        pe.solve(ctx, s, inc, freqs, screen, **kw)  # untimed first call
        best = 1e30
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = pe.solve(ctx, s, inc, freqs, screen, **kw)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return out[1], best * 1e3

    for i in range(2):
        n = int(rng.integers(100_000, 500_001))
        sc = scenes.composite(seed=int(rng.integers(1 << 30)), n_points=n)
        s = pe.Scene.from_scene(ctx, sc, view_res=256)
        inc = scenes.azimuth_sweep(az, 30.0)
        ref, t_ref = timed(s, inc, dict(screen=512))
        ms["plain_512"].append(t_ref)
        for k, kw in forms.items():
            r, t = timed(s, inc, kw)
            err[k].append(T.rmse_db(r, ref))
            ms[k].append(t)
        s.close()
    net.close()
    out = {"plain_512": dict(rmse_db=0.0, ms=float(np.mean(ms["plain_512"])),
                             solves_per_s=1e3 / float(np.mean(ms["plain_512"])))}
    for k in forms:
        out[k] = dict(rmse_db=float(np.mean(err[k])), ms=float(np.mean(ms[k])),
                      solves_per_s=1e3 / float(np.mean(ms[k])))
    d = out["densified_512"]
    cheaper = [k for k in ("plain_128", "plain_256", "plain_512_fp32", "plain_512")
               if out[k]["rmse_db"] <= d["rmse_db"] and out[k]["solves_per_s"] >= d["solves_per_s"]]
    out["densified_beats_plain_at_equal_error"] = not cheaper
    out["plain_forms_at_least_as_accurate_and_fast"] = cheaper
    out["fp32_beats_plain_at_equal_error"] = bool(
        out["plain_512_fp32"]["rmse_db"] <= 0.01 and
        out["plain_512_fp32"]["solves_per_s"] > out["plain_512"]["solves_per_s"])
    out["train_s"] = t_train
    out["note"] = ("solve = 18 incidences x 16 frequencies, single bounce, on held-out scenes; "
                   "errors vs the plain 512^2 trace")
    if log:
        log("densifier claim: " + ", ".join(f"{k} {v['rmse_db']:.2f} dB {v['solves_per_s']:.0f}/s"
                                            for k, v in out.items() if isinstance(v, dict)))
    return out


def next_rows(pe, ctx, sc, xyz_dev, nrm_dev, view_res, log=None):
    """One timed call of each extension row beside the hot path (GPU wall time, the device
    synchronised on both sides; one untimed call first): learned-GFB fusion on the synthetic
    OctAR (eight 512^2 sensor views of first-hit buffers, 256^3 grid), the fused splats traced
    with and without the Eq. (23) normal blending, the OctAR 3-bounce monostatic sweep, a
    bistatic sweep, the finite-K tube raster and PCA normals on the composite."""
    import numpy as np
    import torch
    import scenes

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    out = {}
    oc = scenes.octar()
    views = scenes.octar_views()
    os_ = pe.Scene.from_scene(ctx, oc, view_res=512, view_dirs=views)
    info = os_.info()
    _, dg, ng, mg = pe.make_pair(ctx, os_, views, 256, 256)
    side = 2.0 * float(oc.meta["half"])
    fz, ms = timed(lambda: pe.fuse_gfbs(ctx, views, dg, ng, mg, info["centre"], info["R"],
                                        grid=256, grid_side=side))
    out["fusion"] = dict(views=8, res=512, grid=256, splats=int(fz["xyz"].shape[0]), ms=ms)
    eps = 0.5 * float(oc.radius)
    inc = scenes.azimuth_sweep(np.arange(0.0, 360.0, 10.0), 30.0)
    for name, blend in (("fused_sweep", 0.0), ("fused_sweep_eq23", side / 256)):
        fs = pe.Scene(ctx, fz["xyz"], fz["nrm"], fz["radius"], view_dirs=views, view_res=512,
                      blend_radius=blend)
        (_, _, st), ms = timed(lambda: pe.solve(ctx, fs, inc, [5e9], 512, max_bounces=3, eps=eps))
        out[name] = dict(incidences=len(inc), screen=512, bounces=3, blend_radius=blend, ms=ms,
                         ray_bounces_per_s=st["ray_queries"] / (ms * 1e-3))
        fs.close()
    (_, _, st), ms = timed(lambda: pe.solve(ctx, os_, inc, [5e9], 512, max_bounces=3, eps=eps))
    out["octar_sweep"] = dict(points=int(oc.n), incidences=len(inc), screen=512, bounces=3, ms=ms,
                              ray_bounces_per_s=st["ray_queries"] / (ms * 1e-3))
    binc = scenes.azimuth_sweep([40.0, 130.0], 30.0)
    obs = -scenes.azimuth_sweep(np.arange(0.0, 360.0, 22.5), 20.0)
    (_, _, st), ms = timed(lambda: pe.solve(ctx, os_, binc, [3e9, 5e9], 512, max_bounces=3,
                                            eps=eps, obs_dir=obs))
    out["bistatic"] = dict(incidences=2, observations=len(obs), freqs=2, bounces=3, ms=ms,
                           rcs_samples_per_s=2 * len(obs) * 2 / (ms * 1e-3))
    os_.close()
    s = pe.Scene(ctx, xyz_dev, nrm_dev, sc.radius, view_res=view_res)
    d = np.array([0.3, -0.4, -0.866])
    _, ms = timed(lambda: pe.render_tube_topk(ctx, s, d / np.linalg.norm(d), 1024, 1024,
                                              2.0 * float(sc.radius), 4))
    out["topk_raster"] = dict(screen=1024, K=4, points=int(sc.n), ms=ms)
    s.close()
    xyz = torch.from_numpy(np.ascontiguousarray(sc.xyz, dtype=np.float32)).cuda()
    _, ms = timed(lambda: pe.estimate_normals(ctx, xyz, 16))
    out["pca_normals"] = dict(points=int(sc.n), k=16, ms=ms)
    if log:
        log("next rows: " + ", ".join(f"{k} {v['ms']:.1f} ms" for k, v in out.items()))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=2_000_000)
    ap.add_argument("--screen", type=int, default=1024)
    ap.add_argument("--n-az", type=int, default=360)
    ap.add_argument("--n-freq", type=int, default=64)
    ap.add_argument("--bounces", type=int, default=4)
    ap.add_argument("--precision", default="fp64phase", choices=["fp64phase", "fp32", "fp64acc"])
    ap.add_argument("--secondary", default="splats", choices=["splats", "views"],
                    help="bounce geometry of the timed steps: every splat through the "
                         "object-space hierarchy, or what the aggregation views retain")
    ap.add_argument("--compare-steps", type=int, default=2,
                    help="timed steps of the other bounce geometry, reported beside (0 = skip)")
    ap.add_argument("--cpu-az", type=int, default=36,
                    help="azimuths the CPU oracle solves in full (0 = skip the CPU leg)")
    ap.add_argument("--cpu-sample", type=int, default=2000,
                    help="pixel rays traced by the brute-force oracle")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="Poisson serving window (0 = skip the serving measurement)")
    ap.add_argument("--serve-8gb-seconds", type=float, default=20.0,
                    help="Poisson window of the same load under an 8 GiB budget (0 = skip)")
    ap.add_argument("--serve-scenes", type=int, default=64, help="serving scene pool size")
    ap.add_argument("--no-densifier", action="store_true")
    ap.add_argument("--claim-steps", type=int, default=1500,
                    help="training steps of the densified-vs-plain comparison (0 = skip)")
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the fusion / OctAR / bistatic / finite-K / PCA-normals timings")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the hot path shards by "
              "incidence angle with no exchange, see the design notes.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2408_15583_amd as pe
    import scenes

    if args.copy_calib:
        n = (1 << 30) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return

    t_gen = time.perf_counter()
    sc, sw = scenes.workload_composite(n_points=args.points, n_az=args.n_az, screen=args.screen,
                                       n_freq=args.n_freq, max_bounces=args.bounces)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] scene generated: {sc.n} points, radius {sc.radius*1e3:.2f} mm, "
          f"eps {sw.eps*1e3:.2f} mm ({t_gen:.1f} s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda")
    xyz = torch.from_numpy(np.ascontiguousarray(sc.xyz)).to(dev)
    nrm = torch.from_numpy(np.ascontiguousarray(sc.nrm, dtype=np.float32)).to(dev)
    torch.cuda.synchronize()
    ctx = pe.Context(0)

    def step(secondary=args.secondary):
        s = pe.Scene(ctx, xyz, nrm, sc.radius, view_res=sw.view_res)
        E, rcs, st = pe.solve(ctx, s, sw.inc_dir, sw.freq_hz, sw.screen,
                              max_bounces=sw.max_bounces, eps=sw.eps, precision=args.precision,
                              secondary=secondary)
        s.close()
        return E, rcs, st

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    ctx.kernel_stats(reset=True)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    queries = 0.0
    terms = 0.0
    march_rays = 0.0
    march_hits = 0.0
    last = None
    for i in range(args.steps):
        last = step()
        queries += last[2]["ray_queries"]
        terms += last[2]["po_terms"]
        march_rays += last[2]["march_rays"]
        march_hits += last[2]["march_hits"]
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_profiling(False)
    ks = ctx.kernel_stats(reset=True)
    dt = t1 - t0
    ms_step = 1e3 * dt / args.steps
    E, rcs, st = last
    finite = np.isfinite(rcs[..., 0, 0]).all() and np.isfinite(rcs[..., 1, 1]).all()

    # dominant kernel and its roofline: HIP events on the launch stream over the timed steps
    groups = dict(ks)
    for prefix in ("march", "bvh"):
        part = {k: v for k, v in ks.items() if k.startswith(prefix + "_b")}
        if part:
            for k in part:
                groups.pop(k)
            groups[prefix] = (sum(v[0] for v in part.values()), sum(v[1] for v in part.values()))
    name, (tot_ms, launches) = max(groups.items(), key=lambda kv: kv[1][0])
    avg_ms = tot_ms / max(launches, 1)
    if name in ("march", "bvh"):
        # algorithmic bytes of one bounce (the secondary-hit pass and its apply) per live ray:
        # the ray state, 76 B (18 fp32 + fp64 path + u32 pixel id), read once and written once
        # for the rays that continue; the SoA state the library keeps is 97 B (21 fp32: the
        # incoming direction and the two incident polarisations kept whole, + fp64 path + u8
        # bounce count + u32 facet index), reported beside.  Scene data and view pyramids are
        # not counted.
        rays = march_rays / args.steps
        hits = march_hits / args.steps
        per_step_bytes = 76.0 * rays + 76.0 * hits
        per_launch = per_step_bytes / (launches / args.steps)
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        soa_launch = (97.0 * rays + 97.0 * hits + rays) / (launches / args.steps)
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS,
                    traffic=march_traffic() if name == "march" else bvh_traffic(),
                    kernel="k_march" if name == "march" else "k_trace_bvh",
                    avg_launch_ms=avg_ms, launches=launches, bytes_per_launch=per_launch,
                    soa_bytes_per_launch=soa_launch,
                    soa_frac=soa_launch / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    rays_per_s=rays / (tot_ms / args.steps * 1e-3),
                    note="76 B state read per live ray + 76 B write per continuing ray "
                         "(soa_*: the 97 B SoA state + 1 B flag)")
    elif name == "po_sum":
        per_launch_terms = terms / launches
        achieved = per_launch_terms * po_slots_per_term() / (avg_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP32_LANE_OPS / 1e12,
                    unit="T lane-op/s", frac=achieved / (FP32_LANE_OPS / 1e12), traffic=None,
                    kernel="k_po_sum", avg_launch_ms=avg_ms, launches=launches)
    else:
        roof = dict(bound="hbm", achieved=None, peak=HBM_PEAK_GBS, unit="GB/s", frac=None,
                    traffic=None, kernel=name, avg_launch_ms=avg_ms, launches=launches)

    out = {
        "metric": "ray-bounces/s + RCS samples/s at <=0.1 dB error; p50/p99 solve latency",
        "value": queries / dt,
        "unit": "ray-bounces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f32+f64phase",
        "data": "synthetic",
        "config": {"workload": f"composite 12 primitives, {sc.n} points, {sw.screen}^2 screen, "
                               f"6 views at {sw.view_res}^2, {len(sw.inc_dir)} azimuths at 30 deg "
                               f"elevation, {len(sw.freq_hz)} freqs 2-12 GHz, <= {sw.max_bounces} "
                               "bounces, monostatic",
                   "secondary": args.secondary, "precision": args.precision},
        "rcs_samples_per_s": len(sw.inc_dir) * len(sw.freq_hz) * args.steps / dt,
        "ray_queries_per_step": queries / args.steps,
        "po_terms_per_step": terms / args.steps,
        "march_cap_hits": st["march_cap_hits"],
        "rcs_finite": bool(finite),
        "roofline": roof,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in sorted(ks.items(),
                                                                        key=lambda kv: -kv[1][0])},
    }
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    gpu_rcs = {args.secondary: rcs}
    other = "views" if args.secondary == "splats" else "splats"
    if args.compare_steps > 0:
        # the other bounce geometry on the same workload, timed the same way (fewer steps)
        step(other)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q2 = 0.0
        for _ in range(args.compare_steps):
            _, rcs2, st2 = step(other)
            q2 += st2["ray_queries"]
        torch.cuda.synchronize()
        dt2 = time.perf_counter() - t0
        gpu_rcs[other] = rcs2
        out["compare"] = {"secondary": other, "steps": args.compare_steps,
                          "ms_per_step": 1e3 * dt2 / args.compare_steps, "value": q2 / dt2,
                          "unit": "ray-bounces/s"}
        log(f"{other}: {1e3 * dt2 / args.compare_steps:.1f} ms per step")
    out["next_rows"] = None if args.no_next_rows else next_rows(pe, ctx, sc, xyz, nrm, sw.view_res,
                                                                      log=log)
    out["densifier"] = None if args.no_densifier else densifier_bench(pe, ctx, log=log)
    if not args.no_densifier and args.claim_steps > 0:
        out["densifier"]["vs_plain"] = densifier_claim(pe, ctx, train_steps=args.claim_steps,
                                                       log=log)
    out["serving"] = (serving(pe, ctx, args.serve_seconds, n_scenes=args.serve_scenes, log=log,
                              budget_8gb_seconds=args.serve_8gb_seconds)
                      if args.serve_seconds > 0 else None)
    if args.cpu_az > 0:
        log("CPU oracle leg ...")
        out["cpu_baseline"] = cpu_baseline(sc, sw, args.cpu_az, args.cpu_sample, gpu_rcs)
        acc = out["cpu_baseline"]["accuracy"]
        # error of the timed result against the exact oracle on the oracle's azimuths
        out["accuracy_vs_oracle"] = acc.get(args.secondary)
        log("accuracy: " + ", ".join(f"{m} median {a['median_db']:.4f} / p99 {a['p99_db']:.3f} / "
                                     f"max {a['max_db']:.3f} dB" for m, a in acc.items()))
    else:
        out["cpu_baseline"] = None
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
