"""Gain of the learned densifier (Sec. III-A) on held-out synthetic scenes.

A densifier trained on the GPU for a short schedule on seeded composite scenes must bring the
single-bounce monostatic RCS from the half-resolution TUBE buffer closer to the plain
first-hit trace at the full screen than the same coarse buffer does without the network
(depth-gradient normals, Eq. (16)): the network alone (no fallback) must cut the coarse
buffer's error by at least 20 %.  A fallback threshold that no output can meet must reproduce
the plain solve exactly.  Errors are RMSE in dB over azimuths and frequencies of
the co-polarised channels within 30 dB of each curve's peak.  The trained network is never
stored: every run trains from the same seeds.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_densifier_beats_coarse_buffer():
    import torch
    import paper_2408_15583_amd as pe
    from paper_2408_15583_amd import train_densifier as T
    assert torch.cuda.is_available()
    ctx = pe.Context(0)
    data = T.make_dataset(pe, ctx, n_scenes=8, views=48, h=128, seed=11,
                          n_lo=100_000, n_hi=300_000)
    net = pe.Densifier(ctx, base=32, seed=5)
    hist = T.train(net, data, steps=1500, batch=8, lr0=1e-3, decay_every=500, seed=5)
    assert np.isfinite([h[0] for h in hist]).all()
    assert np.mean([h[0] for h in hist[-50:]]) < 0.5 * np.mean([h[0] for h in hist[:50]])
    res = T.evaluate(pe, ctx, net, n_scenes=2, az=np.arange(0, 360, 20.0), el=30.0,
                     freqs=np.linspace(2e9, 12e9, 16), screen=256, seed=1234,
                     n_lo=100_000, n_hi=300_000, max_uncertain=1.0)
    for r in res:
        print(f"GAIN N={r['n']} coarse {r['coarse']:.3f} dB densified {r['densified']:.3f} dB "
              f"fallbacks {r['fallbacks']:.0f}")
    assert all(r["fallbacks"] == 0 for r in res)
    coarse = np.mean([r["coarse"] for r in res])
    dens = np.mean([r["densified"] for r in res])
    assert dens < 0.8 * coarse, (dens, coarse)
    # a fallback threshold no output can meet sends every incidence to the plain path, whose
    # result must then be the plain solve's, bit for bit
    import scenes
    sc = scenes.composite(seed=77, n_points=150_000)
    s = pe.Scene.from_scene(ctx, sc, view_res=256)
    inc = scenes.azimuth_sweep([0.0, 90.0, 200.0], 30.0)
    f = np.linspace(2e9, 12e9, 4)
    E0, _, _ = pe.solve(ctx, s, inc, f, 256)
    E1, _, st = pe.solve(ctx, s, inc, f, 256, densifier=net, max_uncertain=1e-9)
    assert st["densifier_fallbacks"] == 3
    assert np.array_equal(E0, E1)
    s.close()
    net.close()
    ctx.close()
