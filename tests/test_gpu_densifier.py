"""Densifier kernels (bf16 MFMA convolutions, fp32 accumulation) vs the FP64 oracle of
oracle/nn.py, through the C ABI on a HIP device.

The oracle runs on the same parameters, with the weights the GPU reads in bf16 (the MFMA
convolutions) rounded to bf16 first, so the comparison measures only the kernels' arithmetic:
bf16 activations and gradients through about 30 layers forward and as many backward.

Element-wise bar, from bf16's unit roundoff u = 2^-9 and the network's depth: the oracle is run
again K times with every intermediate tensor of the forward and the backward multiplied by
(1 + delta), delta uniform in [-u, u] per element (oracle forward/backward's q hook).  The
per-element RMS deviation s of those runs is how much each output moves under rounding of bf16
size at every layer; depth and conditioning (LayerNorm, the non-differentiable point of the
normal sine loss, saturated sigmoids) enter through the network itself.  Every element of the
forward outputs, the loss terms and every parameter gradient must satisfy
|gpu - oracle| <= 32 (s + 0.1 rms(s)), and each tensor rms|gpu - oracle| <= 6 rms(s).  The factor
covers that the GPU's rounding is deterministic (equal values round alike, so sums of many equal
terms, such as a bias gradient over saturated pixels, accumulate it coherently) and the sampling
error of s from K runs; measured, the bulk sits at err ~ s (median ratio ~1).

Shapes: 2 images of 16^2 (ragged 32-pixel tiles, flat chunk sums; the 3 x 3 layers of 16-pixel
images on 16 x 8 halo tiles, the smaller ones on the flat k_conv_fwd tiles), and 256^2 -> 512^2
(the densifier's configured resolution): every 3 x 3 layer on k_conv3_halo's 8-row tiles with
64- and 32-channel outputs (three taps per K step), the 1 x 1 layers on 64-pixel k_conv_fwd tiles with 128-
and 32-channel outputs, k_conv_wgrad chunks of 576 pixels (18 K steps per block) with the tree
reduction over 114 chunks; 4 images of 256^2 forward adds the 64 x 64 tile.
"""
import numpy as np
import pytest

import oracle
import scenes
from oracle import nn as N

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import torch
    import paper_2408_15583_amd as pe_mod
    assert torch.cuda.is_available()
    return pe_mod


@pytest.fixture(scope="module")
def ctx(pe):
    c = pe.Context(0)
    yield c
    c.close()


def bf16(a):
    """Round to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mfma_weight(name):
    return name.endswith(".w") and not name.endswith(".dw.w") and name != "stem.w"


def oracle_params(net):
    P = {}
    for k, v in net.get_dict("params").items():
        P[k] = bf16(v) if mfma_weight(k) else v.astype(np.float64)
    return P


def batch(seed, n=2, h=16, w=16):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.2, 1.0, (n, h, w)) * (rng.uniform(size=(n, h, w)) < 0.8)
    dg = rng.uniform(0.2, 0.8, (n, 2 * h, 2 * w))
    ng = rng.normal(size=(n, 2 * h, 2 * w, 3))
    ng[..., 2] = np.abs(ng[..., 2]) + 0.5
    ng /= np.linalg.norm(ng, axis=-1, keepdims=True)
    mg = (rng.uniform(size=(n, 2 * h, 2 * w)) < 0.7).astype(np.float64)
    return x, dg, ng, mg


def to_dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrays]


def test_registry_matches_oracle(pe, ctx):
    net = pe.Densifier(ctx, base=32, seed=1)
    ref = N.init_params(base=32, seed=0)
    got = {n: s for n, _, s in net.tensors()}
    assert set(got) == set(ref)
    for k, v in ref.items():
        assert got[k] == v.shape, k
    net.close()


U_BF16 = 2.0 ** -9
Z_ELEM, Z_RMS = 32.0, 6.0


def oracle_outputs(P, x, dg, ng, mg, q=N._same, grads=True):
    """Forward outputs (depth, unit normal, hit probability), loss terms and gradients."""
    (dp, npr, lp), cache = N.forward(P, x[..., None], q)
    out = dict(d=dp, n=npr / np.linalg.norm(npr, axis=-1, keepdims=True), p=N.sigmoid(lp))
    if grads:
        L, parts, (gd, gn, gl) = N.losses(dp, npr, lp, dg, ng, mg)
        out["loss"] = np.array([L] + list(parts))
        out.update({"G_" + k: v for k, v in N.backward(P, cache, gd, gn, gl, q).items()})
    return out


def rounding_spread(P, x, dg, ng, mg, nom, K, seed, grads=True):
    """Per-element RMS deviation of K oracle runs under bf16-sized relative perturbations of
    every intermediate tensor."""
    rng = np.random.default_rng(seed)

    def q(t):
        return t * (1.0 + rng.uniform(-U_BF16, U_BF16, t.shape))

    acc = {k: np.zeros_like(v) for k, v in nom.items()}
    for _ in range(K):
        e = oracle_outputs(P, x, dg, ng, mg, q, grads)
        for k in acc:
            acc[k] += (e[k] - nom[k]) ** 2
    return {k: np.sqrt(v / K) for k, v in acc.items()}


def check_elementwise(gpu, nom, s, tag):
    worst = []
    for k, o in nom.items():
        g = np.asarray(gpu[k], np.float64).reshape(o.shape)
        err = np.abs(g - o)
        rs = float(np.sqrt((s[k] ** 2).mean()))
        ratio = float((err / (s[k] + 0.1 * rs)).max())
        rms_ratio = float(np.sqrt((err ** 2).mean()) / rs)
        worst.append((ratio, rms_ratio, k))
    worst.sort(reverse=True)
    for r, rr, k in worst[:8]:
        print(f"{tag} {k:18s} max err/(s + 0.1 rms s) {r:6.2f}  rms err / rms s {rr:5.2f}")
    bad = [(k, r, rr) for r, rr, k in worst if not (r <= Z_ELEM and rr <= Z_RMS)]
    assert not bad, bad


def gpu_outputs(net, x, dg, ng, mg, grads=True):
    xd, dgd, ngd, mgd = to_dev(x, dg, ng, mg)
    d, n, p = [t.cpu().numpy() for t in net.infer(xd)]
    out = dict(d=d, n=n, p=p)
    if grads:
        p_before = net.get("params")
        out["loss"] = np.array(net.train_step(xd, dgd, ngd, mgd, lr=0.0))
        out.update({"G_" + k: v for k, v in net.get_dict("grads").items()})
        assert np.array_equal(net.get("params"), p_before)  # lr = 0 leaves them untouched
    return out


@pytest.mark.parametrize("n,h", [(2, 16), (1, 256)])
def test_forward_and_gradients_elementwise(pe, ctx, n, h):
    net = pe.Densifier(ctx, base=32, seed=3)
    P = oracle_params(net)
    x, dg, ng, mg = batch(5, n=n, h=h, w=h)
    gpu = gpu_outputs(net, x, dg, ng, mg)
    net.close()
    nom = oracle_outputs(P, x, dg, ng, mg)
    s = rounding_spread(P, x, dg, ng, mg, nom, K=8, seed=11)
    check_elementwise(gpu, nom, s, f"{n}x{h}^2")


def test_forward_batch4_full_size_elementwise(pe, ctx):
    net = pe.Densifier(ctx, base=32, seed=3)
    P = oracle_params(net)
    x, dg, ng, mg = batch(6, n=4, h=256, w=256)
    gpu = gpu_outputs(net, x, dg, ng, mg, grads=False)
    net.close()
    nom = oracle_outputs(P, x, dg, ng, mg, grads=False)
    s = rounding_spread(P, x, dg, ng, mg, nom, K=6, seed=12, grads=False)
    check_elementwise(gpu, nom, s, "4x256^2 forward")


_SEPARATE_CONVS = """
import sys
import numpy as np
import torch
assert torch.cuda.is_available()
import paper_2408_15583_amd as pe
ctx = pe.Context(0)
net = pe.Densifier(ctx, base=32, seed=1)
g = torch.Generator(device="cpu").manual_seed(0)
x = (torch.rand((2, 256, 256), generator=g) * (torch.rand((2, 256, 256), generator=g) < 0.7)).cuda()
np.savez(sys.argv[1], *[o.cpu().numpy() for o in net.infer(x)])
net.close()
ctx.close()
"""


def test_fused_block_mlp_matches_separate_convolutions(pe, ctx, tmp_path):
    """Inference runs each wide-image ConvNeXt block's two 1 x 1 convolutions as one kernel that
    keeps the hidden activation in LDS; it does the same arithmetic in the same order, so the
    outputs equal those of the two separate convolutions (selected in a child process by
    PE_NN_UNFUSED) bit for bit."""
    import os
    import subprocess
    import sys
    import torch
    net = pe.Densifier(ctx, base=32, seed=1)
    g = torch.Generator(device="cpu").manual_seed(0)
    x = (torch.rand((2, 256, 256), generator=g) * (torch.rand((2, 256, 256), generator=g) < 0.7)).cuda()
    fused = [o.cpu().numpy() for o in net.infer(x)]
    net.close()
    out = tmp_path / "separate.npz"
    env = dict(os.environ, PE_NN_UNFUSED="1")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run([sys.executable, "-c", _SEPARATE_CONVS, str(out)], env=env, cwd=root,
                   check=True, timeout=240)
    sep = np.load(out)
    for i, a in enumerate(fused):
        assert np.array_equal(a, sep[f"arr_{i}"]), f"output {i} differs"


def test_adamw_step_matches_oracle(pe, ctx):
    net = pe.Densifier(ctx, base=32, seed=4)
    x, dg, ng, mg = batch(6)
    xd, dgd, ngd, mgd = to_dev(x, dg, ng, mg)
    net.train_step(xd, dgd, ngd, mgd, lr=0.0)          # step 1 fills the moments
    p0, m0, v0 = net.get("params"), net.get("m"), net.get("v")
    net.train_step(xd, dgd, ngd, mgd, lr=1e-3, weight_decay=0.01)  # step 2
    g = net.get("grads")
    p1 = net.get("params")
    pe_, me, ve = N.adamw_step(p0.astype(np.float64), g.astype(np.float64), m0.astype(np.float64),
                               v0.astype(np.float64), 2, lr=1e-3, wd=0.01)
    assert np.allclose(net.get("m"), me, rtol=1e-5, atol=1e-12)
    assert np.allclose(net.get("v"), ve, rtol=1e-5, atol=1e-15)
    assert np.allclose(p1, pe_, rtol=1e-5, atol=1e-7)
    net.close()


def test_training_is_deterministic_and_checkpoint_resumes(pe, ctx, tmp_path):
    x, dg, ng, mg = batch(7)
    xd, dgd, ngd, mgd = to_dev(x, dg, ng, mg)
    a = pe.Densifier(ctx, base=32, seed=9)
    b = pe.Densifier(ctx, base=32, seed=9)
    la = [a.train_step(xd, dgd, ngd, mgd, lr=1e-3) for _ in range(3)]
    lb = [b.train_step(xd, dgd, ngd, mgd, lr=1e-3) for _ in range(2)]
    path = tmp_path / "ck.bin"
    b.save(path)
    c = pe.Densifier(ctx, base=32, seed=123)
    c.load(path)
    assert np.array_equal(c.get("params"), b.get("params"))
    lc = c.train_step(xd, dgd, ngd, mgd, lr=1e-3)
    assert lc == la[2] and lb[:2] == la[:2]
    assert np.array_equal(c.get("params"), a.get("params"))
    with pytest.raises(pe.PEError):
        pe.Densifier(ctx, base=64, seed=0).load(path)
    for n in (a, b, c):
        n.close()


def test_loss_decreases_on_fixed_batch(pe, ctx):
    net = pe.Densifier(ctx, base=32, seed=2)
    x, dg, ng, mg = batch(8)
    xd, dgd, ngd, mgd = to_dev(x, dg, ng, mg)
    first = net.train_step(xd, dgd, ngd, mgd, lr=2e-3)[0]
    for _ in range(40):
        last = net.train_step(xd, dgd, ngd, mgd, lr=2e-3)[0]
    assert last < 0.7 * first, (first, last)
    net.close()


def test_make_pair_matches_oracle_buffers(pe, ctx):
    sc = scenes.dihedral()
    s = pe.Scene.from_scene(ctx, sc, view_res=64)
    o = oracle.OracleScene(sc, grid=64)
    c, R = o.frame()
    D = 2 * R
    az = np.deg2rad(30.0)
    k = -np.array([np.cos(az), np.sin(az), 0.2])
    k /= np.linalg.norm(k)
    h = w = 32
    coarse, dgt, ngt, mgt = [t.cpu().numpy()[0] for t in pe.make_pair(ctx, s, k[None], h, w,
                                                                        tube_px=2.0)]
    # targets vs the oracle DISK buffer at 2h x 2w
    dep, idx, nrm, mask = o.render_disk(k, 2 * w, 2 * h)
    agree = (mgt > 0.5) == (mask > 0)
    assert agree.mean() >= 0.999
    both = (mgt > 0.5) & (mask > 0)
    assert np.abs(dgt[both] * D - dep[both]).max() <= 1e-5 * D
    _, du, dv = o.screen(k, 2 * w, 2 * h)
    u, v = du / np.linalg.norm(du), dv / np.linalg.norm(dv)
    nv = np.stack([nrm @ u, nrm @ v, -(nrm @ k)], axis=-1)
    assert np.abs(ngt[both] - nv[both]).max() < 1e-4
    # coarse input vs the oracle TUBE buffer at h x w
    pitch = D / w
    tdep, tidx = o.render_tube(k, w, h, 2.0 * pitch)
    thit = tidx >= 0
    ghit = coarse > 0
    assert (thit == ghit).mean() >= 0.99
    bb = thit & ghit
    assert np.abs((1 - coarse[bb]) * D - tdep[bb]).max() <= 1e-5 * D
    # with the K-point heap of Algorithm 1 (K = 4): vs the oracle's heap buffer; fp32 and fp64
    # may break near-ties between candidates differently, so depths agree on >= 99 % of hits
    c4 = pe.make_pair(ctx, s, k[None], h, w, tube_px=2.0, tube_k=4)[0].cpu().numpy()[0]
    kdep, kidx = o.render_tube_topk(k, w, h, 2.0 * pitch, 4)[:2]
    khit, g4 = kidx >= 0, c4 > 0
    assert (khit == g4).mean() >= 0.99
    bb = khit & g4
    assert (np.abs((1 - c4[bb]) * D - kdep[bb]) <= 1e-5 * D).mean() >= 0.99
    s.close()


def test_coarse_and_densified_geometry_run(pe, ctx):
    sc = scenes.plate()
    s = pe.Scene.from_scene(ctx, sc, view_res=64)
    k = np.array([[-1.0, 0.0, 0.0]])  # broadside: the plate lies on x = 0
    f = np.array([10e9])
    _, r_plain, _ = pe.solve(ctx, s, k, f, 128)
    _, r_coarse, st_c = pe.solve(ctx, s, k, f, 128, geometry="coarse")
    assert abs(r_coarse[0, 0, 0, 0, 0] - r_plain[0, 0, 0, 0, 0]) < 1.0
    net = pe.Densifier(ctx, base=32, seed=0)
    E, r_d, st_d = pe.solve(ctx, s, k, f, 128, densifier=net)
    assert np.isfinite(E).all()
    assert st_d["densifier_fallbacks"] in (0.0, 1.0)
    with pytest.raises(pe.PEError):
        pe.solve(ctx, s, k, f, 128, max_bounces=2, geometry="coarse")
    with pytest.raises(pe.PEError):
        pe.solve(ctx, s, k, f, 120, densifier=net)
    net.close()
    s.close()
