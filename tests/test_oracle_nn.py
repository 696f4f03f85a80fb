"""Pins of the FP64 densifier oracle (CPU): finite differences of every backward pass, an
explicit-loop convolution, PyTorch CPU as an independent implementation of convolution and
pixel shuffle, and closed-form special cases of the losses of Eq. (17)-(21)."""
import math

import numpy as np
import pytest

from oracle import nn as N


def fd_check(f, x, analytic, n=12, h=1e-6, rtol=1e-5, seed=0):
    rng = np.random.default_rng(seed)
    flat = x.reshape(-1)
    idx = rng.choice(flat.size, size=min(n, flat.size), replace=False)
    for i in idx:
        old = flat[i]
        flat[i] = old + h
        fp = f()
        flat[i] = old - h
        fm = f()
        flat[i] = old
        num = (fp - fm) / (2 * h)
        a = analytic.reshape(-1)[i]
        assert abs(num - a) <= rtol * max(1.0, abs(num), abs(a)), (i, num, a)


def test_conv2d_explicit_loop():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 5, 4, 3))
    w = rng.normal(size=(2, 3, 3, 3))
    b = rng.normal(size=2)
    y = N.conv2d(x, w, b)
    for i in range(5):
        for j in range(4):
            for o in range(2):
                s = b[o]
                for a in range(3):
                    for c in range(3):
                        ii, jj = i + a - 1, j + c - 1
                        if 0 <= ii < 5 and 0 <= jj < 4:
                            s += np.dot(x[0, ii, jj], w[o, a, c])
                assert abs(y[0, i, j, o] - s) < 1e-12


def test_conv2d_matches_torch_cpu():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 6, 7, 4))
    w = rng.normal(size=(5, 3, 3, 4))
    b = rng.normal(size=5)
    y = N.conv2d(x, w, b)
    yt = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2),
                                    torch.from_numpy(w).permute(0, 3, 1, 2),
                                    torch.from_numpy(b), padding=1).permute(0, 2, 3, 1).numpy()
    assert np.allclose(y, yt, atol=1e-12)


def test_pixel_shuffle_matches_torch_cpu():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(3).normal(size=(2, 3, 4, 8))
    y = N.pixel_shuffle(x)
    yt = torch.nn.functional.pixel_shuffle(torch.from_numpy(x).permute(0, 3, 1, 2), 2)
    assert np.array_equal(y, yt.permute(0, 2, 3, 1).numpy())
    assert np.array_equal(N.pixel_unshuffle(y), x)


def test_conv2d_backward_fd():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(1, 5, 6, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    R = rng.normal(size=(1, 5, 6, 4))
    dx, dw, db = N.conv2d_backward(x, w, R)
    f = lambda: (N.conv2d(x, w, b) * R).sum()
    fd_check(f, x, dx)
    fd_check(f, w, dw)
    fd_check(f, b, db)


def test_dwconv_backward_fd():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(1, 8, 9, 3))
    w = rng.normal(size=(3, 7, 7))
    b = rng.normal(size=3)
    R = rng.normal(size=x.shape)
    dx, dw, db = N.dwconv_backward(x, w, R)
    f = lambda: (N.dwconv(x, w, b) * R).sum()
    fd_check(f, x, dx)
    fd_check(f, w, dw)
    fd_check(f, b, db)


def test_layernorm_and_backward():
    rng = np.random.default_rng(6)
    x = rng.normal(2.0, 3.0, size=(1, 3, 4, 8))
    g = rng.normal(1, 0.1, size=8)
    b = rng.normal(0, 0.1, size=8)
    y, _ = N.layernorm(x, np.ones(8), np.zeros(8))
    assert np.allclose(y.mean(-1), 0, atol=1e-12)
    assert np.allclose(y.var(-1), 1, atol=1e-5)
    R = rng.normal(size=x.shape)
    _, cache = N.layernorm(x, g, b)
    dx, dg, db = N.layernorm_backward(cache, g, R)
    f = lambda: (N.layernorm(x, g, b)[0] * R).sum()
    fd_check(f, x, dx)
    fd_check(f, g, dg)
    fd_check(f, b, db)


def test_gelu_and_backward():
    x = np.linspace(-4, 4, 41)
    assert abs(N.gelu(np.array([0.0]))[0]) == 0
    assert abs(N.gelu(np.array([10.0]))[0] - 10) < 1e-12
    ref = 0.5 * x * (1 + np.array([math.erf(v / math.sqrt(2)) for v in x]))
    assert np.allclose(N.gelu(x), ref)
    R = np.random.default_rng(7).normal(size=x.shape)
    fd_check(lambda: (N.gelu(x) * R).sum(), x, N.gelu_backward(x, R), n=41)


def test_maxpool_backward_fd():
    rng = np.random.default_rng(8)
    x = rng.normal(size=(1, 6, 4, 3))
    y, arg = N.maxpool2(x)
    assert y[0, 0, 0, 0] == x[0, :2, :2, 0].max()
    R = rng.normal(size=y.shape)
    dx = N.maxpool2_backward(arg, R, x.shape)
    fd_check(lambda: (N.maxpool2(x)[0] * R).sum(), x, dx, n=30, h=1e-7)


def _loss_inputs(seed, H=6, W=7):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.2, 0.8, (2, H, W))
    n = rng.normal(size=(2, H, W, 3))
    lg = rng.normal(size=(2, H, W))
    dg = rng.uniform(0.2, 0.8, (2, H, W))
    ng = rng.normal(size=(2, H, W, 3))
    ng /= np.linalg.norm(ng, axis=-1, keepdims=True)
    mg = (rng.uniform(size=(2, H, W)) < 0.7).astype(np.float64)
    return d, n, lg, dg, ng, mg


def test_losses_backward_fd():
    d, n, lg, dg, ng, mg = _loss_inputs(9)
    L, parts, (gd, gn, gl) = N.losses(d, n, lg, dg, ng, mg)
    f = lambda: N.losses(d, n, lg, dg, ng, mg)[0]
    fd_check(f, d, gd, n=30)
    fd_check(f, n, gn, n=30)
    fd_check(f, lg, gl, n=30)
    l1, l2, l3, l4 = N.LAMBDAS
    assert abs(L - (l1 * parts[0] + l2 * parts[1] + l3 * parts[2] + l4 * parts[3])) < 1e-12
    assert (l1, l2, l3, l4) == (1.0, 0.5, 1.0, 0.5)


def test_losses_special_cases():
    d, n, lg, dg, ng, mg = _loss_inputs(10)
    # identical geometry: depth, normal and gradient terms vanish
    L, parts, _ = N.losses(dg.copy(), 2.5 * ng, lg, dg, ng, mg)
    assert parts[0] == 0 and parts[1] < 1e-12 and parts[3] < 1e-12
    # perpendicular normals: sine = 1
    perp = np.cross(ng, np.array([0.3, -0.5, 0.8]))
    L, parts, _ = N.losses(dg, perp, lg, dg, ng, np.ones_like(mg))
    assert abs(parts[1] - 1.0) < 1e-12
    # focal with gamma = 0 is alpha-balanced cross-entropy: 0.5 * BCE at alpha = 0.5
    old = N.FOCAL_GAMMA
    try:
        N.FOCAL_GAMMA = 0.0
        _, parts, _ = N.losses(d, n, lg, dg, ng, mg)
        h = 1.0 / (1.0 + np.exp(-lg))
        bce = -(mg * np.log(h) + (1 - mg) * np.log(1 - h)).mean()
        assert abs(parts[2] - 0.5 * bce) < 1e-12
    finally:
        N.FOCAL_GAMMA = old


def test_focal_loss_saturated_logits():
    """Eq. (19) at logits far beyond where 1 - h underflows: the loss of a wrong confident
    prediction grows like (1 - alpha) |logit| (and alpha |logit| for a missed hit), with slope
    1 - alpha (alpha); a right confident prediction costs nothing."""
    one = np.ones((1, 1, 1))
    z = np.zeros((1, 1, 1))
    nrm, ng = np.ones((1, 1, 1, 3)), np.ones((1, 1, 1, 3))
    for lg, m, loss, slope in ((40.0, 0.0, 0.5 * 40.0, 0.5), (-60.0, 1.0, 0.5 * 60.0, -0.5),
                               (40.0, 1.0, 0.0, 0.0), (-60.0, 0.0, 0.0, 0.0)):
        _, parts, (_, _, gl) = N.losses(0.5 * one, nrm, lg * one, 0.5 * one, ng, m * one)
        assert abs(parts[2] - loss) < 1e-12, (lg, m, parts[2])
        assert abs(gl[0, 0, 0] - slope) < 1e-12, (lg, m, gl[0, 0, 0])


def test_network_backward_fd():
    rng = np.random.default_rng(11)
    P = N.init_params(base=4, seed=1)
    x = rng.uniform(0, 1, (1, 16, 16, 1))
    d_t, n_t, l_t = rng.normal(size=(1, 32, 32)), rng.normal(size=(1, 32, 32, 3)), rng.normal(size=(1, 32, 32))
    (dp, npr, lp), cache = N.forward(P, x)
    assert dp.shape == (1, 32, 32) and npr.shape == (1, 32, 32, 3) and lp.shape == (1, 32, 32)
    G = N.backward(P, cache, d_t, n_t, l_t)
    assert set(G) == set(P)

    def f():
        (a, b, c), _ = N.forward(P, x)
        return (a * d_t).sum() + (b * n_t).sum() + (c * l_t).sum()

    for name in ["stem.w", "enc0.dw.w", "enc0.ln.g", "enc1.pw1.w", "enc3.pw2.b", "down2.w",
                 "depth.up3.w", "nrm.fuse1.w", "mask.out.b", "depth.fuse2.b"]:
        fd_check(f, P[name], G[name], n=4, h=1e-5, rtol=1e-5)


def test_adamw_first_step():
    """First AdamW step moves each weight by lr * (sign(g) + wd * p) (bias-corrected moments)."""
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 2.0])
    p2, m, v = N.adamw_step(p, g, np.zeros(3), np.zeros(3), 1, lr=1e-3, wd=0.01)
    assert np.allclose(p2, p - 1e-3 * (np.sign(g) * (np.abs(g) / (np.abs(g) + 1e-8)) + 0.01 * p))


@pytest.mark.parametrize("bias", [0.0, 1.5])
def test_depth_output_is_coarse_depth_plus_head(bias):
    """With the depth head's last convolution reduced to a bias b, the depth output is the
    coarse depth 1 - x of the input pixel each output pixel lies in (0 where the input is
    empty) plus b input-pixel pitches of depth, b / max(H, W) in t/D (here 8 x 16 inputs)."""
    rng = np.random.default_rng(12)
    P = N.init_params(base=4, seed=3)
    P["depth.out.w"][:] = 0.0
    P["depth.out.b"][:] = bias
    x = rng.uniform(0.1, 1.0, (2, 8, 16, 1)) * (rng.uniform(size=(2, 8, 16, 1)) < 0.7)
    (d, _, _), _ = N.forward(P, x)
    for n in range(2):
        for i in range(16):
            for j in range(32):
                v = x[n, i // 2, j // 2, 0]
                assert d[n, i, j] == pytest.approx((1.0 - v if v > 0 else 0.0) + bias / 16.0,
                                                   abs=1e-15)
