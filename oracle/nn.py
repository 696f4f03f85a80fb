"""FP64 reference of the learned densifier -- TEST INFRASTRUCTURE ONLY.

Plain NumPy definitions of every layer the densifier uses, with hand-written backward passes,
and the training losses of Sec. III-A, Eq. (17)-(21).  Only tests use this module; the HIP
library never imports it.  Layout: NHWC activations, convolution weights [Cout][KH][KW][Cin].

Network (a reading of Fig. 2/3, whose drawings are not in the text): a U-Net whose encoder
uses ConvNeXt blocks (depthwise 7x7, LayerNorm over channels, 1x1 expand x4, GELU, 1x1
project, residual), max-pooling down, sub-pixel convolution (conv + pixel shuffle) up, one
shared encoder and three decoder heads (depth, normal, hit logit) -- the time complexity
M1 (L_e + 3 L_d) of Sec. III-C counts three decoders.  Outputs are at twice the input size.

The depth output is the coarse depth 1 - x of the input pixel the output pixel lies in (0
where the input is empty) plus the depth head's value in units of one input pixel pitch
(t/D per pitch = 1 / max(H, W) for a screen of side D): the head learns a correction of a few
pixels at unit scale, which keeps the bf16 activations of the HIP network precise to a small
fraction of a pixel of depth.  (The paper does not state how the depth head is parametrised.)

Losses (Eq. (17)-(21)): L1 depth squared error (mean over target hits), L2 sine of the angle
between predicted and target normals (mean over target hits), L3 alpha-balanced focal loss on
the hit probability (alpha = 0.5, gamma = 2, mean over all pixels), L4 sine of the angle between
the depth-gradient normals (-du, -dv, 1) of prediction and target (mean over target pixels whose
right and lower neighbours are hits), L = L1 + 0.5 L2 + L3 + 0.5 L4.

Pins: tests/test_oracle_nn.py (finite differences of every backward, explicit-loop convolution,
closed-form special cases of the losses).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

LAMBDAS = (1.0, 0.5, 1.0, 0.5)   # Eq. (21)
FOCAL_ALPHA = 0.5                # Eq. (19)
FOCAL_GAMMA = 2.0
LN_EPS = 1e-6


# ------------------------------------------------------------------------------ convolution --

def _pad(x, p):
    return np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))


def conv2d(x, w, b=None):
    """Stride 1, zero padding (K-1)/2.  y[n,i,j,o] = sum_{a,c,ci} x[n,i+a-p,j+c-p,ci] w[o,a,c,ci]."""
    N, H, W, Ci = x.shape
    Co, KH, KW, _ = w.shape
    p = (KH - 1) // 2
    xp = _pad(x, p)
    y = np.zeros((N, H, W, Co))
    for a in range(KH):
        for c in range(KW):  # one tap: a (pixels x Ci) by (Ci x Co) product
            xs = xp[:, a:a + H, c:c + W, :].reshape(-1, Ci)
            y += (xs @ w[:, a, c, :].T).reshape(N, H, W, Co)
    if b is not None:
        y += b
    return y


def conv2d_backward(x, w, dy):
    N, H, W, Ci = x.shape
    Co, KH, KW, _ = w.shape
    p = (KH - 1) // 2
    xp = _pad(x, p)
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    d2 = dy.reshape(-1, Co)
    for a in range(KH):
        for c in range(KW):
            dw[:, a, c, :] = d2.T @ xp[:, a:a + H, c:c + W, :].reshape(-1, Ci)
            dxp[:, a:a + H, c:c + W, :] += (d2 @ w[:, a, c, :]).reshape(N, H, W, Ci)
    dx = dxp[:, p:p + H, p:p + W, :]
    db = dy.sum(axis=(0, 1, 2))
    return dx, dw, db


def dwconv(x, w, b):
    """Depthwise KxK (per channel), zero padding (K-1)/2.  w [C][K][K]."""
    N, H, W, C = x.shape
    K = w.shape[1]
    p = (K - 1) // 2
    xp = _pad(x, p)
    y = np.zeros_like(x)
    for a in range(K):
        for c in range(K):
            y += xp[:, a:a + H, c:c + W, :] * w[:, a, c]
    return y + b


def dwconv_backward(x, w, dy):
    N, H, W, C = x.shape
    K = w.shape[1]
    p = (K - 1) // 2
    xp = _pad(x, p)
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for a in range(K):
        for c in range(K):
            dw[:, a, c] = np.einsum("nhwc,nhwc->c", dy, xp[:, a:a + H, c:c + W, :])
            dxp[:, a:a + H, c:c + W, :] += dy * w[:, a, c]
    return dxp[:, p:p + H, p:p + W, :], dw, dy.sum(axis=(0, 1, 2))


# ------------------------------------------------------------------------- normalisation --

def layernorm(x, g, b, eps=LN_EPS):
    """Over the channel axis of each pixel; returns y and the cache for backward."""
    mu = x.mean(-1, keepdims=True)
    var = ((x - mu) ** 2).mean(-1, keepdims=True)
    rstd = 1.0 / np.sqrt(var + eps)
    xh = (x - mu) * rstd
    return xh * g + b, (xh, rstd)


def layernorm_backward(cache, g, dy):
    xh, rstd = cache
    C = xh.shape[-1]
    dxh = dy * g
    dx = rstd * (dxh - dxh.mean(-1, keepdims=True) - xh * (dxh * xh).mean(-1, keepdims=True))
    return dx, (dy * xh).sum(axis=(0, 1, 2)), dy.sum(axis=(0, 1, 2))


# ---------------------------------------------------------------------------- activations --

_erf = special.erf


def gelu(x):
    """Exact GELU, x Phi(x)."""
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_backward(x, dy):
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return dy * (cdf + x * pdf)


def sigmoid(x):
    return special.expit(x)


# ------------------------------------------------------------------------ resampling --

def maxpool2(x):
    """2x2 max pooling, stride 2; ties keep the first element in (0,0),(0,1),(1,0),(1,1) order."""
    N, H, W, C = x.shape
    blocks = x.reshape(N, H // 2, 2, W // 2, 2, C).transpose(0, 1, 3, 5, 2, 4).reshape(
        N, H // 2, W // 2, C, 4)
    arg = blocks.argmax(-1)
    return blocks.max(-1), arg


def maxpool2_backward(arg, dy, shape):
    N, H, W, C = shape
    d = np.zeros((N, H // 2, W // 2, C, 4))
    np.put_along_axis(d, arg[..., None], dy[..., None], axis=-1)
    return d.reshape(N, H // 2, W // 2, C, 2, 2).transpose(0, 1, 4, 2, 5, 3).reshape(N, H, W, C)


def pixel_shuffle(x):
    """[N,H,W,4C] -> [N,2H,2W,C]; input channel c*4 + 2*dy + dx goes to pixel (2i+dy, 2j+dx)."""
    N, H, W, C4 = x.shape
    C = C4 // 4
    return x.reshape(N, H, W, C, 2, 2).transpose(0, 1, 4, 2, 5, 3).reshape(N, 2 * H, 2 * W, C)


def pixel_unshuffle(y):
    N, H2, W2, C = y.shape
    return y.reshape(N, H2 // 2, 2, W2 // 2, 2, C).transpose(0, 1, 3, 5, 2, 4).reshape(
        N, H2 // 2, W2 // 2, 4 * C)


# --------------------------------------------------------------------------------- losses --

def losses(depth, nrm, logit, depth_gt, nrm_gt, mask_gt):
    """Eq. (17)-(21) on [N,H,W] maps (nrm: [N,H,W,3]).  Returns (L, (L1, L2, L3, L4), grads)
    with grads = (d depth, d nrm, d logit)."""
    m = mask_gt.astype(np.float64)
    nv = max(m.sum(), 1.0)
    # L1: squared depth error over target hits
    e = depth - depth_gt
    L1 = (m * e * e).sum() / nv
    g_depth = 2.0 * m * e / nv
    # L2: |n_p x n_g| / (|n_p| |n_g|) over target hits
    cr = np.cross(nrm, nrm_gt)
    crn = np.linalg.norm(cr, axis=-1)
    npn = np.linalg.norm(nrm, axis=-1)
    ngn = np.linalg.norm(nrm_gt, axis=-1)
    den = np.maximum(npn * ngn, 1e-12)
    s = crn / den
    L2 = (m * s).sum() / nv
    # d s / d n_p: s = |c|/(|p||g|), c = p x g
    with np.errstate(invalid="ignore", divide="ignore"):
        u = np.where(crn[..., None] > 0, cr / np.maximum(crn, 1e-30)[..., None], 0.0)
    dcrn_dp = np.cross(nrm_gt, u)  # d|p x g|/dp = g x (c/|c|)
    ds_dp = dcrn_dp / den[..., None] - (s / np.maximum(npn, 1e-30) ** 2)[..., None] * nrm
    g_nrm = (m / nv)[..., None] * ds_dp
    # L3: alpha-balanced focal loss over all pixels (Eq. (19)), with h, 1 - h and their logs
    # taken from the logit itself so that saturated logits keep their exact value
    h, hb = sigmoid(logit), sigmoid(-logit)
    lh, l1h = -np.logaddexp(0.0, -logit), -np.logaddexp(0.0, logit)  # log h, log(1 - h)
    a, gm = FOCAL_ALPHA, FOCAL_GAMMA
    pos = -a * hb ** gm * lh
    neg = -(1 - a) * h ** gm * l1h
    l3 = np.where(mask_gt > 0, pos, neg)
    L3 = l3.mean()
    # d/dlogit, using dh/dlogit = h (1 - h)
    dpos = a * hb ** gm * (gm * h * lh - hb)
    dneg = (1 - a) * h ** gm * (h - gm * hb * l1h)
    g_logit = np.where(mask_gt > 0, dpos, dneg) / l3.size
    # L4: depth-gradient normals (-du, -dv, 1), forward differences, pixels whose right and
    # lower neighbours are also target hits
    N, H, W = depth.shape
    valid = m[:, :-1, :-1] * m[:, 1:, :-1] * m[:, :-1, 1:]
    nv4 = max(valid.sum(), 1.0)

    def grad_nrm(d):
        du = d[:, :-1, 1:] - d[:, :-1, :-1]
        dv = d[:, 1:, :-1] - d[:, :-1, :-1]
        return np.stack([-du, -dv, np.ones_like(du)], axis=-1)

    Pp = grad_nrm(depth)
    Pg = grad_nrm(depth_gt)
    c4 = np.cross(Pp, Pg)
    c4n = np.linalg.norm(c4, axis=-1)
    ppn = np.linalg.norm(Pp, axis=-1)
    pgn = np.linalg.norm(Pg, axis=-1)
    s4 = c4n / (ppn * pgn)
    L4 = (valid * s4).sum() / nv4
    with np.errstate(invalid="ignore", divide="ignore"):
        u4 = np.where(c4n[..., None] > 0, c4 / np.maximum(c4n, 1e-30)[..., None], 0.0)
    ds4 = np.cross(Pg, u4) / (ppn * pgn)[..., None] - (s4 / ppn ** 2)[..., None] * Pp
    w4 = (valid / nv4)[..., None] * ds4  # d L4 / d Pp
    g4 = np.zeros_like(depth)
    # Pp = (-(d[i,j+1]-d[i,j]), -(d[i+1,j]-d[i,j]), 1)
    g4[:, :-1, 1:] += -w4[..., 0]
    g4[:, :-1, :-1] += w4[..., 0]
    g4[:, 1:, :-1] += -w4[..., 1]
    g4[:, :-1, :-1] += w4[..., 1]
    l1, l2, l3w, l4 = LAMBDAS
    L = l1 * L1 + l2 * L2 + l3w * L3 + l4 * L4
    grads = (l1 * g_depth + l4 * g4, l2 * g_nrm, l3w * g_logit)
    return L, (L1, L2, L3, L4), grads


# ---------------------------------------------------------------------------- the network --

def init_params(base=8, seed=0, in_ch=1):
    """Parameter dict of the U-Net with channels base, 2, 4, 8 x base.  Weights ~ N(0, 2/fan_in)."""
    rng = np.random.default_rng(seed)
    C = [base, 2 * base, 4 * base, 8 * base]
    P = {}

    def conv(name, co, k, ci):
        P[name + ".w"] = rng.normal(0, math.sqrt(2.0 / (k * k * ci)), (co, k, k, ci))
        P[name + ".b"] = rng.normal(0, 0.01, co)

    def block(name, c):
        P[name + ".dw.w"] = rng.normal(0, math.sqrt(2.0 / 49), (c, 7, 7))
        P[name + ".dw.b"] = rng.normal(0, 0.01, c)
        P[name + ".ln.g"] = 1.0 + rng.normal(0, 0.05, c)
        P[name + ".ln.b"] = rng.normal(0, 0.05, c)
        conv(name + ".pw1", 4 * c, 1, c)
        conv(name + ".pw2", c, 1, 4 * c)

    conv("stem", C[0], 3, in_ch)
    block("enc0", C[0])
    for l in range(1, 4):
        conv(f"down{l}", C[l], 1, C[l - 1])
        block(f"enc{l}", C[l])
    for head, co in (("depth", 1), ("nrm", 3), ("mask", 1)):
        for l in (3, 2, 1):
            conv(f"{head}.up{l}", 4 * C[l - 1], 3, C[l])
            conv(f"{head}.fuse{l}", C[l - 1], 3, 2 * C[l - 1])
        conv(f"{head}.out", 4 * co, 3, C[0])
    return P


def _same(t):
    return t


def _block_fwd(P, name, x, q=_same):
    c = {}
    c["x"] = x
    c["dw"] = q(dwconv(x, P[name + ".dw.w"], P[name + ".dw.b"]))
    ln, c["lnc"] = layernorm(c["dw"], P[name + ".ln.g"], P[name + ".ln.b"])
    c["ln"] = q(ln)
    c["z1"] = q(conv2d(c["ln"], P[name + ".pw1.w"], P[name + ".pw1.b"]))
    c["a1"] = q(gelu(c["z1"]))
    y = q(x + conv2d(c["a1"], P[name + ".pw2.w"], P[name + ".pw2.b"]))
    return y, c


def _block_bwd(P, name, c, dy, G, q=_same):
    da1, G[name + ".pw2.w"], G[name + ".pw2.b"] = conv2d_backward(c["a1"], P[name + ".pw2.w"], dy)
    dz1 = q(gelu_backward(c["z1"], q(da1)))
    dln, G[name + ".pw1.w"], G[name + ".pw1.b"] = conv2d_backward(c["ln"], P[name + ".pw1.w"], dz1)
    ddw, G[name + ".ln.g"], G[name + ".ln.b"] = layernorm_backward(c["lnc"], P[name + ".ln.g"],
                                                                   q(dln))
    dx, G[name + ".dw.w"], G[name + ".dw.b"] = dwconv_backward(c["x"], P[name + ".dw.w"], q(ddw))
    return q(q(dx) + dy)


def forward(P, x, q=_same):
    """x [N,H,W,in_ch] -> (depth [N,2H,2W], nrm [N,2H,2W,3], logit [N,2H,2W]), cache.

    q is applied to every intermediate tensor (identity by default): a test passes a random
    relative perturbation of rounding size to measure how each output responds to rounding at
    every layer (the conditioning of the network at that input)."""
    cache = {}
    z = q(conv2d(x, P["stem.w"], P["stem.b"]))
    cache["x"] = x
    cache["stem_z"] = z
    a = q(gelu(z))
    skips = []
    h, cache["enc0"] = _block_fwd(P, "enc0", a, q)
    skips.append(h)
    for l in range(1, 4):
        p, arg = maxpool2(h)
        cache[f"pool{l}"] = (arg, h.shape, p)
        d = q(conv2d(p, P[f"down{l}.w"], P[f"down{l}.b"]))
        h, cache[f"enc{l}"] = _block_fwd(P, f"enc{l}", d, q)
        cache[f"down{l}_in"] = p
        skips.append(h)
    outs = {}
    for head in ("depth", "nrm", "mask"):
        hc = {}
        u = skips[3]
        for l in (3, 2, 1):
            zu = q(conv2d(u, P[f"{head}.up{l}.w"], P[f"{head}.up{l}.b"]))
            sh = pixel_shuffle(zu)
            cat = np.concatenate([sh, skips[l - 1]], axis=-1)
            zf = q(conv2d(cat, P[f"{head}.fuse{l}.w"], P[f"{head}.fuse{l}.b"]))
            hc[l] = (u, cat, zf)
            u = q(gelu(zf))
        zo = q(conv2d(u, P[f"{head}.out.w"], P[f"{head}.out.b"]))
        hc["out_in"] = u
        outs[head] = pixel_shuffle(zo)
        cache["head_" + head] = hc
    cache["skips"] = skips
    # the depth head predicts a correction to the coarse depth t/D = 1 - x (0 where the coarse
    # buffer is empty), repeated over each 2 x 2 block of output pixels
    x0 = x[..., 0]
    base = np.where(x0 > 0, 1.0 - x0, 0.0).repeat(2, axis=1).repeat(2, axis=2)
    scale = depth_scale(x)
    return (outs["depth"][..., 0] * scale + base, outs["nrm"], outs["mask"][..., 0]), cache


def depth_scale(x):
    """t/D of one input pixel pitch: the unit of the depth head."""
    return 1.0 / max(x.shape[1], x.shape[2])


def backward(P, cache, d_depth, d_nrm, d_logit, q=_same):
    """Parameter gradients from the output gradients; q as in forward, on every intermediate
    gradient (not on the parameter gradients themselves)."""
    G = {}
    skips = cache["skips"]
    dskips = [np.zeros_like(s) for s in skips]
    sc = depth_scale(cache["x"])
    for head, dout in (("depth", sc * d_depth[..., None]), ("nrm", d_nrm),
                       ("mask", d_logit[..., None])):
        hc = cache["head_" + head]
        dzo = q(pixel_unshuffle(dout))
        du, G[f"{head}.out.w"], G[f"{head}.out.b"] = conv2d_backward(hc["out_in"], P[f"{head}.out.w"], dzo)
        for l in (1, 2, 3):
            u_in, cat, zf = hc[l]
            dzf = q(gelu_backward(zf, q(du)))
            dcat, G[f"{head}.fuse{l}.w"], G[f"{head}.fuse{l}.b"] = conv2d_backward(cat, P[f"{head}.fuse{l}.w"], dzf)
            dcat = q(dcat)
            cs = dcat.shape[-1] // 2
            dsh, dskip = dcat[..., :cs], dcat[..., cs:]
            dskips[l - 1] += dskip
            dzu = pixel_unshuffle(dsh)
            du, G[f"{head}.up{l}.w"], G[f"{head}.up{l}.b"] = conv2d_backward(u_in, P[f"{head}.up{l}.w"], dzu)
        dskips[3] += q(du)
    dh = q(dskips[3])
    for l in (3, 2, 1):
        dd = _block_bwd(P, f"enc{l}", cache[f"enc{l}"], dh, G, q)
        dp, G[f"down{l}.w"], G[f"down{l}.b"] = conv2d_backward(cache[f"down{l}_in"], P[f"down{l}.w"], dd)
        arg, shape, _ = cache[f"pool{l}"]
        dh = q(maxpool2_backward(arg, q(dp), shape) + dskips[l - 1])
    da = _block_bwd(P, "enc0", cache["enc0"], dh, G, q)
    dz = q(gelu_backward(cache["stem_z"], da))
    _, G["stem.w"], G["stem.b"] = conv2d_backward(cache["x"], P["stem.w"], dz)
    return G


def adamw_step(p, g, m, v, t, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
    """Decoupled weight decay (the AdamW optimiser of Sec. IV-A's training recipe)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v
