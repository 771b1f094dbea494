"""FP64 reference of the learned upsampler (the network that turns a
half-resolution, one-level-coarser render into the full-resolution frame).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only tests, the smoke
check and the benchmark's CPU-baseline leg use it; the GPU library neither
imports it nor shares code with it.

The paper reduces the rays cast per frame by rendering in a cheaper space and
resampling (Sec 5.3, wrapped space); here the cheaper render is half the
resolution at the next pyramid level and the resampling is learned. Every
operation is written out from its definition in double precision:

* input x0 [N, H, W, 8]: premultiplied R, G, B, alpha, a depth code, zeros;
* conv3x3 with zero padding, weights w[tap = 3 dy + dx][c_in][c_out];
* h1 = relu(conv(x0)), h2 = relu(conv(h1)), h3 = relu(conv(h2)),
  o = conv(h3) (20 used channels of 32);
* full-resolution pixel (2y + sy, 2x + sx) takes the five channels
  o[y, x, 5 s .. 5 s + 4] with s = 2 sy + sx (pixel shuffle): four colour
  residuals added to the bilinear upsampling of x0's colour, and z, whose
  square predicts the pixel's squared RGB error;
* bilinear upsampling by two with half-pixel centres: full-resolution pixel
  X samples low-resolution coordinate (X + 1/2) / 2 - 1/2, edges clamped.

At inference (``forward(..., skip_empty=True)``) a low-resolution pixel
whose 9 x 9 neighbourhood of x0 (the network's receptive field: four stacked
3 x 3 convolutions; pixels outside the image count as zero) holds no nonzero
value yields background: rgba 0 at its four full-resolution pixels and a
predicted error of 0. Its bilinear base is 0 anyway (the base reads the
1-pixel ring); only the network's constant response to an empty input is
dropped. Training evaluates the network everywhere.

``loss_and_grads`` gives the training loss (mean squared RGBA error plus the
error head's mean squared error against the actual per-pixel RMS RGB error,
held constant) and its gradients by backpropagation written out step by
step. Pinned in tests against scipy's correlation, explicit loops and
central finite differences.
"""
from __future__ import annotations

import numpy as np

C_IN, C_HID, C_OUT, C_USED = 8, 32, 32, 20
LAYERS = ((C_IN, C_HID), (C_HID, C_HID), (C_HID, C_HID), (C_HID, C_OUT))
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]  # tap t = 3 (dy+1) + (dx+1)


def conv3x3(x, w, b):
    """y[n, y, x, co] = b[co] + sum_t sum_ci x[n, y+dy_t, x+dx_t, ci] w[t, ci, co],
    x outside the image taken as 0."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci), dtype=np.float64)
    xp[:, 1:H + 1, 1:W + 1] = x
    out = np.broadcast_to(np.asarray(b, np.float64), (N, H, W, w.shape[2])).copy()
    for t, (dy, dx) in enumerate(TAPS):
        out += xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W] @ w[t]
    return out


def conv3x3_input_grad(g, w):
    """d/dx of sum(g * conv3x3(x, w, b)): each output gradient flows back
    through every tap to the input pixel it read."""
    N, H, W, Co = g.shape
    dxp = np.zeros((N, H + 2, W + 2, w.shape[1]), dtype=np.float64)
    for t, (dy, dx) in enumerate(TAPS):
        dxp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W] += g @ w[t].T
    return dxp[:, 1:H + 1, 1:W + 1]


def conv3x3_weight_grad(x, g):
    """d/dw of sum(g * conv3x3(x, w, b)) (and d/db)."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci), dtype=np.float64)
    xp[:, 1:H + 1, 1:W + 1] = x
    dw = np.zeros((9, Ci, g.shape[3]), dtype=np.float64)
    for t, (dy, dx) in enumerate(TAPS):
        dw[t] = xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W].reshape(-1, Ci).T @ \
            g.reshape(-1, g.shape[3])
    return dw, g.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def bilinear_up2(img):
    """[N, H, W, C] -> [N, 2H, 2W, C] with half-pixel centres, clamped edges."""
    N, H, W, C = img.shape

    def axis(n):
        X = np.arange(2 * n)
        u = (X + 0.5) / 2.0 - 0.5
        i0 = np.floor(u).astype(np.int64)
        f = u - i0
        return np.clip(i0, 0, n - 1), np.clip(i0 + 1, 0, n - 1), f

    y0, y1, fy = axis(H)
    x0, x1, fx = axis(W)
    a = img[:, y0][:, :, x0]
    b = img[:, y0][:, :, x1]
    c = img[:, y1][:, :, x0]
    d = img[:, y1][:, :, x1]
    fx = fx[None, None, :, None]
    fy = fy[None, :, None, None]
    top = a + (b - a) * fx
    bot = c + (d - c) * fx
    return top + (bot - top) * fy


def pixel_shuffle(o):
    """[N, H, W, >= 20] -> [N, 2H, 2W, 5]: sub-pixel (sy, sx) of (y, x) takes
    channels 5 s .. 5 s + 4, s = 2 sy + sx."""
    N, H, W, _ = o.shape
    out = np.zeros((N, 2 * H, 2 * W, 5), dtype=np.float64)
    for sy in (0, 1):
        for sx in (0, 1):
            s = 2 * sy + sx
            out[:, sy::2, sx::2] = o[..., 5 * s:5 * s + 5]
    return out


def pixel_unshuffle(g, channels=C_OUT):
    """Adjoint of pixel_shuffle (gradients back to the 20 used channels)."""
    N, H2, W2, _ = g.shape
    out = np.zeros((N, H2 // 2, W2 // 2, channels), dtype=np.float64)
    for sy in (0, 1):
        for sx in (0, 1):
            s = 2 * sy + sx
            out[..., 5 * s:5 * s + 5] = g[:, sy::2, sx::2]
    return out


def empty_neighbourhood(x0, radius=4):
    """[N, H, W] booleans: no nonzero channel of x0 within `radius` pixels
    (a (2 radius + 1)^2 window; outside the image counts as zero)."""
    x0 = np.asarray(x0)
    N, H, W, _ = x0.shape
    nz = np.any(x0 != 0, axis=-1)
    pad = np.zeros((N, H + 2 * radius, W + 2 * radius), dtype=bool)
    pad[:, radius:radius + H, radius:radius + W] = nz
    anyv = np.zeros((N, H, W), dtype=bool)
    for dy in range(2 * radius + 1):
        for dx in range(2 * radius + 1):
            anyv |= pad[:, dy:dy + H, dx:dx + W]
    return ~anyv


def forward(params, x0, act_round=None, skip_empty=False):
    """params: list of (w, b) per layer. Returns (rgba [N,2H,2W,4], z
    [N,2H,2W], cache for backpropagation). act_round, if given, is applied
    to every hidden activation (the precision they are stored in). With
    skip_empty (inference), pixels with an empty neighbourhood yield 0."""
    h = [np.asarray(x0, np.float64)]
    pre = []
    for i, (w, b) in enumerate(params):
        a = conv3x3(h[-1], w, b)
        pre.append(a)
        if i < len(params) - 1:
            r = relu(a)
            h.append(act_round(r) if act_round is not None else r)
        else:
            h.append(a)
    sh = pixel_shuffle(h[-1])
    base = bilinear_up2(h[0][..., :4])
    rgba = base + sh[..., :4]
    z = sh[..., 4]
    if skip_empty:
        e = np.repeat(np.repeat(empty_neighbourhood(h[0]), 2, axis=1), 2, axis=2)
        rgba = np.where(e[..., None], 0.0, rgba)
        z = np.where(e, 0.0, z)
    return rgba, z, (h, pre)


def loss_and_grads(params, x0, target, err_weight=1.0, act_round=None):
    """Loss = mean over full-resolution pixels and RGBA of the squared error
    + err_weight * mean over pixels of (z - e)^2, e = sqrt(mean over RGB of
    the squared error) held constant. Returns (loss, grads [(dw, db)])."""
    rgba, z, (h, pre) = forward(params, x0, act_round)
    target = np.asarray(target, np.float64)
    P = rgba.shape[0] * rgba.shape[1] * rgba.shape[2]
    diff = rgba - target
    e = np.sqrt((diff[..., :3] ** 2).mean(axis=-1))
    loss = (diff ** 2).sum() / (4 * P) + err_weight * ((z - e) ** 2).sum() / P
    g_sh = np.zeros(rgba.shape[:3] + (5,), dtype=np.float64)
    g_sh[..., :4] = 2.0 * diff / (4 * P)
    g_sh[..., 4] = err_weight * 2.0 * (z - e) / P
    g = pixel_unshuffle(g_sh)
    grads = [None] * len(params)
    for i in reversed(range(len(params))):
        dw, db = conv3x3_weight_grad(h[i], g)
        grads[i] = (dw, db)
        if i > 0:
            g = conv3x3_input_grad(g, params[i][0]) * (pre[i - 1] > 0)
    return loss, grads


def psnr(a, b):
    """PSNR over premultiplied RGB with peak 1 (per frame)."""
    mse = float(((np.asarray(a, np.float64)[..., :3] - np.asarray(b, np.float64)[..., :3]) ** 2)
                .mean())
    return float("inf") if mse == 0.0 else 10.0 * np.log10(1.0 / mse)


def depth_code(depth, diag):
    """The depth channel of the input: 1 / (1 + t / diag), 0 where no sample
    reached the depth threshold (t = +inf)."""
    d = np.asarray(depth, np.float64)
    return np.where(np.isfinite(d), 1.0 / (1.0 + d / diag), 0.0)


def to_bf16(x):
    """Round to the nearest bfloat16 (ties to even), as float64."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
