"""Pins of the upsampler reference (oracle/upsampler.py), on the CPU:
convolution against scipy's correlation, gradients against central finite
differences, pixel shuffle against explicit loops and its adjoint, bilinear
upsampling against scipy's zoom, bfloat16 rounding against torch."""
import numpy as np
import pytest
from scipy import ndimage, signal

from oracle import upsampler as U


def rand_params(rng, layers=U.LAYERS, scale=0.2):
    return [(rng.normal(size=(9, ci, co)) * scale, rng.normal(size=co) * 0.05)
            for ci, co in layers]


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 9, 3))
    w = rng.normal(size=(9, 3, 4))
    b = rng.normal(size=4)
    got = U.conv3x3(x, w, b)
    for n in range(2):
        for co in range(4):
            ref = np.full((7, 9), b[co])
            for ci in range(3):
                k = w[:, ci, co].reshape(3, 3)  # k[dy + 1, dx + 1]
                ref += signal.correlate(x[n, :, :, ci], k, mode="same")
            assert np.allclose(got[n, :, :, co], ref, atol=1e-12)


def test_input_and_weight_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 5, 6, 3))
    w = rng.normal(size=(9, 3, 2))
    b = rng.normal(size=2)
    g = rng.normal(size=(1, 5, 6, 2))
    f = lambda x_, w_, b_: float((U.conv3x3(x_, w_, b_) * g).sum())
    dx = U.conv3x3_input_grad(g, w)
    dw, db = U.conv3x3_weight_grad(x, g)
    h = 1e-6
    for arr, grad, name in ((x, dx, "x"), (w, dw, "w"), (b, db, "b")):
        d = rng.normal(size=arr.shape)
        args = {"x": x, "w": w, "b": b}
        up = dict(args, **{name: arr + h * d})
        dn = dict(args, **{name: arr - h * d})
        num = (f(up["x"], up["w"], up["b"]) - f(dn["x"], dn["w"], dn["b"])) / (2 * h)
        assert abs(num - (grad * d).sum()) < 1e-6 * max(1.0, abs(num))


def test_pixel_shuffle_explicit_and_adjoint():
    rng = np.random.default_rng(3)
    o = rng.normal(size=(2, 3, 4, 32))
    s = U.pixel_shuffle(o)
    for n in range(2):
        for y in range(6):
            for x in range(8):
                k = 2 * (y % 2) + (x % 2)
                assert np.array_equal(s[n, y, x], o[n, y // 2, x // 2, 5 * k:5 * k + 5])
    g = rng.normal(size=s.shape)
    assert abs((s * g).sum() - (o * U.pixel_unshuffle(g)).sum()) < 1e-10


def test_bilinear_up2_matches_scipy_zoom():
    rng = np.random.default_rng(4)
    img = rng.normal(size=(1, 5, 7, 2))
    got = U.bilinear_up2(img)
    for c in range(2):
        ref = ndimage.zoom(img[0, :, :, c], 2, order=1, mode="nearest", grid_mode=True)
        assert np.allclose(got[0, :, :, c], ref, atol=1e-12)
    const = np.full((1, 4, 4, 1), 0.3)
    assert np.allclose(U.bilinear_up2(const), 0.3, atol=1e-15)


def test_loss_gradients_match_finite_differences():
    """With the error head off (err_weight 0) the loss is the plain mean
    squared error: backpropagation must match central differences for every
    layer's weights and biases."""
    rng = np.random.default_rng(5)
    params = rand_params(rng)
    x0 = rng.uniform(0, 1, size=(1, 4, 5, U.C_IN))
    target = rng.uniform(0, 1, size=(1, 8, 10, 4))
    _, grads = U.loss_and_grads(params, x0, target, err_weight=0.0)
    h = 1e-6
    for layer in range(4):
        w, b = params[layer]
        for k, arr in ((0, w), (1, b)):
            d = rng.normal(size=arr.shape)
            up = list(params)
            dn = list(params)
            up[layer] = (w + h * d, b) if k == 0 else (w, b + h * d)
            dn[layer] = (w - h * d, b) if k == 0 else (w, b - h * d)
            num = (U.loss_and_grads(up, x0, target, 0.0)[0] -
                   U.loss_and_grads(dn, x0, target, 0.0)[0]) / (2 * h)
            assert abs(num - (grads[layer][k] * d).sum()) < 1e-6 * max(1e-3, abs(num)), layer


def test_error_head_gradient_with_frozen_target():
    """The error-head term's gradient treats e as a constant: perturbing only
    the last layer's z-channels moves z and not the colour, so e is fixed
    and finite differences must match."""
    rng = np.random.default_rng(6)
    params = rand_params(rng)
    x0 = rng.uniform(0, 1, size=(1, 3, 4, U.C_IN))
    target = rng.uniform(0, 1, size=(1, 6, 8, 4))
    _, grads = U.loss_and_grads(params, x0, target, err_weight=1.0)
    w, b = params[3]
    d = np.zeros_like(w)
    d[:, :, [4, 9, 14, 19]] = rng.normal(size=(9, w.shape[1], 4))  # z channels only
    h = 1e-6
    up = params[:3] + [(w + h * d, b)]
    dn = params[:3] + [(w - h * d, b)]
    num = (U.loss_and_grads(up, x0, target)[0] - U.loss_and_grads(dn, x0, target)[0]) / (2 * h)
    assert abs(num - (grads[3][0] * d).sum()) < 1e-6 * max(1e-3, abs(num))


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(size=1000) * 10 ** rng.uniform(-3, 3, 1000),
                        [0.0, 1.0, -2.5, 1.00390625, 1.005859375]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.to_bf16(x), ref)


def test_psnr_and_depth_code():
    a = np.zeros((4, 4, 4))
    b = a.copy()
    b[..., :3] = 0.01
    assert abs(U.psnr(a, b) - 40.0) < 1e-9
    assert U.psnr(a, a) == float("inf")
    assert np.allclose(U.depth_code([0.0, 221.7, np.inf], 221.7), [1.0, 0.5, 0.0])


def test_empty_neighbourhood_matches_a_maximum_filter():
    """The inference rule's neighbourhood (radius 4 = the receptive field of
    four 3x3 layers) equals scipy's 9x9 maximum filter of the nonzero mask
    with zero outside the image; one lit pixel lights exactly its 9x9 block."""
    from scipy.ndimage import maximum_filter
    rng = np.random.default_rng(21)
    x0 = np.zeros((2, 23, 31, 8))
    lit = rng.uniform(size=(2, 23, 31)) < 0.01
    x0[lit, rng.integers(0, 5)] = rng.uniform(0.1, 1.0, size=lit.sum())
    want = ~maximum_filter(np.any(x0 != 0, axis=-1), size=(1, 9, 9), mode="constant", cval=0)
    assert np.array_equal(U.empty_neighbourhood(x0), want)
    one = np.zeros((1, 20, 20, 8))
    one[0, 7, 12, 4] = 0.5
    ne = ~U.empty_neighbourhood(one)[0]
    ys, xs = np.nonzero(ne)
    assert (ys.min(), ys.max(), xs.min(), xs.max()) == (3, 11, 8, 16) and ne.sum() == 81


def test_skip_empty_drops_only_the_constant_response():
    """With skip_empty, pixels with an empty neighbourhood give 0 (their
    bilinear base is already 0); every other pixel is unchanged."""
    rng = np.random.default_rng(22)
    params = [(rng.normal(size=(9, ci, co)) * 0.2, rng.normal(size=co) * 0.1)
              for ci, co in U.LAYERS]
    x0 = np.zeros((1, 26, 30, 8))
    x0[0, 3:9, 4:12, :5] = rng.uniform(0, 1, size=(6, 8, 5))
    rgba, z, _ = U.forward(params, x0)
    srgba, sz, _ = U.forward(params, x0, skip_empty=True)
    e = np.repeat(np.repeat(U.empty_neighbourhood(x0), 2, axis=1), 2, axis=2)[0]
    assert e.any() and (~e).any()
    assert np.array_equal(srgba[0][~e], rgba[0][~e]) and np.array_equal(sz[0][~e], z[0][~e])
    assert np.all(srgba[0][e] == 0) and np.all(sz[0][e] == 0)
    base = U.bilinear_up2(x0[..., :4])[0]
    assert np.all(base[e] == 0)
    assert np.abs(rgba[0][e]).max() > 0  # the network alone would not give 0 there
