"""GPU parity of the learned upsampler's MFMA kernels against the FP64
reference (oracle/upsampler.py).

Each convolution layer is checked on the GPU's own input of that layer
(bf16-stored activations): hidden layers within one bfloat16 step, the last
(FP32) layer and the upsampled output to FP32 accumulation error. Gradients
of the training loss must point the same way as the reference's (bf16
gradients on the GPU), Adam's first step is checked in closed form, and a
small problem must train.
"""
import sys

import numpy as np
import pytest

from oracle import upsampler as U

pytestmark = pytest.mark.gpu

N, H, W = 2, 19, 23  # ragged against the 64-pixel waves
SCALE = 50.0


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU (no CPU fallback exists)"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bf16_params(rng, scale=0.25):
    out = []
    for ci, co in U.LAYERS:
        w = U.to_bf16(rng.normal(size=(9, ci, co)) * scale / np.sqrt(9 * min(ci, 5 if ci == 8
                                                                               else ci)))
        b = rng.normal(size=co).astype(np.float32).astype(np.float64) * 0.05
        out.append((w, b))
    return out


def inputs(rng):
    import torch
    rgba = rng.uniform(0, 1, size=(N, H, W, 4)).astype(np.float32)
    rgba[..., :3] *= rgba[..., 3:4]
    depth = rng.uniform(0, 300, size=(N, H, W)).astype(np.float32)
    depth[rng.uniform(size=depth.shape) < 0.2] = np.inf
    return rgba, depth, torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda()


def x0_reference(rgba, depth):
    """The input tensor as the prep kernel builds it (FP32 arithmetic, then
    bfloat16)."""
    inv = np.float32(1.0 / SCALE)
    code = np.where(np.isfinite(depth), np.float32(1) / (np.float32(1) + depth * inv),
                    np.float32(0)).astype(np.float32)
    x0 = np.zeros((N, H, W, 8))
    x0[..., :4] = U.to_bf16(rgba)
    x0[..., 4] = U.to_bf16(code)
    return x0


def test_forward_layers_match_reference():
    import torch

    from paper_1804_08197_amd import upsampler as up
    rng = np.random.default_rng(11)
    params = bf16_params(rng)
    rgba, depth, trgba, tdepth = inputs(rng)
    u = up.Upsampler(N * H * W)
    try:
        u.set_weights(up.pack(params))
        u.set_fused(False)  # layer by layer: the activations stay readable
        out = torch.full((N, 2 * H, 2 * W, 4), float("nan"), device="cuda")
        err = torch.full((N, 2 * H, 2 * W), float("nan"), device="cuda")
        mse = u.forward(trgba, tdepth, SCALE, out, err, predict=True)
        P = N * H * W
        x0 = u.read_buffer(0, (N, H, W, 8), "bf16")
        assert np.array_equal(x0, x0_reference(rgba, depth))
        prev = x0
        for layer in range(3):
            got = u.read_buffer(1 + layer, (N, H, W, 32), "bf16")
            w, b = params[layer]
            ref = U.to_bf16(U.relu(U.conv3x3(prev, w, b)))
            ulp = np.maximum(np.abs(ref), 1e-30) * 2.0 ** -7
            bad = np.abs(got - ref) > ulp
            assert bad.mean() < 2e-3 and np.abs(got - ref).max() <= 2 * ulp.max(), layer
            log("layer %d: %.4f%% of values one bf16 step off" % (layer + 1, 100 * bad.mean()))
            prev = got
        o = u.read_buffer(4, (N, H, W, 32), "f32")
        w, b = params[3]
        oref = U.conv3x3(prev, w, b)
        assert np.abs(o - oref).max() <= 1e-5 * max(1.0, np.abs(oref).max())
        # upsampled output from the GPU's o and x0
        sh = U.pixel_shuffle(o)
        ref_rgba = U.bilinear_up2(x0[..., :4]) + sh[..., :4]
        assert np.abs(out.cpu().numpy() - ref_rgba).max() <= 1e-5
        assert np.allclose(err.cpu().numpy(), sh[..., 4] ** 2, rtol=1e-5, atol=1e-7)
        assert np.allclose(mse, (sh[..., 4] ** 2).reshape(N, -1).mean(axis=1), rtol=1e-5)
        assert P == 874
    finally:
        u.close()


@pytest.mark.parametrize("shape", [(2, 19, 23), (3, 45, 70), (1, 1, 1), (1, 16, 16),
                                   (1, 33, 17)])
def test_fused_inference_equals_the_layered_path(shape):
    """The fused tile kernel must give the layer-by-layer output bit for bit
    (same MFMA products in the same order, same epilogues, zero padding) on
    ragged sizes spanning several 16 x 16 tiles; the predicted per-image
    errors agree to double rounding."""
    import torch

    from paper_1804_08197_amd import upsampler as up
    n, h, w = shape
    rng = np.random.default_rng(20 + h * w)
    params = bf16_params(rng, 0.5)
    rgba = rng.uniform(0, 1, size=(n, h, w, 4)).astype(np.float32)
    rgba[..., :3] *= rgba[..., 3:4]
    depth = rng.uniform(0, 300, size=(n, h, w)).astype(np.float32)
    depth[rng.uniform(size=depth.shape) < 0.2] = np.inf
    trgba, tdepth = torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda()
    u = up.Upsampler(n * h * w)
    try:
        u.set_weights(up.pack(params))
        res = []
        for fused in (False, True):
            u.set_fused(fused)
            out = torch.full((n, 2 * h, 2 * w, 4), float("nan"), device="cuda")
            err = torch.full((n, 2 * h, 2 * w), float("nan"), device="cuda")
            mse = u.forward(trgba, tdepth, SCALE, out, err, predict=True)
            res.append((out.cpu().numpy(), err.cpu().numpy(), mse))
        (o0, e0, m0), (o1, e1, m1) = res
        assert np.isfinite(o1).all() and np.isfinite(e1).all()
        assert np.array_equal(o0, o1) and np.array_equal(e0, e1)
        assert np.allclose(m0, m1, rtol=1e-12, atol=0)
        log("%s: fused == layered, mse %s" % (shape, m1))
    finally:
        u.close()



def test_layered_predicted_error_is_deterministic():
    """The layer-by-layer path adds the predicted error in a fixed order
    (per-chunk partials, then a fixed-order sum): repeated launches give the
    same per-image sums bit for bit, and the fallback flag agrees with
    them."""
    import torch

    from paper_1804_08197_amd import upsampler as up
    n, h, w = 3, 61, 77
    rng = np.random.default_rng(44)
    rgba = rng.uniform(0, 1, size=(n, h, w, 4)).astype(np.float32)
    rgba[..., :3] *= rgba[..., 3:4]
    depth = rng.uniform(0, 300, size=(n, h, w)).astype(np.float32)
    trgba, tdepth = torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda()
    u = up.Upsampler(n * h * w)
    try:
        u.set_weights(up.pack(bf16_params(rng, 0.5)))
        u.set_fused(False)
        out = torch.empty((n, 2 * h, 2 * w, 4), device="cuda")
        sums = [u.forward(trgba, tdepth, SCALE, out, predict=True) for _ in range(4)]
        for m in sums[1:]:
            assert np.array_equal(m, sums[0])
        assert np.all(sums[0] > 0)
    finally:
        u.close()

def test_gradients_match_reference():
    import torch

    from paper_1804_08197_amd import upsampler as up
    rng = np.random.default_rng(12)
    params = bf16_params(rng)
    rgba, depth, trgba, tdepth = inputs(rng)
    target = rng.uniform(0, 1, size=(N, 2 * H, 2 * W, 4)).astype(np.float32)
    u = up.Upsampler(N * H * W)
    try:
        u.set_weights(up.pack(params))
        loss, g = u.gradients(trgba, tdepth, SCALE, torch.from_numpy(target).cuda(), 0.5)
        x0 = x0_reference(rgba, depth)
        ref_loss, ref_grads = U.loss_and_grads(params, x0, target, 0.5, act_round=U.to_bf16)
        assert abs(loss - ref_loss) <= 1e-3 * ref_loss
        got = up.unpack(g)
        for layer in range(4):
            for k in range(2):
                a = np.asarray(got[layer][k], np.float64).ravel()
                r = ref_grads[layer][k].ravel()
                cos = a @ r / (np.linalg.norm(a) * np.linalg.norm(r))
                rel = np.linalg.norm(a - r) / np.linalg.norm(r)
                log("layer %d %s: cos %.6f rel %.2e" % (layer + 1, "wb"[k], cos, rel))
                assert cos > 0.999 and rel < 0.05, (layer, k)
    finally:
        u.close()


def test_first_adam_step_closed_form():
    """From zero optimiser state Adam's first bias-corrected step is
    -lr g / (|g| + eps) for every weight."""
    import torch

    from paper_1804_08197_amd import upsampler as up
    rng = np.random.default_rng(13)
    params = bf16_params(rng)
    _, _, trgba, tdepth = inputs(rng)
    target = torch.from_numpy(rng.uniform(0, 1, size=(N, 2 * H, 2 * W, 4)).astype(np.float32))
    target = target.cuda()
    u = up.Upsampler(N * H * W)
    try:
        w0 = up.pack(params)
        u.set_weights(w0)
        _, g = u.gradients(trgba, tdepth, SCALE, target, 1.0)
        lr = 1e-3
        u.train_step(trgba, tdepth, SCALE, target, lr, 1.0)
        w1 = u.get_weights()
        expect = w0.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
        live = (np.abs(g) > 1e-12) | (g == 0)  # squares of tinier gradients underflow
        assert np.abs(w1 - expect)[live].max() <= 1e-6
        assert live.mean() > 0.99
    finally:
        u.close()


def test_training_fits_a_small_problem():
    """Targets made by a fixed random network of the same shape: training
    from another random start must cut the loss by a large factor."""
    import torch

    from paper_1804_08197_amd import upsampler as up
    rng = np.random.default_rng(14)
    teacher = bf16_params(rng, 0.5)
    _, _, trgba, tdepth = inputs(rng)
    t = up.Upsampler(N * H * W)
    u = up.Upsampler(N * H * W)
    try:
        t.set_weights(up.pack(teacher))
        target = torch.empty(N, 2 * H, 2 * W, 4, device="cuda")
        t.forward(trgba, tdepth, SCALE, target)
        u.set_weights(up.pack(bf16_params(rng, 0.25)))
        first = None
        for i in range(300):
            loss = u.train_step(trgba, tdepth, SCALE, target, 3e-3, 0.0, want_loss=True)
            first = loss if first is None else first
        log("loss %.3e -> %.3e" % (first, loss))
        assert loss < 0.1 * first
    finally:
        t.close()
        u.close()


def test_bad_arguments():
    import torch

    from paper_1804_08197_amd import sg
    from paper_1804_08197_amd import upsampler as up
    u = up.Upsampler(100)
    try:
        x = torch.zeros(1, 10, 11, 4, device="cuda")
        d = torch.zeros(1, 10, 11, device="cuda")
        o = torch.zeros(1, 20, 22, 4, device="cuda")
        with pytest.raises(sg.SgError):
            u.forward(x, d, SCALE, o)  # 110 pixels > 100
        with pytest.raises(sg.SgError):
            u.set_weights(np.zeros(5, np.float32))
        with pytest.raises(sg.SgError):
            u.forward(x[:, :5], d[:, :5], -1.0, o)
    finally:
        u.close()


def test_device_fallback_flag_matches_the_host_decision():
    """sg_up_forward_flag: the same image as sg_up_forward and a flag equal
    to the host-side decision (predicted PSNR below the threshold) for
    thresholds on both sides of the prediction."""
    import math

    import torch

    from paper_1804_08197_amd import upsampler as up
    rng = np.random.default_rng(15)
    params = bf16_params(rng)
    _, _, trgba, tdepth = inputs(rng)
    u = up.Upsampler(N * H * W)
    try:
        u.set_weights(up.pack(params))
        ref = torch.empty(N, 2 * H, 2 * W, 4, device="cuda")
        mse = u.forward(trgba, tdepth, SCALE, ref, predict=True)
        pred = 10 * math.log10(1.0 / float(np.mean(mse)))
        flag = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        for thr in (pred - 1.0, pred + 1.0, -math.inf, math.inf):
            out = torch.full_like(ref, float("nan"))
            u.forward_flag(trgba, tdepth, SCALE, out, thr, flag)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            assert int(flag.item()) == int(pred < thr), (thr, pred)
    finally:
        u.close()


@pytest.mark.parametrize("lod", [False, True])
def test_device_decided_path_equals_the_host_decided_path(lod):
    """UpsampledPath.render_device (decision on the device, conditional
    full-resolution render) gives the frame UpsampledPath.render gives:
    the upsampled image when the prediction passes, the plain render when
    it does not."""
    import math

    import torch

    import gen
    from paper_1804_08197_amd import sg
    from paper_1804_08197_amd import upsample as U
    from paper_1804_08197_amd import upsampler as up
    from tests.helpers import gpu_volume
    vol = gen.random_volume((48, 40, 56), 31, dtype=np.uint8)
    h = gpu_volume([vol], 16, 3, [gen.tf_identity()], [(0, 255)])
    W2, H2 = 70, 46
    vs = gen.stereo(np.array([150.0, -90.0, 80.0]), np.array([28.0, 20.0, 24.0]), 4.0, W2, H2,
                    0.5, 0.5 * W2 / H2)
    u = up.Upsampler(2 * (H2 // 2) * (W2 // 2))
    try:
        u.set_weights(up.pack(bf16_params(np.random.default_rng(16))))
        path = U.UpsampledPath(h, u, 100.0, {"ert": 0.99, "skip_empty": 1}, W2, H2, 2, lod=lod)
        pred = path.predicted_psnr(vs)
        flag = torch.zeros(1, dtype=torch.int32, device="cuda")
        for thr in (pred - 1.0, pred + 1.0):
            path.threshold_db = thr
            want, fell = path.render(vs)
            want = want.clone()
            path.out.fill_(float("nan"))
            got = path.render_device(vs, flag)
            torch.cuda.synchronize()
            assert bool(flag.item()) == fell == (pred < thr)
            assert torch.equal(got, want), thr
        assert math.isfinite(pred)
    finally:
        u.close()
        sg.sg_volume_destroy(h)


@pytest.mark.parametrize("shape", [(2, 45, 70), (1, 33, 17), (3, 40, 48)])
def test_empty_neighbourhoods_yield_background(shape):
    """Sparse inputs (empty tiles, partly empty tiles, ragged edges): the
    fused kernel equals the layered path bit for bit, and the layered output
    equals the FP64 reconstruction from its own buffers with the inference
    rule (background where the 9x9 neighbourhood of x0 is empty)."""
    import torch

    from paper_1804_08197_amd import upsampler as up
    n, h, w = shape
    rng = np.random.default_rng(30 + h + w)
    params = bf16_params(rng, 0.5)
    rgba = np.zeros((n, h, w, 4), np.float32)
    depth = np.full((n, h, w), np.inf, np.float32)
    for i in range(n):
        for _ in range(3):  # a few small patches of content
            y0, x0_ = rng.integers(0, h), rng.integers(0, w)
            sl = (i, slice(y0, min(h, y0 + 3)), slice(x0_, min(w, x0_ + 4)))
            a = rng.uniform(0.2, 1.0, size=rgba[sl].shape[:-1] + (1,)).astype(np.float32)
            rgba[sl] = np.concatenate([rng.uniform(0, 1, size=a.shape[:-1] + (3,)) * a, a], -1)
            depth[sl] = rng.uniform(10, 300, size=depth[sl].shape)
    trgba, tdepth = torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda()
    u = up.Upsampler(n * h * w)
    try:
        u.set_weights(up.pack(params))
        res = []
        for fused in (False, True):
            u.set_fused(fused)
            out = torch.full((n, 2 * h, 2 * w, 4), float("nan"), device="cuda")
            err = torch.full((n, 2 * h, 2 * w), float("nan"), device="cuda")
            mse = u.forward(trgba, tdepth, SCALE, out, err, predict=True)
            res.append((out.cpu().numpy(), err.cpu().numpy(), mse))
            if not fused:
                x0 = u.read_buffer(0, (n, h, w, 8), "bf16")
                o = u.read_buffer(4, (n, h, w, 32), "f32")
        (o0, e0, m0), (o1, e1, m1) = res
        assert np.array_equal(o0, o1) and np.array_equal(e0, e1)
        assert np.allclose(m0, m1, rtol=1e-12, atol=0)
        empty = np.repeat(np.repeat(U.empty_neighbourhood(x0), 2, axis=1), 2, axis=2)
        assert empty.any() and (~empty).any()
        sh = U.pixel_shuffle(o)
        ref = np.where(empty[..., None], 0.0, U.bilinear_up2(x0[..., :4]) + sh[..., :4])
        assert np.abs(o0 - ref).max() <= 1e-5
        assert np.array_equal(e0[empty], np.zeros(empty.sum(), np.float32))
        assert np.allclose(e0[~empty], (sh[..., 4] ** 2)[~empty], rtol=1e-5, atol=1e-7)
        log("%s: %.1f%% of output pixels background" % (shape, 100 * empty.mean()))
    finally:
        u.close()


def block_mask(rgba, depth):
    """Per 8 x 8-pixel block: any pixel with a nonzero rgba component or a
    finite depth (the render's tile_any rule)."""
    n, h, w = depth.shape
    nz = (rgba != 0).any(-1) | np.isfinite(depth)
    mh, mw = (h + 7) // 8, (w + 7) // 8
    pad = np.zeros((n, mh * 8, mw * 8), bool)
    pad[:, :h, :w] = nz
    return pad.reshape(n, mh, 8, mw, 8).any(axis=(2, 4)).astype(np.uint8)


def test_content_mask_drives_the_same_frame():
    """The fused network runs only on tiles the content mask marks (dilated
    by the layers' reach); all others are background without a look at the
    input. Every source of the mask (built by the call, computed here, all
    ones) gives the layered path's output bit for bit, over two calls in a
    row with different inputs and sizes (the tile lists' counters start at
    zero on each call), on sparse and dense inputs."""
    import torch

    from paper_1804_08197_amd import upsampler as up
    rng = np.random.default_rng(77)
    params = bf16_params(rng, 0.5)
    u = up.Upsampler(2 * 96 * 130)
    try:
        u.set_weights(up.pack(params))
        for (n, h, w), sparse in (((2, 96, 130), True), ((1, 37, 53), False),
                                  ((2, 61, 45), True)):
            rgba = np.zeros((n, h, w, 4), np.float32)
            depth = np.full((n, h, w), np.inf, np.float32)
            if sparse:
                for i in range(n):
                    for _ in range(4):
                        y0, x0_ = rng.integers(0, h), rng.integers(0, w)
                        sl = (i, slice(y0, min(h, y0 + 2)), slice(x0_, min(w, x0_ + 3)))
                        a = rng.uniform(0.2, 1.0, size=rgba[sl].shape[:-1] + (1,))
                        rgba[sl] = np.concatenate([rng.uniform(0, 1, a.shape[:-1] + (3,)) * a, a],
                                                  -1).astype(np.float32)
                        depth[sl] = rng.uniform(10, 300, size=depth[sl].shape)
            else:
                rgba[:] = rng.uniform(0, 1, size=rgba.shape)
                depth[:] = rng.uniform(0, 300, size=depth.shape)
            trgba, tdepth = torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda()
            mask = block_mask(rgba, depth)
            masks = {"built": None, "given": torch.from_numpy(mask).cuda(),
                     "ones": torch.ones(mask.shape, dtype=torch.uint8, device="cuda")}
            u.set_fused(False)
            ref = torch.full((n, 2 * h, 2 * w, 4), float("nan"), device="cuda")
            ref_err = torch.full((n, 2 * h, 2 * w), float("nan"), device="cuda")
            m_ref = u.forward(trgba, tdepth, SCALE, ref, ref_err, predict=True)
            u.set_fused(True)
            for name, m in masks.items():
                out = torch.full_like(ref, float("nan"))
                err = torch.full_like(ref_err, float("nan"))
                mse = u.forward(trgba, tdepth, SCALE, out, err, predict=True, content=m)
                assert torch.equal(out, ref), (n, h, w, name)
                assert torch.equal(err, ref_err), (n, h, w, name)
                assert np.allclose(mse, m_ref, rtol=1e-12, atol=0), (n, h, w, name)
            log("%s sparse=%s: %d of %d blocks with content, all masks == layered" % (
                (n, h, w), sparse, int(mask.sum()), mask.size))
    finally:
        u.close()


def test_render_tile_mask_feeds_the_network():
    """The half-resolution render's own tile_any mask, handed to the network,
    gives the frame the network gives when it builds the mask itself (and
    the mask equals the 8 x 8-block rule applied to the render's output)."""
    import torch

    import gen
    from paper_1804_08197_amd import sg
    from paper_1804_08197_amd import upsampler as up
    from tests.helpers import gpu_volume
    vol = gen.random_volume((48, 40, 56), 33, dtype=np.uint8)
    h = gpu_volume([vol], 16, 3, [gen.tf_identity()], [(0, 255)])
    W2, H2 = 150, 94
    vs = gen.stereo(np.array([150.0, -90.0, 80.0]), np.array([28.0, 20.0, 24.0]), 4.0, W2, H2,
                    0.5, 0.5 * W2 / H2)
    n, hh, ww = 2, H2 // 2, W2 // 2
    u = up.Upsampler(n * hh * ww)
    try:
        u.set_weights(up.pack(bf16_params(np.random.default_rng(18))))
        rgba = torch.empty(n, hh, ww, 4, device="cuda")
        depth = torch.empty(n, hh, ww, device="cuda")
        tiles = torch.full((n, (hh + 7) // 8, (ww + 7) // 8), 7, dtype=torch.uint8, device="cuda")
        half = [dict(v, width=ww, height=hh, tile_any=tiles[i]) for i, v in enumerate(vs)]
        sg.sg_render_views(h, half, {"ert": 0.99, "skip_empty": 1, "lod": 0, "bias": 1,
                                     "depth_alpha": 0.5}, list(rgba), list(depth))
        torch.cuda.synchronize()
        want_mask = block_mask(rgba.cpu().numpy(), depth.cpu().numpy())
        assert np.array_equal(tiles.cpu().numpy(), want_mask)
        assert want_mask.any() and not want_mask.all()
        outs = []
        for m in (None, tiles):
            out = torch.full((n, 2 * hh, 2 * ww, 4), float("nan"), device="cuda")
            mse = u.forward(rgba, depth, 100.0, out, predict=True, content=m)
            outs.append((out, mse))
        assert torch.equal(outs[0][0], outs[1][0])
        assert np.array_equal(outs[0][1], outs[1][1])
    finally:
        u.close()
        sg.sg_volume_destroy(h)


def test_full_size_stereo_input_sampled_parity():
    """The benchmark's network input (two eyes of 720 x 800, sparse content
    as in the blob scene): fused inference equals the layered path bit for
    bit over the whole frame; at sampled pixels (corners, edges, tile seams,
    content) every layer of the layered path matches the FP64 reference on
    the GPU's own input of that layer (the bars of the small case); the
    whole upsampled output matches its FP64 reconstruction from the GPU's x0
    and last layer with the inference rule."""
    import torch

    from paper_1804_08197_amd import upsampler as up
    n, h, w = 2, 800, 720
    rng = np.random.default_rng(41)
    params = bf16_params(rng, 0.5)
    rgba = np.zeros((n, h, w, 4), np.float32)
    depth = np.full((n, h, w), np.inf, np.float32)
    yy, xx = np.mgrid[0:h, 0:w]
    centres = []
    for i in range(n):
        for _ in range(6):  # discs of content
            cy, cx, r = rng.integers(0, h), rng.integers(0, w), rng.integers(20, 90)
            m = (yy - cy) ** 2 + (xx - cx) ** 2 < r * r
            a = rng.uniform(0.1, 1.0, size=m.sum()).astype(np.float32)
            rgba[i][m] = np.stack([rng.uniform(0, 1, m.sum()) * a, rng.uniform(0, 1, m.sum()) * a,
                                   rng.uniform(0, 1, m.sum()) * a, a], -1)
            depth[i][m] = rng.uniform(10, 300, m.sum())
            centres.append((i, int(cy), int(cx)))
    trgba, tdepth = torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda()
    u = up.Upsampler(n * h * w)
    try:
        u.set_weights(up.pack(params))
        res = []
        for fused in (True, False):
            u.set_fused(fused)
            out = torch.full((n, 2 * h, 2 * w, 4), float("nan"), device="cuda")
            err = torch.full((n, 2 * h, 2 * w), float("nan"), device="cuda")
            mse = u.forward(trgba, tdepth, SCALE, out, err, predict=True)
            res.append((out.cpu().numpy(), err.cpu().numpy(), mse))
        (o1, e1, m1), (o0, e0, m0) = res  # fused, then layered (buffers readable)
        assert np.array_equal(o0, o1) and np.array_equal(e0, e1)
        assert np.allclose(m0, m1, rtol=1e-12, atol=0)
        # sampled pixels: corners, edges, 16-pixel tile seams, content
        pix = [(i, y, x) for i in range(n) for y in (0, h - 1) for x in (0, w - 1)]
        pix += [(i, 15, 16) for i in range(n)] + [(i, 400, 367) for i in range(n)]
        pix += [(i, min(h - 1, max(0, cy + int(rng.integers(-30, 31)))),
                 min(w - 1, max(0, cx + int(rng.integers(-30, 31))))) for i, cy, cx in centres]
        pix += [(int(rng.integers(0, n)), int(rng.integers(0, h)), int(rng.integers(0, w)))
                for _ in range(40)]

        def conv_at(inp, wgt, b, i, y, x):
            c = inp.shape[-1]
            crop = np.zeros((1, 3, 3, c))
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if 0 <= y + dy < h and 0 <= x + dx < w:
                        crop[0, dy + 1, dx + 1] = inp[i, y + dy, x + dx]
            return U.conv3x3(crop, wgt, b)[0, 1, 1]

        x0 = u.read_buffer(0, (n, h, w, 8), "bf16")
        assert np.array_equal(x0, x0_reference_of(rgba, depth))
        prev = x0
        bad = total = 0
        for layer in range(3):
            got = u.read_buffer(1 + layer, (n, h, w, 32), "bf16")
            wgt, b = params[layer]
            for i, y, x in pix:
                ref = U.to_bf16(U.relu(conv_at(prev, wgt, b, i, y, x)))
                ulp = np.maximum(np.abs(ref), 1e-30) * 2.0 ** -7
                d = np.abs(got[i, y, x] - ref)
                assert (d <= 2 * ulp.max()).all(), (layer, i, y, x)
                bad += int((d > ulp).sum())
                total += d.size
            prev = got
        assert bad <= max(4, 2e-3 * total)
        o = u.read_buffer(4, (n, h, w, 32), "f32")
        wgt, b = params[3]
        for i, y, x in pix:
            oref = conv_at(prev, wgt, b, i, y, x)
            assert np.abs(o[i, y, x] - oref).max() <= 1e-5 * max(1.0, np.abs(oref).max())
        empty = np.repeat(np.repeat(U.empty_neighbourhood(x0), 2, axis=1), 2, axis=2)
        assert empty.any() and (~empty).any()
        sh = U.pixel_shuffle(o)
        ref = np.where(empty[..., None], 0.0, U.bilinear_up2(x0[..., :4]) + sh[..., :4])
        assert np.abs(o0 - ref).max() <= 1e-5
        log("full size: %d sampled pixels, %.4f%% one bf16 step off, %.1f%% background" % (
            len(pix), 100.0 * bad / total, 100 * empty.mean()))
    finally:
        u.close()


def x0_reference_of(rgba, depth):
    """x0_reference for any input shape."""
    inv = np.float32(1.0 / SCALE)
    code = np.where(np.isfinite(depth), np.float32(1) / (np.float32(1) + depth * inv),
                    np.float32(0)).astype(np.float32)
    x0 = np.zeros(rgba.shape[:-1] + (8,))
    x0[..., :4] = U.to_bf16(rgba)
    x0[..., 4] = U.to_bf16(code)
    return x0

