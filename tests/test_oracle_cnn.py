"""Pins of the predictor network's CPU oracle (oracle/cnn.py) against things
other than itself: brute-force loops, scipy's correlation, finite differences,
the adjoint identity, torch's Adam and torch's bfloat16 conversion."""
import numpy as np
import pytest
import scipy.signal
import torch

from oracle import cnn

RNG = np.random.default_rng(1234)


def _brute_conv(x, w, b):
    """Pure-Python loops straight from the definition (tiny inputs only)."""
    n, d, h, wd, ci = x.shape
    co = w.shape[0]
    y = np.zeros((n, d, h, wd, co))
    for nn in range(n):
        for z in range(d):
            for yy in range(h):
                for xx in range(wd):
                    for o in range(co):
                        s = b[o]
                        for kz in range(3):
                            for ky in range(3):
                                for kx in range(3):
                                    zz, y2, x2 = z + kz - 1, yy + ky - 1, xx + kx - 1
                                    if 0 <= zz < d and 0 <= y2 < h and 0 <= x2 < wd:
                                        t = (kz * 3 + ky) * 3 + kx
                                        for c in range(ci):
                                            s += w[o, t, c] * x[nn, zz, y2, x2, c]
                        y[nn, z, yy, xx, o] = s
    return y


def test_conv_matches_brute_force():
    x = RNG.standard_normal((2, 3, 4, 5, 3))
    w = RNG.standard_normal((2, 27, 3))
    b = RNG.standard_normal(2)
    assert np.allclose(cnn.conv3d(x, w, b), _brute_conv(x, w, b), rtol=1e-13, atol=1e-13)


def test_conv_matches_scipy_correlate():
    """Per (output, input) channel pair the convolution is scipy's 'same'
    correlation with the 3x3x3 kernel w[o, :, c]; a transposed channel pair or
    a mirrored tap fails this."""
    x = RNG.standard_normal((1, 6, 5, 7, 3))
    w = RNG.standard_normal((4, 27, 3))
    y = cnn.conv3d(x, w)
    for o in range(4):
        ref = sum(scipy.signal.correlate(x[0, ..., c], w[o, :, c].reshape(3, 3, 3), mode="same",
                                         method="direct") for c in range(3))
        assert np.allclose(y[0, ..., o], ref, rtol=1e-12, atol=1e-12)


def test_wgrad_and_bias_grad_by_finite_differences():
    x = RNG.standard_normal((2, 4, 3, 5, 3))
    w = RNG.standard_normal((2, 27, 3))
    b = RNG.standard_normal(2)
    gz = RNG.standard_normal((2, 4, 3, 5, 2))
    gw, gb = cnn.conv3d_wgrad(x, gz)
    L = lambda w_, b_: float(np.sum(gz * cnn.conv3d(x, w_, b_)))
    h = 1e-3   # L is linear in (w, b): central differences are exact up to rounding
    for idx in [(0, 0, 0), (1, 13, 2), (0, 26, 1), (1, 5, 0), (0, 21, 2)]:
        e = np.zeros_like(w)
        e[idx] = h
        fd = (L(w + e, b) - L(w - e, b)) / (2 * h)
        assert abs(fd - gw[idx]) < 1e-9 * max(1.0, abs(fd))
    for o in range(2):
        e = np.zeros(2)
        e[o] = h
        fd = (L(w, b + e) - L(w, b - e)) / (2 * h)
        assert abs(fd - gb[o]) < 1e-9 * max(1.0, abs(fd))


def test_dgrad_by_finite_differences_and_adjoint():
    x = RNG.standard_normal((1, 4, 5, 3, 2))
    w = RNG.standard_normal((3, 27, 2))
    gz = RNG.standard_normal((1, 4, 5, 3, 3))
    gx = cnn.conv3d_dgrad(gz, w)
    # adjoint: <conv(x), gz> = <x, dgrad(gz)>
    assert np.isclose(np.sum(cnn.conv3d(x, w) * gz), np.sum(x * gx), rtol=1e-12)
    L = lambda x_: float(np.sum(gz * cnn.conv3d(x_, w)))
    h = 1e-3
    for idx in [(0, 0, 0, 0, 0), (0, 3, 4, 2, 1), (0, 1, 2, 1, 0), (0, 2, 0, 2, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (L(x + e) - L(x - e)) / (2 * h)
        assert abs(fd - gx[idx]) < 1e-9 * max(1.0, abs(fd))


def test_network_gradients_by_finite_differences():
    """Backpropagation through 3 layers (ReLU between) against central
    differences of the loss itself."""
    chans = [3, 5, 4, 1]
    params = [(RNG.standard_normal((chans[k + 1], 27, chans[k])) * 0.3, RNG.standard_normal(chans[k + 1]) * 0.1)
              for k in range(3)]
    x = RNG.standard_normal((2, 3, 4, 3, 3))
    t = RNG.standard_normal((2, 3, 4, 3))
    loss, grads = cnn.loss_and_grads(params, x, t)
    h = 1e-6
    for k in range(3):
        w, b = params[k]
        for idx in [(0, 13, 0), (w.shape[0] - 1, 4, w.shape[2] - 1), (0, 26, w.shape[2] // 2)]:
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            lp = cnn.loss_and_grads(params[:k] + [(wp, b)] + params[k + 1:], x, t)[0]
            lm = cnn.loss_and_grads(params[:k] + [(wm, b)] + params[k + 1:], x, t)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[k][0][idx]) < 1e-6 * max(1e-2, abs(fd)), (k, idx, fd, grads[k][0][idx])
        bp, bm = b.copy(), b.copy()
        bp[0] += h
        bm[0] -= h
        fd = (cnn.loss_and_grads(params[:k] + [(w, bp)] + params[k + 1:], x, t)[0]
              - cnn.loss_and_grads(params[:k] + [(w, bm)] + params[k + 1:], x, t)[0]) / (2 * h)
        assert abs(fd - grads[k][1][0]) < 1e-6 * max(1e-2, abs(fd))


def test_mse_matches_torch():
    y = RNG.standard_normal((2, 3, 4))
    t = RNG.standard_normal((2, 3, 4))
    loss, g = cnn.mse(y, t)
    yt = torch.tensor(y, requires_grad=True)
    lt = torch.nn.functional.mse_loss(yt, torch.tensor(t))
    lt.backward()
    assert np.isclose(loss, lt.item(), rtol=1e-14)
    assert np.allclose(g, yt.grad.numpy(), rtol=1e-14)


def test_adam_matches_torch_optim():
    w0 = RNG.standard_normal(50)
    w = torch.tensor(w0.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    ww, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        g = RNG.standard_normal(50)
        opt.zero_grad()
        w.grad = torch.tensor(g)
        opt.step()
        ww, m, v = cnn.adam(ww, g, m, v, t, 3e-3)
        assert np.allclose(ww, w.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_bf16_round_matches_torch():
    a = np.concatenate([RNG.standard_normal(4000) * 10.0 ** RNG.integers(-6, 6, 4000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8)]])
    a32 = a.astype(np.float32)
    ref = torch.tensor(a32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(a32), ref)
    # ties go to even: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    assert cnn.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert cnn.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def test_block_means_of_known_fields():
    """Means of linear ramps over 8-cell blocks are the ramps at block
    centres; the ragged last block averages the cells it holds."""
    nz, ny, nx = 12, 8, 20
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rho = 1.0 + 0.01 * x
    u = np.stack([0.1 * y, 0.2 * z, -0.05 * x + 0.3 * z]).astype(np.float64)
    m = cnn.block_means(rho, u, (8, 8, 8))
    assert m.shape == (2, 1, 3, 4)
    cx = np.array([3.5, 11.5, 17.5])          # block centres in x (last block: cells 16..19)
    cz = np.array([3.5, 9.5])                 # in z (last block: cells 8..11)
    for k in range(2):
        for i in range(3):
            assert np.allclose(m[k, 0, i], [0.01 * cx[i], 0.1 * 3.5, 0.2 * cz[k], -0.05 * cx[i] + 0.3 * cz[k]],
                               rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("planted", ["mirror", "transpose", "no_bias"])
def test_planted_mistakes_are_caught(planted, monkeypatch):
    """Each plausible slip in the convolution fails the scipy or brute-force
    pin above: the pins have teeth."""
    x = RNG.standard_normal((1, 3, 3, 4, 2))
    w = RNG.standard_normal((2, 27, 2))
    b = RNG.standard_normal(2)
    good = _brute_conv(x, w, b)
    if planted == "mirror":
        bad = cnn.conv3d(x, w[:, ::-1, :], b)
    elif planted == "transpose":
        bad = cnn.conv3d(x, w.transpose(2, 1, 0), b)
    else:
        bad = cnn.conv3d(x, w)
    assert not np.allclose(bad, good, rtol=1e-6, atol=1e-6)
