"""FP64 CPU oracle of the learned refinement-flag predictor's network.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The network is not part
of the paper; the quantity it predicts is the block maximum of the kinetic
sensor (Sec. 3.2, blocks of Sec. 3.4), which the LBM oracle computes.

Everything here is a plain definition written out in float64 numpy:
  * a 3x3x3 cross-correlation with zero padding ("same" size) mapping Ci to
    Co channels, activations channels-last (n, d, h, w, c), weights
    w[co, tap, ci] with tap = (kz*3 + ky)*3 + kx reading the input at offset
    (kz-1, ky-1, kx-1);
  * its gradients with respect to the weights, the bias and the input;
  * ReLU, the mean squared error of output channel 0, and the Adam update
    (Kingma & Ba, 2015, Algorithm 1, bias-corrected moments);
  * rounding of float32 values to bfloat16 (round to nearest, ties to even),
    so that a test can give both sides the same product inputs.

Pins (tests/test_oracle_cnn.py): brute-force loops and scipy.signal.correlate
for the convolution, central finite differences for every gradient (exact up
to rounding for the linear maps), the adjoint identity, torch.optim.Adam for
the update, torch's bfloat16 conversion for the rounding.  No function here is
"parity unpinned".
"""
from __future__ import annotations

import numpy as np

TAPS = [(kz, ky, kx) for kz in range(3) for ky in range(3) for kx in range(3)]


def bf16_round(a) -> np.ndarray:
    """float32(a) rounded to bfloat16 (nearest, ties to even), as float64.
    Finite inputs only."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))


def conv3d(x, w, b=None):
    """y[n, v, o] = sum_{tap, c} w[o, tap, c] x[n, v + off(tap), c] + b[o]."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, d, h, wd, _ = x.shape
    xp = _pad(x)
    y = np.zeros((n, d, h, wd, w.shape[0]))
    for t, (kz, ky, kx) in enumerate(TAPS):
        y += xp[:, kz:kz + d, ky:ky + h, kx:kx + wd, :] @ w[:, t, :].T
    if b is not None:
        y += np.asarray(b, dtype=np.float64)
    return y


def conv3d_wgrad(x, gz):
    """Gradients of sum(gz * conv3d(x, w, b)) with respect to w and b:
    gw[o, tap, c] = sum_{n, v} gz[n, v, o] x[n, v + off(tap), c],
    gb[o] = sum_{n, v} gz[n, v, o]."""
    x = np.asarray(x, dtype=np.float64)
    gz = np.asarray(gz, dtype=np.float64)
    n, d, h, wd, ci = x.shape
    co = gz.shape[-1]
    xp = _pad(x)
    gzf = gz.reshape(-1, co)
    gw = np.empty((co, 27, ci))
    for t, (kz, ky, kx) in enumerate(TAPS):
        gw[:, t, :] = gzf.T @ xp[:, kz:kz + d, ky:ky + h, kx:kx + wd, :].reshape(-1, ci)
    return gw, gzf.sum(axis=0)


def conv3d_dgrad(gz, w):
    """Gradient of sum(gz * conv3d(x, w, b)) with respect to x:
    gx[n, v, c] = sum_{tap, o} w[o, tap, c] gz[n, v - off(tap), o]."""
    gz = np.asarray(gz, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, d, h, wd, _ = gz.shape
    gp = _pad(gz)
    gx = np.zeros((n, d, h, wd, w.shape[2]))
    for t, (kz, ky, kx) in enumerate(TAPS):
        gx += gp[:, 2 - kz:2 - kz + d, 2 - ky:2 - ky + h, 2 - kx:2 - kx + wd, :] @ w[:, t, :]
    return gx


def relu(a):
    return np.maximum(a, 0.0)


def mse(y0, target):
    """Mean squared error of output channel 0 and its gradient."""
    e = np.asarray(y0, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(e * e)), 2.0 * e / e.size


def _ident(a):
    return a


def forward(params, x, q=None):
    """Network forward: conv + ReLU on every layer but the last.  params is a
    list of (w, b); returns the list of layer outputs (post-activation).
    q, if given, rounds both operands of every convolution product (e.g.
    bf16_round, the precision the matrix-core kernels multiply in)."""
    q = q or _ident
    acts = []
    a = np.asarray(x, dtype=np.float64)
    for k, (w, b) in enumerate(params):
        z = conv3d(q(a), q(w), b)
        a = relu(z) if k + 1 < len(params) else z
        acts.append(a)
    return acts


def loss_and_grads(params, x, target, q=None):
    """MSE of the last layer's channel 0 against target (n, d, h, w) and the
    gradient of every (w, b) by backpropagation; q as in forward."""
    q = q or _ident
    acts = forward(params, x, q)
    loss, g0 = mse(acts[-1][..., 0], target)
    g = np.zeros_like(acts[-1])
    g[..., 0] = g0
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        if k + 1 < len(params):
            g = g * (acts[k] > 0.0)
        inp = x if k == 0 else acts[k - 1]
        grads[k] = conv3d_wgrad(q(inp), q(g))
        if k > 0:
            g = conv3d_dgrad(q(g), q(params[k][0]))
    return loss, grads


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at t >= 1; returns the new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def block_means(rho, u, block, rho0=1.0):
    """Per-block means of (rho - rho0, u_x, u_y, u_z) over the cells of each
    block (ragged edge blocks average the cells they hold).  rho (nz, ny, nx),
    u (3, nz, ny, nx); returns (nbz, nby, nbx, 4)."""
    nz, ny, nx = rho.shape
    bx, by, bz = block
    nb = ((nz + bz - 1) // bz, (ny + by - 1) // by, (nx + bx - 1) // bx)
    out = np.empty(nb + (4,))
    fields = [rho - rho0, u[0], u[1], u[2]]
    for k in range(nb[0]):
        for j in range(nb[1]):
            for i in range(nb[2]):
                sl = (slice(k * bz, (k + 1) * bz), slice(j * by, (j + 1) * by), slice(i * bx, (i + 1) * bx))
                for c in range(4):
                    out[k, j, i, c] = fields[c][sl].mean()
    return out
