"""Learned refinement-flag predictor on top of the kinetic sensor.

The sensor's block maxima M_b (Sec. 3.2, blocks of Sec. 3.4) say where the
mesh must be fine now; regridding every so many steps wants to know where it
must be fine by the next regrid.  ``FlagPredictor`` is a small 3D CNN over
the block grid that predicts log10 M_b `horizon` steps ahead.  Two forms:

* the configured one reads the per-block means of (rho - rho0, u) only (4
  channels) and predicts log10 M_b at the horizon directly (standardised
  with the training targets' mean and spread);
* an extension also reads log10 M_b now and one horizon earlier (6
  channels: the sensor and its recent trend) and predicts the change of
  log10 M_b, so that "no change" (reusing the current flags) is what an
  untrained network returns.

Every product runs in the matrix-core kernels of liblbm.so (bindings in
``cnn``): forward, data and weight gradients, ReLU backward, the loss and
Adam.  Torch provides device memory and the stream; numpy only marshals the
small per-block feature arrays (4096 blocks x 6 values at 128^3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import cnn
from .abi import LbmError

LOG_FLOOR = 1e-12   # block maxima below this are taken as this before log10


def _check(st, what):
    if st != 0:
        raise LbmError(st, f"{what} failed")


def log_sensor(bm):
    return np.log10(np.maximum(np.asarray(bm, dtype=np.float64), LOG_FLOOR))


def features(means, bm, bm_prev=None):
    """Raw per-block features [nbz, nby, nbx, 5 or 6]: (rho - rho0, u,
    [log10 M one horizon earlier,] log10 M); log10 M now is the last."""
    parts = [np.asarray(means, dtype=np.float64)]
    if bm_prev is not None:
        parts.append(log_sensor(bm_prev)[..., None])
    parts.append(log_sensor(bm)[..., None])
    return np.concatenate(parts, axis=-1)


@dataclass
class Normalizer:
    """Per-channel affine map of the raw features, fitted on training data."""
    mean: np.ndarray
    scale: np.ndarray

    @staticmethod
    def fit(raw):
        flat = np.asarray(raw, dtype=np.float64).reshape(-1, raw.shape[-1])
        sd = flat.std(axis=0)
        return Normalizer(flat.mean(axis=0), np.where(sd > 0, 1.0 / np.maximum(sd, 1e-30), 1.0))

    def __call__(self, raw):
        return (np.asarray(raw, dtype=np.float64) - self.mean) * self.scale


class _Layer:
    def __init__(self, ci, co, relu, rng, device):
        self.ci, self.co, self.relu = ci, co, relu
        std = math.sqrt(2.0 / (27 * ci)) if relu else 0.1 * math.sqrt(1.0 / (27 * ci))
        w = rng.standard_normal((co, 27, ci)) * std
        self.w = torch.tensor(w, dtype=torch.float32, device=device)
        self.b = torch.zeros(co, dtype=torch.float32, device=device)
        self.gw = torch.zeros_like(self.w)
        self.gb = torch.zeros_like(self.b)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.packed = torch.zeros(cnn.lbm_cnn_packed_size(co, ci), dtype=torch.int16, device=device)
        self.packed_flip = torch.zeros(cnn.lbm_cnn_packed_size(ci, co), dtype=torch.int16, device=device)

    def pack(self, stream):
        _check(cnn.lbm_cnn_pack_weights(self.w, self.co, self.ci, 0, self.packed, stream), "pack")
        _check(cnn.lbm_cnn_pack_weights(self.w, self.co, self.ci, 1, self.packed_flip, stream), "pack flip")


class FlagPredictor:
    """channels: (input, hidden..., 1); 3x3x3 convolutions, ReLU between."""

    def __init__(self, channels=(6, 16, 16, 16, 1), seed=0, device="cuda", stream=None, residual=True):
        """residual: the network learns the change of log10 M_b from the last
        input channel (log10 M_b now); else it learns log10 M_b itself."""
        self.residual = residual
        self.device = torch.device(device)
        self.stream = stream
        rng = np.random.default_rng(seed)
        self.channels = tuple(channels)
        self.layers = [_Layer(channels[k], channels[k + 1], k + 2 < len(channels), rng, self.device)
                       for k in range(len(channels) - 1)]
        self.t = 0
        # optimizer hyperparameters and step in device memory (lbm_cnn_adam_begin)
        self.hyper = torch.zeros(cnn.LBM_CNN_HYPER_FLOATS, dtype=torch.float32, device=self.device)
        self.normalizer = None
        self.y_offset, self.y_scale = 0.0, 1.0
        self._bufs = {}
        self._pack()

    # -- buffers ---------------------------------------------------------------
    def _pack(self):
        for L in self.layers:
            L.pack(self.stream)

    def _buffers(self, shape):
        if shape not in self._bufs:
            n, d, h, w = shape
            nv = n * d * h * w
            z = lambda c: torch.zeros(nv * cnn.pad4(c), dtype=torch.float32, device=self.device)
            acts = [z(L.co) for L in self.layers]
            grads = [z(c) for c in self.channels[:-1]] + [z(self.channels[-1])]
            ws = max(cnn.lbm_cnn_wgrad_workspace(n, d, h, w, L.ci, L.co) for L in self.layers) // 4
            # per-layer partial sums of the weight gradients, kept until the
            # fused fold-and-Adam launches of a training step
            works = [torch.zeros(cnn.lbm_cnn_wgrad_workspace(n, d, h, w, L.ci, L.co) // 4, dtype=torch.float32,
                                 device=self.device) for L in self.layers]
            self._bufs[shape] = dict(x=z(self.channels[0]), acts=acts, grads=grads, works=works,
                                     work=torch.zeros(ws, dtype=torch.float32, device=self.device),
                                     target=torch.zeros(nv, dtype=torch.float32, device=self.device),
                                     loss=torch.zeros(cnn.LBM_CNN_LOSS_FLOATS, dtype=torch.float32,
                                                      device=self.device))
        return self._bufs[shape]

    def load_input(self, x, shape):
        """x: float array (n, d, h, w, C0) (already normalized) -> device."""
        B = self._buffers(shape)
        c4 = cnn.pad4(self.channels[0])
        xp = np.zeros(shape + (c4,), dtype=np.float32)
        xp[..., :self.channels[0]] = x
        B["x"].copy_(torch.from_numpy(xp.reshape(-1)))
        return B

    # -- network -----------------------------------------------------------------
    def forward_device(self, shape):
        """Runs the layers on the loaded input; returns the last activation."""
        B = self._buffers(shape)
        n, d, h, w = shape
        a = B["x"]
        for L, out in zip(self.layers, B["acts"]):
            _check(cnn.lbm_cnn_conv3d_forward(a, n, d, h, w, L.ci, L.packed, L.co, L.b, L.relu, None, out,
                                              self.stream), "conv forward")
            a = out
        return a

    def backward_device(self, shape, partials=False):
        """Gradients of the loss whose output gradient is in grads[-1]; with
        `partials`, the weight gradients stay as per-layer partial sums for
        adam_step_partials (which folds them)."""
        B = self._buffers(shape)
        n, d, h, w = shape
        nv = n * d * h * w
        g = B["grads"][-1]
        L = self.layers[-1]
        if L.relu:   # the output layer's own ReLU (the layers below fuse theirs into the data gradient)
            _check(cnn.lbm_cnn_relu_backward(B["acts"][-1], g, nv * cnn.pad4(L.co), self.stream), "relu bwd")
        for k in range(len(self.layers) - 1, -1, -1):
            L = self.layers[k]
            inp = B["x"] if k == 0 else B["acts"][k - 1]
            if partials and k > 0:
                # weight-gradient partials and the data gradient (through the
                # ReLU of layer k - 1) in one launch
                gin = B["grads"][k]
                mask = B["acts"][k - 1] if self.layers[k - 1].relu else None
                _check(cnn.lbm_cnn_backward_layer(inp, g, n, d, h, w, L.ci, L.co, B["works"][k], L.packed_flip,
                                                  mask, gin, self.stream), "backward layer")
                g = gin
                continue
            if partials:
                _check(cnn.lbm_cnn_conv3d_wgrad_partials(inp, g, n, d, h, w, L.ci, L.co, B["works"][k],
                                                         self.stream), "wgrad partials")
            else:
                _check(cnn.lbm_cnn_conv3d_wgrad(inp, g, n, d, h, w, L.ci, L.co, B["work"], L.gw, L.gb,
                                                self.stream), "wgrad")
            if k > 0:
                # gradient at the input of layer k, through the ReLU of layer k - 1
                gin = B["grads"][k]
                mask = B["acts"][k - 1] if self.layers[k - 1].relu else None
                _check(cnn.lbm_cnn_conv3d_forward(g, n, d, h, w, L.co, L.packed_flip, L.ci, None, 0, mask, gin,
                                                  self.stream), "dgrad")
                g = gin

    def load_batch(self, x, target):
        """Copies a batch to the device: x (n, d, h, w, C0) normalized inputs,
        target (n, d, h, w).  Returns its shape."""
        shape = tuple(target.shape)
        B = self.load_input(x, shape)
        B["target"].copy_(torch.from_numpy(np.ascontiguousarray(target, dtype=np.float32).reshape(-1)))
        return shape

    def loss_and_grads_device(self, shape, partials=False):
        """Loss and gradients (in each layer's gw, gb; with `partials`, as
        per-layer partial sums) on the loaded batch; returns the device loss
        tensor (element 0)."""
        B = self._buffers(shape)
        y = self.forward_device(shape)
        nv = int(np.prod(shape))
        _check(cnn.lbm_cnn_mse(y, cnn.pad4(self.channels[-1]), B["target"], nv, B["grads"][-1], B["loss"],
                               self.stream), "mse")
        self.backward_device(shape, partials)
        return B["loss"]

    def loss_and_grads(self, x, target):
        """Loss (float) and gradients (in each layer's gw, gb) on a batch.
        x (n, d, h, w, C0) normalized inputs, target (n, d, h, w)."""
        return self.loss_and_grads_device(self.load_batch(x, target))[0]

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step of every parameter; the hyperparameters and the step
        count go through device memory (so the step can be graph-captured)."""
        self.t += 1
        _check(cnn.lbm_cnn_adam_begin(self.hyper, lr, beta1, beta2, eps, self.stream), "adam begin")
        for L in self.layers:   # weights, bias and both packed forms in one launch per layer
            _check(cnn.lbm_cnn_adam_layer(L.w, L.b, L.gw, L.gb, L.mw, L.vw, L.mb, L.vb, L.co, L.ci, L.packed,
                                          L.packed_flip, self.hyper, self.stream), "adam")

    def adam_step_partials(self, shape, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """adam_step from the per-layer partial sums that
        backward_device(shape, partials=True) left: each layer's fold and
        update in one launch (the same bits; gw, gb are filled too)."""
        B = self._buffers(shape)
        n, d, h, w = shape
        self.t += 1
        _check(cnn.lbm_cnn_adam_begin(self.hyper, lr, beta1, beta2, eps, self.stream), "adam begin")
        layers = [dict(w=L.w, b=L.b, work=work, mw=L.mw, vw=L.vw, mb=L.mb, vb=L.vb, packed=L.packed,
                       packed_flip=L.packed_flip, gw=L.gw, gb=L.gb, co=L.co, ci=L.ci)
                  for L, work in zip(self.layers, B["works"])]
        if len(layers) <= cnn.LBM_CNN_MAX_LAYERS:   # every layer's fold and update in one launch
            _check(cnn.lbm_cnn_adam_layers_fold(layers, n, d, h, w, self.hyper, self.stream), "adam fold")
        else:
            for L, work in zip(self.layers, B["works"]):
                _check(cnn.lbm_cnn_adam_layer_fold(L.w, L.b, work, n, d, h, w, L.mw, L.vw, L.mb, L.vb, L.co,
                                                   L.ci, L.packed, L.packed_flip, self.hyper, L.gw, L.gb,
                                                   self.stream), "adam fold")

    def train_step(self, shape, lr):
        """One training iteration (forward, loss, backward, Adam) on the
        loaded batch, without host transfers: a layer's weight-gradient
        partials and data gradient share a launch, and the folds of all
        layers run inside one Adam launch (12 launches)."""
        self.loss_and_grads_device(shape, partials=True)
        self.adam_step_partials(shape, lr)

    def capture_train_step(self, shape, lr):
        """A HIP graph of one training iteration on the loaded batch at a
        fixed learning rate; each replay advances the device step count.
        Count replays with `replayed(n)` to keep the host step count."""
        self._buffers(shape)
        g = torch.cuda.CUDAGraph()
        saved, t0 = self.stream, self.t
        self.stream = None       # launch on the capture stream
        try:
            with torch.cuda.graph(g):
                self.train_step(shape, lr)
        finally:
            self.stream, self.t = saved, t0
        return g

    def replayed(self, n):
        self.t += n

    def predict_raw(self, x):
        """Network output channel 0 for normalized inputs x (n, d, h, w, C0)."""
        shape = tuple(x.shape[:4])
        self.load_input(x, shape)
        y = self.forward_device(shape)
        c4 = cnn.pad4(self.channels[-1])
        return y.view(-1, c4)[:, 0].cpu().numpy().astype(np.float64).reshape(shape)

    # -- the flag predictor ------------------------------------------------------
    def _target_scale(self, raw, target_log):
        """(offset, scale) with network output = (learned quantity - offset) * scale."""
        y = np.asarray(target_log, dtype=np.float64)
        if self.residual:
            return 0.0, 1.0
        sd = float(y.std())
        return float(y.mean()), (1.0 / sd if sd > 0 else 1.0)

    def _learned(self, raw, target_log):
        """What the network output stands for: the change of log10 M_b from
        the last input channel (residual), else log10 M_b itself."""
        y = np.asarray(target_log, dtype=np.float64)
        return y - raw[..., -1] if self.residual else y

    def fit(self, raw, target_log, iters=1500, batch=8, lr=2e-3, seed=0, log_every=0):
        """Trains on raw features [S, nbz, nby, nbx, C0] to predict
        target_log [S, nbz, nby, nbx] = log10 M_b at the horizon (residual:
        as target - log10 M_b now, the last channel; else the standardised
        target).  Cosine learning rate from lr over `iters` Adam steps on
        random batches.  Returns the loss history."""
        self.normalizer = Normalizer.fit(raw)
        xs = self.normalizer(raw)
        self.y_offset, self.y_scale = self._target_scale(raw, target_log)
        dy = (self._learned(raw, target_log) - self.y_offset) * self.y_scale
        rng = np.random.default_rng(seed)
        hist = []
        S = raw.shape[0]
        for it in range(iters):
            idx = rng.choice(S, size=min(batch, S), replace=False)
            shape = self.load_batch(xs[idx], dy[idx])
            loss = self.loss_and_grads_device(shape, partials=True)[0]
            self.adam_step_partials(shape, lr * 0.5 * (1.0 + math.cos(math.pi * it / iters)))
            if log_every and (it % log_every == 0 or it + 1 == iters):
                hist.append((it, float(loss.item())))
        return hist

    def predict_log(self, raw):
        """Predicted log10 M_b at the horizon for raw features [S, ..., C0]."""
        if self.normalizer is None:
            raise RuntimeError("the predictor has not been fitted")
        y = self.predict_raw(self.normalizer(raw)) / self.y_scale + self.y_offset
        return raw[..., -1] + y if self.residual else y


def snapshot_run(Blocks, desc, snapshots, horizon, warm, history=True):
    """Runs one grid and records (raw features at t, log10 M_b at t + horizon)
    for t = warm + horizon * j, j < snapshots.  With history the features
    hold log10 M_b at t - horizon too (warm >= 2 horizon; else warm >=
    horizon).  Returns (raw, target_log) or None if the run goes non-finite."""
    if warm < (2 * horizon if history else horizon):
        raise ValueError("warm must leave room for the sensor history")
    blk = Blocks(desc)
    try:
        raw, tgt = [], []
        start = warm - (horizon if history else 0)
        blk.step_n(start - 1, 0)
        blk.step_n(1, 1)
        bm, _, _, bad = blk.sensor_flags()
        prev = None
        if history:
            prev = bm
            blk.step_n(horizon, horizon)
            bm, _, _, bad = blk.sensor_flags()
        cur = features(blk.block_means(), bm, prev)
        for _ in range(snapshots):
            blk.step_n(horizon, horizon)
            nxt, _, _, bad = blk.sensor_flags()
            if bad or not np.isfinite(cur).all():
                return None
            raw.append(cur)
            tgt.append(log_sensor(nxt))
            cur = features(blk.block_means(), nxt, bm if history else None)
            bm = nxt
        return np.stack(raw), np.stack(tgt)
    finally:
        blk.close()


def flag_scores(pred_flags, true_flags):
    """(precision, recall) of boolean refine flags."""
    tp = float(np.sum(pred_flags & true_flags))
    p = tp / max(1.0, float(np.sum(pred_flags)))
    r = tp / max(1.0, float(np.sum(true_flags)))
    return p, r
