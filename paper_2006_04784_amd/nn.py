"""Learned PSD warm start: the network's parameter and activation buffers and
the calls that run it (argument marshalling only; every arithmetic step runs
in the library's HIP kernels, see fch_nn_* in include/fch.h).

The network maps (u^n, u^{n-1}, k_{n+1}, k_n) to a correction of the
extrapolated first PSD iterate u^n + (k_{n+1}/k_n)(u^n - u^{n-1}) of eq.
recurrence.  Six 3x3 periodic convolutions, 32 channels, SiLU, BF16 weights
and activations with FP32 accumulation; the output layer starts at zero, so
the untrained network reproduces the plain extrapolation.  PSD then iterates
from the corrected guess to the same stopping tolerance.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import fch

LAYERS = (32, 32, 32, 32, 32, 16)   # output channels per layer (16: padded output layer)
CH = 32                              # channels of every activation tensor
IN_CH = 3                            # used input channels: u^n, d/s, log10 k


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _chk(code):
    fch._check(code)


class WarmStartNet:
    def __init__(self, H, W, batch, seed=0, device="cuda:0"):
        if H % 16 or W % 32:
            raise ValueError("H must be a multiple of 16 and W of 32")
        self.H, self.W, self.B = H, W, batch
        self.dev = torch.device(device)
        sizes = [9 * c * CH + c for c in LAYERS]
        self.offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        n = int(self.offs[-1])
        self.nparam = n
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.P = torch.zeros(n, **f32)
        self.G = torch.zeros(n, **f32)
        self.M = torch.zeros(n, **f32)
        self.V = torch.zeros(n, **f32)
        self.PB = torch.zeros(n, dtype=torch.bfloat16, device=self.dev)
        self.set_params(self.init_params(seed))
        act = (batch, H, W, CH)
        bf = dict(dtype=torch.bfloat16, device=self.dev)
        self.x = torch.zeros(act, **bf)
        self.z = [torch.zeros(act, **bf) for _ in LAYERS[:-1]]
        self.y = [torch.zeros(act, **bf) for _ in LAYERS[:-1]]
        self.dz = [torch.zeros(act, **bf) for _ in range(2)]
        self.wt = torch.zeros(9 * CH * CH, **bf)
        self.o = torch.zeros((batch, H, W), **f32)
        self.target = torch.zeros((batch, H, W), **f32)
        self.scale = torch.zeros(batch, dtype=torch.float64, device=self.dev)
        self.kk = torch.zeros((batch, 2), dtype=torch.float64, device=self.dev)
        self.fwork = torch.zeros(int(fch.lib().fch_nn_features_work_doubles(batch)),
                                 dtype=torch.float64, device=self.dev)
        L = fch.lib()
        self.scratch = torch.zeros(int(L.fch_nn_bwd_w_scratch_floats(batch, H, W)), **f32)
        self.nblocks = 256
        self.loss_parts = torch.zeros(self.nblocks, **f32)
        self.loss = torch.zeros(1, **f32)
        self.step = 0

    # ---- parameters --------------------------------------------------------
    @staticmethod
    def init_params(seed):
        """He-normal hidden layers (seeded), zero output layer, zero biases.
        Weights of the unused input channels of the first layer are zero."""
        rng = np.random.default_rng(seed)
        out = []
        for i, cout in enumerate(LAYERS):
            w = np.zeros((9, cout, CH))
            cin = IN_CH if i == 0 else CH
            if i < len(LAYERS) - 1:
                w[:, :, :cin] = rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), size=(9, cout, cin))
            out.append((w, np.zeros(cout)))
        return out

    def set_params(self, params):
        flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])
        self.P.copy_(torch.from_numpy(flat.astype(np.float32)))
        _chk(fch.lib().fch_nn_to_bf16(self.nparam, _p(self.P), _p(self.PB), None))

    def get_params(self):
        flat = self.P.cpu().numpy().astype(np.float64)
        out = []
        for i, cout in enumerate(LAYERS):
            a = flat[self.offs[i]:self.offs[i + 1]]
            out.append((a[:9 * cout * CH].reshape(9, cout, CH), a[9 * cout * CH:].copy()))
        return out

    def save_params(self, path):
        """Writes the FP32 master parameters and the layer widths to an .npz
        file (plain arrays, no pickles) at exactly `path`."""
        with open(path, "wb") as fh:
            np.savez(fh, params=self.P.cpu().numpy(), layers=np.array(LAYERS, dtype=np.int64),
                     ch=np.int64(CH), in_ch=np.int64(IN_CH))

    def load_params(self, path):
        """Reads parameters written by save_params (same architecture)."""
        with np.load(path, allow_pickle=False) as z:
            if (tuple(int(c) for c in z["layers"]) != tuple(LAYERS) or int(z["ch"]) != CH
                    or int(z["in_ch"]) != IN_CH):
                raise ValueError("%s: parameters of another architecture" % path)
            p = np.asarray(z["params"])
        if p.dtype != np.float32 or p.shape != (self.nparam,) or not np.isfinite(p).all():
            raise ValueError("%s: expected %d finite float32 parameters" % (path, self.nparam))
        self.P.copy_(torch.from_numpy(p))
        _chk(fch.lib().fch_nn_to_bf16(self.nparam, _p(self.P), _p(self.PB), None))

    def get_grads(self):
        flat = self.G.cpu().numpy().astype(np.float64)
        out = []
        for i, cout in enumerate(LAYERS):
            a = flat[self.offs[i]:self.offs[i + 1]]
            out.append((a[:9 * cout * CH].reshape(9, cout, CH), a[9 * cout * CH:].copy()))
        return out

    def _w(self, i):
        return C.c_void_p(self.PB.data_ptr() + 2 * int(self.offs[i]))

    def _b(self, i):
        return C.c_void_p(self.P.data_ptr() + 4 * int(self.offs[i] + 9 * LAYERS[i] * CH))

    def _g(self, i):
        return C.c_void_p(self.G.data_ptr() + 4 * int(self.offs[i]))

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)

    # ---- passes ------------------------------------------------------------
    def forward(self, nb, keep_z=True):
        """keep_z=False (inference) skips storing the pre-activations, which only
        the backward pass reads."""
        L, s, H, W = fch.lib(), self._stream(), self.H, self.W
        inp = self.x
        for i, cout in enumerate(LAYERS):
            if cout == CH:
                _chk(L.fch_nn_conv_fwd(nb, H, W, cout, _p(inp), self._w(i), self._b(i),
                                       _p(self.z[i]) if keep_z else None, _p(self.y[i]), None,
                                       s))
                inp = self.y[i]
            else:
                _chk(L.fch_nn_conv_fwd(nb, H, W, cout, _p(inp), self._w(i), self._b(i),
                                       None, None, _p(self.o), s))
        return self.o[:nb]

    def backward(self, nb):
        """MSE of the output against self.target, then all gradients into G;
        returns the loss tensor (device)."""
        L, s, H, W = fch.lib(), self._stream(), self.H, self.W
        n = nb * H * W
        _chk(L.fch_nn_mse(n, _p(self.o), _p(self.target), _p(self.dz[0]), _p(self.loss_parts),
                          self.nblocks, s))
        _chk(L.fch_nn_reduce(self.nblocks, 1, _p(self.loss_parts), _p(self.loss), s))
        cur = 0
        for i in range(len(LAYERS) - 1, -1, -1):
            inp = self.x if i == 0 else self.y[i - 1]
            _chk(L.fch_nn_conv_bwd_w(nb, H, W, LAYERS[i], _p(self.dz[cur]), _p(inp), self._g(i),
                                     _p(self.scratch), s))
            if i > 0:
                _chk(L.fch_nn_conv_bwd_data(nb, H, W, LAYERS[i], _p(self.dz[cur]), self._w(i),
                                            _p(self.z[i - 1]), _p(self.dz[1 - cur]),
                                            _p(self.wt), s))
                cur = 1 - cur
        return self.loss

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _chk(fch.lib().fch_nn_adam(self.nparam, _p(self.P), _p(self.G), _p(self.M), _p(self.V),
                                   _p(self.PB), lr, b1, b2, eps, self.step, self._stream()))

    def train_step(self, nb, lr=1e-3):
        self.forward(nb)
        loss = self.backward(nb)
        self.adam(lr)
        return loss

    # ---- features and guesses ------------------------------------------------
    def features(self, u_n, u_nm1, k, u_np1=None):
        """u_*: float64 (nb, H, W) device tensors, k: (nb, 2) = (k_{n+1}, k_n)."""
        nb = u_n.shape[0]
        self.kk[:nb].copy_(k)
        _chk(fch.lib().fch_nn_features(nb, self.H, self.W, _p(u_n), _p(u_nm1), _p(u_np1),
                                       _p(self.kk), _p(self.x),
                                       _p(self.target) if u_np1 is not None else None,
                                       _p(self.scale), _p(self.fwork), self._stream()))
        return nb

    def guess(self, u_n, u_nm1, k, out=None):
        """Physical guess for u^{n+1} of nb samples (float64 (nb, H, W))."""
        nb = self.features(u_n, u_nm1, k)
        self.forward(nb, keep_z=False)
        out = torch.empty_like(u_n) if out is None else out
        _chk(fch.lib().fch_nn_guess(nb, self.H, self.W, _p(u_n), _p(u_nm1), _p(self.kk),
                                    _p(self.scale), _p(self.o), _p(out), self._stream()))
        return out
