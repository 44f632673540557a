"""Learned seed slope for the exact LMS search (binding over lms_net_* in liblms.so).

A small point-set network predicts the LMS line's angle. Its slope is passed to
`lms_solve` as a seed slope, so the screen starts from the exact width at that
slope. Every candidate pair is still screened and the result stays exact
whatever the network predicts, since F(theta) >= the optimal width for every
theta (Eq. (1)). The forward, backward and Adam steps run in the library's
HIP kernels; this module only allocates device buffers and marshals
pointers.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _check, _stream, load

N_PARAMS = 8642
HIDDEN = 64
MAX_POINTS = 2048  # points the network pools per set (larger sets are read strided)
# packed parameter layout (row-major W[out][in])
LAYOUT = (("W1", (HIDDEN, 2)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (HIDDEN, HIDDEN)), ("b3", (HIDDEN,)), ("W4", (2, HIDDEN)), ("b4", (2,)))


def _lib():
    L = load()
    if not getattr(L, "_lms_net_ready", False):
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.lms_net_prepare.argtypes = [vp, vp, i64, vp, vp, vp]
        L.lms_net_forward.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.lms_net_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
        f = ctypes.c_float
        L.lms_net_adam.argtypes = [vp, vp, vp, vp, i64, f, f, f, f, vp]
        L.lms_net_slopes.argtypes = [vp, vp, i64, vp, vp]
        L.lms_net_infer.argtypes = [vp, vp, vp, i64, i64, ctypes.c_int32, vp, vp, vp]
        for fn in ("lms_net_prepare", "lms_net_forward", "lms_net_backward", "lms_net_adam",
                   "lms_net_slopes", "lms_net_infer"):
            getattr(L, fn).restype = ctypes.c_int
        L._lms_net_ready = True
    return L


def pack(params: dict) -> np.ndarray:
    """Dict of arrays -> packed FP32 vector."""
    return np.concatenate([np.asarray(params[k], dtype=np.float32).reshape(-1) for k, _ in LAYOUT])


def unpack(vec) -> dict:
    v = np.asarray(vec, dtype=np.float64).reshape(-1)
    out, o = {}, 0
    for k, shp in LAYOUT:
        m = int(np.prod(shp))
        out[k] = v[o:o + m].reshape(shp)
        o += m
    return out


def _offsets_dev(offsets, device):
    if isinstance(offsets, torch.Tensor):
        return offsets.to(device=device, dtype=torch.int64).contiguous()
    return torch.as_tensor(np.asarray(offsets, dtype=np.int64), device=device)


class SeedNet:
    """Network parameters (FP32 masters on the device) with Adam state."""

    def __init__(self, params=None, device="cuda:0", seed: int = 0):
        self.device = torch.device(device)
        if params is None:
            g = torch.Generator().manual_seed(seed)
            parts = []
            for k, shp in LAYOUT:
                if k.startswith("W"):
                    lim = math.sqrt(6.0 / shp[1])
                    parts.append((torch.rand(shp, generator=g, dtype=torch.float64) * 2 - 1) * lim)
                else:
                    parts.append(torch.zeros(shp, dtype=torch.float64))
            vec = torch.cat([p.reshape(-1) for p in parts]).to(torch.float32)
        elif isinstance(params, dict):
            vec = torch.from_numpy(pack(params))
        else:
            vec = torch.as_tensor(np.asarray(params, dtype=np.float32))
        assert vec.numel() == N_PARAMS
        self.P = vec.to(self.device).contiguous()
        self.m = torch.zeros_like(self.P)
        self.v = torch.zeros_like(self.P)
        self.step = 0

    # -- data ---------------------------------------------------------------
    def prepare(self, xy: torch.Tensor, offsets, stream=None):
        """Normalised FP32 points (N, 2) and per-set (cx, cy, sx, sy)."""
        off = _offsets_dev(offsets, self.device)
        B = off.numel() - 1
        pts = torch.empty((xy.shape[0], 2), dtype=torch.float32, device=self.device)
        scale = torch.empty((B, 4), dtype=torch.float64, device=self.device)
        _check(_lib().lms_net_prepare(xy.data_ptr(), off.data_ptr(), B, pts.data_ptr(),
                                      scale.data_ptr(), _stream(stream)))
        return pts, scale, off

    # -- passes ---------------------------------------------------------------
    def forward(self, pts: torch.Tensor, off: torch.Tensor, want_g: bool = True, stream=None):
        B = off.numel() - 1
        out = torch.empty((B, 2), dtype=torch.float32, device=self.device)
        g = torch.empty((B, HIDDEN), dtype=torch.float32, device=self.device) if want_g else None
        _check(_lib().lms_net_forward(self.P.data_ptr(), pts.data_ptr(), off.data_ptr(), B,
                                      out.data_ptr(), None if g is None else g.data_ptr(),
                                      _stream(stream)))
        return out, g

    def gradient(self, pts, off, target, stream=None):
        """Mean-loss gradient (N_PARAMS,), per-set losses (B,) and outputs."""
        B = off.numel() - 1
        out, g = self.forward(pts, off, True, stream)
        grad_set = torch.empty((B, N_PARAMS), dtype=torch.float32, device=self.device)
        grad = torch.empty(N_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(B, dtype=torch.float32, device=self.device)
        target = target.to(device=self.device, dtype=torch.float32).contiguous()
        _check(_lib().lms_net_backward(self.P.data_ptr(), pts.data_ptr(), off.data_ptr(), B,
                                       target.data_ptr(), out.data_ptr(), g.data_ptr(),
                                       grad_set.data_ptr(), grad.data_ptr(), loss.data_ptr(),
                                       _stream(stream)))
        return grad, loss, out

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        _check(_lib().lms_net_adam(self.P.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                   grad.data_ptr(), self.step, lr, beta1, beta2, eps,
                                   _stream(stream)))

    def train_step(self, pts, off, target, lr=1e-3):
        grad, loss, _ = self.gradient(pts, off, target)
        self.adam(grad, lr)
        return loss

    # -- inference ------------------------------------------------------------
    def predict_slopes(self, xy: torch.Tensor, offsets, max_set: int | None = None,
                       max_points: int = MAX_POINTS, out: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
        """Seed slope per set, FP64 on the device (lms_net_infer: the features
        of each set pooled over many workgroups; a set above max_points points
        is read at evenly strided indices). offsets: host array or device
        tensor (B+1); max_set: the largest set (taken from host offsets)."""
        if isinstance(offsets, torch.Tensor) and offsets.is_cuda:
            off = offsets.to(torch.int64).contiguous()
            if max_set is None:
                max_set = int((off[1:] - off[:-1]).max())
        else:
            h = np.asarray(offsets, dtype=np.int64)
            max_set = int(np.diff(h).max()) if max_set is None else max_set
            off = torch.as_tensor(h, device=self.device)
        B = off.numel() - 1
        theta = torch.empty(B, dtype=torch.float64, device=self.device)
        _check(_lib().lms_net_infer(self.P.data_ptr(), xy.data_ptr(), off.data_ptr(), B,
                                    max_set, max_points, theta.data_ptr(),
                                    None if out is None else out.data_ptr(), _stream(stream)))
        return theta

    # -- persistence ------------------------------------------------------------
    def save(self, path: str):
        np.save(path, self.P.detach().cpu().numpy())

    @classmethod
    def load_weights(cls, path: str, device="cuda:0"):
        return cls(np.load(path), device=device)


def targets_from_slopes(theta: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """(cos 2phi, sin 2phi) of each line's angle in its set's normalised frame."""
    phi = np.arctan(np.asarray(theta) * scale[:, 2] / scale[:, 3])
    return np.stack([np.cos(2 * phi), np.sin(2 * phi)], 1).astype(np.float32)
