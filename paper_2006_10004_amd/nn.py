"""Python binding of the surrogate network's C ABI (include/tvspec_nn.h).

Argument marshalling only: the convolutions, the loss, the gradients and
the optimiser run in the HIP kernels of libtvspec.so.  Tensors are torch
GPU tensors (device memory and streams); bfloat16 tensors are channels-last
where the header says so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .tvspec import _lib, _check, TvspecError  # noqa: F401  (one library, one runtime)

EXPORTS = (
    "tvspec_nn_conv3x3",
    "tvspec_nn_conv3x3_dgrad",
    "tvspec_nn_conv3x3_wgrad",
    "tvspec_net_create",
    "tvspec_net_num_params",
    "tvspec_net_get_params",
    "tvspec_net_set_params",
    "tvspec_net_set_output_scale",
    "tvspec_net_set_loss_floor",
    "tvspec_net_set_grad_clip",
    "tvspec_net_grad_stats",
    "tvspec_net_forward",
    "tvspec_net_forward_checked",
    "tvspec_net_train_step",
    "tvspec_net_last_loss",
    "tvspec_net_loss_grad",
    "tvspec_net_identity_error",
    "tvspec_net_destroy",
)

IN_CHANNELS = 3
BANDS = 4
OUT_CHANNELS = 15
LAYERS = (("e1a", 3, 48), ("e1b", 48, 48), ("e2a", 48, 96), ("e2b", 96, 96), ("e3a", 96, 192),
          ("e3b", 192, 192), ("e4a", 192, 384), ("e4b", 384, 384), ("d3a", 576, 192), ("d3b", 192, 192),
          ("d2a", 288, 96), ("d2b", 96, 96), ("d1a", 144, 48), ("d1b", 48, 48), ("out", 48, 15))

_i, _d, _f, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_float, ctypes.c_void_p
_ll = ctypes.c_longlong
_lib.tvspec_nn_conv3x3.argtypes = [_vp, _i, _i, _i, _i, _vp, _vp, _i, _i, _vp, _i, _vp]
_lib.tvspec_nn_conv3x3.restype = _i
_lib.tvspec_nn_conv3x3_dgrad.argtypes = [_vp, _i, _i, _i, _i, _vp, _i, _vp, _vp, _vp]
_lib.tvspec_nn_conv3x3_dgrad.restype = _i
_lib.tvspec_nn_conv3x3_wgrad.argtypes = [_vp, _vp, _i, _i, _i, _i, _i, _vp, _vp, _vp]
_lib.tvspec_nn_conv3x3_wgrad.restype = _i
_lib.tvspec_net_create.argtypes = [_i, _i, _i, ctypes.c_ulonglong, ctypes.POINTER(_vp)]
_lib.tvspec_net_create.restype = _i
_lib.tvspec_net_num_params.argtypes = [_vp, ctypes.POINTER(_ll)]
_lib.tvspec_net_num_params.restype = _i
_lib.tvspec_net_get_params.argtypes = [_vp, _vp, _ll]
_lib.tvspec_net_get_params.restype = _i
_lib.tvspec_net_set_params.argtypes = [_vp, _vp, _ll]
_lib.tvspec_net_set_params.restype = _i
_lib.tvspec_net_set_output_scale.argtypes = [_vp, _vp]
_lib.tvspec_net_set_output_scale.restype = _i
_lib.tvspec_net_set_loss_floor.argtypes = [_vp, _f]
_lib.tvspec_net_set_loss_floor.restype = _i
_lib.tvspec_net_set_grad_clip.argtypes = [_vp, _f]
_lib.tvspec_net_set_grad_clip.restype = _i
_lib.tvspec_net_grad_stats.argtypes = [_vp, ctypes.POINTER(_f), ctypes.POINTER(_f), ctypes.POINTER(_f)]
_lib.tvspec_net_grad_stats.restype = _i
_lib.tvspec_net_forward.argtypes = [_vp, _vp, _i, _vp, _vp]
_lib.tvspec_net_forward.restype = _i
_lib.tvspec_net_forward_checked.argtypes = [_vp, _vp, _i, _vp, _vp, _vp]
_lib.tvspec_net_forward_checked.restype = _i
_lib.tvspec_net_train_step.argtypes = [_vp, _vp, _vp, _vp, _i, _f, ctypes.POINTER(_f), _vp]
_lib.tvspec_net_last_loss.argtypes = [_vp, ctypes.POINTER(_f), _vp]
_lib.tvspec_net_last_loss.restype = _i
_lib.tvspec_net_train_step.restype = _i
_lib.tvspec_net_loss_grad.argtypes = [_vp, _vp, _vp, _vp, _i, ctypes.POINTER(_f), _vp, _vp]
_lib.tvspec_net_loss_grad.restype = _i
_lib.tvspec_net_identity_error.argtypes = [_vp, _vp, _i, _i, _i, _vp, _vp]
_lib.tvspec_net_identity_error.restype = _i
_lib.tvspec_net_destroy.argtypes = [_vp]
_lib.tvspec_net_destroy.restype = _i


def _stream(t, stream):
    return ctypes.c_void_p((stream if stream is not None else torch.cuda.current_stream(t.device)).cuda_stream)


def _bf16(t, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.bfloat16 or tuple(t.shape) != shape \
            or not t.is_contiguous():
        raise ValueError("%s must be a contiguous bfloat16 GPU tensor of shape %s" % (name, shape))


def tvspec_nn_conv3x3(x, w, bias=None, relu=False, out_f32=False, stream=None):
    """y = act(conv3x3(x, w) + bias): x [B,H,W,Cin], w [Cout,3,3,Cin] bfloat16."""
    B, H, W, Cin = x.shape
    Cout = w.shape[0]
    _bf16(x, (B, H, W, Cin), "x")
    _bf16(w, (Cout, 3, 3, Cin), "w")
    if bias is not None and (bias.dtype != torch.float32 or tuple(bias.shape) != (Cout,)):
        raise ValueError("bias must be float32 [Cout]")
    y = torch.empty((B, H, W, Cout), dtype=torch.float32 if out_f32 else torch.bfloat16, device=x.device)
    _check(_lib.tvspec_nn_conv3x3(x.data_ptr(), B, H, W, Cin, w.data_ptr(),
                                  bias.data_ptr() if bias is not None else None, Cout, 1 if relu else 0,
                                  y.data_ptr(), 1 if out_f32 else 0, _stream(x, stream)))
    return y


def tvspec_nn_conv3x3_dgrad(dy, w, mask=None, stream=None):
    """dx = conv3x3^T(dy) (zero where mask <= 0): dy [B,H,W,Cout], w [Cout,3,3,Cin]."""
    B, H, W, Cout = dy.shape
    Cin = w.shape[3]
    _bf16(dy, (B, H, W, Cout), "dy")
    _bf16(w, (Cout, 3, 3, Cin), "w")
    if mask is not None:
        _bf16(mask, (B, H, W, Cin), "mask")
    dx = torch.empty((B, H, W, Cin), dtype=torch.bfloat16, device=dy.device)
    _check(_lib.tvspec_nn_conv3x3_dgrad(dy.data_ptr(), B, H, W, Cout, w.data_ptr(), Cin,
                                        mask.data_ptr() if mask is not None else None, dx.data_ptr(),
                                        _stream(dy, stream)))
    return dx


def tvspec_nn_conv3x3_wgrad(x, dy, stream=None):
    """(dw [Cout,3,3,Cin], db [Cout]) float32 for x [B,H,W,Cin], dy [B,H,W,Cout]."""
    B, H, W, Cin = x.shape
    Cout = dy.shape[3]
    _bf16(x, (B, H, W, Cin), "x")
    _bf16(dy, (B, H, W, Cout), "dy")
    dw = torch.empty((Cout, 3, 3, Cin), dtype=torch.float32, device=x.device)
    db = torch.empty((Cout,), dtype=torch.float32, device=x.device)
    _check(_lib.tvspec_nn_conv3x3_wgrad(x.data_ptr(), dy.data_ptr(), B, H, W, Cin, Cout, dw.data_ptr(),
                                        db.data_ptr(), _stream(x, stream)))
    return dw, db


def tvspec_net_create(H, W, max_batch, seed=0):
    h = ctypes.c_void_p()
    _check(_lib.tvspec_net_create(int(H), int(W), int(max_batch), int(seed), ctypes.byref(h)))
    return h


def tvspec_net_num_params(h):
    n = _ll(0)
    _check(_lib.tvspec_net_num_params(h, ctypes.byref(n)))
    return n.value


def tvspec_net_get_params(h):
    p = np.empty(tvspec_net_num_params(h), dtype=np.float32)
    _check(_lib.tvspec_net_get_params(h, p.ctypes.data, p.size))
    return p


def tvspec_net_set_params(h, p):
    p = np.ascontiguousarray(p, dtype=np.float32)
    _check(_lib.tvspec_net_set_params(h, p.ctypes.data, p.size))


def tvspec_net_set_output_scale(h, scale):
    s = np.ascontiguousarray(scale, dtype=np.float32)
    if s.shape != (OUT_CHANNELS,):
        raise ValueError("scale must have %d entries" % OUT_CHANNELS)
    _check(_lib.tvspec_net_set_output_scale(h, s.ctypes.data))


def tvspec_net_set_loss_floor(h, kappa):
    _check(_lib.tvspec_net_set_loss_floor(h, float(kappa)))


def tvspec_net_set_grad_clip(h, clip):
    _check(_lib.tvspec_net_set_grad_clip(h, float(clip)))


def tvspec_net_grad_stats(h):
    n, a, sc = _f(0.0), _f(0.0), _f(0.0)
    _check(_lib.tvspec_net_grad_stats(h, ctypes.byref(n), ctypes.byref(a), ctypes.byref(sc)))
    return n.value, a.value, sc.value


def tvspec_net_forward(h, f, out, stream=None):
    _check(_lib.tvspec_net_forward(h, f.data_ptr(), f.shape[0], out.data_ptr(), _stream(f, stream)))


def tvspec_net_forward_checked(h, f, out, err, stream=None):
    _check(_lib.tvspec_net_forward_checked(h, f.data_ptr(), f.shape[0], out.data_ptr(),
                                           err.data_ptr() if err is not None else None, _stream(f, stream)))


def tvspec_net_train_step(h, f, bands, residual, lr, stream=None, sync=True):
    """One step; returns the loss (sync=True) or None (the step is only
    enqueued; tvspec_net_last_loss reads the latest loss later)."""
    loss = _f(0.0)
    _check(_lib.tvspec_net_train_step(h, f.data_ptr(), bands.data_ptr(), residual.data_ptr(), f.shape[0],
                                      float(lr), ctypes.byref(loss) if sync else None, _stream(f, stream)))
    return loss.value if sync else None


def tvspec_net_last_loss(h, stream=None, device=None):
    loss = _f(0.0)
    st = stream.cuda_stream if stream is not None else torch.cuda.current_stream(device).cuda_stream
    _check(_lib.tvspec_net_last_loss(h, ctypes.byref(loss), st))
    return loss.value


def tvspec_net_loss_grad(h, f, bands, residual, grads=True, stream=None):
    loss = _f(0.0)
    g = np.empty(tvspec_net_num_params(h), dtype=np.float32) if grads else None
    _check(_lib.tvspec_net_loss_grad(h, f.data_ptr(), bands.data_ptr(), residual.data_ptr(), f.shape[0],
                                     ctypes.byref(loss), g.ctypes.data if grads else None, _stream(f, stream)))
    return loss.value, g


def tvspec_net_identity_error(f, out, stream=None):
    """Per-image mean |f - sum of bands - residual| of outputs [B,15,H,W]."""
    B, _, H, W = f.shape
    err = torch.empty((B,), dtype=torch.float32, device=f.device)
    _check(_lib.tvspec_net_identity_error(f.data_ptr(), out.data_ptr(), B, H, W, err.data_ptr(),
                                          _stream(f, stream)))
    return err


def tvspec_net_destroy(h):
    _check(_lib.tvspec_net_destroy(h))


def split_params(p):
    """Flat parameter vector -> {name: (w [Cout,3,3,Cin], b [Cout])} (views)."""
    out, off = {}, 0
    for name, ci, co in LAYERS:
        nw = co * 9 * ci
        out[name] = (p[off:off + nw].reshape(co, 3, 3, ci), p[off + nw:off + nw + co])
        off += nw + co
    return out


class Net:
    """The encoder-decoder surrogate (widths 48-96-192-384) for H x W images."""

    def __init__(self, H, W, max_batch, seed=0):
        self.H, self.W, self.max_batch = H, W, max_batch
        self._h = tvspec_net_create(H, W, max_batch, seed)
        self.output_scale = np.ones(OUT_CHANNELS, dtype=np.float32)

    def _check_f(self, f):
        if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.float32 or f.dim() != 4 \
                or tuple(f.shape[1:]) != (IN_CHANNELS, self.H, self.W) or not f.is_contiguous():
            raise ValueError("f must be a contiguous float32 GPU tensor [B,3,%d,%d]" % (self.H, self.W))

    def _check_target(self, f, bands, residual):
        B = f.shape[0]
        for t, shp, nm in ((bands, (B, BANDS, IN_CHANNELS, self.H, self.W), "bands"),
                           (residual, (B, IN_CHANNELS, self.H, self.W), "residual")):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
                    or tuple(t.shape) != shp or not t.is_contiguous():
                raise ValueError("%s must be a contiguous float64 GPU tensor %s" % (nm, shp))

    @property
    def num_params(self):
        return tvspec_net_num_params(self._h)

    def get_params(self):
        return tvspec_net_get_params(self._h)

    def set_params(self, p):
        tvspec_net_set_params(self._h, p)

    def set_output_scale(self, scale):
        """Fixed per-channel output scales [15] (see the header)."""
        tvspec_net_set_output_scale(self._h, scale)
        self.output_scale = np.asarray(scale, dtype=np.float32)

    def set_loss_floor(self, kappa):
        """Floor of the loss's denominators (see the header); 0 = the paper's loss."""
        tvspec_net_set_loss_floor(self._h, kappa)

    def set_grad_clip(self, clip):
        """Gradient-norm clipping factor (see the header); 0 = off."""
        tvspec_net_set_grad_clip(self._h, clip)

    def grad_stats(self):
        """(norm, running average, scale) of the last training step."""
        return tvspec_net_grad_stats(self._h)

    def forward(self, f, out=None, stream=None, identity=False):
        """f [B,3,H,W] float32 -> [B,15,H,W] float32 (4 bands x 3, residual x 3);
        with identity=True also each image's reconstruction-identity error
        [B] (float32, on the device), computed while the output is written."""
        self._check_f(f)
        if out is None:
            out = torch.empty((f.shape[0], OUT_CHANNELS, self.H, self.W), dtype=torch.float32, device=f.device)
        if not identity:
            tvspec_net_forward(self._h, f, out, stream)
            return out
        err = torch.empty((f.shape[0],), dtype=torch.float32, device=f.device)
        tvspec_net_forward_checked(self._h, f, out, err, stream)
        return out, err

    def train_step(self, f, bands, residual, lr, stream=None, sync=True):
        self._check_f(f)
        self._check_target(f, bands, residual)
        return tvspec_net_train_step(self._h, f, bands, residual, lr, stream, sync)

    def last_loss(self, stream=None):
        return tvspec_net_last_loss(self._h, stream)

    def loss_grad(self, f, bands, residual, grads=True, stream=None):
        self._check_f(f)
        self._check_target(f, bands, residual)
        return tvspec_net_loss_grad(self._h, f, bands, residual, grads, stream)

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            tvspec_net_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
