"""ctypes binding of the denoiser's C ABI (include/mcx_nn.h).

Argument marshalling only: every step runs in libmcx's HIP kernels.  Volume
arguments are torch CUDA tensors (device memory and streams are all torch
is used for); parameters move as numpy float32 arrays.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import mcx

EXPORTS = ["mcx_nn_create", "mcx_nn_destroy", "mcx_nn_param_count", "mcx_nn_set_params",
           "mcx_nn_get_params", "mcx_nn_get_grads", "mcx_nn_get_adam", "mcx_nn_set_adam",
           "mcx_nn_forward", "mcx_nn_forward_sym", "mcx_nn_loss_grad",
           "mcx_nn_set_fused_backward", "mcx_nn_adam", "mcx_nn_train_step", "mcx_nn_mirror_xy", "mcx_nn_layer_forward",
           "mcx_nn_layer_backward"]

MCX_NN_CONV3, MCX_NN_DOWN, MCX_NN_UP = 0, 1, 2

_bound = False


def lib() -> C.CDLL:
    global _bound
    L = mcx.lib()
    if not _bound:
        vp, i32, u64, f32 = C.c_void_p, C.c_int32, C.c_uint64, C.c_float
        sig = {
            "mcx_nn_create": (C.c_int, [vp, i32, i32, i32, i32, i32, C.POINTER(vp)]),
            "mcx_nn_destroy": (None, [vp]),
            "mcx_nn_param_count": (u64, [vp]),
            "mcx_nn_set_params": (C.c_int, [vp, vp, u64]),
            "mcx_nn_get_params": (C.c_int, [vp, vp, u64]),
            "mcx_nn_get_grads": (C.c_int, [vp, vp, u64]),
            "mcx_nn_get_adam": (C.c_int, [vp, vp, vp, u64, C.POINTER(i32)]),
            "mcx_nn_set_adam": (C.c_int, [vp, vp, vp, u64, i32]),
            "mcx_nn_forward": (C.c_int, [vp, vp, vp, vp, vp]),
            "mcx_nn_forward_sym": (C.c_int, [vp, vp, vp, vp, i32, vp]),
            "mcx_nn_loss_grad": (C.c_int, [vp, vp, vp, i32, C.POINTER(C.c_double), vp]),
            "mcx_nn_set_fused_backward": (C.c_int, [vp, i32, C.POINTER(i32)]),
            "mcx_nn_adam": (C.c_int, [vp, f32, f32, f32, vp]),
            "mcx_nn_train_step": (C.c_int, [vp, vp, vp, f32, C.POINTER(C.c_double), vp]),
            "mcx_nn_mirror_xy": (C.c_int, [vp, vp, i32, i32, i32, i32, vp]),
            "mcx_nn_layer_forward": (C.c_int, [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp,
                                               i32, i32, vp, vp]),
            "mcx_nn_layer_backward": (C.c_int, [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp,
                                                vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _ptr(t) -> Optional[int]:
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(s):
    import torch
    if s is None:
        s = torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check_volume(t, numel):
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == numel


def mcx_nn_create(channels: Sequence[int], shape, device: int = 0) -> C.c_void_p:
    nz, ny, nx = shape
    ch = (C.c_int32 * len(channels))(*channels)
    out = C.c_void_p()
    mcx._check(lib().mcx_nn_create(ch, len(channels), nx, ny, nz, device, C.byref(out)))
    return out


def mcx_nn_destroy(h):
    if h:
        lib().mcx_nn_destroy(h)


def mcx_nn_param_count(h) -> int:
    return int(lib().mcx_nn_param_count(h))


def mcx_nn_set_params(h, values: np.ndarray):
    v = np.ascontiguousarray(values, np.float32)
    mcx._check(lib().mcx_nn_set_params(h, v.ctypes.data, v.size))


def mcx_nn_get_params(h) -> np.ndarray:
    out = np.empty(mcx_nn_param_count(h), np.float32)
    mcx._check(lib().mcx_nn_get_params(h, out.ctypes.data, out.size))
    return out


def mcx_nn_get_grads(h) -> np.ndarray:
    out = np.empty(mcx_nn_param_count(h), np.float32)
    mcx._check(lib().mcx_nn_get_grads(h, out.ctypes.data, out.size))
    return out


def mcx_nn_get_adam(h):
    """(m, v, step): Adam's moments as numpy float32 arrays and its step count."""
    n = mcx_nn_param_count(h)
    m, v, step = np.empty(n, np.float32), np.empty(n, np.float32), C.c_int32()
    mcx._check(lib().mcx_nn_get_adam(h, m.ctypes.data, v.ctypes.data, n, C.byref(step)))
    return m, v, int(step.value)


def mcx_nn_set_adam(h, m, v, step: int):
    m = np.ascontiguousarray(m, np.float32)
    v = np.ascontiguousarray(v, np.float32)
    if m.size != v.size:
        raise ValueError(f"m has {m.size} values and v {v.size}")
    mcx._check(lib().mcx_nn_set_adam(h, m.ctypes.data, v.ctypes.data, m.size, int(step)))


def mcx_nn_forward(h, phi_in, phi_out=None, u_out=None, stream=None):
    mcx._check(lib().mcx_nn_forward(h, _ptr(phi_in), _ptr(phi_out), _ptr(u_out), _stream(stream)))


def mcx_nn_forward_sym(h, phi_in, phi_out=None, u_out=None, nsym=8, stream=None):
    mcx._check(lib().mcx_nn_forward_sym(h, _ptr(phi_in), _ptr(phi_out), _ptr(u_out), int(nsym),
                                        _stream(stream)))


def mcx_nn_loss_grad(h, phi_in, phi_target, want_loss=True, stream=None,
                     accumulate=False) -> Optional[float]:
    loss = C.c_double()
    mcx._check(lib().mcx_nn_loss_grad(h, _ptr(phi_in), _ptr(phi_target), int(bool(accumulate)),
                                      C.byref(loss) if want_loss else None, _stream(stream)))
    return loss.value if want_loss else None


def mcx_nn_set_fused_backward(h, on: bool) -> int:
    """Switch the fused backward pass; returns the number of folded layers."""
    n = C.c_int32()
    mcx._check(lib().mcx_nn_set_fused_backward(h, int(bool(on)), C.byref(n)))
    return n.value


def mcx_nn_adam(h, lr: float, grad_scale: float = 1.0, max_norm: float = 0.0, stream=None):
    mcx._check(lib().mcx_nn_adam(h, float(lr), float(grad_scale), float(max_norm),
                                 _stream(stream)))


def mcx_nn_train_step(h, phi_in, phi_target, lr: float, want_loss=False, stream=None):
    loss = C.c_double()
    mcx._check(lib().mcx_nn_train_step(h, _ptr(phi_in), _ptr(phi_target), float(lr),
                                       C.byref(loss) if want_loss else None, _stream(stream)))
    return loss.value if want_loss else None


def mcx_nn_mirror_xy(x, op: int, out=None, stream=None):
    """One of the eight x-y symmetries of a (nz, ny, nx) float32 CUDA tensor
    (op bits: 1 mirror x, 2 mirror y, 4 swap x and y first)."""
    import torch
    if out is None:
        out = torch.empty_like(x)
    nz, ny, nx = x.shape
    mcx._check(lib().mcx_nn_mirror_xy(_ptr(x), _ptr(out), nx, ny, nz, int(op), _stream(stream)))
    return out


def mcx_nn_layer_forward(kind, shape, cin, cout, x, w, b=None, skip=None, relu=True, y=None,
                         y_f32=False, stream=None):
    nz, ny, nx = shape
    mcx._check(lib().mcx_nn_layer_forward(kind, nx, ny, nz, cin, cout, _ptr(x), _ptr(w), _ptr(b),
                                          _ptr(skip), int(bool(relu)), int(bool(y_f32)), _ptr(y),
                                          _stream(stream)))
    return y


def mcx_nn_layer_backward(kind, shape, cin, cout, x, w, gy, gx=None, gw=None, gb=None,
                          stream=None):
    nz, ny, nx = shape
    mcx._check(lib().mcx_nn_layer_backward(kind, nx, ny, nz, cin, cout, _ptr(x), _ptr(w), _ptr(gy),
                                           _ptr(gx), _ptr(gw), _ptr(gb), _stream(stream)))


def bf16_bits(x) -> np.ndarray:
    """16-bit patterns of float32 values rounded to BF16, to nearest even,
    NaNs kept quiet (the rounding the kernels apply when they pack weights)."""
    u = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7fffffff) > 0x7f800000
    rne = ((u + 0x7fff + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return np.where(nan, ((u >> 16) | 0x40).astype(np.uint16), rne)


class Denoiser:
    """The U-Net of include/mcx_nn.h on one volume shape."""

    def __init__(self, channels: Sequence[int], shape, device: int = 0):
        self.channels = tuple(int(c) for c in channels)
        self.shape = tuple(int(s) for s in shape)  # (nz, ny, nx)
        self.h = mcx_nn_create(self.channels, self.shape, device)

    @property
    def nparam(self) -> int:
        return mcx_nn_param_count(self.h)

    def set_params(self, values):
        if isinstance(values, (list, tuple)):  # [(w, b), ...] in layer order
            values = np.concatenate([np.concatenate([np.ravel(w), np.ravel(b)]) for w, b in values])
        mcx_nn_set_params(self.h, values)

    def params(self) -> np.ndarray:
        return mcx_nn_get_params(self.h)

    def grads(self) -> np.ndarray:
        return mcx_nn_get_grads(self.h)

    def save(self, path):
        """Checkpoint: parameters, Adam's moments and step count, channels and
        volume shape, as a numpy .npz archive."""
        m, v, step = mcx_nn_get_adam(self.h)
        np.savez(path, params=self.params(), adam_m=m, adam_v=v, step=np.int64(step),
                 channels=np.array(self.channels, np.int64), shape=np.array(self.shape, np.int64))

    def load(self, path):
        """Restore a checkpoint written by save() for the same channels and
        shape (read without unpickling)."""
        with np.load(path, allow_pickle=False) as z:
            if tuple(z["channels"]) != self.channels or tuple(z["shape"]) != self.shape:
                raise ValueError(f"checkpoint is for channels {tuple(z['channels'])} and shape "
                                 f"{tuple(z['shape'])}, not {self.channels} and {self.shape}")
            self.set_params(z["params"])
            mcx_nn_set_adam(self.h, z["adam_m"], z["adam_v"], int(z["step"]))

    def _weight_mask(self) -> np.ndarray:
        """True for the weight entries of the flat parameter vector (layer by
        layer: weights [taps][cin][cout], then the biases)."""
        from .workloads import denoiser_layer_shapes
        parts = []
        for _, taps, ci, co in denoiser_layer_shapes(self.channels):
            parts += [np.ones(taps * ci * co, bool), np.zeros(co, bool)]
        mask = np.concatenate(parts)
        if mask.size != self.nparam:
            raise ValueError("parameter layout does not match the network")
        return mask

    def save_inference(self, path, meta: Optional[dict] = None):
        """Inference checkpoint: the weights as the BF16 values the matrix
        cores use (round to nearest even, stored as their 16-bit patterns),
        the biases in FP32, channels, volume shape and a JSON string of
        `meta` (provenance).  Half the size of the FP32 parameters; a network
        loaded from it computes exactly what the saved one computes."""
        import json
        p = self.params().astype(np.float32)
        mask = self._weight_mask()
        np.savez(path, weights_bf16=bf16_bits(p[mask]), biases=p[~mask],
                 channels=np.array(self.channels, np.int64), shape=np.array(self.shape, np.int64),
                 meta=np.array(json.dumps(meta or {})))

    def load_inference(self, path) -> dict:
        """Parameters from save_inference() (read without unpickling); the
        Adam state is left as it is.  Returns the provenance dict."""
        import json
        with np.load(path, allow_pickle=False) as z:
            if tuple(z["channels"]) != self.channels or tuple(z["shape"]) != self.shape:
                raise ValueError(f"checkpoint is for channels {tuple(z['channels'])} and shape "
                                 f"{tuple(z['shape'])}, not {self.channels} and {self.shape}")
            mask = self._weight_mask()
            p = np.empty(mask.size, np.float32)
            p[mask] = (z["weights_bf16"].astype(np.uint32) << 16).view(np.float32)
            p[~mask] = z["biases"]
            meta = json.loads(str(z["meta"]))
        self.set_params(p)
        return meta

    def _vol(self, t):
        _check_volume(t, int(np.prod(self.shape)))
        return t

    def forward(self, phi_in, phi_out=None, u_out=None, stream=None, symmetries=1):
        """Denoise; with symmetries = 2, 4 or 8 the outputs of that many
        x-y symmetries of the input are averaged (mcx_nn_forward_sym)."""
        import torch
        self._vol(phi_in)
        if phi_out is None and u_out is None:
            phi_out = torch.empty_like(phi_in)
        if symmetries == 1:
            mcx_nn_forward(self.h, phi_in, phi_out, u_out, stream)
        else:
            mcx_nn_forward_sym(self.h, phi_in, phi_out, u_out, symmetries, stream)
        return phi_out if phi_out is not None else u_out

    def loss_grad(self, phi_in, phi_target, want_loss=True, stream=None, accumulate=False):
        return mcx_nn_loss_grad(self.h, self._vol(phi_in), self._vol(phi_target), want_loss, stream,
                                accumulate)

    def set_fused_backward(self, on: bool) -> int:
        return mcx_nn_set_fused_backward(self.h, on)

    def adam(self, lr, grad_scale=1.0, max_norm=0.0, stream=None):
        mcx_nn_adam(self.h, lr, grad_scale, max_norm, stream)

    def train_step(self, phi_in, phi_target, lr, want_loss=False, stream=None):
        return mcx_nn_train_step(self.h, self._vol(phi_in), self._vol(phi_target), lr, want_loss,
                                 stream)

    def close(self):
        if self.h:
            mcx_nn_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
