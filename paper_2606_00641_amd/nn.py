"""Python binding of include/vlbm_nn.h (argument marshalling only): the learned
coarse-grid correction network, restriction and corrected coarse stepping."""
from __future__ import annotations

import ctypes

import numpy as np

from . import vlbm as _v

_lib = _v.lib()
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)

_sigs = {
    "vlbm_nn_create": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.POINTER(_vp)],
    "vlbm_nn_num_params": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "vlbm_nn_set_weights": [_vp, _fp, ctypes.c_size_t],
    "vlbm_nn_get_weights": [_vp, _fp, ctypes.c_size_t],
    "vlbm_nn_set_norm": [_vp, _dp, _dp, _dp, _dp],
    "vlbm_nn_forward": [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "vlbm_nn_loss_grad": [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dp, _fp],
    "vlbm_nn_adam_step": [_vp, ctypes.c_float],
    "vlbm_nn_adam_config": [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float],
    "vlbm_nn_train_step": [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                           ctypes.c_float, _dp],
    "vlbm_restrict": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                      ctypes.c_int32, _vp, _vp, _vp],
    "vlbm_step_corrected": [_vp, _vp, ctypes.c_int32, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int64)],
    "vlbm_inject": [_vp, _vp],
}
for _name, _args in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_int
_lib.vlbm_nn_destroy.argtypes = [_vp]
_lib.vlbm_nn_destroy.restype = None
_lib.vlbm_nn_last_error.argtypes = [_vp]
_lib.vlbm_nn_last_error.restype = ctypes.c_char_p


def _check(status, nn=None):
    if status != _v.VLBM_OK:
        msg = _lib.vlbm_nn_last_error(nn)
        raise _v.VlbmError(status, msg.decode() if msg else "")


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


def _d(a):
    a = np.ascontiguousarray(a, np.float64)
    return a, a.ctypes.data_as(_dp)


class Net:
    """Owns one ``vlbm_nn``; methods map one-to-one onto the C ABI.  dim = 2: 3x3
    kernels, fields [C, batch, ny, nx]; dim = 3: 3x3x3 kernels, fields
    [C, batch, nz, ny, nx] (torch FP32 device tensors, channel-major)."""

    def __init__(self, cin=8, width=32, layers=4, stream=None, dim=2):
        h = ctypes.c_void_p()
        _check(_lib.vlbm_nn_create(dim, cin, width, layers, stream, ctypes.byref(h)))
        self.h = h
        self.cin, self.width, self.layers, self.dim = cin, width, layers, dim

    def _shape(self, X):
        """(batch, nx, ny, nz) of a channel-major field."""
        if self.dim == 2:
            C, B, ny, nx = X.shape
            return B, nx, ny, 1
        C, B, nz, ny, nx = X.shape
        return B, nx, ny, nz

    def vlbm_nn_num_params(self):
        n = ctypes.c_size_t()
        _check(_lib.vlbm_nn_num_params(self.h, ctypes.byref(n)), self.h)
        return n.value

    def vlbm_nn_set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        _check(_lib.vlbm_nn_set_weights(self.h, w.ctypes.data_as(_fp), w.size), self.h)

    def vlbm_nn_get_weights(self):
        w = np.empty(self.vlbm_nn_num_params(), np.float32)
        _check(_lib.vlbm_nn_get_weights(self.h, w.ctypes.data_as(_fp), w.size), self.h)
        return w

    def vlbm_nn_set_norm(self, in_mean, in_std, out_mean, out_std):
        arrs = [_d(a) for a in (in_mean, in_std, out_mean, out_std)]
        _check(_lib.vlbm_nn_set_norm(self.h, *[p for _, p in arrs]), self.h)

    def vlbm_nn_forward(self, X, out):
        """X, out: torch FP32 device tensors of the network's field shape."""
        if tuple(out.shape) != tuple(X.shape):
            raise ValueError("out must have the shape of X")
        _check(_lib.vlbm_nn_forward(self.h, _dev(X), _dev(out), *self._shape(X)), self.h)
        return out

    def vlbm_nn_loss_grad(self, X, T, want_grad=True):
        loss = ctypes.c_double()
        g = np.empty(self.vlbm_nn_num_params(), np.float32) if want_grad else None
        _check(_lib.vlbm_nn_loss_grad(self.h, _dev(X), _dev(T), *self._shape(X), ctypes.byref(loss),
                                      g.ctypes.data_as(_fp) if g is not None else None), self.h)
        return loss.value, g

    def vlbm_nn_adam_step(self, lr):
        _check(_lib.vlbm_nn_adam_step(self.h, lr), self.h)

    def vlbm_nn_adam_config(self, b1=0.9, b2=0.999, eps=1e-8):
        _check(_lib.vlbm_nn_adam_config(self.h, b1, b2, eps), self.h)

    def vlbm_nn_train_step(self, X, T, lr, want_loss=False):
        loss = ctypes.c_double()
        _check(_lib.vlbm_nn_train_step(self.h, _dev(X), _dev(T), *self._shape(X), lr,
                                       ctypes.byref(loss) if want_loss else None), self.h)
        return loss.value if want_loss else None

    def vlbm_nn_destroy(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.vlbm_nn_destroy(self.h)
            self.h = ctypes.c_void_p()

    close = vlbm_nn_destroy

    def __del__(self):
        try:
            self.vlbm_nn_destroy()
        except Exception:
            pass


def vlbm_restrict(Qf, r, out, rz=None, minus=None, stream=None):
    """Qf: torch FP32 device [K, nz, ny, nx]; out: [K, nz/rz, ny/r, nx/r].  rz defaults
    to r for a 3D field (nz > 1 means 3D unless rz=1 is given for a 2D batch)."""
    K, nz, ny, nx = Qf.shape
    if rz is None:
        rz = r if nz > 1 else 1
    st = _lib.vlbm_restrict(_dev(Qf), K, nx, ny, nz, r, rz, _dev(minus) if minus is not None else None,
                            _dev(out), stream)
    if st != _v.VLBM_OK:
        raise _v.VlbmError(st, "vlbm_restrict: bad shapes")
    return out


def vlbm_step_corrected(sim, net, n, bound_corr, bound_divb_rel, bound_divb_abs=0.0, project_totals=True):
    """Advance the coarse context `sim` (a vlbm.Vlbm) n steps with the correction
    (projected to zero lattice totals unless project_totals is False); returns the
    number of fallbacks."""
    b, bp = _d(bound_corr)
    nfb = ctypes.c_int64()
    st = _lib.vlbm_step_corrected(sim.ctx, net.h, int(n), bp, float(bound_divb_rel), float(bound_divb_abs),
                                  1 if project_totals else 0, ctypes.byref(nfb))
    if st != _v.VLBM_OK:
        msg = _lib.vlbm_nn_last_error(net.h)
        raise _v.VlbmError(st, msg.decode() if msg else "")
    return nfb.value


def vlbm_inject(sim, dQ):
    """f += w_i dQ_k on the context `sim` (a vlbm.Vlbm) at its current step; dQ: torch
    FP32 device tensor [8, nz, ny, nx]."""
    st = _lib.vlbm_inject(sim.ctx, _dev(dQ))
    if st != _v.VLBM_OK:
        raise _v.VlbmError(st, "vlbm_inject: needs an initialised periodic ideal-MHD context without a body")

