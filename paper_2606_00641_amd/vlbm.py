"""Python binding of the C ABI in include/vlbm.h (argument marshalling only).

Every step of the method runs in the HIP library ``libvlbm.so``; this module only
converts Python/numpy/torch arguments to the C calls of the same names.  It raises
at import time if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvlbm.so")

KMAX = 26
VLBM_OK, VLBM_ERR_ARG, VLBM_ERR_OOM, VLBM_ERR_HIP, VLBM_ERR_STATE, VLBM_ERR_NONFINITE = 0, -1, -2, -3, -4, -5
VLBM_D2Q5, VLBM_D3Q7 = 0, 1
VLBM_IDEAL, VLBM_RESISTIVE, VLBM_EULER, VLBM_NAVIER_CAUCHY, VLBM_RESISTIVE_2D = 0, 1, 2, 3, 4
VLBM_F64, VLBM_F32, VLBM_F16DEV, VLBM_BF16DEV = 0, 1, 2, 3
VLBM_BC_PERIODIC, VLBM_BC_INFLOW_EQ, VLBM_BC_ZERO_GRAD = 0, 1, 2
STORAGE = {"f64": VLBM_F64, "f32": VLBM_F32, "f16": VLBM_F16DEV, "bf16": VLBM_BF16DEV}
ELEM_BYTES = {VLBM_F64: 8, VLBM_F32: 4, VLBM_F16DEV: 2, VLBM_BF16DEV: 2}


class VlbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"vlbm status {status}: {msg}")
        self.status = status


class vlbm_params(ctypes.Structure):
    """Mirror of ``vlbm_params`` (include/vlbm.h)."""

    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("lattice", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("powell", ctypes.c_int32),
        ("divb_mode", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("flux_scale", ctypes.c_double),
        ("w0", ctypes.c_double),
        ("tau", ctypes.c_double * KMAX),
        ("dt", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("eta0", ctypes.c_double),
        ("j_c", ctypes.c_double),
        ("tau_M", ctypes.c_double),
        ("tau_H", ctypes.c_double),
        ("bc", ctypes.c_int32 * 6),
        ("inflow_Q", ctypes.c_double * 8),
        ("rest_Q", ctypes.POINTER(ctypes.c_double)),
        ("scale", ctypes.c_double * KMAX),
        ("pop_buffer", ctypes.c_void_p),
        ("pop_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("block_x", ctypes.c_int32),
        ("body", ctypes.c_int32),
        ("body_c0", ctypes.c_double * 3),
        ("body_v", ctypes.c_double * 3),
        ("body_R0", ctypes.c_double),
        ("body_a", ctypes.c_double * 4),
        ("body_d", (ctypes.c_double * 3) * 4),
        ("body_b", ctypes.c_double * 4),
        ("body_e", (ctypes.c_double * 3) * 4),
        ("body_m", ctypes.c_double * 3),
        ("collision", ctypes.c_int32),
        ("trt_magic", ctypes.c_double),
        ("lame_lambda", ctypes.c_double),
        ("lame_mu", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("mrt_tau_e", ctypes.c_double),
        ("mrt_tau_d", ctypes.c_double),
        ("source", ctypes.c_int32),
    ]


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()'); there is no CPU fallback")
    # torch is imported first so that its HIP runtime is the one the library binds to:
    # the process then holds a single runtime, shared by the library's calls and the
    # torch tensors and streams handed to it
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    P = ctypes.POINTER(vlbm_params)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    sigs = {
        "vlbm_params_default": [P],
        "vlbm_population_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "vlbm_create": [P, ctypes.POINTER(vp)],
        "vlbm_init_fields": [vp, vp, ctypes.c_int, ctypes.c_int],
        "vlbm_step": [vp, ctypes.c_int32],
        "vlbm_moments": [vp, vp, ctypes.c_int, ctypes.c_int, dp],
        "vlbm_moments_noalloc": [vp, vp, dp],
        "vlbm_gather_cells": [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp],
        "vlbm_get_populations": [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int64)],
        "vlbm_set_populations": [vp, vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64],
        "vlbm_get_codec": [vp, dp, dp],
        "vlbm_get_step": [vp, ctypes.POINTER(ctypes.c_int64)],
        "vlbm_copy_kernel": [vp, vp, ctypes.c_size_t, vp],
        "vlbm_body_loads": [vp, dp],
    }
    for name, argtypes in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = argtypes
        fn.restype = ctypes.c_int
    L.vlbm_destroy.argtypes = [vp]
    L.vlbm_destroy.restype = None
    L.vlbm_last_error.argtypes = [vp]
    L.vlbm_last_error.restype = ctypes.c_char_p
    return L


_lib = load_library()


def lib():
    return _lib


def _check(status, ctx=None):
    if status != VLBM_OK:
        msg = _lib.vlbm_last_error(ctx)
        raise VlbmError(status, msg.decode() if msg else "")
    return status


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def make_params(lattice="D2Q5", shape=(64, 64, 1), model="ideal", storage="f32", gamma=5.0 / 3.0,
                flux_scale=0.2, tau=0.6, powell=True, divb_mode=0, dt=0.0, mu=0.0, eta0=0.0,
                j_c=0.0, tau_M=1.0, tau_H=1.0, w0=0.0, bc=None, inflow_Q=None, scale=None,
                stream=None, block_x=0, body=None, collision="bgk", trt_magic=0.25, lame_lambda=1.0, lame_mu=1.0,
                rho0=1.0, mrt_tau_e=1.0, mrt_tau_d=1.0, source="direct"):
    p = vlbm_params()
    _check(_lib.vlbm_params_default(ctypes.byref(p)))
    p.lattice = VLBM_D3Q7 if str(lattice).upper() == "D3Q7" else VLBM_D2Q5
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    p.model = {"ideal": VLBM_IDEAL, "resistive": VLBM_RESISTIVE, "euler": VLBM_EULER,
               "navier_cauchy": VLBM_NAVIER_CAUCHY, "resistive_2d": VLBM_RESISTIVE_2D}[model] \
            if isinstance(model, str) \
        else int(model)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.gamma = gamma
    p.flux_scale = flux_scale
    p.w0 = w0
    taus = [float(tau)] * KMAX if np.ndim(tau) == 0 else list(map(float, tau))
    taus += [taus[-1]] * (KMAX - len(taus))
    for k in range(KMAX):
        p.tau[k] = taus[k]
    p.powell = 1 if powell else 0
    p.divb_mode = int(divb_mode)
    p.dt, p.mu, p.eta0, p.j_c, p.tau_M, p.tau_H = dt, mu, eta0, j_c, tau_M, tau_H
    if bc is not None:
        for f in range(6):
            p.bc[f] = int(bc[f])
    if inflow_Q is not None:
        for k in range(8):
            p.inflow_Q[k] = float(inflow_Q[k])
    if scale is not None:
        for k, v in enumerate(scale):
            p.scale[k] = float(v)
    p.stream = stream
    p.block_x = int(block_x)
    p.collision = {"bgk": 0, "trt": 1, "rlb": 2, "mrt": 3}[collision] if isinstance(collision, str) else int(collision)
    p.mrt_tau_e, p.mrt_tau_d = float(mrt_tau_e), float(mrt_tau_d)
    p.source = {"direct": 0, "guo": 1, "chai": 2}[source] if isinstance(source, str) else int(source)
    p.trt_magic = float(trt_magic)
    p.lame_lambda, p.lame_mu, p.rho0 = float(lame_lambda), float(lame_mu), float(rho0)
    if body is not None:
        p.body = int(body.get("mode", 1))
        for a in range(3):
            p.body_c0[a] = body["c0"][a]
            p.body_v[a] = body["v"][a]
            p.body_m[a] = body["m"][a]
        p.body_R0 = body["R0"]
        for j in range(4):
            p.body_a[j] = body["a"][j]
            p.body_b[j] = body["b"][j]
            for a in range(3):
                p.body_d[j][a] = body["d"][j][a]
                p.body_e[j][a] = body["e"][j][a]
    return p


class Vlbm:
    """Owns one ``vlbm_ctx``.  Methods map one-to-one onto the C ABI."""

    def __init__(self, params: vlbm_params, rest_Q=None, pop_tensor=None):
        self.params = params
        self._rest = None
        if rest_Q is not None:
            self._rest = np.ascontiguousarray(rest_Q, np.float64)
            params.rest_Q = _dptr(self._rest)
        self._pop_tensor = pop_tensor
        if pop_tensor is not None:
            params.pop_buffer = pop_tensor.data_ptr()
            params.pop_bytes = pop_tensor.numel() * pop_tensor.element_size()
        self.K = {VLBM_RESISTIVE: 26, VLBM_EULER: 5, VLBM_NAVIER_CAUCHY: 9, VLBM_RESISTIVE_2D: 13}.get(params.model, 8)
        self.dim = 3 if params.lattice == VLBM_D3Q7 else 2
        self.Q = 2 * self.dim + 1
        self.shape = (params.nx, params.ny, params.nz)
        self.N = params.nx * params.ny * params.nz
        ctx = ctypes.c_void_p()
        _check(_lib.vlbm_create(ctypes.byref(params), ctypes.byref(ctx)), None)
        self.ctx = ctx

    # -- C ABI -----------------------------------------------------------------
    def vlbm_init_fields(self, Q):
        """Q: numpy [K, ...] (host) or torch tensor on the GPU, FP64 or FP32."""
        if _is_torch(Q):
            Qt = Q.contiguous()
            assert Qt.numel() == self.K * self.N
            f32 = 1 if str(Qt.dtype) == "torch.float32" else 0
            _check(_lib.vlbm_init_fields(self.ctx, ctypes.c_void_p(Qt.data_ptr()), 1 if Qt.is_cuda else 0, f32),
                   self.ctx)
        else:
            Qh = np.ascontiguousarray(Q)
            if Qh.dtype not in (np.float64, np.float32):
                Qh = Qh.astype(np.float64)
            assert Qh.size == self.K * self.N, (Qh.shape, self.K, self.N)
            _check(_lib.vlbm_init_fields(self.ctx, Qh.ctypes.data_as(ctypes.c_void_p), 0,
                                         1 if Qh.dtype == np.float32 else 0), self.ctx)

    def vlbm_step(self, n):
        _check(_lib.vlbm_step(self.ctx, int(n)), self.ctx)

    def vlbm_moments(self, out=None, f32=False, with_field=True, raise_nonfinite=True):
        """Returns (Q [K, N] numpy FP64/FP32 or the given torch tensor, totals [K+5])."""
        totals = np.zeros(self.K + 5, np.float64)
        if out is not None and _is_torch(out):
            st = _lib.vlbm_moments(self.ctx, ctypes.c_void_p(out.data_ptr()), 1,
                                   1 if str(out.dtype) == "torch.float32" else 0, _dptr(totals))
            Q = out
        elif with_field:
            Q = np.empty((self.K, self.N), np.float32 if f32 else np.float64)
            st = _lib.vlbm_moments(self.ctx, Q.ctypes.data_as(ctypes.c_void_p), 0, 1 if f32 else 0,
                                   _dptr(totals))
        else:
            Q = None
            st = _lib.vlbm_moments(self.ctx, None, 0, 0, _dptr(totals))
        if st != VLBM_OK and not (st == VLBM_ERR_NONFINITE and not raise_nonfinite):
            _check(st, self.ctx)
        return Q, totals

    def vlbm_moments_noalloc(self, out):
        """vlbm_moments without device allocations: out is a torch FP64 device tensor
        of K x N values; returns (out, totals [K+5])."""
        assert _is_torch(out) and str(out.dtype) == "torch.float64" and out.is_cuda and out.is_contiguous()
        assert out.numel() == self.K * self.N
        totals = np.zeros(self.K + 5, np.float64)
        _check(_lib.vlbm_moments_noalloc(self.ctx, ctypes.c_void_p(out.data_ptr()), _dptr(totals)), self.ctx)
        return out, totals

    def vlbm_gather_cells(self, cells):
        cells = np.ascontiguousarray(cells, np.int64)
        out = np.empty((len(cells), self.K, self.Q), np.float64)
        _check(_lib.vlbm_gather_cells(self.ctx, cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      len(cells), _dptr(out)), self.ctx)
        return out

    def population_bytes(self):
        n = ctypes.c_size_t()
        _check(_lib.vlbm_population_bytes(ctypes.byref(self.params), ctypes.byref(n)))
        return n.value

    def vlbm_get_populations(self):
        nbytes = self.population_bytes()
        buf = np.empty(nbytes, np.uint8)
        par = ctypes.c_int32()
        step = ctypes.c_int64()
        _check(_lib.vlbm_get_populations(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), nbytes,
                                         ctypes.byref(par), ctypes.byref(step)), self.ctx)
        return buf, par.value, step.value

    def vlbm_set_populations(self, buf, parity, step):
        buf = np.ascontiguousarray(buf, np.uint8)
        _check(_lib.vlbm_set_populations(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes,
                                         int(parity), int(step)), self.ctx)

    def vlbm_get_codec(self):
        rest = np.zeros(self.K)
        sc = np.zeros(self.K)
        _check(_lib.vlbm_get_codec(self.ctx, _dptr(rest), _dptr(sc)), self.ctx)
        return rest, sc

    def vlbm_get_step(self):
        s = ctypes.c_int64()
        _check(_lib.vlbm_get_step(self.ctx, ctypes.byref(s)), self.ctx)
        return s.value

    def vlbm_body_loads(self):
        """Loads on the homogenized body for the next step: dict(force [3], torque [3],
        energy, flux) (include/vlbm.h)."""
        out = np.zeros(8)
        _check(_lib.vlbm_body_loads(self.ctx, _dptr(out)), self.ctx)
        return dict(force=out[0:3].copy(), torque=out[3:6].copy(), energy=float(out[6]), flux=float(out[7]))

    def vlbm_destroy(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            _lib.vlbm_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    close = vlbm_destroy

    def __del__(self):
        try:
            self.vlbm_destroy()
        except Exception:
            pass


def vlbm_copy_kernel(dst_tensor, src_tensor, stream=None):
    nbytes = min(dst_tensor.numel() * dst_tensor.element_size(), src_tensor.numel() * src_tensor.element_size())
    nbytes -= nbytes % 16
    _check(_lib.vlbm_copy_kernel(ctypes.c_void_p(dst_tensor.data_ptr()), ctypes.c_void_p(src_tensor.data_ptr()),
                                 nbytes, stream))
    return nbytes
