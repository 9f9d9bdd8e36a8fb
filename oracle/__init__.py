"""Plain FP64 CPU oracle of the VLBM for MHD -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never touches it, and it never touches the product path: the two
share no code, header, table or constant.

* ``vlbm_ref.c`` -- the lattice Boltzmann update of the paper (Sec. 2.2-2.3),
  two-lattice push streaming, FP64, OpenMP over cells.
* ``conv_ref.py`` -- the learned-correction network, restriction and gate in
  FP64 numpy (plain shifted sums).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libvlbm_ref.so")

KMAX = 26


_SO32 = os.path.join(_HERE, "libvlbm_ref_f32.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, IEEE semantics, OpenMP), and the same
    source with every double replaced by float: the oracle's formulas evaluated in
    FP32 arithmetic, the yardstick of what FP32 evaluation of the method can reach
    (used only to derive FP32 tolerances)."""
    gen = os.path.join(_HERE, "_build")
    os.makedirs(gen, exist_ok=True)
    for name in ("vlbm_ref.c", "vlbm_ref.h"):
        with open(os.path.join(_HERE, name)) as fh:
            text = fh.read().replace("double", "float").replace("fabs(", "fabsf(")
        with open(os.path.join(gen, name), "w") as fh:
            fh.write(text)
    newest = max(os.path.getmtime(os.path.join(_HERE, n)) for n in ("vlbm_ref.c", "vlbm_ref.h"))
    for out, src in ((_SO, _HERE), (_SO32, gen)):
        if force or not os.path.exists(out) or os.path.getmtime(out) < newest:
            tmp = out + ".tmp"
            subprocess.check_call(
                ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-I", src,
                 "-o", tmp, os.path.join(src, "vlbm_ref.c"), "-lm"])
            os.replace(tmp, out)
    return _SO


class Params(ctypes.Structure):
    """Mirror of ``vref_params`` in ``vlbm_ref.h``."""

    _fields_ = [
        ("dim", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("powell", ctypes.c_int32),
        ("divb_mode", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("s", ctypes.c_double),
        ("w0", ctypes.c_double),
        ("tau", ctypes.c_double * KMAX),
        ("dt", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("eta0", ctypes.c_double),
        ("j_c", ctypes.c_double),
        ("tau_M", ctypes.c_double),
        ("tau_H", ctypes.c_double),
        ("bc", ctypes.c_int32 * 6),
        ("body", ctypes.c_int32),
        ("inflow_Q", ctypes.c_double * 8),
        ("body_c0", ctypes.c_double * 3),
        ("body_v", ctypes.c_double * 3),
        ("body_R0", ctypes.c_double),
        ("body_a", ctypes.c_double * 4),
        ("body_d", (ctypes.c_double * 3) * 4),
        ("body_b", ctypes.c_double * 4),
        ("body_e", (ctypes.c_double * 3) * 4),
        ("body_m", ctypes.c_double * 3),
        ("collision", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
        ("trt_magic", ctypes.c_double),
        ("lame_lambda", ctypes.c_double),
        ("lame_mu", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("mrt_tau_e", ctypes.c_double),
        ("mrt_tau_d", ctypes.c_double),
        ("source", ctypes.c_int32),
        ("reserved3", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER(Params)
        dp = ctypes.POINTER(ctypes.c_double)
        L.vref_nvars.argtypes = [P]
        L.vref_ndirs.argtypes = [P]
        L.vref_flux_source.argtypes = [P, dp, dp, dp, dp, dp]
        L.vref_equilibrium.argtypes = [P, dp, dp]
        L.vref_equilibrium.restype = None
        L.vref_collide.argtypes = [P, dp, dp, dp]
        L.vref_collide_many.argtypes = [P, ctypes.c_long, dp, dp]
        L.vref_collide_at.argtypes = [P, ctypes.c_long, dp, ctypes.POINTER(ctypes.c_int32), ctypes.c_double, dp]
        L.vref_init.argtypes = [P, dp, dp]
        L.vref_run.argtypes = [P, dp, dp, ctypes.c_int]
        L.vref_run_src.argtypes = [P, dp, dp, dp, ctypes.c_int]
        L.vref_source_field.argtypes = [P, dp, dp]
        L.vref_moments.argtypes = [P, dp, dp, dp, dp]
        L.vref_run_bc.argtypes = [P, dp, dp, ctypes.c_int, ctypes.c_int]
        L.vref_solid.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.vref_porosity.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.vref_porosity.restype = ctypes.c_double
        L.vref_set_threads.argtypes = [ctypes.c_int]
        L.vref_set_threads.restype = None
        _lib = L
    return _lib


class use_library:
    """Temporarily route every call of this module through another build of the
    oracle (used by the tests that plant a mistake in a copy of the oracle source
    and check that the pins catch it)."""

    def __init__(self, path):
        self.path = path
        self.saved = None

    def __enter__(self):
        global _lib, _SO
        self.saved = (_lib, _SO)
        _lib, _SO = None, self.path
        return lib()

    def __exit__(self, *exc):
        global _lib, _SO
        _lib, _SO = self.saved
        return False


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile a (modified) copy of the oracle source to ``out_path``."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-I", _HERE, "-o", out_path, src, "-lm"])
    return out_path


def source_text() -> str:
    with open(os.path.join(_HERE, "vlbm_ref.c")) as fh:
        return fh.read()


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(dim=2, shape=(64, 64, 1), model=0, gamma=5.0 / 3.0, s=0.2, w0=None,
                tau=0.6, powell=1, divb_mode=0, dt=0.0, mu=0.0, eta0=0.0, j_c=0.0,
                tau_M=1.0, tau_H=1.0, collision=0, trt_magic=0.25, lame_lambda=1.0, lame_mu=1.0,
                rho0=1.0, mrt_tau_e=1.0, mrt_tau_d=1.0, source=0) -> Params:
    p = Params()
    p.dim = dim
    p.nx, p.ny, p.nz = shape
    p.model = model
    p.powell = powell
    p.divb_mode = divb_mode
    p.gamma = gamma
    p.s = s
    p.w0 = (1.0 / 3.0 if dim == 2 else 0.25) if w0 is None else w0
    if np.ndim(tau) == 0:
        taus = np.full(KMAX, float(tau))
    else:
        t = [float(v) for v in tau]
        taus = np.array(t + [t[-1]] * (KMAX - len(t)))
    for k in range(KMAX):
        p.tau[k] = float(taus[k])
    p.dt, p.mu, p.eta0, p.j_c, p.tau_M, p.tau_H = dt, mu, eta0, j_c, tau_M, tau_H
    p.collision = int(collision)
    p.trt_magic = float(trt_magic)
    p.lame_lambda, p.lame_mu, p.rho0 = float(lame_lambda), float(lame_mu), float(rho0)
    p.mrt_tau_e, p.mrt_tau_d = float(mrt_tau_e), float(mrt_tau_d)
    p.source = {"direct": 0, "guo": 1, "chai": 2}[source] if isinstance(source, str) else int(source)
    return p


def nvars(p):
    return {1: 26, 2: 5, 3: 9, 4: 13}.get(p.model, 8)


def ndirs(p):
    return 2 * p.dim + 1


def ncells(p):
    return p.nx * p.ny * p.nz


def init(p, Q):
    """f := f^eq(Q); Q is [K, nz, ny, nx] or [K, N]; returns f [K, Q, N]."""
    K, NQ, N = nvars(p), ndirs(p), ncells(p)
    Q = np.ascontiguousarray(np.asarray(Q, np.float64).reshape(K, N))
    f = np.empty((K, NQ, N), np.float64)
    lib().vref_init(ctypes.byref(p), _ptr(Q), _ptr(f))
    return f


def run(p, f, nsteps, sprev=None):
    """Advance populations f [K, Q, N] in place by nsteps; returns #unphysical cell-steps.
    sprev [K, N]: the Chai source's previous-step source (required for p.source == 2,
    updated in place; start it with source_field)."""
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
    work = np.empty_like(f)
    if p.source == 2:
        assert sprev is not None and sprev.dtype == np.float64 and sprev.flags["C_CONTIGUOUS"]
    return lib().vref_run_src(ctypes.byref(p), _ptr(f), _ptr(work), _ptr(sprev), int(nsteps))


def source_field(p, f):
    """The source S~ [K, N] of the state held by f (the Chai scheme's starting sprev)."""
    out = np.empty((nvars(p), ncells(p)), np.float64)
    lib().vref_source_field(ctypes.byref(p), _ptr(np.ascontiguousarray(f)), _ptr(out))
    return out


def set_boundaries(p, bc=None, inflow_Q=None, body=None, body_mode=1):
    """bc: 6 face kinds (0 periodic, 1 inflow, 2 zero gradient); body: dict with c0, v,
    R0, a[4], d[4][3], b[4], e[4][3], m[3] (or None); body_mode 1 bounce-back,
    2 homogenized."""
    if bc is not None:
        for j in range(6):
            p.bc[j] = int(bc[j])
    if inflow_Q is not None:
        for k in range(8):
            p.inflow_Q[k] = float(inflow_Q[k])
    p.body = 0
    if body is not None:
        p.body = int(body_mode)
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


def run_bc(p, f, nsteps, t0=0):
    """Advance f in place with the boundary kinds / body of p; returns #bad cell-steps."""
    assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
    work = np.empty_like(f)
    return lib().vref_run_bc(ctypes.byref(p), _ptr(f), _ptr(work), int(nsteps), int(t0))


def solid_mask(p, t):
    m = np.zeros((p.nz, p.ny, p.nx), np.uint8)
    for z in range(p.nz):
        for y in range(p.ny):
            for x in range(p.nx):
                m[z, y, x] = lib().vref_solid(ctypes.byref(p), x, y, z, float(t))
    return m


def porosity(p, t):
    """Lattice porosity d [nz, ny, nx] of the homogenized body at time t."""
    L = lib()
    d = np.empty((p.nz, p.ny, p.nx))
    for z in range(p.nz):
        for y in range(p.ny):
            for x in range(p.nx):
                d[z, y, x] = L.vref_porosity(ctypes.byref(p), x, y, z, float(t))
    return d


def moments(p, f):
    """Returns (Q [K, N], dlat [N], totals [K+5])."""
    K, N = nvars(p), ncells(p)
    Q = np.empty((K, N), np.float64)
    d = np.empty(N, np.float64)
    t = np.empty(K + 5, np.float64)
    lib().vref_moments(ctypes.byref(p), _ptr(np.ascontiguousarray(f)), _ptr(Q), _ptr(d), _ptr(t))
    return Q, d, t


def collide(p, fcell):
    """One-cell collision: fcell [K, Q] -> (fstar [K, Q], dlat, bad)."""
    fcell = np.ascontiguousarray(fcell, np.float64)
    out = np.empty_like(fcell)
    dl = ctypes.c_double(0.0)
    bad = lib().vref_collide(ctypes.byref(p), _ptr(fcell), _ptr(out), ctypes.byref(dl))
    return out, dl.value, bad


def collide_many(p, fcells):
    """Collision of n independent cells: fcells [n, K, Q] -> fstar [n, K, Q]."""
    fcells = np.ascontiguousarray(fcells, np.float64)
    out = np.empty_like(fcells)
    lib().vref_collide_many(ctypes.byref(p), fcells.shape[0], _ptr(fcells), _ptr(out))
    return out


def collide_at(p, fcells, xyz, t):
    """Collision of n cells fcells [n, K, Q] at coordinates xyz [n, 3] and time t
    (homogenized toward the body if p.body == 2) -> fstar [n, K, Q]."""
    fcells = np.ascontiguousarray(fcells, np.float64)
    xyz = np.ascontiguousarray(xyz, np.int32)
    out = np.empty_like(fcells)
    lib().vref_collide_at(ctypes.byref(p), fcells.shape[0], _ptr(fcells),
                          xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(t), _ptr(out))
    return out


def equilibrium(p, Qcell):
    Qcell = np.ascontiguousarray(Qcell, np.float64)
    out = np.empty((nvars(p), ndirs(p)), np.float64)
    lib().vref_equilibrium(ctypes.byref(p), _ptr(Qcell), _ptr(out))
    return out


def flux_source(p, Qcell, J=None):
    K = nvars(p)
    Qcell = np.ascontiguousarray(Qcell, np.float64)
    J = np.zeros((K, 3)) if J is None else np.ascontiguousarray(J, np.float64)
    Phi = np.empty((K, 3))
    S = np.empty(K)
    dl = ctypes.c_double(0.0)
    bad = lib().vref_flux_source(ctypes.byref(p), _ptr(Qcell), _ptr(J), _ptr(Phi), _ptr(S),
                                 ctypes.byref(dl))
    return Phi, S, dl.value, bad


def num_threads():
    return lib().vref_num_threads()


def set_threads(n):
    """Number of OpenMP threads of the oracle's loops from now on."""
    lib().vref_set_threads(int(n))


def _as_f32(t):
    if t is ctypes.c_double:
        return ctypes.c_float
    if hasattr(t, "_length_"):
        return _as_f32(t._type_) * t._length_
    return t


class Params32(ctypes.Structure):
    """``vref_params`` of the FP32-arithmetic build (every double is a float)."""

    _fields_ = [(n, _as_f32(t)) for n, t in Params._fields_]


def _copy_struct(src, dst):
    """Field-by-field copy between the FP64 and FP32 parameter mirrors."""
    def cp(a, b):
        for j in range(len(a)):
            if hasattr(a[j], "__len__"):
                cp(a[j], b[j])
            else:
                b[j] = a[j]
    for n, _ in Params._fields_:
        v = getattr(src, n)
        if hasattr(v, "__len__"):
            cp(v, getattr(dst, n))
        else:
            setattr(dst, n, v)


def run_fp32(p, Q, nsteps):
    """The oracle's update evaluated entirely in FP32 (init, nsteps steps); returns
    the moments [K, N] as float64.  A precision yardstick, not a reference."""
    if not os.path.exists(_SO32):
        build(force=True)
    L = ctypes.CDLL(_SO32)
    fp = ctypes.POINTER(ctypes.c_float)
    q = Params32()
    _copy_struct(p, q)
    K, NQ, N = nvars(p), ndirs(p), ncells(p)
    Q32 = np.ascontiguousarray(np.asarray(Q, np.float64).reshape(K, N), np.float32)
    f = np.empty((K, NQ, N), np.float32)
    work = np.empty_like(f)
    L.vref_init(ctypes.byref(q), Q32.ctypes.data_as(fp), f.ctypes.data_as(fp))
    sp = None
    if p.source == 2:
        sp = np.empty((K, N), np.float32)
        L.vref_source_field(ctypes.byref(q), f.ctypes.data_as(fp), sp.ctypes.data_as(fp))
    L.vref_run_src(ctypes.byref(q), f.ctypes.data_as(fp), work.ctypes.data_as(fp),
                   sp.ctypes.data_as(fp) if sp is not None else None, int(nsteps))
    out = np.empty((K, N), np.float32)
    L.vref_moments(ctypes.byref(q), f.ctypes.data_as(fp), out.ctypes.data_as(fp), None, None)
    return out.astype(np.float64)


def body_loads(p, f, t):
    """What one homogenized step at time t moves from the fluid to the body, and the
    magnetic flux through the body's surface -- the per-step integrals the paper's
    showcase reports (Sec. 5: net magnetic flux, force, torque, electromagnetic work),
    for the homogenized body of Sec. 2.4.

    The collision relaxes every conserved variable toward its homogenized value, so a
    cell's zeroth moments change by omega_k (Q^_k - Q_k): momentum by omega_m rho (u^ - u)
    = omega_m rho (1 - d) (u^B - u), energy by omega_E (e^ - e_tot) (rho and p kept,
    e^ = p/(gamma-1) + rho|u^|^2/2 + |B^|^2/2).  The body receives the opposite:
    force = -sum omega_m rho (u^ - u), torque = -sum (x - c(t)) x omega_m rho (u^ - u)
    about the body's centre, work = -sum omega_E (e^ - e_tot) (all per step, cell volume
    1, flux units).  omega_k: 1/tau_k (BGK), 1/tau+_k (TRT: the zeroth moment is carried
    by the symmetric halves), 1 (RLB: f* = f^eq(Q^) + ..., whose zeroth moment is Q^).
    Flux: half the surface integral of |B . n|, the surface measure being |grad d| dV,
    1 across the one-cell ramp 0 < d < 1 of the porosity: flux = 1/2 sum_ramp |B . r/|r||.
    Returns dict(force [3], torque [3], work, flux)."""
    K = nvars(p)
    Q, _, _ = moments(p, f)
    Q = Q.reshape(K, p.nz, p.ny, p.nx)
    d = porosity(p, t)
    c = np.array([p.body_c0[a] + t * p.body_v[a] for a in range(3)])
    z, y, x = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
    r = np.stack([x - c[0], y - c[1], z - c[2]]).astype(np.float64)
    r2 = (r ** 2).sum(0)
    m = np.array([p.body_m[a] for a in range(3)])
    R0 = p.body_R0
    with np.errstate(divide="ignore", invalid="ignore"):
        mr = (m[:, None, None, None] * r).sum(0)
        Bout = (3.0 * mr * r - m[:, None, None, None] * r2) / r2 ** 2.5
    Bin = np.broadcast_to((2.0 * m / R0 ** 3)[:, None, None, None], r.shape)
    BB = np.where(r2 < R0 * R0, Bin, Bout)
    rho, E, B = Q[0], Q[4], Q[5:8]
    u = Q[1:4] / rho
    gm1 = p.gamma - 1.0
    pres = gm1 * (E - 0.5 * rho * (u ** 2).sum(0) - 0.5 * (B ** 2).sum(0))
    ub = np.array([p.body_v[a] for a in range(3)]) / p.s
    uh = d * u + (1.0 - d) * ub[:, None, None, None]
    Bh = d * B + np.where(d < 1.0, (1.0 - d) * BB, 0.0)
    Eh = pres / gm1 + 0.5 * rho * (uh ** 2).sum(0) + 0.5 * (Bh ** 2).sum(0)
    tau = np.array([p.tau[k] for k in range(K)])
    if p.collision == 0:
        om = 1.0 / tau
    elif p.collision == 1:
        om = 1.0 / (0.5 + p.trt_magic / (tau - 0.5))
    else:
        om = np.ones(K)
    dM = om[1:4, None, None, None] * rho * (uh - u)
    dM = np.where(d < 1.0, dM, 0.0)
    dE = np.where(d < 1.0, om[4] * (Eh - E), 0.0)
    force = -dM.reshape(3, -1).sum(1)
    torque = -np.cross(r, dM, axis=0).reshape(3, -1).sum(1)
    ramp = (d > 0.0) & (d < 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        Bn = np.abs((B * r).sum(0)) / np.sqrt(r2)
    flux = 0.5 * Bn[ramp].sum()
    return dict(force=force, torque=torque, work=-dE.sum(), flux=flux)
