"""C-ABI checks that need no GPU: the library loads, exports every function the
public headers declare, the binding's struct mirrors the header layout, and
parameter validation rejects bad inputs before any device call."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = []
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(vlbm_[a-z0-9_]+)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def vb():
    from paper_2606_00641_amd import vlbm
    return vlbm


def test_library_exports_every_declared_symbol(vb):
    names = declared_functions()
    assert len(names) >= 14
    L = ctypes.CDLL(vb.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_params_layout_matches_header(vb, tmp_path):
    fields = [f[0] for f in vb.vlbm_params._fields_]
    src = tmp_path / "off.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "vlbm.h"\nint main(void){\n'
                   + 'printf("%zu\\n", sizeof(vlbm_params));\n'
                   + "".join(f'printf("%zu\\n", offsetof(vlbm_params, {f}));\n' for f in fields)
                   + "return 0;}\n")
    exe = tmp_path / "off"
    subprocess.check_call(["gcc", "-I", INCLUDE, str(src), "-o", str(exe)])
    out = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert out[0] == ctypes.sizeof(vb.vlbm_params)
    for f, off in zip(fields, out[1:]):
        assert getattr(vb.vlbm_params, f).offset == off, f


def _status(vb, **kw):
    p = vb.make_params(**kw)
    ctx = ctypes.c_void_p()
    st = vb.lib().vlbm_create(ctypes.byref(p), ctypes.byref(ctx))
    msg = vb.lib().vlbm_last_error(None).decode()
    return st, msg, ctx


_QIN = [1.0, 3.0, 0.0, 0.0, 10.0, 0.3, 0.1, 0.0]
_BODY_OK = dict(c0=[4, 4, 4], v=[0, 0, 0], R0=2.0, a=[0] * 4, d=[[1, 0, 0]] * 4, b=[0] * 4, e=[[1, 0, 0]] * 4,
                m=[0, 0, 0])
_BODY_NEG = dict(_BODY_OK, R0=-1.0)


@pytest.mark.parametrize("kw,needle", [
    (dict(tau=0.5), "tau"),
    (dict(tau=float("nan")), "tau"),
    (dict(gamma=1.0), "gamma"),
    (dict(flux_scale=0.0), "flux_scale"),
    (dict(shape=(0, 4, 1)), "extent"),
    (dict(model="resistive"), "D3Q7"),
    (dict(storage=7), "storage"),
    (dict(lattice="D3Q7", shape=(8, 8, 8), model="resistive", dt=0.0, tau_M=0.01, tau_H=0.01), "tau_M"),
    (dict(divb_mode=1), "divb_mode"),
    (dict(block_x=100), "block_x"),
    (dict(shape=(2048, 2048, 1024), lattice="D3Q7"), "2^31"),
    (dict(lattice="D3Q7", shape=(8, 8, 8), bc=(1, 0, 0, 0, 0, 0), inflow_Q=_QIN), "neither"),
    (dict(lattice="D3Q7", shape=(8, 8, 8), bc=(3, 3, 0, 0, 0, 0), inflow_Q=_QIN), "vlbm_bc"),
    (dict(bc=(1, 2, 0, 0, 0, 0), inflow_Q=_QIN), "D3Q7 ideal"),
    (dict(lattice="D3Q7", shape=(8, 8, 8), model="resistive", dt=0.1, bc=(1, 2, 0, 0, 0, 0), inflow_Q=_QIN),
     "D3Q7 ideal"),
    (dict(lattice="D3Q7", shape=(2, 8, 8), bc=(1, 2, 0, 0, 0, 0), inflow_Q=_QIN), ">= 3"),
    (dict(lattice="D3Q7", shape=(8, 8, 8), bc=(1, 2, 0, 0, 0, 0), inflow_Q=[0.0] * 8), "density"),
    (dict(lattice="D3Q7", shape=(8, 8, 8), body=_BODY_NEG), "body_R0"),
    (dict(body=_BODY_OK), "D3Q7 ideal"),
])
def test_create_rejects_bad_parameters(vb, kw, needle):
    st, msg, ctx = _status(vb, **kw)
    assert st == vb.VLBM_ERR_ARG
    assert ctx.value is None
    assert needle in msg


def test_struct_size_mismatch_rejected(vb):
    p = vb.make_params()
    p.struct_size = 12
    ctx = ctypes.c_void_p()
    assert vb.lib().vlbm_create(ctypes.byref(p), ctypes.byref(ctx)) == vb.VLBM_ERR_ARG
    assert "ABI" in vb.lib().vlbm_last_error(None).decode()


def test_population_bytes(vb):
    p = vb.make_params(lattice="D3Q7", shape=(256, 256, 256), storage="f32")
    n = ctypes.c_size_t()
    assert vb.lib().vlbm_population_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    plane = 256 ** 3 * 4 + 4096  # 4 KiB-rounded plane plus the 4 KiB stagger
    assert n.value == 8 * 7 * plane
    p = vb.make_params(lattice="D3Q7", shape=(256, 256, 256), storage="f16", model="resistive",
                       dt=1e-3, tau_M=0.01, tau_H=0.01)
    assert vb.lib().vlbm_population_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    assert n.value == 26 * 7 * (256 ** 3 * 2 + 4096)


def test_null_safety(vb):
    L = vb.lib()
    L.vlbm_destroy(None)
    assert L.vlbm_step(None, 1) == vb.VLBM_ERR_ARG
    assert L.vlbm_create(None, None) == vb.VLBM_ERR_ARG
    assert L.vlbm_copy_kernel(None, None, 16, None) == vb.VLBM_ERR_ARG
    assert L.vlbm_body_loads(None, None) == vb.VLBM_ERR_ARG
