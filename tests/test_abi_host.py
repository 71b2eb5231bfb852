"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/lbm.h declares, and rejects invalid parameter sets with
the documented status codes before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_2003_06342_amd import inputs as I
from paper_2003_06342_amd import lbm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    return lbm.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "lbm_step" in names and "lbm_create" in names
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_error_string(lib):
    assert b"gfx950" in lib.lbm_version()
    assert lib.lbm_last_error() is not None


def _c_layout():
    """sizeof(lbm_params) and the offset of every field, from the C header
    compiled by the host C compiler."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    names = [f[0] for f in lbm.lbm_params._fields_]
    body = "\n".join(f'  printf("{n} %zu\\n", offsetof(lbm_params, {n}));' for n in names)
    src = ("#include <stdio.h>\n#include <stddef.h>\n#include \"lbm.h\"\nint main(void){\n"
           '  printf("sizeof %zu\\n", sizeof(lbm_params));\n' + body + "\n  return 0;\n}\n")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (ln.split() for ln in out.splitlines())}


def test_struct_layout_matches_header():
    """The ctypes mirror of lbm_params has the C size and every field at the
    C offset (same order, types and padding)."""
    lay = _c_layout()
    assert C.sizeof(lbm.lbm_params) == lay["sizeof"]
    for name, _ in lbm.lbm_params._fields_:
        assert getattr(lbm.lbm_params, name).offset == lay[name], name


def _status(prm, storage="f32"):
    lib = lbm.load_library()
    p = lbm.make_params(prm, storage)
    n = C.c_size_t()
    return lib.lbm_workspace_size(C.byref(p), C.byref(n)), n.value


def test_workspace_size_valid(lib):
    prm = I.film2d_params(130, 66)
    st, n = _status(prm)
    assert st == lbm.LBM_OK
    # 27 populations x 2 buffers x pitch 192 x 66 x 4 B at least
    assert n >= 2 * 27 * 192 * 66 * 4


@pytest.mark.parametrize("key,val", [("nu_l", 0.0), ("mobility", -1.0), ("alpha_g", 0.0),
                                     ("W", 0.0), ("rho_g", 0.0)])
def test_rejects_nonpositive_transport(lib, key, val):
    prm = I.film2d_params(64, 32)
    prm[key] = val
    st, _ = _status(prm)
    assert st == lbm.LBM_E_INVAL
    assert key.encode() in lib.lbm_last_error()


def test_rejects_bad_lattice_and_dims(lib):
    prm = I.film2d_params(64, 32)
    prm["lat_g"] = "D3Q7"
    assert _status(prm)[0] == lbm.LBM_E_UNSUPPORTED
    prm = I.film2d_params(64, 32)
    prm["nz"] = 2
    assert _status(prm)[0] == lbm.LBM_E_INVAL


def test_phase_change_needs_heat(lib):
    p = lbm.make_params(I.film2d_params(16, 16), "f32")
    p.flags = lbm.LBM_NS | lbm.LBM_PHASE_CHANGE
    n = C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(p), C.byref(n)) == lbm.LBM_E_INVAL


def test_null_arguments(lib):
    assert lib.lbm_step(None, 1) == lbm.LBM_E_INVAL
    assert lib.lbm_sync(None) == lbm.LBM_E_INVAL
    out = C.c_void_p()
    p = lbm.make_params(I.film2d_params(16, 16), "f32")
    assert lib.lbm_create(C.byref(p), None, 0, None, C.byref(out)) == lbm.LBM_E_INVAL
    assert out.value is None


def test_walled_axis_needs_two_nodes(lib):
    assert _status(I.film2d_params(16, 1))[0] == lbm.LBM_E_INVAL   # y walls, one row
    assert b"walled axis" in lib.lbm_last_error()
    assert _status(I.film2d_params(16, 2))[0] == lbm.LBM_OK
    prm = I.film2d_params(1, 8)   # x periodic: one column is allowed
    assert _status(prm)[0] == lbm.LBM_OK


def test_extended_options_validated(lib):
    """MRT has no D3Q19 basis (NS in 3-D), the local div(u phi) needs the NS
    and heat families, unknown collision / gradient codes are rejected; the
    supported combinations pass."""
    p3 = I.film3d_params(32, nz=24)
    p3["collision"] = "mrt"
    assert _status(p3)[0] == lbm.LBM_E_UNSUPPORTED
    p3["ns"] = False
    assert _status(p3)[0] == lbm.LBM_OK
    p2 = I.film2d_params(16, 8)
    p2.update(div_local=True, heat=False, phase_change=False)
    assert _status(p2)[0] == lbm.LBM_E_INVAL
    p2 = I.film2d_params(16, 8)
    p2.update(div_local=True, collision="trt", grad_scheme="biased2")
    assert _status(p2)[0] == lbm.LBM_OK
    p = lbm.make_params(I.film2d_params(16, 8), "f32")
    p.collision = 7
    n = C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(p), C.byref(n)) == lbm.LBM_E_INVAL
    p = lbm.make_params(I.film2d_params(16, 8), "f32")
    p.grad_scheme = 3
    assert lib.lbm_workspace_size(C.byref(p), C.byref(n)) == lbm.LBM_E_INVAL
    p = lbm.make_params(dict(I.film2d_params(16, 8), collision="mrt",
                             mrt_rates=[[1.0] * 4, [1.0, 2.0, 1.0, 1.0], [1.0] * 4]), "f32")
    assert lib.lbm_workspace_size(C.byref(p), C.byref(n)) == lbm.LBM_E_INVAL


def test_open_faces_validated(lib):
    """An open (pressure) face of f needs a walled axis; unknown kinds and a
    non-finite face pressure are rejected; the film with an open top passes."""
    p = I.film2d_params(16, 8)
    p["f_open"] = [[False, False], [False, True], [False, False]]
    assert _status(p)[0] == lbm.LBM_OK
    p["f_open"] = [[True, False], [False, False], [False, False]]   # x is periodic
    assert _status(p)[0] == lbm.LBM_E_INVAL
    assert b"walled axis" in lib.lbm_last_error()
    q = lbm.make_params(I.film2d_params(16, 8), "f32")
    q.f_bc[1][1] = 5
    n = C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(q), C.byref(n)) == lbm.LBM_E_INVAL
    q = lbm.make_params(I.film2d_params(16, 8), "f32")
    q.f_bc[1][1] = lbm.LBM_FBC_PRESSURE
    q.p_wall[1][1] = float("nan")
    assert lib.lbm_workspace_size(C.byref(q), C.byref(n)) == lbm.LBM_E_INVAL


def test_stream_probe_library_loads_and_checks_arguments():
    """The measurement probes bench.py times beside the step (their own
    library, outside the C ABI) are built, export their launchers, and
    reject null buffers, grids below 3 x 3 and misaligned copies before any
    device call."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "benchprobe",
                        "libstream_probe.so")
    if not os.path.exists(path):
        pytest.fail("libstream_probe.so is not built (run __graft_entry__.build())")
    p = C.CDLL(path)
    f = p.stream_probe_pull_pattern
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    assert f(None, None, 64, 64, None) != 0
    assert f(C.c_void_p(16), C.c_void_p(32), 2, 64, None) != 0
    g = p.stream_probe_copy16
    g.restype = C.c_int
    g.argtypes = [C.c_void_p, C.c_void_p, C.c_longlong, C.c_int, C.c_void_p]
    assert g(None, None, 1024, 0, None) != 0
    assert g(C.c_void_p(16), C.c_void_p(32), 1000, 0, None) != 0   # not a multiple of 16
    assert g(C.c_void_p(8), C.c_void_p(32), 1024, 1, None) != 0    # misaligned source


def test_d2q5_lattice_validated(lib):
    """2-D takes D2Q5 for g and s (the same for both; f stays D2Q9), and the
    workspace holds 9 + 5 + 5 populations; mixed or 3-D use is rejected."""
    p = I.film2d_params(130, 66, lat_g="D2Q5", lat_s="D2Q5")
    st, n = _status(p)
    assert st == lbm.LBM_OK
    assert n >= 2 * 19 * 192 * 66 * 4
    assert n < _status(I.film2d_params(130, 66))[1]
    p["lat_s"] = "D2Q9"
    assert _status(p)[0] == lbm.LBM_E_UNSUPPORTED
    p = I.film2d_params(16, 8, lat_f="D2Q5", lat_g="D2Q5", lat_s="D2Q5")
    assert _status(p)[0] == lbm.LBM_E_UNSUPPORTED
    p3 = I.film3d_params(32, nz=24)
    p3["lat_g"] = "D2Q5"
    assert _status(p3)[0] == lbm.LBM_E_UNSUPPORTED
