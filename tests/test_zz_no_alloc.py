"""lbm_backward_static (the adjoint entry point that allocates nothing: its
workspace is the library's static device scratch) against lbm_backward with
a caller workspace, through the C ABI: two calls in a row, the second on a
smaller grid, and the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2003_06342_amd import inputs as I
from paper_2003_06342_amd import lbm
from tests._parity import need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu


def _case(nx, ny, h0):
    prm = I.film2d_params(nx, ny)
    prm["gravity"] = [0.0, -2e-4, 0.0]
    phi0, T0, _ = I.film2d_fields(prm, seed=2, h0=h0, amp=1.5)
    return prm, phi0, T0, I.wall_T_row(nx, seed=3)


def _grads(prm, phi0, T0, Tw, n, storage, static):
    sim = lbm.Sim(prm, storage)
    sim.set_wall_T(1, 0, Tw)
    sim.init(phi0, T0)
    sim.forward_taped(n)
    N = prm["nx"] * prm["ny"]
    gphi = np.full((prm["ny"], prm["nx"]), 1.0 / N)
    gT = np.linspace(0.0, 1.0, N).reshape(prm["ny"], prm["nx"]) / N
    if static:
        g = sim.backward_static(gphi, gT=gT)
        out = {k: v.cpu().numpy() for k, v in g.items()}
    else:
        # lbm_backward with a caller workspace whose bytes start as 0xff (NaN
        # in FP32 and FP64): the entry point may not rely on zeroed memory
        n_ws = C.c_size_t()
        lbm._check(sim.lib.lbm_adjoint_workspace_size(sim.ctx, C.byref(n_ws)))
        ws = torch.full((n_ws.value + 256,), 255, dtype=torch.uint8, device="cuda")
        ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
        dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda").contiguous()
        gp, gt = dev(gphi), dev(gT)
        ny, nx = gphi.shape
        o = {"phi0": torch.empty((ny, nx), dtype=torch.float64, device="cuda"),
             "T0": torch.empty((ny, nx), dtype=torch.float64, device="cuda"),
             "Tw": torch.empty(nx, dtype=torch.float64, device="cuda")}
        P = lambda t: C.c_void_p(t.data_ptr())
        none = C.c_void_p(None)
        lbm._check(sim.lib.lbm_backward(sim.ctx, P(gp), P(gt), none, none, lbm.LBM_DT_F64,
                                        C.c_void_p(ptr), n_ws, P(o["phi0"]), P(o["T0"]), P(o["Tw"]),
                                        1, 0, lbm.LBM_DT_F64))
        out = {k: v.cpu().numpy() for k, v in o.items()}
    sim.sync()
    sim.close()
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_static_scratch_backward_matches_workspace_backward(storage):
    need_gpu()
    # first call: 96 x 64 (ragged in x); second call: a smaller grid, so the
    # scratch still holds the first call's larger intermediates
    for (nx, ny, h0, n) in ((96, 64, 10.0, 40), (70, 40, 8.0, 25)):
        prm, phi0, T0, Tw = _case(nx, ny, h0)
        say(f"[no-alloc] {storage} {nx}x{ny} {n} steps")
        ref = _grads(prm, phi0, T0, Tw, n, storage, static=False)
        got = _grads(prm, phi0, T0, Tw, n, storage, static=True)
        errs = {k: rel_l2(got[k], ref[k]) for k in ref}
        say(f"[no-alloc] {storage} {nx}x{ny}: {errs}")
        for k, e in errs.items():
            assert np.isfinite(got[k]).all(), k
            assert e <= 1e-12, (k, errs)


def test_static_scratch_size_limit():
    need_gpu()
    prm = I.film2d_params(1024, 1024)
    sim = lbm.Sim(prm, "f64")
    n_ws = C.c_size_t()
    lbm._check(sim.lib.lbm_adjoint_workspace_size(sim.ctx, C.byref(n_ws)))
    assert n_ws.value > lbm.LBM_STATIC_SCRATCH_BYTES
    none = C.c_void_p(None)
    g = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
    st = sim.lib.lbm_backward_static(sim.ctx, C.c_void_p(g.data_ptr()), none, none, none,
                                     lbm.LBM_DT_F64, none, none, none, 1, 0, lbm.LBM_DT_F64)
    assert st == lbm.LBM_E_NOMEM
    assert b"static scratch" in sim.lib.lbm_last_error()
    sim.close()
