"""The largest 2-D grids the library accepts: the 2-D kernels address a
population family (nine planes) with 32-bit byte offsets, so 9 x pitch x ny
x element size must stay below 2^32.  At nx = 16384 this allows ny = 7281
for FP32, 3640 for FP64 and 14563 for 16-bit storage; one more row is
rejected.  Two steps of a film whose interface runs along the top rows (the
highest offsets) are compared with the oracle on 64-column windows at the
floor and at the top, one across the periodic seam, more than 11 nodes (two
steps' reach) inside each window's artificial edges: FP64 within 1e-10,
FP32 within max(1e-5, 3 x the windows' float32 floor) (the pressure about
its mean varies little inside a 40-node window, so its relative error sits
at the FP32 rounding of p), FP16 within the 16-bit bars."""
import numpy as np
import pytest
import torch

from oracle.lbm_oracle import Model
from paper_2003_06342_amd import inputs as I
from tests._parity import compare, need_gpu, say

pytestmark = pytest.mark.gpu

NX = 16384
ELEM = {"f32": 4, "f64": 8, "f16dev": 2}


def max_rows(storage):
    return (2 ** 32 - 1) // (9 * NX * ELEM[storage])


def _window(prm, phi0, T0, n, r0, rows, c0, width, dtype=torch.float64):
    """Oracle on rows r0 .. r0+rows-1 and `width` columns from c0 (wrapped);
    the window's own walls stand in for the rows beyond it."""
    p = dict(prm, nx=width, ny=rows)
    cols = (c0 + np.arange(width)) % prm["nx"]
    M = Model(p, dtype=dtype)
    st = M.run(M.init(phi0[:, r0:r0 + rows][:, :, cols], T0[:, r0:r0 + rows][:, :, cols]), n)
    return {k: v.double().numpy() for k, v in M.fields(st).items()}


@pytest.mark.parametrize("storage", ["f32", "f64", "f16dev"])
def test_largest_accepted_2d_grid(storage):
    from paper_2003_06342_amd import lbm
    need_gpu()
    ny = max_rows(storage)
    prm = I.film2d_params(NX, ny, wavelength=512.0)
    with pytest.raises(lbm.LBMError):
        lbm.Sim(dict(prm, ny=ny + 1), storage)
    phi0, T0, _ = I.film2d_fields(prm, seed=4, h0=ny - 30.0, amp=4.0, wavelength=512.0)
    n, R, Wd, m = 2, 48, 64, 11
    keys = ("phi", "T", "ux", "uy", "uz", "p")
    wins = []
    floor = {}
    for (r0, c0) in ((0, NX - 20), (0, 7000), (ny - R, NX - 20), (ny - R, 3000)):
        ref = _window(prm, phi0, T0, n, r0, R, c0, Wd)
        # meaningful rows: away from the artificial edge (the top of a floor
        # window, the bottom of a top window) and from the window's x edges
        rs = slice(0, R - m) if r0 == 0 else slice(m, R)
        cut = lambda w: {k: w[k][:, rs, m:Wd - m] for k in keys}
        wins.append((r0, c0, rs, cut(ref)))
        if storage == "f32":   # the float32 floor of the windows: the oracle in float32
            for k, e in compare(cut(_window(prm, phi0, T0, n, r0, R, c0, Wd, torch.float32)),
                                cut(ref)).items():
                floor[k] = max(floor.get(k, 0.0), e)
    bars = {"f64": {k: 1e-10 for k in ("phi", "T", "umag", "p")},
            "f32": {k: max(1e-5, 3.0 * floor.get(k, 0.0)) for k in ("phi", "T", "umag", "p")},
            "f16dev": {"phi": 1e-4, "T": 1e-3, "umag": 1e-3, "p": 1e-3}}[storage]
    say(f"[maxsize] {storage}: {NX} x {ny}, {n} steps")
    sim = lbm.Sim(prm, storage)
    sim.init(phi0, T0)
    sim.step(n)
    f = sim.fields()
    worst = {}
    for (r0, c0, rs, ref) in wins:
        rows = torch.arange(r0, r0 + R, device=f["phi"].device)[rs]
        cols = torch.tensor(((c0 + np.arange(Wd)) % NX)[m:Wd - m], device=f["phi"].device)
        g = {k: f[k].index_select(1, rows).index_select(2, cols).double().cpu().numpy() for k in keys}
        for k, e in compare(g, ref).items():
            worst[k] = max(worst.get(k, 0.0), e)
    sim.sync()
    sim.close()
    del f
    torch.cuda.empty_cache()
    say(f"[maxsize] {storage}: worst window errors {worst} | bars {bars}")
    for k in ("phi", "T", "umag", "p"):
        assert worst[k] <= bars[k], (storage, k, worst, bars)
