"""Pin P16: the oracle's reverse pass (torch.autograd through the FP64 step)
against central finite differences of the oracle itself, on tiny grids."""
import numpy as np
import pytest
import torch

from oracle.lbm_oracle import F64, Model
from paper_2003_06342_amd import inputs as I


def _loss_fn(p, T0, nsteps):
    def fn(phi0, Tw):
        M = Model(p, T_wall_faces={(1, 0): Tw.reshape(1, 1, -1)})
        st = M.init(phi0, T0)
        st = M.run(st, nsteps)
        return M.fields(st)["phi"].mean()       # vapour fraction (R23)
    return fn


def test_gradcheck_film_tiny():
    nx, ny = 6, 8
    p = I.film2d_params(nx, ny)
    p["gravity"] = [0.0, -1e-3, 0.0]
    phi0, T0, Tw = I.film2d_fields(p, seed=2, h0=3.0, amp=0.7)
    T0 = torch.tensor(T0)
    fn = _loss_fn(p, T0, 3)
    phi = torch.tensor(phi0, requires_grad=True)
    tw = torch.tensor(I.wall_T_row(nx, seed=3), requires_grad=True)
    assert torch.autograd.gradcheck(fn, (phi, tw), eps=1e-6, atol=1e-9, rtol=1e-5)


def test_dot_product_tangent_vs_adjoint():
    """<J v, w> == <v, J^T w> for the map phi0 -> phi_T (forward-mode via
    torch.func.jvp against reverse mode)."""
    nx, ny = 6, 7
    p = I.film2d_params(nx, ny)
    phi0, T0, _ = I.film2d_fields(p, seed=5, h0=3.0, amp=0.5)

    def fmap(phi):
        M = Model(p)
        st = M.run(M.init(phi, T0), 3)
        return M.fields(st)["phi"]
    x = torch.tensor(phi0)
    g = torch.Generator().manual_seed(0)
    v = torch.randn(x.shape, generator=g, dtype=F64)
    w = torch.randn(x.shape, generator=g, dtype=F64)
    _, Jv = torch.func.jvp(fmap, (x,), (v,))
    _, vjp = torch.func.vjp(fmap, x)
    JTw, = vjp(w)
    a = float((Jv * w).sum())
    b = float((v * JTw).sum())
    assert a == pytest.approx(b, rel=1e-12)
