"""Pins of the oracle's biased directional derivatives (reading R27; Sec.
3.4, the first- and second-order upwind differences listed after Eq.
Laplacian as alternatives to the central Eq. DerivDirec_Grad).

* Polynomial exactness of the difference along a lattice velocity c: the
  first-order form phi(x + c) - phi(x) is exact on linear fields, the
  second-order form [-phi(x + 2c) + 4 phi(x + c) - 3 phi(x)] / 2 on
  quadratics; the first-order form is off by c.H.c / 2 on a quadratic.
* Convergence orders on a smooth periodic field: 1 and 2.
* Special cases that reduce to the central scheme: on a field linear in y
  whose wall value continues the line (so every ghost layer lies on it),
  one step of each scheme equals the central step to round-off; on a
  quadratic, the second-order scheme equals the central one on every node
  that no ghost reaches within the initialisation and one step.
* phi stays conserved under every scheme (the phase-field source keeps the
  central normal): the sum of phi over a periodic box without production
  after 40 steps, to round-off.
* The momentum moment of the NS source at u = 0: sum_i c_i S^f_i equals
  c_s^2 (mu G + F_n) with G the central gradient for the first-order form
  (the biased sum telescopes onto Eq. Grad) and G = 2 G_h - G_2h (central
  gradients with steps 1 and 2) for the second-order form.

A planted mistake in a subclass (the wrong sign of the -3 phi(x) term)
fails the quadratic check.
"""
import math

import numpy as np
import pytest
import torch

from oracle.lbm_oracle import F64, Macros, Model, lattice
from paper_2003_06342_amd import inputs as I


def _model(scheme, nx=12, ny=10, walls=False, cls=Model, **kw):
    p = I.base_params(dim=2, nx=nx, ny=ny, ns=True, heat=True, **I.FB)
    p["grad_scheme"] = scheme
    if walls:
        p["bc"] = ["periodic", "wall", "periodic"]
    p.update(kw)
    return cls(p)


def _macros_with_pad(M, pad2):
    """A Macros carrying only the two-layer padded phi (what cproj reads)."""
    z = torch.zeros(M.shape, dtype=F64)
    return Macros(z, [z, z, z], z, [z, z, z], z, z, [z, z, z], [z, z, z], [z, z, z], z, z, z,
                  z, z, z, z, pad2)


def _poly_pad(M, fn):
    """fn sampled on the node centres of the grid plus two ghost layers (in
    z the single plane repeats, as the periodic wrap of nz = 1 gives)."""
    nz, ny, nx = M.shape
    x = np.arange(-2, nx + 2) + 0.5
    y = np.arange(-2, ny + 2) + 0.5
    X, Y = np.meshgrid(x, y)
    return torch.tensor(np.repeat(fn(X, Y)[None], nz + 4, axis=0), dtype=F64)


def _interior(a):
    return a[0]


@pytest.mark.parametrize("scheme,exact_on", [("biased1", "linear"), ("biased2", "quadratic")])
def test_directional_difference_exact_on_polynomials(scheme, exact_on):
    M = _model(scheme)
    if exact_on == "linear":
        fn = lambda X, Y: 0.3 + 0.07 * X - 0.11 * Y
        grad = lambda X, Y: (0.07 + 0 * X, -0.11 + 0 * Y)
    else:
        fn = lambda X, Y: 0.3 + 0.07 * X - 0.11 * Y + 0.013 * X * X - 0.021 * X * Y + 0.008 * Y * Y
        grad = lambda X, Y: (0.07 + 0.026 * X - 0.021 * Y, -0.11 - 0.021 * X + 0.016 * Y)
    m = _macros_with_pad(M, _poly_pad(M, fn))
    nz, ny, nx = M.shape
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    gx, gy = grad(X, Y)
    for c in lattice("D2Q9").c[1:]:
        d = _interior(M.cproj(m, c)).numpy()
        # the difference along c at x equals the derivative along c at x for
        # the first-order form on lines only; the second-order one is exact
        # on quadratics at x itself
        exact = c[0] * gx + c[1] * gy
        assert np.abs(d - exact).max() < 1e-13, (c, np.abs(d - exact).max())


def test_first_order_difference_misses_curvature():
    """phi(x + c) - phi(x) on a quadratic is c.grad + c.H.c / 2: the half
    curvature term, which the second-order form removes."""
    M = _model("biased1")
    a, b = 0.013, 0.008
    fn = lambda X, Y: a * X * X + b * Y * Y
    m = _macros_with_pad(M, _poly_pad(M, fn))
    nz, ny, nx = M.shape
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    for c in lattice("D2Q9").c[1:]:
        d = _interior(M.cproj(m, c)).numpy()
        exact = c[0] * 2 * a * X + c[1] * 2 * b * Y
        assert np.allclose(d - exact, a * c[0] ** 2 + b * c[1] ** 2, atol=1e-13)


@pytest.mark.parametrize("scheme,order", [("biased1", 1), ("biased2", 2)])
def test_convergence_order_on_smooth_field(scheme, order):
    errs = []
    for n in (16, 32, 64):
        M = _model(scheme, nx=n, ny=n)
        k = 2 * math.pi / n
        m = _macros_with_pad(M, _poly_pad(M, lambda X, Y: np.sin(k * X) * np.cos(2 * k * Y)))
        X, Y = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5)
        e = 0.0
        for c in lattice("D2Q9").c[1:]:
            exact = c[0] * k * np.cos(k * X) * np.cos(2 * k * Y) \
                - c[1] * 2 * k * np.sin(k * X) * np.sin(2 * k * Y)
            # derivatives per lattice spacing; compare relative to the scale k
            e = max(e, np.abs(_interior(M.cproj(m, c)).numpy() - exact).max() / k)
        errs.append(e)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.15 for r in rates), (errs, rates)


def _step_once(M, phi0, T0):
    st = M.step(M.init(phi0, T0))
    return st


def test_linear_field_all_schemes_agree_after_one_step():
    """phi linear in y with phi_w at the walls on the same line: every ghost
    layer continues the line, every directional difference is exact, so the
    first step is the same for all three schemes."""
    nx, ny = 8, 12
    b = 0.06
    a0 = 0.2
    y = np.arange(ny) + 0.5
    phi = np.broadcast_to((a0 + b * y)[:, None], (ny, nx))[None].copy()
    T0 = np.full_like(phi, 0.4) + 0.05 * phi
    wall = dict(phi_wall=[[0.0, 0.0], [a0, a0 + b * ny], [0.0, 0.0]])
    out = {}
    for scheme in ("central", "biased1", "biased2"):
        M = _model(scheme, nx=nx, ny=ny, walls=True, **wall)
        st = _step_once(M, phi, T0)
        out[scheme] = torch.cat([st.f, st.g, st.s]).numpy()
    for scheme in ("biased1", "biased2"):
        d = np.abs(out[scheme] - out["central"]).max()
        assert d < 1e-14, (scheme, d)
    # and the schemes do act: on a curved field they differ
    phi_c = phi + 0.03 * np.sin(2 * np.pi * (np.arange(nx) + 0.5) / nx)[None, None, :]
    r = {}
    for sch in ("central", "biased1"):
        st = _step_once(_model(sch, nx=nx, ny=ny, walls=True, **wall), phi_c, T0)
        r[sch] = torch.cat([st.f, st.g, st.s]).numpy()
    assert np.abs(r["biased1"] - r["central"]).max() > 1e-6


def test_quadratic_field_second_order_equals_central_away_from_ghosts():
    nx, ny = 10, 14
    y = np.arange(ny) + 0.5
    x = np.arange(nx) + 0.5
    prof = 0.2 + 0.05 * y - 0.0021 * y * y
    phi = np.broadcast_to(prof[:, None], (ny, nx))[None] + 0.0 * x[None, None, :]
    T0 = 0.3 + 0.1 * phi
    st = {}
    for scheme in ("central", "biased2"):
        M = _model(scheme, nx=nx, ny=ny, walls=True)
        st[scheme] = _step_once(M, phi, T0)
    # the initial f differs on rows 0, 1 (their differences reach ghosts);
    # the step's u there enters div(u phi) on row 2, whose s collides
    # differently; rows 4 .. ny - 5 receive populations collided at rows
    # 3 .. ny - 4 only, which see neither
    sl = slice(4, ny - 4)
    for fam in ("f", "g", "s"):
        a = getattr(st["biased2"], fam)[:, 0, sl]
        c = getattr(st["central"], fam)[:, 0, sl]
        assert float((a - c).abs().max()) < 1e-14, fam


@pytest.mark.parametrize("scheme", ["biased1", "biased2"])
def test_momentum_moment_of_ns_source_at_rest(scheme):
    """u = 0 (init, NS on, no flow): sum_i c_i S^f_i against the closed form."""
    nx = ny = 12
    M = _model(scheme, nx=nx, ny=ny, gravity=[0.0, -1e-3, 0.0])
    k = 2 * math.pi / nx
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    phi = torch.tensor((0.5 + 0.3 * np.sin(k * X) * np.cos(k * Y))[None], dtype=F64)
    P = M.ghost_pad(phi, "phi")
    gphi = M.grad(P)
    lphi = M.laplacian(P, phi)
    mu, rho, F = M.forces(phi, gphi, lphi)
    z = torch.zeros_like(phi)
    m = Macros(phi, gphi, lphi, [z, z, z], mu, rho,
               [(M.rho_g - M.rho_l) * g for g in gphi], F, [z, z, z], z, z, z, z, z, z, z,
               M.ghost_pad_wide(phi, "phi", 2))
    _, S = M.f_terms(m)
    L = M.Lf
    mom = [sum(L.c[i][a] * S[i] for i in range(L.Q) if L.c[i][a]) for a in range(2)]
    ph = phi[0].numpy()

    def central(step):   # (1/c_s^2) sum_i w_i c_i phi(x + step c_i) / step
        g = [np.zeros_like(ph), np.zeros_like(ph)]
        for i in range(1, 9):
            c = L.c[i]
            sh = np.roll(ph, (-step * c[1], -step * c[0]), axis=(0, 1))
            for a in range(2):
                g[a] += L.w[i] * c[a] * sh / (L.cs2 * step)
        return g
    G = central(1) if scheme == "biased1" else [2 * a - b for a, b in zip(central(1), central(2))]
    Fn = [(rho - M.rho_l) * M.grav[a] for a in range(2)]
    for a in range(2):
        expect = L.cs2 * (mu[0].numpy() * G[a] + Fn[a][0].numpy())
        assert np.abs(mom[a][0].numpy() - expect).max() < 1e-15, (scheme, a)


class _WrongSign(Model):
    """Planted mistake: +3 phi(x) in the second-order difference."""

    def cproj(self, m, c):
        if self.grad_scheme != "biased2" or all(x == 0 for x in c):
            return super().cproj(m, c)
        nz, ny, nx = self.shape

        def at(k):
            return m.phi_pad2[2 + k * c[2]:2 + k * c[2] + nz, 2 + k * c[1]:2 + k * c[1] + ny,
                              2 + k * c[0]:2 + k * c[0] + nx]
        return 0.5 * (-at(2) + 4.0 * at(1) + 3.0 * at(0))


def test_planted_sign_error_fails_quadratic_check():
    M = _model("biased2", cls=_WrongSign)
    fn = lambda X, Y: 0.3 + 0.07 * X - 0.11 * Y + 0.013 * X * X
    m = _macros_with_pad(M, _poly_pad(M, fn))
    nz, ny, nx = M.shape
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    c = (1, 0, 0)
    d = _interior(M.cproj(m, c)).numpy()
    assert np.abs(d - (0.07 + 0.026 * X)).max() > 0.1


@pytest.mark.parametrize("scheme", ["biased1", "biased2"])
def test_phi_conserved_under_biased_schemes(scheme):
    nx, ny = 24, 20
    p = I.base_params(dim=2, nx=nx, ny=ny, ns=True, heat=True, phase_change=False, **I.FB)
    p["grad_scheme"] = scheme
    p["gravity"] = [0.0, -2e-4, 0.0]
    M = Model(p)
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    r = np.sqrt((X - 11.3) ** 2 + (Y - 9.1) ** 2)
    phi0 = (0.5 * (1 - np.tanh(2 * (r - 6.0) / 4.0)))[None]
    T0 = 0.2 + 0.1 * np.cos(2 * np.pi * X / nx)[None]
    st0 = M.init(phi0, T0)
    st = M.run(st0, 40)
    m0, m1 = float(M.macros(st0).phi.sum()), float(M.macros(st).phi.sum())
    assert abs(m1 - m0) <= 1e-13 * abs(m0), (m0, m1)
    # the scheme acts: the flow differs from the central run
    pc = dict(p, grad_scheme="central")
    Mc = Model(pc)
    uc = Mc.macros(Mc.run(Mc.init(phi0, T0), 40)).u[0]
    assert float((M.macros(st).u[0] - uc).abs().max()) > 1e-8
