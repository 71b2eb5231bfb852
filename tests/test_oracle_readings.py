"""Pins of oracle readings the closed-form cases do not reach.

* R13, no-slip velocity ghost u_g = -u_b in div(u phi): a manufactured
  field with u odd and phi - phi_w odd about both half-way walls, whose
  analytic extension beyond the wall is exactly the ghost rule.  The wall
  rows of the oracle's div(u phi) equal the central stencil (Eq. Grad)
  applied to the analytic extension to round-off, and converge at second
  order to the analytic divergence.
* R13, edges crossed by two walls: a hand-computed 3 x 3 box for the
  stream (the higher axis gives the anti-bounce-back value) and for the
  stencil ghosts (x ghosts first, then y ghosts of the x-padded field).
* R9, n = grad phi / sqrt(|grad phi|^2 + eps^2) with eps = 1e-3: exact on
  linear ramps over five decades of slope, and its effect on the planar
  interface of Sec. 2.1 at W = 4, 8, 16: second-order convergence to the
  tanh profile where the counter term's strength 4 phi (1 - phi) / W is
  above 10 eps, and a tail deviation below phi* = eps W / 4, the level at
  which the regularised counter flux vanishes.

* R8, div(u phi) as the central stencil of Eq. Grad on each u_a phi: its
  Fourier symbol sin(k) on a periodic lattice (D2Q9 and D3Q19), exact for a
  product of two modes.
* R10, the linear interpolation of alpha(phi): the steady series
  conduction across a static interface between walls at T = 1 and T = 0.

Each pin comes with a planted mistake in a subclass of the oracle (a flipped
ghost sign, a swapped axis order, the product rule in place of the stencil
on the product, a harmonic alpha) that the same check rejects.
"""
import math

import numpy as np
import pytest
import torch

from oracle.lbm_oracle import F64, Model
from paper_2003_06342_amd import inputs as I


# ---------------------------------------------------------------------------
# R13: no-slip velocity ghost in div(u phi)
# ---------------------------------------------------------------------------

PHI_W = 1.0


def _fields(x, y, nx, ny):
    """Manufactured u_x, u_y, phi at points (x, y): u odd and phi - phi_w
    odd about y = 0 and y = ny (both walls)."""
    s = np.sin(np.pi * y / ny)
    kx = 2 * np.pi * x / nx
    ux = 0.01 * (1 + 0.5 * np.cos(kx)) * s
    uy = 0.02 * np.sin(kx) * s
    phi = PHI_W - 0.4 * (1 + 0.3 * np.cos(kx)) * s
    return ux, uy, phi


def _div_exact(x, y, nx, ny):
    """Analytic d(u_x phi)/dx + d(u_y phi)/dy of _fields."""
    s = np.sin(np.pi * y / ny)
    ds = np.pi / ny * np.cos(np.pi * y / ny)
    k = 2 * np.pi / nx
    kx = k * x
    A, dA = 0.01 * (1 + 0.5 * np.cos(kx)), -0.005 * k * np.sin(kx)
    B, dB = 0.02 * np.sin(kx), 0.02 * k * np.cos(kx)
    C, dC = 0.4 * (1 + 0.3 * np.cos(kx)), -0.12 * k * np.sin(kx)
    phi = PHI_W - C * s
    dphidx, dphidy = -dC * s, -C * ds
    return (dA * s) * phi + (A * s) * dphidx + (B * ds) * phi + (B * s) * dphidy


def _wall_model(nx, ny, cls=Model):
    p = I.base_params(dim=2, nx=nx, ny=ny, ns=True, heat=True)
    p["bc"] = ["periodic", "wall", "periodic"]
    p["phi_wall"] = [[0.0, 0.0], [PHI_W, PHI_W], [0.0, 0.0]]
    return cls(p)


def _oracle_div(M, nx, ny):
    xc = np.arange(nx) + 0.5
    yc = np.arange(ny) + 0.5
    X, Y = np.meshgrid(xc, yc)
    ux, uy, phi = _fields(X, Y, nx, ny)
    t = lambda a: torch.tensor(a[None], dtype=F64)
    u = [t(ux), t(uy), torch.zeros(1, ny, nx, dtype=F64)]
    P = M.ghost_pad(t(phi), "phi")
    return M.divergence(u, P)[0].numpy()


def _stencil_on_extension(nx, ny):
    """Eq. Grad's central stencil on the analytic u_a phi, evaluated on node
    centres including the ghost rows y = -1/2 and y = ny + 1/2."""
    w = {(0, 0): 4 / 9}
    for c in ((1, 0), (0, 1), (-1, 0), (0, -1)):
        w[c] = 1 / 9
    for c in ((1, 1), (-1, 1), (-1, -1), (1, -1)):
        w[c] = 1 / 36
    xc = np.arange(nx) + 0.5
    yc = np.arange(ny) + 0.5
    X, Y = np.meshgrid(xc, yc)
    D = np.zeros((ny, nx))
    for (cx, cy), wi in w.items():
        if (cx, cy) == (0, 0):
            continue
        uxp, uyp, pp = _fields(X + cx, Y + cy, nx, ny)
        uxm, uym, pm = _fields(X - cx, Y - cy, nx, ny)
        D += 3 * wi * (cx * (uxp * pp - uxm * pm) + cy * (uyp * pp - uym * pm)) / 2
    return D


def test_noslip_velocity_ghost_in_divergence():
    nx, ny = 24, 20
    D = _oracle_div(_wall_model(nx, ny), nx, ny)
    ref = _stencil_on_extension(nx, ny)
    assert np.abs(D - ref).max() < 1e-15
    # the wall rows are where the ghost enters
    assert np.abs(ref[0]).max() > 1e-3 and np.abs(ref[-1]).max() > 1e-3


def test_noslip_velocity_ghost_converges_to_analytic_divergence():
    errs = []
    for n in (16, 32, 64):
        D = _oracle_div(_wall_model(n, n), n, n)
        xc = np.arange(n) + 0.5
        ex = np.stack([_div_exact(xc, 0.5, n, n), _div_exact(xc, n - 0.5, n, n)])
        errs.append(np.abs(D[[0, -1]] - ex).max() / np.abs(ex).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


class _FlippedGhost(Model):
    """Planted mistake: a velocity ghost of +u_b instead of -u_b."""

    def ghost_pad(self, v, kind):
        if kind != "anti":
            return super().ghost_pad(v, kind)
        out = v
        for a in range(3):
            d = 2 - a
            n = out.shape[d]
            first, last = out.narrow(d, 0, 1), out.narrow(d, n - 1, 1)
            lo, hi = (first, last) if self.wall[a] else (last, first)
            out = torch.cat([lo, out, hi], dim=d)
        return out


def test_flipped_velocity_ghost_is_detected():
    nx, ny = 24, 20
    D = _oracle_div(_wall_model(nx, ny, _FlippedGhost), nx, ny)
    ref = _stencil_on_extension(nx, ny)
    assert np.abs(D - ref).max() > 1e-4
    assert np.abs(D[1:-1] - ref[1:-1]).max() < 1e-15   # only the wall rows differ


# ---------------------------------------------------------------------------
# R13: edges crossed by two walls (3 x 3 box, walls on x and y)
# ---------------------------------------------------------------------------

PW = [[0.2, 0.4], [0.7, 0.9], [0.0, 0.0]]     # phi_wall[axis][side]
TW = [[0.05, 0.15], [0.35, 0.55], [0.0, 0.0]]  # T_wall[axis][side]


def _box(cls=Model):
    p = I.base_params(dim=2, nx=3, ny=3, ns=True, heat=True)
    p["bc"] = ["wall", "wall", "periodic"]
    p["phi_wall"] = PW
    p["T_wall"] = TW
    return cls(p)


def _box_phi():
    return np.array([[0.1 * (1 + x + 3 * y) for x in range(3)] for y in range(3)])


def test_box_corner_stencil_ghosts():
    M = _box()
    phi = _box_phi()
    P = M.ghost_pad(torch.tensor(phi[None]), "phi")[1].numpy()   # [y + 1][x + 1]
    # x ghosts first: P(-1, y) = 2 phi_w[x][lo] - phi(0, y); then the y ghosts
    # of the x-padded rows, corners included
    assert P[1, 0] == pytest.approx(2 * 0.2 - phi[0, 0], abs=1e-15)
    assert P[0, 1] == pytest.approx(2 * 0.7 - phi[0, 0], abs=1e-15)
    assert P[0, 0] == pytest.approx(2 * 0.7 - (2 * 0.2 - phi[0, 0]), abs=1e-15)
    assert P[0, 4] == pytest.approx(2 * 0.7 - (2 * 0.4 - phi[0, 2]), abs=1e-15)
    assert P[4, 0] == pytest.approx(2 * 0.9 - (2 * 0.2 - phi[2, 0]), abs=1e-15)
    assert P[4, 4] == pytest.approx(2 * 0.9 - (2 * 0.4 - phi[2, 2]), abs=1e-15)
    # the velocity ghosts compose the same way (two sign flips at a corner)
    U = M.ghost_pad(torch.tensor(phi[None]), "anti")[1].numpy()
    assert U[0, 0] == pytest.approx(phi[0, 0], abs=1e-15)
    assert U[0, 2] == pytest.approx(-phi[0, 1], abs=1e-15)


def _post():
    """Distinct post-collision values per population and node: [9][1][3][3]."""
    v = np.arange(9 * 9, dtype=np.float64).reshape(9, 1, 3, 3) * 0.01 + 0.003
    return torch.tensor(v)


def test_box_corner_stream_higher_axis_wins():
    M = _box()
    L = M.Lg
    post = _post()
    wall_val = [[torch.tensor(v, dtype=F64) for v in side] for side in PW]
    new = M.stream(post, L, "abb", wall_val)[:, 0].numpy()      # [i][y][x]
    pv = post[:, 0].numpy()
    i = 5                                      # c = (1, 1)
    j = L.opp[i]
    w = L.w[i]
    # node (0, 0): the source (-1, -1) is beyond both walls: the y wall's value
    assert new[i, 0, 0] == pytest.approx(-pv[j, 0, 0] + 2 * w * PW[1][0], abs=1e-15)
    # node (x=0, y=1): beyond the x wall only
    assert new[i, 1, 0] == pytest.approx(-pv[j, 1, 0] + 2 * w * PW[0][0], abs=1e-15)
    # node (x=1, y=0): beyond the y wall only
    assert new[i, 0, 1] == pytest.approx(-pv[j, 0, 1] + 2 * w * PW[1][0], abs=1e-15)
    # node (1, 1): an ordinary pull from (0, 0)
    assert new[i, 1, 1] == pytest.approx(pv[i, 0, 0], abs=1e-15)
    # the opposite corner for c = (-1, -1) (i = 7): the y wall at the top
    i, j, w = 7, L.opp[7], L.w[7]
    assert new[i, 2, 2] == pytest.approx(-pv[j, 2, 2] + 2 * w * PW[1][1], abs=1e-15)
    # bounce-back (f): both walls give the same value at a corner
    nf = M.stream(post, M.Lf, "bb")[:, 0].numpy()
    assert nf[5, 0, 0] == pytest.approx(pv[M.Lf.opp[5], 0, 0], abs=1e-15)


class _SwappedAxes(Model):
    """Planted mistake: the lower axis' wall value wins at a corner."""

    def stream(self, post, L, kind, wall_val=None):
        wall = self.wall
        self.wall = list(wall)
        out = []
        for i in range(L.Q):
            c = L.c[i]
            v = torch.roll(post[i], shifts=(c[2], c[1], c[0]), dims=(0, 1, 2))
            for a in (2, 1, 0):
                if not wall[a] or c[a] == 0:
                    continue
                side = 0 if c[a] > 0 else 1
                mask = self._boundary_mask(a, side)
                repl = post[L.opp[i]] if kind == "bb" else \
                    -post[L.opp[i]] + 2.0 * L.w[i] * wall_val[a][side]
                v = torch.where(mask, repl, v)
            out.append(v)
        return torch.stack(out)


def test_swapped_corner_precedence_is_detected():
    M = _SwappedAxes(_box().prm)
    L = M.Lg
    post = _post()
    wall_val = [[torch.tensor(v, dtype=F64) for v in side] for side in PW]
    new = M.stream(post, L, "abb", wall_val)[:, 0].numpy()
    pv = post[:, 0].numpy()
    right = -pv[L.opp[5], 0, 0] + 2 * L.w[5] * PW[1][0]
    assert abs(new[5, 0, 0] - right) > 1e-3


# ---------------------------------------------------------------------------
# R9: regularised interface normal
# ---------------------------------------------------------------------------

def test_normal_regularisation_on_linear_ramps():
    """On phi = 1/2 + a (x - x_c) the Eq. Grad stencil is exact, so the
    oracle's normal must be a / sqrt(a^2 + eps^2) with the default eps =
    1e-3, for slopes from 1e-5 (eps dominates) to 1e-1 (unit normal)."""
    nx, ny = 8, 6
    for a in (1e-5, 1e-4, 1e-3, 1e-2, 1e-1):
        p = I.base_params(dim=2, nx=nx, ny=ny, ns=False, heat=False, phase_change=False)
        p["bc"] = ["wall", "periodic", "periodic"]
        xc = np.arange(nx) + 0.5
        # the Dirichlet ghost continues the ramp exactly when phi_w lies on it
        p["phi_wall"] = [[0.5 - a * nx / 2, 0.5 + a * nx / 2], [0, 0], [0, 0]]
        M = Model(p)
        phi = 0.5 + a * (xc - nx / 2)
        st = M.init(np.broadcast_to(phi, (1, ny, nx)).copy())
        m = M.macros(st)
        n = m.n[0].numpy()
        want = a / math.sqrt(a * a + 1e-6)
        assert np.abs(n - want).max() <= 1e-12 * max(1.0, want), (a, n.ravel()[:3], want)
        assert np.abs(m.n[1].numpy()).max() == 0.0


@pytest.mark.slow
def test_planar_interface_with_regularised_normal():
    """Planar slab (two interfaces) started on the tanh profile, relaxed for
    3 W^2 / M steps at W = 4, 8, 16 with eps = 1e-3.  Where the counter term's
    strength k = 4 phi (1 - phi) / W exceeds 10 eps, the profile stays on tanh
    with a second-order error in 1/W; below, the regularised counter flux
    (zero where k < eps) lets the tails depart by less than phi* = eps W / 4."""
    eps = 1e-3
    core = []
    for W in (4.0, 8.0, 16.0):
        nx = int(24 * W)
        p = I.base_params(dim=2, nx=nx, ny=1, ns=False, heat=False, phase_change=False,
                          W=W, mobility=0.1, eps_n=eps)
        M = Model(p)
        x = np.arange(nx) + 0.5
        x1, x2 = nx / 4, 3 * nx / 4
        ex = 0.5 * (1 + np.tanh(2 * (x - x1) / W)) * 0.5 * (1 + np.tanh(2 * (x2 - x) / W))
        st = M.run(M.init(ex.reshape(1, 1, nx)), int(3 * W * W / 0.1))
        phi = M.fields(st)["phi"][0, 0].numpy()
        k = 4 * ex * (1 - ex) / W
        inner = k > 10 * eps
        core.append(np.abs(phi - ex)[inner].max())
        tail = np.abs(phi - ex)[~inner].max()
        assert tail < eps * W / 4, (W, tail)
    assert core[0] / core[1] > 3 and core[1] / core[2] > 3, core
    assert core[2] < 5e-4, core


# ---------------------------------------------------------------------------
# R8: div(u phi) is the central stencil of Eq. Grad applied to each product
# u_a phi.  On a periodic lattice the stencil's Fourier symbol along an axis
# is sin(k) for every isotropic lattice (sum_i w_i c_ia^2 = c_s^2): it maps
# sin(k x) to sin(k) cos(k x).  With u_x = U cos(k2 x) and phi = sin(k1 x),
# u_x phi = U/2 [sin((k1 + k2) x) + sin((k1 - k2) x)], so the oracle's
# divergence must equal U/2 [sin(k1 + k2) cos((k1 + k2) x) + sin(k1 - k2)
# cos((k1 - k2) x)] exactly (round-off), in 2-D (D2Q9) and 3-D (D3Q19).
# ---------------------------------------------------------------------------

def _periodic_model(dim, n, cls=Model):
    if dim == 2:
        p = I.base_params(dim=2, nx=n, ny=6, ns=True, heat=True)
        p["bc"] = ["periodic", "periodic", "periodic"]
    else:
        p = I.base_params(dim=3, nx=n, ny=5, nz=4, ns=True, heat=True, lat_f="D3Q19",
                          lat_g="D3Q7", lat_s="D3Q7")
        p["bc"] = ["periodic", "periodic", "periodic"]
    return cls(p)


def _symbol_case(M, n, axis):
    """u along `axis` = U cos(k2 s), phi = sin(k1 s) with s the coordinate on
    that axis; returns the oracle's div(u phi) and the closed form."""
    shape = M.shape
    k1, k2, U = 2 * np.pi * 3 / n, 2 * np.pi * 5 / n, 0.02
    s = np.arange(n, dtype=np.float64)
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    phi = np.broadcast_to(np.sin(k1 * s).reshape(bshape), shape).copy()
    ua = np.broadcast_to((U * np.cos(k2 * s)).reshape(bshape), shape).copy()
    u = [torch.zeros(shape, dtype=F64) for _ in range(3)]
    u[axis] = torch.tensor(ua)
    D = M.divergence(u, M.ghost_pad(torch.tensor(phi), "phi")).numpy()
    ex = 0.5 * U * (np.sin(k1 + k2) * np.cos((k1 + k2) * s)
                    + np.sin(k1 - k2) * np.cos((k1 - k2) * s))
    return D, np.broadcast_to(ex.reshape(bshape), shape)


@pytest.mark.parametrize("dim,axis", [(2, 0), (2, 1), (3, 0), (3, 2)])
def test_divergence_fourier_symbol(dim, axis):
    n = 24
    M = _periodic_model(dim, n)
    if axis == 1 and dim == 2:
        # the y axis of the 2-D model has 6 nodes: use a square grid instead
        p = dict(M.prm, nx=n, ny=n)
        M = Model(p)
    if axis == 2:
        p = dict(M.prm, nz=n)
        M = Model(p)
    D, ex = _symbol_case(M, n, axis)
    assert np.abs(D - ex).max() < 1e-15
    assert np.abs(ex).max() > 1e-3


class _ProductRuleDivergence(Model):
    """Planted mistake: div(u phi) as u . grad(phi) + phi div(u), each with
    the central stencil (equal in the continuum, not on the lattice)."""

    def divergence(self, u, phi_padded):
        gphi = self.grad(phi_padded)
        phi = phi_padded[1:-1, 1:-1, 1:-1]
        D = torch.zeros(self.shape, dtype=self.dt)
        for a in range(3):
            D = D + u[a] * gphi[a] + phi * self.grad(self.ghost_pad(u[a], "anti"))[a]
        return D


def test_divergence_symbol_rejects_product_rule():
    n = 24
    M = _periodic_model(2, n, _ProductRuleDivergence)
    D, ex = _symbol_case(M, n, 0)
    assert np.abs(D - ex).max() > 1e-4


# ---------------------------------------------------------------------------
# R10: alpha(phi) = (1 - phi) alpha_l + phi alpha_g.  A static interface
# (heat only: no flow, no phase change) across a column between walls at
# T = 1 and T = 0 conducts in series.  With alpha constant over each node's
# unit cell, the continuum steady state of (alpha T')' = 0 is linear in
# each cell with slope proportional to 1 / alpha_i; at the node centre
#   T_i = 1 - (sum_{j<i} 1/alpha_j + 1/(2 alpha_i)) / sum_j 1/alpha_j.
# The oracle's steady state follows it for the linear interpolation, and a
# harmonic interpolation (the form of Eq. Viscosity) misses it by 6e-2.
# ---------------------------------------------------------------------------

class _HarmonicDiffusivity(Model):
    """Planted mistake: alpha interpolated harmonically."""

    def diffusivity(self, phi):
        al, ag = self.prm["alpha_l"], self.prm["alpha_g"]
        return al * ag / (phi * al + (1.0 - phi) * ag)


def _layered_column(cls, ny=16, al=0.05, ag=0.25, W=4.0, nsteps=2000):
    p = I.base_params(dim=2, nx=1, ny=ny, ns=False, heat=True, phase_change=False,
                      alpha_l=al, alpha_g=ag, W=W)
    p["bc"] = ["periodic", "wall", "periodic"]
    p["phi_wall"] = [[0.0, 0.0], [0.0, 1.0], [0.0, 0.0]]
    p["T_wall"] = [[0.0, 0.0], [1.0, 0.0], [0.0, 0.0]]
    M = cls(p)
    y = np.arange(ny) + 0.5
    st = M.init(I.tanh_profile(y - ny / 2, W)[None, :, None], (1.0 - y / ny)[None, :, None])
    f = M.fields(M.run(st, nsteps))
    phi = f["phi"][0, :, 0].numpy()
    r = 1.0 / ((1.0 - phi) * al + phi * ag)
    R = np.concatenate([[0.0], np.cumsum(r)])
    T_series = 1.0 - 0.5 * (R[:-1] + R[1:]) / R[-1]
    return np.abs(f["T"][0, :, 0].numpy() - T_series).max()


def test_layered_conduction_follows_linear_diffusivity():
    assert _layered_column(Model) < 1e-3


def test_layered_conduction_rejects_harmonic_diffusivity():
    assert _layered_column(_HarmonicDiffusivity) > 1e-2
