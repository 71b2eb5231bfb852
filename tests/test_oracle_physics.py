"""Oracle pins on closed-form solutions: planar tanh interface (P8), Laplace
law (P9), Gaussian heat kernel (P10), 1-D Stefan problem (P11) and the
layered Poiseuille flow (P12)."""
import math

import numpy as np
import pytest
import torch
from scipy import special

from oracle.lbm_oracle import F64, Model
from paper_2003_06342_amd import inputs as I
from tests.test_constants import stefan_xi


def _interface_positions(phi_line):
    """x where a 1-D profile (node centres i + 1/2) crosses 1/2."""
    x = np.arange(len(phi_line)) + 0.5
    out = []
    for i in range(len(phi_line) - 1):
        a, b = phi_line[i] - 0.5, phi_line[i + 1] - 0.5
        if a == 0:
            out.append(x[i])
        elif a * b < 0:
            out.append(x[i] + a / (a - b))
    return out


def test_planar_interface_relaxes_to_tanh():
    """P8: a slab started with twice the width relaxes to 1/2[1+tanh(2 zeta/W)]
    (Eq. Kernel-Function), centred where it started (CAC, no flow)."""
    nx, W = 96, 4.0
    p = I.base_params(dim=2, nx=nx, ny=1, ns=False, heat=False, phase_change=False,
                      W=W, mobility=0.1)
    M = Model(p)
    x = np.arange(nx) + 0.5
    x1, x2 = 24.0, 72.0
    wide = 0.5 * (1 + np.tanh(2 * (x - x1) / (2 * W))) * 0.5 * (1 + np.tanh(2 * (x2 - x) / (2 * W)))
    st = M.init(wide.reshape(1, 1, nx))
    st = M.run(st, 3000)
    phi = M.fields(st)["phi"][0, 0].numpy()
    exact = 0.5 * (1 + np.tanh(2 * (x - x1) / W)) * 0.5 * (1 + np.tanh(2 * (x2 - x) / W))
    assert np.abs(phi - exact).max() < 0.015
    pos = _interface_positions(phi)
    assert pos[0] == pytest.approx(x1, abs=0.05) and pos[1] == pytest.approx(x2, abs=0.05)
    # the unrelaxed start was far from it
    assert np.abs(wide - exact).max() > 0.1


@pytest.mark.slow
def test_laplace_law_static_drop():
    """P9: p_in - p_out = sigma / R (Eq. LaplaceLaw) for the static drop;
    in/out means over r < R - 2W and r > R + 2W (reading R22)."""
    n, R = 64, 16.0
    p = I.drop_params(n)
    M = Model(p)
    phi0, _ = I.drop_fields(p, radius=R)
    st = M.init(phi0)
    st = M.run(st, 2000)
    x = np.arange(n) + 0.5
    r = np.sqrt((x[None, :] - n / 2) ** 2 + (x[:, None] - n / 2) ** 2)
    dps = []
    for _ in range(10):            # average out the slowly decaying acoustic mode
        st = M.run(st, 100)
        pp = M.fields(st)["p"][0].numpy()
        dps.append(pp[r < R - 2 * p["W"]].mean() - pp[r > R + 2 * p["W"]].mean())
    # R/W = 4: the diffuse interface lowers the jump by a few per cent
    assert np.mean(dps) == pytest.approx(p["sigma"] / R, rel=0.1)


def test_gaussian_heat_kernel():
    """P10: pure diffusion (phi uniform, u = 0) of a Gaussian matches
    T = A (s^2/(s^2 + 2 alpha t))^(d/2) exp(-r^2 / (2 (s^2 + 2 alpha t)))
    with alpha = tau_s c_s^2, and sum(T) is exact."""
    n, s, A, alpha, t = 64, 4.0, 1.0, 0.1, 200
    p = I.base_params(dim=2, nx=n, ny=n, ns=False, heat=True, phase_change=True,
                      alpha_l=alpha, alpha_g=alpha)
    M = Model(p)
    T0 = I.gaussian_T(p, A, s)
    st = M.init(np.zeros_like(T0), T0)
    st = M.run(st, t)
    T = M.fields(st)["T"][0].numpy()
    s2 = s * s + 2 * alpha * t
    x = np.arange(n) + 0.5
    r2 = (x[None, :] - n / 2) ** 2 + (x[:, None] - n / 2) ** 2
    exact = A * (s * s / s2) * np.exp(-r2 / (2 * s2))
    assert np.linalg.norm(T - exact) / np.linalg.norm(exact) < 5e-3   # O((dx/s)^2)
    assert T.sum() == pytest.approx(T0.sum(), rel=1e-13)


@pytest.mark.slow
@pytest.mark.parametrize("case", ["equal", "ratio10"])
def test_stefan_problem(case):
    """P11: 1-D Stefan problem of Sec. 4.2 (D2Q9 phi + T, u = 0, anti-bounce-
    back walls in x): interface position 2 xi sqrt(alpha_l t) and the erf
    liquid profile, xi from the transcendental equation with reading R15."""
    nx, t = 160, 8000
    theta_w, theta_inf = -0.3, 0.3
    if case == "equal":
        a_l = a_g = 0.14
        theta_I = 0.0
    else:
        a_l, a_g, theta_I = 0.14, 0.014, 0.05
    p = I.base_params(dim=2, nx=nx, ny=1, ns=False, heat=True, phase_change=True,
                      alpha_l=a_l, alpha_g=a_g, mobility=0.08, W=3.0, L_over_cp=1.0,
                      T_sat=0.0, theta_I=theta_I)
    p["bc"] = ["wall", "periodic", "periodic"]
    p["phi_wall"] = [[0.0, 1.0], [0, 0], [0, 0]]
    p["T_wall"] = [[theta_w, theta_inf], [0, 0], [0, 0]]
    M = Model(p)
    x = np.arange(nx) + 0.5
    phi0 = 0.5 * (1 + np.tanh(2 * x / p["W"]))
    st = M.init(phi0.reshape(1, 1, nx), np.full((1, 1, nx), theta_inf))
    st = M.run(st, t)
    f = M.fields(st)
    phi = f["phi"][0, 0].numpy()
    xI = _interface_positions(phi)[0]
    xi = stefan_xi(theta_w, theta_inf, theta_I, a_l / a_g)
    exact = 2 * xi * math.sqrt(a_l * t)
    assert xI == pytest.approx(exact, rel=0.05)
    theta = f["T"][0, 0].numpy()
    liq = x < xI - 2 * p["W"]
    th_l = theta_w + (theta_I - theta_w) * special.erf(x / (2 * math.sqrt(a_l * t))) / special.erf(xi)
    assert np.abs(theta[liq] - th_l[liq]).max() < 0.02


@pytest.mark.slow
def test_layered_poiseuille():
    """P12: two layers of viscosity ratio 3 (Sec. 4.1.2, Eq.
    AnalyticalSol_Poiseuille-1), body force G, half-way bounce-back walls;
    harmonic viscosity (Eq. Viscosity).  The printed linear term carries a
    minus sign that violates no-slip at y = -h; the profile below is the one
    that satisfies both walls and stress continuity (linear term +)."""
    h = 16
    ny = 2 * h
    nu_A, nu_B, uc = 0.1, 0.3, 5e-5
    eta_A, eta_B = nu_A, nu_B              # rho = 1 in both layers
    G = uc * (eta_A + eta_B) / h ** 2
    p = I.base_params(dim=2, nx=1, ny=ny, heat=False, phase_change=False,
                      nu_l=nu_A, nu_g=nu_B, rho_l=1.0, rho_g=1.0, mobility=0.1, W=4.0, sigma=0.0)
    p["bc"] = ["periodic", "wall", "periodic"]
    p["phi_wall"] = [[0, 0], [0.0, 1.0], [0, 0]]
    p["body_force"] = [G, 0.0, 0.0]
    M = Model(p)
    y = np.arange(ny) + 0.5
    phi0 = 0.5 * (1 + np.tanh(2 * (y - h) / p["W"]))
    st = M.init(phi0.reshape(1, ny, 1))
    st = M.run(st, 8000)
    ux = M.fields(st)["ux"][0, :, 0].numpy()
    Y = (y - h) / h
    k = (eta_A - eta_B) / (eta_A + eta_B)
    exact = np.where(Y <= 0,
                     G * h * h / (2 * eta_A) * (-Y ** 2 + Y * k + 2 * eta_A / (eta_A + eta_B)),
                     G * h * h / (2 * eta_B) * (-Y ** 2 + Y * k + 2 * eta_B / (eta_A + eta_B)))
    assert np.abs(ux - exact).max() / exact.max() < 0.03
