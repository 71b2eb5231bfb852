"""Pins on constants the paper prints (golden values in tests/golden)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize, special

from paper_2003_06342_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_coefficient_A_from_integrals():
    """App. B: A = (G + J U) / (2 I) with phi0 = tanh kernel, p_phi = phi0(1-phi0),
    h0 = phi0, W = 2 sqrt 2; integrals by quadrature vs the printed closed
    forms and A = 10/48."""
    W = 2.0 * math.sqrt(2.0)
    phi0 = lambda z: 0.5 * (1.0 + math.tanh(2.0 * z / W))
    dphi = lambda z: (4.0 / W) * phi0(z) * (1.0 - phi0(z))   # Eq. Norm_GradPhi
    pphi = lambda z: phi0(z) * (1.0 - phi0(z))
    L = 60.0
    Ival = integrate.quad(lambda z: dphi(z) ** 2, -L, L, limit=200)[0]
    Jval = integrate.quad(lambda z: dphi(z) * pphi(z), -L, L, limit=200)[0]
    Uval = integrate.quad(phi0, -L, 0.0, limit=200)[0]
    inner = lambda z: integrate.quad(phi0, 0.0, z, limit=200)[0]
    Gval = integrate.quad(lambda z: dphi(z) * pphi(z) * inner(z), -L, L, limit=200)[0]
    assert Ival == pytest.approx(1.0 / (3.0 * math.sqrt(2.0)), rel=1e-9)
    assert Jval == pytest.approx(1.0 / 6.0, rel=1e-9)
    assert Uval == pytest.approx(math.log(2.0) / math.sqrt(2.0), rel=1e-9)
    assert Gval == pytest.approx(-(12.0 * math.log(2.0) - 10.0) / (72.0 * math.sqrt(2.0)), rel=1e-7)
    A = (Gval + Jval * Uval) / (2.0 * Ival)
    assert A == pytest.approx(GOLD["coefficient_A"]["A"], rel=1e-7)
    assert I.base_params()["A_coef"] == pytest.approx(10.0 / 48.0, rel=1e-15)


def _stefan_residual(xi, theta_w, theta_inf, theta_I, r_lg):
    """Transcendental equation of Sec. 4.2 with the right-hand side read as
    -xi sqrt(pi) / (theta_w - theta_I) (reading R15); r_lg = alpha_l/alpha_g."""
    lhs = (math.exp(-xi * xi) / math.erf(xi)
           + math.sqrt(1.0 / r_lg) * (theta_I - theta_inf) / (theta_I - theta_w)
           * math.exp(-xi * xi * r_lg) / math.erfc(xi * math.sqrt(r_lg)))
    return lhs + xi * math.sqrt(math.pi) / (theta_w - theta_I)


def stefan_xi(theta_w, theta_inf, theta_I, r_lg):
    return optimize.brentq(_stefan_residual, 1e-4, 3.0, args=(theta_w, theta_inf, theta_I, r_lg),
                           xtol=1e-14)


def test_stefan_xi_equal_diffusivities():
    g = GOLD["stefan_xi_equal_diffusivities"]
    xi = stefan_xi(g["theta_w"], g["theta_inf"], g["theta_I"], 1.0)
    assert round(xi, 6) == pytest.approx(g["xi"], abs=1.5e-6)


def test_stefan_xi_unequal_diffusivities():
    g = GOLD["stefan_xi_unequal_diffusivities"]
    for case in g["cases"]:
        xi = stefan_xi(g["theta_w"], g["theta_inf"], g["theta_I"], case["ratio_l_over_g"])
        assert xi == pytest.approx(case["xi"], abs=1.5e-6), case


def test_stefan_printed_rhs_does_not_reproduce():
    """The right-hand side as printed (-xi sqrt(pi)/theta_w) misses the
    printed xi when theta_I != 0 (why reading R15 is taken)."""
    g = GOLD["stefan_xi_unequal_diffusivities"]
    case = g["cases"][0]
    def printed(xi):
        r = case["ratio_l_over_g"]
        lhs = (math.exp(-xi * xi) / math.erf(xi)
               + math.sqrt(1.0 / r) * (g["theta_I"] - g["theta_inf"]) / (g["theta_I"] - g["theta_w"])
               * math.exp(-xi * xi * r) / math.erfc(xi * math.sqrt(r)))
        return lhs + xi * math.sqrt(math.pi) / g["theta_w"]
    xi = optimize.brentq(printed, 1e-4, 3.0)
    assert abs(xi - case["xi"]) > 1e-2


def test_film_table_dimensionless_numbers():
    """Sec. 5.1: lambda_s, lambda_c, Gr, Pr, Ja, t_s from the table."""
    t = GOLD["film_boiling_table"]
    lam_s = math.sqrt(t["sigma"] / ((t["rho_l"] - t["rho_g"]) * t["g_y"]))
    assert lam_s == pytest.approx(t["lambda_s"], rel=1e-3)
    assert 2 * math.pi * lam_s == pytest.approx(t["lambda_c"], rel=1e-3)
    Gr = t["rho_g"] * t["g_y"] * (t["rho_l"] - t["rho_g"]) * lam_s ** 3 / (t["rho_g"] ** 2 * t["nu_g"] ** 2)
    assert Gr == pytest.approx(t["Gr"], rel=1e-3)
    assert t["nu_g"] / t["alpha_g"] == pytest.approx(t["Pr"], rel=1e-12)
    assert math.sqrt(lam_s / t["g_y"]) == pytest.approx(t["t_s"], rel=2e-3)


def test_film_lattice_set_matches_table():
    """The lattice film-boiling set is the table converted with dx, dt."""
    t = GOLD["film_boiling_table"]
    dx, dt = t["dx"], t["dt"]
    k = dt / dx ** 2
    assert I.FB["nu_g"] == pytest.approx(t["nu_g"] * k, rel=1e-12)
    assert I.FB["nu_l"] == pytest.approx(t["nu_l"] * k, rel=1e-12)
    assert I.FB["alpha_g"] == pytest.approx(t["alpha_g"] * k, rel=1e-12)
    assert I.FB["alpha_l"] == pytest.approx(t["alpha_l"] * k, rel=1e-12)
    assert I.FB["mobility"] == pytest.approx(t["mobility"] * k, rel=1e-12)
    assert I.FB["W"] == pytest.approx(t["W"] / dx, rel=1e-12)
    assert I.FB["sigma"] == pytest.approx(t["sigma"] * dt ** 2 / dx ** 3, rel=1e-12)
    # Prandtl number is unit-free
    assert I.FB["nu_g"] / I.FB["alpha_g"] == pytest.approx(t["Pr"], rel=1e-12)


def test_film_gravity_gives_paper_wavelength_ratio():
    for lam in (1024.0, 512.0, 256.0):
        g = I.film_gravity(lam)
        lam_c = 2 * math.pi * math.sqrt(I.FB["sigma"] / ((I.FB["rho_l"] - I.FB["rho_g"]) * g))
        assert lam / lam_c == pytest.approx(0.64 / 0.2738, rel=1e-12)
    assert I.film_gravity(1024.0) == pytest.approx(3.29e-7, rel=2e-3)
