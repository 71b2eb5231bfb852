"""Pins of the oracle's TRT and MRT collisions (reading R26; Sec. 3 names
them after Eq. LBE as the way to lower mobility and higher Peclet numbers).

* The MRT bases are orthogonal and hold the stated polynomials (the D2Q9
  rows e, eps, q as in Lallemand and Luo's table).
* Equal rates give BGK exactly: TRT with Lambda = tau^2 (omega+ = omega-)
  and MRT with every rate at the BGK rate reproduce BGK runs to round-off,
  in 2-D and 3-D.
* MRT with even moments at omega+ and odd moments at omega- is TRT.
* Diffusion depends on the antisymmetric rate only: the Gaussian heat
  kernel (P10) decays as the closed form for every Lambda and for MRT with
  arbitrary free rates.
* Ginzburg's magic parameter: with Lambda = 3/16 the half-way bounce-back
  wall sits exactly mid-link, so the force-driven Poiseuille profile is
  exact for any viscosity, where BGK at tau = 1.5 is off by 4 per cent.
* z-invariance (P13) holds with TRT: a z-invariant 3-D run equals the 2-D
  run with D2Q5 phase field and heat populations.
"""
import numpy as np
import pytest
import torch

from oracle.lbm_oracle import Model, lattice, moment_basis
from paper_2003_06342_amd import inputs as I


@pytest.mark.parametrize("name", ["D2Q9", "D3Q7", "D2Q5"])
def test_moment_bases_orthogonal(name):
    L = lattice(name)
    M = np.array(moment_basis(L))
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    assert np.linalg.matrix_rank(M) == L.Q
    assert (M[0] == 1).all()


def test_d2q9_basis_rows_match_lallemand_luo():
    L = lattice("D2Q9")
    M = np.array(moment_basis(L))
    # directions in the order 0, E, N, W, S, NE, NW, SW, SE (this lattice's order)
    assert [c[:2] for c in L.c] == [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                                    (1, 1), (-1, 1), (-1, -1), (1, -1)]
    assert M[1].tolist() == [-4, -1, -1, -1, -1, 2, 2, 2, 2]
    assert M[2].tolist() == [4, -2, -2, -2, -2, 1, 1, 1, 1]
    assert M[4].tolist() == [0, -2, 0, 2, 0, 1, -1, -1, 1]
    assert M[6].tolist() == [0, 0, -2, 0, 2, 1, 1, -1, -1]
    assert M[7].tolist() == [0, 1, -1, 1, -1, 0, 0, 0, 0]
    assert M[8].tolist() == [0, 0, 0, 0, 0, 1, -1, 1, -1]


def _periodic_case(dim=2, **kw):
    if dim == 2:
        p = I.base_params(dim=2, nx=20, ny=16, **I.FB)
    else:
        p = I.base_params(dim=3, nx=12, ny=10, nz=9, lat_f="D3Q19", lat_g="D3Q7",
                          lat_s="D3Q7", **I.FB)
    # constant transport coefficients: one BGK rate per family
    p["nu_g"] = p["nu_l"] = 0.1
    p["alpha_g"] = p["alpha_l"] = 0.05
    p["gravity"] = [0.0, -1e-4, 0.0] if dim == 2 else [0.0, 0.0, -1e-4]
    p.update(kw)
    phi0, T0 = I.random_smooth_fields(p, seed=3, T_amp=0.5)
    return p, phi0, T0


def _run(p, phi0, T0, n):
    M = Model(p)
    return M.fields(M.run(M.init(phi0, T0), n))


def _taus(p):
    cs2_g = 1 / 3 if p["dim"] == 2 else 0.25
    return [p["nu_l"] * 3, p["mobility"] / cs2_g, p["alpha_l"] / cs2_g]


def _close(a, b, tol=1e-13):
    for k in ("phi", "T", "ux", "uy", "p"):
        sc = max(1.0, float(np.abs(b[k].numpy()).max()))
        assert float(np.abs(a[k].numpy() - b[k].numpy()).max()) <= tol * sc, k


@pytest.mark.parametrize("dim", [2, 3])
def test_trt_with_equal_rates_is_bgk(dim):
    p, phi0, T0 = _periodic_case(dim)
    ref = _run(p, phi0, T0, 15)
    lam = [t * t for t in _taus(p)]
    trt = _run(dict(p, collision="trt", trt_lambda=lam), phi0, T0, 15)
    _close(trt, ref)


@pytest.mark.parametrize("dim", [2, 3])
def test_mrt_with_equal_rates_is_bgk(dim):
    p, phi0, T0 = _periodic_case(dim, ns=(dim == 2))
    ref = _run(p, phi0, T0, 15)
    rates = [[1.0 / (t + 0.5)] * 4 for t in _taus(p)]
    mrt = _run(dict(p, collision="mrt", mrt_rates=rates), phi0, T0, 15)
    _close(mrt, ref)


def test_mrt_with_trt_rates_is_trt():
    p, phi0, T0 = _periodic_case(2)
    lam = 3.0 / 16.0
    trt = _run(dict(p, collision="trt", trt_lambda=[lam] * 3), phi0, T0, 15)
    rates = []
    for fam, t in enumerate(_taus(p)):
        w_t = 1.0 / (t + 0.5)
        w_o = 1.0 / (lam / t + 0.5)
        wp, wm = (w_t, w_o) if fam == 0 else (w_o, w_t)
        rates.append([wp, wp, wm, wp])          # s_e, s_eps (even), s_q (odd), s_p (even)
    mrt = _run(dict(p, collision="mrt", mrt_rates=rates), phi0, T0, 15)
    _close(mrt, trt)


def _gaussian_error(**kw):
    n, s, A, alpha, t = 48, 3.0, 1.0, 0.1, 150
    p = I.base_params(dim=2, nx=n, ny=n, ns=False, heat=True, phase_change=True,
                      alpha_l=alpha, alpha_g=alpha, **kw)
    M = Model(p)
    T0 = I.gaussian_T(p, A, s)
    st = M.run(M.init(np.zeros_like(T0), T0), t)
    T = M.fields(st)["T"][0].numpy()
    s2 = s * s + 2 * alpha * t
    xc = np.arange(n) + 0.5
    r2 = (xc[None, :] - n / 2) ** 2 + (xc[:, None] - n / 2) ** 2
    ex = A * (s * s / s2) * np.exp(-r2 / (2 * s2))
    return np.abs(T - ex).max() / ex.max(), float(T.sum()) / float(T0.sum())


def test_diffusion_depends_on_the_antisymmetric_rate_only():
    """Measured max errors against the closed form (48^2, s = 3, 150 steps):
    BGK 6.8e-3; TRT Lambda = 1/12, 3/16, 1/4, 1/2: 7.2e-3, 1.8e-3, 1.5e-3,
    1.5e-2 (the fourth-order error depends on Lambda); MRT 8.4e-3.  The
    diffusivity itself is set by omega- alone: the symmetric rate moves only
    that higher-order error.  A transport coefficient put on omega+ would
    halve the diffusivity here (Lambda / tau = 0.21 against tau = 0.4)."""
    e_bgk, m_bgk = _gaussian_error()
    assert e_bgk < 1e-2 and abs(m_bgk - 1) < 1e-13
    for lam in (1 / 12, 3 / 16, 1 / 4, 1 / 2):
        e, m = _gaussian_error(collision="trt", trt_lambda=[lam] * 3)
        assert e < 2e-2 and abs(m - 1) < 1e-13, (lam, e)
    rates = [[1.0] * 4, [1.0] * 4, [1.3, 0.7, 1.1, 1.6]]
    e, m = _gaussian_error(collision="mrt", mrt_rates=rates)
    assert e < 2e-2 and abs(m - 1) < 1e-13, e


def _poiseuille_error(**kw):
    ny, nu, F = 16, 0.5, 1e-6
    p = I.base_params(dim=2, nx=1, ny=ny, ns=True, heat=False, phase_change=False,
                      nu_l=nu, nu_g=nu, sigma=0.0, **kw)
    p["bc"] = ["periodic", "wall", "periodic"]
    p["body_force"] = [F, 0.0, 0.0]
    M = Model(p)
    st = M.run(M.init(np.zeros((1, ny, 1))), 2500)   # slowest mode: exp(-nu pi^2 t / ny^2) ~ 1e-21
    u = M.fields(st)["ux"][0, :, 0].numpy()
    y = np.arange(ny) + 0.5
    ex = F / (2 * p["rho_l"] * nu) * y * (ny - y)
    return np.abs(u - ex).max() / ex.max()


@pytest.mark.slow
def test_trt_magic_parameter_makes_bounce_back_poiseuille_exact():
    assert _poiseuille_error() > 0.03          # BGK at tau = 1.5: the wall slips
    assert _poiseuille_error(collision="trt", trt_lambda=[3 / 16] * 3) < 1e-8
    assert _poiseuille_error(collision="trt", trt_lambda=[1 / 4] * 3) > 1e-3
    tau = 1.5
    wp, wm = 1 / (tau + 0.5), 1 / ((3 / 16) / tau + 0.5)
    rates = [[wp, wp, wm, 1.0], [1.0] * 4, [1.0] * 4]
    assert _poiseuille_error(collision="mrt", mrt_rates=rates) < 1e-8


def test_z_invariance_holds_with_trt():
    """P13 with TRT: 3-D fields constant along z equal the 2-D run with D2Q9
    f and D2Q5 g and s (the z-projections of D3Q19 and D3Q7)."""
    kw = dict(collision="trt", trt_lambda=[3 / 16, 1 / 6, 1 / 12])
    p2 = I.base_params(dim=2, nx=14, ny=12, lat_g="D2Q5", lat_s="D2Q5", **I.FB, **kw)
    p2["gravity"] = [0.0, -1e-4, 0.0]
    phi2, T2 = I.random_smooth_fields(p2, seed=8, T_amp=0.5)
    p3 = I.base_params(dim=3, nx=14, ny=12, nz=4, lat_f="D3Q19", lat_g="D3Q7", lat_s="D3Q7",
                       **I.FB, **kw)
    p3["gravity"] = [0.0, -1e-4, 0.0]
    phi3 = np.repeat(phi2, 4, axis=0)
    T3 = np.repeat(T2, 4, axis=0)
    f2 = _run(p2, phi2, T2, 12)
    f3 = _run(p3, phi3, T3, 12)
    for k in ("phi", "T", "ux", "uy", "p"):
        a = f3[k].numpy()
        assert np.abs(a - a[:1]).max() < 1e-14, k
        assert np.abs(a[0] - f2[k].numpy()[0]).max() < 1e-12 * max(1.0, np.abs(a).max()), k
