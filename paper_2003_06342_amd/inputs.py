"""Seeded synthetic workloads: parameter sets and initial fields.

This module is shared by the FP64 oracle's tests and by the HIP path's
callers.  It holds no step of the lattice-Boltzmann method: it only builds
plain parameter dictionaries and initial fields (numpy, float64) from a
seed.  Every random number comes from ``numpy.random.default_rng(seed)``
(PCG64).

Field layout: C-ordered ``[nz, ny, nx]`` arrays (``nz == 1`` in 2-D); node
``(i, j, k)`` has its centre at ``(i + 1/2, j + 1/2, k + 1/2)`` so that a
half-way wall lies on the coordinate planes 0 and ``n``.

Parameter sets follow the paper:
  * film boiling: Tab. "FilmBoiling_Parameters" (Sec. 5.1) converted to
    lattice units with dx = 1.25e-3 and dt = 7.5e-5 (nu, alpha and M times
    dt/dx^2 = 48, W/dx = 4, sigma*dt^2/dx^3 = 0.0144), with rho_g = 1,
    rho_l = 10, T_w = 1, T_sat = 0 and L/Cp = 10 (Jacob number 0.1), and
    gravity set so that the perturbation wavelength over the critical
    wavelength lambda_c = 2*pi*sqrt(sigma/((rho_l-rho_g) g)) (Sec. 5.1)
    equals the paper's 0.64 / 0.2738;
  * static drop: Laplace-law set-up of Sec. 4.1.2 scaled to a 128^2 box.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# ---------------------------------------------------------------------------
# parameter dictionaries (plain numbers; each side derives its own
# relaxation rates from them)
# ---------------------------------------------------------------------------

_BASE = dict(
    dim=2, nx=1, ny=1, nz=1,
    lat_f="D2Q9", lat_g="D2Q9", lat_s="D2Q9",
    ns=True, heat=True, phase_change=True,
    visc_linear=False, geq_cac=False,
    nu_l=0.1, nu_g=0.1, mobility=0.02, alpha_l=0.1, alpha_g=0.1,
    W=4.0, sigma=1e-3, rho_l=10.0, rho_g=1.0,
    L_over_cp=1.0, T_sat=0.0, theta_I=0.0, A_coef=10.0 / 48.0,
    gravity=[0.0, 0.0, 0.0],
    body_force=[0.0, 0.0, 0.0],
    bc=["periodic", "periodic", "periodic"],
    phi_wall=[[0.0, 0.0], [0.0, 0.0], [0.0, 0.0]],
    T_wall=[[0.0, 0.0], [0.0, 0.0], [0.0, 0.0]],
    f_open=[[False, False], [False, False], [False, False]],   # open (pressure) faces of f
    p_wall=[[0.0, 0.0], [0.0, 0.0], [0.0, 0.0]],               # their pressure
    eps_n=1e-3,
    div_local=False,
    collision="bgk",                  # "bgk" | "trt" | "mrt"
    trt_lambda=[0.25, 0.25, 0.25],    # TRT magic parameter of f, g, s
    mrt_rates=[[1.0] * 4, [1.0] * 4, [1.0] * 4],   # MRT s_e, s_eps, s_q, s_p of f, g, s
    grad_scheme="central",            # "central" | "biased1" | "biased2"
    check_every=0,
)


def base_params(**kw) -> dict:
    p = copy.deepcopy(_BASE)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = copy.deepcopy(v)
    return p


# Film-boiling lattice set (paper's table x 48 for the diffusivities).
FB = dict(nu_g=0.024, nu_l=0.144, alpha_g=0.12, alpha_l=0.012,
          mobility=0.0816, W=4.0, sigma=0.0144, theta_I=0.0,
          rho_g=1.0, rho_l=10.0, T_sat=0.0, L_over_cp=10.0)

# Ratio lambda / lambda_c used by the paper's node/antinode run (Sec. 5.2).
LAMBDA_OVER_LAMBDA_C = 0.64 / 0.2738


def film_gravity(wavelength: float, sigma: float = FB["sigma"],
                 rho_l: float = FB["rho_l"], rho_g: float = FB["rho_g"]) -> float:
    """Gravity magnitude that puts ``wavelength`` at 0.64/0.2738 lambda_c."""
    lam_c = wavelength / LAMBDA_OVER_LAMBDA_C
    lam_s = lam_c / (2.0 * math.pi)
    return sigma / ((rho_l - rho_g) * lam_s * lam_s)


def film2d_params(nx: int, ny: int, wavelength: float | None = None, **kw) -> dict:
    """2-D film boiling: x periodic, walls at y = 0 and y = ny."""
    lam = float(nx if wavelength is None else wavelength)
    p = base_params(dim=2, nx=nx, ny=ny, nz=1, **FB)
    p["gravity"] = [0.0, -film_gravity(lam), 0.0]
    p["bc"] = ["periodic", "wall", "periodic"]
    p["phi_wall"] = [[0.0, 0.0], [1.0, 1.0], [0.0, 0.0]]   # vapour at both walls
    p["T_wall"] = [[0.0, 0.0], [1.0, 0.0], [0.0, 0.0]]     # heated floor, T_sat top
    for k, v in kw.items():
        p[k] = v
    return p


def film3d_params(n: int, wavelength: float | None = None, nz: int | None = None,
                  **kw) -> dict:
    """3-D film boiling: x, y periodic, walls at z = 0 and z = nz."""
    lam = float(n if wavelength is None else wavelength)
    p = base_params(dim=3, nx=n, ny=n, nz=n if nz is None else nz,
                    lat_f="D3Q19", lat_g="D3Q7", lat_s="D3Q7", **FB)
    p["gravity"] = [0.0, 0.0, -film_gravity(lam)]
    p["bc"] = ["periodic", "periodic", "wall"]
    p["phi_wall"] = [[0.0, 0.0], [0.0, 0.0], [1.0, 1.0]]
    p["T_wall"] = [[0.0, 0.0], [0.0, 0.0], [1.0, 0.0]]
    for k, v in kw.items():
        p[k] = v
    return p


# Multi-mode film boiling (Sec. 5.3, the 4096 x 3072 run): the paper's
# domain 5.12 x 3.84 at dx = 1.25e-3, the film-boiling set with gravity
# such that the critical wavelength spans the same number of nodes as for
# the lambda = 512 set (lambda_c = 512 * 0.2738 / 0.64 = 219 nodes, the
# paper's 0.2738 / dx), and two Jacob numbers through L/Cp (T_w - T_sat = 1).
MULTIMODE_LAMBDA_C = 512.0 / LAMBDA_OVER_LAMBDA_C


def multimode_params(nx: int = 4096, ny: int = 3072, jacob: float = 0.1, **kw) -> dict:
    """Multi-mode film: x periodic, walls at y = 0 and y = ny; Ja = Cp (T_w -
    T_sat) / L, so L/Cp = 1 / Ja with T_w = 1 and T_sat = 0."""
    p = film2d_params(nx, ny, wavelength=512.0)
    p["L_over_cp"] = 1.0 / jacob
    for k, v in kw.items():
        p[k] = v
    return p


def multimode_modes(nx: int, seed: int, count: int = 16,
                    lam_c: float = MULTIMODE_LAMBDA_C) -> np.ndarray:
    """Wavelengths of the multi-mode initial interface: `count` values drawn
    uniformly in [0.5 lambda_c, 1.5 sqrt(3) lambda_c] (Sec. 5.3), each
    snapped to nx / k with k the nearest integer >= 1 so that every mode is
    periodic on the x-periodic domain."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.5 * lam_c, 1.5 * math.sqrt(3.0) * lam_c, count)
    k = np.maximum(1, np.rint(nx / lam))
    return nx / k


def multimode_fields(p: dict, seed: int = 7, y0: float = 24.0, y1: float = 0.75,
                     count: int = 16):
    """Vapour film h(x) = y0 + y1 sum_i sin(2 pi x / lambda_i) (Sec. 5.3) with
    the modes of multimode_modes.  Defaults: y0 = 0.03 / dx = 24 nodes as in
    the single-mode run, and y1 = (0.015 / dx) / 16 = 0.75 nodes, so that h
    stays within the single-mode run's printed range [y0 - 12, y0 + 12]
    nodes.  T = T_w (1 - y / h) below the film, T_sat above; u = 0, p = 0.
    Returns (phi0, T0, modes)."""
    nx, ny, W = p["nx"], p["ny"], p["W"]
    lam = multimode_modes(nx, seed, count)
    x = _centres(nx)
    y = _centres(ny)
    h = y0 + y1 * np.sin(2.0 * np.pi * x[None, :] / lam[:, None]).sum(axis=0)
    H = h[None, :]
    Y = y[:, None]
    phi = tanh_profile(H - Y, W)
    Tw, Tsat = p["T_wall"][1][0], p["T_sat"]
    T = np.where(Y < H, Tsat + (Tw - Tsat) * (1.0 - Y / H), Tsat)
    return phi[None].copy(), T[None].copy(), lam


def drop_params(n: int = 128, **kw) -> dict:
    """Static drop, periodic box, heat off (Laplace-law set-up)."""
    p = base_params(dim=2, nx=n, ny=n, nz=1, heat=False, phase_change=False,
                    nu_l=0.1, nu_g=0.1, mobility=0.02, W=4.0, sigma=1e-3,
                    rho_l=10.0, rho_g=1.0)
    for k, v in kw.items():
        p[k] = v
    return p


# ---------------------------------------------------------------------------
# initial fields
# ---------------------------------------------------------------------------

def _centres(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) + 0.5


def tanh_profile(signed_dist: np.ndarray, W: float) -> np.ndarray:
    """Diffuse-interface profile 1/2 [1 + tanh(2 d / W)] (Sec. 2.1 kernel)."""
    return 0.5 * (1.0 + np.tanh(2.0 * signed_dist / W))


def film2d_fields(p: dict, seed: int = 0, h0: float = 64.0, amp: float = 4.0,
                  wavelength: float | None = None, Tw=None):
    """Vapour film of height h(x) = h0 + amp cos(2 pi x / lambda) + U(-1/2, 1/2)
    above the heated floor.  Returns (phi0, T0, Tw_row) as float64 arrays
    of shape [1, ny, nx] and [nx]."""
    nx, ny, W = p["nx"], p["ny"], p["W"]
    lam = float(nx if wavelength is None else wavelength)
    rng = np.random.default_rng(seed)
    x = _centres(nx)
    y = _centres(ny)
    h = h0 + amp * np.cos(2.0 * np.pi * x / lam) + rng.uniform(-0.5, 0.5, nx)
    Tw_row = (np.full(nx, p["T_wall"][1][0]) if Tw is None
              else np.asarray(Tw, dtype=np.float64).reshape(nx))
    H = h[None, :]
    Y = y[:, None]
    phi = tanh_profile(H - Y, W)
    Tsat = p["T_sat"]
    T = np.where(Y < H, Tsat + (Tw_row[None, :] - Tsat) * (1.0 - Y / H), Tsat)
    return phi[None].copy(), T[None].copy(), Tw_row.copy()


def film3d_fields(p: dict, seed: int = 1, h0: float = 32.0, amp: float = 3.0,
                  wavelength: float | None = None):
    """Vapour film of height h(x,y) = h0 + amp cos(2 pi x/l) cos(2 pi y/l)
    + U(-1/2, 1/2) above the heated floor z = 0.  Returns (phi0, T0) of shape
    [nz, ny, nx]."""
    nx, ny, nz, W = p["nx"], p["ny"], p["nz"], p["W"]
    lam = float(nx if wavelength is None else wavelength)
    rng = np.random.default_rng(seed)
    x = _centres(nx)
    y = _centres(ny)
    z = _centres(nz)
    h = (h0 + amp * np.cos(2 * np.pi * x[None, :] / lam)
         * np.cos(2 * np.pi * y[:, None] / lam)
         + rng.uniform(-0.5, 0.5, (ny, nx)))
    H = h[None, :, :]
    Z = z[:, None, None]
    phi = tanh_profile(H - Z, W)
    Tw, Tsat = p["T_wall"][2][0], p["T_sat"]
    T = np.where(Z < H, Tsat + (Tw - Tsat) * (1.0 - Z / H), Tsat)
    return np.ascontiguousarray(phi), np.ascontiguousarray(T)


def drop_fields(p: dict, radius: float = 32.0, centre=None):
    """Liquid drop (phi = 0 inside) of the given radius in vapour."""
    nx, ny, W = p["nx"], p["ny"], p["W"]
    cx, cy = (nx / 2.0, ny / 2.0) if centre is None else centre
    x = _centres(nx)[None, :]
    y = _centres(ny)[:, None]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    phi = tanh_profile(r - radius, W)
    return phi[None].copy(), np.zeros_like(phi)[None].copy()


def random_smooth_fields(p: dict, seed: int, phi_amp: float = 0.5,
                         T_amp: float = 0.1):
    """Smooth random fields (a few Fourier modes) for conservation tests on
    periodic boxes.  phi stays inside (0, 1)."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")
    phi = np.full((nz, ny, nx), 0.5)
    T = np.zeros((nz, ny, nx))
    for _ in range(3):
        kx, ky = rng.integers(1, 3, 2)
        kz = rng.integers(1, 3) if nz > 1 else 0
        ph = rng.uniform(0, 2 * np.pi, 2)
        arg = 2 * np.pi * (kx * x / nx + ky * y / ny + (kz * z / nz if nz > 1 else 0))
        phi += phi_amp / 3.0 * 0.9 * np.sin(arg + ph[0])
        T += T_amp / 3.0 * np.cos(arg + ph[1])
    return phi, T


def gaussian_T(p: dict, amp: float, s: float, centre=None):
    """Gaussian temperature bump T = amp exp(-r^2 / (2 s^2))."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")
    if centre is None:
        centre = (nx / 2.0, ny / 2.0, nz / 2.0)
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2
    if nz > 1:
        r2 = r2 + (z - centre[2]) ** 2
    return amp * np.exp(-r2 / (2.0 * s * s))


def wall_T_row(nx: int, seed: int = 3, mean: float = 1.0, std: float = 0.05):
    """Seeded wall-temperature row T_w(x) ~ N(mean, std^2)."""
    return np.random.default_rng(seed).normal(mean, std, nx)


def random_directions(n: int, count: int, seed: int = 4):
    """Unit-norm random directions (for finite-difference checks)."""
    v = np.random.default_rng(seed).normal(size=(count, n))
    return v / np.linalg.norm(v, axis=1, keepdims=True)
