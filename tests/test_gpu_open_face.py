"""GPU parity of open (pressure) faces of f (reading R29: pressure
anti-bounce-back, zero-gradient velocity ghost) against the FP64 oracle, in
2-D (open top of the film; a pressure-driven channel with both x faces open
and no-slip y walls, so corners join an open and a no-slip face) and 3-D
(open top of the film), including an initial velocity field whose ghosts
enter div(u phi) at the open face, and under the extended step (TRT,
biased2 derivatives, local div(u phi)).  FP64 within 1e-10, FP32 within
max(1e-5, 3 x the float32 floor)."""
import numpy as np
import pytest

from paper_2003_06342_amd import inputs as I
from tests._parity import (compare, fp32_bars, fp32_floor, gpu_run, need_gpu, oracle_run, say)

pytestmark = pytest.mark.gpu

OPEN_TOP_2D = dict(f_open=[[False, False], [False, True], [False, False]],
                   p_wall=[[0.0, 0.0], [0.0, 1e-4], [0.0, 0.0]])


def _keys(prm):
    return ["phi"] + (["T"] if prm["heat"] else []) + (["umag", "p"] if prm["ns"] else [])


def _check(name, prm, phi0, T0, n, storage, tol, u0=None):
    need_gpu()
    say(f"[open] {name}: storage={storage} steps={n}")
    ref = oracle_run(prm, phi0, T0, n, u0=u0)
    gpu = gpu_run(prm, phi0, T0, n, storage, u0=u0)
    errs = compare(gpu, ref)
    say(f"[open] {name}: errors {errs}")
    for k in _keys(prm):
        assert errs[k] <= tol, (k, errs)


def film2d_open(**kw):
    prm = I.film2d_params(130, 66)
    prm["gravity"] = [0.0, -2e-5, 0.0]
    prm.update(OPEN_TOP_2D)
    prm.update(kw)
    phi0, T0, _ = I.film2d_fields(prm, seed=0, h0=12.0, amp=2.0)
    return prm, phi0, T0


def test_film2d_open_top_f64():
    prm, phi0, T0 = film2d_open()
    _check("film2d_open_top", prm, phi0, T0, 60, "f64", 1e-10)


def test_film2d_open_top_with_initial_velocity_f64():
    prm, phi0, T0 = film2d_open()
    ny, nx = phi0.shape[1:]
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    ux = 1e-3 * np.sin(2 * np.pi * x)[None, :] * np.sin(np.pi * y / 2)[:, None]
    uy = 1e-3 * np.cos(2 * np.pi * x)[None, :] * y[:, None]
    u0 = [ux[None], uy[None], np.zeros_like(ux)[None]]
    _check("film2d_open_top_u0", prm, phi0, T0, 20, "f64", 1e-10, u0=u0)


def test_film2d_open_top_f32():
    prm, phi0, T0 = film2d_open()
    need_gpu()
    floor, ref = fp32_floor(prm, phi0, T0, 100)
    gpu = gpu_run(prm, phi0, T0, 100, "f32")
    errs = compare(gpu, ref)
    bars = fp32_bars(floor)
    say(f"[open] film2d_open_top f32: gpu {errs} | fp32 floor {floor}")
    for k in _keys(prm):
        assert errs[k] <= bars[k], (k, errs, floor)


def test_pressure_driven_channel_f64():
    nx, ny = 70, 20
    p = I.base_params(dim=2, nx=nx, ny=ny, ns=True, heat=True, phase_change=False,
                      nu_l=0.1, nu_g=0.05, rho_l=1.0, rho_g=0.5, sigma=1e-4,
                      collision="trt", trt_lambda=[3.0 / 16.0, 0.25, 0.25])
    p["bc"] = ["wall", "wall", "periodic"]
    p["phi_wall"] = [[0.0, 0.0], [0.0, 0.0], [0.0, 0.0]]
    p["T_wall"] = [[0.3, 0.1], [0.2, 0.2], [0.0, 0.0]]
    p["f_open"] = [[True, True], [False, False], [False, False]]
    p["p_wall"] = [[2e-4, 0.0], [0.0, 0.0], [0.0, 0.0]]
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    phi0 = I.tanh_profile(np.sqrt((X - 30.0) ** 2 + (Y - 10.0) ** 2) - 5.0, 4.0)[None]
    T0 = (0.2 + 0.05 * np.cos(2 * np.pi * X / nx))[None]
    _check("channel_open_x", p, phi0, T0, 150, "f64", 1e-10)


def test_film3d_open_top_f64():
    prm = I.film3d_params(36, nz=37)
    prm["ny"] = 20
    prm["gravity"] = [0.0, 0.0, -5e-5]
    prm["f_open"] = [[False, False], [False, False], [False, True]]
    prm["p_wall"] = [[0.0, 0.0], [0.0, 0.0], [0.0, 1e-4]]
    phi0, T0 = I.film3d_fields(prm, seed=1, h0=8.0, amp=1.5, wavelength=36.0)
    _check("film3d_open_top", prm, phi0, T0, 20, "f64", 1e-10)


@pytest.mark.parametrize("dim", [2, 3])
def test_open_top_16bit_storage(dim):
    """Open top with FP16-deviation storage (the open face's reflected f is
    stored against f's global reference like every other slot): within the
    16-bit bars of the closed film (phi 1e-4, T, |u| and p 1e-3)."""
    if dim == 2:
        prm, phi0, T0 = film2d_open()
        n = 60
    else:
        prm = I.film3d_params(36, nz=37)
        prm["ny"] = 20
        prm["gravity"] = [0.0, 0.0, -5e-5]
        prm["f_open"] = [[False, False], [False, False], [False, True]]
        prm["p_wall"] = [[0.0, 0.0], [0.0, 0.0], [0.0, 1e-4]]
        phi0, T0 = I.film3d_fields(prm, seed=1, h0=8.0, amp=1.5, wavelength=36.0)
        n = 20
    need_gpu()
    say(f"[open] {dim}-D open top f16dev: steps={n}")
    ref = oracle_run(prm, phi0, T0, n)
    errs = compare(gpu_run(prm, phi0, T0, n, "f16dev"), ref)
    say(f"[open] {dim}-D open top f16dev: errors {errs}")
    for k, bar in {"phi": 1e-4, "T": 1e-3, "umag": 1e-3, "p": 1e-3}.items():
        assert errs[k] <= bar, (k, errs)


EXT_ALL = dict(collision="trt", trt_lambda=[0.25, 3.0 / 16.0, 0.3], grad_scheme="biased2",
               div_local=True)


@pytest.mark.parametrize("dim", [2, 3])
def test_open_top_with_extended_step_f64(dim):
    """The open top under the extended step (TRT collision, biased2
    derivatives, local div(u phi)): the open face's reflected f enters the
    TRT pairs and the biased differences read phi ghosts beyond it; FP64
    within 1e-10."""
    if dim == 2:
        prm, phi0, T0 = film2d_open(**EXT_ALL)
        _check("film2d_open_top_ext", prm, phi0, T0, 60, "f64", 1e-10)
    else:
        prm = I.film3d_params(80, nz=37)
        prm["ny"] = 20
        prm["gravity"] = [0.0, 0.0, -5e-5]
        prm["f_open"] = [[False, False], [False, False], [False, True]]
        prm["p_wall"] = [[0.0, 0.0], [0.0, 0.0], [0.0, 1e-4]]
        prm.update(EXT_ALL)
        phi0, T0 = I.film3d_fields(prm, seed=1, h0=8.0, amp=1.5, wavelength=80.0)
        _check("film3d_open_top_ext", prm, phi0, T0, 20, "f64", 1e-10)


def test_open_top_with_extended_step_f32():
    """The same 2-D case with FP32 storage (64 x 16 tiles, the extended
    kernel), within max(1e-5, 3 x the float32 floor)."""
    prm, phi0, T0 = film2d_open(**EXT_ALL)
    n = 60
    need_gpu()
    floor, ref = fp32_floor(prm, phi0, T0, n)
    errs = compare(gpu_run(prm, phi0, T0, n, "f32"), ref)
    bars = fp32_bars(floor)
    say(f"[open] film2d_open_top_ext f32: {errs} | floor {floor}")
    for k in _keys(prm):
        assert errs[k] <= bars[k], (k, errs, floor)


@pytest.mark.parametrize("dim", [2, 3])
def test_open_top_with_extended_step_16bit(dim):
    """The open top under the extended step with FP16-deviation storage
    (64 x 8 tiles in 2-D, 64 x 16 x 16 in 3-D, the extended kernels): within
    the 16-bit bars (phi 1e-4; T, |u| and p 1e-3)."""
    if dim == 2:
        prm, phi0, T0 = film2d_open(**EXT_ALL)
        n = 60
    else:
        prm = I.film3d_params(80, nz=37)
        prm["ny"] = 20
        prm["gravity"] = [0.0, 0.0, -5e-5]
        prm["f_open"] = [[False, False], [False, False], [False, True]]
        prm["p_wall"] = [[0.0, 0.0], [0.0, 0.0], [0.0, 1e-4]]
        prm.update(EXT_ALL)
        phi0, T0 = I.film3d_fields(prm, seed=1, h0=8.0, amp=1.5, wavelength=80.0)
        n = 20
    need_gpu()
    say(f"[open] ext 16-bit dim={dim}: {n} steps")
    errs = compare(gpu_run(prm, phi0, T0, n, "f16dev"), oracle_run(prm, phi0, T0, n))
    say(f"[open] ext 16-bit dim={dim}: {errs}")
    for k, bar in {"phi": 1e-4, "T": 1e-3, "umag": 1e-3, "p": 1e-3}.items():
        assert errs[k] <= bar, (dim, k, errs)
