"""GPU parity of the extended step kernels (through the C ABI) against the
FP64 oracle: TRT and MRT collisions (reading R26), the biased directional
derivatives of the NS source (R27) and the local div(u phi) (R8b), alone and
combined, in 2-D and 3-D, on ragged tiles with walls.

Bars: FP64 storage within 1e-10 relative L2 (rounding order only); FP32
storage within max(1e-5, 3 x the FP32 rounding floor the oracle itself
shows when evaluated in float32 on the same case); FP16-deviation storage
within 1e-3 on phi, T, |u| and p."""
import numpy as np
import pytest

from paper_2003_06342_amd import inputs as I
from tests._parity import (compare, fp32_bars, fp32_floor, gpu_run, need_gpu, oracle_run, say)

pytestmark = pytest.mark.gpu

TRT = dict(collision="trt", trt_lambda=[0.25, 3.0 / 16.0, 0.3])
MRT = dict(collision="mrt", mrt_rates=[[1.1, 1.2, 1.3, 1.4], [1.0, 1.15, 1.25, 1.35],
                                       [1.05, 1.2, 1.3, 1.1]])
VARIANTS = {
    "trt": TRT,
    "mrt": MRT,
    "biased1": dict(grad_scheme="biased1"),
    "biased2": dict(grad_scheme="biased2"),
    "div_local": dict(div_local=True),
    "trt+biased2+div_local": dict(TRT, grad_scheme="biased2", div_local=True),
    "mrt+biased1": dict(MRT, grad_scheme="biased1"),
}


def film2d(nx=130, ny=66, h0=12.0, amp=2.0, **kw):
    prm = I.film2d_params(nx, ny)
    prm["gravity"] = [0.0, -2e-5, 0.0]
    prm.update(kw)
    phi0, T0, _ = I.film2d_fields(prm, seed=0, h0=h0, amp=amp)
    return prm, phi0, T0


def film3d(nx=36, ny=20, nz=37, h0=8.0, amp=1.5, **kw):
    prm = I.film3d_params(nx, nz=nz)
    prm["ny"] = ny
    prm["gravity"] = [0.0, 0.0, -5e-5]
    prm.update(kw)
    phi0, T0 = I.film3d_fields(prm, seed=1, h0=h0, amp=amp, wavelength=float(nx))
    return prm, phi0, T0


def _keys(prm):
    return ["phi"] + (["T"] if prm["heat"] else []) + (["umag", "p"] if prm["ns"] else [])


def _check(name, prm, phi0, T0, nsteps, storage, tol):
    need_gpu()
    dims = f"{prm['nx']}x{prm['ny']}" + (f"x{prm['nz']}" if prm["dim"] == 3 else "")
    say(f"[ext] {name}: {dims} storage={storage} steps={nsteps}")
    ref = oracle_run(prm, phi0, T0, nsteps)
    gpu = gpu_run(prm, phi0, T0, nsteps, storage)
    errs = compare(gpu, ref)
    say(f"[ext] {name}: errors {errs}")
    for k in _keys(prm):
        assert errs[k] <= tol, (k, errs)
    return errs


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_film2d_f64(variant):
    prm, phi0, T0 = film2d(**VARIANTS[variant])
    _check(f"film2d_{variant}", prm, phi0, T0, 60, "f64", 1e-10)


def test_film2d_on_x_walls_f64():
    """The film turned on its side (walls on x, periodic y): the x ghosts of
    the second-order biased differences and of the local divergence."""
    prm, phi0, T0 = film2d(**VARIANTS["trt+biased2+div_local"])
    nx, ny = 70, 44
    prm.update(nx=nx, ny=ny, bc=["wall", "periodic", "periodic"],
               phi_wall=[[1.0, 1.0], [0.0, 0.0], [0.0, 0.0]],
               T_wall=[[1.0, 0.0], [0.0, 0.0], [0.0, 0.0]], gravity=[-2e-5, 0.0, 0.0])
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    h = 10.0 + 1.5 * np.cos(2 * np.pi * y / ny)
    phi0 = I.tanh_profile(h[:, None] - x[None, :], prm["W"])[None]
    T0 = np.where(x[None, :] < h[:, None], 1.0 - x[None, :] / h[:, None], 0.0)[None]
    _check("film2d_xwalls_ext", prm, phi0, T0, 40, "f64", 1e-10)


def test_heat_only_mrt_and_ns_only_trt_f64():
    """Family subsets: heat + phase field without NS under MRT; NS + phase
    field without heat under TRT with the second-order biased scheme."""
    prm, phi0, T0 = film2d(ns=False, **MRT)
    _check("film2d_noNS_mrt", prm, phi0, T0, 50, "f64", 1e-10)
    p = I.drop_params(64)
    p.update(TRT, grad_scheme="biased2")
    phi, T = I.drop_fields(p, radius=14.0)
    _check("drop64_trt_biased2", p, phi, T, 50, "f64", 1e-10)


@pytest.mark.parametrize("variant", ["trt", "trt+biased2+div_local"])
def test_film2d_f32(variant):
    prm, phi0, T0 = film2d(**VARIANTS[variant])
    nsteps = 100
    need_gpu()
    floor, ref = fp32_floor(prm, phi0, T0, nsteps)
    gpu = gpu_run(prm, phi0, T0, nsteps, "f32")
    errs = compare(gpu, ref)
    bars = fp32_bars(floor)
    say(f"[ext] film2d_{variant} f32: gpu {errs} | fp32 floor {floor}")
    for k in _keys(prm):
        assert errs[k] <= bars[k], (k, errs, floor)


def test_film2d_f16dev_trt():
    prm, phi0, T0 = film2d(**TRT)
    _check("film2d_trt_f16dev", prm, phi0, T0, 60, "f16dev", 1e-3)


@pytest.mark.parametrize("variant", ["trt", "biased2", "div_local", "trt+biased2+div_local"])
def test_film3d_f64(variant):
    prm, phi0, T0 = film3d(**VARIANTS[variant])
    _check(f"film3d_{variant}", prm, phi0, T0, 20, "f64", 1e-10)


def test_film3d_mrt_without_ns_f64():
    """MRT is built for the D3Q7 families (phase field and heat)."""
    prm, phi0, T0 = film3d(ns=False, **MRT)
    _check("film3d_noNS_mrt", prm, phi0, T0, 20, "f64", 1e-10)


@pytest.mark.parametrize("variant", ["trt", "trt+biased2+div_local"])
def test_film3d_f32(variant):
    """The FP32 extended 3-D step runs on 64 x 16 tiles: 80 columns give one
    full and one ragged tile in x, 20 rows one full and one ragged in y."""
    prm, phi0, T0 = film3d(nx=80, **VARIANTS[variant])
    nsteps = 20
    need_gpu()
    floor, ref = fp32_floor(prm, phi0, T0, nsteps)
    gpu = gpu_run(prm, phi0, T0, nsteps, "f32")
    errs = compare(gpu, ref)
    bars = fp32_bars(floor)
    say(f"[ext] film3d_{variant} f32: gpu {errs} | fp32 floor {floor}")
    for k in _keys(prm):
        assert errs[k] <= bars[k], (k, errs, floor)


def test_film3d_f16dev_trt_biased2():
    prm, phi0, T0 = film3d(nx=80, **VARIANTS["trt+biased2+div_local"])
    _check("film3d_trt+biased2+div_local_f16dev", prm, phi0, T0, 20, "f16dev", 1e-3)


def test_film2d_on_x_walls_f16dev():
    """The extended step on the film turned on its side, FP16-deviation
    storage: the 16-bit codec's wall links along x (g referenced to the
    node's own phi beyond a wall), within 1e-3."""
    prm, phi0, T0 = film2d(**VARIANTS["trt+biased2+div_local"])
    nx, ny = 70, 44
    prm.update(nx=nx, ny=ny, bc=["wall", "periodic", "periodic"],
               phi_wall=[[1.0, 1.0], [0.0, 0.0], [0.0, 0.0]],
               T_wall=[[1.0, 0.0], [0.0, 0.0], [0.0, 0.0]], gravity=[-2e-5, 0.0, 0.0])
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    h = 10.0 + 1.5 * np.cos(2 * np.pi * y / ny)
    phi0 = I.tanh_profile(h[:, None] - x[None, :], prm["W"])[None]
    T0 = np.where(x[None, :] < h[:, None], 1.0 - x[None, :] / h[:, None], 0.0)[None]
    _check("film2d_xwalls_ext_f16dev", prm, phi0, T0, 40, "f16dev", 1e-3)
