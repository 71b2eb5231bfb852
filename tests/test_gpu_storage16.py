"""16-bit deviation storage (FP16 / BF16, FP32 arithmetic) against the FP64
oracle.  The bar for compressed storage is 1e-3 relative L2 on phi and T;
|u| and p (small signals) are bounded by the FP32 path's errors plus the
storage rounding and are reported."""
import numpy as np
import pytest

from paper_2003_06342_amd import inputs as I
from tests._parity import compare, gpu_run, need_gpu, oracle_run, say

pytestmark = pytest.mark.gpu


def _film2d():
    prm = I.film2d_params(130, 66)
    prm["gravity"] = [0.0, -2e-5, 0.0]
    phi0, T0, _ = I.film2d_fields(prm, seed=0, h0=12.0, amp=2.0)
    return prm, phi0, T0


def _film3d():
    prm = I.film3d_params(36, nz=37)
    prm["ny"] = 20
    prm["gravity"] = [0.0, 0.0, -5e-5]
    phi0, T0 = I.film3d_fields(prm, seed=1, h0=8.0, amp=1.5, wavelength=36.0)
    return prm, phi0, T0


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
@pytest.mark.parametrize("case,steps", [("film2d", 100), ("film3d", 40)])
def test_deviation_storage(storage, case, steps):
    need_gpu()
    prm, phi0, T0 = _film2d() if case == "film2d" else _film3d()
    say(f"[storage16] {case} {storage} steps={steps}")
    ref = oracle_run(prm, phi0, T0, steps)
    g16 = gpu_run(prm, phi0, T0, steps, storage)
    g32 = gpu_run(prm, phi0, T0, steps, "f32")
    e16, e32 = compare(g16, ref), compare(g32, ref)
    say(f"[storage16] {case} {storage}: {e16} | f32 {e32}")
    assert all(np.isfinite(v) for v in e16.values())
    bar = 1e-3 if storage == "f16dev" else 1e-2
    assert e16["phi"] <= bar and e16["T"] <= bar, e16
