"""16-bit deviation storage (FP16 / BF16, FP32 arithmetic) against the FP64
oracle.  f is stored as (v - w_i ref_f) * 2^k with a global reference; g as
deviations from w_i phi of the node that reads the slot (its lagged phi), s
as deviations from w_i T(x) of the node x that stored it (a T_ref plane).

Measured (relative L2 after 100 steps in 2-D, 40 in 3-D): FP16 phi 7e-6 /
5e-6, T 7e-5 / 1.3e-4, |u| 3.5e-4 / 4e-4, p 7.6e-4 / 5e-4 (2-D / 3-D).  The
per-node references took T from 5e-3 and phi from 5e-4.  BF16 is about 8x
worse (3 fewer mantissa bits).

Bars: FP16 within the 1e-3 compressed-storage target on every field (phi
1e-4; T, |u| and p, about its mean, 1e-3).  The largest FP16 pressure error
of the 16-bit GPU tests is 8.4e-4 (the 2-D TRT film).  BF16 misses the 1e-3
target for |u| and p; its bars record the measured levels with margin."""
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
    bars = ({"phi": 1e-4, "T": 1e-3, "umag": 1e-3, "p": 1e-3} if storage == "f16dev" else
            {"phi": 1e-3, "T": 5e-3, "umag": 2e-2, "p": 5e-2})
    for k, bar in bars.items():
        assert e16[k] <= bar, (k, e16)
    # the compressed path is never better than FP32 storage
    assert e16["phi"] >= e32["phi"]


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_film3d_16bit_step_tiles_interior(storage):
    """The 16-bit 3-D step's 64 x 16 tiles with interior (seam-free) tiles in
    x and y and ragged last tiles: 200 x 56 x 20, 40 steps, same bars as the
    film3d case above."""
    need_gpu()
    prm = I.film3d_params(200, nz=20, wavelength=100.0)
    prm["ny"] = 56
    prm["gravity"] = [0.0, 0.0, -5e-5]
    phi0, T0 = I.film3d_fields(prm, seed=3, h0=6.0, amp=1.5, wavelength=100.0)
    steps = 40
    say(f"[storage16] film3d 200x56x20 {storage} steps={steps}")
    ref = oracle_run(prm, phi0, T0, steps)
    e16 = compare(gpu_run(prm, phi0, T0, steps, storage), ref)
    say(f"[storage16] film3d 200x56x20 {storage}: {e16}")
    bars = ({"phi": 1e-4, "T": 1e-3, "umag": 1e-3, "p": 1e-3} if storage == "f16dev" else
            {"phi": 1e-3, "T": 5e-3, "umag": 2e-2, "p": 5e-2})
    for k, bar in bars.items():
        assert e16[k] <= bar, (k, e16)


def test_compressed_storage_64cubed_instance_of_512cubed_run():
    """The error instance of the 512^3 compressed-storage workload: a 64^3
    film (z = 16 + 3 cos cos + noise, seed 6) with the 512^3 run's lattice
    parameters (its gravity), FP16 / BF16 / FP32 storage against the FP64
    oracle after 100 steps.  This instance enters the vapour-side
    sharpening regime at about 150 steps: the oracle evaluated in float32
    departs from FP64 by 5e-7 (phi) at 100 steps but 1.9e-3 at 200 and
    2.9e-3 at 300, so a comparison of storage precisions is meaningful only
    before the onset."""
    need_gpu()
    prm = I.film3d_params(64, wavelength=512.0)
    phi0, T0 = I.film3d_fields(prm, seed=6, h0=16.0, amp=3.0, wavelength=64.0)
    steps = 100
    say(f"[storage16] 64^3 instance: oracle {steps} steps")
    ref = oracle_run(prm, phi0, T0, steps)
    errs = {}
    for st in ("f32", "f16dev", "bf16dev"):
        errs[st] = compare(gpu_run(prm, phi0, T0, steps, st), ref)
        say(f"[storage16] 64^3 {st}: {errs[st]}")
    for k in ("phi", "T", "umag"):
        assert errs["f16dev"][k] <= 1e-3, ("f16dev", k, errs["f16dev"])
        assert errs["bf16dev"][k] <= 2e-2, ("bf16dev", k, errs["bf16dev"])
    assert errs["f16dev"]["p"] <= 1e-3
    for k in ("phi", "T", "umag", "p"):
        assert errs["f32"][k] <= 1e-5, ("f32", k, errs["f32"])


def test_deviation_storage_full_size_bench_grid():
    """FP16 and BF16 storage on the benchmark grid itself (1024 x 2048 film,
    seed 0), in the launch configuration bench.py times (64 x 4 tiles, one
    node per lane): 20 steps against the FP64 oracle, with the 2-D bars
    above."""
    need_gpu()
    prm = I.film2d_params(1024, 2048)
    phi0, T0, _ = I.film2d_fields(prm, seed=0, h0=64.0, amp=4.0)
    n = 20
    say(f"[storage16] full size 1024x2048: oracle {n} steps")
    ref = oracle_run(prm, phi0, T0, n)
    for storage, bars in (("f16dev", {"phi": 1e-4, "T": 1e-3, "umag": 1e-3, "p": 1e-3}),
                          ("bf16dev", {"phi": 1e-3, "T": 5e-3, "umag": 2e-2, "p": 5e-2})):
        e = compare(gpu_run(prm, phi0, T0, n, storage), ref)
        say(f"[storage16] full size {storage}: {e}")
        for k, bar in bars.items():
            assert e[k] <= bar, (storage, k, e)

