"""The binomial tape policy (LBM_TAPE_BINOMIAL) against the sqrt(T) policy
through the C ABI: both reverse sweeps run the same adjoint kernels on the
same recomputed states in the same order, so the gradients must agree bit
for bit, for step counts that exercise every branch of the schedule (one
step, no free slot, the spine, the recursion); the binomial tape is
smaller for long runs."""
import ctypes as C

import numpy as np
import pytest

from paper_2003_06342_amd import inputs as I
from tests._parity import need_gpu, say

pytestmark = pytest.mark.gpu


def _grads(prm, phi0, T0, Tw, n, storage, policy):
    from paper_2003_06342_amd import lbm
    sim = lbm.Sim(prm, storage)
    sim.set_wall_T(1, 0, Tw)
    sim.init(phi0, T0)
    sim.forward_taped(n, policy)
    N = prm["nx"] * prm["ny"]
    g = sim.backward(np.full((prm["ny"], prm["nx"]), 1.0 / N),
                     gT=np.full((prm["ny"], prm["nx"]), 0.5 / N))
    out = {k: v.cpu().numpy() for k, v in g.items()}
    size = C.c_size_t()
    lbm._check(sim.lib.lbm_tape_size(sim.ctx, int(n), int(policy), C.byref(size)))
    sim.sync()
    sim.close()
    return out, size.value


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 3, 7, 40])
def test_binomial_equals_sqrt_bitwise(storage, n):
    need_gpu()
    from paper_2003_06342_amd import lbm
    prm = I.film2d_params(70, 34)
    prm["gravity"] = [0.0, -2e-4, 0.0]
    phi0, T0, _ = I.film2d_fields(prm, seed=2, h0=6.0, amp=1.5)
    Tw = I.wall_T_row(70, seed=3)
    say(f"[tape] {storage} n={n}: sqrt vs binomial")
    a, sa = _grads(prm, phi0, T0, Tw, n, storage, lbm.LBM_TAPE_SQRT)
    b, sb = _grads(prm, phi0, T0, Tw, n, storage, lbm.LBM_TAPE_BINOMIAL)
    for k in ("phi0", "T0", "Tw"):
        assert np.array_equal(a[k], b[k]), (k, np.abs(a[k] - b[k]).max())
        assert np.isfinite(a[k]).all() and np.abs(a[k]).max() > 0
    say(f"[tape] {storage} n={n}: identical; tape bytes sqrt {sa}, binomial {sb}")
    if n >= 40:
        assert sb < sa
