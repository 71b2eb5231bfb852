"""Write tests/golden/adjoint_fp32_floor.json: the rounding floor of any FP32
evaluation of the adjoint on the 512 x 512 film recipe, from the oracle only.

The oracle's reverse pass (torch.autograd, per-step segments checkpointed so
that 512 x 512 fits in memory) is evaluated in float32 and in float64 on the
recipe the GPU adjoint test uses (lambda = 512 gravity, h = 32 + 2 cos +
noise with seed 2, T_w ~ N(1, 0.05^2) with seed 3).  The gradients of
V = mean phi^N are projected on the test's 16 random unit directions of T_w
(seed 4) and of phi0 (seed 5); the stored floor per kind is the relative L2,
over the 16 directions, of the float32 projections against the float64
ones: the same metric the test applies to the GPU adjoint against central
differences.

Usage: python tests/golden/make_adjoint_fp32_floor.py 300 [1000 ...]
(several minutes of CPU per step count and precision).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.lbm_oracle import F64, Model, State  # noqa: E402
from paper_2003_06342_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fp32_floor.json")
NX = NY = 512
SEG = 5


def grads(n: int, dtype):
    prm = I.film2d_params(NX, NY)
    phi0, T0, _ = I.film2d_fields(prm, seed=2, h0=32.0, amp=2.0)
    Tw = I.wall_T_row(NX, seed=3)
    phi = torch.tensor(phi0, dtype=dtype, requires_grad=True)
    tw = torch.tensor(Tw, dtype=dtype, requires_grad=True)
    M = Model(prm, T_wall_faces={(1, 0): tw.reshape(1, 1, -1)}, dtype=dtype)
    st = M.init(phi, torch.tensor(T0, dtype=dtype))

    def seg(k, f, g, s, pp, qp):
        x = State(f, g, s, pp, qp)
        for _ in range(k):
            x = M.step(x)
        return x.f, x.g, x.s, x.phi_prev, x.q_prev

    t = (st.f, st.g, st.s, st.phi_prev, st.q_prev)
    done = 0
    while done < n:
        k = min(SEG, n - done)
        t = checkpoint(seg, k, *t, use_reentrant=True)
        done += k
    V = M.fields(State(*t))["phi"].mean()
    V.backward()
    return tw.grad.double().numpy(), phi.grad.double().numpy()[0]


def rel_l2(x, ref):
    x, ref = np.asarray(x), np.asarray(ref)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def main(steps):
    torch.set_num_threads(min(8, os.cpu_count() or 1))
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_about"] = ("FP32 rounding floor of the 512 x 512 film adjoint (oracle reverse pass in "
                      "float32 vs float64), relative L2 over 16 random directions per kind; "
                      "written by make_adjoint_fp32_floor.py from the oracle only")
    dirs_tw = I.random_directions(NX, 16, seed=4)
    dirs_phi = I.random_directions(NX * NY, 16, seed=5)
    for n in steps:
        t0 = time.time()
        gtw64, gphi64 = grads(n, F64)
        gtw32, gphi32 = grads(n, torch.float32)
        p = lambda g, d: [float(np.dot(g.ravel(), d[k].ravel())) for k in range(16)]
        rec = {"Tw": rel_l2(p(gtw32, dirs_tw), p(gtw64, dirs_tw)),
               "phi0": rel_l2(p(gphi32, dirs_phi), p(gphi64, dirs_phi)),
               "Tw_full_gradient": rel_l2(gtw32, gtw64),
               "phi0_full_gradient": rel_l2(gphi32, gphi64)}
        data[str(n)] = rec
        print(n, rec, f"{time.time() - t0:.0f} s", flush=True)
        json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [300])
