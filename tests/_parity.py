"""Shared helpers of the GPU parity tests: run the HIP path and the FP64
oracle on the same seeded inputs and compare fields."""
from __future__ import annotations

import sys
import time

import numpy as np
import torch

from oracle.lbm_oracle import Model
from paper_2003_06342_amd import lbm

FIELD_KEYS = ("phi", "T", "p", "ux", "uy", "uz")


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def need_gpu():
    assert torch.cuda.is_available(), "GPU test run without a HIP device"
    import os
    assert os.path.exists(lbm.LIB_PATH), "liblbm.so not built"


def rel_l2(x, ref, about_mean=False):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if about_mean:
        x = x - x.mean()
        ref = ref - ref.mean()
    den = np.linalg.norm(ref)
    num = np.linalg.norm(x - ref)
    return num / den if den > 0 else num


def oracle_run(prm, phi0, T0, nsteps, Tw_face=None, u0=None, p0=None):
    faces = None
    if Tw_face is not None:
        axis, side, arr = Tw_face
        shp = [1, 1, 1]
        if axis == 1:
            shp[2] = arr.shape[-1]
        faces = {(axis, side): torch.tensor(np.asarray(arr, dtype=np.float64).reshape(shp))}
    M = Model(prm, T_wall_faces=faces)
    st = M.init(phi0, T0, u0, p0)
    st = M.run(st, nsteps)
    f = M.fields(st)
    out = {k: v.detach().numpy() for k, v in f.items()}
    out["diag"] = M.diagnostics(st)
    return out


def gpu_run(prm, phi0, T0, nsteps, storage, Tw_face=None, u0=None, p0=None, chunks=None):
    sim = lbm.Sim(prm, storage)
    if Tw_face is not None:
        axis, side, arr = Tw_face
        sim.set_wall_T(axis, side, np.asarray(arr, dtype=np.float64))
    sim.init(phi0, T0, u0, p0)
    if chunks is None:
        sim.step(nsteps)
    else:
        for c in chunks:
            sim.step(c)
    f = sim.fields()
    out = {k: v.double().cpu().numpy() for k, v in f.items()}
    out["diag"] = sim.diagnostics(check=False)
    sim.sync()
    sim.close()
    return out


def compare(gpu, ref, keys=("phi", "T", "umag", "p")):
    """Relative L2 per field: phi, T, |u|, p about its mean."""
    errs = {}
    for k in keys:
        if k == "umag":
            g = np.sqrt(gpu["ux"] ** 2 + gpu["uy"] ** 2 + gpu["uz"] ** 2)
            r = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2 + ref["uz"] ** 2)
            errs[k] = rel_l2(g, r)
        elif k == "p":
            errs[k] = rel_l2(gpu["p"], ref["p"], about_mean=True)
        else:
            errs[k] = rel_l2(gpu[k], ref[k])
    return errs


class Timer:
    def __enter__(self):
        self.t = time.time()
        return self

    def __exit__(self, *a):
        self.dt = time.time() - self.t


def fp32_floor(prm, phi0, T0, nsteps):
    """Relative L2 between the oracle evaluated in float32 and in float64 on
    the same inputs: the rounding floor of any FP32 implementation of the
    scheme on this case (nothing here comes from the HIP path)."""
    ref = oracle_run(prm, phi0, T0, nsteps)
    M = Model(prm, dtype=torch.float32)
    st = M.run(M.init(phi0, T0), nsteps)
    f = {k: v.double().numpy() for k, v in M.fields(st).items()}
    return compare(f, ref), ref


def fp32_bars(floor, tol=1e-5, factor=3.0):
    """The 1e-5 relative-L2 bar where FP32 arithmetic allows it, else
    `factor` times the measured FP32 floor of the case."""
    return {k: max(tol, factor * v) for k, v in floor.items()}
