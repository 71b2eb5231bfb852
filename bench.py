"""Throughput benchmark of the fused phase-change LBM step on one MI355X.

Headline workload: 2-D film boiling on 1024 x 2048 nodes, D2Q9 for f, g and
s, FP32 storage (the film-boiling parameter set of the paper's Sec. 5.1 in
lattice units; seeded synthetic initial film).  A step is one fused pass of
the whole hot path over the grid.  Prints ONE JSON line.

  value      MLUPS = nodes * steps / seconds / 1e6 (the paper's metric, Sec. 3.5)
  roofline   HBM-bound: algorithmic bytes per node update (populations read
             once and written once plus the lagged phi and q) over the step
             kernel's average launch duration: HIP events on its launch
             stream around the timed steps, divided by their number
  cpu_baseline  the FP64 oracle timed on a bounded sample of the same
             workload on this host's cores
  context.pattern_probe  a compute-free kernel with the step's exact HBM
             access pattern, and a plain copy of the same bytes: the
             bandwidth the device gives this pattern
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS + % HBM roofline, FP32 & FP16-store vs FP64 oracle error; adjoint/fwd"


def bytes_per_node(dim: int, q_total: int, storage: str) -> int:
    """Algorithmic bytes per node update: every population read once and
    written once, plus phi_prev and q_prev read and written (FP32, FP64 for
    FP64 storage)."""
    pe = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}[storage]
    se = 8 if storage == "f64" else 4
    return q_total * pe * 2 + 2 * se * 2


def impl_bytes_per_node(dim: int, q_total: int, storage: str) -> int:
    """Bytes per node update this implementation moves at best: the
    algorithmic bytes plus, for 16-bit storage, the per-node temperature
    reference plane of the s family (FP32, read and written)."""
    extra = 2 * 4 if storage in ("f16dev", "bf16dev") else 0
    return bytes_per_node(dim, q_total, storage) + extra


# sources of the dominant kernel (k_step2d); HBM counters recorded under
# profiles/ are used only while these are unchanged
STEP2D_SOURCES = ("lbm_device.h", "lbm_kernels.h", "lbm_tile2d.h", "lbm_step2d.hip")


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2003_06342_amd", "csrc")
    for name in STEP2D_SOURCES:
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def time_variant(prm, fields, storage, steps, warmup):
    import torch
    from paper_2003_06342_amd import lbm
    sim = lbm.Sim(prm, storage)
    sim.init(*fields)
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = sim.stream
    # whole-job timing of exactly `steps` steps (host clock), and the average
    # launch duration of the step kernel from HIP events on its launch stream
    # around the same timed region (each step is one kernel launch)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms = ev0.elapsed_time(ev1) / steps
    diag = sim.diagnostics(check=False)
    sim.close()
    n = prm["nx"] * prm["ny"] * prm["nz"]
    return dict(ms_per_step=1e3 * dt / steps, mlups=n * steps / dt / 1e6, kernel_ms=kern_ms,
                nodes=n, finite=diag["nonfinite"] == 0)


def adjoint_ratio(nx=512, ny=512, nsteps=200):
    """Time of the reverse sweep per step (segment recompute included) over
    the forward step time, FP32, film recipe at 512 x 512."""
    import numpy as np
    import torch
    from paper_2003_06342_amd import inputs as I
    from paper_2003_06342_amd import lbm
    prm = I.film2d_params(nx, ny)
    phi0, T0, _ = I.film2d_fields(prm, seed=2, h0=32.0, amp=2.0)
    sim = lbm.Sim(prm, "f32")
    sim.set_wall_T(1, 0, I.wall_T_row(nx, seed=3))
    sim.init(phi0, T0)
    sim.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(nsteps)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / nsteps
    sim.init(phi0, T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.forward_taped(nsteps)
    torch.cuda.synchronize()
    t_tape = (time.perf_counter() - t0) / nsteps
    g = np.full((ny, nx), 1.0 / (nx * ny))
    sim.backward(g)   # warm-up of the adjoint kernels
    torch.cuda.synchronize()
    sim.init(phi0, T0)
    sim.forward_taped(nsteps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.backward(g)
    torch.cuda.synchronize()
    t_bwd = (time.perf_counter() - t0) / nsteps
    sim.close()
    # sqrt(T) checkpointing: segments of K = ceil(sqrt(N)) steps; the reverse
    # sweep recomputes K - 1 steps per segment (taped forward steps)
    K = math.ceil(math.sqrt(nsteps))
    nseg = (nsteps + K - 1) // K
    t_adj = t_bwd - (nsteps - nseg) * t_tape / nsteps
    return dict(grid=f"{nx}x{ny}", steps=nsteps, fwd_ms=round(1e3 * t_fwd, 4),
                taped_fwd_ms=round(1e3 * t_tape, 4), bwd_ms_per_step=round(1e3 * t_bwd, 4),
                ratio_with_recompute=round(t_bwd / t_fwd, 3),
                ratio_adjoint_kernels=round(t_adj / t_fwd, 3))


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prm, fields, budget_s=12.0):
    """FP64 oracle on the same grid, timed on this host's cores: as many
    whole steps as fit about budget_s with all threads torch uses, then
    with one thread (at most a few steps)."""
    import torch
    from oracle.lbm_oracle import Model
    M = Model(prm)
    n = prm["nx"] * prm["ny"] * prm["nz"]

    def timed(budget, kmax):
        st = M.init(*fields)
        t0 = time.perf_counter()
        st = M.step(st)
        one = time.perf_counter() - t0
        k = max(1, min(kmax, int(budget / max(one, 1e-3)) - 1))
        t0 = time.perf_counter()
        for _ in range(k):
            st = M.step(st)
        return k, time.perf_counter() - t0

    nthreads = torch.get_num_threads()
    k, dt = timed(budget_s, 20)
    torch.set_num_threads(1)
    try:
        k1, dt1 = timed(budget_s, 4)
    finally:
        torch.set_num_threads(nthreads)
    return dict(value=n * k / dt / 1e6, unit="MLUPS", cores=nthreads, kind="oracle",
                value_1thread=n * k1 / dt1 / 1e6, cpu_model=cpu_model(), nproc=os.cpu_count(),
                sample=f"{k} FP64 oracle steps of the full {prm['nx']}x{prm['ny']} film grid on "
                       f"{nthreads} threads ({dt:.1f} s), and {k1} on 1 thread ({dt1:.1f} s), each "
                       f"after 1 untimed step")


def traffic_entry(name: str, nodes: int):
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != kernel_sources_hash():
        return None
    return d.get("bytes_per_launch")


def pattern_probe(nx=1024, ny=2048, reps=50):
    """Bandwidth of the step's HBM access pattern with no arithmetic: the
    probe kernel copies the 29 planes of the FP32 2-D step (27 populations
    read at the pull offsets, phi_prev and q_prev) over the interior nodes
    of the headline grid.  Beside it, copies of the same byte count: a
    hand-written 16-byte streaming copy (plain and non-temporal) and torch's
    copy_.  All timed with HIP events on the launch stream."""
    import ctypes
    import torch
    path = os.path.join(ROOT, "benchprobe", "libstream_probe.so")
    if not os.path.exists(path):
        raise ImportError(f"{path} not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    lib.stream_probe_pull_pattern.restype = ctypes.c_int
    lib.stream_probe_pull_pattern.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_void_p]
    lib.stream_probe_copy16.restype = ctypes.c_int
    lib.stream_probe_copy16.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong,
                                        ctypes.c_int, ctypes.c_void_p]
    n = 29 * nx * ny
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()

    def probe():
        rc = lib.stream_probe_pull_pattern(a.data_ptr(), b.data_ptr(), nx, ny, st.cuda_stream)
        if rc != 0:
            raise RuntimeError(f"probe launch failed ({rc})")

    def copy16(nt):
        def run():
            rc = lib.stream_probe_copy16(a.data_ptr(), b.data_ptr(), 4 * n, nt, st.cuda_stream)
            if rc != 0:
                raise RuntimeError(f"copy16 launch failed ({rc})")
        return run

    def timed(fn):
        for _ in range(5):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_p = timed(probe)
    ms_16 = timed(copy16(0))
    ms_16nt = timed(copy16(1))
    ms_c = timed(lambda: b.copy_(a))
    bytes_p = 2 * 29 * 4 * (nx - 2) * (ny - 2)
    bytes_c = 2 * 4 * n
    del a, b
    torch.cuda.empty_cache()
    gbs = lambda by, ms: round(by / ms / 1e6, 1)
    return {"pull_pattern_ms": round(ms_p, 5), "pull_pattern_GBs": gbs(bytes_p, ms_p),
            "copy16_same_bytes_ms": round(ms_16, 5), "copy16_same_bytes_GBs": gbs(bytes_c, ms_16),
            "copy16_nt_same_bytes_ms": round(ms_16nt, 5),
            "copy16_nt_same_bytes_GBs": gbs(bytes_c, ms_16nt),
            "torch_copy_same_bytes_ms": round(ms_c, 5),
            "torch_copy_same_bytes_GBs": gbs(bytes_c, ms_c)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 512 MiB device copy (HBM counter calibration)")
    ap.add_argument("--only", choices=["film3d256", "adjoint", "film2d_f16dev", "film3d512_f32",
                                       "film3d512_f16dev", "multimode_f32", "multimode_f16dev",
                                       "film2d_ext", "film3d256_ext"],
                    help="run one secondary measurement alone (for profiling) and print it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU slab decomposition is design-only)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2003_06342_amd import inputs as I
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.only == "film3d256":
        p3 = I.film3d_params(256)
        f3 = I.film3d_fields(p3, seed=1, h0=32.0, amp=3.0)
        r = time_variant(p3, f3, "f32", args.steps, args.warmup)
        print(json.dumps({"film3d_256^3_f32": r}), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps({"adjoint_512x512_f32": adjoint_ratio()}), flush=True)
        return
    if args.only in ("film3d512_f32", "film3d512_f16dev"):
        st = args.only.split("_")[1]
        p5 = I.film3d_params(512)
        f5 = I.film3d_fields(p5, seed=5, h0=64.0, amp=6.0)
        r = time_variant(p5, f5, st, args.steps, args.warmup)
        print(json.dumps({f"film3d_512^3_{st}": r}), flush=True)
        return
    if args.only in ("multimode_f32", "multimode_f16dev"):
        st = args.only.split("_")[1]
        pm = I.multimode_params(4096, 3072, jacob=0.1)
        fm = I.multimode_fields(pm, seed=7)[:2]
        r = time_variant(pm, fm, st, args.steps, args.warmup)
        print(json.dumps({f"multimode_4096x3072_Ja0.1_{st}": r}), flush=True)
        return
    if args.only in ("film2d_ext", "film3d256_ext"):
        # the extended step with every option at once: TRT collision, biased2
        # directional derivatives and the local div(u phi)
        ext = dict(collision="trt", trt_lambda=[0.25, 3.0 / 16.0, 0.25], grad_scheme="biased2",
                   div_local=True)
        if args.only == "film2d_ext":
            pe = dict(I.film2d_params(1024, 2048), **ext)
            fe = I.film2d_fields(pe, seed=0, h0=64.0, amp=4.0)[:2]
            name = "film2d_1024x2048_f32_trt_biased2_divlocal"
        else:
            pe = dict(I.film3d_params(256), **ext)
            fe = I.film3d_fields(pe, seed=1, h0=32.0, amp=3.0)
            name = "film3d_256^3_f32_trt_biased2_divlocal"
        r = time_variant(pe, fe, "f32", args.steps, args.warmup)
        print(json.dumps({name: r}), flush=True)
        return
    if args.only == "film2d_f16dev":
        p2 = I.film2d_params(1024, 2048)
        f2 = I.film2d_fields(p2, seed=0, h0=64.0, amp=4.0)[:2]
        r = time_variant(p2, f2, "f16dev", args.steps, args.warmup)
        print(json.dumps({"film2d_1024x2048_f16dev": r}), flush=True)
        return

    nx, ny = 1024, 2048
    prm = I.film2d_params(nx, ny)
    phi0, T0, _ = I.film2d_fields(prm, seed=0, h0=64.0, amp=4.0)
    fields = (phi0, T0)
    head = time_variant(prm, fields, "f32", args.steps, args.warmup)
    bpn = bytes_per_node(2, 27, "f32")
    achieved = bpn * head["nodes"] / (head["kernel_ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(head["mlups"], 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2-D film boiling, D2Q9 f+g+s, FP32 populations",
                   "nx": nx, "ny": ny, "global_batch": nx * ny, "seq_len": 1,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_entry("k_step2d_film1024x2048_f32", head["nodes"]),
                     "kernel": "k_step2d<float,float,NS,HEAT,STEP,16,EXT=false,NTS=true,D2Q9>",
                     "bytes_per_node": bpn, "kernel_ms": round(head["kernel_ms"], 5)},
        "context": {"paper_K80_MLUPS_1024x1024": 80.96, "paper_Xeon16c_MLUPS_1024x1024": 11.97},
    }
    if not head["finite"]:
        out["warning"] = "non-finite values after the timed run"
    # the device's bandwidth on this kernel's access pattern without compute
    out["context"]["pattern_probe"] = pattern_probe(nx, ny)
    if not args.no_variants:
        var = {}

        def record(name, prm_v, fields_v, st, q, steps, warm):
            r = time_variant(prm_v, fields_v, st, steps, warm)
            b = bytes_per_node(prm_v["dim"], q, st)
            bi = impl_bytes_per_node(prm_v["dim"], q, st)
            rate = r["nodes"] / (r["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
            var[name] = dict(mlups=round(r["mlups"], 1), kernel_ms=round(r["kernel_ms"], 5),
                             bytes_per_node=b, hbm_frac=round(b * rate, 4))
            if bi != b:   # 16-bit storage: the per-node T_ref plane, reported apart
                var[name]["impl_bytes_per_node"] = bi
                var[name]["impl_hbm_frac"] = round(bi * rate, 4)
        for st in ("f64", "f16dev", "bf16dev"):
            record(f"film2d_1024x2048_{st}", prm, fields, st, 27, max(20, args.steps // 4), 5)
        # the extended step options (TRT / MRT collision, biased directional
        # derivatives, local div(u phi)): the same bytes as the default step
        ext_opts = {"trt": dict(collision="trt", trt_lambda=[0.25, 3.0 / 16.0, 0.25]),
                    "mrt": dict(collision="mrt", mrt_rates=[[1.1, 1.2, 1.3, 1.4]] * 3),
                    "biased2": dict(grad_scheme="biased2"),
                    "div_local": dict(div_local=True)}
        for name, kw in ext_opts.items():
            record(f"film2d_1024x2048_f32_{name}", dict(prm, **kw), fields, "f32", 27,
                   max(20, args.steps // 4), 5)
        # second 2-D workload: the multi-mode film of Sec. 5.3 (4096 x 3072)
        for ja in (0.1, 0.025):
            pm = I.multimode_params(4096, 3072, jacob=ja)
            fm = I.multimode_fields(pm, seed=7)[:2]
            for st in (("f32", "f16dev") if ja == 0.1 else ("f32",)):
                record(f"multimode_4096x3072_Ja{ja}_{st}", pm, fm, st, 27, max(20, args.steps // 4), 5)
            del fm
        # the adjoint first: after the 3-D grids (tens of GB) it times slower
        try:
            var["adjoint_512x512_f32"] = adjoint_ratio()
        except Exception as e:  # report, do not hide the headline
            var["adjoint_512x512_f32"] = {"error": str(e)}
        p3 = I.film3d_params(256)
        f3 = I.film3d_fields(p3, seed=1, h0=32.0, amp=3.0)
        record("film3d_256^3_f32", p3, f3, "f32", 33, 20, 3)
        for name in ("trt", "biased2"):
            record(f"film3d_256^3_f32_{name}", dict(p3, **ext_opts[name]), f3, "f32", 33, 20, 3)
        p5 = I.film3d_params(512)
        f5 = I.film3d_fields(p5, seed=5, h0=64.0, amp=6.0)
        for st in ("f32", "f16dev", "bf16dev"):
            record(f"film3d_512^3_{st}", p5, f5, st, 33, 10, 2)
        del f5
        torch.cuda.empty_cache()
        out["variants"] = var
    if args.copy_calib:
        # 512 MiB device copy (16-byte accesses), then a scaled copy of a float
        # view offset by one element, which cannot be vectorised (4-byte
        # accesses per lane, like the populations in the step kernels)
        x = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        xf, yf = x.view(torch.float32), y.view(torch.float32)
        xf.fill_(1.0)
        for _ in range(3):
            torch.mul(xf[1:], 2.0, out=yf[1:])
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = x.numel()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prm, fields)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
