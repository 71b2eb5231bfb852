"""Python binding of the C ABI in include/lbm.h (ctypes; marshalling only).

Every step of the method runs in the HIP library ``liblbm.so``; this module
only builds the parameter struct, hands device pointers of torch tensors to
the library and wraps status codes in exceptions.  Importing it fails
loudly if the library has not been built (``python -m
paper_2003_06342_amd.build`` or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_HIP, LBM_E_STATE, LBM_E_UNSTABLE, LBM_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
LBM_D2Q9, LBM_D2Q5, LBM_D3Q7, LBM_D3Q19 = 9, 5, 7, 19
ST = {"f64": 0, "f32": 1, "f16dev": 2, "bf16dev": 3}
LBM_BC_PERIODIC, LBM_BC_WALL = 0, 1
LBM_NS, LBM_HEAT, LBM_PHASE_CHANGE, LBM_VISC_LINEAR, LBM_GEQ_CAC, LBM_DIV_LOCAL = \
    1, 2, 4, 8, 16, 32
COLL = {"bgk": 0, "trt": 1, "mrt": 2}
GRAD = {"central": 0, "biased1": 1, "biased2": 2}
LBM_TAPE_SQRT, LBM_TAPE_BINOMIAL = 0, 1
LBM_DT_F32, LBM_DT_F64 = 0, 1
LBM_FBC_NOSLIP, LBM_FBC_PRESSURE = 0, 1
LBM_STATIC_SCRATCH_BYTES = 128 << 20   # include/lbm.h
FIELDS = ["phi", "p", "ux", "uy", "uz", "T"]          # bit order of LBM_FIELD_*
LAT = {"D2Q9": LBM_D2Q9, "D2Q5": LBM_D2Q5, "D3Q7": LBM_D3Q7, "D3Q19": LBM_D3Q19}


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


class lbm_params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("lat_f", C.c_int32), ("lat_g", C.c_int32), ("lat_s", C.c_int32),
        ("storage", C.c_int32), ("flags", C.c_uint32),
        ("nu_l", C.c_double), ("nu_g", C.c_double), ("mobility", C.c_double),
        ("alpha_l", C.c_double), ("alpha_g", C.c_double),
        ("W", C.c_double), ("sigma", C.c_double), ("rho_l", C.c_double), ("rho_g", C.c_double),
        ("L_over_cp", C.c_double), ("T_sat", C.c_double), ("theta_I", C.c_double),
        ("A_coef", C.c_double),
        ("gravity", C.c_double * 3), ("body_force", C.c_double * 3),
        ("bc", C.c_int32 * 3),
        ("phi_wall", (C.c_double * 2) * 3), ("T_wall", (C.c_double * 2) * 3),
        ("eps_n", C.c_double),
        ("collision", C.c_int32),
        ("trt_lambda", C.c_double * 3),
        ("mrt_rates", (C.c_double * 4) * 3),
        ("grad_scheme", C.c_int32),
        ("check_every", C.c_int32),
        ("f_bc", (C.c_int32 * 2) * 3),
        ("p_wall", (C.c_double * 2) * 3),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbm.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built; run __graft_entry__.build() first")
    # torch ships its own HIP runtime; importing it first makes the library
    # bind to that same runtime (whose memory and streams it is given)
    # instead of loading a second one, which then sees no device
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, I32, I64, SZ, U32, D = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_uint32, C.c_double
    sig = {
        "lbm_workspace_size": (I32, [C.POINTER(lbm_params), C.POINTER(SZ)]),
        "lbm_create": (I32, [C.POINTER(lbm_params), P, SZ, P, C.POINTER(P)]),
        "lbm_init_fields": (I32, [P, P, P, P, P, I32]),
        "lbm_set_wall_T": (I32, [P, I32, I32, P, I32]),
        "lbm_step": (I32, [P, I64]),
        "lbm_get_fields": (I32, [P, U32, P, I32]),
        "lbm_diagnostics": (I32, [P, C.POINTER(D)]),
        "lbm_state_size": (I32, [P, C.POINTER(SZ)]),
        "lbm_get_state": (I32, [P, P, SZ]),
        "lbm_set_state": (I32, [P, P, SZ]),
        "lbm_get_step": (I32, [P, C.POINTER(I64)]),
        "lbm_sync": (I32, [P]),
        "lbm_tape_size": (I32, [P, I64, I32, C.POINTER(SZ)]),
        "lbm_forward_taped": (I32, [P, I64, I32, P, SZ]),
        "lbm_adjoint_workspace_size": (I32, [P, C.POINTER(SZ)]),
        "lbm_backward": (I32, [P, P, P, P, P, I32, P, SZ, P, P, P, I32, I32, I32]),
        "lbm_backward_static": (I32, [P, P, P, P, P, I32, P, P, P, I32, I32, I32]),
        "lbm_destroy": (None, [P]),
        "lbm_last_error": (C.c_char_p, []),
        "lbm_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != LBM_OK:
        raise LBMError(status, _lib.lbm_last_error().decode())


def make_params(prm: dict, storage: str) -> lbm_params:
    """Marshal a workload parameter dict into the C struct."""
    p = lbm_params()
    p.dim, p.nx, p.ny, p.nz = prm["dim"], prm["nx"], prm["ny"], prm["nz"]
    p.lat_f, p.lat_g, p.lat_s = LAT[prm["lat_f"]], LAT[prm["lat_g"]], LAT[prm["lat_s"]]
    p.storage = ST[storage]
    flags = 0
    flags |= LBM_NS if prm["ns"] else 0
    flags |= LBM_HEAT if prm["heat"] else 0
    flags |= LBM_PHASE_CHANGE if (prm["phase_change"] and prm["heat"]) else 0
    flags |= LBM_VISC_LINEAR if prm["visc_linear"] else 0
    flags |= LBM_GEQ_CAC if prm["geq_cac"] else 0
    flags |= LBM_DIV_LOCAL if prm.get("div_local", False) else 0
    p.flags = flags
    p.collision = COLL[prm.get("collision", "bgk")]
    lam = prm.get("trt_lambda", (0.25, 0.25, 0.25))
    rates = prm.get("mrt_rates", ((1.0,) * 4,) * 3)
    for k in range(3):
        p.trt_lambda[k] = float(lam[k])
        for r in range(4):
            p.mrt_rates[k][r] = float(rates[k][r])
    p.grad_scheme = GRAD[prm.get("grad_scheme", "central")]
    p.check_every = int(prm.get("check_every", 0))
    f_open = prm.get("f_open", [[False, False]] * 3)
    p_wall = prm.get("p_wall", [[0.0, 0.0]] * 3)
    for a in range(3):
        for s in range(2):
            p.f_bc[a][s] = LBM_FBC_PRESSURE if f_open[a][s] else LBM_FBC_NOSLIP
            p.p_wall[a][s] = float(p_wall[a][s])
    for k in ("nu_l", "nu_g", "mobility", "alpha_l", "alpha_g", "W", "sigma", "rho_l", "rho_g",
              "L_over_cp", "T_sat", "theta_I", "A_coef", "eps_n"):
        setattr(p, k, float(prm[k]))
    for a in range(3):
        p.gravity[a] = float(prm["gravity"][a])
        p.body_force[a] = float(prm.get("body_force", [0, 0, 0])[a])
        p.bc[a] = LBM_BC_WALL if prm["bc"][a] == "wall" else LBM_BC_PERIODIC
        for s in range(2):
            p.phi_wall[a][s] = float(prm["phi_wall"][a][s])
            p.T_wall[a][s] = float(prm["T_wall"][a][s])
    return p


def workspace_size(prm: dict, storage: str) -> int:
    lib = load_library()
    p = make_params(prm, storage)
    n = C.c_size_t()
    _check(lib.lbm_workspace_size(C.byref(p), C.byref(n)))
    return n.value


class Sim:
    """One simulation context on a HIP device; memory comes from torch."""

    def __init__(self, prm: dict, storage: str = "f32", device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.prm = prm
        self.storage = storage
        self.device = torch.device(device)
        self.shape = (prm["nz"], prm["ny"], prm["nx"])
        self._p = make_params(prm, storage)
        n = C.c_size_t()
        _check(self.lib.lbm_workspace_size(C.byref(self._p), C.byref(n)))
        # 256 extra bytes so the workspace can be aligned to 256
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        _check(self.lib.lbm_create(C.byref(self._p), C.c_void_p(aligned), C.c_size_t(n.value),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------
    def _dev(self, arr, dtype=None):
        torch = self.torch
        if arr is None:
            return None
        t = torch.as_tensor(arr)
        if dtype is None:
            dtype = torch.float64 if t.dtype == torch.float64 else torch.float32
        return t.to(device=self.device, dtype=dtype).contiguous()

    @staticmethod
    def _ptr(t):
        return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)

    # -- API ---------------------------------------------------------------
    def init(self, phi0, T0=None, u0=None, p0=None, dtype="f64"):
        torch = self.torch
        dt = torch.float64 if dtype == "f64" else torch.float32
        phi = self._dev(np.asarray(phi0).reshape(self.shape) if not isinstance(phi0, torch.Tensor)
                        else phi0.reshape(self.shape), dt)
        T = None
        if T0 is not None:
            T = self._dev(T0 if isinstance(T0, torch.Tensor) else np.asarray(T0), dt).reshape(self.shape)
        elif self.prm["heat"]:
            T = torch.zeros(self.shape, dtype=dt, device=self.device)
        u = None
        if u0 is not None:
            u = torch.stack([self._dev(np.asarray(c) if not isinstance(c, torch.Tensor) else c, dt)
                             .reshape(self.shape) for c in u0]).contiguous()
        p = None if p0 is None else self._dev(p0, dt).reshape(self.shape).contiguous()
        self._keep = (phi, T, u, p)
        _check(self.lib.lbm_init_fields(self.ctx, self._ptr(phi), self._ptr(T), self._ptr(u),
                                        self._ptr(p), LBM_DT_F64 if dtype == "f64" else LBM_DT_F32))
        return self

    def set_wall_T(self, axis: int, side: int, face):
        t = self._dev(face, self.torch.float64).contiguous()
        self._keep_face = t
        _check(self.lib.lbm_set_wall_T(self.ctx, axis, side, self._ptr(t), LBM_DT_F64))

    def step(self, n: int = 1):
        _check(self.lib.lbm_step(self.ctx, int(n)))
        return self

    def fields(self, names=("phi", "p", "ux", "uy", "uz", "T"), dtype="f64") -> dict:
        torch = self.torch
        mask = 0
        for k in names:
            mask |= 1 << FIELDS.index(k)
        sel = [k for k in FIELDS if mask & (1 << FIELDS.index(k))]
        dt = torch.float64 if dtype == "f64" else torch.float32
        out = torch.empty((len(sel),) + self.shape, dtype=dt, device=self.device)
        _check(self.lib.lbm_get_fields(self.ctx, mask, self._ptr(out),
                                       LBM_DT_F64 if dtype == "f64" else LBM_DT_F32))
        return {k: out[i] for i, k in enumerate(sel)}

    def diagnostics(self, check: bool = True) -> dict:
        buf = (C.c_double * 5)()
        st = self.lib.lbm_diagnostics(self.ctx, buf)
        if check:
            _check(st)
        return dict(mass=buf[0], enthalpy=buf[1], vapour=buf[2], umax=buf[3], nonfinite=buf[4],
                    status=st)

    def state_size(self) -> int:
        n = C.c_size_t()
        _check(self.lib.lbm_state_size(self.ctx, C.byref(n)))
        return n.value

    def get_state(self):
        n = self.state_size()
        t = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        _check(self.lib.lbm_get_state(self.ctx, self._ptr(t), n))
        return t

    def set_state(self, t):
        _check(self.lib.lbm_set_state(self.ctx, self._ptr(t), t.numel()))

    def sync(self):
        _check(self.lib.lbm_sync(self.ctx))

    # -- adjoint -----------------------------------------------------------
    @staticmethod
    def _aligned(n: int, device):
        import torch
        t = torch.empty(n + 256, dtype=torch.uint8, device=device)
        off = (-t.data_ptr()) % 256
        return t, t.data_ptr() + off

    def forward_taped(self, nsteps: int, policy: int = LBM_TAPE_SQRT):
        """Advance nsteps from a fresh init recording the tape for backward()."""
        n = C.c_size_t()
        _check(self.lib.lbm_tape_size(self.ctx, int(nsteps), int(policy), C.byref(n)))
        self._tape, ptr = self._aligned(n.value, self.device)
        _check(self.lib.lbm_forward_taped(self.ctx, int(nsteps), int(policy), C.c_void_p(ptr), n))
        return self

    def backward(self, gphi=None, tw_face=(1, 0), gT=None) -> dict:
        """Gradients of a loss with dL/dphi^N = gphi and dL/dT^N = gT (arrays
        [ny][nx], each optional) with respect to phi0, T0 and the
        wall-temperature face tw_face."""
        torch = self.torch
        shp = self.shape[1:]
        g = None if gphi is None else self._dev(gphi, torch.float64).reshape(shp).contiguous()
        gt = None if gT is None else self._dev(gT, torch.float64).reshape(shp).contiguous()
        n = C.c_size_t()
        _check(self.lib.lbm_adjoint_workspace_size(self.ctx, C.byref(n)))
        ws, ptr = self._aligned(n.value, self.device)
        nx, ny = self.prm["nx"], self.prm["ny"]
        dphi = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        dT0 = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        face_len = nx if tw_face[0] == 1 else ny
        dTw = torch.empty(face_len, dtype=torch.float64, device=self.device)
        none = C.c_void_p(None)
        _check(self.lib.lbm_backward(self.ctx, self._ptr(g), self._ptr(gt), none, none, LBM_DT_F64,
                                     C.c_void_p(ptr), n, self._ptr(dphi), self._ptr(dT0),
                                     self._ptr(dTw), int(tw_face[0]), int(tw_face[1]), LBM_DT_F64))
        self._keep_ws = ws
        return dict(phi0=dphi, T0=dT0, Tw=dTw)

    def backward_static(self, gphi=None, tw_face=(1, 0), gT=None) -> dict:
        """backward() through lbm_backward_static: no workspace argument (the
        library's static device scratch); same seeds and outputs."""
        torch = self.torch
        shp = self.shape[1:]
        g = None if gphi is None else self._dev(gphi, torch.float64).reshape(shp).contiguous()
        gt = None if gT is None else self._dev(gT, torch.float64).reshape(shp).contiguous()
        nx, ny = self.prm["nx"], self.prm["ny"]
        dphi = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        dT0 = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        face_len = nx if tw_face[0] == 1 else ny
        dTw = torch.empty(face_len, dtype=torch.float64, device=self.device)
        none = C.c_void_p(None)
        _check(self.lib.lbm_backward_static(self.ctx, self._ptr(g), self._ptr(gt), none, none,
                                            LBM_DT_F64, self._ptr(dphi), self._ptr(dT0),
                                            self._ptr(dTw), int(tw_face[0]), int(tw_face[1]),
                                            LBM_DT_F64))
        self._keep_seeds = (g, gt)
        return dict(phi0=dphi, T0=dT0, Tw=dTw)

    @property
    def steps_taken(self) -> int:
        v = C.c_int64()
        _check(self.lib.lbm_get_step(self.ctx, C.byref(v)))
        return v.value
