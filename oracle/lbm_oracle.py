"""Plain FP64 reference of the phase-change lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written with PyTorch
CPU ops in float64 so that ``torch.autograd`` provides an independent
reverse pass.  No blocking, fusion or reordering: each function is one step
of the scheme in the paper's order and notation.

Paper: Verdier, Kestener, Cartalade, "Performance portability of lattice
Boltzmann methods for two-phase flows with phase change" (arXiv 2003.06342).

Model (Sec. 2): conservative Allen-Cahn phase field phi (phi = 1 gas,
phi = 0 liquid) with production m''' (Eqs. CAC_ChgtPhase, ProductionRate),
incompressible Navier-Stokes with surface tension mu grad(phi) and buoyancy
(Eqs. ConservMasse_ChgtPhase, ConvservQDM_ChgtPhase, Force_Total,
SuperficialTensionForce, ChemicalPotential) and the heat equation with the
latent-heat source (Eq. Temperature_ChgtPhase).

Scheme (Sec. 3): three BGK populations f (NS), g (phi), s (T) in barred
variables (Eqs. VariableChange_f, VariableChange_feq, LBE), equilibria
Feq_NS_Incompr, Geq_Allen-Cahn_Eq, Seq_Temp with Gamma_i (Eq.
FunctionGamma), sources Forcing, MicroProduction, SourceTerm_AllenCahn,
Def_SourceTerms_Temp, moments Velocity, Pressure, Moment_Phi, Moment_Temp,
directional-derivative gradient and Laplacian (Eqs. DerivDirec_Grad, Grad,
DerivDirect_Laplacian, Laplacian), anti-bounce-back Dirichlet walls (Sec.
3.3) and half-way bounce-back no-slip walls (Sec. 4.1.2, Poiseuille).

Readings where the paper is silent or inconsistent (the GPU path takes the
same ones):
  R1  D2Q9 weights 4/9, 1/9, 1/36 (not printed); D3Q7 order +x,+y,+z,-x,-y,-z.
  R2  every "3" of Eqs. Grad / Laplacian is 1/c_s^2 of the stencil lattice;
      each population uses its own lattice's c_s^2 (1/3 D2Q9, D3Q19; 1/4
      D3Q7, D2Q5).
  R3  stencils use D2Q9 in 2-D and D3Q19 in 3-D whatever the g/s lattice.
  R4  heat source S^s_i = -w_i (L/Cp) [d_t phi + div(u phi)] (sign fixed by
      Eqs. Heat-Equation_dimensionless and Moment_Temp).
  R5  buoyancy F_v = (rho(phi) - rho_l) g with g the gravity acceleration
      vector (points down): upward on vapour, zero in liquid.
  R6  the production term in Eq. Moment_Phi is lagged by one step (q_prev).
  R7  d_t phi = phi^n - phi^{n-1} (0 at the first step).
  R8  div(u phi) = sum_a of the a-th component of the Eq. Grad stencil applied
      to u_a phi.
  R8b with div_local: u.grad(phi) + phi div(u), div(u) from Eq.
      ConservMasse_ChgtPhase with the previous step's production.
  R9  n = grad(phi) / sqrt(|grad(phi)|^2 + eps^2), eps = 1e-3: far below
      interface gradients (~1/W), far above round-off gradients in the bulk
      phases, where a smaller eps turns round-off into O(phi(1-phi)) forcing.
  R10 alpha(phi) = (1 - phi) alpha_l + phi alpha_g, used for tau_s and in q.
  R12 init: populations = equilibrium - S/2 at the initial fields with
      d_t phi = 0 and div(u phi) from u0, so the moments return the inputs.
  R13 half-way walls between node rows; stencil ghosts phi_g = 2 phi_w - phi_b
      and u_g = -u_b; at an edge crossed by two walls the wall of the higher
      axis (z over y over x) gives the anti-bounce-back value.
  R17 the u of the current step enters Gamma_i of all three families.
  R18 the pressure moment uses the current step's q.
  R26 TRT and MRT (named in Sec. 3 after Eq. LBE as the way to lower
      mobility and higher Peclet numbers; not written out in the paper) act
      on the same barred variables as BGK: the non-equilibrium plus half the
      source, a_i = pop_i - eq_i + S_i/2, relaxes and S_i is added, so equal
      rates give BGK exactly.  TRT (Ginzburg) relaxes the parts of a
      symmetric and antisymmetric under c -> -c with omega+ and omega-; the
      transport coefficient keeps its BGK rate (omega+ for the viscosity of
      f, omega- for the mobility of g and the diffusivity of s) and the other
      rate follows from Lambda = (1/omega+ - 1/2)(1/omega- - 1/2).  MRT
      (d'Humieres) relaxes a in an orthogonal moment basis: D2Q9 rho, e, eps,
      jx, qx, jy, qy, pxx, pxy (Lallemand and Luo); D3Q7 1, cx, cy, cz,
      7c^2 - 6, 2cx^2 - cy^2 - cz^2, cy^2 - cz^2.  Transport moments at the
      BGK rate (pxx, pxy for f; j for g and s), the others at the free rates
      (s_e for rho and e, s_eps, s_q for q (and j of f), s_p for the
      second-order moments of g and s).
  R29 an open face of f (flag per face): the pressure anti-bounce-back
      f_i = -f*_{i'} + 2 w_i p_w, the even part of Eq. Feq_NS_Incompr at the
      face pressure with its O(u^2) terms dropped (Ginzburg's rule for a
      Dirichlet condition on the zeroth moment), and a stencil ghost
      u_g = u_b (zero normal gradient) instead of the no-slip -u_b.  g and s
      keep their Dirichlet anti-bounce-back.  Lets net evaporation leave a
      closed box, whose gauge pressure otherwise drifts.
  R27 biased directional derivatives (Sec. 3.4, after Eq. Laplacian: the
      first- and second-order upwind differences phi(x + c) - phi(x) and
      [-phi(x + 2c) + 4 phi(x + c) - 3 phi(x)] / 2, offered there as
      alternatives to the central Eq. DerivDirec_Grad for low-density
      regions, where the central form misses the velocity profile) replace
      c_i . grad(phi) where the NS source projects it on its own direction
      c_i: c_i . grad(rho) and the surface tension mu c_i . grad(phi) of Eq.
      Forcing.  Every vector use of grad(phi) (u . grad(rho), u . F, the
      velocity and pressure moments, the normal n) and the Laplacian keep
      the central stencils, and so does c_i . n of Eq. SourceTerm_AllenCahn:
      its zeroth moment must vanish for phi to stay conserved, which a
      biased difference would break (sum_i w_i [phi(x + c_i) - phi(x)] is a
      Laplacian).  Ghosts two nodes beyond a wall mirror the second node
      (R13).
Pinned readings beyond the closed forms: R8 (the Fourier symbol of the
central stencil on u_a phi, and second-order convergence of the wall rows),
R9 (linear ramps and the planar interface), R10 (steady series conduction
across a static interface), R7 (the enthalpy invariant, which a lag that is
not advanced breaks), R6 (the exact discrete mass balance of the lagged
production) and R13 (manufactured ghosts, hand-computed edges).  Parity
unpinned beyond self-consistency and invariants: chaotic trajectories after
pinch-off.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import torch

F64 = torch.float64


# ---------------------------------------------------------------------------
# Lattices (Sec. 3, lattice definitions; weights of D2Q9 and D2Q5: R1)
# ---------------------------------------------------------------------------

@dataclass
class Lattice:
    name: str
    c: list          # Q tuples (cx, cy, cz)
    w: list          # Q weights
    cs2: float       # lattice speed of sound squared
    opp: list        # index of -c_i

    @property
    def Q(self) -> int:
        return len(self.w)


def _make(name, c, w, cs2):
    opp = [c.index(tuple(-v for v in ci)) for ci in c]
    return Lattice(name, [tuple(ci) for ci in c], list(w), cs2, opp)


def lattice(name: str) -> Lattice:
    if name == "D2Q9":
        c = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
             (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
        w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
        return _make(name, c, w, 1 / 3)
    if name == "D2Q5":   # z-projection of D3Q7 (used by the z-invariance pin)
        c = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0)]
        w = [1 / 2] + [1 / 8] * 4
        return _make(name, c, w, 1 / 4)
    if name == "D3Q7":
        c = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
             (-1, 0, 0), (0, -1, 0), (0, 0, -1)]
        w = [1 / 4] + [1 / 8] * 6
        return _make(name, c, w, 1 / 4)
    if name == "D3Q19":
        c = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
             (-1, 0, 0), (0, -1, 0), (0, 0, -1),
             (1, 1, 0), (-1, 1, 0), (1, -1, 0), (-1, -1, 0),
             (1, 0, 1), (-1, 0, 1), (1, 0, -1), (-1, 0, -1),
             (0, 1, 1), (0, -1, 1), (0, 1, -1), (0, -1, -1)]
        w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
        return _make(name, c, w, 1 / 3)
    raise ValueError(name)


# ---------------------------------------------------------------------------
# State and intermediate fields
# ---------------------------------------------------------------------------

@dataclass
class State:
    """Post-streaming barred populations at time n plus the lagged scalars.

    f: [Qf, nz, ny, nx] or None (NS off); g: [Qg, ...]; s: [Qs, ...] or None
    (heat off); phi_prev = phi^{n-1} (R7); q_prev = q^{n-1} (R6)."""
    f: Optional[torch.Tensor]
    g: torch.Tensor
    s: Optional[torch.Tensor]
    phi_prev: torch.Tensor
    q_prev: torch.Tensor


@dataclass
class Macros:
    phi: torch.Tensor
    grad_phi: list
    lap_phi: torch.Tensor
    n: list
    mu: torch.Tensor
    rho: torch.Tensor
    grad_rho: list
    F: list
    u: list
    dtphi: torch.Tensor
    D: torch.Tensor
    T: torch.Tensor
    q: torch.Tensor
    p: torch.Tensor
    alpha: torch.Tensor
    nu: torch.Tensor
    phi_pad2: Optional[torch.Tensor] = None   # phi with two ghost layers (R27)


def _tensor_axis(a: int) -> int:
    """Lattice axis a (0=x, 1=y, 2=z) -> dim of a [nz, ny, nx] tensor."""
    return 2 - a


class Model:
    """Parameters plus the step of the scheme (all lattice units, dx = dt = 1).

    ``prm`` is the plain parameter dict built by the workload module.
    ``T_wall_faces`` optionally replaces the scalar wall temperature of a
    face by a per-node face array: key (axis, side) -> tensor broadcastable
    to [nz, ny, nx] (size 1 along ``axis``).

    ``dtype`` is float64 for the oracle proper.  float32 evaluates the same
    arithmetic in single precision; it is used only to measure the rounding
    floor that any FP32 implementation of the scheme has on a given case."""

    def __init__(self, prm: dict, T_wall_faces: Optional[dict] = None, dtype=F64):
        self.prm = prm
        self.dt = dtype
        self.dim = int(prm["dim"])
        self.shape = (int(prm["nz"]), int(prm["ny"]), int(prm["nx"]))
        self.ns = bool(prm["ns"])
        self.heat = bool(prm["heat"])
        self.phase_change = bool(prm["phase_change"]) and self.heat
        self.visc_linear = bool(prm["visc_linear"])
        self.geq_cac = bool(prm["geq_cac"])
        self.Lf = lattice(prm["lat_f"])
        self.Lg = lattice(prm["lat_g"])
        self.Ls = lattice(prm["lat_s"])
        self.Lst = lattice("D2Q9" if self.dim == 2 else "D3Q19")   # R3
        for key, v in (("nu_l", prm["nu_l"]), ("nu_g", prm["nu_g"]),
                       ("mobility", prm["mobility"]), ("alpha_l", prm["alpha_l"]),
                       ("alpha_g", prm["alpha_g"])):
            if not v > 0:
                raise ValueError(f"{key} must be > 0")
        self.W = float(prm["W"])
        self.sigma = float(prm["sigma"])
        self.rho_l = float(prm["rho_l"])
        self.rho_g = float(prm["rho_g"])
        self.Lcp = float(prm["L_over_cp"])
        self.T_sat = float(prm["T_sat"])
        self.theta_I = float(prm["theta_I"])
        self.A = float(prm["A_coef"])
        self.M = float(prm["mobility"])
        self.grav = [float(v) for v in prm["gravity"]]
        self.body = [float(v) for v in prm.get("body_force", (0.0, 0.0, 0.0))]
        self.eps = float(prm.get("eps_n", 1e-3))
        self.div_local = bool(prm.get("div_local", False))
        if self.div_local and not (self.ns and self.heat):
            raise ValueError("div_local needs the NS and heat families")
        self.grad_scheme = prm.get("grad_scheme", "central")
        if self.grad_scheme not in ("central", "biased1", "biased2"):
            raise ValueError(self.grad_scheme)
        self.collision = prm.get("collision", "bgk")
        if self.collision not in ("bgk", "trt", "mrt"):
            raise ValueError(self.collision)
        self.trt_lambda = [float(v) if v > 0 else 0.25
                           for v in prm.get("trt_lambda", (0.25, 0.25, 0.25))]
        self.mrt_rates = [[float(r) for r in fam]
                          for fam in prm.get("mrt_rates", ((1.0,) * 4,) * 3)]
        # Eq. Def_K-H
        self.K = 1.5 * self.W * self.sigma
        self.H = 12.0 * self.sigma / self.W
        self.wall = [prm["bc"][a] == "wall" for a in range(3)]
        self.phi_w = [[float(prm["phi_wall"][a][s]) for s in range(2)] for a in range(3)]
        # open faces of f (R29): pressure anti-bounce-back instead of no-slip
        fo = prm.get("f_open", [[False, False]] * 3)
        pw = prm.get("p_wall", [[0.0, 0.0]] * 3)
        self.f_open = [[bool(fo[a][s]) and self.wall[a] for s in range(2)] for a in range(3)]
        self.p_w = [[float(pw[a][s]) for s in range(2)] for a in range(3)]
        self.T_w = [[torch.tensor(float(prm["T_wall"][a][s]), dtype=self.dt)
                     for s in range(2)] for a in range(3)]
        if T_wall_faces:
            for (a, s), arr in T_wall_faces.items():
                self.T_w[a][s] = torch.as_tensor(arr, dtype=self.dt)

    # -- closures (Sec. 2) --------------------------------------------------

    def density(self, phi):
        """Eq. Density."""
        return phi * self.rho_g + (1.0 - phi) * self.rho_l

    def viscosity(self, phi):
        """Eq. Viscosity (harmonic) or Eq. Visco_lin."""
        nl, ng = self.prm["nu_l"], self.prm["nu_g"]
        if self.visc_linear:
            return (1.0 - phi) * nl + phi * ng
        return nl * ng / (phi * nl + (1.0 - phi) * ng)

    def diffusivity(self, phi):
        """Thermal diffusivity interpolation (R10)."""
        return (1.0 - phi) * self.prm["alpha_l"] + phi * self.prm["alpha_g"]

    # -- ghosts and stencils (Sec. 3.4) ---------------------------------------

    def ghost_pad(self, v, kind: str):
        """Pad a [nz, ny, nx] field by one ghost layer on every axis.

        Periodic axes wrap; wall axes use the half-way mirror (R13):
        'phi' -> 2 phi_w - v_b, 'anti' -> -v_b (no-slip velocity)."""
        out = v
        for a in range(3):
            d = _tensor_axis(a)
            n = out.shape[d]
            first = out.narrow(d, 0, 1)
            last = out.narrow(d, n - 1, 1)
            if not self.wall[a]:
                lo, hi = last, first
            elif kind == "phi":
                lo = 2.0 * self.phi_w[a][0] - first
                hi = 2.0 * self.phi_w[a][1] - last
            elif kind == "anti":
                # no-slip: u_g = -u_b; an open face (R29): u_g = u_b
                lo = first if self.f_open[a][0] else -first
                hi = last if self.f_open[a][1] else -last
            else:
                raise ValueError(kind)
            out = torch.cat([lo, out, hi], dim=d)
        return out

    def ghost_pad_wide(self, v, kind: str, width: int):
        """ghost_pad with `width` ghost layers: periodic axes wrap; the
        ghost k nodes beyond a wall mirrors the k-th node from it (R13)."""
        out = v
        for a in range(3):
            d = _tensor_axis(a)
            n = out.shape[d]
            idx = torch.arange(width)
            if not self.wall[a]:
                lo = out.index_select(d, (n - width + idx) % n)
                hi = out.index_select(d, idx % n)
            else:
                lo = out.index_select(d, torch.flip(idx, [0]))       # ghost -k <- node k-1
                hi = out.index_select(d, n - 1 - idx)                # ghost n-1+k <- node n-k
                if kind == "phi":
                    lo = 2.0 * self.phi_w[a][0] - lo
                    hi = 2.0 * self.phi_w[a][1] - hi
                else:
                    raise ValueError(kind)
            out = torch.cat([lo, out, hi], dim=d)
        return out

    def cproj(self, m, c):
        """c . grad(phi) for a lattice velocity c under the directional-
        derivative scheme (R27): the projection of the Eq. Grad vector
        (central), or the first- / second-order biased difference along c."""
        if all(x == 0 for x in c):
            return torch.zeros(self.shape, dtype=self.dt)
        if self.grad_scheme == "central":
            return sum(c[a] * m.grad_phi[a] for a in range(3) if c[a] != 0)
        nz, ny, nx = self.shape

        def at(k):   # phi(x + k c) from the two-layer padded field
            return m.phi_pad2[2 + k * c[2]:2 + k * c[2] + nz, 2 + k * c[1]:2 + k * c[1] + ny,
                              2 + k * c[0]:2 + k * c[0] + nx]
        if self.grad_scheme == "biased1":
            return at(1) - at(0)
        return 0.5 * (-at(2) + 4.0 * at(1) - 3.0 * at(0))

    def _shift(self, padded, e):
        """padded value at x + e for every interior node x."""
        nz, ny, nx = self.shape
        ex, ey, ez = e
        return padded[1 + ez:1 + ez + nz, 1 + ey:1 + ey + ny, 1 + ex:1 + ex + nx]

    def grad(self, padded):
        """Eqs. DerivDirec_Grad and Grad: (1/c_s^2) sum_i w_i e_i [v(x+e_i) -
        v(x-e_i)] / 2 over the stencil lattice (R2, R3)."""
        L = self.Lst
        out = [torch.zeros(self.shape, dtype=self.dt) for _ in range(3)]
        for i in range(1, L.Q):
            e = L.c[i]
            dd = 0.5 * (self._shift(padded, e) - self._shift(padded, tuple(-x for x in e)))
            for a in range(3):
                if e[a] != 0:
                    out[a] = out[a] + L.w[i] * e[a] * dd
        return [o / L.cs2 for o in out]

    def laplacian(self, padded, centre):
        """Eqs. DerivDirect_Laplacian and Laplacian."""
        L = self.Lst
        out = torch.zeros(self.shape, dtype=self.dt)
        for i in range(1, L.Q):
            e = L.c[i]
            out = out + L.w[i] * (self._shift(padded, e) - 2.0 * centre
                                  + self._shift(padded, tuple(-x for x in e)))
        return out / L.cs2

    # -- moments and closures at the current populations (S1-S7) -------------

    def forces(self, phi, grad_phi, lap_phi):
        """Chemical potential (Eq. ChemicalPotential with Eq. Def_K-H), surface
        tension mu grad(phi) (Eq. SuperficialTensionForce) and buoyancy (R5);
        F_tot = F_s + F_v (Eq. Force_Total) plus an optional uniform body
        force (the pressure-gradient surrogate of the Poiseuille case)."""
        mu = 4.0 * self.H * phi * (phi - 1.0) * (phi - 0.5) - self.K * lap_phi
        rho = self.density(phi)
        F = [mu * grad_phi[a] + (rho - self.rho_l) * self.grav[a] + self.body[a]
             for a in range(3)]
        return mu, rho, F

    def divergence(self, u, phi_padded):
        """div(u phi) with the central directional-derivative stencil (R8)."""
        D = torch.zeros(self.shape, dtype=self.dt)
        for a in range(3):
            prod = self.ghost_pad(u[a], "anti") * phi_padded
            D = D + self.grad(prod)[a]
        return D

    def divergence_term(self, u, phi_padded, grad_phi, phi, q_prev):
        """The div(u phi) of the latent-heat source: R8 (central stencil), or
        with ``div_local`` (R8b) u.grad(phi) + phi div(u), where div(u) =
        mdot (1/rho_g - 1/rho_l) (Eq. ConservMasse_ChgtPhase) with the
        production of the previous step, mdot = rho_g q_prev (as R6)."""
        if not self.div_local:
            return self.divergence(u, phi_padded)
        udg = sum(u[a] * grad_phi[a] for a in range(3))
        return udg + phi * self.rho_g * q_prev * (1.0 / self.rho_g - 1.0 / self.rho_l)

    def production(self, phi, T, alpha):
        """q = m'''/rho_g of Eq. ProductionRate with theta = (Cp/L)(T - T_sat)."""
        if not self.phase_change:
            return torch.zeros_like(phi)
        theta = (T - self.T_sat) / self.Lcp
        return -(4.0 * alpha / (self.A * self.W * self.W)) * (self.theta_I - theta) \
            * phi * (1.0 - phi)

    def macros(self, st: State, u_prescribed=None) -> Macros:
        # S1: Eq. Moment_Phi, production lagged (R6)
        phi = st.g.sum(0) + 0.5 * st.q_prev
        # S2: stencils and closures
        P = self.ghost_pad(phi, "phi")
        gphi = self.grad(P)
        lphi = self.laplacian(P, phi)
        norm = torch.sqrt(gphi[0] ** 2 + gphi[1] ** 2 + gphi[2] ** 2 + self.eps ** 2)
        n = [gphi[a] / norm for a in range(3)]
        mu, rho, F = self.forces(phi, gphi, lphi)
        grho = [(self.rho_g - self.rho_l) * gphi[a] for a in range(3)]
        # S3: Eq. Velocity
        if self.ns:
            Lf = self.Lf
            u = []
            for a in range(3):
                m1 = sum(st.f[i] * Lf.c[i][a] for i in range(Lf.Q) if Lf.c[i][a] != 0)
                if isinstance(m1, int):
                    m1 = torch.zeros(self.shape, dtype=self.dt)
                u.append((m1 / Lf.cs2 + 0.5 * F[a]) / rho)
        elif u_prescribed is not None:
            u = [torch.as_tensor(u_prescribed[a], dtype=self.dt) * torch.ones(self.shape, dtype=self.dt)
                 for a in range(3)]
        else:
            u = [torch.zeros(self.shape, dtype=self.dt) for _ in range(3)]
        # S4: time derivative (R7) and divergence (R8)
        dtphi = phi - st.phi_prev
        alpha = self.diffusivity(phi)
        if self.heat:
            D = self.divergence_term(u, P, gphi, phi, st.q_prev)
            # S5: Eq. Moment_Temp
            T = st.s.sum(0) - 0.5 * self.Lcp * (dtphi + D)
        else:
            D = torch.zeros(self.shape, dtype=self.dt)
            T = torch.zeros(self.shape, dtype=self.dt)
        # S6: Eq. ProductionRate
        q = self.production(phi, T, alpha)
        # S7: Eq. Pressure (R18)
        if self.ns:
            cs2 = self.Lf.cs2
            mdot = self.rho_g * q
            udr = sum(u[a] * grho[a] for a in range(3))
            p = st.f.sum(0) + 0.5 * (cs2 * udr + rho * cs2 * mdot
                                     * (1.0 / self.rho_g - 1.0 / self.rho_l))
        else:
            p = torch.zeros(self.shape, dtype=self.dt)
        return Macros(phi, gphi, lphi, n, mu, rho, grho, F, u, dtphi, D, T, q, p,
                      alpha, self.viscosity(phi), self._pad2(phi))

    def _pad2(self, phi):
        return None if self.grad_scheme == "central" else self.ghost_pad_wide(phi, "phi", 2)

    # -- equilibria, sources, collision (S8-S10) --------------------------------

    def gamma(self, L: Lattice, u):
        """Eq. FunctionGamma for every direction: list of Q tensors."""
        uu = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
        out = []
        for i in range(L.Q):
            cu = sum(L.c[i][a] * u[a] for a in range(3) if L.c[i][a] != 0)
            if isinstance(cu, int):
                cu = torch.zeros(self.shape, dtype=self.dt)
            out.append(L.w[i] * (1.0 + cu / L.cs2 + cu * cu / (2.0 * L.cs2 ** 2)
                                 - uu / (2.0 * L.cs2)))
        return out

    def f_terms(self, m: Macros):
        """Eq. Feq_NS_Incompr and source S^f = F^f + P^f (Eqs. Forcing,
        MicroProduction).  Returns (feq, S) lists."""
        L = self.Lf
        Gm = self.gamma(L, m.u)
        cs2 = L.cs2
        prod = m.rho * cs2 * self.rho_g * m.q * (1.0 / self.rho_g - 1.0 / self.rho_l)
        feq, S = [], []
        biased = self.grad_scheme != "central"
        if biased:
            # R27: the projections on c_i of grad(rho) and of the surface
            # tension use the biased directional derivative; u . X keeps the
            # Eq. Grad vector
            u_grho = sum(m.u[a] * m.grad_rho[a] for a in range(3))
            u_F = sum(m.u[a] * m.F[a] for a in range(3))
            Fn = [(m.rho - self.rho_l) * self.grav[a] + self.body[a] for a in range(3)]
        for i in range(L.Q):
            feq.append(L.w[i] * m.p + m.rho * cs2 * (Gm[i] - L.w[i]))
            if biased:
                cp = self.cproj(m, L.c[i])
                c_grho = (self.rho_g - self.rho_l) * cp
                c_F = m.mu * cp + sum(L.c[i][a] * Fn[a] for a in range(3) if L.c[i][a] != 0)
                Ff = ((Gm[i] - L.w[i]) * cs2 * (c_grho - u_grho) + Gm[i] * (c_F - u_F))
            else:
                Ff = 0.0
                for a in range(3):
                    Ff = Ff + (L.c[i][a] - m.u[a]) * ((Gm[i] - L.w[i]) * cs2 * m.grad_rho[a]
                                                      + Gm[i] * m.F[a])
            S.append(Ff + L.w[i] * prod)
        return feq, S

    def g_terms(self, m: Macros):
        """Eq. Geq_Allen-Cahn_Eq with S^g = F^g + P^g (Eq. SourceTerm_AllenCahn),
        or, with ``geq_cac``, the equivalent Eq. Geq_AC-1 with only P^g."""
        L = self.Lg
        Gm = self.gamma(L, m.u)
        k = (4.0 / self.W) * m.phi * (1.0 - m.phi)
        geq, S = [], []
        for i in range(L.Q):
            cn = sum(L.c[i][a] * m.n[a] for a in range(3) if L.c[i][a] != 0)
            Fg = k * L.w[i] * cn
            Pg = L.w[i] * m.q
            if self.geq_cac:
                geq.append(m.phi * Gm[i] + self.M * Fg / L.cs2)
                S.append(Pg + 0.0 * m.phi)
            else:
                geq.append(m.phi * Gm[i])
                S.append(Fg + Pg)
        return geq, S

    def s_terms(self, m: Macros):
        """Eq. Seq_Temp with S^s_i = -w_i (L/Cp)[d_t phi + div(u phi)] (R4)."""
        L = self.Ls
        Gm = self.gamma(L, m.u)
        src = -self.Lcp * (m.dtphi + m.D)
        return [m.T * Gm[i] for i in range(L.Q)], [L.w[i] * src for i in range(L.Q)]

    @staticmethod
    def bgk(pop_i, eq_i, S_i, omega):
        """Eq. LBE with Eq. VariableChange_feq: bar-eq = eq - S/2."""
        return pop_i - omega * (pop_i - (eq_i - 0.5 * S_i)) + S_i

    @staticmethod
    def trt(L: Lattice, pop, eq, S, om_plus, om_minus):
        """Two-relaxation-time collision (R26): a = pop - eq + S/2 split into
        its parts symmetric and antisymmetric under c_i -> -c_i."""
        a = [pop[i] - eq[i] + 0.5 * S[i] for i in range(L.Q)]
        out = []
        for i in range(L.Q):
            j = L.opp[i]
            sym = 0.5 * (a[i] + a[j])
            anti = 0.5 * (a[i] - a[j])
            out.append(pop[i] - om_plus * sym - om_minus * anti + S[i])
        return torch.stack(out)

    @staticmethod
    def mrt(L: Lattice, pop, eq, S, rates):
        """Multiple-relaxation-time collision (R26): the moments m_k =
        sum_i M_ki a_i of a = pop - eq + S/2 relax with rates[k]; M has
        orthogonal rows, so the inverse map is M^T divided by the squared row
        norms."""
        Mx = moment_basis(L)
        Q = L.Q
        norms = [sum(Mx[k][i] ** 2 for i in range(Q)) for k in range(Q)]
        a = [pop[i] - eq[i] + 0.5 * S[i] for i in range(Q)]
        m = [sum(Mx[k][i] * a[i] for i in range(Q) if Mx[k][i] != 0) for k in range(Q)]
        dm = [rates[k] * m[k] / norms[k] for k in range(Q)]
        out = []
        for i in range(Q):
            back = sum(Mx[k][i] * dm[k] for k in range(Q) if Mx[k][i] != 0)
            out.append(pop[i] - back + S[i])
        return torch.stack(out)

    def relax(self, family: int, L: Lattice, pop, eq, S, tau):
        """Collision of one family (0 f, 1 g, 2 s) whose transport
        coefficient gives tau (tau = diffusivity / c_s^2, a number or a
        per-node tensor): BGK (Eq. LBE), TRT or MRT (R26)."""
        om = 1.0 / (tau + 0.5)
        if self.collision == "bgk":
            return torch.stack([self.bgk(pop[i], eq[i], S[i], om) for i in range(L.Q)])
        if self.collision == "trt":
            lam = self.trt_lambda[family]
            other = 1.0 / (lam / tau + 0.5)      # (1/w - 1/2) = Lambda / tau
            if family == 0:
                return self.trt(L, pop, eq, S, om, other)
            return self.trt(L, pop, eq, S, other, om)
        s_e, s_eps, s_q, s_p = self.mrt_rates[family]
        if L.name == "D2Q9":
            if family == 0:   # rho, e, eps, jx, qx, jy, qy, pxx, pxy
                rates = [s_e, s_e, s_eps, s_q, s_q, s_q, s_q, om, om]
            else:
                rates = [s_e, s_e, s_eps, om, s_q, om, s_q, s_p, s_p]
        elif L.name in ("D3Q7", "D2Q5") and family != 0:
            if L.name == "D3Q7":   # 1, cx, cy, cz, 7c^2 - 6, 2cx^2 - cy^2 - cz^2, cy^2 - cz^2
                rates = [s_e, om, om, om, s_e, s_p, s_p]
            else:                  # 1, cx, cy, 5c^2 - 4, cx^2 - cy^2
                rates = [s_e, om, om, s_e, s_p]
        else:
            raise ValueError(f"MRT is not defined here for {L.name} (family {family})")
        return self.mrt(L, pop, eq, S, rates)

    def collide(self, st: State, m: Macros):
        out_f = out_s = None
        if self.ns:
            feq, S = self.f_terms(m)
            out_f = self.relax(0, self.Lf, st.f, feq, S, m.nu / self.Lf.cs2)   # nu = tau_f c_s^2
        geq, S = self.g_terms(m)
        out_g = self.relax(1, self.Lg, st.g, geq, S, self.M / self.Lg.cs2)     # M = tau_g c_s^2
        if self.heat:
            seq, S = self.s_terms(m)
            out_s = self.relax(2, self.Ls, st.s, seq, S, m.alpha / self.Ls.cs2)  # alpha = tau_s c_s^2
        return out_f, out_g, out_s

    # -- streaming with walls (S11) ---------------------------------------------

    def _boundary_mask(self, a: int, side: int):
        d = _tensor_axis(a)
        n = self.shape[d]
        idx = torch.arange(n)
        m = (idx == 0) if side == 0 else (idx == n - 1)
        shape = [1, 1, 1]
        shape[d] = n
        return m.reshape(shape)

    def stream(self, post, L: Lattice, kind: str, wall_val=None):
        """Pull streaming new_i(x) = post_i(x - c_i) (periodic roll); at a wall
        the link reflects: bounce-back new_i = post_{i'} ('bb', an open face of
        f instead -post_{i'} + 2 w_i p_w, R29) or anti-bounce-back
        new_i = -post_{i'} + 2 w_i V_w ('abb', Sec. 3.3)."""
        out = []
        for i in range(L.Q):
            c = L.c[i]
            v = torch.roll(post[i], shifts=(c[2], c[1], c[0]), dims=(0, 1, 2))
            for a in range(3):          # higher axis applied last wins (R13)
                if not self.wall[a] or c[a] == 0:
                    continue
                side = 0 if c[a] > 0 else 1
                mask = self._boundary_mask(a, side)
                if kind == "bb":
                    repl = (-post[L.opp[i]] + 2.0 * L.w[i] * self.p_w[a][side]
                            if self.f_open[a][side] else post[L.opp[i]])
                else:
                    repl = -post[L.opp[i]] + 2.0 * L.w[i] * wall_val[a][side]
                v = torch.where(mask, repl, v)
            out.append(v)
        return torch.stack(out)

    # -- one time step ------------------------------------------------------------

    def step(self, st: State, u_prescribed=None) -> State:
        m = self.macros(st, u_prescribed)
        pf, pg, ps = self.collide(st, m)
        phiw = [[torch.tensor(v, dtype=self.dt) for v in side] for side in self.phi_w]
        nf = self.stream(pf, self.Lf, "bb") if self.ns else None
        ng = self.stream(pg, self.Lg, "abb", phiw)
        ns_ = self.stream(ps, self.Ls, "abb", self.T_w) if self.heat else None
        return State(nf, ng, ns_, m.phi, m.q)

    def run(self, st: State, nsteps: int, u_prescribed=None) -> State:
        for _ in range(nsteps):
            st = self.step(st, u_prescribed)
        return st

    # -- initialisation (R12) ---------------------------------------------------

    def init(self, phi0, T0=None, u0=None, p0=None) -> State:
        phi = torch.as_tensor(phi0, dtype=self.dt).reshape(self.shape)
        T = (torch.zeros(self.shape, dtype=self.dt) if (T0 is None or not self.heat)
             else torch.as_tensor(T0, dtype=self.dt).reshape(self.shape))
        u = ([torch.zeros(self.shape, dtype=self.dt) for _ in range(3)] if u0 is None
             else [torch.as_tensor(u0[a], dtype=self.dt).reshape(self.shape) for a in range(3)])
        if not self.ns and u0 is None:
            u = [torch.zeros(self.shape, dtype=self.dt) for _ in range(3)]
        p = (torch.zeros(self.shape, dtype=self.dt) if p0 is None
             else torch.as_tensor(p0, dtype=self.dt).reshape(self.shape))
        P = self.ghost_pad(phi, "phi")
        gphi = self.grad(P)
        lphi = self.laplacian(P, phi)
        norm = torch.sqrt(gphi[0] ** 2 + gphi[1] ** 2 + gphi[2] ** 2 + self.eps ** 2)
        n = [gphi[a] / norm for a in range(3)]
        mu, rho, F = self.forces(phi, gphi, lphi)
        grho = [(self.rho_g - self.rho_l) * gphi[a] for a in range(3)]
        alpha = self.diffusivity(phi)
        q = self.production(phi, T, alpha) if self.heat else torch.zeros(self.shape, dtype=self.dt)
        # the first step's div term sees q_prev = q(phi0, T0)
        D = (self.divergence_term(u, P, gphi, phi, q) if self.heat
             else torch.zeros(self.shape, dtype=self.dt))
        zero = torch.zeros(self.shape, dtype=self.dt)
        m = Macros(phi, gphi, lphi, n, mu, rho, grho, F, u, zero, D, T, q, p, alpha,
                   self.viscosity(phi), self._pad2(phi))
        f = g = s = None
        if self.ns:
            feq, S = self.f_terms(m)
            f = torch.stack([feq[i] - 0.5 * S[i] for i in range(self.Lf.Q)])
        geq, S = self.g_terms(m)
        g = torch.stack([geq[i] - 0.5 * S[i] for i in range(self.Lg.Q)])
        if self.heat:
            seq, S = self.s_terms(m)
            s = torch.stack([seq[i] - 0.5 * S[i] for i in range(self.Ls.Q)])
        return State(f, g, s, phi.clone(), q)

    # -- outputs ----------------------------------------------------------------

    def fields(self, st: State, u_prescribed=None) -> dict:
        """phi, p, u, T from the current populations (S1-S7)."""
        m = self.macros(st, u_prescribed)
        return dict(phi=m.phi, p=m.p, ux=m.u[0], uy=m.u[1], uz=m.u[2], T=m.T)

    def diagnostics(self, st: State) -> dict:
        """FP64 sums: Phi = sum phi, E = sum T + (L/Cp)(Phi + Phi_prev)/2,
        vapour fraction Phi/N, max|u|."""
        m = self.macros(st)
        Phi = m.phi.sum()
        Phi_prev = st.phi_prev.sum()
        E = m.T.sum() + self.Lcp * 0.5 * (Phi + Phi_prev)
        umag = torch.sqrt(m.u[0] ** 2 + m.u[1] ** 2 + m.u[2] ** 2)
        N = m.phi.numel()
        return dict(mass=float(Phi), enthalpy=float(E), vapour=float(Phi) / N,
                    umax=float(umag.max()))


def moment_basis(L: Lattice):
    """Orthogonal moment basis of the MRT collision (R26) as a Q x Q list:
    row k holds polynomial k evaluated at the lattice velocities c_i.
    D2Q9 (Lallemand and Luo): 1, e = -4 + 3c^2, eps = 4 - 21c^2/2 + 9c^4/2,
    cx, qx = (3c^2 - 5)cx, cy, qy = (3c^2 - 5)cy, cx^2 - cy^2, cx cy.
    D3Q7: 1, cx, cy, cz, 7c^2 - 6, 2cx^2 - cy^2 - cz^2, cy^2 - cz^2.
    D2Q5: 1, cx, cy, 5c^2 - 4, cx^2 - cy^2."""
    def c2(c):
        return c[0] ** 2 + c[1] ** 2 + c[2] ** 2
    if L.name == "D2Q9":
        polys = [lambda c: 1.0,
                 lambda c: -4.0 + 3.0 * c2(c),
                 lambda c: 4.0 - 10.5 * c2(c) + 4.5 * c2(c) ** 2,
                 lambda c: float(c[0]),
                 lambda c: (3.0 * c2(c) - 5.0) * c[0],
                 lambda c: float(c[1]),
                 lambda c: (3.0 * c2(c) - 5.0) * c[1],
                 lambda c: float(c[0] ** 2 - c[1] ** 2),
                 lambda c: float(c[0] * c[1])]
    elif L.name == "D3Q7":
        polys = [lambda c: 1.0,
                 lambda c: float(c[0]),
                 lambda c: float(c[1]),
                 lambda c: float(c[2]),
                 lambda c: 7.0 * c2(c) - 6.0,
                 lambda c: float(2 * c[0] ** 2 - c[1] ** 2 - c[2] ** 2),
                 lambda c: float(c[1] ** 2 - c[2] ** 2)]
    elif L.name == "D2Q5":
        polys = [lambda c: 1.0,
                 lambda c: float(c[0]),
                 lambda c: float(c[1]),
                 lambda c: 5.0 * c2(c) - 4.0,
                 lambda c: float(c[0] ** 2 - c[1] ** 2)]
    else:
        raise ValueError(f"no MRT basis for {L.name}")
    return [[p(ci) for ci in L.c] for p in polys]


def relative_l2(x, ref, about_mean: bool = False) -> float:
    x = torch.as_tensor(x, dtype=F64)
    ref = torch.as_tensor(ref, dtype=F64)
    if about_mean:
        x = x - x.mean()
        ref = ref - ref.mean()
    den = float(torch.linalg.vector_norm(ref))
    num = float(torch.linalg.vector_norm(x - ref))
    return num / den if den > 0 else num
