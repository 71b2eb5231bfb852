"""Oracle pins on exact discrete invariants: init round trip (R12), mass
conservation without sources (P6), the enthalpy invariant that fixes the
heat-source sign (P7) and the backward time derivative (R7), the discrete
mass balance of the lagged production (R6), z-invariance 3-D == 2-D (P13)
and the buoyancy sign (R5)."""
import numpy as np
import pytest
import torch

from oracle.lbm_oracle import F64, Model
from paper_2003_06342_amd import inputs as I


def test_init_returns_inputs_exactly():
    """R12: the moments of the initial populations return phi0, T0, u0, p0."""
    p = I.film2d_params(12, 10)
    M = Model(p)
    phi0, T0, _ = I.film2d_fields(p, seed=0, h0=4.0, amp=1.0)
    rng = np.random.default_rng(7)
    u0 = [rng.normal(0, 1e-3, M.shape), rng.normal(0, 1e-3, M.shape), np.zeros(M.shape)]
    p0 = rng.normal(0, 1e-3, M.shape)
    st = M.init(phi0, T0, u0, p0)
    f = M.fields(st)
    assert torch.allclose(f["phi"], torch.tensor(phi0), atol=1e-14)
    assert torch.allclose(f["T"], torch.tensor(T0), atol=1e-14)
    assert torch.allclose(f["ux"], torch.tensor(u0[0]), atol=1e-15)
    assert torch.allclose(f["uy"], torch.tensor(u0[1]), atol=1e-15)
    assert torch.allclose(f["p"], torch.tensor(p0), atol=1e-15)


def test_mass_conserved_without_sources():
    """P6: heat off, periodic: sum(phi) is conserved to round-off."""
    p = I.drop_params(48, sigma=1e-3)
    M = Model(p)
    phi0, _ = I.drop_fields(p, radius=12.0)
    st = M.init(phi0)
    m0 = M.diagnostics(st)["mass"]
    st = M.run(st, 300)
    m1 = M.diagnostics(st)["mass"]
    assert abs(m1 - m0) / m0 < 1e-13
    assert M.diagnostics(st)["umax"] > 0  # the flow is not trivially zero


@pytest.mark.parametrize("dim", [2, 3])
def test_enthalpy_invariant_periodic(dim):
    """P7: periodic, full coupling: E = sum T + (L/Cp)(Phi^n + Phi^{n-1})/2
    is conserved to round-off (holds only with the minus sign of R4)."""
    if dim == 2:
        p = I.base_params(dim=2, nx=24, ny=20, **I.FB)
    else:
        p = I.base_params(dim=3, nx=10, ny=8, nz=9, lat_f="D3Q19", lat_g="D3Q7", lat_s="D3Q7", **I.FB)
    p["gravity"] = [0.0, -1e-4, 0.0] if dim == 2 else [0.0, 0.0, -1e-4]
    M = Model(p)
    phi0, T0 = I.random_smooth_fields(p, seed=11, T_amp=0.5)
    st = M.init(phi0, T0)
    E0 = M.diagnostics(st)["enthalpy"]
    Es = []
    for _ in range(4):
        st = M.run(st, 15)
        Es.append(M.diagnostics(st)["enthalpy"])
    d = M.diagnostics(st)
    assert d["umax"] > 1e-6
    scale = float(np.abs(T0).sum() + p["L_over_cp"] * np.abs(phi0).sum())
    assert max(abs(e - E0) for e in Es) / scale < 1e-13
    # sum(phi) is NOT conserved here (production is on): the invariant is non-trivial
    assert abs(M.diagnostics(st)["mass"] - float(phi0.sum())) > 1e-6


def test_enthalpy_flips_with_wrong_heat_sign():
    """Planting the printed '+' sign of the heat source in the oracle breaks P7."""
    p = I.base_params(dim=2, nx=16, ny=12, **I.FB)
    M = Model(p)
    orig = M.s_terms

    def plus_sign(m):
        seq, S = orig(m)
        return seq, [-x for x in S]
    M.s_terms = plus_sign
    phi0, T0 = I.random_smooth_fields(p, seed=2, T_amp=0.5)
    st = M.init(phi0, T0)
    E0 = M.diagnostics(st)["enthalpy"]
    st = M.run(st, 20)
    assert abs(M.diagnostics(st)["enthalpy"] - E0) > 1e-6


def test_z_invariance_3d_equals_2d():
    """P13: z-invariant data on D3Q19 (f) + D3Q7 (g, s) with D3Q19 stencils
    equals the 2-D run on D2Q9 (f) + D2Q5 (g, s) with D2Q9 stencils."""
    nx, ny = 16, 14
    p2 = I.film2d_params(nx, ny, lat_g="D2Q5", lat_s="D2Q5")
    p2["gravity"] = [0.0, -2e-5, 0.0]
    p3 = I.film2d_params(nx, ny, lat_g="D3Q7", lat_s="D3Q7")
    p3.update(dim=3, nz=3, lat_f="D3Q19")
    p3["gravity"] = [0.0, -2e-5, 0.0]
    M2, M3 = Model(p2), Model(p3)
    phi0, T0, _ = I.film2d_fields(p2, seed=0, h0=5.0, amp=1.5)
    s2 = M2.init(phi0, T0)
    s3 = M3.init(np.repeat(phi0, 3, axis=0), np.repeat(T0, 3, axis=0))
    s2 = M2.run(s2, 40)
    s3 = M3.run(s3, 40)
    f2, f3 = M2.fields(s2), M3.fields(s3)
    for k in ("phi", "T", "p", "ux", "uy"):
        for z in range(3):
            assert torch.allclose(f3[k][z], f2[k][0], atol=1e-13, rtol=0), k
    assert float(f2["uy"].abs().max()) > 1e-5


def test_buoyant_bubble_rises():
    """R5: a vapour bubble in liquid under gravity -y moves up (+y)."""
    nx, ny = 32, 48
    p = I.film2d_params(nx, ny, heat=False, phase_change=False)
    p["gravity"] = [0.0, -2e-5, 0.0]
    p["phi_wall"] = [[0, 0], [0.0, 0.0], [0, 0]]       # liquid at both walls
    M = Model(p)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    r = np.sqrt((x[None, :] - 16) ** 2 + (y[:, None] - 18) ** 2)
    phi0 = (0.5 * (1 + np.tanh(2 * (8 - r) / p["W"])))[None]
    st = M.init(phi0)
    yc = lambda ph: float((ph[0] * torch.tensor(y)[:, None]).sum() / ph[0].sum())
    y0 = yc(M.fields(st)["phi"])
    st = M.run(st, 400)
    f = M.fields(st)
    assert yc(f["phi"]) > y0 + 0.05
    assert float(f["uy"][0].max()) > 0


def test_enthalpy_invariant_pins_the_backward_time_derivative():
    """R7: the invariant of P7 holds because dphi/dt is the backward
    difference phi^n - phi^{n-1} with phi^{n-1} advanced every step.  A lag
    that is not advanced (phi_prev kept at phi^0) breaks it."""
    from oracle.lbm_oracle import State

    class StaleLag(Model):
        def step(self, st, u_prescribed=None):
            new = super().step(st, u_prescribed)
            return State(new.f, new.g, new.s, st.phi_prev, new.q_prev)

    p = I.base_params(dim=2, nx=16, ny=12, **I.FB)
    p["gravity"] = [0.0, -1e-4, 0.0]
    phi0, T0 = I.random_smooth_fields(p, seed=11, T_amp=0.5)
    drift = {}
    for name, cls in (("backward", Model), ("stale", StaleLag)):
        M = cls(p)
        st = M.init(phi0, T0)
        E0 = M.diagnostics(st)["enthalpy"]
        st = M.run(st, 20)
        drift[name] = abs(M.diagnostics(st)["enthalpy"] - E0)
    scale = float(np.abs(T0).sum() + p["L_over_cp"] * np.abs(phi0).sum())
    assert drift["backward"] / scale < 1e-13
    assert drift["stale"] / scale > 1e-8, drift


def _mass_balance_residual(p, cls, nsteps=10):
    """Largest |Phi^{n+1} - Phi^n - [(3 - w)/2 Q^n + (w - 1)/2 Q^{n-1}]| over
    the run, relative to max |Q^n| (Phi = sum phi, Q = sum q over the
    periodic domain, w the BGK rate of g)."""
    M = cls(p)
    st = M.init(*I.random_smooth_fields(p, seed=11, T_amp=0.5))
    w = 1.0 / (3.0 * p["mobility"] + 0.5)
    Phi, Q, Qp = [], [], []
    for _ in range(nsteps):
        m = M.macros(st)
        Phi.append(float(m.phi.sum()))
        Q.append(float(m.q.sum()))
        Qp.append(float(st.q_prev.sum()))
        st = M.step(st)
    Phi, Q, Qp = map(np.array, (Phi, Q, Qp))
    pred = 0.5 * (3.0 - w) * Q[:-1] + 0.5 * (w - 1.0) * Qp[:-1]
    return np.abs(np.diff(Phi) - pred).max() / np.abs(Q).max()


@pytest.mark.parametrize("mobility", [0.0816, 0.02])
def test_mass_balance_pins_the_lagged_production(mobility):
    """R6: phi = sum g + q^{n-1}/2 (the production lagged one step).  Summed
    over a periodic domain, the BGK collision of g with its production
    source P^g_i = w_i q gives the exact discrete balance
        Phi^{n+1} - Phi^n = (3 - w)/2 Q^n + (w - 1)/2 Q^{n-1},
    weights summing to one (no production is lost), with w = 1/(3 M + 1/2).
    It holds to round-off at two mobilities; dropping the lag term from the
    phi moment breaks it."""
    p = I.base_params(dim=2, nx=16, ny=12, **dict(I.FB, mobility=mobility))
    p["gravity"] = [0.0, -1e-4, 0.0]
    assert _mass_balance_residual(p, Model) < 1e-11

    class NoLag(Model):
        def macros(self, st, u_prescribed=None):
            from oracle.lbm_oracle import State
            st0 = State(st.f, st.g, st.s, st.phi_prev, torch.zeros_like(st.q_prev))
            return super().macros(st0, u_prescribed)
    assert _mass_balance_residual(p, NoLag) > 1e-3
