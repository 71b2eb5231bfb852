"""P17: brute force on tiny inputs.  One time step of the 2-D scheme written
as plain scalar loops over nodes and directions (Python floats, no arrays),
straight from the step's definitions: Eqs. Moment_Phi (production lagged,
R6), DerivDirec_Grad / Grad and DerivDirect_Laplacian / Laplacian with
half-way wall ghosts (R13), NormalVector (R9), ChemicalPotential, Density,
Force_Total (R5), Velocity, the backward time derivative (R7), the central
div(u phi) (R8), Moment_Temp (R4), ProductionRate, Pressure (R18),
FunctionGamma, Feq_NS_Incompr, Forcing, MicroProduction,
Geq_Allen-Cahn_Eq, SourceTerm_AllenCahn, Seq_Temp, the BGK collision of
Eq. LBE with the variable change, and pull streaming with bounce-back and
anti-bounce-back links (Sec. 3.3; the y wall wins at a corner).  It is
compared with the vectorised oracle on 6 x 5 grids over several steps, and
a planted sign mistake in the oracle is shown to fail the comparison."""
import math

import numpy as np
import pytest

from oracle.lbm_oracle import Model
from paper_2003_06342_amd import inputs as I

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
WT = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
OPP = [next(j for j in range(9) if CX[j] == -CX[i] and CY[j] == -CY[i]) for i in range(9)]
CS2 = 1.0 / 3.0


def brute_step(prm, f, g, s, phip, qp):
    """One step; f, g, s: [9][ny][nx] nested lists of pulled populations,
    phip, qp: [ny][nx].  Returns the next (f, g, s, phip, qp)."""
    nx, ny = prm["nx"], prm["ny"]
    wallx, wally = prm["bc"][0] == "wall", prm["bc"][1] == "wall"
    rl, rg = prm["rho_l"], prm["rho_g"]
    W, sig = prm["W"], prm["sigma"]
    K, H = 1.5 * W * sig, 12.0 * sig / W
    M, Lcp = prm["mobility"], prm["L_over_cp"]
    grav, body = prm["gravity"], prm["body_force"]
    eps = prm["eps_n"]
    X, Y = range(nx), range(ny)

    phi = [[sum(g[i][y][x] for i in range(9)) + 0.5 * qp[y][x] for x in X] for y in Y]

    def ghost(field, x, y, kind, wx_val, wy_val):
        """field at (x, y), x and y at most one node outside: periodic wrap,
        or the half-way mirror: 'phi' 2 V_w - v, 'anti' -v (x first, then y)."""
        def at_x(xx, yy):
            if 0 <= xx < nx:
                return field[yy][xx]
            if not wallx:
                return field[yy][xx % nx]
            m = 0 if xx < 0 else nx - 1
            v = field[yy][m]
            return 2.0 * wx_val[0 if xx < 0 else 1] - v if kind == "phi" else -v
        if 0 <= y < ny:
            return at_x(x, y)
        if not wally:
            return at_x(x, y % ny)
        m = 0 if y < 0 else ny - 1
        v = at_x(x, m)
        return 2.0 * wy_val[0 if y < 0 else 1] - v if kind == "phi" else -v

    pwx, pwy = prm["phi_wall"][0], prm["phi_wall"][1]
    P = lambda x, y: ghost(phi, x, y, "phi", pwx, pwy)
    gx = [[0.0] * nx for _ in Y]
    gy = [[0.0] * nx for _ in Y]
    lap = [[0.0] * nx for _ in Y]
    for y in Y:
        for x in X:
            ax = ay = l = 0.0
            for i in range(1, 9):
                pp, pm = P(x + CX[i], y + CY[i]), P(x - CX[i], y - CY[i])
                ax += WT[i] * CX[i] * 0.5 * (pp - pm)
                ay += WT[i] * CY[i] * 0.5 * (pp - pm)
                l += WT[i] * (pp - 2.0 * phi[y][x] + pm)
            gx[y][x], gy[y][x], lap[y][x] = ax / CS2, ay / CS2, l / CS2

    ux = [[0.0] * nx for _ in Y]
    uy = [[0.0] * nx for _ in Y]
    node = {}
    for y in Y:
        for x in X:
            ph = phi[y][x]
            mu = 4.0 * H * ph * (ph - 1.0) * (ph - 0.5) - K * lap[y][x]
            rho = ph * rg + (1.0 - ph) * rl
            F = [mu * gx[y][x] + (rho - rl) * grav[0] + body[0],
                 mu * gy[y][x] + (rho - rl) * grav[1] + body[1]]
            mx = sum(f[i][y][x] * CX[i] for i in range(9))
            my = sum(f[i][y][x] * CY[i] for i in range(9))
            ux[y][x] = (mx / CS2 + 0.5 * F[0]) / rho
            uy[y][x] = (my / CS2 + 0.5 * F[1]) / rho
            nrm = math.sqrt(gx[y][x] ** 2 + gy[y][x] ** 2 + eps * eps)
            node[(x, y)] = dict(mu=mu, rho=rho, F=F, n=(gx[y][x] / nrm, gy[y][x] / nrm))

    zero = (0.0, 0.0)
    UX = lambda x, y: ghost(ux, x, y, "anti", zero, zero)
    UY = lambda x, y: ghost(uy, x, y, "anti", zero, zero)
    post_f = [[[0.0] * nx for _ in Y] for _ in range(9)]
    post_g = [[[0.0] * nx for _ in Y] for _ in range(9)]
    post_s = [[[0.0] * nx for _ in Y] for _ in range(9)]
    new_phip = [[0.0] * nx for _ in Y]
    new_qp = [[0.0] * nx for _ in Y]
    for y in Y:
        for x in X:
            d = node[(x, y)]
            ph, rho, F = phi[y][x], d["rho"], d["F"]
            u = (ux[y][x], uy[y][x])
            dtphi = ph - phip[y][x]
            alpha = (1.0 - ph) * prm["alpha_l"] + ph * prm["alpha_g"]
            D = 0.0
            for i in range(1, 9):
                xp, yp, xm, ym = x + CX[i], y + CY[i], x - CX[i], y - CY[i]
                vp = (UX(xp, yp) * P(xp, yp), UY(xp, yp) * P(xp, yp))
                vm = (UX(xm, ym) * P(xm, ym), UY(xm, ym) * P(xm, ym))
                D += WT[i] * 0.5 * (CX[i] * (vp[0] - vm[0]) + CY[i] * (vp[1] - vm[1]))
            D /= CS2
            T = sum(s[i][y][x] for i in range(9)) - 0.5 * Lcp * (dtphi + D)
            theta = (T - prm["T_sat"]) / Lcp
            q = -(4.0 * alpha / (prm["A_coef"] * W * W)) * (prm["theta_I"] - theta) * ph * (1.0 - ph) \
                if prm["phase_change"] else 0.0
            grho = ((rg - rl) * gx[y][x], (rg - rl) * gy[y][x])
            pfac = rg * (1.0 / rg - 1.0 / rl)
            p = sum(f[i][y][x] for i in range(9)) + 0.5 * (
                CS2 * (u[0] * grho[0] + u[1] * grho[1]) + rho * CS2 * q * pfac)
            nu_l, nu_g = prm["nu_l"], prm["nu_g"]
            nu = nu_l * nu_g / (ph * nu_l + (1.0 - ph) * nu_g)
            om_f = 1.0 / (nu / CS2 + 0.5)
            om_g = 1.0 / (M / CS2 + 0.5)
            om_s = 1.0 / (alpha / CS2 + 0.5)
            uu = u[0] * u[0] + u[1] * u[1]
            for i in range(9):
                cu = CX[i] * u[0] + CY[i] * u[1]
                G = WT[i] * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2))
                feq = WT[i] * p + rho * CS2 * (G - WT[i])
                Sf = sum((c - uc) * ((G - WT[i]) * CS2 * gr + G * Fa)
                         for c, uc, gr, Fa in zip((CX[i], CY[i]), u, grho, F)) \
                    + WT[i] * rho * CS2 * q * pfac
                post_f[i][y][x] = f[i][y][x] - om_f * (f[i][y][x] - (feq - 0.5 * Sf)) + Sf
                cn = CX[i] * d["n"][0] + CY[i] * d["n"][1]
                geq = ph * G
                Sg = (4.0 / W) * ph * (1.0 - ph) * WT[i] * cn + WT[i] * q
                post_g[i][y][x] = g[i][y][x] - om_g * (g[i][y][x] - (geq - 0.5 * Sg)) + Sg
                seq = T * G
                Ss = -WT[i] * Lcp * (dtphi + D)
                post_s[i][y][x] = s[i][y][x] - om_s * (s[i][y][x] - (seq - 0.5 * Ss)) + Ss
            new_phip[y][x], new_qp[y][x] = ph, q

    def stream(post, kind):
        out = [[[0.0] * nx for _ in Y] for _ in range(9)]
        for i in range(9):
            for y in Y:
                for x in X:
                    sx, sy = x - CX[i], y - CY[i]
                    oy = wally and CY[i] != 0 and not (0 <= sy < ny)
                    ox = wallx and CX[i] != 0 and not (0 <= sx < nx)
                    if oy or ox:
                        # the y wall wins at a corner
                        a, side = (1, 0 if sy < 0 else 1) if oy else (0, 0 if sx < 0 else 1)
                        r = post[OPP[i]][y][x]
                        if kind == "g":
                            r = -r + 2.0 * WT[i] * prm["phi_wall"][a][side]
                        elif kind == "s":
                            r = -r + 2.0 * WT[i] * prm["T_wall"][a][side]
                        out[i][y][x] = r
                    else:
                        out[i][y][x] = post[i][sy % ny][sx % nx]
        return out

    return stream(post_f, "f"), stream(post_g, "g"), stream(post_s, "s"), new_phip, new_qp


def _lists(st):
    t = lambda a: a.detach().numpy()[:, 0].tolist() if a.dim() == 4 else a.detach().numpy()[0].tolist()
    return t(st.f), t(st.g), t(st.s), t(st.phi_prev), t(st.q_prev)


def _case(box):
    prm = I.film2d_params(6, 5)
    prm["gravity"] = [0.0, -3e-3, 0.0]
    prm["body_force"] = [2e-4, 0.0, 0.0]
    prm["theta_I"] = 0.05
    if box:
        prm["bc"] = ["wall", "wall", "periodic"]
        prm["phi_wall"] = [[0.3, 0.6], [1.0, 0.8], [0.0, 0.0]]
        prm["T_wall"] = [[0.2, 0.4], [1.0, 0.1], [0.0, 0.0]]
    rng = np.random.default_rng(11)
    y = np.arange(5) + 0.5
    phi0 = (0.5 * (1 + np.tanh(2 * (y[:, None] - 2.2 + 0.4 * rng.standard_normal((1, 6))) / prm["W"])))
    phi0 = np.clip(phi0 + 0.02 * rng.standard_normal((5, 6)), 0.0, 1.0)[None]
    T0 = (1.0 - 0.15 * y[:, None] + 0.05 * rng.standard_normal((5, 6)))[None]
    u0 = [1e-2 * rng.standard_normal((1, 5, 6)), 1e-2 * rng.standard_normal((1, 5, 6)),
          np.zeros((1, 5, 6))]
    return prm, phi0, T0, u0


@pytest.mark.parametrize("box", [False, True])
def test_bruteforce_step_equals_oracle(box):
    prm, phi0, T0, u0 = _case(box)
    M = Model(prm)
    st = M.init(phi0, T0, u0)
    b = _lists(st)
    for n in range(4):
        st = M.step(st)
        b = brute_step(prm, *b)
        o = _lists(st)
        for name, x, y in zip(("f", "g", "s", "phi_prev", "q_prev"), b, o):
            x, y = np.asarray(x), np.asarray(y)
            assert np.abs(x - y).max() <= 1e-13 * max(1.0, np.abs(y).max()), (box, n, name)
    # the run is not trivial: the flow, the production and the heat moved
    f = M.fields(st)
    assert float(f["ux"].abs().max()) > 1e-3 and float(st.q_prev.abs().max()) > 1e-5


def test_bruteforce_detects_a_planted_oracle_mistake(monkeypatch):
    """A sign flipped in the oracle's div(u phi) is caught at the first step."""
    prm, phi0, T0, u0 = _case(False)
    M = Model(prm)
    st = M.init(phi0, T0, u0)
    b = brute_step(prm, *_lists(st))
    orig = Model.divergence
    monkeypatch.setattr(Model, "divergence", lambda self, u, P: -orig(self, u, P))
    o = _lists(M.step(st))
    worst = max(np.abs(np.asarray(x) - np.asarray(y)).max() for x, y in zip(b, o))
    assert worst > 1e-8
