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
a planted sign mistake in the oracle is shown to fail the comparison.  The
3-D step (D3Q19 f and stencils, D3Q7 g and s with c_s^2 = 1/4, walls on z)
is checked the same way on a 4 x 3 x 6 film."""
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


# ---------------------------------------------------------------------------
# 3-D: D3Q19 f and stencils, D3Q7 g and s (each population with its own c_s^2,
# R2 and R3), walls on z.  Written over dictionaries keyed by node; lattice
# tables built here from their definitions.
# ---------------------------------------------------------------------------

def _d3q19():
    c = [(0, 0, 0)]
    c += [v for a in range(3) for v in (tuple(1 if b == a else 0 for b in range(3)),
                                         tuple(-1 if b == a else 0 for b in range(3)))]
    c += [(sx, sy, 0) for sx in (1, -1) for sy in (1, -1)]
    c += [(sx, 0, sz) for sx in (1, -1) for sz in (1, -1)]
    c += [(0, sy, sz) for sy in (1, -1) for sz in (1, -1)]
    w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    return c, w, 1.0 / 3.0


def _d3q7():
    c = [(0, 0, 0)] + [v for a in range(3) for v in (tuple(1 if b == a else 0 for b in range(3)),
                                                     tuple(-1 if b == a else 0 for b in range(3)))]
    return c, [1 / 4] + [1 / 8] * 6, 0.25


def brute_step_3d(prm, f, g, s, phip, qp):
    """f, g, s: dict node -> list of populations (own lattice order);
    phip, qp: dict node -> float.  Walls on z only (x, y periodic)."""
    nx, ny, nz = prm["nx"], prm["ny"], prm["nz"]
    CF, WF, C2F = _d3q19()
    CG, WG, C2G = _d3q7()
    rl, rg = prm["rho_l"], prm["rho_g"]
    W, sig = prm["W"], prm["sigma"]
    K, H = 1.5 * W * sig, 12.0 * sig / W
    M, Lcp = prm["mobility"], prm["L_over_cp"]
    grav, body, eps = prm["gravity"], prm["body_force"], prm["eps_n"]
    nodes = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
    add = lambda p, c, k=1: (p[0] + k * c[0], p[1] + k * c[1], p[2] + k * c[2])
    phi = {p: sum(g[p]) + 0.5 * qp[p] for p in nodes}

    def ghost(field, p, kind, vw):
        x, y, z = p[0] % nx, p[1] % ny, p[2]
        if 0 <= z < nz:
            return field[(x, y, z)]
        v = field[(x, y, 0 if z < 0 else nz - 1)]
        return 2.0 * vw[0 if z < 0 else 1] - v if kind == "phi" else -v

    P = lambda p: ghost(phi, p, "phi", prm["phi_wall"][2])
    d = {}
    for p in nodes:
        gr = [0.0, 0.0, 0.0]
        lap = 0.0
        for c, w in zip(CF[1:], WF[1:]):
            pp, pm = P(add(p, c)), P(add(p, c, -1))
            for a in range(3):
                gr[a] += w * c[a] * 0.5 * (pp - pm)
            lap += w * (pp - 2.0 * phi[p] + pm)
        gr = [v / C2F for v in gr]
        lap /= C2F
        ph = phi[p]
        mu = 4.0 * H * ph * (ph - 1.0) * (ph - 0.5) - K * lap
        rho = ph * rg + (1.0 - ph) * rl
        F = [mu * gr[a] + (rho - rl) * grav[a] + body[a] for a in range(3)]
        m = [sum(fi * c[a] for fi, c in zip(f[p], CF)) for a in range(3)]
        u = [(m[a] / C2F + 0.5 * F[a]) / rho for a in range(3)]
        nrm = math.sqrt(sum(v * v for v in gr) + eps * eps)
        d[p] = dict(gr=gr, lap=lap, mu=mu, rho=rho, F=F, u=u, n=[v / nrm for v in gr])
    U = lambda p, a: ghost({q: d[q]["u"][a] for q in nodes}, p, "anti", (0.0, 0.0))
    Ucache = {}

    def u_at(p, a):
        key = (p, a)
        if key not in Ucache:
            Ucache[key] = U(p, a)
        return Ucache[key]

    post = {}
    out_phip, out_qp = {}, {}
    for p in nodes:
        e = d[p]
        ph, rho, F, u = phi[p], e["rho"], e["F"], e["u"]
        dtphi = ph - phip[p]
        alpha = (1.0 - ph) * prm["alpha_l"] + ph * prm["alpha_g"]
        D = 0.0
        for c, w in zip(CF[1:], WF[1:]):
            qp_, qm_ = add(p, c), add(p, c, -1)
            for a in range(3):
                if c[a]:
                    D += w * c[a] * 0.5 * (u_at(qp_, a) * P(qp_) - u_at(qm_, a) * P(qm_))
        D /= C2F
        T = sum(s[p]) - 0.5 * Lcp * (dtphi + D)
        theta = (T - prm["T_sat"]) / Lcp
        q = -(4.0 * alpha / (prm["A_coef"] * W * W)) * (prm["theta_I"] - theta) * ph * (1.0 - ph)
        grho = [(rg - rl) * v for v in e["gr"]]
        pfac = rg * (1.0 / rg - 1.0 / rl)
        pr = sum(f[p]) + 0.5 * (C2F * sum(u[a] * grho[a] for a in range(3)) + rho * C2F * q * pfac)
        nu = prm["nu_l"] * prm["nu_g"] / (ph * prm["nu_l"] + (1.0 - ph) * prm["nu_g"])
        uu = sum(v * v for v in u)

        def gamma(c, w, cs2):
            cu = sum(c[a] * u[a] for a in range(3))
            return w * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2))
        om = 1.0 / (nu / C2F + 0.5)
        pf = []
        for fi, c, w in zip(f[p], CF, WF):
            G = gamma(c, w, C2F)
            feq = w * pr + rho * C2F * (G - w)
            S = sum((c[a] - u[a]) * ((G - w) * C2F * grho[a] + G * F[a]) for a in range(3)) \
                + w * rho * C2F * q * pfac
            pf.append(fi - om * (fi - (feq - 0.5 * S)) + S)
        omg = 1.0 / (M / C2G + 0.5)
        oms = 1.0 / (alpha / C2G + 0.5)
        pg, ps = [], []
        for gi, si, c, w in zip(g[p], s[p], CG, WG):
            G = gamma(c, w, C2G)
            cn = sum(c[a] * e["n"][a] for a in range(3))
            Sg = (4.0 / W) * ph * (1.0 - ph) * w * cn + w * q
            pg.append(gi - omg * (gi - (ph * G - 0.5 * Sg)) + Sg)
            Ss = -w * Lcp * (dtphi + D)
            ps.append(si - oms * (si - (T * G - 0.5 * Ss)) + Ss)
        post[p] = (pf, pg, ps)
        out_phip[p], out_qp[p] = ph, q

    def stream(k, C, W_, kind):
        out = {}
        opp = [C.index(tuple(-v for v in c)) for c in C]
        for p in nodes:
            vals = []
            for i, c in enumerate(C):
                src = add(p, c, -1)
                if not (0 <= src[2] < nz):   # a z wall link reflects at the node
                    side = 0 if src[2] < 0 else 1
                    r = post[p][k][opp[i]]
                    if kind == "g":
                        r = -r + 2.0 * W_[i] * prm["phi_wall"][2][side]
                    elif kind == "s":
                        r = -r + 2.0 * W_[i] * prm["T_wall"][2][side]
                    vals.append(r)
                else:
                    vals.append(post[(src[0] % nx, src[1] % ny, src[2])][k][i])
            out[p] = vals
        return out

    return (stream(0, CF, WF, "f"), stream(1, CG, WG, "g"), stream(2, CG, WG, "s"), out_phip, out_qp)


def test_bruteforce_step_equals_oracle_3d():
    """Four steps of a 4 x 3 x 6 film (walls on z, x and y periodic) with an
    initial velocity: the scalar 3-D step equals the oracle's populations to
    1e-13 (mapped between the two lattice orderings by their velocities)."""
    prm = I.film3d_params(4, nz=6)
    prm["ny"] = 3
    prm["gravity"] = [0.0, 0.0, -3e-3]
    prm["body_force"] = [2e-4, -1e-4, 0.0]
    prm["theta_I"] = 0.05
    rng = np.random.default_rng(5)
    z = np.arange(6) + 0.5
    phi0 = 0.5 * (1 + np.tanh(2 * (z[:, None, None] - 2.7 + 0.4 * rng.standard_normal((1, 3, 4))) / prm["W"]))
    phi0 = np.clip(phi0 + 0.02 * rng.standard_normal((6, 3, 4)), 0.0, 1.0)
    T0 = 1.0 - 0.15 * z[:, None, None] + 0.05 * rng.standard_normal((6, 3, 4))
    u0 = [1e-2 * rng.standard_normal((6, 3, 4)) for _ in range(3)]
    Mo = Model(prm)
    st = Mo.init(phi0, T0, u0)
    CF, CG = _d3q19()[0], _d3q7()[0]
    perm_f = [CF.index(tuple(int(v) for v in c)) for c in Mo.Lf.c]   # oracle index -> ours
    perm_g = [CG.index(tuple(int(v) for v in c)) for c in Mo.Lg.c]
    nodes = [(x, y, zz) for zz in range(6) for y in range(3) for x in range(4)]

    def to_ours(pop, perm, Q):
        a = pop.detach().numpy()
        out = {}
        for (x, y, zz) in nodes:
            v = [0.0] * Q
            for i in range(Q):
                v[perm[i]] = float(a[i, zz, y, x])
            out[(x, y, zz)] = v
        return out
    b = (to_ours(st.f, perm_f, 19), to_ours(st.g, perm_g, 7), to_ours(st.s, perm_g, 7),
         {p: float(st.phi_prev[p[2], p[1], p[0]]) for p in nodes},
         {p: float(st.q_prev[p[2], p[1], p[0]]) for p in nodes})
    for n in range(4):
        st = Mo.step(st)
        b = brute_step_3d(prm, *b)
        o = (to_ours(st.f, perm_f, 19), to_ours(st.g, perm_g, 7), to_ours(st.s, perm_g, 7))
        for name, mine, ref in zip(("f", "g", "s"), b[:3], o):
            worst = max(abs(mine[p][i] - ref[p][i]) for p in nodes for i in range(len(ref[p])))
            scale = max(1.0, max(abs(v) for p in nodes for v in ref[p]))
            assert worst <= 1e-13 * scale, (n, name, worst)
        for name, mine, ref in (("phi_prev", b[3], st.phi_prev), ("q_prev", b[4], st.q_prev)):
            worst = max(abs(mine[p] - float(ref[p[2], p[1], p[0]])) for p in nodes)
            assert worst <= 1e-13, (n, name, worst)
    f = Mo.fields(st)
    assert float(f["uz"].abs().max()) > 1e-4 and float(st.q_prev.abs().max()) > 1e-5
