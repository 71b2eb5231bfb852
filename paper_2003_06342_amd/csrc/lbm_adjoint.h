// Hand-written adjoint of the 2-D (D2Q9 x 3) node update.
//
// The forward step at a node maps its pulled populations P (f, g, s), the
// phase field phi, its stencils (grad phi, lap phi), the velocity u, the
// divergence D = div(u phi) and phi_prev to the post-collision populations
// and the production q (Secs. 2-3; same closures and collisions as the
// fused kernel).  node_adj applies the transposed Jacobian of that map to
// the adjoints of its outputs.  u_fwd / u_adj do the same for the velocity
// closure u = (3 sum f c + F/2)/rho (Eq. Velocity) with F from Eqs.
// ChemicalPotential and Force_Total.  The functions are __host__ __device__
// so that a host program can check them against finite differences.
#pragma once

#include <math.h>

namespace lbm {
namespace adj {

struct W9 {
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return v[i];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

// Constants of the node map (lattice units; c_s^2 = 1/3 for all families).
template <class Real>
struct NodeConst {
  Real rho_l, rho_g, K, H, four_over_W, eps2;
  Real grav[2], body[2];
  Real nu_l, nu_g, alpha_l, alpha_g;
  Real Lcp, T_sat, theta_I, qcoef, prod_fac;
  Real omega_g, M_over_cs2g;
  int visc_linear, geq_cac, phase_change;
};

template <class Real>
struct NodeIn {
  Real Pf[9], Pg[9], Ps[9];
  Real phi, gphi[2], lphi, u[2], D, phip;
};

template <class Real>
struct NodeOut {
  Real Af[9], Ag[9], As[9];
  Real q;
};

template <class Real>
struct NodeAdjIn {          // adjoints of the node inputs
  Real Pf[9], Pg[9], Ps[9];
  Real phi, gphi[2], lphi, u[2], D, phip;
};

template <class Real>
__host__ __device__ inline Real viscosity_of(const NodeConst<Real>& c, Real phi, Real& dnu) {
  if (c.visc_linear) {
    dnu = c.nu_g - c.nu_l;
    return ((Real)1 - phi) * c.nu_l + phi * c.nu_g;
  }
  const Real den = phi * c.nu_l + ((Real)1 - phi) * c.nu_g;
  const Real nu = c.nu_l * c.nu_g / den;
  dnu = -nu * (c.nu_l - c.nu_g) / den;
  return nu;
}

// Forward node map (reference form of the fused kernel's phase 3).
template <class Real>
__host__ __device__ inline void node_fwd(const NodeConst<Real>& c, const NodeIn<Real>& in,
                                         NodeOut<Real>& out) {
  const Real cs2 = (Real)(1.0 / 3.0);
  const Real phi = in.phi;
  const Real rho = phi * c.rho_g + ((Real)1 - phi) * c.rho_l;
  const Real mu = (Real)4 * c.H * phi * (phi - (Real)1) * (phi - (Real)0.5) - c.K * in.lphi;
  Real F[2], grho[2], n[2];
  const Real drho = c.rho_g - c.rho_l;
  const Real r = (Real)1 / sqrt(in.gphi[0] * in.gphi[0] + in.gphi[1] * in.gphi[1] + c.eps2);
  for (int a = 0; a < 2; ++a) {
    F[a] = mu * in.gphi[a] + (rho - c.rho_l) * c.grav[a] + c.body[a];
    grho[a] = drho * in.gphi[a];
    n[a] = in.gphi[a] * r;
  }
  const Real dtphi = phi - in.phip;
  Real m0s = 0, m0f = 0;
  for (int i = 0; i < 9; ++i) {
    m0s += in.Ps[i];
    m0f += in.Pf[i];
  }
  const Real T = m0s - (Real)0.5 * c.Lcp * (dtphi + in.D);
  const Real alpha = ((Real)1 - phi) * c.alpha_l + phi * c.alpha_g;
  const Real theta = (T - c.T_sat) / c.Lcp;
  const Real q = c.phase_change ? -c.qcoef * alpha * (c.theta_I - theta) * phi * ((Real)1 - phi)
                                : (Real)0;
  const Real ug = in.u[0] * grho[0] + in.u[1] * grho[1];
  const Real uF = in.u[0] * F[0] + in.u[1] * F[1];
  const Real rc = rho * cs2;
  const Real p = m0f + (Real)0.5 * (cs2 * ug + rc * q * c.prod_fac);
  Real dnu;
  const Real nu = viscosity_of(c, phi, dnu);
  const Real omf = (Real)1 / ((Real)3 * nu + (Real)0.5);
  const Real oms = (Real)1 / ((Real)3 * alpha + (Real)0.5);
  const Real omg = c.omega_g;
  const Real huu = (Real)1.5 * (in.u[0] * in.u[0] + in.u[1] * in.u[1]);
  const Real kk = c.four_over_W * phi * ((Real)1 - phi);
  const Real src = -c.Lcp * (dtphi + in.D);
  for (int i = 0; i < 9; ++i) {
    const Real w = (Real)W9::w(i);
    const Real cx = (Real)W9::cx(i), cy = (Real)W9::cy(i);
    const Real cu = cx * in.u[0] + cy * in.u[1];
    const Real dG = w * (cu * ((Real)3 + (Real)4.5 * cu) - huu);
    // f
    const Real X = cs2 * (cx * grho[0] + cy * grho[1] - ug);
    const Real Y = cx * F[0] + cy * F[1] - uF;
    const Real S = dG * X + (w + dG) * Y + w * rc * q * c.prod_fac;
    const Real feq = w * p + rc * dG;
    out.Af[i] = ((Real)1 - omf) * in.Pf[i] + omf * feq + ((Real)1 - (Real)0.5 * omf) * S;
    // g
    const Real geq = phi * (w + dG);
    const Real Fg = w * kk * (cx * n[0] + cy * n[1]);
    const Real Pgs = w * q;
    if (c.geq_cac)
      out.Ag[i] = ((Real)1 - omg) * in.Pg[i] + omg * (geq + c.M_over_cs2g * Fg) +
                  ((Real)1 - (Real)0.5 * omg) * Pgs;
    else
      out.Ag[i] = ((Real)1 - omg) * in.Pg[i] + omg * geq + ((Real)1 - (Real)0.5 * omg) * (Fg + Pgs);
    // s
    const Real seq = T * (w + dG);
    const Real Ss = w * src;
    out.As[i] = ((Real)1 - oms) * in.Ps[i] + oms * seq + ((Real)1 - (Real)0.5 * oms) * Ss;
  }
  out.q = q;
}

// Transposed Jacobian of node_fwd: given adjoints of (Af, Ag, As, q) return
// adjoints of every input.  Statement-by-statement reverse of node_fwd.
template <class Real>
__host__ __device__ inline void node_adj(const NodeConst<Real>& c, const NodeIn<Real>& in,
                                         const NodeOut<Real>& lo, NodeAdjIn<Real>& li) {
  const Real cs2 = (Real)(1.0 / 3.0);
  // ---- recompute the forward intermediates ----
  const Real phi = in.phi;
  const Real rho = phi * c.rho_g + ((Real)1 - phi) * c.rho_l;
  const Real mu = (Real)4 * c.H * phi * (phi - (Real)1) * (phi - (Real)0.5) - c.K * in.lphi;
  Real F[2], grho[2], n[2];
  const Real drho = c.rho_g - c.rho_l;
  const Real r = (Real)1 / sqrt(in.gphi[0] * in.gphi[0] + in.gphi[1] * in.gphi[1] + c.eps2);
  for (int a = 0; a < 2; ++a) {
    F[a] = mu * in.gphi[a] + (rho - c.rho_l) * c.grav[a] + c.body[a];
    grho[a] = drho * in.gphi[a];
    n[a] = in.gphi[a] * r;
  }
  const Real dtphi = phi - in.phip;
  Real m0s = 0;
  for (int i = 0; i < 9; ++i) m0s += in.Ps[i];
  const Real T = m0s - (Real)0.5 * c.Lcp * (dtphi + in.D);
  const Real alpha = ((Real)1 - phi) * c.alpha_l + phi * c.alpha_g;
  const Real theta = (T - c.T_sat) / c.Lcp;
  const Real pp = phi * ((Real)1 - phi);
  const Real q = c.phase_change ? -c.qcoef * alpha * (c.theta_I - theta) * pp : (Real)0;
  const Real ug = in.u[0] * grho[0] + in.u[1] * grho[1];
  const Real uF = in.u[0] * F[0] + in.u[1] * F[1];
  const Real rc = rho * cs2;
  Real m0f = 0;
  for (int i = 0; i < 9; ++i) m0f += in.Pf[i];
  const Real p = m0f + (Real)0.5 * (cs2 * ug + rc * q * c.prod_fac);
  Real dnu;
  const Real nu = viscosity_of(c, phi, dnu);
  const Real omf = (Real)1 / ((Real)3 * nu + (Real)0.5);
  const Real oms = (Real)1 / ((Real)3 * alpha + (Real)0.5);
  const Real omg = c.omega_g;
  const Real huu = (Real)1.5 * (in.u[0] * in.u[0] + in.u[1] * in.u[1]);
  const Real kk = c.four_over_W * pp;
  const Real src = -c.Lcp * (dtphi + in.D);

  // ---- adjoint accumulators ----
  Real l_phi = 0, l_rho = 0, l_mu = 0, l_F[2] = {0, 0}, l_grho[2] = {0, 0}, l_n[2] = {0, 0};
  Real l_dtphi = 0, l_T = 0, l_alpha = 0, l_q = lo.q, l_p = 0, l_rc = 0;
  Real l_ug = 0, l_uF = 0, l_omf = 0, l_oms = 0, l_huu = 0, l_kk = 0, l_src = 0;
  Real l_u[2] = {0, 0};
  Real l_m0f = 0;
  for (int i = 0; i < 9; ++i) {
    li.Pf[i] = 0;
    li.Pg[i] = 0;
    li.Ps[i] = 0;
  }
  for (int i = 0; i < 9; ++i) {
    const Real w = (Real)W9::w(i);
    const Real cx = (Real)W9::cx(i), cy = (Real)W9::cy(i);
    const Real cu = cx * in.u[0] + cy * in.u[1];
    const Real dG = w * (cu * ((Real)3 + (Real)4.5 * cu) - huu);
    Real l_dG = 0;
    // s: As = (1-oms) Ps + oms seq + (1 - oms/2) Ss
    {
      const Real lA = lo.As[i];
      const Real seq = T * (w + dG);
      const Real Ss = w * src;
      li.Ps[i] += ((Real)1 - oms) * lA;
      l_oms += lA * (-in.Ps[i] + seq - (Real)0.5 * Ss);
      const Real l_seq = oms * lA;
      l_T += l_seq * (w + dG);
      l_dG += l_seq * T;
      l_src += ((Real)1 - (Real)0.5 * oms) * lA * w;
    }
    // g
    {
      const Real lA = lo.Ag[i];
      const Real cn = cx * n[0] + cy * n[1];
      li.Pg[i] += ((Real)1 - omg) * lA;
      const Real l_geq = omg * lA;
      Real l_Fg, l_Pgs;
      if (c.geq_cac) {
        l_Fg = l_geq * c.M_over_cs2g;
        l_Pgs = ((Real)1 - (Real)0.5 * omg) * lA;
      } else {
        l_Fg = ((Real)1 - (Real)0.5 * omg) * lA;
        l_Pgs = l_Fg;
      }
      l_phi += l_geq * (w + dG);
      l_dG += l_geq * phi;
      l_kk += l_Fg * w * cn;
      l_n[0] += l_Fg * w * kk * cx;
      l_n[1] += l_Fg * w * kk * cy;
      l_q += l_Pgs * w;
    }
    // f
    {
      const Real lA = lo.Af[i];
      const Real X = cs2 * (cx * grho[0] + cy * grho[1] - ug);
      const Real Y = cx * F[0] + cy * F[1] - uF;
      const Real S = dG * X + (w + dG) * Y + w * rc * q * c.prod_fac;
      const Real feq = w * p + rc * dG;
      li.Pf[i] += ((Real)1 - omf) * lA;
      l_omf += lA * (-in.Pf[i] + feq - (Real)0.5 * S);
      const Real l_feq = omf * lA;
      l_p += l_feq * w;
      l_rc += l_feq * dG;
      l_dG += l_feq * rc;
      const Real l_S = ((Real)1 - (Real)0.5 * omf) * lA;
      l_dG += l_S * (X + Y);
      const Real l_X = l_S * dG;
      const Real l_Y = l_S * (w + dG);
      l_rc += l_S * w * q * c.prod_fac;
      l_q += l_S * w * rc * c.prod_fac;
      l_grho[0] += cs2 * cx * l_X;
      l_grho[1] += cs2 * cy * l_X;
      l_ug -= cs2 * l_X;
      l_F[0] += cx * l_Y;
      l_F[1] += cy * l_Y;
      l_uF -= l_Y;
    }
    // dG = w (cu (3 + 4.5 cu) - huu)
    const Real l_cu = l_dG * w * ((Real)3 + (Real)9 * cu);
    l_huu -= l_dG * w;
    l_u[0] += cx * l_cu;
    l_u[1] += cy * l_cu;
  }
  // src = -Lcp (dtphi + D)
  l_dtphi += -c.Lcp * l_src;
  Real l_D = -c.Lcp * l_src;
  // huu = 1.5 |u|^2
  l_u[0] += (Real)3 * in.u[0] * l_huu;
  l_u[1] += (Real)3 * in.u[1] * l_huu;
  // kk = (4/W) phi (1 - phi)
  l_phi += l_kk * c.four_over_W * ((Real)1 - (Real)2 * phi);
  // omegas
  const Real l_nu = l_omf * (-(Real)3 * omf * omf);
  l_alpha += l_oms * (-(Real)3 * oms * oms);
  l_phi += l_nu * dnu;
  // p = m0f + 0.5 (cs2 ug + rc q pf)
  l_m0f += l_p;
  l_ug += (Real)0.5 * cs2 * l_p;
  l_rc += (Real)0.5 * q * c.prod_fac * l_p;
  l_q += (Real)0.5 * rc * c.prod_fac * l_p;
  // rc = rho cs2
  l_rho += cs2 * l_rc;
  // ug = u.grho ; uF = u.F
  for (int a = 0; a < 2; ++a) {
    l_u[a] += grho[a] * l_ug + F[a] * l_uF;
    l_grho[a] += in.u[a] * l_ug;
    l_F[a] += in.u[a] * l_uF;
  }
  for (int i = 0; i < 9; ++i) li.Pf[i] += l_m0f;
  // q = -qcoef alpha (theta_I - theta) phi (1 - phi)
  if (c.phase_change) {
    l_alpha += l_q * (-c.qcoef * (c.theta_I - theta) * pp);
    const Real l_theta = l_q * (c.qcoef * alpha * pp);
    l_phi += l_q * (-c.qcoef * alpha * (c.theta_I - theta)) * ((Real)1 - (Real)2 * phi);
    l_T += l_theta / c.Lcp;
  }
  // alpha
  l_phi += l_alpha * (c.alpha_g - c.alpha_l);
  // T = m0s - 0.5 Lcp (dtphi + D)
  for (int i = 0; i < 9; ++i) li.Ps[i] += l_T;
  l_dtphi += -(Real)0.5 * c.Lcp * l_T;
  l_D += -(Real)0.5 * c.Lcp * l_T;
  // dtphi = phi - phip
  l_phi += l_dtphi;
  li.phip = -l_dtphi;
  // n = gphi r, r = (|g|^2 + eps2)^(-1/2)
  Real l_g[2];
  {
    const Real ln_dot_g = l_n[0] * in.gphi[0] + l_n[1] * in.gphi[1];
    for (int a = 0; a < 2; ++a) l_g[a] = r * l_n[a] - r * r * r * in.gphi[a] * ln_dot_g;
  }
  // grho = drho gphi ; F = mu gphi + (rho - rho_l) g + body
  for (int a = 0; a < 2; ++a) {
    l_g[a] += drho * l_grho[a] + mu * l_F[a];
    l_mu += l_F[a] * in.gphi[a];
    l_rho += l_F[a] * c.grav[a];
  }
  // mu = 4H phi (phi-1)(phi-1/2) - K lphi
  l_phi += l_mu * (Real)4 * c.H * ((Real)3 * phi * phi - (Real)3 * phi + (Real)0.5);
  const Real l_lphi = -c.K * l_mu;
  // rho
  l_phi += l_rho * drho;
  li.phi = l_phi;
  li.gphi[0] = l_g[0];
  li.gphi[1] = l_g[1];
  li.lphi = l_lphi;
  li.u[0] = l_u[0];
  li.u[1] = l_u[1];
  li.D = l_D;
}

// u = (3 m1 + F/2) / rho with m1 = sum f_i c_i and F from phi, grad phi,
// lap phi (Eq. Velocity, Eq. Force_Total with Eq. ChemicalPotential).
template <class Real>
__host__ __device__ inline void u_fwd(const NodeConst<Real>& c, const Real* Pf, Real phi,
                                      const Real* gphi, Real lphi, Real* u) {
  const Real rho = phi * c.rho_g + ((Real)1 - phi) * c.rho_l;
  const Real mu = (Real)4 * c.H * phi * (phi - (Real)1) * (phi - (Real)0.5) - c.K * lphi;
  Real m[2] = {0, 0};
  for (int i = 0; i < 9; ++i) {
    m[0] += (Real)W9::cx(i) * Pf[i];
    m[1] += (Real)W9::cy(i) * Pf[i];
  }
  for (int a = 0; a < 2; ++a) {
    const Real F = mu * gphi[a] + (rho - c.rho_l) * c.grav[a] + c.body[a];
    u[a] = ((Real)3 * m[a] + (Real)0.5 * F) / rho;
  }
}

// Adjoint of u_fwd at a point whose forward velocity u (u_fwd's output) is
// known: the populations enter only through m1, so they are not needed.
// Adds to lPf, and returns adjoints of phi, gphi, lphi.
template <class Real>
__host__ __device__ inline void u_adj_at(const NodeConst<Real>& c, const Real* u, Real phi,
                                         const Real* gphi, Real lphi, const Real* lu, Real* lPf,
                                         Real& l_phi, Real* l_g, Real& l_lphi) {
  const Real rho = phi * c.rho_g + ((Real)1 - phi) * c.rho_l;
  const Real mu = (Real)4 * c.H * phi * (phi - (Real)1) * (phi - (Real)0.5) - c.K * lphi;
  Real l_m[2], l_rho = 0, l_mu = 0;
  for (int a = 0; a < 2; ++a) {
    l_m[a] = (Real)3 * lu[a] / rho;
    const Real l_F = (Real)0.5 * lu[a] / rho;
    l_rho += -lu[a] * u[a] / rho;
    l_mu += l_F * gphi[a];
    l_g[a] = mu * l_F;
    l_rho += l_F * c.grav[a];
  }
  for (int i = 0; i < 9; ++i) lPf[i] += (Real)W9::cx(i) * l_m[0] + (Real)W9::cy(i) * l_m[1];
  l_phi = l_mu * (Real)4 * c.H * ((Real)3 * phi * phi - (Real)3 * phi + (Real)0.5) +
          l_rho * (c.rho_g - c.rho_l);
  l_lphi = -c.K * l_mu;
}

// Adjoint of u_fwd from its inputs.
template <class Real>
__host__ __device__ inline void u_adj(const NodeConst<Real>& c, const Real* Pf, Real phi,
                                      const Real* gphi, Real lphi, const Real* lu, Real* lPf,
                                      Real& l_phi, Real* l_g, Real& l_lphi) {
  Real u[2];
  u_fwd(c, Pf, phi, gphi, lphi, u);
  u_adj_at(c, u, phi, gphi, lphi, lu, lPf, l_phi, l_g, l_lphi);
}

// Initial populations (barred equilibria minus half the source at u = 0,
// d_t phi = 0, D = 0) and the production, as a function of phi, its
// stencils and T.  Outputs the post-streaming values and q.
template <class Real>
__host__ __device__ inline void init_fwd(const NodeConst<Real>& c, Real phi, const Real* gphi,
                                         Real lphi, Real T, NodeOut<Real>& out) {
  NodeIn<Real> in;
  // an init node equals a node map at u = 0, D = 0, phip = phi with
  // populations that are all zero and omega = 1 ... written out instead:
  const Real cs2 = (Real)(1.0 / 3.0);
  const Real rho = phi * c.rho_g + ((Real)1 - phi) * c.rho_l;
  const Real mu = (Real)4 * c.H * phi * (phi - (Real)1) * (phi - (Real)0.5) - c.K * lphi;
  Real F[2], n[2];
  const Real r = (Real)1 / sqrt(gphi[0] * gphi[0] + gphi[1] * gphi[1] + c.eps2);
  for (int a = 0; a < 2; ++a) {
    F[a] = mu * gphi[a] + (rho - c.rho_l) * c.grav[a] + c.body[a];
    n[a] = gphi[a] * r;
  }
  const Real alpha = ((Real)1 - phi) * c.alpha_l + phi * c.alpha_g;
  const Real theta = (T - c.T_sat) / c.Lcp;
  const Real q = c.phase_change
                     ? -c.qcoef * alpha * (c.theta_I - theta) * phi * ((Real)1 - phi)
                     : (Real)0;
  const Real rc = rho * cs2;
  const Real kk = c.four_over_W * phi * ((Real)1 - phi);
  (void)in;
  for (int i = 0; i < 9; ++i) {
    const Real w = (Real)W9::w(i);
    const Real cx = (Real)W9::cx(i), cy = (Real)W9::cy(i);
    const Real S = w * (cx * F[0] + cy * F[1]) + w * rc * q * c.prod_fac;
    out.Af[i] = -(Real)0.5 * S;
    const Real Fg = w * kk * (cx * n[0] + cy * n[1]);
    const Real Pg = w * q;
    out.Ag[i] = c.geq_cac ? phi * w + c.M_over_cs2g * Fg - (Real)0.5 * Pg
                          : phi * w - (Real)0.5 * (Fg + Pg);
    out.As[i] = T * w;
  }
  out.q = q;
}

// Adjoint of init_fwd: adjoints of phi, gphi, lphi, T.
template <class Real>
__host__ __device__ inline void init_adj(const NodeConst<Real>& c, Real phi, const Real* gphi,
                                         Real lphi, Real T, const NodeOut<Real>& lo, Real& l_phi,
                                         Real* l_g, Real& l_lphi, Real& l_T) {
  const Real cs2 = (Real)(1.0 / 3.0);
  const Real rho = phi * c.rho_g + ((Real)1 - phi) * c.rho_l;
  const Real mu = (Real)4 * c.H * phi * (phi - (Real)1) * (phi - (Real)0.5) - c.K * lphi;
  const Real r = (Real)1 / sqrt(gphi[0] * gphi[0] + gphi[1] * gphi[1] + c.eps2);
  Real n[2];
  for (int a = 0; a < 2; ++a) n[a] = gphi[a] * r;
  const Real alpha = ((Real)1 - phi) * c.alpha_l + phi * c.alpha_g;
  const Real theta = (T - c.T_sat) / c.Lcp;
  const Real pp = phi * ((Real)1 - phi);
  const Real q = c.phase_change ? -c.qcoef * alpha * (c.theta_I - theta) * pp : (Real)0;
  const Real rc = rho * cs2;
  const Real kk = c.four_over_W * pp;
  Real l_F[2] = {0, 0}, l_n[2] = {0, 0}, l_rc = 0, l_q = lo.q, l_kk = 0;
  l_phi = 0;
  l_T = 0;
  for (int i = 0; i < 9; ++i) {
    const Real w = (Real)W9::w(i);
    const Real cx = (Real)W9::cx(i), cy = (Real)W9::cy(i);
    // f: -S/2
    const Real l_S = -(Real)0.5 * lo.Af[i];
    l_F[0] += l_S * w * cx;
    l_F[1] += l_S * w * cy;
    l_rc += l_S * w * q * c.prod_fac;
    l_q += l_S * w * rc * c.prod_fac;
    // g
    const Real lA = lo.Ag[i];
    const Real cn = cx * n[0] + cy * n[1];
    l_phi += lA * w;
    const Real l_Fg = c.geq_cac ? lA * c.M_over_cs2g : -(Real)0.5 * lA;
    const Real l_Pg = -(Real)0.5 * lA;
    l_kk += l_Fg * w * cn;
    l_n[0] += l_Fg * w * kk * cx;
    l_n[1] += l_Fg * w * kk * cy;
    l_q += l_Pg * w;
    // s
    l_T += lo.As[i] * w;
  }
  Real l_alpha = 0;
  if (c.phase_change) {
    l_alpha += l_q * (-c.qcoef * (c.theta_I - theta) * pp);
    l_T += l_q * (c.qcoef * alpha * pp) / c.Lcp;
    l_phi += l_q * (-c.qcoef * alpha * (c.theta_I - theta)) * ((Real)1 - (Real)2 * phi);
  }
  l_phi += l_alpha * (c.alpha_g - c.alpha_l);
  l_phi += l_kk * c.four_over_W * ((Real)1 - (Real)2 * phi);
  Real l_rho = cs2 * l_rc, l_mu = 0;
  {
    const Real ln_dot_g = l_n[0] * gphi[0] + l_n[1] * gphi[1];
    for (int a = 0; a < 2; ++a) l_g[a] = r * l_n[a] - r * r * r * gphi[a] * ln_dot_g;
  }
  for (int a = 0; a < 2; ++a) {
    l_g[a] += mu * l_F[a];
    l_mu += l_F[a] * gphi[a];
    l_rho += l_F[a] * c.grav[a];
  }
  l_phi += l_mu * (Real)4 * c.H * ((Real)3 * phi * phi - (Real)3 * phi + (Real)0.5);
  l_lphi = -c.K * l_mu;
  l_phi += l_rho * (c.rho_g - c.rho_l);
}

}  // namespace adj
}  // namespace lbm
