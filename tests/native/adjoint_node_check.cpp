// Host check of the hand-written per-node adjoints in lbm_adjoint.h:
// <lambda_out, (fwd(x + e d) - fwd(x - e d)) / 2e> == <adj(lambda_out), d>
// for random inputs, directions and output adjoints (double precision).
#define __host__
#define __device__
#include <cmath>
#include <cstdio>
#include <random>

#include "../../paper_2003_06342_amd/csrc/lbm_adjoint.h"

using namespace lbm::adj;
using R = double;

static std::mt19937_64 rng(12345);
static double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static NodeConst<R> make_const(int cac, int lin, int pc) {
  NodeConst<R> c{};
  c.rho_l = 10; c.rho_g = 1; const double W = 4, sigma = 0.0144;
  c.K = 1.5 * W * sigma; c.H = 12 * sigma / W; c.four_over_W = 4 / W; c.eps2 = 1e-6;
  c.grav[0] = 0; c.grav[1] = -3e-5; c.body[0] = 1e-6; c.body[1] = 0;
  c.nu_l = 0.144; c.nu_g = 0.024; c.alpha_l = 0.012; c.alpha_g = 0.12;
  c.Lcp = 10; c.T_sat = 0; c.theta_I = 0.01; c.qcoef = 4.0 / ((10.0 / 48.0) * W * W);
  c.prod_fac = 1.0 * (1.0 / 1.0 - 1.0 / 10.0);
  c.omega_g = 1.0 / (0.0816 * 3 + 0.5); c.M_over_cs2g = 0.0816 * 3;
  c.visc_linear = lin; c.geq_cac = cac; c.phase_change = pc;
  return c;
}

static void rand_in(NodeIn<R>& in) {
  for (int i = 0; i < 9; ++i) {
    in.Pf[i] = U(-1e-2, 1e-2); in.Pg[i] = U(0, 0.3); in.Ps[i] = U(0, 0.2);
  }
  in.phi = U(0.1, 0.9); in.gphi[0] = U(-0.2, 0.2); in.gphi[1] = U(-0.2, 0.2); in.lphi = U(-0.05, 0.05);
  in.u[0] = U(-1e-2, 1e-2); in.u[1] = U(-1e-2, 1e-2); in.D = U(-1e-3, 1e-3); in.phip = in.phi + U(-1e-3, 1e-3);
}

// flatten NodeIn to a vector view
static const int NIN = 27 + 8;
static R* at(NodeIn<R>& in, int k) {
  if (k < 9) return &in.Pf[k];
  if (k < 18) return &in.Pg[k - 9];
  if (k < 27) return &in.Ps[k - 18];
  switch (k - 27) {
    case 0: return &in.phi; case 1: return &in.gphi[0]; case 2: return &in.gphi[1]; case 3: return &in.lphi;
    case 4: return &in.u[0]; case 5: return &in.u[1]; case 6: return &in.D; default: return &in.phip;
  }
}
static R adj_at(NodeAdjIn<R>& li, int k) {
  if (k < 9) return li.Pf[k];
  if (k < 18) return li.Pg[k - 9];
  if (k < 27) return li.Ps[k - 18];
  switch (k - 27) {
    case 0: return li.phi; case 1: return li.gphi[0]; case 2: return li.gphi[1]; case 3: return li.lphi;
    case 4: return li.u[0]; case 5: return li.u[1]; case 6: return li.D; default: return li.phip;
  }
}
static R dot_out(const NodeOut<R>& a, const NodeOut<R>& b) {
  R s = a.q * b.q;
  for (int i = 0; i < 9; ++i) s += a.Af[i] * b.Af[i] + a.Ag[i] * b.Ag[i] + a.As[i] * b.As[i];
  return s;
}

int main() {
  int fails = 0;
  double worst = 0;
  for (int cfg = 0; cfg < 8; ++cfg) {
    const NodeConst<R> c = make_const(cfg & 1, (cfg >> 1) & 1, (cfg >> 2) & 1 ? 0 : 1);
    for (int trial = 0; trial < 20; ++trial) {
      NodeIn<R> x; rand_in(x);
      NodeOut<R> lo;
      for (int i = 0; i < 9; ++i) { lo.Af[i] = U(-1, 1); lo.Ag[i] = U(-1, 1); lo.As[i] = U(-1, 1); }
      lo.q = U(-1, 1);
      double d[NIN];
      for (int k = 0; k < NIN; ++k) d[k] = U(-1, 1) * (k < 27 ? 1e-2 : (k == 27 || k == 34 ? 0.1 : 0.05));
      // node map
      NodeAdjIn<R> li; node_adj(c, x, lo, li);
      double lhs = 0, rhs = 0;
      for (int k = 0; k < NIN; ++k) rhs += adj_at(li, k) * d[k];
      const double eps = 1e-5;
      NodeIn<R> xp = x, xm = x;
      for (int k = 0; k < NIN; ++k) { *at(xp, k) += eps * d[k]; *at(xm, k) -= eps * d[k]; }
      NodeOut<R> op, om; node_fwd(c, xp, op); node_fwd(c, xm, om);
      NodeOut<R> dd;
      for (int i = 0; i < 9; ++i) { dd.Af[i] = (op.Af[i] - om.Af[i]) / (2 * eps); dd.Ag[i] = (op.Ag[i] - om.Ag[i]) / (2 * eps); dd.As[i] = (op.As[i] - om.As[i]) / (2 * eps); }
      dd.q = (op.q - om.q) / (2 * eps);
      lhs = dot_out(lo, dd);
      double rel = std::fabs(lhs - rhs) / std::fmax(std::fabs(lhs), 1e-12);
      worst = std::fmax(worst, rel);
      if (rel > 1e-6) { ++fails; std::printf("node cfg %d trial %d: fd %.12e adj %.12e rel %.3e\n", cfg, trial, lhs, rhs, rel); }
      // u closure
      R lu[2] = {U(-1, 1), U(-1, 1)};
      R lPf[9] = {0}; R lphi, lg[2], llphi;
      u_adj(c, x.Pf, x.phi, x.gphi, x.lphi, lu, lPf, lphi, lg, llphi);
      double rhs2 = lphi * d[27] + lg[0] * d[28] + lg[1] * d[29] + llphi * d[30];
      for (int i = 0; i < 9; ++i) rhs2 += lPf[i] * d[i];
      R up[2], um[2];
      u_fwd(c, xp.Pf, xp.phi, xp.gphi, xp.lphi, up);
      u_fwd(c, xm.Pf, xm.phi, xm.gphi, xm.lphi, um);
      double lhs2 = lu[0] * (up[0] - um[0]) / (2 * eps) + lu[1] * (up[1] - um[1]) / (2 * eps);
      rel = std::fabs(lhs2 - rhs2) / std::fmax(std::fabs(lhs2), 1e-12);
      worst = std::fmax(worst, rel);
      if (rel > 1e-6) { ++fails; std::printf("u cfg %d trial %d: fd %.12e adj %.12e rel %.3e\n", cfg, trial, lhs2, rhs2, rel); }
      // init map (phi, gphi, lphi, T)
      const R T = U(-0.5, 1.0), dT = U(-0.1, 0.1);
      R l_phi, l_g[2], l_lphi, l_T;
      init_adj(c, x.phi, x.gphi, x.lphi, T, lo, l_phi, l_g, l_lphi, l_T);
      double rhs3 = l_phi * d[27] + l_g[0] * d[28] + l_g[1] * d[29] + l_lphi * d[30] + l_T * dT;
      NodeOut<R> ip, im;
      init_fwd(c, xp.phi, xp.gphi, xp.lphi, T + eps * dT, ip);
      init_fwd(c, xm.phi, xm.gphi, xm.lphi, T - eps * dT, im);
      NodeOut<R> di;
      for (int i = 0; i < 9; ++i) { di.Af[i] = (ip.Af[i] - im.Af[i]) / (2 * eps); di.Ag[i] = (ip.Ag[i] - im.Ag[i]) / (2 * eps); di.As[i] = (ip.As[i] - im.As[i]) / (2 * eps); }
      di.q = (ip.q - im.q) / (2 * eps);
      const double lhs3 = dot_out(lo, di);
      rel = std::fabs(lhs3 - rhs3) / std::fmax(std::fabs(lhs3), 1e-12);
      worst = std::fmax(worst, rel);
      if (rel > 1e-6) { ++fails; std::printf("init cfg %d trial %d: fd %.12e adj %.12e rel %.3e\n", cfg, trial, lhs3, rhs3, rel); }
    }
  }
  std::printf("adjoint node checks: %d failures, worst relative mismatch %.3e\n", fails, worst);
  return fails ? 1 : 0;
}
