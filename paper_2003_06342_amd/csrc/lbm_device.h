// Device-side building blocks of the phase-change LBM step (gfx950).
//
// Lattices, 16-bit deviation codecs, the kernel argument block and the
// per-node physics (closures, equilibria, sources and BGK collision) shared
// by the 2-D and 3-D fused kernels.  Paper: arXiv 2003.06342, Secs. 2-3.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace lbm {

// ---------------------------------------------------------------------------
// Lattices (Sec. 3).  D2Q9 weights 4/9, 1/9, 1/36; D3Q7 c_s^2 = 1/4 with
// w0 = 1/4, w = 1/8; D3Q19 w0 = 1/3, w = 1/18, 1/36.  Order of D3Q7: rest,
// +x, +y, +z, -x, -y, -z.
// ---------------------------------------------------------------------------
struct D2Q9 {
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return v[i];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  static constexpr double cs2 = 1.0 / 3.0;
};

struct D3Q7 {
  static constexpr int Q = 7;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[7] = {0, 1, 0, 0, -1, 0, 0};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[7] = {0, 0, 1, 0, 0, -1, 0};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int i) {
    constexpr int v[7] = {0, 0, 0, 1, 0, 0, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[7] = {0, 4, 5, 6, 1, 2, 3};
    return v[i];
  }
  __host__ __device__ static constexpr double w(int i) { return i == 0 ? 0.25 : 0.125; }
  static constexpr double cs2 = 0.25;
};

struct D3Q19 {
  static constexpr int Q = 19;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[19] = {0, 1, 0, 0, -1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[19] = {0, 0, 1, 0, 0, -1, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int i) {
    constexpr int v[19] = {0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[19] = {0, 4, 5, 6, 1, 2, 3, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    return v[i];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  static constexpr double cs2 = 1.0 / 3.0;
};

// ---------------------------------------------------------------------------
// Population storage codecs.  Identity for float/double; for 16-bit storage
// h = round_to_nearest_even((v - w_i ref) * 2^k), v = h * 2^-k + w_i ref.
// ---------------------------------------------------------------------------
template <class Real, class Store>
struct Codec {
  __device__ static inline Real dec(Store v, Real, Real) { return (Real)v; }
  __device__ static inline Store enc(Real v, Real, Real) { return (Store)v; }
};
template <>
struct Codec<float, __half> {
  __device__ static inline float dec(__half v, float wref, float inv_scale) {
    return fmaf(__half2float(v), inv_scale, wref);
  }
  __device__ static inline __half enc(float v, float wref, float scale) {
    return __float2half_rn((v - wref) * scale);
  }
};
template <>
struct Codec<float, __hip_bfloat16> {
  __device__ static inline float dec(__hip_bfloat16 v, float wref, float inv_scale) {
    return fmaf(__bfloat162float(v), inv_scale, wref);
  }
  __device__ static inline __hip_bfloat16 enc(float v, float wref, float scale) {
    return __float2bfloat16((v - wref) * scale);
  }
};

// Lagged scalars (phi_prev, q_prev): double for FP64 storage, float otherwise.
template <class Store> struct ScalarOf { using T = float; };
template <> struct ScalarOf<double> { using T = double; };

// ---------------------------------------------------------------------------
// Kernel argument block (passed by value).
// ---------------------------------------------------------------------------
template <class Real, class Store>
struct KArgs {
  using Sc = typename ScalarOf<Store>::T;
  int nx, ny, nz;
  int px;                 // row pitch (elements), multiple of 64
  long long slab;         // px * ny * nz
  int wall[3];            // axis is walled (else periodic)
  int off_f, off_g, off_s;  // first population plane of each family
  // populations: read A, write B
  const Store* __restrict__ A;
  Store* __restrict__ B;
  const Sc* __restrict__ A_phip;   // phi^{n-1}
  const Sc* __restrict__ A_qp;     // q^{n-1}
  Sc* __restrict__ B_phip;
  Sc* __restrict__ B_qp;
  // per-node wall temperature on each walled face: [axis][side]
  const Real* __restrict__ Tw[3][2];
  Real phi_w[3][2];
  // codec constants per family (f, g, s)
  Real ref[3], scale[3], inv_scale[3];
  // physics
  Real rho_l, rho_g, K, H, four_over_W, eps2;
  Real grav[3], body[3];
  Real nu_l, nu_g, alpha_l, alpha_g;
  Real Lcp, inv_Lcp, T_sat, theta_I, qcoef;   // qcoef = 4 / (A W^2)
  Real omega_g, M_over_cs2g;
  Real prod_fac;          // rho_g (1/rho_g - 1/rho_l): P^f = w rho c_s^2 q prod_fac
  int visc_linear, geq_cac, phase_change;
  // macro output (MODE_MACRO): planes of nx*ny*nz
  void* out;
  int out_f64;
  uint32_t out_mask;
  double* partials;       // per-block diagnostics partials
};

__device__ inline int wrap1(int s, int n) {   // s in [-1, n]
  return s < 0 ? s + n : (s >= n ? s - n : s);
}
__device__ inline int wrapmod(int s, int n) {
  int r = s % n;
  return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------
// Per-node physics.  Everything a node needs once its populations are
// gathered, phi and its stencils are known and u is known.
// ---------------------------------------------------------------------------
template <class Real>
struct NodeMacro {
  Real phi, gphi[3], lphi;
  Real rho, mu, F[3], grho[3], n[3];
  Real u[3];
  Real dtphi, D, T, q, p, alpha, nu;
};

// Chemical potential (Eq. ChemicalPotential with Eq. Def_K-H), density
// (Eq. Density), surface tension + buoyancy + body force (Eqs. Force_Total,
// SuperficialTensionForce; buoyancy (rho - rho_l) g).
template <class Real, class A>
__device__ inline void forces(const A& a, Real phi, const Real* gphi, Real lphi, Real& rho,
                              Real& mu, Real* F) {
  rho = phi * a.rho_g + ((Real)1 - phi) * a.rho_l;
  mu = (Real)4 * a.H * phi * (phi - (Real)1) * (phi - (Real)0.5) - a.K * lphi;
  const Real drho = rho - a.rho_l;
#pragma unroll
  for (int d = 0; d < 3; ++d) F[d] = mu * gphi[d] + drho * a.grav[d] + a.body[d];
}

template <class Real>
__device__ inline Real rsqrt_t(Real v) { return (Real)1 / sqrt(v); }
template <>
__device__ inline float rsqrt_t<float>(float v) { return 1.0f / sqrtf(v); }

// Production q = m'''/rho_g (Eq. ProductionRate) with linear alpha(phi).
template <class Real, class A>
__device__ inline Real production(const A& a, Real phi, Real T, Real alpha) {
  if (!a.phase_change) return (Real)0;
  const Real theta = (T - a.T_sat) * a.inv_Lcp;
  return -(a.qcoef * alpha) * (a.theta_I - theta) * phi * ((Real)1 - phi);
}

// Gamma_i of Eq. FunctionGamma.
template <class Lat, class Real>
__device__ inline Real gamma_i(int i, const Real* u, Real uu) {
  const Real inv_cs2 = (Real)(1.0 / Lat::cs2);
  const Real cu = (Real)Lat::cx(i) * u[0] + (Real)Lat::cy(i) * u[1] + (Real)Lat::cz(i) * u[2];
  return (Real)Lat::w(i) *
         ((Real)1 + cu * inv_cs2 + (Real)0.5 * cu * cu * inv_cs2 * inv_cs2 - (Real)0.5 * uu * inv_cs2);
}

// f family: Eq. Feq_NS_Incompr, S^f = F^f + P^f (Eqs. Forcing, MicroProduction),
// collision Eq. LBE with bar-eq = eq - S/2.
template <class Lat, class Real>
__device__ inline void collide_f(Real* f, const NodeMacro<Real>& m, Real prodP, Real omega) {
  const Real cs2 = (Real)Lat::cs2;
  const Real uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const Real w = (Real)Lat::w(i);
    const Real G = gamma_i<Lat>(i, m.u, uu);
    const Real feq = w * m.p + m.rho * cs2 * (G - w);
    const Real c[3] = {(Real)Lat::cx(i), (Real)Lat::cy(i), (Real)Lat::cz(i)};
    Real Ff = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) Ff += (c[d] - m.u[d]) * ((G - w) * cs2 * m.grho[d] + G * m.F[d]);
    const Real S = Ff + w * prodP;
    f[i] = f[i] - omega * (f[i] - feq + (Real)0.5 * S) + S;
  }
}

// g family: Eq. Geq_Allen-Cahn_Eq with S^g = F^g + P^g (Eq.
// SourceTerm_AllenCahn), or the CAC equilibrium form (Eq. Geq_AC-1).
template <class Lat, class Real, class A>
__device__ inline void collide_g(const A& a, Real* g, const NodeMacro<Real>& m) {
  const Real uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
  const Real k = a.four_over_W * m.phi * ((Real)1 - m.phi);
  const Real om = a.omega_g;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const Real w = (Real)Lat::w(i);
    const Real G = gamma_i<Lat>(i, m.u, uu);
    const Real cn = (Real)Lat::cx(i) * m.n[0] + (Real)Lat::cy(i) * m.n[1] + (Real)Lat::cz(i) * m.n[2];
    const Real Fg = k * w * cn;
    const Real Pg = w * m.q;
    if (a.geq_cac) {
      const Real geq = m.phi * G + a.M_over_cs2g * Fg;
      g[i] = g[i] - om * (g[i] - geq + (Real)0.5 * Pg) + Pg;
    } else {
      const Real S = Fg + Pg;
      g[i] = g[i] - om * (g[i] - m.phi * G + (Real)0.5 * S) + S;
    }
  }
}

// s family: Eq. Seq_Temp with S^s_i = -w_i (L/Cp)[d_t phi + div(u phi)].
template <class Lat, class Real, class A>
__device__ inline void collide_s(const A& a, Real* s, const NodeMacro<Real>& m, Real omega) {
  const Real uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
  const Real src = -a.Lcp * (m.dtphi + m.D);
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const Real w = (Real)Lat::w(i);
    const Real G = gamma_i<Lat>(i, m.u, uu);
    const Real S = w * src;
    s[i] = s[i] - omega * (s[i] - m.T * G + (Real)0.5 * S) + S;
  }
}

// Viscosity (Eq. Viscosity / Visco_lin) and diffusivity (linear).
template <class Real, class A>
__device__ inline Real viscosity(const A& a, Real phi) {
  if (a.visc_linear) return ((Real)1 - phi) * a.nu_l + phi * a.nu_g;
  return a.nu_l * a.nu_g / (phi * a.nu_l + ((Real)1 - phi) * a.nu_g);
}
template <class Real, class A>
__device__ inline Real diffusivity(const A& a, Real phi) {
  return ((Real)1 - phi) * a.alpha_l + phi * a.alpha_g;
}

}  // namespace lbm
