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

#include <type_traits>

namespace lbm {

// ---------------------------------------------------------------------------
// Lattices (Sec. 3).  D2Q9 weights 4/9, 1/9, 1/36; D3Q7 c_s^2 = 1/4 with
// w0 = 1/4, w = 1/8; D3Q19 w0 = 1/3, w = 1/18, 1/36.  Order of D3Q7: rest,
// +x, +y, +z, -x, -y, -z.
// ---------------------------------------------------------------------------
struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
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

// D2Q5: the z-projection of D3Q7 (w0 = 1/2, w = 1/8, c_s^2 = 1/4), for the
// phase-field and heat populations of 2-D runs that cross-check the 3-D path.
// Order: rest, +x, +y, -x, -y.
struct D2Q5 {
  static constexpr int Q = 5;
  static constexpr int D = 2;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[5] = {0, 1, 0, -1, 0};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[5] = {0, 0, 1, 0, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[5] = {0, 3, 4, 1, 2};
    return v[i];
  }
  __host__ __device__ static constexpr double w(int i) { return i == 0 ? 0.5 : 0.125; }
  static constexpr double cs2 = 0.25;
};

struct D3Q7 {
  static constexpr int Q = 7;
  static constexpr int D = 3;
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
  static constexpr int D = 3;
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

// 16-bit storage keeps the s family as deviations from w_i T_ref(x), with
// T_ref(x) the temperature of the node x that stored the population (one
// scalar plane, written with the populations).  A slot (i, x) is always
// encoded and decoded against T_ref(x), so pull and store agree.  The g
// family is kept as deviations from w_i phi(y), with y = x + c_i the node
// that reads slot (i, x) at the next step (x itself where x + c_i lies
// beyond a wall): the writer takes phi(y) from its LDS tile, the reader its
// own phi_prev, which is the same value.  A gather then needs one reference
// per node instead of one per link.
template <class Real, class Store>
constexpr bool kNodeRef = !std::is_same<Real, Store>::value;

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
  int q_gs;                 // populations of the phase-field (and heat) family
  // populations: read A, write B
  const Store* __restrict__ A;
  Store* __restrict__ B;
  const Sc* __restrict__ A_phip;   // phi^{n-1}
  const Sc* __restrict__ A_qp;     // q^{n-1}
  // 16-bit storage: per-node reference of the s family (the node's T when
  // it stored its populations); null for FP32 / FP64
  const Sc* __restrict__ A_Tref;
  Sc* __restrict__ B_Tref;
  Sc* __restrict__ B_phip;
  Sc* __restrict__ B_qp;
  // per-node wall temperature on each walled face: [axis][side]
  const Real* __restrict__ Tw[3][2];
  Real phi_w[3][2];
  // open (pressure) faces of f: pressure anti-bounce-back at p_w.  The
  // gathers apply a wall link of f as f_sg r + w_i f_pw2 without a branch:
  // (1, 0) on a no-slip face, (-1, 2 p_w) on an open one
  int f_open[3][2];
  Real p_w[3][2];
  Real f_sg[3][2], f_pw2[3][2];
  // codec constants per family (f, g, s)
  Real ref[3], scale[3], inv_scale[3];
  // physics
  Real rho_l, rho_g, K, H, four_over_W, eps2;
  Real grav[3], body[3];
  Real nu_l, nu_g, alpha_l, alpha_g;
  Real Lcp, inv_Lcp, T_sat, theta_I, qcoef;   // qcoef = 4 / (A W^2)
  Real omega_g, M_over_cs2g;
  Real prod_fac;          // rho_g (1/rho_g - 1/rho_l): P^f = w rho c_s^2 q prod_fac
  int visc_linear, geq_cac, phase_change, div_local;
  // collision (LBM_COLL_*): TRT magic parameters and MRT free rates per family
  int coll;
  Real lam[3];
  Real mrt[3][4];
  int grad_scheme;        // LBM_GRAD_*
  int nt;                 // launch the non-temporal-store step kernel (state beyond the last-level cache)
  // macro output (MODE_MACRO): planes of nx*ny*nz
  void* out;
  int out_f64;
  uint32_t out_mask;
  double* partials;       // per-block diagnostics partials
};

// Load / store element `idx` (32-bit, non-negative) of a uniform plane
// pointer.  The byte offset is formed in 32 bits and zero-extended so the
// compiler can use the scalar-base + 32-bit vector-offset addressing form
// instead of 64-bit per-lane address arithmetic.
template <class T>
__device__ __forceinline__ T ld_plane(const T* __restrict__ plane, unsigned idx) {
  return *(const T*)((const char*)plane + (size_t)(idx * (unsigned)sizeof(T)));
}
// Store of the step's output: written once and not read again before the
// next step.  NT (chosen per launch: the two state buffers exceed the 256 MiB
// last-level cache): 4- and 8-byte values go out as non-temporal stores,
// which keep them from displacing the halo pulls in L2 (FP32 steps: 1024 x
// 2048 0.105 -> 0.100 ms, 4096 x 3072 0.611 -> 0.571 ms, 256^3 1.456 ->
// 1.385 ms); on grids whose state stays in that cache they would send the
// next step's reads to HBM (512 x 512 FP32 0.0138 -> 0.0173 ms).  16-bit
// values use plain stores (non-temporal 2-byte stores made the FP16 1024 x
// 2048 step 0.092 -> 0.099 ms).  Non-temporal loads of the s family (read
// once) did not help.  A compile-time choice: a run-time branch between the
// two stores is merged by the compiler into one plain store.
template <bool NT, class T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  if constexpr (NT && std::is_arithmetic<T>::value && sizeof(T) >= 4)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
template <bool NT = false, class T>
__device__ __forceinline__ void st_plane(T* __restrict__ plane, unsigned idx, T v) {
  st_stream<NT>((T*)((char*)plane + (size_t)(idx * (unsigned)sizeof(T))), v);
}

// Element `idx` of a family block (all planes of one population family)
// addressed with a 32-bit byte offset; the caller guarantees the family
// block is below 4 GiB.
template <class T>
__device__ __forceinline__ T ld_fam(const T* __restrict__ fam, unsigned idx) {
  return *(const T*)((const char*)fam + (size_t)(idx * (unsigned)sizeof(T)));
}
template <bool NT, class T>
__device__ __forceinline__ void st_fam(T* __restrict__ fam, unsigned idx, T v) {
  st_stream<NT>((T*)((char*)fam + (size_t)(idx * (unsigned)sizeof(T))), v);
}

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

// c_i . v over the lattice's non-zero components only (after unrolling the
// direction loop the components are constants, so zero terms vanish).
template <class Lat, class Real>
__device__ __forceinline__ Real cdot(int i, const Real* v) {
  const int c0 = Lat::cx(i), c1 = Lat::cy(i), c2 = Lat::cz(i);
  Real r = c0 ? (Real)c0 * v[0] : (Real)0;
  if (c1) r = c0 ? r + (Real)c1 * v[1] : (Real)c1 * v[1];
  if (c2) r = (c0 || c1) ? r + (Real)c2 * v[2] : (Real)c2 * v[2];
  return r;
}

template <class Lat, class Real>
__device__ __forceinline__ Real dotD(const Real* a, const Real* b) {
  Real r = a[0] * b[0] + a[1] * b[1];
  if (Lat::D == 3) r += a[2] * b[2];
  return r;
}

// Gamma_i of Eq. FunctionGamma split as w_i + dGamma_i with
// dGamma_i = w_i [cu/c_s^2 + cu^2/(2 c_s^4) - u.u/(2 c_s^2)] computed directly
// (no cancellation against w_i: the deviation carries the flow).
template <class Lat, class Real>
__device__ __forceinline__ Real dgamma_i(int i, const Real* u, Real huu) {
  const Real inv_cs2 = (Real)(1.0 / Lat::cs2);
  const Real h = (Real)(0.5 / (Lat::cs2 * Lat::cs2));
  if (Lat::cx(i) == 0 && Lat::cy(i) == 0 && Lat::cz(i) == 0) return -(Real)Lat::w(i) * huu;
  const Real cu = cdot<Lat>(i, u);
  return (Real)Lat::w(i) * (cu * (inv_cs2 + h * cu) - huu);
}
template <class Lat, class Real>
__device__ __forceinline__ Real gamma_huu(const Real* u) {   // u.u / (2 c_s^2)
  return (Real)(0.5 / Lat::cs2) * dotD<Lat>(u, u);
}
template <class Lat, class Real>
__device__ __forceinline__ Real gamma_i(int i, const Real* u, Real huu) {
  return (Real)Lat::w(i) + dgamma_i<Lat>(i, u, huu);
}

// BGK with the barred equilibrium (Eqs. VariableChange_feq, LBE):
// v - w (v - eq + S/2) + S = (1 - w) v + w eq + (1 - w/2) S.
template <class Real>
struct Relax {
  Real om, om1, om2;
  __device__ __forceinline__ explicit Relax(Real omega)
      : om(omega), om1((Real)1 - omega), om2((Real)1 - (Real)0.5 * omega) {}
  __device__ __forceinline__ Real operator()(Real v, Real eq, Real S) const {
    return fma(om1, v, fma(om, eq, om2 * S));
  }
};

// f family: Eq. Feq_NS_Incompr, S^f = F^f + P^f (Eqs. Forcing, MicroProduction).
// With Gamma_i = w_i + dGamma_i:
//   f^eq_i = w_i p + rho c_s^2 dGamma_i,
//   F^f_i  = dGamma_i X_i + Gamma_i Y_i,
//   X_i = c_s^2 (c_i - u).grad(rho),  Y_i = (c_i - u).F.
template <class Lat, class Real>
__device__ inline void collide_f(Real* f, const NodeMacro<Real>& m, Real prodP, Real omega) {
  const Real cs2 = (Real)Lat::cs2;
  const Real huu = gamma_huu<Lat>(m.u);
  const Real rc = m.rho * cs2;
  const Real ug = cs2 * dotD<Lat>(m.u, m.grho);
  const Real uF = dotD<Lat>(m.u, m.F);
  const Relax<Real> R(omega);
  Real cg2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) cg2[d] = cs2 * m.grho[d];
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const Real w = (Real)Lat::w(i);
    const Real dG = dgamma_i<Lat>(i, m.u, huu);
    const Real X = cdot<Lat>(i, cg2) - ug;
    const Real Y = cdot<Lat>(i, m.F) - uF;
    const Real S = fma(dG, X, (w + dG) * Y) + w * prodP;
    const Real feq = fma(w, m.p, rc * dG);
    f[i] = R(f[i], feq, S);
  }
}

// g family: Eq. Geq_Allen-Cahn_Eq with S^g = F^g + P^g (Eq.
// SourceTerm_AllenCahn), or the CAC equilibrium form (Eq. Geq_AC-1).
template <class Lat, class Real, class A>
__device__ inline void collide_g(const A& a, Real* g, const NodeMacro<Real>& m) {
  const Real huu = gamma_huu<Lat>(m.u);
  const Real k = a.four_over_W * m.phi * ((Real)1 - m.phi);
  Real kn[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) kn[d] = k * m.n[d];
  const Relax<Real> R(a.omega_g);
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const Real w = (Real)Lat::w(i);
    const Real geq = fma(m.phi, dgamma_i<Lat>(i, m.u, huu), m.phi * w);   // phi Gamma_i
    const Real Fg = w * cdot<Lat>(i, kn);
    const Real Pg = w * m.q;
    if (a.geq_cac)
      g[i] = R(g[i], fma(a.M_over_cs2g, Fg, geq), Pg);
    else
      g[i] = R(g[i], geq, Fg + Pg);
  }
}

// s family: Eq. Seq_Temp with S^s_i = -w_i (L/Cp)[d_t phi + div(u phi)].
template <class Lat, class Real, class A>
__device__ inline void collide_s(const A& a, Real* s, const NodeMacro<Real>& m, Real omega) {
  const Real huu = gamma_huu<Lat>(m.u);
  const Real src = -a.Lcp * (m.dtphi + m.D);
  const Relax<Real> R(omega);
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const Real w = (Real)Lat::w(i);
    const Real seq = fma(m.T, dgamma_i<Lat>(i, m.u, huu), m.T * w);   // T Gamma_i
    s[i] = R(s[i], seq, w * src);
  }
}

// ---------------------------------------------------------------------------
// Collision operators of the extended step kernels (Sec. 3: TRT and MRT are
// named after Eq. LBE as the way to reach lower mobility and higher Peclet
// numbers).  All three act on the barred variables: with
// a_i = v_i - eq_i + S_i/2 (non-equilibrium part plus half the source) the
// post-collision value is a_i - Delta_i + eq_i + S_i/2, and
//   BGK: Delta = omega a;
//   TRT: the parts of a symmetric and antisymmetric under c -> -c relax at
//        omega+ and omega-; the transport coefficient keeps the BGK rate
//        (omega+ for the viscosity of f, omega- for the mobility of g and the
//        diffusivity of s) and the other rate follows from the magic
//        parameter Lambda = (1/omega+ - 1/2)(1/omega- - 1/2);
//   MRT: a relaxes in an orthogonal moment basis, moment k at rate r_k
//        (Delta = M^T diag(r_k / |M_k|^2) M a).
// ---------------------------------------------------------------------------
enum { COLL_BGK = 0, COLL_TRT = 1, COLL_MRT = 2 };
enum { GRAD_CENTRAL = 0, GRAD_BIASED1 = 1, GRAD_BIASED2 = 2 };

// Moment bases.  rate(fam, k) selects the rate of moment k for family fam
// (0 f, 1 g, 2 s) from {s_e, s_eps, s_q, s_p, omega}: the transport moments
// take the BGK rate omega (index 4).
template <class Lat>
struct MrtBasis {
  static constexpr bool ok = false;
  __host__ __device__ static constexpr double M(int, int) { return 0.0; }
  __host__ __device__ static constexpr int rate(int, int) { return 4; }
};
// D2Q9 (Lallemand and Luo): 1, e = 3c^2 - 4, eps = 4 - 21c^2/2 + 9c^4/2,
// cx, qx = (3c^2 - 5) cx, cy, qy = (3c^2 - 5) cy, cx^2 - cy^2, cx cy.
template <>
struct MrtBasis<D2Q9> {
  static constexpr bool ok = true;
  __host__ __device__ static constexpr double M(int k, int i) {
    const double cx = D2Q9::cx(i), cy = D2Q9::cy(i), c2 = cx * cx + cy * cy;
    switch (k) {
      case 0: return 1.0;
      case 1: return 3.0 * c2 - 4.0;
      case 2: return 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
      case 3: return cx;
      case 4: return (3.0 * c2 - 5.0) * cx;
      case 5: return cy;
      case 6: return (3.0 * c2 - 5.0) * cy;
      case 7: return cx * cx - cy * cy;
      default: return cx * cy;
    }
  }
  __host__ __device__ static constexpr int rate(int fam, int k) {
    // f: rho, e at s_e; eps at s_eps; j and q at s_q; stress at omega
    // g, s: rho, e at s_e; eps at s_eps; j at omega; q at s_q; pxx, pxy at s_p
    constexpr int rf[9] = {0, 0, 1, 2, 2, 2, 2, 4, 4};
    constexpr int rg[9] = {0, 0, 1, 4, 2, 4, 2, 3, 3};
    return fam == 0 ? rf[k] : rg[k];
  }
};
// D3Q7: 1, cx, cy, cz, 7c^2 - 6, 2cx^2 - cy^2 - cz^2, cy^2 - cz^2 (g and s).
template <>
struct MrtBasis<D3Q7> {
  static constexpr bool ok = true;
  __host__ __device__ static constexpr double M(int k, int i) {
    const double cx = D3Q7::cx(i), cy = D3Q7::cy(i), cz = D3Q7::cz(i);
    const double c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
      case 0: return 1.0;
      case 1: return cx;
      case 2: return cy;
      case 3: return cz;
      case 4: return 7.0 * c2 - 6.0;
      case 5: return 2.0 * cx * cx - cy * cy - cz * cz;
      default: return cy * cy - cz * cz;
    }
  }
  __host__ __device__ static constexpr int rate(int, int k) {
    constexpr int r[7] = {0, 4, 4, 4, 0, 3, 3};
    return r[k];
  }
};
// D2Q5: 1, cx, cy, 5c^2 - 4, cx^2 - cy^2 (g and s).
template <>
struct MrtBasis<D2Q5> {
  static constexpr bool ok = true;
  __host__ __device__ static constexpr double M(int k, int i) {
    const double cx = D2Q5::cx(i), cy = D2Q5::cy(i), c2 = cx * cx + cy * cy;
    switch (k) {
      case 0: return 1.0;
      case 1: return cx;
      case 2: return cy;
      case 3: return 5.0 * c2 - 4.0;
      default: return cx * cx - cy * cy;
    }
  }
  __host__ __device__ static constexpr int rate(int, int k) {
    constexpr int r[5] = {0, 4, 4, 0, 3};
    return r[k];
  }
};
template <class Lat>
__host__ __device__ constexpr double mrt_norm2(int k) {
  double s = 0.0;
  for (int i = 0; i < Lat::Q; ++i) s += MrtBasis<Lat>::M(k, i) * MrtBasis<Lat>::M(k, i);
  return s;
}

// One family's collision in the general form.  eqs(i, eq, S) gives the
// equilibrium and the source of direction i; om is the family's BGK rate.
template <class Lat, int FAM, class Real, class A, class EqS>
__device__ __forceinline__ void relax_general(const A& a, Real om, Real* v, const EqS& eqs) {
  constexpr int Q = Lat::Q;
  Real b[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    Real eq, S;
    eqs(i, eq, S);
    const Real h = (Real)0.5 * S;
    v[i] = v[i] - eq + h;   // a_i
    b[i] = eq + h;
  }
  if (a.coll == COLL_TRT) {
    const Real tau = (Real)1 / om - (Real)0.5;
    const Real oth = (Real)1 / (a.lam[FAM] / tau + (Real)0.5);
    const Real op = FAM == 0 ? om : oth, on = FAM == 0 ? oth : om;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int j = Lat::opp(i);
      if (j < i) continue;
      if (j == i) {
        v[i] = b[i] + ((Real)1 - op) * v[i];
        continue;
      }
      const Real sym = (Real)0.5 * (v[i] + v[j]), anti = (Real)0.5 * (v[i] - v[j]);
      const Real vi = b[i] + v[i] - op * sym - on * anti;
      const Real vj = b[j] + v[j] - op * sym + on * anti;
      v[i] = vi;
      v[j] = vj;
    }
  } else if (a.coll == COLL_MRT) {
    if constexpr (MrtBasis<Lat>::ok) {
      const Real r[5] = {a.mrt[FAM][0], a.mrt[FAM][1], a.mrt[FAM][2], a.mrt[FAM][3], om};
      Real dm[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        Real mk = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const double c = MrtBasis<Lat>::M(k, i);
          if (c != 0.0) mk += (Real)c * v[i];
        }
        dm[k] = r[MrtBasis<Lat>::rate(FAM, k)] * mk * (Real)(1.0 / mrt_norm2<Lat>(k));
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        Real back = 0;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const double c = MrtBasis<Lat>::M(k, i);
          if (c != 0.0) back += (Real)c * dm[k];
        }
        v[i] = b[i] + v[i] - back;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = b[i] + ((Real)1 - om) * v[i];
  }
}

// The three families in the general form.  cproj(i) is c_i . grad(phi) as
// the step's directional-derivative scheme gives it: the projection of the
// Eq. Grad vector (central), or the first- or second-order biased
// directional derivative of Sec. 3.4 along c_i.  It enters the terms of the
// NS source that project grad(phi) on the population's direction:
// c_i . grad(rho) and the surface tension mu c_i . grad(phi) of Eq.
// Forcing.  The phase-field source keeps c_i . n of the Eq. Grad vector:
// its zeroth moment must vanish for phi to stay conserved.
template <class Lat, class Real, class A, class Proj>
__device__ inline void collide_f_ext(const A& a, Real* f, const NodeMacro<Real>& m, Real prodP,
                                     Real om, const Proj& cproj) {
  const Real cs2 = (Real)Lat::cs2;
  const Real huu = gamma_huu<Lat>(m.u);
  const Real rc = m.rho * cs2;
  const Real drho = a.rho_g - a.rho_l;
  const Real ug = cs2 * dotD<Lat>(m.u, m.grho);
  const Real uF = dotD<Lat>(m.u, m.F);
  Real Fn[3];   // buoyancy and body force: F without the surface tension
#pragma unroll
  for (int d = 0; d < 3; ++d) Fn[d] = (m.rho - a.rho_l) * a.grav[d] + a.body[d];
  relax_general<Lat, 0>(a, om, f, [&](int i, Real& eq, Real& S) {
    const Real w = (Real)Lat::w(i);
    const Real dG = dgamma_i<Lat>(i, m.u, huu);
    const Real cp = cproj(i);
    const Real X = cs2 * drho * cp - ug;
    const Real Y = m.mu * cp + cdot<Lat>(i, Fn) - uF;
    S = fma(dG, X, (w + dG) * Y) + w * prodP;
    eq = fma(w, m.p, rc * dG);
  });
}

template <class Lat, class Real, class A>
__device__ inline void collide_g_ext(const A& a, Real* g, const NodeMacro<Real>& m) {
  const Real huu = gamma_huu<Lat>(m.u);
  const Real k = a.four_over_W * m.phi * ((Real)1 - m.phi);
  Real kn[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) kn[d] = k * m.n[d];
  relax_general<Lat, 1>(a, a.omega_g, g, [&](int i, Real& eq, Real& S) {
    const Real w = (Real)Lat::w(i);
    const Real geq = fma(m.phi, dgamma_i<Lat>(i, m.u, huu), m.phi * w);   // phi Gamma_i
    const Real Fg = w * cdot<Lat>(i, kn);
    const Real Pg = w * m.q;
    if (a.geq_cac) {
      eq = fma(a.M_over_cs2g, Fg, geq);
      S = Pg;
    } else {
      eq = geq;
      S = Fg + Pg;
    }
  });
}

template <class Lat, class Real, class A>
__device__ inline void collide_s_ext(const A& a, Real* s, const NodeMacro<Real>& m, Real om) {
  const Real huu = gamma_huu<Lat>(m.u);
  const Real src = -a.Lcp * (m.dtphi + m.D);
  relax_general<Lat, 2>(a, om, s, [&](int i, Real& eq, Real& S) {
    const Real w = (Real)Lat::w(i);
    eq = fma(m.T, dgamma_i<Lat>(i, m.u, huu), m.T * w);   // T Gamma_i
    S = w * src;
  });
}

// c_i . grad(phi) of a lattice direction (cx, cy, cz) for the scheme
// `scheme`: the projection of the Eq. Grad vector g, or the biased
// directional derivatives of Sec. 3.4, phi(x + c) - phi(x) and
// [-phi(x + 2c) + 4 phi(x + c) - 3 phi(x)] / 2, from at(s) = phi(x + s c).
template <class Real, class At>
__device__ __forceinline__ Real dir_deriv(int scheme, int cx, int cy, int cz, const Real* g,
                                          const At& at) {
  if (cx == 0 && cy == 0 && cz == 0) return (Real)0;
  if (scheme == GRAD_CENTRAL) {
    Real r = cx ? (Real)cx * g[0] : (Real)0;
    if (cy) r = cx ? r + (Real)cy * g[1] : (Real)cy * g[1];
    if (cz) r = (cx || cy) ? r + (Real)cz * g[2] : (Real)cz * g[2];
    return r;
  }
  const Real c = at(0), p1 = at(1);
  if (scheme == GRAD_BIASED1) return p1 - c;
  return (Real)0.5 * ((Real)4 * p1 - at(2) - (Real)3 * c);
}

// div(u phi) in the local form (flag LBM_DIV_LOCAL): u . grad(phi) +
// phi div(u), with div(u) = m''' (1/rho_g - 1/rho_l) from Eq.
// ConservMasse_ChgtPhase and the production of the previous step.
template <class Real, class A>
__device__ __forceinline__ Real div_local_term(const A& a, const Real* u, const Real* gphi,
                                               Real phi, Real q_prev) {
  return u[0] * gphi[0] + u[1] * gphi[1] + u[2] * gphi[2] + phi * a.prod_fac * q_prev;
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
