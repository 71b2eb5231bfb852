// 2-D fused time step (D2Q9 for f, g and s; D2Q9 stencils) for gfx950.
//
// One workgroup owns a tile of 64 columns (one wave64 per row) and runs
// three LDS phases per step:
//   1. phi = sum g_bar + q_prev/2 (Eq. Moment_Phi, lagged production) on the
//      tile plus a 2-node halo, pulled straight from buffer A with the wall
//      links applied; stored in LDS.  Wall ghosts 2 phi_w - phi_b.
//   2. u (Eq. Velocity) on the tile plus a 1-node halo: directional-derivative
//      gradient and Laplacian of phi from LDS (Eqs. Grad, Laplacian),
//      chemical potential, forces and the first moment of the pulled f.
//      Stored in LDS.  No-slip ghosts -u_b.
//   3. every tile node: pull s, moments (Eqs. Pressure, Moment_Temp),
//      d_t phi, div(u phi) from LDS, production (Eq. ProductionRate),
//      equilibria, sources, BGK collision; write to buffer B (pull scheme:
//      the next step's gather does the streaming).
// The time step runs one tile node per lane (16 rows on 1024 lanes for FP32,
// 4 rows on 256 lanes for 16-bit and FP64 storage).  Each lane stages its own
// node first in phases 1 and 2 and keeps the g and f it pulled there in
// registers for phase 3, so every population of the tile is read from A
// once; only the halo nodes are pulled again, by the neighbouring tiles,
// mostly from L2.  The halo recomputation keeps every step one kernel with
// no grid-wide synchronisation.  Each population is written once to B.
#include "lbm_device.h"
#include "lbm_kernels.h"
#include "lbm_tile2d.h"

namespace lbm {

// Lanes per workgroup: one tile node per lane for the time step's 4-, 8-
// and 16-row tiles, 512 for the 64-row tiles of the fields pass.
template <int TY>
struct StepTile {
  static constexpr int NT = TY <= 16 ? TX2 * TY : 512;
};

template <class Store, class Real, bool NS, bool HEAT, int MODE, bool FAST, int TY, bool EXT, bool NTS,
          class LG>
__device__ __forceinline__ void step_tile2d(const KArgs<Real, Store>& a, Real (*sphi)[R1X],
                                            Real (*sux)[R2X], Real (*suy)[R2X], int x0, int y0) {
  using C = Codec<Real, Store>;
  using Sc = typename ScalarOf<Store>::T;
  const int tid = threadIdx.x;
  constexpr int NT = StepTile<TY>::NT;
  // the step keeps the g and f that phases 1-2 pulled for the lane's node
  constexpr bool CARRY = MODE == MODE_STEP && NT == TX2 * TY;
  Real gk[LG::Q], fk[9];
  stage2d<Store, Real, NS, HEAT, FAST, TY, NT, CARRY, LG>(a, sphi, sux, suy, x0, y0, gk, fk);

  // ---- phase 3: the tile's nodes ------------------------------------------
  double acc_phi = 0, acc_T = 0, acc_phip = 0, acc_umax = 0, acc_bad = 0;
  const int lx = tid % TX2;
  for (int r = tid / TX2; r < TY; r += NT / TX2) {
    const int x = x0 + lx, y = y0 + r;
    if (x >= a.nx || y >= a.ny) continue;
    const unsigned node = (unsigned)(y * a.px + x);
    NodeMacro<Real> m;
    m.phi = sphi[r + 2][lx + 2];
    stencil2d<Real, R1X>(sphi, r + 2, lx + 2, m.gphi, m.lphi);
    forces(a, m.phi, m.gphi, m.lphi, m.rho, m.mu, m.F);
    const Real drho = a.rho_g - a.rho_l;
    const Real inrm = rsqrt_t<Real>(m.gphi[0] * m.gphi[0] + m.gphi[1] * m.gphi[1] + a.eps2);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      m.grho[d] = drho * m.gphi[d];
      m.n[d] = m.gphi[d] * inrm;
    }
    // c_i . grad(phi) for the extended kernels' sources (central or biased)
    auto cproj = [&](int i) -> Real {
      const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
      return dir_deriv<Real>(a.grad_scheme, cx, cy, 0, m.gphi,
                             [&](int st) { return sphi[r + 2 + st * cy][lx + 2 + st * cx]; });
    };
    (void)cproj;
    m.u[0] = m.u[1] = m.u[2] = 0;
    Real f[9];
    Real m0f = 0;
    if constexpr (NS && HEAT) {
      m.u[0] = sux[r + 1][lx + 1];
      m.u[1] = suy[r + 1][lx + 1];
    } else if constexpr (NS) {
      // without the heat family u is not staged in LDS: take it from the
      // local f before the phase field collides with it
      gather2d<D2Q9, 0, FAST>(a, x, y, f);
      Real mx = 0, my = 0;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        m0f += f[i];
        if (D2Q9::cx(i)) mx += (Real)D2Q9::cx(i) * f[i];
        if (D2Q9::cy(i)) my += (Real)D2Q9::cy(i) * f[i];
      }
      const Real ir = (Real)1 / m.rho;
      m.u[0] = ((Real)3 * mx + (Real)0.5 * m.F[0]) * ir;
      m.u[1] = ((Real)3 * my + (Real)0.5 * m.F[1]) * ir;
    }
    const Real phip = (Real)ld_plane(a.A_phip, node);
    m.dtphi = m.phi - phip;
    m.alpha = diffusivity(a, m.phi);
    m.D = 0;
    m.T = 0;
    m.q = 0;
    // One family live at a time: heat (gives T and q), then phi, then NS
    // (needs q for the pressure moment and the production source).
    if constexpr (HEAT) {
      Real s[LG::Q];
      gather2d<LG, 2, FAST>(a, x, y, s);
      if constexpr (NS) {
        if constexpr (EXT || MODE == MODE_MACRO) {
          if (a.div_local)
            m.D = div_local_term(a, m.u, m.gphi, m.phi, (Real)ld_plane(a.A_qp, node));
          else
            m.D = divergence2d<Real>(sphi, sux, suy, r + 1, lx + 1);
        } else {
          m.D = divergence2d<Real>(sphi, sux, suy, r + 1, lx + 1);
        }
      }
      Real m0s = 0;
#pragma unroll
      for (int i = 0; i < LG::Q; ++i) m0s += s[i];
      m.T = m0s - (Real)0.5 * a.Lcp * (m.dtphi + m.D);
      m.q = production(a, m.phi, m.T, m.alpha);
      if constexpr (MODE == MODE_STEP) {
        const Real om = (Real)1 / (m.alpha * (Real)(1.0 / LG::cs2) + (Real)0.5);   // alpha = tau c_s^2
        if constexpr (EXT)
          collide_s_ext<LG>(a, s, m, om);
        else
          collide_s<LG>(a, s, m, om);
        // 16-bit storage: the s deviations are about this node's own T
        const Real Tref = kNodeRef<Real, Store> ? (Real)(Sc)m.T : a.ref[2];
        store_family<LG, NTS>(a, a.off_s, 2, node, s, Tref);
        if constexpr (kNodeRef<Real, Store>) st_plane<NTS>(a.B_Tref, node, (Sc)m.T);
      }
    }
    if constexpr (MODE == MODE_STEP) {
      Real g[LG::Q];
      if constexpr (CARRY) {
#pragma unroll
        for (int i = 0; i < LG::Q; ++i) g[i] = gk[i];
      } else {
        gather2d<LG, 1, FAST>(a, x, y, g);
      }
      if constexpr (EXT)
        collide_g_ext<LG>(a, g, m);
      else
        collide_g<LG>(a, g, m);
      if constexpr (kNodeRef<Real, Store>) {
        // slot i is read by x + c_i and decoded against that node's phi
        // (its phi_prev next step, in LDS now); where x + c_i lies beyond a
        // wall, x reads the slot back itself
        store_family_ref<LG, NTS>(a, a.off_g, 1, node, g, [&](int i) -> Real {
          const int cx = LG::cx(i), cy = LG::cy(i);
          if (!FAST) {
            const bool out = (cx != 0 && a.wall[0] && (x + cx < 0 || x + cx >= a.nx)) ||
                             (cy != 0 && a.wall[1] && (y + cy < 0 || y + cy >= a.ny));
            if (out) return m.phi;
          }
          return sphi[r + 2 + cy][lx + 2 + cx];
        });
      } else {
        store_family<LG, NTS>(a, a.off_g, 1, node, g, a.ref[1]);
      }
    }
    const Real cs2 = (Real)(1.0 / 3.0);
    m.p = 0;
    if constexpr (NS) {
      if constexpr (HEAT) {
        if constexpr (CARRY) {
#pragma unroll
          for (int i = 0; i < 9; ++i) f[i] = fk[i];
        } else {
          gather2d<D2Q9, 0, FAST>(a, x, y, f);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) m0f += f[i];
      }
      const Real udr = m.u[0] * m.grho[0] + m.u[1] * m.grho[1];
      m.p = m0f + (Real)0.5 * (cs2 * udr + m.rho * cs2 * m.q * a.prod_fac);
      if constexpr (MODE == MODE_STEP) {
        m.nu = viscosity(a, m.phi);
        const Real om = (Real)1 / (m.nu * (Real)3 + (Real)0.5);
        if constexpr (EXT)
          collide_f_ext<D2Q9>(a, f, m, m.rho * cs2 * m.q * a.prod_fac, om, cproj);
        else
          collide_f<D2Q9>(f, m, m.rho * cs2 * m.q * a.prod_fac, om);
        store_family<D2Q9, NTS>(a, a.off_f, 0, node, f, a.ref[0]);
      }
    }
    if constexpr (MODE == MODE_STEP) {
      st_plane<NTS>(a.B_phip, node, (Sc)m.phi);
      st_plane<NTS>(a.B_qp, node, (Sc)m.q);
    } else {
      const long long plane = (long long)a.nx * a.ny * a.nz;
      const long long idx = (long long)y * a.nx + x;
      const Real vals[6] = {m.phi, m.p, m.u[0], m.u[1], (Real)0, m.T};
      int k = 0;
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        if (a.out_mask & (1u << b)) {
          if (a.out_f64)
            ((double*)a.out)[k * plane + idx] = (double)vals[b];
          else
            ((float*)a.out)[k * plane + idx] = (float)vals[b];
          ++k;
        }
      }
      if (a.partials) {
        acc_phi += (double)m.phi;
        acc_T += (double)m.T;
        acc_phip += (double)phip;
        const double um = sqrt((double)m.u[0] * m.u[0] + (double)m.u[1] * m.u[1]);
        acc_umax = fmax(acc_umax, um);
        const bool bad = !(isfinite((double)m.phi) && isfinite((double)m.T) && isfinite(um) &&
                           isfinite((double)m.p));
        acc_bad += bad ? 1.0 : 0.0;
      }
    }
  }
  if constexpr (MODE == MODE_MACRO) {
    if (a.partials) block_partials(acc_phi, acc_T, acc_phip, acc_umax, acc_bad, a.partials);
  }
}

template <class Store, class Real, bool NS, bool HEAT, int MODE, int TY, bool EXT, bool NTS, class LG>
__device__ __forceinline__ void step2d_body(const KArgs<Real, Store>& a) {
  __shared__ Real sphi[Tile2<TY>::R1Y][R1X];
  __shared__ Real sux[Tile2<TY>::R2Y][R2X];
  __shared__ Real suy[Tile2<TY>::R2Y][R2X];
  const int tiles_x = (a.nx + TX2 - 1) / TX2;
  const int ntiles = tiles_x * ((a.ny + TY - 1) / TY);
  // XCD-aware order: hardware deals blocks to the 8 XCDs round-robin.  Each
  // XCD gets one contiguous band of tiles, so neighbouring tiles share an L2;
  // for the 16-row tiles of grids of 32 or more tile columns each XCD takes
  // runs of four tile rows in turn instead (FP32 4096 x 3072: 0.558 against
  // 0.574 ms with bands; 1024 x 2048: 0.104 against 0.097 ms the other way
  // round; the 8-row 16-bit tiles are faster with bands at both sizes).
  int t = blockIdx.x;
  if (TY != 16 || tiles_x < 32) {
    const int full = (ntiles / 8) * 8;
    if (t < full) t = (t % 8) * (full / 8) + t / 8;
  } else {
    const int C = 4 * tiles_x;
    const int full = (ntiles / (8 * C)) * (8 * C);
    if (t < full) {
      const int xcd = t % 8, k = t / 8;
      t = (k / C) * (8 * C) + xcd * C + (k % C);
    }
  }
  const int x0 = (t % tiles_x) * TX2, y0 = (t / tiles_x) * TY;
  // interior tile: every source node of the 2-halo region (3 nodes out)
  // lies inside the domain, so no wall link and no periodic wrap occurs
  const bool interior = x0 >= 3 && x0 + TX2 + 3 <= a.nx && y0 >= 3 && y0 + TY + 3 <= a.ny;
  if (interior)
    step_tile2d<Store, Real, NS, HEAT, MODE, true, TY, EXT, NTS, LG>(a, sphi, sux, suy, x0, y0);
  else
    step_tile2d<Store, Real, NS, HEAT, MODE, false, TY, EXT, NTS, LG>(a, sphi, sux, suy, x0, y0);
}

// EXT: the extended step (TRT / MRT collision, biased directional
// derivatives, local div(u phi)), selected at run time from the arguments;
// the default kernels are BGK with central derivatives.
template <class Store, class Real, bool NS, bool HEAT, int MODE, int TY, bool EXT, bool NTS, class LG>
__global__ __launch_bounds__(StepTile<TY>::NT) void k_step2d(const KArgs<Real, Store> a) {
  step2d_body<Store, Real, NS, HEAT, MODE, TY, EXT, NTS, LG>(a);
}

// 16-bit storage: at most 128 VGPRs (4 waves per SIMD).  The codec constants
// and per-node references pushed the 64-row tile kernel past that (0.200 ->
// 0.136 ms at 1024 x 2048 with the cap); the 8-row carry kernel fits under it.
template <class Store, class Real, bool NS, bool HEAT, int MODE, int TY, bool EXT, bool NTS, class LG>
__global__ __launch_bounds__(StepTile<TY>::NT) __attribute__((amdgpu_waves_per_eu(4))) void k_step2d_w4(
    const KArgs<Real, Store> a) {
  step2d_body<Store, Real, NS, HEAT, MODE, TY, EXT, NTS, LG>(a);
}

// Initialisation: populations = equilibrium - S/2 at the given fields with
// d_t phi = 0 and div(u0 phi0) from u0; written as the pre-image of the pull
// gather (each value goes to the slot the next gather reads it from).
template <class Store, class Real, bool NS, bool HEAT, class LG>
__global__ __launch_bounds__(256) void k_init2d(const KArgs<Real, Store> a, const void* phi0,
                                                const void* T0, const void* u0, const void* p0,
                                                int f64) {
  using C = Codec<Real, Store>;
  using Sc = typename ScalarOf<Store>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  auto ld = [&](const void* p, int plane, int xx, int yy) -> Real {
    const long long i = (long long)plane * a.nx * a.ny + (long long)yy * a.nx + xx;
    return f64 ? (Real)((const double*)p)[i] : (Real)((const float*)p)[i];
  };
  // phi with Dirichlet ghosts, u with no-slip ghosts (x ghost then y ghost)
  auto phi_at = [&](int xx, int yy) -> Real {
    Real sgn = 1, add = 0;
    if (a.wall[1] && (yy < 0 || yy >= a.ny)) {
      add = (Real)2 * a.phi_w[1][yy < 0 ? 0 : 1];
      sgn = -1;
      yy = mirror(yy, a.ny);
    } else if (!a.wall[1]) yy = wrapmod(yy, a.ny);
    Real v;
    if (a.wall[0] && (xx < 0 || xx >= a.nx)) {
      v = (Real)2 * a.phi_w[0][xx < 0 ? 0 : 1] - ld(phi0, 0, mirror(xx, a.nx), yy);
    } else {
      if (!a.wall[0]) xx = wrapmod(xx, a.nx);
      v = ld(phi0, 0, xx, yy);
    }
    return add + sgn * v;
  };
  // u ghost: -u_b beyond a no-slip face, u_b beyond an open face of f
  auto u_at = [&](int comp, int xx, int yy) -> Real {
    if (!u0) return 0;
    Real sgn = 1;
    if (a.wall[1] && (yy < 0 || yy >= a.ny)) {
      if (!a.f_open[1][yy < 0 ? 0 : 1]) sgn = -sgn;
      yy = mirror(yy, a.ny);
    } else if (!a.wall[1]) yy = wrap1(yy, a.ny);
    if (a.wall[0] && (xx < 0 || xx >= a.nx)) {
      if (!a.f_open[0][xx < 0 ? 0 : 1]) sgn = -sgn;
      xx = mirror(xx, a.nx);
    } else if (!a.wall[0]) xx = wrap1(xx, a.nx);
    return sgn * ld(u0, comp, xx, yy);
  };
  Real P[3][3];
  for (int j = -1; j <= 1; ++j)
    for (int i = -1; i <= 1; ++i) P[j + 1][i + 1] = phi_at(x + i, y + j);
  NodeMacro<Real> m;
  m.phi = P[1][1];
  {
    Real gx = 0, gy = 0, l = 0;
    for (int i = 1; i < 9; ++i) {
      const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
      const Real w = (Real)D2Q9::w(i);
      const Real p = P[1 + cy][1 + cx], mm = P[1 - cy][1 - cx];
      gx += w * (Real)cx * (Real)0.5 * (p - mm);
      gy += w * (Real)cy * (Real)0.5 * (p - mm);
      l += w * (p - (Real)2 * m.phi + mm);
    }
    m.gphi[0] = gx * (Real)3;
    m.gphi[1] = gy * (Real)3;
    m.gphi[2] = 0;
    m.lphi = l * (Real)3;
  }
  forces(a, m.phi, m.gphi, m.lphi, m.rho, m.mu, m.F);
  const Real inrm = rsqrt_t<Real>(m.gphi[0] * m.gphi[0] + m.gphi[1] * m.gphi[1] + a.eps2);
  for (int d = 0; d < 3; ++d) {
    m.grho[d] = (a.rho_g - a.rho_l) * m.gphi[d];
    m.n[d] = m.gphi[d] * inrm;
  }
  m.u[0] = NS ? u_at(0, x, y) : (Real)0;
  m.u[1] = NS ? u_at(1, x, y) : (Real)0;
  m.u[2] = 0;
  m.dtphi = 0;
  m.D = 0;
  m.alpha = diffusivity(a, m.phi);
  m.T = HEAT ? ld(T0, 0, x, y) : (Real)0;
  m.q = HEAT ? production(a, m.phi, m.T, m.alpha) : (Real)0;
  if (HEAT && NS && a.div_local) {
    // the first step's local form sees q_prev = q(phi0, T0)
    m.D = div_local_term(a, m.u, m.gphi, m.phi, m.q);
  } else if (HEAT && NS && u0) {
    Real d = 0;
    for (int i = 1; i < 9; ++i) {
      const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
      const Real w = (Real)D2Q9::w(i);
      const Real pp = phi_at(x + cx, y + cy), pm = phi_at(x - cx, y - cy);
      if (cx) d += w * (Real)cx * (Real)0.5 * (u_at(0, x + cx, y + cy) * pp - u_at(0, x - cx, y - cy) * pm);
      if (cy) d += w * (Real)cy * (Real)0.5 * (u_at(1, x + cx, y + cy) * pp - u_at(1, x - cx, y - cy) * pm);
    }
    m.D = d * (Real)3;
  }
  m.p = (NS && p0) ? ld(p0, 0, x, y) : (Real)0;
  const Real cs2 = (Real)(1.0 / 3.0);
  // populations = eq - S/2, written out: f on D2Q9, g and s on LG
  Real f[9], g[LG::Q], s[LG::Q];
  const bool biased = a.grad_scheme != GRAD_CENTRAL;
  if (NS) {
    const Real a0 = gamma_huu<D2Q9>(m.u);
    for (int i = 0; i < 9; ++i) {
      const Real w = (Real)D2Q9::w(i);
      const Real G = gamma_i<D2Q9>(i, m.u, a0);
      const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
      const Real c[3] = {(Real)cx, (Real)cy, (Real)0};
      Real Ff = 0;
      if (biased) {
        // biased schemes: c_i . grad(phi) of the NS source is the
        // directional derivative along c_i
        const Real cp = dir_deriv<Real>(a.grad_scheme, cx, cy, 0, m.gphi,
                                        [&](int st) { return phi_at(x + st * cx, y + st * cy); });
        const Real ug = cs2 * (m.u[0] * m.grho[0] + m.u[1] * m.grho[1]);
        const Real uF = m.u[0] * m.F[0] + m.u[1] * m.F[1];
        const Real drb = m.rho - a.rho_l;
        const Real cFn = c[0] * (drb * a.grav[0] + a.body[0]) + c[1] * (drb * a.grav[1] + a.body[1]);
        Ff = (G - w) * (cs2 * (a.rho_g - a.rho_l) * cp - ug) + G * (m.mu * cp + cFn - uF);
      } else {
        for (int d = 0; d < 3; ++d) Ff += (c[d] - m.u[d]) * ((G - w) * cs2 * m.grho[d] + G * m.F[d]);
      }
      const Real S = Ff + w * m.rho * cs2 * m.q * a.prod_fac;
      f[i] = w * m.p + m.rho * cs2 * (G - w) - (Real)0.5 * S;
    }
  }
  {
    const Real a0 = gamma_huu<LG>(m.u);
    for (int i = 0; i < LG::Q; ++i) {
      const Real w = (Real)LG::w(i);
      const Real G = gamma_i<LG>(i, m.u, a0);
      const Real cn = (Real)LG::cx(i) * m.n[0] + (Real)LG::cy(i) * m.n[1];
      const Real Fg = a.four_over_W * m.phi * ((Real)1 - m.phi) * w * cn;
      const Real Pg = w * m.q;
      g[i] = a.geq_cac ? m.phi * G + a.M_over_cs2g * Fg - (Real)0.5 * Pg
                       : m.phi * G - (Real)0.5 * (Fg + Pg);
      if (HEAT) s[i] = m.T * G - (Real)0.5 * (w * (-a.Lcp * (m.dtphi + m.D)));
    }
  }
  // scatter to the pre-image slots: slot i of node x - c_i, or at a wall link
  // slot i' of node x itself (it is read back reflected)
  auto scatter = [&](auto lat, int fam, const Real* v) {
    using L = decltype(lat);
    const int off = fam == 0 ? a.off_f : (fam == 1 ? a.off_g : a.off_s);
    for (int i = 0; i < L::Q; ++i) {
      const int cx = L::cx(i), cy = L::cy(i);
      int sx = x - cx, sy = y - cy;
      const bool oy = cy != 0 && a.wall[1] && (sy < 0 || sy >= a.ny);
      const bool ox = cx != 0 && !oy && a.wall[0] && (sx < 0 || sx >= a.nx);
      const Real w = (Real)L::w(i);
      if (oy || ox) {
        const long long node = (long long)y * a.px + x;
        const int ax = oy ? 1 : 0;
        const int side = oy ? (sy < 0 ? 0 : 1) : (sx < 0 ? 0 : 1);
        Real val, ref;
        if (fam == 0) {
          // bounce-back returns the slot as is; an open face returns
          // -slot + 2 w_i p_w, so its slot holds 2 w_i p_w - f_i
          val = a.f_open[ax][side] ? (Real)2 * w * a.p_w[ax][side] - v[i] : v[i];
          ref = a.ref[0];
        } else if (fam == 1) {
          val = (Real)2 * w * a.phi_w[ax][side] - v[i];
          ref = kNodeRef<Real, Store> ? (Real)(Sc)m.phi : a.ref[1];   // read by this node
        } else {
          val = (Real)2 * w * (oy ? a.Tw[1][side][x] : a.Tw[0][side][y]) - v[i];
          ref = kNodeRef<Real, Store> ? (Real)(Sc)m.T : a.ref[2];     // slot at this node
        }
        a.B[(long long)(off + L::opp(i)) * a.slab + node] = C::enc(val, w * ref, a.scale[fam]);
      } else {
        if (!a.wall[0]) sx = wrap1(sx, a.nx);
        if (!a.wall[1]) sy = wrap1(sy, a.ny);
        const long long node = (long long)sy * a.px + sx;
        // 16-bit storage: a g slot is encoded against the phi of the node
        // that reads it (this one), an s slot against the T0 of the node
        // that owns it, (sx, sy)
        const Real ref = fam == 0 ? a.ref[0]
                                  : (kNodeRef<Real, Store>
                                         ? (fam == 1 ? (Real)(Sc)m.phi : (Real)(Sc)ld(T0, 0, sx, sy))
                                         : a.ref[fam]);
        a.B[(long long)(off + i) * a.slab + node] = C::enc(v[i], w * ref, a.scale[fam]);
      }
    }
  };
  if (NS) scatter(D2Q9{}, 0, f);
  scatter(LG{}, 1, g);
  if (HEAT) scatter(LG{}, 2, s);
  const long long node = (long long)y * a.px + x;
  a.B_phip[node] = (Sc)m.phi;
  a.B_qp[node] = (Sc)m.q;
  if constexpr (kNodeRef<Real, Store>)
    if (HEAT) a.B_Tref[node] = (Sc)m.T;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class Store, class Real>
static hipError_t launch_step2d_t(const KArgs<Real, Store>& a, int ns, int heat, int mode,
                                  hipStream_t st) {
  // MODE_MACRO always uses 64-row tiles: its per-block partials are sized by
  // step2d_blocks.  The step runs one tile node per lane: 16 rows (1024
  // lanes) for FP32, 8 rows (512 lanes) for 16-bit storage and 4 rows (256
  // lanes) for FP64 storage, whose kernel holds more registers.  Measured at
  // 1024 x 2048: FP32 0.108 ms (0.120 with 4 rows, 0.110 with 8); FP64 0.204
  // (0.228 with 8).  FP16, with the g reference per reading node: 0.0748 ms
  // (0.0774 with 4 rows, 0.0838 with 16), 512 x 512 0.0136 (0.0153 with 4).
  // At 512 x 512 FP32 0.016 ms (0.018 with 4 rows).
  constexpr bool st16 = sizeof(Store) == 2;
  constexpr bool small_tiles = st16 || sizeof(Store) == 8;
  const int ty = mode != MODE_STEP ? 64 : (st16 ? 8 : (small_tiles ? 4 : 16));
  const int tiles = ((a.nx + TX2 - 1) / TX2) * ((a.ny + ty - 1) / ty);
  // D2Q5 phase-field and heat populations run the extended kernels
  const bool d2q5 = a.q_gs == 5;
  const bool ext = a.coll != COLL_BGK || a.grad_scheme != GRAD_CENTRAL || a.div_local || d2q5;
#define LBM_K(NSV, HV, MV, TYV, EV, NTV, LGV)                                                   \
  do {                                                                                          \
    if constexpr (st16)                                                                         \
      hipLaunchKernelGGL((k_step2d_w4<Store, Real, NSV, HV, MV, TYV, EV, NTV, LGV>), dim3(tiles), \
                         dim3(StepTile<TYV>::NT), 0, st, a);                                    \
    else                                                                                        \
      hipLaunchKernelGGL((k_step2d<Store, Real, NSV, HV, MV, TYV, EV, NTV, LGV>), dim3(tiles),  \
                         dim3(StepTile<TYV>::NT), 0, st, a);                                    \
  } while (0)
// the default and the extended step with or without non-temporal stores;
// the extended step on D2Q5 phase-field and heat populations with plain
// stores
#define LBM_L(NSV, HV, MV, TYV)                                      \
  do {                                                               \
    if (ext && d2q5) LBM_K(NSV, HV, MV, TYV, true, false, D2Q5);     \
    else if (ext && a.nt) LBM_K(NSV, HV, MV, TYV, true, true, D2Q9); \
    else if (ext) LBM_K(NSV, HV, MV, TYV, true, false, D2Q9);        \
    else if (a.nt) LBM_K(NSV, HV, MV, TYV, false, true, D2Q9);  \
    else LBM_K(NSV, HV, MV, TYV, false, false, D2Q9);           \
  } while (0)
#define LBM_L2(NSV, HV, MV)                            \
  if constexpr (st16) LBM_L(NSV, HV, MV, 8);              \
  else if constexpr (small_tiles) LBM_L(NSV, HV, MV, 4);  \
  else LBM_L(NSV, HV, MV, 16)
#define LBM_M(NSV, HV)                                                \
  do {                                                                \
    if (d2q5) LBM_K(NSV, HV, MODE_MACRO, 64, false, false, D2Q5);     \
    else LBM_K(NSV, HV, MODE_MACRO, 64, false, false, D2Q9);          \
  } while (0)
  if (mode == MODE_STEP) {
    if (ns && heat) { LBM_L2(true, true, MODE_STEP); }
    else if (ns) { LBM_L2(true, false, MODE_STEP); }
    else if (heat) { LBM_L2(false, true, MODE_STEP); }
    else { LBM_L2(false, false, MODE_STEP); }
  } else {
    // the fields pass takes the local div(u phi) at run time
    if (ns && heat) LBM_M(true, true);
    else if (ns) LBM_M(true, false);
    else if (heat) LBM_M(false, true);
    else LBM_M(false, false);
  }
#undef LBM_M
#undef LBM_L2
#undef LBM_L
#undef LBM_K
  return hipGetLastError();
}

template <class Store, class Real>
static hipError_t launch_init2d_t(const KArgs<Real, Store>& a, int ns, int heat, const void* phi0,
                                  const void* T0, const void* u0, const void* p0, int f64,
                                  hipStream_t st) {
  dim3 block(256), grid((a.nx + 255) / 256, a.ny);
#define LBM_I(NSV, HV)                                                                          \
  do {                                                                                          \
    if (a.q_gs == 5)                                                                            \
      hipLaunchKernelGGL((k_init2d<Store, Real, NSV, HV, D2Q5>), grid, block, 0, st, a, phi0, T0, \
                         u0, p0, f64);                                                          \
    else                                                                                        \
      hipLaunchKernelGGL((k_init2d<Store, Real, NSV, HV, D2Q9>), grid, block, 0, st, a, phi0, T0, \
                         u0, p0, f64);                                                          \
  } while (0)
  if (ns && heat) LBM_I(true, true);
  else if (ns) LBM_I(true, false);
  else if (heat) LBM_I(false, true);
  else LBM_I(false, false);
#undef LBM_I
  return hipGetLastError();
}

int step2d_blocks(int nx, int ny) { return ((nx + TX2 - 1) / TX2) * ((ny + TY2 - 1) / TY2); }

#define LBM_INST(STORE, REAL)                                                                 \
  hipError_t launch_step2d(const KArgs<REAL, STORE>& a, int ns, int heat, int mode,           \
                           hipStream_t st) {                                                  \
    return launch_step2d_t<STORE, REAL>(a, ns, heat, mode, st);                               \
  }                                                                                           \
  hipError_t launch_init2d(const KArgs<REAL, STORE>& a, int ns, int heat, const void* phi0,   \
                           const void* T0, const void* u0, const void* p0, int f64,           \
                           hipStream_t st) {                                                  \
    return launch_init2d_t<STORE, REAL>(a, ns, heat, phi0, T0, u0, p0, f64, st);              \
  }
LBM_INST(double, double)
LBM_INST(float, float)
LBM_INST(__half, float)
LBM_INST(__hip_bfloat16, float)
#undef LBM_INST

}  // namespace lbm
