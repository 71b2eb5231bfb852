// 3-D fused time step for gfx950: D3Q19 for f, D3Q7 for g and s, D3Q19
// stencils (directional-derivative gradient and Laplacian, Sec. 3.4).
//
// 2.5-D blocking: a workgroup (256 lanes) owns a TX x TY column of nodes (64 x 16
// for the FP32 and 16-bit steps, 32 x 16 otherwise)
// over a chunk of z planes and marches up z with rolling LDS rings:
//   phase 1, plane k+2: phi = sum g_bar + q_prev/2 on the tile + 2-halo
//                       (5-plane ring);
//   phase 2, plane k+1: u (Eq. Velocity) on the tile + 1-halo from the phi
//                       ring and the pulled f (3-plane ring);
//   phase 3, plane k  : moments, div(u phi), production, equilibria,
//                       sources and BGK collision of f, g, s; write B.
// Walls are on z (half-way; bounce-back for f, anti-bounce-back for g, s);
// x and y are periodic.  A ghost plane beyond a wall is computed at its
// mirror plane and transformed (2 phi_w - phi, -u).
#include <type_traits>

#include "lbm_device.h"
#include "lbm_kernels.h"

namespace lbm {

// Tile shape: TX x TY nodes per plane, marching over ZC planes, 256 lanes.
template <int TX_, int TY_, int ZC_>
struct Shape3 {
  static constexpr int TX = TX_, TY = TY_, ZC = ZC_, NT = 256;
  static constexpr int P1X = TX + 4, P1Y = TY + 4;   // phi plane region
  static constexpr int P2X = TX + 2, P2Y = TY + 2;   // u plane region
};
// 32 x 16: FP64 storage, the extended step, and the fields / diagnostics
// pass.  64 x 16 over 32-plane chunks: the FP32 step (256^3 1.32 ms against
// 1.35 on 128 x 8 and 1.77 on 32 x 16; 512^3 10.42 against 10.47 on 128 x
// 8): wider rows than 32 cut the x-halo share of the pulls, and 16 rows
// keep the y halo small.
using ShapeStd3 = Shape3<32, 16, 32>;
using ShapeWide3 = Shape3<64, 16, 32>;
// 64 x 16 over 16-plane chunks: the 16-bit step (512^3 FP16 11.1 against
// 12.2 ms on 32 x 16 and 11.6 on 128 x 8 with 32-plane chunks; 64-column rows
// are whole 128-byte lines of 2-byte values; 16-plane chunks 10.77 against
// 10.92 ms with 32 and 11.08 with 8)
using ShapeMid3 = Shape3<64, 16, 16>;
constexpr int NPHI = 5, NU = 3;

__device__ inline int slot5(int p) { return (p + 10) % NPHI; }
__device__ inline int slot3(int p) { return (p + 9) % NU; }

// Pull the Q populations of family FAM arriving at node (x, y, z); z walls
// reflect at the node (bounce-back f, anti-bounce-back g, s).  XYIN: the
// caller guarantees no x/y source crosses the periodic seam.  A link that
// crosses a z wall (c_z = +1 at z = 0, c_z = -1 at z = nz - 1) reads the
// opposite slot of the node itself; slot and transform are selected, not
// branched on, so the loads of all Q links issue back to back.
// NTL: non-temporal loads (the last read of these populations this step).
template <class Lat, int FAM, bool XYIN, bool NTL = false, class Real, class Store>
__device__ inline void gather3d(const KArgs<Real, Store>& a, int x, int y, int z, Real* v) {
  using C = Codec<Real, Store>;
  const int off = FAM == 0 ? a.off_f : (FAM == 1 ? a.off_g : a.off_s);
  const Real ref = a.ref[FAM], inv = a.inv_scale[FAM];
  const Store* __restrict__ base = a.A + (size_t)off * (size_t)a.slab;
  const int pz = a.px * a.ny;
  const unsigned node = (unsigned)(z * pz + y * a.px + x);
  // 16-bit storage: g is stored as deviations from w_i phi_prev of the node
  // that reads it (one reference per node), s as deviations from w_i T_ref
  // of the node that stored it (one reference per link)
  constexpr bool NREF = FAM == 2 && kNodeRef<Real, Store>;
  constexpr bool GREF = FAM == 1 && kNodeRef<Real, Store>;
  const typename KArgs<Real, Store>::Sc* __restrict__ rplane = a.A_Tref;
  const Real gref = GREF ? (Real)a.A_phip[node] : ref;
  // this plane's wall links (uniform) and the family's wall values
  const bool wlo = a.wall[2] && z == 0, whi = a.wall[2] && z == a.nz - 1;
  Real V[2] = {(Real)0, (Real)0};
  if constexpr (FAM == 1) {
    V[0] = a.phi_w[2][0];
    V[1] = a.phi_w[2][1];
  } else if constexpr (FAM == 2) {
    if (wlo) V[0] = a.Tw[2][0][y * a.nx + x];
    if (whi) V[1] = a.Tw[2][1][y * a.nx + x];
  }
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const int cx = Lat::cx(i), cy = Lat::cy(i), cz = Lat::cz(i);
    const bool oz = cz > 0 ? wlo : (cz < 0 ? whi : false);
    const int side = cz > 0 ? 0 : 1;
    unsigned src;
    if (XYIN) {
      int dz = -cz;
      if (cz != 0 && !a.wall[2]) dz = wrap1(z - cz, a.nz) - z;
      src = (unsigned)((int)node - cx - cy * a.px + dz * pz);
    } else {
      int sx = x - cx, sy = y - cy, sz = z - cz;
      if (cx != 0) sx = wrap1(sx, a.nx);
      if (cy != 0) sy = wrap1(sy, a.ny);
      if (cz != 0 && !a.wall[2]) sz = wrap1(sz, a.nz);
      src = (unsigned)(sz * pz + sy * a.px + sx);
    }
    const int slot = oz ? Lat::opp(i) : i;
    const unsigned at = oz ? node : src;
    const Real wr = NREF ? (Real)Lat::w(i) * (Real)rplane[at] : (Real)Lat::w(i) * gref;
    const Store* sp = &(base + (size_t)slot * (size_t)a.slab)[at];
    Store raw;
    if constexpr (NTL && sizeof(Store) == 2)
      raw = __builtin_bit_cast(Store, __builtin_nontemporal_load((const unsigned short*)sp));
    else if constexpr (NTL)
      raw = __builtin_nontemporal_load(sp);
    else
      raw = *sp;
    const Real r = C::dec(raw, wr, inv);
    Real rw;
    if constexpr (FAM != 0)
      rw = -r + (Real)2 * (Real)Lat::w(i) * V[side];
    else   // bounce-back, or pressure anti-bounce-back on an open face
      rw = a.f_sg[2][side] * r + (Real)Lat::w(i) * a.f_pw2[2][side];
    v[i] = oz ? rw : r;
  }
}

// Output store of the 3-D step: non-temporal (NT) also for 2-byte
// populations, which gain here (512^3 FP16 11.10 -> 10.92 ms), unlike the
// 2-D step's 4-row tiles.
template <bool NT, class T>
__device__ __forceinline__ void st_stream3(T* p, T v) {
  if constexpr (NT && sizeof(T) == 2)
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), (unsigned short*)p);
  else
    st_stream<NT>(p, v);
}
template <class Lat, bool NT = false, class Real, class Store, class RefI>
__device__ inline void store3d_ref(const KArgs<Real, Store>& a, int off, int fam, unsigned node,
                                   const Real* v, const RefI& refi) {
  using C = Codec<Real, Store>;
  Store* __restrict__ base = a.B + (size_t)off * (size_t)a.slab;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    st_stream3<NT>(&(base + (size_t)i * (size_t)a.slab)[node],
                   C::enc(v[i], (Real)Lat::w(i) * refi(i), a.scale[fam]));
}
template <class Lat, bool NT = false, class Real, class Store>
__device__ inline void store3d(const KArgs<Real, Store>& a, int off, int fam, unsigned node,
                               const Real* v, Real ref) {
  using C = Codec<Real, Store>;
  Store* __restrict__ base = a.B + (size_t)off * (size_t)a.slab;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    st_stream3<NT>(&(base + (size_t)i * (size_t)a.slab)[node], C::enc(v[i], (Real)Lat::w(i) * ref, a.scale[fam]));
}

// D3Q19 directional-derivative gradient and Laplacian from the phi ring
// (each direction/opposite pair taken once with weight 2: exact rewrite).
template <class S, class Real>
__device__ inline void stencil3d(const Real (*sphi)[S::P1Y][S::P1X], int p, int ry, int rx, Real* g,
                                 Real& lap) {
  const Real c = sphi[slot5(p)][ry][rx];
  Real gx = 0, gy = 0, gz = 0, l = 0, wsum = 0;
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    if (i > D3Q19::opp(i)) continue;
    const int cx = D3Q19::cx(i), cy = D3Q19::cy(i), cz = D3Q19::cz(i);
    const Real w = (Real)D3Q19::w(i);
    const Real pp = sphi[slot5(p + cz)][ry + cy][rx + cx];
    const Real pm = sphi[slot5(p - cz)][ry - cy][rx - cx];
    if (cx) gx += w * (Real)cx * (pp - pm);
    if (cy) gy += w * (Real)cy * (pp - pm);
    if (cz) gz += w * (Real)cz * (pp - pm);
    l += w * (pp + pm);
    wsum += w;
  }
  g[0] = gx * (Real)3;
  g[1] = gy * (Real)3;
  g[2] = gz * (Real)3;
  lap = (l - (Real)2 * wsum * c) * (Real)6;
}

template <class S, class Real>
__device__ inline Real divergence3d(const Real (*sphi)[S::P1Y][S::P1X],
                                    const Real (*su)[3][S::P2Y][S::P2X],
                                    int p, int ry, int rx) {
  // ry, rx: u-region coordinates of the node; phi region is offset by 1
  Real d = 0;
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    if (i > D3Q19::opp(i)) continue;
    const int cx = D3Q19::cx(i), cy = D3Q19::cy(i), cz = D3Q19::cz(i);
    const Real w = (Real)D3Q19::w(i);
    const Real pp = sphi[slot5(p + cz)][ry + 1 + cy][rx + 1 + cx];
    const Real pm = sphi[slot5(p - cz)][ry + 1 - cy][rx + 1 - cx];
    const int sp = slot3(p + cz), sm = slot3(p - cz);
    if (cx) d += w * (Real)cx * (su[sp][0][ry + cy][rx + cx] * pp - su[sm][0][ry - cy][rx - cx] * pm);
    if (cy) d += w * (Real)cy * (su[sp][1][ry + cy][rx + cx] * pp - su[sm][1][ry - cy][rx - cx] * pm);
    if (cz) d += w * (Real)cz * (su[sp][2][ry + cy][rx + cx] * pp - su[sm][2][ry - cy][rx - cx] * pm);
  }
  return d * (Real)3;
}

__device__ inline int mirror3(int g, int n) { return g < 0 ? -1 - g : 2 * n - 1 - g; }

// Plane index -> (domain plane, ghost?) for z.
__device__ inline int zplane(int p, int nz, int wall, bool& ghost) {
  ghost = false;
  if (wall) {
    if (p < 0 || p >= nz) {
      ghost = true;
      return mirror3(p, nz);
    }
    return p;
  }
  return wrapmod(p, nz);
}

template <class S, class Store, class Real, bool NS, bool HEAT, int MODE, bool XYIN, bool EXT, bool NTS>
__device__ __forceinline__ void march3d(const KArgs<Real, Store>& a, Real (*sphi)[S::P1Y][S::P1X],
                                        Real (*su)[3][S::P2Y][S::P2X], int x0, int y0, int z0, int z1) {
  using Sc = typename ScalarOf<Store>::T;
  const int tid = threadIdx.x;
  const int pz = a.px * a.ny;

  auto phase1 = [&](int p) {
    bool ghost;
    const int zz = zplane(p, a.nz, a.wall[2], ghost);
    const int s = slot5(p);
    const Real pw = ghost ? a.phi_w[2][p < 0 ? 0 : 1] : (Real)0;
    for (int k = tid; k < S::P1X * S::P1Y; k += S::NT) {
      const int ry = k / S::P1X, rx = k - ry * S::P1X;
      int gx = x0 - 2 + rx, gy = y0 - 2 + ry;
      if (!XYIN) {
        gx = wrapmod(gx, a.nx);
        gy = wrapmod(gy, a.ny);
      }
      Real g[7];
      gather3d<D3Q7, 1, XYIN>(a, gx, gy, zz, g);
      Real sum = 0;
#pragma unroll
      for (int i = 0; i < 7; ++i) sum += g[i];
      const Real v = sum + (Real)0.5 * (Real)a.A_qp[(unsigned)(zz * pz + gy * a.px + gx)];
      sphi[s][ry][rx] = ghost ? (Real)2 * pw - v : v;
    }
  };

  auto phase2 = [&](int p) {
    bool ghost;
    const int zz = zplane(p, a.nz, a.wall[2], ghost);
    // a ghost u plane is minus u at the mirror plane, whose phi stencil is in the ring
    const int pm = ghost ? (p < 0 ? -1 - p : 2 * a.nz - 1 - p) : p;
    const int s = slot3(p);
    for (int k = tid; k < S::P2X * S::P2Y; k += S::NT) {
      const int ry = k / S::P2X, rx = k - ry * S::P2X;
      int gx = x0 - 1 + rx, gy = y0 - 1 + ry;
      if (!XYIN) {
        gx = wrapmod(gx, a.nx);
        gy = wrapmod(gy, a.ny);
      }
      Real gphi[3], lphi, rho, mu, F[3];
      stencil3d<S, Real>(sphi, pm, ry + 1, rx + 1, gphi, lphi);
      forces(a, sphi[slot5(pm)][ry + 1][rx + 1], gphi, lphi, rho, mu, F);
      Real f[19];
      gather3d<D3Q19, 0, XYIN>(a, gx, gy, zz, f);
      Real m[3] = {0, 0, 0};
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        if (D3Q19::cx(i)) m[0] += (Real)D3Q19::cx(i) * f[i];
        if (D3Q19::cy(i)) m[1] += (Real)D3Q19::cy(i) * f[i];
        if (D3Q19::cz(i)) m[2] += (Real)D3Q19::cz(i) * f[i];
      }
      const Real ir = (Real)1 / rho;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const Real u = ((Real)3 * m[d] + (Real)0.5 * F[d]) * ir;
        // ghost plane: -u beyond a no-slip face, u beyond an open one
        su[s][d][ry][rx] = (ghost && !a.f_open[2][p < 0 ? 0 : 1]) ? -u : u;
      }
    }
  };

  double acc_phi = 0, acc_T = 0, acc_phip = 0, acc_umax = 0, acc_bad = 0;

  auto phase3 = [&](int k) {
    const int cs = slot5(k);
    (void)cs;
    for (int t = tid; t < S::TX * S::TY; t += S::NT) {
      const int ly = t / S::TX, lx = t - ly * S::TX;
      const int x = x0 + lx, y = y0 + ly, z = k;
      if (x >= a.nx || y >= a.ny) continue;
      const unsigned node = (unsigned)(z * pz + y * a.px + x);
      NodeMacro<Real> m;
      m.phi = sphi[slot5(k)][ly + 2][lx + 2];
      stencil3d<S, Real>(sphi, k, ly + 2, lx + 2, m.gphi, m.lphi);
      forces(a, m.phi, m.gphi, m.lphi, m.rho, m.mu, m.F);
      const Real drho = a.rho_g - a.rho_l;
      const Real inrm = rsqrt_t<Real>(m.gphi[0] * m.gphi[0] + m.gphi[1] * m.gphi[1] +
                                      m.gphi[2] * m.gphi[2] + a.eps2);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        m.grho[d] = drho * m.gphi[d];
        m.n[d] = m.gphi[d] * inrm;
      }
      // c_i . grad(phi) for the extended kernels' sources (central or biased)
      auto cproj = [&](int cx, int cy, int cz) -> Real {
        return dir_deriv<Real>(a.grad_scheme, cx, cy, cz, m.gphi, [&](int st) {
          return sphi[slot5(k + st * cz)][ly + 2 + st * cy][lx + 2 + st * cx];
        });
      };
      (void)cproj;
      m.u[0] = m.u[1] = m.u[2] = 0;
      Real f[19];
      Real m0f = 0;
      if constexpr (NS && HEAT) {
#pragma unroll
        for (int d = 0; d < 3; ++d) m.u[d] = su[slot3(k)][d][ly + 1][lx + 1];
      } else if constexpr (NS) {
        gather3d<D3Q19, 0, XYIN, true>(a, x, y, z, f);   // read once (no phase 2)
        Real mm[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < 19; ++i) {
          m0f += f[i];
          if (D3Q19::cx(i)) mm[0] += (Real)D3Q19::cx(i) * f[i];
          if (D3Q19::cy(i)) mm[1] += (Real)D3Q19::cy(i) * f[i];
          if (D3Q19::cz(i)) mm[2] += (Real)D3Q19::cz(i) * f[i];
        }
        const Real ir = (Real)1 / m.rho;
#pragma unroll
        for (int d = 0; d < 3; ++d) m.u[d] = ((Real)3 * mm[d] + (Real)0.5 * m.F[d]) * ir;
      }
      const Real phip = (Real)a.A_phip[node];
      m.dtphi = m.phi - phip;
      m.alpha = diffusivity(a, m.phi);
      m.D = 0;
      m.T = 0;
      m.q = 0;
      if constexpr (HEAT) {
        Real s[7];
        gather3d<D3Q7, 2, XYIN, true>(a, x, y, z, s);   // s is read once per step
        if constexpr (NS) {
          if constexpr (EXT || MODE == MODE_MACRO) {
            if (a.div_local)
              m.D = div_local_term(a, m.u, m.gphi, m.phi, (Real)a.A_qp[node]);
            else
              m.D = divergence3d<S, Real>(sphi, su, k, ly + 1, lx + 1);
          } else {
            m.D = divergence3d<S, Real>(sphi, su, k, ly + 1, lx + 1);
          }
        }
        Real m0s = 0;
#pragma unroll
        for (int i = 0; i < 7; ++i) m0s += s[i];
        m.T = m0s - (Real)0.5 * a.Lcp * (m.dtphi + m.D);
        m.q = production(a, m.phi, m.T, m.alpha);
        if constexpr (MODE == MODE_STEP) {
          const Real om = (Real)1 / (m.alpha * (Real)4 + (Real)0.5);   // c_s^2 = 1/4
          if constexpr (EXT)
            collide_s_ext<D3Q7>(a, s, m, om);
          else
            collide_s<D3Q7>(a, s, m, om);
          const Real Tref = kNodeRef<Real, Store> ? (Real)(Sc)m.T : a.ref[2];
          store3d<D3Q7, NTS>(a, a.off_s, 2, node, s, Tref);
          if constexpr (kNodeRef<Real, Store>) st_stream<NTS>(&a.B_Tref[node], (Sc)m.T);
        }
      }
      if constexpr (MODE == MODE_STEP) {
        Real g[7];
        gather3d<D3Q7, 1, XYIN, true>(a, x, y, z, g);   // the last read of g this step
        if constexpr (EXT)
          collide_g_ext<D3Q7>(a, g, m);
        else
          collide_g<D3Q7>(a, g, m);
        if constexpr (kNodeRef<Real, Store>) {
          // slot i is read by x + c_i and decoded against that node's phi
          // (in the ring now); beyond a z wall, x reads it back itself
          store3d_ref<D3Q7, NTS>(a, a.off_g, 1, node, g, [&](int i) -> Real {
            const int cx = D3Q7::cx(i), cy = D3Q7::cy(i), cz = D3Q7::cz(i);
            if (cz != 0 && a.wall[2] && (z + cz < 0 || z + cz >= a.nz)) return m.phi;
            return sphi[slot5(k + cz)][ly + 2 + cy][lx + 2 + cx];
          });
        } else {
          store3d<D3Q7, NTS>(a, a.off_g, 1, node, g, a.ref[1]);
        }
      }
      const Real cs2 = (Real)(1.0 / 3.0);
      m.p = 0;
      if constexpr (NS) {
        if constexpr (HEAT) {
          gather3d<D3Q19, 0, XYIN, true>(a, x, y, z, f);   // the last read of f this step
#pragma unroll
          for (int i = 0; i < 19; ++i) m0f += f[i];
        }
        const Real udr = m.u[0] * m.grho[0] + m.u[1] * m.grho[1] + m.u[2] * m.grho[2];
        m.p = m0f + (Real)0.5 * (cs2 * udr + m.rho * cs2 * m.q * a.prod_fac);
        if constexpr (MODE == MODE_STEP) {
          m.nu = viscosity(a, m.phi);
          const Real om = (Real)1 / (m.nu * (Real)3 + (Real)0.5);
          if constexpr (EXT)
            collide_f_ext<D3Q19>(a, f, m, m.rho * cs2 * m.q * a.prod_fac, om, [&](int i) {
              return cproj(D3Q19::cx(i), D3Q19::cy(i), D3Q19::cz(i));
            });
          else
            collide_f<D3Q19>(f, m, m.rho * cs2 * m.q * a.prod_fac, om);
          store3d<D3Q19, NTS>(a, a.off_f, 0, node, f, a.ref[0]);
        }
      }
      if constexpr (MODE == MODE_STEP) {
        st_stream<NTS>(&a.B_phip[node], (Sc)m.phi);
        st_stream<NTS>(&a.B_qp[node], (Sc)m.q);
      } else {
        const long long plane = (long long)a.nx * a.ny * a.nz;
        const long long idx = ((long long)z * a.ny + y) * a.nx + x;
        const Real vals[6] = {m.phi, m.p, m.u[0], m.u[1], m.u[2], m.T};
        int kk = 0;
#pragma unroll
        for (int b = 0; b < 6; ++b) {
          if (a.out_mask & (1u << b)) {
            if (a.out_f64) ((double*)a.out)[kk * plane + idx] = (double)vals[b];
            else ((float*)a.out)[kk * plane + idx] = (float)vals[b];
            ++kk;
          }
        }
        if (a.partials) {
          acc_phi += (double)m.phi;
          acc_T += (double)m.T;
          acc_phip += (double)phip;
          const double um = sqrt((double)m.u[0] * m.u[0] + (double)m.u[1] * m.u[1] +
                                 (double)m.u[2] * m.u[2]);
          acc_umax = fmax(acc_umax, um);
          const bool bad = !(isfinite((double)m.phi) && isfinite((double)m.T) && isfinite(um) &&
                             isfinite((double)m.p));
          acc_bad += bad ? 1.0 : 0.0;
        }
      }
    }
  };

  // prologue: phi planes z0-2 .. z0+1, u planes z0-1 .. z0
  for (int p = z0 - 2; p <= z0 + 1; ++p) phase1(p);
  __syncthreads();
  if constexpr (NS && HEAT) {
    for (int p = z0 - 1; p <= z0; ++p) phase2(p);
    __syncthreads();
  }
  for (int k = z0; k < z1; ++k) {
    phase1(k + 2);
    __syncthreads();
    if constexpr (NS && HEAT) {
      phase2(k + 1);
      __syncthreads();
    }
    phase3(k);
    __syncthreads();
  }
  if constexpr (MODE == MODE_MACRO) {
    if (a.partials) block_partials(acc_phi, acc_T, acc_phip, acc_umax, acc_bad, a.partials);
  }
}

// EXT: the extended step (TRT / MRT collision, biased directional
// derivatives, local div(u phi)), selected at run time from the arguments.
template <class S, class Store, class Real, bool NS, bool HEAT, int MODE, bool EXT, bool NTS>
__global__ __launch_bounds__(S::NT) void k_step3d(const KArgs<Real, Store> a) {
  __shared__ Real sphi[NPHI][S::P1Y][S::P1X];
  __shared__ Real su[NU][3][S::P2Y][S::P2X];
  const int tx = (a.nx + S::TX - 1) / S::TX, ty = (a.ny + S::TY - 1) / S::TY;
  const int zc = (a.nz + S::ZC - 1) / S::ZC;
  const int ntiles = tx * ty * zc;
  int t = blockIdx.x;
  const int full = (ntiles / 8) * 8;
  if (t < full) t = (t % 8) * (full / 8) + t / 8;
  const int ix = t % tx, iy = (t / tx) % ty, iz = t / (tx * ty);
  const int x0 = ix * S::TX, y0 = iy * S::TY, z0 = iz * S::ZC;
  const int z1 = min(z0 + S::ZC, a.nz);
  const bool xyin = x0 >= 3 && x0 + S::TX + 3 <= a.nx && y0 >= 3 && y0 + S::TY + 3 <= a.ny;
  if (xyin)
    march3d<S, Store, Real, NS, HEAT, MODE, true, EXT, NTS>(a, sphi, su, x0, y0, z0, z1);
  else
    march3d<S, Store, Real, NS, HEAT, MODE, false, EXT, NTS>(a, sphi, su, x0, y0, z0, z1);
}

// Initialisation (3-D): equilibrium - S/2 at the initial fields, scattered
// to the pre-image slots of the pull gather.
template <class Store, class Real, bool NS, bool HEAT>
__global__ __launch_bounds__(256) void k_init3d(const KArgs<Real, Store> a, const void* phi0,
                                                const void* T0, const void* u0, const void* p0,
                                                int f64) {
  using C = Codec<Real, Store>;
  using Sc = typename ScalarOf<Store>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.nx || y >= a.ny || z >= a.nz) return;
  const long long plane = (long long)a.nx * a.ny * a.nz;
  auto ld = [&](const void* p, int comp, int xx, int yy, int zz) -> Real {
    const long long i = comp * plane + ((long long)zz * a.ny + yy) * a.nx + xx;
    return f64 ? (Real)((const double*)p)[i] : (Real)((const float*)p)[i];
  };
  auto phi_at = [&](int xx, int yy, int zz) -> Real {
    xx = wrapmod(xx, a.nx);
    yy = wrapmod(yy, a.ny);
    if (a.wall[2] && (zz < 0 || zz >= a.nz))
      return (Real)2 * a.phi_w[2][zz < 0 ? 0 : 1] - ld(phi0, 0, xx, yy, mirror3(zz, a.nz));
    if (!a.wall[2]) zz = wrapmod(zz, a.nz);
    return ld(phi0, 0, xx, yy, zz);
  };
  auto u_at = [&](int c, int xx, int yy, int zz) -> Real {
    if (!u0) return 0;
    xx = wrap1(xx, a.nx);
    yy = wrap1(yy, a.ny);
    if (a.wall[2] && (zz < 0 || zz >= a.nz)) {
      const Real ub = ld(u0, c, xx, yy, mirror3(zz, a.nz));
      return a.f_open[2][zz < 0 ? 0 : 1] ? ub : -ub;
    }
    if (!a.wall[2]) zz = wrap1(zz, a.nz);
    return ld(u0, c, xx, yy, zz);
  };
  NodeMacro<Real> m;
  m.phi = phi_at(x, y, z);
  {
    Real g[3] = {0, 0, 0}, l = 0;
    for (int i = 1; i < 19; ++i) {
      const int cx = D3Q19::cx(i), cy = D3Q19::cy(i), cz = D3Q19::cz(i);
      const Real w = (Real)D3Q19::w(i);
      const Real pp = phi_at(x + cx, y + cy, z + cz), pm = phi_at(x - cx, y - cy, z - cz);
      g[0] += w * (Real)cx * (Real)0.5 * (pp - pm);
      g[1] += w * (Real)cy * (Real)0.5 * (pp - pm);
      g[2] += w * (Real)cz * (Real)0.5 * (pp - pm);
      l += w * (pp - (Real)2 * m.phi + pm);
    }
    for (int d = 0; d < 3; ++d) m.gphi[d] = g[d] * (Real)3;
    m.lphi = l * (Real)3;
  }
  forces(a, m.phi, m.gphi, m.lphi, m.rho, m.mu, m.F);
  const Real inrm = rsqrt_t<Real>(m.gphi[0] * m.gphi[0] + m.gphi[1] * m.gphi[1] +
                                  m.gphi[2] * m.gphi[2] + a.eps2);
  for (int d = 0; d < 3; ++d) {
    m.grho[d] = (a.rho_g - a.rho_l) * m.gphi[d];
    m.n[d] = m.gphi[d] * inrm;
    m.u[d] = NS ? u_at(d, x, y, z) : (Real)0;
  }
  m.dtphi = 0;
  m.D = 0;
  m.alpha = diffusivity(a, m.phi);
  m.T = HEAT ? ld(T0, 0, x, y, z) : (Real)0;
  m.q = HEAT ? production(a, m.phi, m.T, m.alpha) : (Real)0;
  if (HEAT && NS && a.div_local) {
    // the first step's local form sees q_prev = q(phi0, T0)
    m.D = div_local_term(a, m.u, m.gphi, m.phi, m.q);
  } else if (HEAT && NS && u0) {
    Real d = 0;
    for (int i = 1; i < 19; ++i) {
      const int c[3] = {D3Q19::cx(i), D3Q19::cy(i), D3Q19::cz(i)};
      const Real w = (Real)D3Q19::w(i);
      const Real pp = phi_at(x + c[0], y + c[1], z + c[2]), pm = phi_at(x - c[0], y - c[1], z - c[2]);
      for (int k = 0; k < 3; ++k)
        if (c[k])
          d += w * (Real)c[k] * (Real)0.5 *
               (u_at(k, x + c[0], y + c[1], z + c[2]) * pp - u_at(k, x - c[0], y - c[1], z - c[2]) * pm);
    }
    m.D = d * (Real)3;
  }
  m.p = (NS && p0) ? ld(p0, 0, x, y, z) : (Real)0;
  const bool biased = a.grad_scheme != GRAD_CENTRAL;
  // biased schemes: c_i . grad(phi) is the directional derivative along c_i
  auto cproj = [&](int cx, int cy, int cz) -> Real {
    return dir_deriv<Real>(a.grad_scheme, cx, cy, cz, m.gphi, [&](int st) {
      return phi_at(x + st * cx, y + st * cy, z + st * cz);
    });
  };
  const Real cs2 = (Real)(1.0 / 3.0);
  const int pz = a.px * a.ny;
  const Real a0f = gamma_huu<D3Q19>(m.u), a0g = gamma_huu<D3Q7>(m.u);
  // f (D3Q19)
  if (NS) {
    for (int i = 0; i < 19; ++i) {
      const Real w = (Real)D3Q19::w(i);
      const Real G = gamma_i<D3Q19>(i, m.u, a0f);
      const Real c[3] = {(Real)D3Q19::cx(i), (Real)D3Q19::cy(i), (Real)D3Q19::cz(i)};
      Real Ff = 0;
      if (biased) {
        const Real cp = cproj(D3Q19::cx(i), D3Q19::cy(i), D3Q19::cz(i));
        Real ug = 0, uF = 0, cFn = 0;
        const Real drb = m.rho - a.rho_l;
        for (int d = 0; d < 3; ++d) {
          ug += m.u[d] * m.grho[d];
          uF += m.u[d] * m.F[d];
          cFn += c[d] * (drb * a.grav[d] + a.body[d]);
        }
        Ff = (G - w) * (cs2 * (a.rho_g - a.rho_l) * cp - cs2 * ug) + G * (m.mu * cp + cFn - uF);
      } else {
        for (int d = 0; d < 3; ++d) Ff += (c[d] - m.u[d]) * ((G - w) * cs2 * m.grho[d] + G * m.F[d]);
      }
      const Real S = Ff + w * m.rho * cs2 * m.q * a.prod_fac;
      const Real val = w * m.p + m.rho * cs2 * (G - w) - (Real)0.5 * S;
      const int sz = z - D3Q19::cz(i);
      if (a.wall[2] && (sz < 0 || sz >= a.nz)) {
        const unsigned node = (unsigned)(z * pz + y * a.px + x);
        // an open face returns -slot + 2 w_i p_w: its slot holds 2 w_i p_w - f_i
        const int side = sz < 0 ? 0 : 1;
        const Real sv = a.f_open[2][side] ? (Real)2 * w * a.p_w[2][side] - val : val;
        a.B[(size_t)(a.off_f + D3Q19::opp(i)) * a.slab + node] = C::enc(sv, w * a.ref[0], a.scale[0]);
      } else {
        const int sx = wrap1(x - D3Q19::cx(i), a.nx), sy = wrap1(y - D3Q19::cy(i), a.ny);
        const int szz = a.wall[2] ? sz : wrap1(sz, a.nz);
        const unsigned node = (unsigned)(szz * pz + sy * a.px + sx);
        a.B[(size_t)(a.off_f + i) * a.slab + node] = C::enc(val, w * a.ref[0], a.scale[0]);
      }
    }
  }
  // g and s (D3Q7)
  for (int i = 0; i < 7; ++i) {
    const Real w = (Real)D3Q7::w(i);
    const Real G = gamma_i<D3Q7>(i, m.u, a0g);
    const Real cn = (Real)D3Q7::cx(i) * m.n[0] + (Real)D3Q7::cy(i) * m.n[1] + (Real)D3Q7::cz(i) * m.n[2];
    const Real Fg = a.four_over_W * m.phi * ((Real)1 - m.phi) * w * cn;
    const Real Pg = w * m.q;
    const Real gv = a.geq_cac ? m.phi * G + a.M_over_cs2g * Fg - (Real)0.5 * Pg
                              : m.phi * G - (Real)0.5 * (Fg + Pg);
    const Real sv = m.T * G - (Real)0.5 * (w * (-a.Lcp * (m.dtphi + m.D)));
    const int sz = z - D3Q7::cz(i);
    if (a.wall[2] && (sz < 0 || sz >= a.nz)) {
      const int side = sz < 0 ? 0 : 1;
      const unsigned node = (unsigned)(z * pz + y * a.px + x);
      const int j = D3Q7::opp(i);
      const Real gr = kNodeRef<Real, Store> ? (Real)(Sc)m.phi : a.ref[1];   // read by this node
      a.B[(size_t)(a.off_g + j) * a.slab + node] =
          C::enc((Real)2 * w * a.phi_w[2][side] - gv, w * gr, a.scale[1]);
      if (HEAT) {
        const Real tr = kNodeRef<Real, Store> ? (Real)(Sc)m.T : a.ref[2];   // slot at this node
        a.B[(size_t)(a.off_s + j) * a.slab + node] =
            C::enc((Real)2 * w * a.Tw[2][side][y * a.nx + x] - sv, w * tr, a.scale[2]);
      }
    } else {
      const int sx = wrap1(x - D3Q7::cx(i), a.nx), sy = wrap1(y - D3Q7::cy(i), a.ny);
      const int szz = a.wall[2] ? sz : wrap1(sz, a.nz);
      const unsigned node = (unsigned)(szz * pz + sy * a.px + sx);
      // 16-bit storage: the g slot is encoded against the phi of the node
      // that reads it (this one)
      const Real gr = kNodeRef<Real, Store> ? (Real)(Sc)m.phi : a.ref[1];
      a.B[(size_t)(a.off_g + i) * a.slab + node] = C::enc(gv, w * gr, a.scale[1]);
      if (HEAT) {
        // the slot belongs to node (sx, sy, szz): its reference is that node's T0
        const Real tr = kNodeRef<Real, Store> ? (Real)(Sc)ld(T0, 0, sx, sy, szz) : a.ref[2];
        a.B[(size_t)(a.off_s + i) * a.slab + node] = C::enc(sv, w * tr, a.scale[2]);
      }
    }
  }
  const unsigned node = (unsigned)(z * pz + y * a.px + x);
  a.B_phip[node] = (Sc)m.phi;
  a.B_qp[node] = (Sc)m.q;
  if constexpr (kNodeRef<Real, Store>)
    if (HEAT) a.B_Tref[node] = (Sc)m.T;
}

template <class S>
static int blocks3d(int nx, int ny, int nz) {
  return ((nx + S::TX - 1) / S::TX) * ((ny + S::TY - 1) / S::TY) * ((nz + S::ZC - 1) / S::ZC);
}

template <class Store, class Real>
static hipError_t launch_step3d_t(const KArgs<Real, Store>& a, int ns, int heat, int mode,
                                  hipStream_t st) {
  // the FP32 step on the wide shape; everything else (and the fields pass,
  // whose per-block partials are sized by step3d_blocks) on the standard one
  const bool ext = a.coll != COLL_BGK || a.grad_scheme != GRAD_CENTRAL || a.div_local;
  constexpr bool kWide = std::is_same<Store, float>::value;
  constexpr bool kMid = sizeof(Store) == 2;
#define LBM_K(SH, NSV, HV, MV, EV, NTV)                                                        \
  hipLaunchKernelGGL((k_step3d<SH, Store, Real, NSV, HV, MV, EV, NTV>),                         \
                     dim3(blocks3d<SH>(a.nx, a.ny, a.nz)), dim3(SH::NT), 0, st, a)
// the step, default or extended, on the FP32 / 16-bit / FP64 shape with or
// without non-temporal stores (the extended FP64 step with plain stores);
// the fields pass on the standard shape
#define LBM_L(NSV, HV, MV)                                                                   \
  do {                                                                                       \
    if constexpr (MV == MODE_STEP) {                                                         \
      if (ext) {                                                                             \
        if constexpr (kWide) {                                                               \
          if (a.nt) LBM_K(ShapeWide3, NSV, HV, MV, true, true);                              \
          else LBM_K(ShapeWide3, NSV, HV, MV, true, false);                                  \
        } else if constexpr (kMid) {                                                         \
          if (a.nt) LBM_K(ShapeMid3, NSV, HV, MV, true, true);                               \
          else LBM_K(ShapeMid3, NSV, HV, MV, true, false);                                   \
        } else {                                                                             \
          LBM_K(ShapeStd3, NSV, HV, MV, true, false);                                        \
        }                                                                                    \
      } else if constexpr (kWide) {                                                          \
        if (a.nt) LBM_K(ShapeWide3, NSV, HV, MV, false, true);                               \
        else LBM_K(ShapeWide3, NSV, HV, MV, false, false);                                   \
      } else if constexpr (kMid) {                                                           \
        if (a.nt) LBM_K(ShapeMid3, NSV, HV, MV, false, true);                                \
        else LBM_K(ShapeMid3, NSV, HV, MV, false, false);                                    \
      } else {                                                                               \
        if (a.nt) LBM_K(ShapeStd3, NSV, HV, MV, false, true);                                \
        else LBM_K(ShapeStd3, NSV, HV, MV, false, false);                                    \
      }                                                                                      \
    } else {                                                                                 \
      LBM_K(ShapeStd3, NSV, HV, MV, false, false);                                           \
    }                                                                                        \
  } while (0)
  if (mode == MODE_STEP) {
    if (ns && heat) LBM_L(true, true, MODE_STEP);
    else if (ns) LBM_L(true, false, MODE_STEP);
    else if (heat) LBM_L(false, true, MODE_STEP);
    else LBM_L(false, false, MODE_STEP);
  } else {
    if (ns && heat) LBM_L(true, true, MODE_MACRO);
    else if (ns) LBM_L(true, false, MODE_MACRO);
    else if (heat) LBM_L(false, true, MODE_MACRO);
    else LBM_L(false, false, MODE_MACRO);
  }
#undef LBM_L
#undef LBM_K
  return hipGetLastError();
}

template <class Store, class Real>
static hipError_t launch_init3d_t(const KArgs<Real, Store>& a, int ns, int heat, const void* phi0,
                                  const void* T0, const void* u0, const void* p0, int f64,
                                  hipStream_t st) {
  dim3 block(256), grid((a.nx + 255) / 256, a.ny, a.nz);
#define LBM_I(NSV, HV) \
  hipLaunchKernelGGL((k_init3d<Store, Real, NSV, HV>), grid, block, 0, st, a, phi0, T0, u0, p0, f64)
  if (ns && heat) LBM_I(true, true);
  else if (ns) LBM_I(true, false);
  else if (heat) LBM_I(false, true);
  else LBM_I(false, false);
#undef LBM_I
  return hipGetLastError();
}

int step3d_blocks(int nx, int ny, int nz) {
  return blocks3d<ShapeStd3>(nx, ny, nz);
}

#define LBM_INST(STORE, REAL)                                                                 \
  hipError_t launch_step3d(const KArgs<REAL, STORE>& a, int ns, int heat, int mode,           \
                           hipStream_t st) {                                                  \
    return launch_step3d_t<STORE, REAL>(a, ns, heat, mode, st);                               \
  }                                                                                           \
  hipError_t launch_init3d(const KArgs<REAL, STORE>& a, int ns, int heat, const void* phi0,   \
                           const void* T0, const void* u0, const void* p0, int f64,           \
                           hipStream_t st) {                                                  \
    return launch_init3d_t<STORE, REAL>(a, ns, heat, phi0, T0, u0, p0, f64, st);              \
  }
LBM_INST(double, double)
LBM_INST(float, float)
LBM_INST(__half, float)
LBM_INST(__hip_bfloat16, float)
#undef LBM_INST

}  // namespace lbm
