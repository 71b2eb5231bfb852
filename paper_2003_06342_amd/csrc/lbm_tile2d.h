// 2-D tile machinery shared by the forward step and its adjoint: pulls with
// wall links, the directional-derivative stencils, div(u phi), and the
// LDS staging of phi (tile + 2-halo) and u (tile + 1-halo).
#pragma once

#include "lbm_device.h"

namespace lbm {

// Tiles are 64 columns wide (one wave64 per row) and TY rows high.  Tile2
// gives the default lane count (512 for 64 rows, else 256); the time step
// runs one tile node per lane (4 or 16 rows) and the fields pass 64 rows;
// the adjoint's local kernel uses 8 rows on 256 lanes.
constexpr int TX2 = 64, TY2 = 64, NT2 = 512;
constexpr int R1X = TX2 + 4, R1Y = TY2 + 4;   // phi region (halo 2)
constexpr int R2X = TX2 + 2, R2Y = TY2 + 2;   // u region (halo 1)
template <int TY>
struct Tile2 {
  static constexpr int NT = TY >= 64 ? 512 : 256;
  static constexpr int R1Y = TY + 4, R2Y = TY + 2;
};

// Pull the Q populations of family FAM (0 f, 1 g, 2 s) arriving at node
// (x, y).  A link whose source lies beyond a wall reflects at the node:
// bounce-back for f, anti-bounce-back -v_{i'} + 2 w_i V_w for g and s
// (Sec. 3.3).  The y wall takes precedence over the x wall at corners.
// FAST: the caller guarantees that no source node of this tile lies beyond
// a wall or across a periodic seam, so every pull is the uniform plane
// pointer shifted by -(c_x + c_y px) and indexed by the node's lane offset.
// BRANCH (the adjoint's local kernel, which runs only with no-slip faces of
// f): each wall link branches to its reflected read; f links bounce back.
template <class Lat, int FAM, bool FAST = false, bool BRANCH = false, class Real, class Store>
__device__ inline void gather2d(const KArgs<Real, Store>& a, int x, int y, Real* v) {
  using C = Codec<Real, Store>;
  const int off = FAM == 0 ? a.off_f : (FAM == 1 ? a.off_g : a.off_s);
  const Real ref = a.ref[FAM], inv = a.inv_scale[FAM];
  // uniform plane base (scalar registers) + 32-bit lane offset
  const Store* __restrict__ base = a.A + (size_t)off * (size_t)a.slab;
  const unsigned node = (unsigned)(y * a.px + x);
  // 16-bit storage: g is stored as deviations from w_i phi_prev of the node
  // that reads it (one reference per node), s as deviations from w_i T_ref
  // of the node that stored it (one reference per link)
  constexpr bool NREF = FAM == 2 && kNodeRef<Real, Store>;
  constexpr bool GREF = FAM == 1 && kNodeRef<Real, Store>;
  const typename KArgs<Real, Store>::Sc* __restrict__ rplane = a.A_Tref;
  const Real gref = GREF ? (Real)ld_plane(a.A_phip, node) : ref;
  if constexpr (FAST) {
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
      const unsigned src = node - (unsigned)(Lat::cx(i) + Lat::cy(i) * a.px);
      const unsigned sl = (unsigned)i * (unsigned)a.slab - (unsigned)(Lat::cx(i) + Lat::cy(i) * a.px);
      const Real r = NREF ? (Real)ld_plane(rplane, src) : gref;
      v[i] = C::dec(ld_fam(base, node + sl), (Real)Lat::w(i) * r, inv);
    }
    return;
  }
  if constexpr (BRANCH) {
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
      const int cx = Lat::cx(i), cy = Lat::cy(i);
      int sx = x - cx, sy = y - cy;
      const bool oy = (cy != 0) && a.wall[1] && (sy < 0 || sy >= a.ny);
      const bool ox = (cx != 0) && !oy && a.wall[0] && (sx < 0 || sx >= a.nx);
      if (oy || ox) {
        const Real wr = NREF ? (Real)Lat::w(i) * (Real)ld_plane(rplane, node) : (Real)Lat::w(i) * gref;
        Real r = C::dec(ld_fam(base, (unsigned)Lat::opp(i) * (unsigned)a.slab + node), wr, inv);
        if (FAM != 0) {
          const int side = oy ? (sy < 0 ? 0 : 1) : (sx < 0 ? 0 : 1);
          const Real V = FAM == 1 ? (oy ? a.phi_w[1][side] : a.phi_w[0][side])
                                  : (oy ? a.Tw[1][side][x] : a.Tw[0][side][y]);
          r = -r + (Real)2 * (Real)Lat::w(i) * V;
        }
        v[i] = r;
      } else {
        if (cx != 0 && !a.wall[0]) sx = wrap1(sx, a.nx);
        if (cy != 0 && !a.wall[1]) sy = wrap1(sy, a.ny);
        const unsigned src = (unsigned)(sy * a.px + sx);
        const Real wr = NREF ? (Real)Lat::w(i) * (Real)ld_plane(rplane, src) : (Real)Lat::w(i) * gref;
        v[i] = C::dec(ld_fam(base, (unsigned)i * (unsigned)a.slab + src), wr, inv);
      }
    }
    return;
  }
  // wall values of the node's links: only a node next to a wall has any
  // (per-node wall temperatures are loaded once here, not per link)
  Real Vy[2] = {(Real)0, (Real)0}, Vx[2] = {(Real)0, (Real)0};
  if constexpr (FAM == 1) {
    Vy[0] = a.phi_w[1][0];
    Vy[1] = a.phi_w[1][1];
    Vx[0] = a.phi_w[0][0];
    Vx[1] = a.phi_w[0][1];
  } else if constexpr (FAM == 2) {
    if (a.wall[1]) {
      if (y == 0) Vy[0] = a.Tw[1][0][x];
      if (y == a.ny - 1) Vy[1] = a.Tw[1][1][x];
    }
    if (a.wall[0]) {
      if (x == 0) Vx[0] = a.Tw[0][0][y];
      if (x == a.nx - 1) Vx[1] = a.Tw[0][1][y];
    }
  }
  // a wall link reads the opposite slot of the node itself; slot, address and
  // transform are selected, not branched on, so the Q loads issue together
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const int cx = Lat::cx(i), cy = Lat::cy(i);
    int sx = x - cx, sy = y - cy;
    const bool oy = (cy != 0) && a.wall[1] && (sy < 0 || sy >= a.ny);
    const bool ox = (cx != 0) && !oy && a.wall[0] && (sx < 0 || sx >= a.nx);
    const bool o = oy || ox;
    if (cx != 0 && !a.wall[0]) sx = wrap1(sx, a.nx);
    if (cy != 0 && !a.wall[1]) sy = wrap1(sy, a.ny);
    const unsigned at = o ? node : (unsigned)(sy * a.px + sx);
    const int slot = o ? Lat::opp(i) : i;
    const Real wr = NREF ? (Real)Lat::w(i) * (Real)ld_plane(rplane, at) : (Real)Lat::w(i) * gref;
    const Real r = C::dec(ld_fam(base, (unsigned)slot * (unsigned)a.slab + at), wr, inv);
    // the crossed face: y (precedence at corners) or x, side from the sign of c
    const int ys = cy > 0 ? 0 : 1, xs = cx > 0 ? 0 : 1;
    Real rw;
    if constexpr (FAM != 0) {
      rw = -r + (Real)2 * (Real)Lat::w(i) * (oy ? Vy[ys] : Vx[xs]);
    } else {   // bounce-back, or pressure anti-bounce-back on an open face
      const Real sg = oy ? a.f_sg[1][ys] : a.f_sg[0][xs];
      const Real pw2 = oy ? a.f_pw2[1][ys] : a.f_pw2[0][xs];
      rw = sg * r + (Real)Lat::w(i) * pw2;
    }
    v[i] = o ? rw : r;
  }
}

// Store the Q post-collision populations of one family at `node` of B, slot
// i encoded against w_i refi(i).
template <class Lat, bool NT = false, class Real, class Store, class RefI>
__device__ inline void store_family_ref(const KArgs<Real, Store>& a, int off, int fam, unsigned node,
                                        const Real* v, const RefI& refi) {
  using C = Codec<Real, Store>;
  Store* __restrict__ base = a.B + (size_t)off * (size_t)a.slab;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    st_fam<NT>(base, (unsigned)i * (unsigned)a.slab + node,
               C::enc(v[i], (Real)Lat::w(i) * refi(i), a.scale[fam]));
}

// Store the Q post-collision populations of one family at `node` of B.
// ref: the deviation reference (the family's global one, or the node's
// T_ref for the s family in 16-bit storage).
template <class Lat, bool NT = false, class Real, class Store>
__device__ inline void store_family(const KArgs<Real, Store>& a, int off, int fam, unsigned node,
                                    const Real* v, Real ref) {
  using C = Codec<Real, Store>;
  Store* __restrict__ base = a.B + (size_t)off * (size_t)a.slab;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    st_fam<NT>(base, (unsigned)i * (unsigned)a.slab + node,
               C::enc(v[i], (Real)Lat::w(i) * ref, a.scale[fam]));
}

// Directional-derivative gradient and Laplacian (Eqs. DerivDirec_Grad, Grad,
// DerivDirect_Laplacian, Laplacian) of a field read through at(dy, dx), the
// value at offset (dx, dy) from the centre.  The sums run over the D2Q9
// directions; a direction and its opposite contribute the same term, so each
// pair is taken once with weight 2 (exact rewrite).
template <class Real, class At>
__device__ __forceinline__ void stencil2d_at(const At& at, Real* g, Real& lap) {
  const Real c = at(0, 0);
  Real gx = 0, gy = 0, l = 0, wsum = 0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    if (i > D2Q9::opp(i)) continue;
    const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
    const Real w = (Real)D2Q9::w(i);
    const Real p = at(cy, cx), m = at(-cy, -cx);
    if (cx) gx += w * (Real)cx * (p - m);
    if (cy) gy += w * (Real)cy * (p - m);
    l += w * (p + m);
    wsum += w;
  }
  g[0] = gx * (Real)3;   // 1/c_s^2
  g[1] = gy * (Real)3;
  g[2] = 0;
  lap = (l - (Real)2 * wsum * c) * (Real)6;
}

template <class Real, int RX>
__device__ __forceinline__ void stencil2d(const Real (*s)[RX], int ry, int rx, Real* g, Real& lap) {
  stencil2d_at<Real>([&](int dy, int dx) { return s[ry + dy][rx + dx]; }, g, lap);
}

// div(u phi): the Eq. Grad stencil applied to u_a phi, a-th component,
// summed; phi(dy, dx), ux(dy, dx), uy(dy, dx) read at offsets from the node.
template <class Real, class P, class UX, class UY>
__device__ __forceinline__ Real divergence2d_at(const P& phi, const UX& ux, const UY& uy) {
  Real d = 0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    if (i > D2Q9::opp(i)) continue;
    const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
    const Real w = (Real)D2Q9::w(i);
    const Real pp = phi(cy, cx), pm = phi(-cy, -cx);
    if (cx != 0) d += w * (Real)cx * (ux(cy, cx) * pp - ux(-cy, -cx) * pm);
    if (cy != 0) d += w * (Real)cy * (uy(cy, cx) * pp - uy(-cy, -cx) * pm);
  }
  return d * (Real)3;
}

template <class Real>
__device__ __forceinline__ Real divergence2d(const Real (*sphi)[R1X], const Real (*sux)[R2X],
                                             const Real (*suy)[R2X], int ry2, int rx2) {
  return divergence2d_at<Real>(
      [&](int dy, int dx) { return sphi[ry2 + 1 + dy][rx2 + 1 + dx]; },
      [&](int dy, int dx) { return sux[ry2 + dy][rx2 + dx]; },
      [&](int dy, int dx) { return suy[ry2 + dy][rx2 + dx]; });
}

// Map a region coordinate to the domain: wraps periodic axes; returns false
// for points beyond a wall (ghosts).
__device__ inline bool to_domain(int& g, int n, int wall) {
  if (wall) return g >= 0 && g < n;
  g = wrapmod(g, n);
  return true;
}

// Mirror of a ghost coordinate across the half-way wall (-1 <-> 0, n <-> n-1).
__device__ inline int mirror(int g, int n) { return g < 0 ? -1 - g : 2 * n - 1 - g; }

// The halo of a region: halo1_rc enumerates the phi region (tile + 2) minus
// the tile, halo2_rc the u region (tile + 1) minus the tile: the rows above
// and below first, then the side columns of the tile rows.
template <int TY>
__device__ __forceinline__ void halo1_rc(int h, int& ry, int& rx) {
  if (h < 2 * R1X) {
    ry = h / R1X;
    rx = h - ry * R1X;
    return;
  }
  h -= 2 * R1X;
  if (h < 2 * R1X) {
    ry = TY + 2 + h / R1X;
    rx = h % R1X;
    return;
  }
  h -= 2 * R1X;
  ry = 2 + (h >> 2);
  const int c = h & 3;
  rx = c < 2 ? c : TX2 + c;
}
template <int TY>
__device__ __forceinline__ void halo2_rc(int h, int& ry, int& rx) {
  if (h < 2 * R2X) {
    ry = h < R2X ? 0 : TY + 1;
    rx = h < R2X ? h : h - R2X;
    return;
  }
  h -= 2 * R2X;
  ry = 1 + (h >> 1);
  rx = (h & 1) ? R2X - 1 : 0;
}

// Stage phi on the tile + 2-halo and (NS && HEAT) u on the tile + 1-halo in
// LDS, with wall ghosts (x ghosts first, then y ghosts, so corners compose).
// NT lanes.  CARRY (NT == TX2 * TY, one tile node per lane): each phase
// stages the lane's own node first and returns the g it pulled for phi in
// gk and the f it pulled for u in fk, so the node update does not pull them
// again; the halo nodes follow.
template <class Store, class Real, bool NS, bool HEAT, bool FAST, int TY = TY2,
          int NT = Tile2<TY>::NT, bool CARRY = false, class LG = D2Q9>
__device__ __forceinline__ void stage2d(const KArgs<Real, Store>& a, Real (*sphi)[R1X],
                                        Real (*sux)[R2X], Real (*suy)[R2X], int x0, int y0,
                                        Real* gk = nullptr, Real* fk = nullptr) {
  static_assert(!CARRY || NT == TX2 * TY, "CARRY needs one tile node per lane");
  const int tid = threadIdx.x;
  // ---- phase 1: phi on the tile + 2-halo --------------------------------
  auto phi_node = [&](int ry, int rx, Real* g) {
    int gx = x0 - 2 + rx, gy = y0 - 2 + ry;
    Real v = 0;
    if (FAST || (to_domain(gx, a.nx, a.wall[0]) && to_domain(gy, a.ny, a.wall[1]))) {
      gather2d<LG, 1, FAST>(a, gx, gy, g);
      Real s = 0;
#pragma unroll
      for (int i = 0; i < LG::Q; ++i) s += g[i];
      v = s + (Real)0.5 * (Real)ld_plane(a.A_qp, (unsigned)(gy * a.px + gx));
    }
    sphi[ry][rx] = v;
  };
  if constexpr (CARRY) {
    phi_node(tid / TX2 + 2, tid % TX2 + 2, gk);
    for (int h = tid; h < R1X * Tile2<TY>::R1Y - TX2 * TY; h += NT) {
      int ry, rx;
      halo1_rc<TY>(h, ry, rx);
      Real g[LG::Q];
      phi_node(ry, rx, g);
    }
  } else {
    for (int k = tid; k < R1X * Tile2<TY>::R1Y; k += NT) {
      const int ry = k / R1X, rx = k - ry * R1X;
      Real g[LG::Q];
      phi_node(ry, rx, g);
    }
  }
  __syncthreads();
  if (!FAST && a.wall[0]) {   // x ghosts first, then y ghosts (corners compose)
    for (int k = tid; k < R1X * Tile2<TY>::R1Y; k += NT) {
      const int ry = k / R1X, rx = k - ry * R1X;
      const int gx = x0 - 2 + rx;
      if (gx < 0 || gx >= a.nx) {
        const int mx = mirror(gx, a.nx) - (x0 - 2);
        if (mx >= 0 && mx < R1X) sphi[ry][rx] = (Real)2 * a.phi_w[0][gx < 0 ? 0 : 1] - sphi[ry][mx];
      }
    }
    __syncthreads();
  }
  if (!FAST && a.wall[1]) {
    for (int k = tid; k < R1X * Tile2<TY>::R1Y; k += NT) {
      const int ry = k / R1X, rx = k - ry * R1X;
      const int gy = y0 - 2 + ry;
      if (gy < 0 || gy >= a.ny) {
        const int my = mirror(gy, a.ny) - (y0 - 2);
        if (my >= 0 && my < Tile2<TY>::R1Y) sphi[ry][rx] = (Real)2 * a.phi_w[1][gy < 0 ? 0 : 1] - sphi[my][rx];
      }
    }
    __syncthreads();
  }

  // ---- phase 2: u on the tile + 1-halo -----------------------------------
  if constexpr (NS && HEAT) {
    auto u_node = [&](int ry, int rx, Real* f) {
      int gx = x0 - 1 + rx, gy = y0 - 1 + ry;
      Real ux = 0, uy = 0;
      if (FAST || (to_domain(gx, a.nx, a.wall[0]) && to_domain(gy, a.ny, a.wall[1]))) {
        Real gphi[3], lphi, rho, mu, F[3];
        stencil2d<Real, R1X>(sphi, ry + 1, rx + 1, gphi, lphi);
        forces(a, sphi[ry + 1][rx + 1], gphi, lphi, rho, mu, F);
        gather2d<D2Q9, 0, FAST>(a, gx, gy, f);
        Real mx = 0, my = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          if (D2Q9::cx(i)) mx += (Real)D2Q9::cx(i) * f[i];
          if (D2Q9::cy(i)) my += (Real)D2Q9::cy(i) * f[i];
        }
        const Real ir = (Real)1 / rho;
        ux = ((Real)3 * mx + (Real)0.5 * F[0]) * ir;
        uy = ((Real)3 * my + (Real)0.5 * F[1]) * ir;
      }
      sux[ry][rx] = ux;
      suy[ry][rx] = uy;
    };
    if constexpr (CARRY) {
      u_node(tid / TX2 + 1, tid % TX2 + 1, fk);
      for (int h = tid; h < R2X * Tile2<TY>::R2Y - TX2 * TY; h += NT) {
        int ry, rx;
        halo2_rc<TY>(h, ry, rx);
        Real f[9];
        u_node(ry, rx, f);
      }
    } else {
      for (int k = tid; k < R2X * Tile2<TY>::R2Y; k += NT) {
        const int ry = k / R2X, rx = k - ry * R2X;
        Real f[9];
        u_node(ry, rx, f);
      }
    }
    __syncthreads();
    if (!FAST && a.wall[0]) {
      for (int k = tid; k < R2X * Tile2<TY>::R2Y; k += NT) {
        const int ry = k / R2X, rx = k - ry * R2X;
        const int gx = x0 - 1 + rx;
        if (gx < 0 || gx >= a.nx) {
          const int mx = mirror(gx, a.nx) - (x0 - 1);
          // no-slip ghost -u_b; open face u_b (zero normal gradient)
          const Real sg = a.f_open[0][gx < 0 ? 0 : 1] ? (Real)1 : (Real)-1;
          if (mx >= 0 && mx < R2X) {
            sux[ry][rx] = sg * sux[ry][mx];
            suy[ry][rx] = sg * suy[ry][mx];
          }
        }
      }
      __syncthreads();
    }
    if (!FAST && a.wall[1]) {
      for (int k = tid; k < R2X * Tile2<TY>::R2Y; k += NT) {
        const int ry = k / R2X, rx = k - ry * R2X;
        const int gy = y0 - 1 + ry;
        if (gy < 0 || gy >= a.ny) {
          const int my = mirror(gy, a.ny) - (y0 - 1);
          const Real sg = a.f_open[1][gy < 0 ? 0 : 1] ? (Real)1 : (Real)-1;
          if (my >= 0 && my < Tile2<TY>::R2Y) {
            sux[ry][rx] = sg * sux[my][rx];
            suy[ry][rx] = sg * suy[my][rx];
          }
        }
      }
      __syncthreads();
    }
  }

}

}  // namespace lbm
