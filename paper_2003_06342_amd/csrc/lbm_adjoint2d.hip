// Adjoint of the 2-D (D2Q9 x 3) fused step, for gradients of a loss of the
// final phase field with respect to the initial phase field and the wall
// temperature (reverse-mode differentiation written by hand; FP32 or FP64).
//
// Forward step n maps the stored state X^n = (A: post-collision populations,
// phi_prev, q_prev) to X^{n+1}.  With lambda = dL/dX, one adjoint step is
//   K_A  local:   recompute phi, u (LDS, as the forward) and the node inputs,
//                 apply node_adj: adjoints of the pulled populations P, of
//                 phi, grad phi, lap phi, u, D at the node; lambda_phi_prev.
//   K_BC, in one tiled kernel:
//     u / D:      transpose of D = div(u phi) (gradient stencil, no-slip and
//                 Dirichlet ghosts), then the adjoint of the velocity closure
//                 (on the tile plus a 1-node halo, totals staged in LDS);
//     phi:        transposed gradient (antisymmetric) and Laplacian
//                 (symmetric) stencils with Dirichlet ghosts; phi = sum g +
//                 q_prev/2 distributes lambda_phi to the pulled g and q_prev.
// The transpose of the pull gather is folded into these kernels: each slot
// of A is read by exactly one pull, so the adjoint of a pulled population is
// stored (K_A) or accumulated (K_BC, for f and g) straight into the slot it
// was read from, in a second buffer that becomes lambda_A of the earlier
// state; anti-bounce-back links of s add 2 w_i lambda to the wall-temperature
// gradient (K_A).  K_C alone (the phi transpose from node fields in memory)
// serves the initial-condition step.  The seed (a loss of phi^N and T^N)
// is a local kernel of its own followed by K_BC.
// Supports at most one walled axis (ghost corners are not differentiated).
#include "lbm_adjoint.h"
#include "lbm_adjargs.h"
#include "lbm_device.h"
#include "lbm_kernels.h"
#include "lbm_tile2d.h"

namespace lbm {

template <class Real>
__device__ inline Real ldp(const Real* p, long long slab, int plane, unsigned node) {
  return p[(size_t)plane * (size_t)slab + node];
}

// Periodic wrap of a coordinate at most two nodes outside [0, n) (the
// stencils here reach x +- 1 around ghost positions x = -1 and x = n), by
// compares instead of an integer division.
__device__ __forceinline__ int wrap2(int s, int n) {
  s += s < 0 ? n : 0;
  s += s < 0 ? n : 0;
  s -= s >= n ? n : 0;
  s -= s >= n ? n : 0;
  return s;
}

// Global-memory phi with Dirichlet ghosts (one walled axis at most).
template <class Real, class Store>
__device__ inline Real phi_g(const KArgs<Real, Store>& a, const Real* fphi, int x, int y) {
  if (a.wall[1] && (y < 0 || y >= a.ny))
    return (Real)2 * a.phi_w[1][y < 0 ? 0 : 1] - fphi[(unsigned)(mirror(y, a.ny) * a.px + wrap2(x, a.nx))];
  if (a.wall[0] && (x < 0 || x >= a.nx))
    return (Real)2 * a.phi_w[0][x < 0 ? 0 : 1] - fphi[(unsigned)(wrap2(y, a.ny) * a.px + mirror(x, a.nx))];
  return fphi[(unsigned)(wrap2(y, a.ny) * a.px + wrap2(x, a.nx))];
}

// A node-valued adjoint field read at (x, y): 0 beyond a wall (no stencil is
// evaluated at ghost nodes), periodic wrap otherwise.
template <class Real, class Store>
__device__ inline Real lfield(const KArgs<Real, Store>& a, const Real* f, int x, int y) {
  if (a.wall[1] && (y < 0 || y >= a.ny)) return 0;
  if (a.wall[0] && (x < 0 || x >= a.nx)) return 0;
  return f[(unsigned)(wrap2(y, a.ny) * a.px + wrap2(x, a.nx))];
}

// Slot of A read by the pull of population i of family fam at node (x, y),
// with the sign of that read (-1 on the anti-bounce-back links of g and s)
// and, for a link reflected at a wall, the wall (axis, side); wax = -1 else.
template <class Real, class Store>
__device__ inline size_t pull_slot(const KArgs<Real, Store>& a, int fam, int i, int x, int y,
                                   Real& sign, int& wax, int& wside) {
  const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
  int sx = x - cx, sy = y - cy;
  const bool oy = cy != 0 && a.wall[1] && (sy < 0 || sy >= a.ny);
  const bool ox = cx != 0 && !oy && a.wall[0] && (sx < 0 || sx >= a.nx);
  wax = -1;
  wside = 0;
  if (oy || ox) {
    sign = fam == 0 ? (Real)1 : (Real)-1;
    wax = oy ? 1 : 0;
    wside = oy ? (sy < 0 ? 0 : 1) : (sx < 0 ? 0 : 1);
    return (size_t)(fam * 9 + D2Q9::opp(i)) * (size_t)a.slab + (unsigned)(y * a.px + x);
  }
  if (!a.wall[0]) sx = wrap1(sx, a.nx);
  if (!a.wall[1]) sy = wrap1(sy, a.ny);
  sign = 1;
  return (size_t)(fam * 9 + i) * (size_t)a.slab + (unsigned)(sy * a.px + sx);
}

// ---------------------------------------------------------------------------
// K_A: local adjoint
// ---------------------------------------------------------------------------
// node_adj keeps the node's inputs, output adjoints and input adjoints live
// together (about 256 VGPRs); two waves per SIMD is the most it reaches
// without heavy spilling.
template <class Real, int TY>
__global__ __launch_bounds__(Tile2<TY>::NT) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_local2d(const KArgs<Real, Real> a,
                                                              const AdjArgs<Real> b) {
  __shared__ Real sphi[Tile2<TY>::R1Y][R1X];
  __shared__ Real sux[Tile2<TY>::R2Y][R2X];
  __shared__ Real suy[Tile2<TY>::R2Y][R2X];
  const int tiles_x = (a.nx + TX2 - 1) / TX2;
  const int t = blockIdx.x;
  const int x0 = (t % tiles_x) * TX2, y0 = (t / tiles_x) * TY;
  stage2d<Real, Real, true, true, false, TY>(a, sphi, sux, suy, x0, y0);
  const int tid = threadIdx.x, lx = tid % TX2;
  for (int r = tid / TX2; r < TY; r += Tile2<TY>::NT / TX2) {
    const int x = x0 + lx, y = y0 + r;
    if (x >= a.nx || y >= a.ny) continue;
    const unsigned node = (unsigned)(y * a.px + x);
    NodeIn<Real> in;
    gather2d<D2Q9, 0, false, true>(a, x, y, in.Pf);
    gather2d<D2Q9, 1, false, true>(a, x, y, in.Pg);
    gather2d<D2Q9, 2, false, true>(a, x, y, in.Ps);
    in.phi = sphi[r + 2][lx + 2];
    Real g3[3];
    stencil2d<Real, R1X>(sphi, r + 2, lx + 2, g3, in.lphi);
    in.gphi[0] = g3[0];
    in.gphi[1] = g3[1];
    in.u[0] = sux[r + 1][lx + 1];
    in.u[1] = suy[r + 1][lx + 1];
    in.D = divergence2d<Real>(sphi, sux, suy, r + 1, lx + 1);
    in.phip = a.A_phip[node];
    NodeOut<Real> lo;
    for (int i = 0; i < 9; ++i) {
      lo.Af[i] = ldp(b.lA, a.slab, i, node);
      lo.Ag[i] = ldp(b.lA, a.slab, 9 + i, node);
      lo.As[i] = ldp(b.lA, a.slab, 18 + i, node);
    }
    lo.q = b.lqp[node];
    NodeAdjIn<Real> li;
    adj::node_adj(b.nc, in, lo, li);
    // adjoints of the pulled populations, stored at the slots they were read
    // from (transpose of the pull)
    Real tw[2][2] = {{0, 0}, {0, 0}};
    const Real* lsets[3] = {li.Pf, li.Pg, li.Ps};
#pragma unroll
    for (int fam = 0; fam < 3; ++fam)
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        Real sg;
        int wax, wsd;
        const size_t slot = pull_slot(a, fam, i, x, y, sg, wax, wsd);
        b.lP[slot] = sg * lsets[fam][i];
        if (fam == 2 && wax >= 0) tw[wax][wsd] += (Real)2 * (Real)D2Q9::w(i) * lsets[fam][i];
      }
    for (int ax = 0; ax < 2; ++ax)
      for (int sd = 0; sd < 2; ++sd)
        if (b.lTw[ax][sd] && tw[ax][sd] != (Real)0) b.lTw[ax][sd][ax == 1 ? x : y] += tw[ax][sd];
    // phi_prev of the next state is this step's phi
    b.lloc[(size_t)LL_PHI * a.slab + node] = li.phi + b.lphip[node];
    b.lloc[(size_t)LL_GX * a.slab + node] = li.gphi[0];
    b.lloc[(size_t)LL_GY * a.slab + node] = li.gphi[1];
    b.lloc[(size_t)LL_LAP * a.slab + node] = li.lphi;
    b.lloc[(size_t)LL_UX * a.slab + node] = li.u[0];
    b.lloc[(size_t)LL_UY * a.slab + node] = li.u[1];
    b.lloc[(size_t)LL_D * a.slab + node] = li.D;
    b.lphip[node] = li.phip;
    b.fphi[node] = in.phi;
    b.fux[node] = in.u[0];
    b.fuy[node] = in.u[1];
  }
}

// Transposed gradient stencil of an adjoint field g_a at (x, y):
// sum over pairs of 3 w_i c_ia [g_a(x - c_i) - g_a(x + c_i)].
template <class Real, class Store>
__device__ inline void grad_T(const KArgs<Real, Store>& a, const Real* gx, const Real* gy, int x,
                              int y, Real* out) {
  Real ox = 0, oy = 0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    if (i > D2Q9::opp(i)) continue;
    const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
    const Real w = (Real)D2Q9::w(i);
    if (cx && gx) ox += w * (Real)cx * (lfield(a, gx, x - cx, y - cy) - lfield(a, gx, x + cx, y + cy));
    if (cy && gy) oy += w * (Real)cy * (lfield(a, gy, x - cx, y - cy) - lfield(a, gy, x + cx, y + cy));
  }
  out[0] = (Real)3 * ox;
  out[1] = (Real)3 * oy;
}

// ---------------------------------------------------------------------------
// The u transpose at one node: transpose of D = div(u phi) and the
// velocity-closure adjoint
// ---------------------------------------------------------------------------
// At domain node (x, y): lambda of P_a = u_a phi from the transposed gradient
// of lambda_D (and from the ghost nodes this node mirrors), then the adjoint
// of the velocity closure.  lPf: the adjoints to add to the node's pulled f;
// L: the node's lambda of phi, grad phi (x, y) and lap phi after this step.
template <class Real>
__device__ inline void u_transpose(const KArgs<Real, Real>& a, const AdjArgs<Real>& b, int x, int y,
                                   Real* lPf, Real* L) {
  const unsigned node = (unsigned)(y * a.px + x);
  const Real* lD = b.lloc + (size_t)LL_D * a.slab;
  const Real phi = b.fphi[node];
  const Real u[2] = {b.fux[node], b.fuy[node]};
  // lambda of P_a = u_a phi at this node
  Real lPa[2];
  grad_T(a, lD, lD, x, y, lPa);
  Real lu[2] = {ldp(b.lloc, a.slab, LL_UX, node) + lPa[0] * phi,
                ldp(b.lloc, a.slab, LL_UY, node) + lPa[1] * phi};
  Real lphi = lPa[0] * u[0] + lPa[1] * u[1];
  // this node as the mirror of a ghost node: P_a(ghost) = -u_a (2 phi_w - phi)
  for (int ax = 0; ax < 2; ++ax) {
    if (!a.wall[ax]) continue;
    const int n = ax == 0 ? a.nx : a.ny, c = ax == 0 ? x : y;
    for (int side = 0; side < 2; ++side) {
      if ((side == 0 && c != 0) || (side == 1 && c != n - 1)) continue;
      const int gx = ax == 0 ? (side == 0 ? -1 : a.nx) : x;
      const int gy = ax == 1 ? (side == 0 ? -1 : a.ny) : y;
      Real lPg[2];
      grad_T(a, lD, lD, gx, gy, lPg);
      const Real phig = (Real)2 * a.phi_w[ax][side] - phi;
      for (int k = 0; k < 2; ++k) {
        lu[k] += -lPg[k] * phig;
        lphi += lPg[k] * u[k];
      }
    }
  }
  // velocity closure at this node (from the forward u: the pulled f enter
  // it only through their first moment)
  Real P[3][3];
  for (int j = -1; j <= 1; ++j)
    for (int i = -1; i <= 1; ++i) P[j + 1][i + 1] = phi_g(a, b.fphi, x + i, y + j);
  Real g[2] = {0, 0}, l = 0, ws = 0;
  for (int i = 1; i < 9; ++i) {
    if (i > D2Q9::opp(i)) continue;
    const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
    const Real w = (Real)D2Q9::w(i);
    const Real p = P[1 + cy][1 + cx], m = P[1 - cy][1 - cx];
    if (cx) g[0] += w * (Real)cx * (p - m);
    if (cy) g[1] += w * (Real)cy * (p - m);
    l += w * (p + m);
    ws += w;
  }
  g[0] *= (Real)3;
  g[1] *= (Real)3;
  const Real lap = (l - (Real)2 * ws * phi) * (Real)6;
#pragma unroll
  for (int i = 0; i < 9; ++i) lPf[i] = 0;
  Real l_phi_u, l_g[2], l_lap;
  adj::u_adj_at(b.nc, u, phi, g, lap, lu, lPf, l_phi_u, l_g, l_lap);
  L[0] = ldp(b.lloc, a.slab, LL_PHI, node) + lphi + l_phi_u;
  L[1] = ldp(b.lloc, a.slab, LL_GX, node) + l_g[0];
  L[2] = ldp(b.lloc, a.slab, LL_GY, node) + l_g[1];
  L[3] = ldp(b.lloc, a.slab, LL_LAP, node) + l_lap;
}

// Add v[i] (times the read's sign) to the nine slots that the pull of
// family fam at (x, y) read; all reads first, then all writes (written as
// nine separate +=, the reads would wait behind the writes: the compiler
// cannot prove the slots distinct).
template <class Real>
__device__ inline void add_pulled(const KArgs<Real, Real>& a, Real* lP, int fam, int x, int y,
                                  const Real* v) {
  size_t slot[9];
  Real old[9], sg[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int wax, wsd;
    slot[i] = pull_slot(a, fam, i, x, y, sg[i], wax, wsd);
    old[i] = lP[slot[i]];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) lP[slot[i]] = old[i] + sg[i] * v[i];
}

// Transposed stencils for lambda_phi at (x, y) (in-domain or ghost position).
template <class Real, class Store>
__device__ inline Real phi_T(const KArgs<Real, Store>& a, const Real* lg_x, const Real* lg_y,
                             const Real* ll, int x, int y, bool self) {
  Real g[2];
  grad_T(a, lg_x, lg_y, x, y, g);
  Real l = 0, ws = 0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    if (i > D2Q9::opp(i)) continue;
    const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
    const Real w = (Real)D2Q9::w(i);
    l += w * (lfield(a, ll, x - cx, y - cy) + lfield(a, ll, x + cx, y + cy));
    ws += w;
  }
  Real out = g[0] + g[1] + (Real)6 * l;
  if (self) out -= (Real)12 * ws * lfield(a, ll, x, y);
  return out;
}

// ---------------------------------------------------------------------------
// K_C: stencil transposes, phi = sum g + q_prev / 2 (initial-condition step)
// ---------------------------------------------------------------------------
template <class Real>
__global__ __launch_bounds__(256) void k_adj_phi2d(const KArgs<Real, Real> a, const AdjArgs<Real> b,
                                                   Real* lphi_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const unsigned node = (unsigned)(y * a.px + x);
  const Real* lgx = b.lloc + (size_t)LL_GX * a.slab;
  const Real* lgy = b.lloc + (size_t)LL_GY * a.slab;
  const Real* ll = b.lloc + (size_t)LL_LAP * a.slab;
  Real lphi = ldp(b.lloc, a.slab, LL_PHI, node) + phi_T(a, lgx, lgy, ll, x, y, true);
  // ghosts 2 phi_w - phi(mirror): their transposed value flows back with -1
  for (int ax = 0; ax < 2; ++ax) {
    if (!a.wall[ax]) continue;
    const int n = ax == 0 ? a.nx : a.ny, c = ax == 0 ? x : y;
    for (int side = 0; side < 2; ++side) {
      if ((side == 0 && c != 0) || (side == 1 && c != n - 1)) continue;
      const int gx = ax == 0 ? (side == 0 ? -1 : a.nx) : x;
      const int gy = ax == 1 ? (side == 0 ? -1 : a.ny) : y;
      lphi -= phi_T(a, lgx, lgy, ll, gx, gy, false);
    }
  }
  if (lphi_out) {   // initial-condition adjoint: lambda of phi0 itself
    lphi_out[(unsigned)(y * a.nx + x)] = lphi;
    return;
  }
  const Real v[9] = {lphi, lphi, lphi, lphi, lphi, lphi, lphi, lphi, lphi};
  add_pulled(a, b.lP, 1, x, y, v);
  b.lqp[node] = (Real)0.5 * lphi;
}

// ---------------------------------------------------------------------------
// K_BC: the u transpose and the phi transpose of one step, fused
// ---------------------------------------------------------------------------
// A workgroup owns a 64 x TY tile, one node per lane.  Phase U runs the u
// transpose on the tile plus a 1-node halo (each lane its own node first,
// then the halo nodes; only a tile node updates its pulled f) and stages the
// node totals of lambda grad phi and lambda lap phi in LDS, 0 beyond a wall.
// Phase Phi applies the transposed stencils from LDS (and at the ghost
// positions a wall-adjacent node mirrors), then phi = sum g + q_prev/2 sends
// lambda_phi to the nine pulled g and to q_prev.
template <class Real, int TY>
__global__ __launch_bounds__(TX2 * TY) void k_adj_uphi2d(const KArgs<Real, Real> a,
                                                        const AdjArgs<Real> b) {
  constexpr int NT = TX2 * TY, RX = R2X, RY = TY + 2;
  __shared__ Real sgx[RY][RX], sgy[RY][RX], slap[RY][RX];
  const int tiles_x = (a.nx + TX2 - 1) / TX2;
  const int t = blockIdx.x;
  const int x0 = (t % tiles_x) * TX2, y0 = (t / tiles_x) * TY;
  const int tid = threadIdx.x, lx = tid % TX2, r = tid / TX2;
  const int x = x0 + lx, y = y0 + r;
  const bool own = x < a.nx && y < a.ny;
  // ---- phase U ------------------------------------------------------------
  auto u_at = [&](int ry, int rx, bool mine) -> Real {
    int gx = x0 - 1 + rx, gy = y0 - 1 + ry;
    Real L[4] = {0, 0, 0, 0};
    const bool beyond = (a.wall[0] && (gx < 0 || gx >= a.nx)) || (a.wall[1] && (gy < 0 || gy >= a.ny));
    if (!beyond) {
      gx = wrapmod(gx, a.nx);
      gy = wrapmod(gy, a.ny);
      Real lPf[9];
      u_transpose(a, b, gx, gy, lPf, L);
      if (mine) add_pulled(a, b.lP, 0, gx, gy, lPf);
    }
    sgx[ry][rx] = L[1];
    sgy[ry][rx] = L[2];
    slap[ry][rx] = L[3];
    return L[0];
  };
  // one loop over the lane's own node (k = tid) and then its halo nodes,
  // so that the u transpose is emitted once
  Real lphi_u = 0;
  for (int k = tid; k < RX * RY; k += NT) {
    int ry = r + 1, rx = lx + 1;
    if (k >= NT) halo2_rc<TY>(k - NT, ry, rx);
    const Real v = u_at(ry, rx, k < NT && own);
    if (k < NT) lphi_u = v;
  }
  __syncthreads();
  if (!own) return;
  // ---- phase Phi ----------------------------------------------------------
  // transposed gradient and Laplacian at region position (ry, rx); points
  // outside the region lie beyond a wall (ghost evaluations only) and are 0
  auto phiT = [&](int ry, int rx, bool self) -> Real {
    auto F = [&](const Real (*s)[RX], int yy, int xx) -> Real {
      return (yy < 0 || yy >= RY || xx < 0 || xx >= RX) ? (Real)0 : s[yy][xx];
    };
    Real ox = 0, oy = 0, l = 0, ws = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      if (i > D2Q9::opp(i)) continue;
      const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
      const Real w = (Real)D2Q9::w(i);
      if (cx) ox += w * (Real)cx * (F(sgx, ry - cy, rx - cx) - F(sgx, ry + cy, rx + cx));
      if (cy) oy += w * (Real)cy * (F(sgy, ry - cy, rx - cx) - F(sgy, ry + cy, rx + cx));
      l += w * (F(slap, ry - cy, rx - cx) + F(slap, ry + cy, rx + cx));
      ws += w;
    }
    Real out = (Real)3 * ox + (Real)3 * oy + (Real)6 * l;
    if (self) out -= (Real)12 * ws * slap[ry][rx];
    return out;
  };
  Real lphi = lphi_u + phiT(r + 1, lx + 1, true);
  // ghosts 2 phi_w - phi(mirror): their transposed value flows back with -1
  for (int ax = 0; ax < 2; ++ax) {
    if (!a.wall[ax]) continue;
    const int n = ax == 0 ? a.nx : a.ny, c = ax == 0 ? x : y;
    for (int side = 0; side < 2; ++side) {
      if ((side == 0 && c != 0) || (side == 1 && c != n - 1)) continue;
      const int gx = ax == 0 ? (side == 0 ? -1 : a.nx) : x;
      const int gy = ax == 1 ? (side == 0 ? -1 : a.ny) : y;
      lphi -= phiT(gy - (y0 - 1), gx - (x0 - 1), false);
    }
  }
  const Real v[9] = {lphi, lphi, lphi, lphi, lphi, lphi, lphi, lphi, lphi};
  add_pulled(a, b.lP, 1, x, y, v);
  b.lqp[(unsigned)(y * a.px + x)] = (Real)0.5 * lphi;
}

// ---------------------------------------------------------------------------
// Seed: a loss of the final fields with dL/dphi^N = gphi and dL/dT^N = gT
// (fields [ny][nx] of Real, each nullable), at the fields of the state X^N
// as the fields pass computes them:
//   phi^N = sum g (pulled) + q_prev / 2,
//   T^N   = sum s (pulled) - (L/Cp)/2 [phi^N - phi_prev + div(u^N phi^N)].
// This kernel recomputes phi and u on the tile in LDS (as the forward), sends
// gT to the pulled s (at the slots they were read from; anti-bounce-back
// links add 2 w_i gT to the wall-temperature gradient) and leaves the node
// adjoints of phi and D for the u / phi transposes (K_BC), which carry them
// to the pulled f and g and to q_prev.
// ---------------------------------------------------------------------------
template <class Real, int TY>
__global__ __launch_bounds__(Tile2<TY>::NT) void k_adj_seed_local2d(const KArgs<Real, Real> a,
                                                                   const AdjArgs<Real> b,
                                                                   const Real* gphi, const Real* gT) {
  __shared__ Real sphi[Tile2<TY>::R1Y][R1X];
  __shared__ Real sux[Tile2<TY>::R2Y][R2X];
  __shared__ Real suy[Tile2<TY>::R2Y][R2X];
  const int tiles_x = (a.nx + TX2 - 1) / TX2;
  const int t = blockIdx.x;
  const int x0 = (t % tiles_x) * TX2, y0 = (t / tiles_x) * TY;
  stage2d<Real, Real, true, true, false, TY>(a, sphi, sux, suy, x0, y0);
  const int tid = threadIdx.x, lx = tid % TX2;
  for (int r = tid / TX2; r < TY; r += Tile2<TY>::NT / TX2) {
    const int x = x0 + lx, y = y0 + r;
    if (x >= a.nx || y >= a.ny) continue;
    const unsigned node = (unsigned)(y * a.px + x);
    const unsigned fidx = (unsigned)(y * a.nx + x);
    const Real gp = gphi ? gphi[fidx] : (Real)0;
    const Real gt = gT ? gT[fidx] : (Real)0;
    const Real hl = (Real)0.5 * b.nc.Lcp * gt;
    Real tw[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
    for (int fam = 0; fam < 3; ++fam)
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        Real sg;
        int wax, wsd;
        const size_t slot = pull_slot(a, fam, i, x, y, sg, wax, wsd);
        b.lP[slot] = fam == 2 ? sg * gt : (Real)0;
        if (fam == 2 && wax >= 0) tw[wax][wsd] += (Real)2 * (Real)D2Q9::w(i) * gt;
      }
    for (int ax = 0; ax < 2; ++ax)
      for (int sd = 0; sd < 2; ++sd)
        if (b.lTw[ax][sd] && tw[ax][sd] != (Real)0) b.lTw[ax][sd][ax == 1 ? x : y] += tw[ax][sd];
    b.lloc[(size_t)LL_PHI * a.slab + node] = gp - hl;
    b.lloc[(size_t)LL_GX * a.slab + node] = 0;
    b.lloc[(size_t)LL_GY * a.slab + node] = 0;
    b.lloc[(size_t)LL_LAP * a.slab + node] = 0;
    b.lloc[(size_t)LL_UX * a.slab + node] = 0;
    b.lloc[(size_t)LL_UY * a.slab + node] = 0;
    b.lloc[(size_t)LL_D * a.slab + node] = -hl;
    b.lphip[node] = hl;
    b.fphi[node] = sphi[r + 2][lx + 2];
    b.fux[node] = sux[r + 1][lx + 1];
    b.fuy[node] = suy[r + 1][lx + 1];
  }
}

// Initial-condition adjoint, local part.  The initial state is the pull
// pre-image of the barred equilibria at (phi0, T0) with u = 0: lambda of
// those post-streaming values is the pull of lambda_A (anti-bounce-back
// slots also carry 2 w_i T_w).  phi0 = phi_prev^0, T0 = sum of the pulled s.
template <class Real>
__global__ __launch_bounds__(256) void k_adj_init_local2d(const KArgs<Real, Real> a,
                                                          const AdjArgs<Real> b, Real* lT0_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const unsigned node = (unsigned)(y * a.px + x);
  // lambda of the post-streaming init values: pull of lambda_A
  NodeOut<Real> lo;
  Real* lsets[3] = {lo.Af, lo.Ag, lo.As};
  Real tw[2][2] = {{0, 0}, {0, 0}};
  for (int fam = 0; fam < 3; ++fam)
    for (int i = 0; i < 9; ++i) {
      const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
      int sx = x - cx, sy = y - cy;
      const bool oy = cy != 0 && a.wall[1] && (sy < 0 || sy >= a.ny);
      const bool ox = cx != 0 && !oy && a.wall[0] && (sx < 0 || sx >= a.nx);
      if (oy || ox) {
        const int j = D2Q9::opp(i);
        const Real la = b.lA[(size_t)(fam * 9 + j) * a.slab + node];
        lsets[fam][i] = fam == 0 ? la : -la;
        if (fam == 2) {
          const int ax = oy ? 1 : 0;
          const int side = oy ? (sy < 0 ? 0 : 1) : (sx < 0 ? 0 : 1);
          tw[ax][side] += (Real)2 * (Real)D2Q9::w(i) * la;
        }
      } else {
        if (!a.wall[0]) sx = wrap1(sx, a.nx);
        if (!a.wall[1]) sy = wrap1(sy, a.ny);
        lsets[fam][i] = b.lA[(size_t)(fam * 9 + i) * a.slab + (unsigned)(sy * a.px + sx)];
      }
    }
  lo.q = b.lqp[node];
  for (int ax = 0; ax < 2; ++ax)
    for (int side = 0; side < 2; ++side)
      if (b.lTw[ax][side] && tw[ax][side] != (Real)0) b.lTw[ax][side][ax == 1 ? x : y] += tw[ax][side];
  // forward init inputs: phi0 and its stencils, T0
  const Real phi = a.A_phip[node];
  Real P[3][3];
  for (int j = -1; j <= 1; ++j)
    for (int i = -1; i <= 1; ++i) P[j + 1][i + 1] = phi_g(a, a.A_phip, x + i, y + j);
  Real g[2] = {0, 0}, l = 0, ws = 0;
  for (int i = 1; i < 9; ++i) {
    if (i > D2Q9::opp(i)) continue;
    const int cx = D2Q9::cx(i), cy = D2Q9::cy(i);
    const Real w = (Real)D2Q9::w(i);
    const Real p = P[1 + cy][1 + cx], m = P[1 - cy][1 - cx];
    if (cx) g[0] += w * (Real)cx * (p - m);
    if (cy) g[1] += w * (Real)cy * (p - m);
    l += w * (p + m);
    ws += w;
  }
  g[0] *= (Real)3;
  g[1] *= (Real)3;
  const Real lap = (l - (Real)2 * ws * phi) * (Real)6;
  Real Ps[9];
  gather2d<D2Q9, 2, false, true>(a, x, y, Ps);
  Real T = 0;
  for (int i = 0; i < 9; ++i) T += Ps[i];
  Real l_phi, l_g[2], l_lap, l_T;
  adj::init_adj(b.nc, phi, g, lap, T, lo, l_phi, l_g, l_lap, l_T);
  b.lloc[(size_t)LL_PHI * a.slab + node] = l_phi + b.lphip[node];
  b.lloc[(size_t)LL_GX * a.slab + node] = l_g[0];
  b.lloc[(size_t)LL_GY * a.slab + node] = l_g[1];
  b.lloc[(size_t)LL_LAP * a.slab + node] = l_lap;
  if (lT0_out) lT0_out[(unsigned)(y * a.nx + x)] = l_T;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class Real>
static dim3 node_grid(const KArgs<Real, Real>& a) {
  return dim3((a.nx + 255) / 256, a.ny);
}

template <class Real>
hipError_t launch_adj_step2d_t(const KArgs<Real, Real>& a, const AdjArgs<Real>& b, hipStream_t st) {
  // Local kernel on 8-row tiles: the re-gathered populations of a tile are
  // still in L2 (512 x 512 FP32, whole reverse step: 71 us against 75 with
  // 4 rows and 86 with 16).  u/phi transposes on 64 x 16 tiles of 1024
  // lanes (70.5 us against 71.2 with 8 rows and 72.7 with 4).
  constexpr int ty = 8;
  const int tiles = ((a.nx + TX2 - 1) / TX2) * ((a.ny + ty - 1) / ty);
  hipLaunchKernelGGL((k_adj_local2d<Real, ty>), dim3(tiles), dim3(Tile2<ty>::NT), 0, st, a, b);
  constexpr int tyb = 16;
  const int tiles_b = ((a.nx + TX2 - 1) / TX2) * ((a.ny + tyb - 1) / tyb);
  hipLaunchKernelGGL((k_adj_uphi2d<Real, tyb>), dim3(tiles_b), dim3(TX2 * tyb), 0, st, a, b);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_adj_seed2d_t(const KArgs<Real, Real>& a, const AdjArgs<Real>& b, const Real* gphi,
                               const Real* gT, hipStream_t st) {
  constexpr int ty = 8;
  const int tiles = ((a.nx + TX2 - 1) / TX2) * ((a.ny + ty - 1) / ty);
  hipLaunchKernelGGL((k_adj_seed_local2d<Real, ty>), dim3(tiles), dim3(Tile2<ty>::NT), 0, st, a, b,
                     gphi, gT);
  constexpr int tyb = 16;
  const int tiles_b = ((a.nx + TX2 - 1) / TX2) * ((a.ny + tyb - 1) / tyb);
  hipLaunchKernelGGL((k_adj_uphi2d<Real, tyb>), dim3(tiles_b), dim3(TX2 * tyb), 0, st, a, b);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_adj_init2d_t(const KArgs<Real, Real>& a, const AdjArgs<Real>& b, Real* dphi0,
                               Real* dT0, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_init_local2d<Real>, node_grid(a), dim3(256), 0, st, a, b, dT0);
  hipLaunchKernelGGL(k_adj_phi2d<Real>, node_grid(a), dim3(256), 0, st, a, b, dphi0);
  return hipGetLastError();
}

#define LBM_ADJ_INST(REAL)                                                                    \
  hipError_t launch_adj_step2d(const KArgs<REAL, REAL>& a, const AdjArgs<REAL>& b,             \
                               hipStream_t st) {                                              \
    return launch_adj_step2d_t<REAL>(a, b, st);                                               \
  }                                                                                           \
  hipError_t launch_adj_seed2d(const KArgs<REAL, REAL>& a, const AdjArgs<REAL>& b,             \
                               const REAL* g, const REAL* gT, hipStream_t st) {               \
    return launch_adj_seed2d_t<REAL>(a, b, g, gT, st);                                        \
  }                                                                                           \
  hipError_t launch_adj_init2d(const KArgs<REAL, REAL>& a, const AdjArgs<REAL>& b, REAL* dphi0, \
                               REAL* dT0, hipStream_t st) {                                   \
    return launch_adj_init2d_t<REAL>(a, b, dphi0, dT0, st);                                   \
  }
LBM_ADJ_INST(float)
LBM_ADJ_INST(double)
#undef LBM_ADJ_INST

}  // namespace lbm
