// C ABI of the phase-change LBM library (see include/lbm.h).
//
// Host side: parameter validation, workspace carving, relaxation rates and
// codec constants, kernel launches on the caller's stream, and the
// deterministic FP64 diagnostics reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_kernels.h"
#include "lbm_adjargs.h"
#include "lbm_tape.h"

using namespace lbm;

namespace {

thread_local std::string g_err = "no error";

lbm_status fail(lbm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
lbm_status fail(lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

lbm_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return LBM_OK;
  return fail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
  int Qf, Qg, Qs, Qtot;
  int px;
  long long slab;
  size_t elem, sc_elem, real_elem;
  size_t pops, scal, faces[3][2], partials;
  int nsc;   // scalar planes per state: phi_prev, q_prev (+ T_ref for 16-bit storage)
  size_t total;
  int nblocks;
};

}  // namespace

struct lbm_ctx {
  lbm_params prm;
  Layout L;
  int ns, heat;
  char* ws;
  void* pops[2];
  void* phip[2];
  void* qp[2];
  void* tref[2];   // 16-bit storage: per-node reference of the s family
  void* tw[3][2];
  double* partials;
  double* red;
  int cur;
  int64_t step;
  int initialized;
  hipStream_t stream;
  double ref[3], scale[3];
  // sqrt(T) tape of the last lbm_forward_taped call
  char* tape;
  size_t tape_bytes;
  int64_t tape_n, tape_k, tape_nsnap, tape_end_step;
  int32_t tape_policy;
  int tape_ready;
  // the current state is step `step` of an lbm_init_fields call with u0 ==
  // NULL (the initialisation the reverse sweep differentiates)
  int fresh_init;
  // this device's copy of the static scratch (lbm_backward_static)
  void* scratch;
};

namespace {

// ---------------------------------------------------------------------------
// Static scratch of lbm_backward_static: the adjoint workspace for callers
// that cannot allocate device memory.  Every device the library runs on
// holds its own copy from module load until the process ends.  In host code
// the symbol is only a host-side stand-in: kernels and copies get the
// device address hipGetSymbolAddress returns for the current device, looked
// up once per device (lbm_create) and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)LBM_STATIC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

lbm_status scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_check(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(LBM_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

int q_of(int lat) { return lat; }

lbm_status validate(const lbm_params* p) {
  if (!p) return fail(LBM_E_INVAL, "params is NULL");
  if (p->dim != 2 && p->dim != 3) return fail(LBM_E_INVAL, "dim must be 2 or 3");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_E_INVAL, "grid sizes must be >= 1");
  if (p->dim == 2) {
    if (p->nz != 1) return fail(LBM_E_INVAL, "2-D needs nz == 1");
    if (p->lat_f != LBM_D2Q9 || (p->lat_g != LBM_D2Q9 && p->lat_g != LBM_D2Q5) ||
        p->lat_s != p->lat_g)
      return fail(LBM_E_UNSUPPORTED,
                  "2-D supports D2Q9 for f and D2Q9 or D2Q5 (the same) for g and s");
    // the 2-halo ghost beyond a wall mirrors the second node from it
    if ((p->bc[0] == LBM_BC_WALL && p->nx < 2) || (p->bc[1] == LBM_BC_WALL && p->ny < 2))
      return fail(LBM_E_INVAL, "a walled axis needs at least 2 nodes");
  } else {
    if (p->lat_f != LBM_D3Q19 || p->lat_g != LBM_D3Q7 || p->lat_s != LBM_D3Q7)
      return fail(LBM_E_UNSUPPORTED, "3-D supports D3Q19 (f) with D3Q7 (g, s)");
    if (p->bc[0] != LBM_BC_PERIODIC || p->bc[1] != LBM_BC_PERIODIC)
      return fail(LBM_E_UNSUPPORTED, "3-D supports walls on z only");
    if (p->bc[2] == LBM_BC_WALL && p->nz < 2) return fail(LBM_E_INVAL, "z walls need nz >= 2");
  }
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != LBM_BC_PERIODIC && p->bc[a] != LBM_BC_WALL)
      return fail(LBM_E_INVAL, "bc[%d] must be LBM_BC_PERIODIC or LBM_BC_WALL", a);
  if (p->storage < LBM_ST_F64 || p->storage > LBM_ST_BF16_DEV)
    return fail(LBM_E_INVAL, "unknown storage %d", p->storage);
  const double pos[] = {p->nu_l, p->nu_g, p->mobility, p->alpha_l, p->alpha_g, p->W, p->rho_l, p->rho_g};
  const char* nm[] = {"nu_l", "nu_g", "mobility", "alpha_l", "alpha_g", "W", "rho_l", "rho_g"};
  for (int i = 0; i < 8; ++i)
    if (!(pos[i] > 0) || !std::isfinite(pos[i]))
      return fail(LBM_E_INVAL, "%s must be finite and > 0 (tau > 0, omega < 2)", nm[i]);
  if ((p->flags & LBM_HEAT) && !(p->L_over_cp > 0)) return fail(LBM_E_INVAL, "L_over_cp must be > 0");
  if ((p->flags & LBM_PHASE_CHANGE) && !(p->flags & LBM_HEAT))
    return fail(LBM_E_INVAL, "LBM_PHASE_CHANGE needs LBM_HEAT");
  if (p->A_coef < 0) return fail(LBM_E_INVAL, "A_coef must be >= 0");
  if (!(p->sigma >= 0)) return fail(LBM_E_INVAL, "sigma must be >= 0");
  if ((long long)p->nx * p->ny * p->nz > (1LL << 31)) return fail(LBM_E_INVAL, "grid too large");
  if (p->collision < LBM_COLL_BGK || p->collision > LBM_COLL_MRT)
    return fail(LBM_E_INVAL, "unknown collision %d", p->collision);
  if (p->collision == LBM_COLL_TRT)
    for (int k = 0; k < 3; ++k)
      if (!(p->trt_lambda[k] >= 0) || !std::isfinite(p->trt_lambda[k]))
        return fail(LBM_E_INVAL, "trt_lambda[%d] must be finite and >= 0 (0 -> 1/4)", k);
  if (p->collision == LBM_COLL_MRT) {
    if (p->dim == 3 && (p->flags & LBM_NS))
      return fail(LBM_E_UNSUPPORTED, "MRT is built for D2Q9 and D3Q7 (not D3Q19)");
    for (int k = 0; k < 3; ++k)
      for (int r = 0; r < 4; ++r)
        if (!(p->mrt_rates[k][r] > 0 && p->mrt_rates[k][r] < 2))
          return fail(LBM_E_INVAL, "mrt_rates[%d][%d] must lie in (0, 2)", k, r);
  }
  if (p->grad_scheme < LBM_GRAD_CENTRAL || p->grad_scheme > LBM_GRAD_BIASED2)
    return fail(LBM_E_INVAL, "unknown grad_scheme %d", p->grad_scheme);
  if ((p->flags & LBM_DIV_LOCAL) && !((p->flags & LBM_NS) && (p->flags & LBM_HEAT)))
    return fail(LBM_E_INVAL, "LBM_DIV_LOCAL needs LBM_NS and LBM_HEAT");
  if (p->check_every < 0) return fail(LBM_E_INVAL, "check_every must be >= 0");
  for (int a = 0; a < 3; ++a)
    for (int sd = 0; sd < 2; ++sd) {
      const int fb = p->f_bc[a][sd];
      if (fb != LBM_FBC_NOSLIP && fb != LBM_FBC_PRESSURE)
        return fail(LBM_E_INVAL, "unknown f_bc[%d][%d] = %d", a, sd, fb);
      if (fb == LBM_FBC_PRESSURE && p->bc[a] != LBM_BC_WALL)
        return fail(LBM_E_INVAL, "f_bc[%d][%d]: an open face needs a walled axis", a, sd);
      if (!std::isfinite(p->p_wall[a][sd])) return fail(LBM_E_INVAL, "p_wall must be finite");
    }
  if (p->dim == 2) {
    // the 2-D kernel addresses each population family with 32-bit byte offsets
    const long long px = (p->nx + 63) / 64 * 64;
    const long long elem = p->storage == LBM_ST_F64 ? 8 : (p->storage == LBM_ST_F32 ? 4 : 2);
    if (9LL * px * p->ny * elem >= (1LL << 32))
      return fail(LBM_E_UNSUPPORTED, "2-D grid too large for 32-bit family offsets");
  }
  return LBM_OK;
}

Layout layout(const lbm_params* p) {
  Layout L{};
  const bool ns = p->flags & LBM_NS, heat = p->flags & LBM_HEAT;
  L.Qf = ns ? q_of(p->lat_f) : 0;
  L.Qg = q_of(p->lat_g);
  L.Qs = heat ? q_of(p->lat_s) : 0;
  L.Qtot = L.Qf + L.Qg + L.Qs;
  L.px = (p->nx + 63) / 64 * 64;
  L.slab = (long long)L.px * p->ny * p->nz;
  L.elem = p->storage == LBM_ST_F64 ? 8 : (p->storage == LBM_ST_F32 ? 4 : 2);
  L.sc_elem = p->storage == LBM_ST_F64 ? 8 : 4;
  L.real_elem = p->storage == LBM_ST_F64 ? 8 : 4;
  L.pops = align256((size_t)L.Qtot * L.slab * L.elem);
  L.scal = align256((size_t)L.slab * L.sc_elem);
  const bool st16 = p->storage == LBM_ST_F16_DEV || p->storage == LBM_ST_BF16_DEV;
  L.nsc = (st16 && heat) ? 3 : 2;
  size_t tot = 2 * L.pops + 2 * (size_t)L.nsc * L.scal;
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) {
      L.faces[a][s] = 0;
      if (p->bc[a] == LBM_BC_WALL) {
        const size_t face = (size_t)n[0] * n[1] * n[2] / n[a];
        L.faces[a][s] = align256(face * L.real_elem);
        tot += L.faces[a][s];
      }
    }
  L.nblocks = p->dim == 2 ? step2d_blocks(p->nx, p->ny) : step3d_blocks(p->nx, p->ny, p->nz);
  L.partials = align256((size_t)(L.nblocks * NPART + 8) * sizeof(double));
  tot += L.partials;
  L.total = tot;
  return L;
}

template <class Real, class Store>
KArgs<Real, Store> make_args(const lbm_ctx* c) {
  const lbm_params& p = c->prm;
  KArgs<Real, Store> a{};
  a.nx = p.nx;
  a.ny = p.ny;
  a.nz = p.nz;
  a.px = c->L.px;
  a.slab = c->L.slab;
  for (int d = 0; d < 3; ++d) a.wall[d] = p.bc[d] == LBM_BC_WALL;
  a.off_f = 0;
  a.off_g = c->L.Qf;
  a.off_s = c->L.Qf + c->L.Qg;
  a.q_gs = c->L.Qg;
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < 2; ++s) {
      a.Tw[d][s] = (const Real*)c->tw[d][s];
      a.phi_w[d][s] = (Real)p.phi_wall[d][s];
      a.f_open[d][s] = p.f_bc[d][s] == LBM_FBC_PRESSURE ? 1 : 0;
      a.p_w[d][s] = (Real)p.p_wall[d][s];
      a.f_sg[d][s] = a.f_open[d][s] ? (Real)-1 : (Real)1;
      a.f_pw2[d][s] = a.f_open[d][s] ? (Real)2 * a.p_w[d][s] : (Real)0;
    }
  for (int k = 0; k < 3; ++k) {
    a.ref[k] = (Real)c->ref[k];
    a.scale[k] = (Real)c->scale[k];
    a.inv_scale[k] = (Real)(1.0 / c->scale[k]);
  }
  const double cs2g = (p.dim == 2 && p.lat_g == LBM_D2Q9) ? 1.0 / 3.0 : 0.25;   // D3Q7, D2Q5: 1/4
  a.rho_l = (Real)p.rho_l;
  a.rho_g = (Real)p.rho_g;
  a.K = (Real)(1.5 * p.W * p.sigma);          // Eq. Def_K-H
  a.H = (Real)(12.0 * p.sigma / p.W);
  a.four_over_W = (Real)(4.0 / p.W);
  const double eps = p.eps_n > 0 ? p.eps_n : 1e-3;
  a.eps2 = (Real)(eps * eps);
  for (int d = 0; d < 3; ++d) {
    a.grav[d] = (Real)p.gravity[d];
    a.body[d] = (Real)p.body_force[d];
  }
  a.nu_l = (Real)p.nu_l;
  a.nu_g = (Real)p.nu_g;
  a.alpha_l = (Real)p.alpha_l;
  a.alpha_g = (Real)p.alpha_g;
  a.Lcp = (Real)p.L_over_cp;
  a.inv_Lcp = (Real)(p.L_over_cp > 0 ? 1.0 / p.L_over_cp : 0.0);
  a.T_sat = (Real)p.T_sat;
  a.theta_I = (Real)p.theta_I;
  const double A = p.A_coef > 0 ? p.A_coef : 10.0 / 48.0;
  a.qcoef = (Real)(4.0 / (A * p.W * p.W));
  a.omega_g = (Real)(1.0 / (p.mobility / cs2g + 0.5));   // M = tau_g c_s^2
  a.M_over_cs2g = (Real)(p.mobility / cs2g);
  a.prod_fac = (Real)(p.rho_g * (1.0 / p.rho_g - 1.0 / p.rho_l));
  a.visc_linear = (p.flags & LBM_VISC_LINEAR) ? 1 : 0;
  a.geq_cac = (p.flags & LBM_GEQ_CAC) ? 1 : 0;
  a.phase_change = (p.flags & LBM_PHASE_CHANGE) ? 1 : 0;
  a.div_local = (p.flags & LBM_DIV_LOCAL) ? 1 : 0;
  a.coll = p.collision;
  for (int k = 0; k < 3; ++k) {
    a.lam[k] = (Real)(p.trt_lambda[k] > 0 ? p.trt_lambda[k] : 0.25);
    for (int r = 0; r < 4; ++r) a.mrt[k][r] = (Real)p.mrt_rates[k][r];
  }
  a.grad_scheme = p.grad_scheme;
  // non-temporal output stores once the two state buffers (populations and
  // lagged planes) exceed the 256 MiB last-level cache (Infinity Cache)
  a.nt = 2 * (c->L.pops + (size_t)c->L.nsc * c->L.scal) > ((size_t)256 << 20) ? 1 : 0;
  const int cur = c->cur;
  a.A = (const Store*)c->pops[cur];
  a.B = (Store*)c->pops[1 - cur];
  a.A_phip = (const typename KArgs<Real, Store>::Sc*)c->phip[cur];
  a.A_qp = (const typename KArgs<Real, Store>::Sc*)c->qp[cur];
  a.B_phip = (typename KArgs<Real, Store>::Sc*)c->phip[1 - cur];
  a.B_qp = (typename KArgs<Real, Store>::Sc*)c->qp[1 - cur];
  a.A_Tref = (const typename KArgs<Real, Store>::Sc*)c->tref[cur];
  a.B_Tref = (typename KArgs<Real, Store>::Sc*)c->tref[1 - cur];
  return a;
}

// Kernel arguments reading state blob `in` and writing state blob `out`
// (blob layout: populations | phi_prev | q_prev [| T_ref], each 256-byte
// aligned).
template <class Real, class Store>
KArgs<Real, Store> make_args_blobs(const lbm_ctx* c, const char* in, char* out) {
  KArgs<Real, Store> a = make_args<Real, Store>(c);
  using Sc = typename KArgs<Real, Store>::Sc;
  a.A = (const Store*)in;
  a.A_phip = (const Sc*)(in + c->L.pops);
  a.A_qp = (const Sc*)(in + c->L.pops + c->L.scal);
  a.B = (Store*)out;
  a.B_phip = (Sc*)(out ? out + c->L.pops : nullptr);
  a.B_qp = (Sc*)(out ? out + c->L.pops + c->L.scal : nullptr);
  a.A_Tref = c->L.nsc == 3 ? (const Sc*)(in + c->L.pops + 2 * c->L.scal) : nullptr;
  a.B_Tref = (c->L.nsc == 3 && out) ? (Sc*)(out + c->L.pops + 2 * c->L.scal) : nullptr;
  return a;
}

// Dispatch a callable on the (Real, Store) pair of the context.
template <class Fn>
hipError_t dispatch(const lbm_ctx* c, Fn&& fn) {
  switch (c->prm.storage) {
    case LBM_ST_F64: return fn(make_args<double, double>(c));
    case LBM_ST_F32: return fn(make_args<float, float>(c));
    case LBM_ST_F16_DEV: return fn(make_args<float, __half>(c));
    default: return fn(make_args<float, __hip_bfloat16>(c));
  }
}

__global__ void k_fill(void* dst, long long n, double v, int f64) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (f64) ((double*)dst)[i] = v;
  else ((float*)dst)[i] = (float)v;
}
__global__ void k_convert(void* dst, int dst_f64, const void* src, int src_f64, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = src_f64 ? ((const double*)src)[i] : (double)((const float*)src)[i];
  if (dst_f64) ((double*)dst)[i] = v;
  else ((float*)dst)[i] = (float)v;
}

__global__ void k_reduce(const double* partials, int nb, double* out) {
  __shared__ double red[NPART][4];
  double s[NPART] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    s[0] += partials[(long long)b * NPART + 0];
    s[1] += partials[(long long)b * NPART + 1];
    s[2] += partials[(long long)b * NPART + 2];
    s[3] = fmax(s[3], partials[(long long)b * NPART + 3]);
    s[4] += partials[(long long)b * NPART + 4];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = 0; k < NPART; ++k) s[k] = (k == 3) ? wave_max_d(s[k]) : wave_sum_d(s[k]);
  if (lane == 0)
    for (int k = 0; k < NPART; ++k) red[k][wv] = s[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < NPART; ++k) {
      double v = red[k][0];
      for (int w = 1; w < 4; ++w) v = (k == 3) ? fmax(v, red[k][w]) : v + red[k][w];
      out[k] = v;
    }
  }
}

}  // namespace

namespace lbm {
hipError_t launch_reduce(const double* partials, int nblocks, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, partials, nblocks, out);
  return hipGetLastError();
}
}  // namespace lbm

extern "C" {

lbm_status lbm_workspace_size(const lbm_params* prm, size_t* bytes) {
  if (!bytes) return fail(LBM_E_INVAL, "bytes is NULL");
  lbm_status s = validate(prm);
  if (s != LBM_OK) return s;
  *bytes = layout(prm).total;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_params* prm, void* ws, size_t bytes, void* stream, lbm_ctx** out) {
  if (!out) return fail(LBM_E_INVAL, "out is NULL");
  *out = nullptr;
  lbm_status s = validate(prm);
  if (s != LBM_OK) return s;
  const Layout L = layout(prm);
  if (!ws) return fail(LBM_E_INVAL, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(LBM_E_INVAL, "workspace must be 256-byte aligned");
  if (bytes < L.total)
    return fail(LBM_E_NOMEM, "workspace has %zu bytes, needs %zu", bytes, L.total);
  void* scr = nullptr;
  s = scratch_of_current_device(&scr);
  if (s != LBM_OK) return s;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_E_NOMEM, "host allocation failed");
  c->scratch = scr;
  c->prm = *prm;
  c->L = L;
  c->ns = (prm->flags & LBM_NS) != 0;
  c->heat = (prm->flags & LBM_HEAT) != 0;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)ws;
  char* p = c->ws;
  c->pops[0] = p;  p += L.pops;
  c->pops[1] = p;  p += L.pops;
  c->phip[0] = p;  p += L.scal;
  c->qp[0] = p;    p += L.scal;
  c->phip[1] = p;  p += L.scal;
  c->qp[1] = p;    p += L.scal;
  c->tref[0] = c->tref[1] = nullptr;
  if (L.nsc == 3) {
    c->tref[0] = p;  p += L.scal;
    c->tref[1] = p;  p += L.scal;
  }
  for (int a = 0; a < 3; ++a)
    for (int sd = 0; sd < 2; ++sd) {
      c->tw[a][sd] = L.faces[a][sd] ? (void*)p : nullptr;
      p += L.faces[a][sd];
    }
  c->partials = (double*)p;
  c->red = c->partials + (size_t)L.nblocks * NPART;
  // 16-bit deviation codec: phi about 1/2, T about the mean wall value,
  // f (gauge pressure) about 0; scale 2^12 keeps |dev| in FP16's normal range.
  double tref = prm->T_sat, cnt = 1;
  for (int a = 0; a < 3; ++a)
    if (prm->bc[a] == LBM_BC_WALL) {
      tref += prm->T_wall[a][0] + prm->T_wall[a][1];
      cnt += 2;
    }
  const bool f16 = prm->storage == LBM_ST_F16_DEV, b16 = prm->storage == LBM_ST_BF16_DEV;
  c->ref[0] = 0.0;
  c->ref[1] = (f16 || b16) ? 0.5 : 0.0;
  c->ref[2] = (f16 || b16) ? tref / cnt : 0.0;
  for (int k = 0; k < 3; ++k) c->scale[k] = f16 ? 4096.0 : 1.0;
  c->cur = 0;
  // wall rows start at the scalar face values
  const int n[3] = {prm->nx, prm->ny, prm->nz};
  for (int a = 0; a < 3; ++a)
    for (int sd = 0; sd < 2; ++sd)
      if (c->tw[a][sd]) {
        const long long face = (long long)n[0] * n[1] * n[2] / n[a];
        hipLaunchKernelGGL(k_fill, dim3((face + 255) / 256), dim3(256), 0, c->stream, c->tw[a][sd],
                           face, prm->T_wall[a][sd], prm->storage == LBM_ST_F64 ? 1 : 0);
      }
  s = hip_check(hipGetLastError(), "lbm_create");
  if (s != LBM_OK) {
    delete c;
    return s;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx* c, const void* phi0, const void* T0, const void* u0,
                           const void* p0, int32_t dtype) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  if (!phi0) return fail(LBM_E_INVAL, "phi0 is NULL");
  if (c->heat && !T0) return fail(LBM_E_INVAL, "T0 is NULL but LBM_HEAT is set");
  if (dtype != LBM_DT_F32 && dtype != LBM_DT_F64) return fail(LBM_E_INVAL, "bad dtype");
  // the init kernel writes the current buffer: pretend it is B of a step
  c->cur = 1;
  const int f64 = dtype == LBM_DT_F64;
  hipError_t e = dispatch(c, [&](auto a) {
    return c->prm.dim == 2 ? launch_init2d(a, c->ns, c->heat, phi0, T0, u0, p0, f64, c->stream)
                           : launch_init3d(a, c->ns, c->heat, phi0, T0, u0, p0, f64, c->stream);
  });
  c->cur = 0;
  c->step = 0;
  c->initialized = 1;
  c->tape_ready = 0;
  c->fresh_init = u0 == nullptr;
  return hip_check(e, "lbm_init_fields");
}

lbm_status lbm_set_wall_T(lbm_ctx* c, int32_t axis, int32_t side, const void* face, int32_t dtype) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  if (axis < 0 || axis > 2 || side < 0 || side > 1) return fail(LBM_E_INVAL, "bad face");
  if (!c->tw[axis][side]) return fail(LBM_E_INVAL, "axis %d is not walled", axis);
  if (!face) return fail(LBM_E_INVAL, "face is NULL");
  if (dtype != LBM_DT_F32 && dtype != LBM_DT_F64) return fail(LBM_E_INVAL, "bad dtype");
  const int n[3] = {c->prm.nx, c->prm.ny, c->prm.nz};
  const long long cnt = (long long)n[0] * n[1] * n[2] / n[axis];
  c->tape_ready = 0;   // a recorded tape would be recomputed with the new wall values
  hipLaunchKernelGGL(k_convert, dim3((cnt + 255) / 256), dim3(256), 0, c->stream, c->tw[axis][side],
                     c->prm.storage == LBM_ST_F64 ? 1 : 0, face, dtype == LBM_DT_F64 ? 1 : 0, cnt);
  return hip_check(hipGetLastError(), "lbm_set_wall_T");
}

static lbm_status run_macro(lbm_ctx* c, uint32_t mask, void* out, int f64, double* partials) {
  hipError_t e = dispatch(c, [&](auto a) {
    a.out = out;
    a.out_f64 = f64;
    a.out_mask = mask;
    a.partials = partials;
    return c->prm.dim == 2 ? launch_step2d(a, c->ns, c->heat, MODE_MACRO, c->stream)
                           : launch_step3d(a, c->ns, c->heat, MODE_MACRO, c->stream);
  });
  return hip_check(e, "macro pass");
}

// FP64 sums of the current fields into r[NPART] (host): sum phi, sum T,
// sum phi_prev, max |u|, count of non-finite nodes.  Synchronises.
static lbm_status reduce_fields(lbm_ctx* c, double* r) {
  lbm_status s = run_macro(c, 0u, nullptr, 0, c->partials);
  if (s != LBM_OK) return s;
  s = hip_check(launch_reduce(c->partials, c->L.nblocks, c->red, c->stream), "reduce");
  if (s != LBM_OK) return s;
  s = hip_check(hipMemcpyAsync(r, c->red, NPART * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                "copy");
  if (s != LBM_OK) return s;
  return hip_check(hipStreamSynchronize(c->stream), "reduce_fields");
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  if (!c->initialized) return fail(LBM_E_STATE, "lbm_step before lbm_init_fields / lbm_set_state");
  if (nsteps < 0) return fail(LBM_E_INVAL, "nsteps < 0");
  const int every = c->prm.check_every;
  for (int64_t k = 0; k < nsteps; ++k) {
    hipError_t e = dispatch(c, [&](auto a) {
      return c->prm.dim == 2 ? launch_step2d(a, c->ns, c->heat, MODE_STEP, c->stream)
                             : launch_step3d(a, c->ns, c->heat, MODE_STEP, c->stream);
    });
    if (e != hipSuccess) return hip_check(e, "lbm_step");
    c->cur = 1 - c->cur;
    ++c->step;
    if (every > 0 && c->step % every == 0) {
      double r[NPART];
      lbm_status s = reduce_fields(c, r);
      if (s != LBM_OK) return s;
      if (r[4] != 0)
        return fail(LBM_E_UNSTABLE, "%.0f non-finite nodes after step %lld", r[4], (long long)c->step);
    }
  }
  return LBM_OK;
}

lbm_status lbm_get_fields(lbm_ctx* c, uint32_t mask, void* out, int32_t dtype) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  if (!c->initialized) return fail(LBM_E_STATE, "lbm_get_fields before initialisation");
  if (mask & ~63u) return fail(LBM_E_INVAL, "unknown field bits");
  if (mask && !out) return fail(LBM_E_INVAL, "out is NULL");
  if (dtype != LBM_DT_F32 && dtype != LBM_DT_F64) return fail(LBM_E_INVAL, "bad dtype");
  if (!mask) return LBM_OK;
  return run_macro(c, mask, out, dtype == LBM_DT_F64, nullptr);
}

lbm_status lbm_diagnostics(lbm_ctx* c, double out[5]) {
  if (!c || !out) return fail(LBM_E_INVAL, "NULL argument");
  if (!c->initialized) return fail(LBM_E_STATE, "lbm_diagnostics before initialisation");
  double r[NPART];
  lbm_status s = reduce_fields(c, r);
  if (s != LBM_OK) return s;
  const double N = (double)c->prm.nx * c->prm.ny * c->prm.nz;
  const double Lcp = c->heat ? c->prm.L_over_cp : 0.0;
  out[0] = r[0];
  out[1] = r[1] + Lcp * 0.5 * (r[0] + r[2]);
  out[2] = r[0] / N;
  out[3] = r[3];
  out[4] = r[4];
  if (r[4] != 0) return fail(LBM_E_UNSTABLE, "%.0f non-finite nodes", r[4]);
  return LBM_OK;
}

lbm_status lbm_state_size(const lbm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(LBM_E_INVAL, "NULL argument");
  *bytes = c->L.pops + (size_t)c->L.nsc * c->L.scal;
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, void* out, size_t bytes) {
  if (!c || !out) return fail(LBM_E_INVAL, "NULL argument");
  if (!c->initialized) return fail(LBM_E_STATE, "no state yet");
  if (bytes < c->L.pops + (size_t)c->L.nsc * c->L.scal)
    return fail(LBM_E_NOMEM, "state buffer too small");
  char* o = (char*)out;
  hipError_t e = hipMemcpyAsync(o, c->pops[c->cur], c->L.pops, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o + c->L.pops, c->phip[c->cur], c->L.scal, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o + c->L.pops + c->L.scal, c->qp[c->cur], c->L.scal, hipMemcpyDeviceToDevice,
                       c->stream);
  if (e == hipSuccess && c->L.nsc == 3)
    e = hipMemcpyAsync(o + c->L.pops + 2 * c->L.scal, c->tref[c->cur], c->L.scal,
                       hipMemcpyDeviceToDevice, c->stream);
  return hip_check(e, "lbm_get_state");
}

lbm_status lbm_set_state(lbm_ctx* c, const void* in, size_t bytes) {
  if (!c || !in) return fail(LBM_E_INVAL, "NULL argument");
  if (bytes < c->L.pops + (size_t)c->L.nsc * c->L.scal)
    return fail(LBM_E_NOMEM, "state buffer too small");
  const char* i = (const char*)in;
  hipError_t e = hipMemcpyAsync(c->pops[c->cur], i, c->L.pops, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->phip[c->cur], i + c->L.pops, c->L.scal, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->qp[c->cur], i + c->L.pops + c->L.scal, c->L.scal, hipMemcpyDeviceToDevice,
                       c->stream);
  if (e == hipSuccess && c->L.nsc == 3)
    e = hipMemcpyAsync(c->tref[c->cur], i + c->L.pops + 2 * c->L.scal, c->L.scal,
                       hipMemcpyDeviceToDevice, c->stream);
  c->initialized = 1;
  c->step = 0;
  c->tape_ready = 0;
  c->fresh_init = 0;
  return hip_check(e, "lbm_set_state");
}

lbm_status lbm_get_step(const lbm_ctx* c, int64_t* out) {
  if (!c || !out) return fail(LBM_E_INVAL, "NULL argument");
  *out = c->step;
  return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx* c) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  return hip_check(hipStreamSynchronize(c->stream), "lbm_sync");
}

void lbm_destroy(lbm_ctx* c) { delete c; }

const char* lbm_last_error(void) { return g_err.c_str(); }

const char* lbm_version(void) { return "lbm-phasechange-gfx950 0.1"; }

}  // extern "C"

// ===========================================================================
// Adjoint: sqrt(T) tape and the reverse sweep (2-D, FP32 / FP64 storage)
// ===========================================================================
namespace {

size_t state_bytes(const lbm_ctx* c) { return c->L.pops + (size_t)c->L.nsc * c->L.scal; }

lbm_status adjoint_supported(const lbm_ctx* c) {
  const lbm_params& p = c->prm;
  if (p.dim != 2) return fail(LBM_E_UNSUPPORTED, "adjoint is built for 2-D only");
  if (p.storage != LBM_ST_F32 && p.storage != LBM_ST_F64)
    return fail(LBM_E_UNSUPPORTED, "adjoint needs FP32 or FP64 storage");
  if (!c->ns || !c->heat) return fail(LBM_E_UNSUPPORTED, "adjoint needs LBM_NS | LBM_HEAT");
  if (p.bc[0] == LBM_BC_WALL && p.bc[1] == LBM_BC_WALL)
    return fail(LBM_E_UNSUPPORTED, "adjoint supports at most one walled axis");
  if (p.lat_g != LBM_D2Q9) return fail(LBM_E_UNSUPPORTED, "adjoint is built for D2Q9 populations");
  if (p.collision != LBM_COLL_BGK) return fail(LBM_E_UNSUPPORTED, "adjoint is built for BGK collision");
  if (p.grad_scheme != LBM_GRAD_CENTRAL)
    return fail(LBM_E_UNSUPPORTED, "adjoint is built for central gradients");
  if (p.flags & LBM_DIV_LOCAL) return fail(LBM_E_UNSUPPORTED, "adjoint is built without LBM_DIV_LOCAL");
  for (int a = 0; a < 3; ++a)
    for (int sd = 0; sd < 2; ++sd)
      if (p.f_bc[a][sd] != LBM_FBC_NOSLIP)
        return fail(LBM_E_UNSUPPORTED, "adjoint is built for no-slip faces of f");
  return LBM_OK;
}

void tape_shape(int64_t n, int64_t& k, int64_t& nsnap) {
  k = 1;
  while (k * k < n) ++k;
  nsnap = (n + k - 1) / k;
}

template <class Real>
NodeConst<Real> node_const(const lbm_ctx* c) {
  const KArgs<Real, Real> a = make_args<Real, Real>(c);
  NodeConst<Real> nc{};
  nc.rho_l = a.rho_l; nc.rho_g = a.rho_g; nc.K = a.K; nc.H = a.H;
  nc.four_over_W = a.four_over_W; nc.eps2 = a.eps2;
  for (int d = 0; d < 2; ++d) { nc.grav[d] = a.grav[d]; nc.body[d] = a.body[d]; }
  nc.nu_l = a.nu_l; nc.nu_g = a.nu_g; nc.alpha_l = a.alpha_l; nc.alpha_g = a.alpha_g;
  nc.Lcp = a.Lcp; nc.T_sat = a.T_sat; nc.theta_I = a.theta_I; nc.qcoef = a.qcoef;
  nc.prod_fac = a.prod_fac; nc.omega_g = a.omega_g; nc.M_over_cs2g = a.M_over_cs2g;
  nc.visc_linear = a.visc_linear; nc.geq_cac = a.geq_cac; nc.phase_change = a.phase_change;
  return nc;
}

size_t adj_ws_bytes(const lbm_ctx* c) {
  const size_t R = c->prm.storage == LBM_ST_F64 ? 8 : 4;
  const size_t plane = align256((size_t)c->L.slab * R);
  const size_t field = align256((size_t)c->prm.nx * c->prm.ny * R);
  size_t tot = (27 + 2 + 27 + LL_N + 3) * plane + 4 * field;
  for (int a = 0; a < 2; ++a)
    if (c->prm.bc[a] == LBM_BC_WALL) tot += 2 * align256((size_t)(a == 0 ? c->prm.ny : c->prm.nx) * R);
  return tot;
}

template <class Real>
lbm_status backward_t(lbm_ctx* c, const void* gphi, const void* gT, int32_t gdt, void* ws, void* d_phi0,
                      void* d_T0, void* d_Tw, int32_t tw_axis, int32_t tw_side, int32_t odt) {
  const size_t R = sizeof(Real);
  const long long nxy = (long long)c->prm.nx * c->prm.ny;
  const size_t plane = align256((size_t)c->L.slab * R);
  const size_t field = align256((size_t)nxy * R);
  char* p = (char*)ws;
  AdjArgs<Real> b{};
  b.lA = (Real*)p;       p += 27 * plane;
  b.lphip = (Real*)p;    p += plane;
  b.lqp = (Real*)p;      p += plane;
  b.lP = (Real*)p;       p += 27 * plane;
  b.lloc = (Real*)p;     p += LL_N * plane;
  b.fphi = (Real*)p;     p += plane;
  b.fux = (Real*)p;      p += plane;
  b.fuy = (Real*)p;      p += plane;
  Real* seed = (Real*)p; p += field;
  Real* seedT = (Real*)p; p += field;
  Real* dphi = (Real*)p; p += field;
  Real* dT0 = (Real*)p;  p += field;
  for (int a = 0; a < 2; ++a)
    for (int sd = 0; sd < 2; ++sd) b.lTw[a][sd] = nullptr;
  for (int a = 0; a < 2; ++a)
    if (c->prm.bc[a] == LBM_BC_WALL) {
      const size_t len = (size_t)(a == 0 ? c->prm.ny : c->prm.nx);
      for (int sd = 0; sd < 2; ++sd) {
        b.lTw[a][sd] = (Real*)p;
        p += align256(len * R);
        // accumulators start at zero (a fill kernel, not a memset node, so
        // that a captured graph replays it correctly)
        hipLaunchKernelGGL(k_fill, dim3((len + 255) / 256), dim3(256), 0, c->stream,
                           (void*)b.lTw[a][sd], (long long)len, 0.0, sizeof(Real) == 8 ? 1 : 0);
      }
    }
  b.nc = node_const<Real>(c);
  const int f64 = sizeof(Real) == 8;
  const size_t ss = state_bytes(c);
  char* snaps = c->tape;
  char* seg = c->tape + (size_t)c->tape_nsnap * ss;
  hipError_t e;
  // seed at the final state (the context's current state): phi^N and T^N
  // as the fields pass computes them, transposed onto lambda of X^N
  const int gdt64 = gdt == LBM_DT_F64 ? 1 : 0;
  if (gphi)
    hipLaunchKernelGGL(k_convert, dim3((nxy + 255) / 256), dim3(256), 0, c->stream, (void*)seed, f64,
                       gphi, gdt64, nxy);
  if (gT)
    hipLaunchKernelGGL(k_convert, dim3((nxy + 255) / 256), dim3(256), 0, c->stream, (void*)seedT, f64,
                       gT, gdt64, nxy);
  {
    KArgs<Real, Real> a = make_args<Real, Real>(c);
    e = launch_adj_seed2d(a, b, gphi ? seed : nullptr, gT ? seedT : nullptr, c->stream);
    if (e != hipSuccess) return hip_check(e, "adjoint seed");
    std::swap(b.lA, b.lP);   // the seed left lambda_A of X^N in lP
  }
  const int64_t N = c->tape_n, K = c->tape_k;
  auto adj_step = [&](const char* state) -> hipError_t {
    KArgs<Real, Real> a = make_args_blobs<Real, Real>(c, state, nullptr);
    hipError_t er = launch_adj_step2d(a, b, c->stream);
    std::swap(b.lA, b.lP);   // the step left lambda_A of its input state in lP
    return er;
  };
  if (c->tape_policy == LBM_TAPE_SQRT) {
    for (int64_t s = c->tape_nsnap - 1; s >= 0; --s) {
      const int64_t n0 = s * K, n1 = std::min<int64_t>(n0 + K, N);
      e = hipMemcpyAsync(seg, snaps + (size_t)s * ss, ss, hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return hip_check(e, "tape restore");
      for (int64_t k = 0; k + 1 < n1 - n0; ++k) {   // recompute the segment's states
        KArgs<Real, Real> a = make_args_blobs<Real, Real>(c, seg + (size_t)k * ss, seg + (size_t)(k + 1) * ss);
        e = launch_step2d(a, c->ns, c->heat, MODE_STEP, c->stream);
        if (e != hipSuccess) return hip_check(e, "segment recompute");
      }
      for (int64_t k = n1 - n0 - 1; k >= 0; --k) {
        e = adj_step(seg + (size_t)k * ss);
        if (e != hipSuccess) return hip_check(e, "adjoint step");
      }
    }
  } else {
    // slots 0 .. nsnap-1 hold checkpoints (slot 0: X^0); two work states follow
    char* w[2] = {snaps + (size_t)c->tape_nsnap * ss, snaps + (size_t)(c->tape_nsnap + 1) * ss};
    hipError_t er = hipSuccess;
    // X of `slot` advanced by `steps` steps (ping-pong through the work states)
    auto advance = [&](int64_t slot, int64_t steps) -> const char* {
      const char* cur = snaps + (size_t)slot * ss;
      for (int64_t k = 0; k < steps && er == hipSuccess; ++k) {
        char* out = w[k & 1];
        KArgs<Real, Real> a = make_args_blobs<Real, Real>(c, cur, out);
        er = launch_step2d(a, c->ns, c->heat, MODE_STEP, c->stream);
        cur = out;
      }
      return cur;
    };
    auto adj = [&](int64_t slot, int64_t k) -> bool {
      const char* x = advance(slot, k);
      if (er == hipSuccess) er = adj_step(x);
      return er == hipSuccess;
    };
    auto store = [&](int64_t slot, int64_t j, int64_t to) -> bool {
      const char* x = advance(slot, j);
      if (er == hipSuccess)
        er = hipMemcpyAsync(snaps + (size_t)to * ss, x, ss, hipMemcpyDeviceToDevice, c->stream);
      return er == hipSuccess;
    };
    binom_reverse(0, N, c->tape_nsnap - 1, 0, true, adj, store);
    if (er != hipSuccess) return hip_check(er, "binomial reverse sweep");
  }
  {  // initial condition: X^0 (the first slot of the last segment restored, or slot 0)
    const char* x0 = c->tape_policy == LBM_TAPE_SQRT ? seg : snaps;
    KArgs<Real, Real> a = make_args_blobs<Real, Real>(c, x0, nullptr);
    e = launch_adj_init2d(a, b, dphi, dT0, c->stream);
    if (e != hipSuccess) return hip_check(e, "adjoint init");
  }
  const int odt64 = odt == LBM_DT_F64 ? 1 : 0;
  if (d_phi0)
    hipLaunchKernelGGL(k_convert, dim3((nxy + 255) / 256), dim3(256), 0, c->stream, d_phi0, odt64,
                       (const void*)dphi, f64, nxy);
  if (d_T0)
    hipLaunchKernelGGL(k_convert, dim3((nxy + 255) / 256), dim3(256), 0, c->stream, d_T0, odt64,
                       (const void*)dT0, f64, nxy);
  if (d_Tw) {
    if (tw_axis < 0 || tw_axis > 1 || tw_side < 0 || tw_side > 1 || !b.lTw[tw_axis][tw_side])
      return fail(LBM_E_INVAL, "wall face (%d, %d) is not a walled face", tw_axis, tw_side);
    const long long len = tw_axis == 0 ? c->prm.ny : c->prm.nx;
    hipLaunchKernelGGL(k_convert, dim3((len + 255) / 256), dim3(256), 0, c->stream, d_Tw, odt64,
                       (const void*)b.lTw[tw_axis][tw_side], f64, len);
  }
  return hip_check(hipGetLastError(), "lbm_backward");
}

}  // namespace

extern "C" {

lbm_status lbm_tape_size(const lbm_ctx* c, int64_t nsteps, int32_t policy, size_t* bytes) {
  if (!c || !bytes) return fail(LBM_E_INVAL, "NULL argument");
  if (nsteps < 1) return fail(LBM_E_INVAL, "nsteps must be >= 1");
  if (policy == LBM_TAPE_BINOMIAL) {
    *bytes = (size_t)(binom_slots(nsteps) + 2) * state_bytes(c);
    return LBM_OK;
  }
  if (policy != LBM_TAPE_SQRT) return fail(LBM_E_INVAL, "unknown tape policy %d", policy);
  int64_t k, ns;
  tape_shape(nsteps, k, ns);
  *bytes = (size_t)(ns + k) * state_bytes(c);
  return LBM_OK;
}

lbm_status lbm_forward_taped(lbm_ctx* c, int64_t nsteps, int32_t policy, void* tape, size_t bytes) {
  if (!c || !tape) return fail(LBM_E_INVAL, "NULL argument");
  lbm_status st = adjoint_supported(c);
  if (st != LBM_OK) return st;
  if (!c->initialized) return fail(LBM_E_STATE, "lbm_forward_taped before initialisation");
  if (!c->fresh_init || c->step != 0)
    return fail(LBM_E_STATE,
                "lbm_forward_taped needs step 0 of lbm_init_fields with u0 == NULL (the reverse sweep "
                "differentiates that initialisation)");
  size_t need;
  st = lbm_tape_size(c, nsteps, policy, &need);
  if (st != LBM_OK) return st;
  if (bytes < need) return fail(LBM_E_NOMEM, "tape has %zu bytes, needs %zu", bytes, need);
  if (((uintptr_t)tape & 255) != 0) return fail(LBM_E_INVAL, "tape must be 256-byte aligned");
  int64_t k, ns;
  if (policy == LBM_TAPE_SQRT) {
    tape_shape(nsteps, k, ns);
  } else {   // binomial: k unused, ns checkpoint slots
    k = 0;
    ns = binom_slots(nsteps);
  }
  const size_t ss = state_bytes(c);
  char* t = (char*)tape;
  auto snap = [&](int64_t s) -> hipError_t {
    char* d = t + (size_t)s * ss;
    hipError_t e = hipMemcpyAsync(d, c->pops[c->cur], c->L.pops, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d + c->L.pops, c->phip[c->cur], c->L.scal, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d + c->L.pops + c->L.scal, c->qp[c->cur], c->L.scal, hipMemcpyDeviceToDevice,
                         c->stream);
    return e;
  };
  c->tape_ready = 0;
  hipError_t e = snap(0);
  if (e != hipSuccess) return hip_check(e, "tape snapshot");
  // binomial: the split states of the reverse sweep's first descent (its
  // right spine) are stored on the way
  std::vector<std::pair<int64_t, int64_t>> spine;
  if (policy == LBM_TAPE_BINOMIAL)
    binom_spine(nsteps, [&](int64_t step, int64_t slot) { spine.emplace_back(step, slot); });
  size_t next = 0;
  for (int64_t n = 1; n <= nsteps; ++n) {
    st = lbm_step(c, 1);
    if (st != LBM_OK) return st;
    if (policy == LBM_TAPE_SQRT && n % k == 0 && n < nsteps) {
      e = snap(n / k);
      if (e != hipSuccess) return hip_check(e, "tape snapshot");
    }
    if (next < spine.size() && n == spine[next].first) {
      e = snap(spine[next].second);
      if (e != hipSuccess) return hip_check(e, "tape snapshot");
      ++next;
    }
  }
  c->tape = t;
  c->tape_bytes = bytes;
  c->tape_n = nsteps;
  c->tape_k = k;
  c->tape_nsnap = ns;
  c->tape_policy = policy;
  c->tape_end_step = c->step;
  c->tape_ready = 1;
  return LBM_OK;
}

lbm_status lbm_adjoint_workspace_size(const lbm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(LBM_E_INVAL, "NULL argument");
  lbm_status st = adjoint_supported(c);
  if (st != LBM_OK) return st;
  *bytes = adj_ws_bytes(c);
  return LBM_OK;
}

lbm_status lbm_backward(lbm_ctx* c, const void* g_phi, const void* g_T, const void* g_u,
                        const void* g_p, int32_t seed_dtype, void* dev_ws, size_t ws_bytes,
                        void* d_phi0, void* d_T0, void* d_Twall, int32_t tw_axis, int32_t tw_side,
                        int32_t out_dtype) {
  if (!c || !dev_ws) return fail(LBM_E_INVAL, "NULL argument");
  if (!g_phi && !g_T) return fail(LBM_E_INVAL, "no seed: g_phi and g_T are both NULL");
  if (g_u || g_p) return fail(LBM_E_UNSUPPORTED, "seeds on u^N and p^N are not built");
  lbm_status st = adjoint_supported(c);
  if (st != LBM_OK) return st;
  if (!c->tape_ready) return fail(LBM_E_STATE, "lbm_backward without a current lbm_forward_taped tape");
  if (c->step != c->tape_end_step)
    return fail(LBM_E_STATE, "the context stepped after lbm_forward_taped");
  if (ws_bytes < adj_ws_bytes(c)) return fail(LBM_E_NOMEM, "adjoint workspace too small");
  if (((uintptr_t)dev_ws & 255) != 0) return fail(LBM_E_INVAL, "workspace must be 256-byte aligned");
  if ((seed_dtype != LBM_DT_F32 && seed_dtype != LBM_DT_F64) ||
      (out_dtype != LBM_DT_F32 && out_dtype != LBM_DT_F64))
    return fail(LBM_E_INVAL, "bad dtype");
  if (d_Twall && (tw_axis < 0 || tw_axis > 1 || tw_side < 0 || tw_side > 1 ||
                  c->prm.bc[tw_axis] != LBM_BC_WALL))
    return fail(LBM_E_INVAL, "wall face (%d, %d) is not a walled face", tw_axis, tw_side);
  if (c->prm.storage == LBM_ST_F64)
    return backward_t<double>(c, g_phi, g_T, seed_dtype, dev_ws, d_phi0, d_T0, d_Twall, tw_axis, tw_side,
                              out_dtype);
  return backward_t<float>(c, g_phi, g_T, seed_dtype, dev_ws, d_phi0, d_T0, d_Twall, tw_axis, tw_side,
                           out_dtype);
}

lbm_status lbm_backward_static(lbm_ctx* c, const void* g_phi, const void* g_T, const void* g_u,
                               const void* g_p, int32_t seed_dtype, void* d_phi0, void* d_T0,
                               void* d_Twall, int32_t tw_axis, int32_t tw_side, int32_t out_dtype) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  lbm_status st = adjoint_supported(c);
  if (st != LBM_OK) return st;
  const size_t need = adj_ws_bytes(c);
  if (need > kScratchBytes)
    return fail(LBM_E_NOMEM, "adjoint workspace of %zu bytes exceeds the static scratch of %zu bytes",
                need, kScratchBytes);
  if (!c->scratch) return fail(LBM_E_STATE, "no static scratch for this context");
  return lbm_backward(c, g_phi, g_T, g_u, g_p, seed_dtype, c->scratch, kScratchBytes, d_phi0, d_T0,
                      d_Twall, tw_axis, tw_side, out_dtype);
}

}  // extern "C"
