// Internal launcher interface between the C ABI (lbm_abi.cpp) and the HIP
// kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include "lbm_device.h"

namespace lbm {

enum { MODE_STEP = 0, MODE_MACRO = 1 };
constexpr int NPART = 5;   // diagnostics partials per block

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ inline double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

// Deterministic block reduction of the FP64 diagnostics (wave shuffles, then
// the waves in order); writes NPART values at partials[blockIdx.x * NPART].
__device__ inline void block_partials(double s_phi, double s_T, double s_phip, double umax,
                                      double bad, double* partials) {
  __shared__ double red[NPART][16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  s_phi = wave_sum_d(s_phi);
  s_T = wave_sum_d(s_T);
  s_phip = wave_sum_d(s_phip);
  umax = wave_max_d(umax);
  bad = wave_sum_d(bad);
  if (lane == 0) {
    red[0][wv] = s_phi;
    red[1][wv] = s_T;
    red[2][wv] = s_phip;
    red[3][wv] = umax;
    red[4][wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double o[NPART] = {0, 0, 0, 0, 0};
    for (int w = 0; w < nw; ++w) {
      o[0] += red[0][w];
      o[1] += red[1][w];
      o[2] += red[2][w];
      o[3] = fmax(o[3], red[3][w]);
      o[4] += red[4][w];
    }
    for (int k = 0; k < NPART; ++k) partials[(long long)blockIdx.x * NPART + k] = o[k];
  }
}

#define LBM_DECL(STORE, REAL)                                                                \
  hipError_t launch_step2d(const KArgs<REAL, STORE>& a, int ns, int heat, int mode,          \
                           hipStream_t st);                                                  \
  hipError_t launch_init2d(const KArgs<REAL, STORE>& a, int ns, int heat, const void* phi0,  \
                           const void* T0, const void* u0, const void* p0, int f64,          \
                           hipStream_t st);                                                  \
  hipError_t launch_step3d(const KArgs<REAL, STORE>& a, int ns, int heat, int mode,          \
                           hipStream_t st);                                                  \
  hipError_t launch_init3d(const KArgs<REAL, STORE>& a, int ns, int heat, const void* phi0,  \
                           const void* T0, const void* u0, const void* p0, int f64,          \
                           hipStream_t st);
LBM_DECL(double, double)
LBM_DECL(float, float)
LBM_DECL(__half, float)
LBM_DECL(__hip_bfloat16, float)
#undef LBM_DECL

int step2d_blocks(int nx, int ny);
int step3d_blocks(int nx, int ny, int nz);

namespace adj { template <class Real> struct NodeConst; }
template <class Real> struct AdjArgs;
#define LBM_ADJ_DECL(REAL)                                                                    \
  hipError_t launch_adj_step2d(const KArgs<REAL, REAL>& a, const AdjArgs<REAL>& b,             \
                               hipStream_t st);                                               \
  hipError_t launch_adj_seed2d(const KArgs<REAL, REAL>& a, const AdjArgs<REAL>& b,             \
                               const REAL* g, const REAL* gT, hipStream_t st);                \
  hipError_t launch_adj_init2d(const KArgs<REAL, REAL>& a, const AdjArgs<REAL>& b, REAL* dphi0, \
                               REAL* dT0, hipStream_t st);
LBM_ADJ_DECL(float)
LBM_ADJ_DECL(double)
#undef LBM_ADJ_DECL

// Sum the per-block partials in a fixed order into out[NPART] (device).
hipError_t launch_reduce(const double* partials, int nblocks, double* out, hipStream_t st);

}  // namespace lbm
