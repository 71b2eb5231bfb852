// Measurement probe (not part of the method): the HBM access pattern of
// one 2-D FP32 step with none of its arithmetic.  Every interior node of an
// nx x ny grid (pitch nx) copies 29 planes of A into B: the 27 population
// planes (three D2Q9 families) read at the pull offsets x - c_i, and the
// two lagged planes (phi_prev, q_prev) read in place; all 29 written in
// place.  One node per lane, as the step kernel.  bench.py times it next to
// a plain device copy of the same byte count, to give the bandwidth that
// this pattern reaches on the device without any compute.
#include <hip/hip_runtime.h>

namespace {

constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

__global__ __launch_bounds__(256) void k_pull_pattern(const float* __restrict__ A,
                                                      float* __restrict__ B, int nx, int ny,
                                                      long long slab) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  // interior nodes only: every pull offset stays inside its plane
  if (x < 1 || x >= nx - 1 || y < 1 || y >= ny - 1) return;
  const long long node = (long long)y * nx + x;
  float v[29];
#pragma unroll
  for (int p = 0; p < 29; ++p) {
    const int i = p % 9;
    const long long off = p < 27 ? (long long)(kCx[i] + kCy[i] * nx) : 0;
    v[p] = A[p * slab + node - off];
  }
#pragma unroll
  for (int p = 0; p < 29; ++p) B[p * slab + node] = v[p];
}

}  // namespace

// A and B: device buffers of 29 * nx * ny floats each.  Returns a hipError_t
// code (0 on success); rejects grids smaller than 3 x 3.
extern "C" int stream_probe_pull_pattern(const float* A, float* B, int nx, int ny, void* stream) {
  if (nx < 3 || ny < 3 || !A || !B) return (int)hipErrorInvalidValue;
  const long long slab = (long long)nx * ny;
  hipLaunchKernelGGL(k_pull_pattern, dim3((nx + 255) / 256, ny), dim3(256), 0,
                     (hipStream_t)stream, A, B, nx, ny, slab);
  return (int)hipGetLastError();
}
