// Measurement probes for bench.py (not part of the method, not in the
// library's C ABI): what the device gives the step's memory traffic with
// none of its arithmetic.
//
//   stream_probe_pull_pattern: the HBM access pattern of one 2-D FP32 step.
//     Every interior node of an nx x ny grid (pitch nx) copies 29 planes of
//     A into B: the 27 population planes (three D2Q9 families) read at the
//     pull offsets x - c_i, and the two lagged planes (phi_prev, q_prev) read
//     in place; all 29 written in place.  One node per lane, as the step.
//   stream_probe_copy16: a plain streaming copy of n bytes with 16-byte
//     loads and stores (four per lane, consecutive lanes on consecutive 16-byte
//     words), optionally with non-temporal hints: the copy ceiling of the
//     device for a given data volume.
#include <hip/hip_runtime.h>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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

// Four 16-byte words per lane: word k of block b, lane t is
// b * 1024 + k * 256 + t, so each load instruction of a wave covers 1 KiB of
// consecutive bytes.  n16 is the word count; the tail is bounds-checked.
template <bool NT>
__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ a, u32x4* __restrict__ b,
                                                long long n16) {
  const long long base = (long long)blockIdx.x * 1024 + threadIdx.x;
  u32x4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long i = base + k * 256;
    if (i < n16) v[k] = NT ? __builtin_nontemporal_load(a + i) : a[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long i = base + k * 256;
    if (i < n16) {
      if (NT)
        __builtin_nontemporal_store(v[k], b + i);
      else
        b[i] = v[k];
    }
  }
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

// Copy nbytes (a multiple of 16; src and dst 16-byte aligned) from src to
// dst.  nontemporal != 0 uses non-temporal loads and stores.  Returns a
// hipError_t code (0 on success).
extern "C" int stream_probe_copy16(const void* src, void* dst, long long nbytes, int nontemporal,
                                   void* stream) {
  if (!src || !dst || nbytes <= 0 || (nbytes & 15) || ((size_t)src & 15) || ((size_t)dst & 15))
    return (int)hipErrorInvalidValue;
  const long long n16 = nbytes / 16;
  const long long blocks = (n16 + 1023) / 1024;
  if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  if (nontemporal)
    hipLaunchKernelGGL(k_copy16<true>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4*)src, (u32x4*)dst, n16);
  else
    hipLaunchKernelGGL(k_copy16<false>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4*)src, (u32x4*)dst, n16);
  return (int)hipGetLastError();
}
