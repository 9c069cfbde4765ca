// GPU-assisted batch unweighting (paper, Sec. 3 and Table 2): the weights of
// a batch, w_i = |M|^2_i * f_i with f_i the Jacobian x PDF factor the host
// sends, are formed on the device where the matrix elements already are, and
// the batch maximum is reduced in parallel so that only one scalar returns.
//
// HBM-bound: 16 bytes read per event (|M|^2 and f), 8 written when the
// weights are kept.  One grid-stride kernel of at most 1024 blocks: each lane
// keeps a running maximum, the wave reduces it with cross-lane moves, the
// block through LDS, and one atomic per block lands on the bit pattern of
// the (non-negative) maximum (a few hundred atomics on one address instead
// of one per wave).  A one-lane fill kernel clears the result first, so the
// pair of launches is stream-ordered and safe to capture in a graph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "me.h"

namespace {

__global__ void max_weight_init(unsigned long long* d_max_bits) { *d_max_bits = 0ull; }

__global__ __launch_bounds__(256) void max_weight_kernel(const double* __restrict__ me,
                                                         const double* __restrict__ f, int64_t n,
                                                         double* __restrict__ w,
                                                         unsigned long long* __restrict__ d_max_bits) {
  double m = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    // weights are non-negative; NaN and negative inputs are clamped to 0 so the
    // integer order of the bit patterns stays the numeric order
    double x = me[i] * f[i];
    if (!(x > 0.0)) x = 0.0;
    if (w) w[i] = x;
    m = fmax(m, x);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  __shared__ double wmax[4];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    if (m > 0.0) atomicMax(d_max_bits, static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}

}  // namespace

extern "C" me_status me_max_weight(const double* d_me, const double* d_factor, int64_t nevt, double* d_w,
                                   double* d_max, void* hip_stream) {
  if (nevt < 0 || !d_max || (nevt > 0 && (!d_me || !d_factor))) return ME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  auto* bits = reinterpret_cast<unsigned long long*>(d_max);
  hipLaunchKernelGGL(max_weight_init, dim3(1), dim3(1), 0, s, bits);
  if (nevt > 0) {
    // four blocks per CU, grid-stride beyond that
    int64_t blocks = (nevt + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(max_weight_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, d_me, d_factor, nevt, d_w,
                       bits);
  }
  return hipGetLastError() == hipSuccess ? ME_OK : ME_EHIP;
}
