// Colour sum on MFMA for the mixed form (one event per lane, 64 events per wave).
//
// For each helicity the wave holds jamp[NCOLOR] (FP32 complex) per lane.
// q_e = x_e^T C x_e + y_e^T C y_e (x = Re jamp, y = Im jamp, C the integer
// colour matrix) is evaluated as the dense product  D = X C  on
// v_mfma_f32_16x16x32_f16 (M = 64 events in 4 tiles, N = K = colours padded to
// 32) followed by the row-wise dot q_e = sum_k X[e][k] D[e][k]:
//   * per (event, helicity) a power-of-two scale 2^-s brings max|jamp| below 1
//     (exact), then X = hi + lo with hi = f16(x), lo = f16(x - hi): about 22
//     significant bits;
//   * C has at most 10 significant bits (integers <= 512 for 4 gluons), so it
//     is exact in FP16 and hi*C, lo*C are exact in the FP32 accumulator;
//   * X goes through LDS to reach the MFMA operand layout (row = event,
//     8 consecutive colours per lane); C is loaded once per kernel into the B
//     operand registers.
// MFMA operand layout (16x16x32, wave64): lane l supplies A[l%16][8(l/16)+j]
// and B[8(l/16)+j][l%16] for j = 0..7, and receives D[4(l/16)+i][l%16] for
// i = 0..3.  Only the pairing of A's and B's K slots matters for the product,
// and both use the same slots.
#pragma once
#include <hip/hip_runtime.h>

#include "helas.hpp"

namespace me {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4v mfma16x16x32(half8 a, half8 b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave LDS: 4 planes (Re hi, Re lo, Im hi, Im lo) of [64 events][32 colours]
// halves plus 64 floats for the results = 16640 bytes.
constexpr int kColourLdsHalves = 4 * 64 * 32;
constexpr int kColourLdsBytes = kColourLdsHalves * 2 + 64 * 4;

template <int NC>
struct ColourB {
  half8 b[2];   // B operand for N-tiles 0 and 1
};

// B operand registers from the integer colour matrix (row-major NC x NC).
template <int NC>
__device__ __forceinline__ ColourB<NC> colour_b(const int* cmat, int lane) {
  ColourB<NC> r;
#pragma unroll
  for (int n = 0; n < 2; ++n) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * (lane / 16) + j, col = 16 * n + lane % 16;
      r.b[n][j] = (k < NC && col < NC) ? _Float16(float(cmat[k * NC + col])) : _Float16(0.0f);
    }
  }
  return r;
}

// Returns sum_kl C_kl Re(conj(jamp_k) jamp_l) for this lane's event; every
// lane of the wave must call it (uniform control flow).
template <int NC>
__device__ __forceinline__ float colour_sum_mfma(const cx<float> (&jamp)[NC], const ColourB<NC>& B,
                                                 _Float16* lds, int lane) {
  static_assert(NC <= 32, "MFMA colour sum handles up to 32 colour flows");
  float* qbuf = reinterpret_cast<float*>(lds + kColourLdsHalves);
  // power-of-two scale: max |component| -> [0.5, 1)
  float m = 0.f;
#pragma unroll
  for (int k = 0; k < NC; ++k) m = fmaxf(m, fmaxf(fabsf(jamp[k].r), fabsf(jamp[k].i)));
  int ex = 0;
  (void)frexpf(m, &ex);
  // write hi/lo planes, rows = events, 32 colours (zero padded)
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    float xr = 0.f, xi = 0.f;
    if (k < NC) { xr = ldexpf(jamp[k].r, -ex); xi = ldexpf(jamp[k].i, -ex); }
    const _Float16 hr = _Float16(xr), hi = _Float16(xi);
    lds[(0 * 64 + lane) * 32 + k] = hr;
    lds[(1 * 64 + lane) * 32 + k] = _Float16(xr - float(hr));
    lds[(2 * 64 + lane) * 32 + k] = hi;
    lds[(3 * 64 + lane) * 32 + k] = _Float16(xi - float(hi));
  }
  wave_lds_sync();
  const int g = lane / 16, c16 = lane % 16;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {           // real, imaginary
      const half8 ahi = *reinterpret_cast<const half8*>(&lds[((2 * ri) * 64 + 16 * t + c16) * 32 + 8 * g]);
      const half8 alo = *reinterpret_cast<const half8*>(&lds[((2 * ri + 1) * 64 + 16 * t + c16) * 32 + 8 * g]);
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        if (16 * n >= NC) continue;
        float4v d = {0.f, 0.f, 0.f, 0.f};
        d = mfma16x16x32(ahi, B.b[n], d);
        d = mfma16x16x32(alo, B.b[n], d);
        // this lane holds D[e][k] for e = 16t + 4g + i, k = 16n + c16
        const int k = 16 * n + c16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = 16 * t + 4 * g + i;
          const float x = float(lds[((2 * ri) * 64 + e) * 32 + k]) + float(lds[((2 * ri + 1) * 64 + e) * 32 + k]);
          part[i] += x * d[i];
        }
      }
    }
    // sum over the 16 lanes of the group (colour index)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = part[i];
      v += __shfl_xor(v, 8, 16);
      v += __shfl_xor(v, 4, 16);
      v += __shfl_xor(v, 2, 16);
      v += __shfl_xor(v, 1, 16);
      if (c16 == i) qbuf[16 * t + 4 * g + i] = v;
    }
  }
  wave_lds_sync();
  const float q = qbuf[lane];
  wave_lds_sync();   // the next call overwrites the planes
  return ldexpf(q, 2 * ex);
}

}  // namespace me
