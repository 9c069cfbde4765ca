// Colour sum on MFMA for the mixed form (one event per lane, 64 events per wave),
// with hi+lo jamps in FP16 or BF16 (below) or with FP32 operands (further down).
//
// For each helicity the wave holds jamp[NCOLOR] (FP32 complex) per lane.
// q_e = x_e^T C x_e + y_e^T C y_e (x = Re jamp, y = Im jamp, C the integer
// colour matrix) is evaluated as the dense product  D' = C X^T  on
// v_mfma_f32_16x16x32_f16 or _bf16 (M = colours, N = 64 events in 4 tiles,
// K = colours, padded to 32), followed by each lane's dot of its own row of D
// with its own jamps:
//   * FP16: per (event, helicity) a power-of-two scale 2^-s brings max|jamp|
//     below 1 (exact), then X = hi + lo with hi = f16(x), lo = f16(x - hi):
//     about 22 significant bits;
//   * BF16: hi = bf16(x), lo = bf16(x - hi), both rounded to nearest even
//     (x - hi is exact in FP32), so |x - hi - lo| <= 2^-8 |x - hi| <=
//     2^-16 |x|: 16 significant bits; BF16 has the exponent range of FP32,
//     so no scale is needed;
//   * C has at most 10 significant bits (integers <= 512 for 4 gluons), so it
//     is exact in FP16; the colour matrices of 6..32 flows have at most 7
//     and are exact in BF16 (8 bits); C*hi and C*lo are exact in the FP32
//     accumulator;
//   * C is the A operand, loaded once per kernel into registers; X reaches
//     the B operand layout through LDS (8 consecutive colours of one event per
//     lane, one 128-bit load); a lane's D' fragment is 4 consecutive colours
//     of one event, stored with one 128-bit write; each lane then reads its own
//     row back.  The staging holds only the colours there are (rows of KP =
//     8 ceil(NC/8) colours, products of MP = 16 ceil(NC/16)): lane groups
//     whose K slots are all padding take zero B operands without reading LDS,
//     and the smaller footprint leaves room for more waves per CU.
// MFMA operand layout (16x16x32, wave64): lane l supplies A[l%16][8(l/16)+j]
// and B[8(l/16)+j][l%16] for j = 0..7, and receives D[4(l/16)+i][l%16] for
// i = 0..3.  Only the pairing of A's and B's K slots matters for the product,
// and both use the same slots.
#pragma once
#include <hip/hip_runtime.h>

#include "helas.hpp"

namespace me {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4v mfma16x16x32(half8 a, half8 b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float4v mfma16x16x32(bf16x8 a, bf16x8 b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Staging of NC colour flows: per wave, hi and lo planes [64 events][KP] of
// 2-byte elements and the product rows [64 events][MP] of floats, reused for
// the real and the imaginary part (g g > t t~ g g: 14 KB; 6 flows: 6 KB).
template <int NC>
struct ColourTile {
  static constexpr int KP = 8 * ((NC + 7) / 8), MP = 16 * ((NC + 15) / 16);
  static constexpr int kLdsBytes = 2 * 64 * KP * 2 + 64 * MP * 4;
};

// hi+lo element types: FP16 with the per-event power-of-two scale (its
// exponent range is narrow), BF16 without
template <class H>
struct HiLo;
template <>
struct HiLo<_Float16> {
  typedef half8 vec;
  static constexpr bool kScale = true;
};
template <>
struct HiLo<__bf16> {
  typedef bf16x8 vec;
  static constexpr bool kScale = false;
};

template <int NC, class H = _Float16>
struct ColourA {
  typename HiLo<H>::vec a[2];   // A operand (colour matrix) for colour tiles 0 and 1
};

// A operand registers from the integer colour matrix (row-major NC x NC):
// lane l holds C[16m + l%16][8(l/16) + j].
template <int NC, class H = _Float16>
__device__ __forceinline__ ColourA<NC, H> colour_a(const int* cmat, int lane) {
  ColourA<NC, H> r;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int row = 16 * m + lane % 16, k = 8 * (lane / 16) + j;
      r.a[m][j] = H((row < NC && k < NC) ? float(cmat[row * NC + k]) : 0.0f);
    }
  }
  return r;
}

// Returns sum_kl C_kl Re(conj(jamp_k) jamp_l) for this lane's event; every
// lane of the wave must call it (uniform control flow).  lds_wave holds
// ColourTile<NC>::kLdsBytes.
template <int NC, class H = _Float16>
__device__ __forceinline__ float colour_sum_mfma(const cx<float> (&jamp)[NC], const ColourA<NC, H>& A,
                                                 void* lds_wave, int lane) {
  static_assert(NC <= 32, "MFMA colour sum handles up to 32 colour flows");
  typedef typename HiLo<H>::vec V;
  constexpr int KP = ColourTile<NC>::KP, MP = ColourTile<NC>::MP;
  H* phi = reinterpret_cast<H*>(lds_wave);
  H* plo = phi + 64 * KP;
  float* drow = reinterpret_cast<float*>(plo + 64 * KP);
  int ex = 0;
  if constexpr (HiLo<H>::kScale) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < NC; ++k) m = fmaxf(m, fmaxf(fabsf(jamp[k].r), fabsf(jamp[k].i)));
    (void)frexpf(m, &ex);
  }
  const int g = lane / 16, c16 = lane % 16;
  const bool live = 8 * g < KP;   // this lane group's K slots hold colours
  float q = 0.f;
#pragma unroll
  for (int ri = 0; ri < 2; ++ri) {
    // this lane's event row: hi/lo pairs, 8 colours per 128-bit store (the
    // padding colours are zeros: they meet zero columns of C, and must not
    // be NaN)
#pragma unroll
    for (int c = 0; c < KP / 8; ++c) {
      V h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 8 * c + j;
        float x = k < NC ? (ri ? jamp[k < NC ? k : 0].i : jamp[k < NC ? k : 0].r) : 0.f;
        if constexpr (HiLo<H>::kScale) x = ldexpf(x, -ex);
        const H hx = H(x);
        h[j] = hx;
        l[j] = H(x - float(hx));
      }
      *reinterpret_cast<V*>(&phi[lane * KP + 8 * c]) = h;
      *reinterpret_cast<V*>(&plo[lane * KP + 8 * c]) = l;
    }
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      V bhi = {}, blo = {};
      if (live) {
        bhi = *reinterpret_cast<const V*>(&phi[(16 * t + c16) * KP + 8 * g]);
        blo = *reinterpret_cast<const V*>(&plo[(16 * t + c16) * KP + 8 * g]);
      }
#pragma unroll
      for (int mt = 0; mt < MP / 16; ++mt) {
        float4v d = {0.f, 0.f, 0.f, 0.f};
        d = mfma16x16x32(A.a[mt], bhi, d);
        d = mfma16x16x32(A.a[mt], blo, d);
        // d[i] = (C X^T)[16mt + 4g + i][16t + c16]
        *reinterpret_cast<float4v*>(&drow[(16 * t + c16) * MP + 16 * mt + 4 * g]) = d;
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < (NC + 3) / 4; ++c) {
      const float4v d = *reinterpret_cast<const float4v*>(&drow[lane * MP + 4 * c]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 4 * c + i;
        if (k < NC) {
          const float x = ri ? jamp[k].i : jamp[k].r;
          q += (HiLo<H>::kScale ? ldexpf(x, -ex) : x) * d[i];
        }
      }
    }
    wave_lds_sync();   // the next pass overwrites the planes and rows
  }
  return HiLo<H>::kScale ? ldexpf(q, 2 * ex) : q;
}

// ---------------------------------------------------------------------------
// The same contraction with FP32 operands on v_mfma_f32_16x16x4_f32: jamps
// and the integer colour matrix are exact FP32 operands, so there is no
// scaling and no hi/lo split, and the result has the rounding of an FP32
// accumulation only.  K runs over colours in steps of 4; in step s lane group
// g supplies colour kappa = S*g + s (S = ceil(NC/4) steps), so each lane
// reads S consecutive colours of one event from LDS.
// Operand layout (16x16x4, wave64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16], and receives D[4(l/16)+i][l%16].

__device__ __forceinline__ float4v mfma16x16x4f32(float a, float b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int NC>
struct ColourA32 {
  static constexpr int S = (NC + 3) / 4;
  float a[2][S];   // A operand (colour matrix) for colour tiles 0 and 1, K steps
};

template <int NC>
__device__ __forceinline__ ColourA32<NC> colour_a32(const int* cmat, int lane) {
  ColourA32<NC> r;
  constexpr int S = ColourA32<NC>::S;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int row = 16 * m + lane % 16, k = S * (lane / 16) + st;
      r.a[m][st] = (row < NC && k < NC) ? float(cmat[row * NC + k]) : 0.f;
    }
  return r;
}

// Per-wave LDS: x rows [64][32] floats (8 KB) and product rows [64][32] (8 KB).
constexpr int kColourLds32Bytes = 2 * 64 * 32 * 4;

template <int NC>
__device__ __forceinline__ float colour_sum_mfma32(const cx<float> (&jamp)[NC], const ColourA32<NC>& A,
                                                   void* lds_wave, int lane) {
  static_assert(NC <= 32, "MFMA colour sum handles up to 32 colour flows");
  constexpr int S = ColourA32<NC>::S;
  float* xrow = reinterpret_cast<float*>(lds_wave);
  float* drow = xrow + 64 * 32;
  const int g = lane / 16, c16 = lane % 16;
  float q = 0.f;
#pragma unroll
  for (int ri = 0; ri < 2; ++ri) {
#pragma unroll
    for (int c = 0; c < (NC + 3) / 4; ++c) {
      float4v v;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 4 * c + i;
        v[i] = k < NC ? (ri ? jamp[k < NC ? k : 0].i : jamp[k < NC ? k : 0].r) : 0.f;
      }
      *reinterpret_cast<float4v*>(&xrow[lane * 32 + 4 * c]) = v;
    }
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float b[S];
#pragma unroll
      for (int st = 0; st < S; ++st) b[st] = xrow[(16 * t + c16) * 32 + S * g + st];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        if (16 * mt >= NC) continue;
        float4v d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < S; ++st) d = mfma16x16x4f32(A.a[mt][st], b[st], d);
        *reinterpret_cast<float4v*>(&drow[(16 * t + c16) * 32 + 16 * mt + 4 * g]) = d;
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < (NC + 3) / 4; ++c) {
      const float4v d = *reinterpret_cast<const float4v*>(&drow[lane * 32 + 4 * c]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 4 * c + i;
        if (k < NC) q += (ri ? jamp[k].i : jamp[k].r) * d[i];
      }
    }
    wave_lds_sync();
  }
  return q;
}

}  // namespace me
