// Event-parallel |M|^2 kernels for gfx950: one event per lane, the helicity
// loop inside the lane (uniform across the wave, no divergence), the colour
// sum and the helicity sum fused in the same kernel so that only the momenta
// are read from and one double per event is written to HBM.
//
// Per process the generator supplies  struct Proc { NPAR, NCOLOR, NHEL, CDEN,
// IDEN, amplitudes<T>(), colour_sum<T>() }.  T = double is the FP64 form;
// T = float is the mixed form (FP32 wavefunctions and vertices, FP64
// momenta, p^2, propagator denominators and helicity-sum accumulation).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "colour_mfma.hpp"
#include "epilogue.hpp"
#include "helas.hpp"
#include "me_types.h"
#include "split.hpp"

namespace me {

template <class T> __device__ __forceinline__ mom<T> neg(const mom<T>& k) {
  return mom<T>{{-k.k[0], -k.k[1], -k.k[2], -k.k[3]}};
}
// 1/(K^2 - m^2 + i m w) from the invariant K^2, formed in FP64 and rounded to T.
template <class T> __device__ __forceinline__ cx<T> prop_den(double k2, double m, double w) {
  const double a = k2 - m * m, b = m * w;
  const double r = 1.0 / (a * a + b * b);
  return cx<T>{T(a * r), T(-b * r)};
}

template <class P, class T>
__global__ __launch_bounds__(256) void me_kernel(const double* __restrict__ mom, int64_t nevt,
                                                 double* __restrict__ out, double* __restrict__ out_hel,
                                                 const MeParams prm) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  double p[P::NPAR][4];
  load_on_shell<P::MASSIVE>(mom + e * (4 * P::NPAR), p, prm.mt);
  double acc = 0.0;
  for (int ih = 0; ih < prm.nhel; ++ih) {
    // Momentum sums and propagator factors are recomputed per helicity where
    // they are used; hiding p from loop-invariant code motion keeps the
    // compiler from hoisting them all and holding them in registers.
#pragma unroll
    for (int i = 0; i < P::NPAR; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) asm volatile("" : "+v"(p[i][c]));
    const unsigned hel = prm.hel[ih];
    cx<T> jamp[P::NCOLOR];
    P::template amplitudes<T>(p, hel, prm, jamp);
    const double q = double(P::template colour_sum<T>(jamp));
    if (out_hel) out_hel[e * P::NHEL + hel] = q * (P::coupling_factor(prm) / P::CDEN);
    acc += q;
  }
  if (out) store_me(prm, out, e, acc * (P::coupling_factor(prm) / (P::CDEN * P::IDEN)));
}

// Propagator factors and polarisation bases (eps_base) of one event in LDS,
// formed once per event before the helicity loop (they do not depend on the
// helicity): slot s of event t at base[s * S + t] (S events per block), so a
// wave's 64 reads of one slot are contiguous; a polarisation base takes five
// slots.  The per-iteration offset passes through an empty asm statement, so
// the reads stay inside the helicity loop where the schedule put them instead
// of being hoisted out of it and held in registers across the loop.
// With M, the cache also holds the schedule's momentum sums (one 16-byte
// entry per slot) and both helicity states of each external spinor (two
// 16-byte halves per state, in separate planes), for the FP32 form: the
// helicity program then reads no momenta at all.
template <class T, int S = 256, bool M = false>
struct LdsKinCache {
  static constexpr bool kCached = true;
  static constexpr bool kMom = M;
  static constexpr bool kLc = false;   // cached factors already hold the light-cone forms
  __device__ __forceinline__ double lcs(int) const { return 0.0; }
  __device__ __forceinline__ double pair(int) const { return 0.0; }
  T* re;
  cx<T>* cxs;
  T* eb;
  int off;
  __device__ __forceinline__ T r(int s) const { return re[s * S + off]; }
  __device__ __forceinline__ cx<T> c(int s) const { return cxs[s * S + off]; }
  __device__ __forceinline__ T r_opq(int s) const {
    int o = off;
    asm volatile("" : "+v"(o));
    return re[s * S + o];
  }
  __device__ __forceinline__ cx<T> c_opq(int s) const {
    int o = off;
    asm volatile("" : "+v"(o));
    return cxs[s * S + o];
  }
  __device__ __forceinline__ epsw<T> eps_at(int j, int o, int lam, bool conj_out) const {
    const T* b = eb + 5 * j * S + o;
    return eps_from_base<T>(b[0], b[S], b[2 * S], b[3 * S], b[4 * S], lam, conj_out);
  }
  __device__ __forceinline__ epsw<T> eps(int j, int lam, bool conj_out) const { return eps_at(j, off, lam, conj_out); }
  __device__ __forceinline__ epsw<T> eps_opq(int j, int lam, bool conj_out) const {
    int o = off;
    asm volatile("" : "+v"(o));
    return eps_at(j, o, lam, conj_out);
  }
  __device__ __forceinline__ void set_eps(int j, T a0, T a1, T a2, T b0, T b1) {
    T* b = eb + 5 * j * S + off;
    b[0] = a0; b[S] = a1; b[2 * S] = a2; b[3 * S] = b0; b[4 * S] = b1;
  }
  __device__ __forceinline__ void set_r(int s, T v) { re[s * S + off] = v; }
  __device__ __forceinline__ void set_c(int s, cx<T> v) { cxs[s * S + off] = v; }
  // momentum sums and spinors (M only), in 16-byte chunks (float4 for
  // FP32, double2 for FP64: NV chunks per momentum, 2 NV per spinor state):
  // chunk h of slot s of event t at km[(s NV + h) S + t]; chunk h of state
  // lam of spinor slot j at ksp[((2j + (lam > 0)) 2 NV + h) S + t]
  using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  static constexpr int NV = sizeof(T) / 4;
  V* km = nullptr;
  V* ksp = nullptr;
  __device__ __forceinline__ static void unpack(const V& v, T* x) {
    if constexpr (sizeof(T) == 8) { x[0] = v.x; x[1] = v.y; }
    else { x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w; }
  }
  __device__ __forceinline__ static V pack(const T* x) {
    if constexpr (sizeof(T) == 8) return V{x[0], x[1]};
    else return V{x[0], x[1], x[2], x[3]};
  }
  __device__ __forceinline__ mom<T> k_at(int s, int o) const {
    mom<T> K;
#pragma unroll
    for (int h = 0; h < NV; ++h) unpack(km[(s * NV + h) * S + o], K.k + h * (4 / NV));
    return K;
  }
  __device__ __forceinline__ mom<T> k(int s) const { return k_at(s, off); }
  __device__ __forceinline__ mom<T> k_opq(int s) const {
    int o = off;
    asm volatile("" : "+v"(o));
    return k_at(s, o);
  }
  __device__ __forceinline__ wf<T> sp_at(int j, int lam, int o) const {
    const int b = (2 * j + (lam > 0 ? 1 : 0)) * 2 * NV;
    T x[8];
#pragma unroll
    for (int h = 0; h < 2 * NV; ++h) unpack(ksp[(b + h) * S + o], x + h * (4 / NV));
    wf<T> w;
#pragma unroll
    for (int c = 0; c < 4; ++c) w.c[c] = cx<T>{x[2 * c], x[2 * c + 1]};
    return w;
  }
  __device__ __forceinline__ wf<T> sp(int j, int lam) const { return sp_at(j, lam, off); }
  __device__ __forceinline__ wf<T> sp_opq(int j, int lam) const {
    int o = off;
    asm volatile("" : "+v"(o));
    return sp_at(j, lam, o);
  }
  __device__ __forceinline__ void set_k(int s, const mom<T>& K) {
#pragma unroll
    for (int h = 0; h < NV; ++h) km[(s * NV + h) * S + off] = pack(K.k + h * (4 / NV));
  }
  __device__ __forceinline__ void set_sp(int j, int lam, const wf<T>& w) {
    const int b = (2 * j + (lam > 0 ? 1 : 0)) * 2 * NV;
    T x[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) { x[2 * c] = w.c[c].r; x[2 * c + 1] = w.c[c].i; }
#pragma unroll
    for (int h = 0; h < 2 * NV; ++h) ksp[(b + h) * S + off] = pack(x + h * (4 / NV));
  }
};

// The kinematic cache in LDS with the vector-ALU colour sum (256-thread
// blocks; per thread KC_RE real and KC_CX complex propagator-factor slots and
// KC_EPS polarisation bases of the form's schedule).  T = float: mixed form
// (out_hel unused); T = double: FP64 form (out_hel as in me_kernel).
template <class P, class T>
__global__ __launch_bounds__(256) void me_kernel_kc(const double* __restrict__ mom, int64_t nevt,
                                                    double* __restrict__ out, double* __restrict__ out_hel,
                                                    const MeParams prm) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int KR = F64 ? P::KC_RE_F64 : P::KC_RE_F32;
  constexpr int KC = F64 ? P::KC_CX_F64 : P::KC_CX_F32;
  constexpr int KE = F64 ? P::KC_EPS_F64 : P::KC_EPS_F32;
  __shared__ T kre[(KR > 0 ? KR : 1) * 256];
  __shared__ cx<T> kcx[(KC > 0 ? KC : 1) * 256];
  __shared__ T keps[5 * (KE > 0 ? KE : 1) * 256];
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  double p[P::NPAR][4];
  load_on_shell<P::MASSIVE>(mom + e * (4 * P::NPAR), p, prm.mt);
  LdsKinCache<T> dc{kre, kcx, keps, int(threadIdx.x)};
  if constexpr (F64) P::template den_fill_f64<T>(p, prm, dc);
  else P::template den_fill_f32<T>(p, prm, dc);
  double acc = 0.0;
  for (int ih = 0; ih < prm.nhel; ++ih) {
#pragma unroll
    for (int i = 0; i < P::NPAR; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) asm volatile("" : "+v"(p[i][c]));
    asm volatile("" : "+v"(dc.off));
    const unsigned hel = prm.hel[ih];
    cx<T> jamp[P::NCOLOR];
    P::template amplitudes<T>(p, hel, prm, jamp, dc);
    const double q = double(P::template colour_sum<T>(jamp));
    if constexpr (F64) {
      if (out_hel) out_hel[e * P::NHEL + hel] = q * (P::coupling_factor(prm) / P::CDEN);
    }
    acc += q;
  }
  if (out) store_me(prm, out, e, acc * (P::coupling_factor(prm) / (P::CDEN * P::IDEN)));
}

// Vector-ALU colour sum with the full kinematic cache (propagator factors,
// polarisation bases, momentum sums and both helicity states of the
// external spinors): a block of W waves evaluates 64 events, wave w the
// helicities w, w + W, ... of each, so one per-event cache, formed by wave 0
// before the helicity loop, serves W lanes.  The helicity program reads no
// momenta, so none stay in registers across the loop.  Each wave's helicity
// partial sums meet in LDS and wave 0 adds them in wave order.  Lanes past
// the end of the batch evaluate the last event again (every wave reaches
// both barriers) and store nothing.  T = float: mixed form (out_hel unused);
// T = double: FP64 form (out_hel as in me_kernel).
template <class P, class T, int W>
__global__ __launch_bounds__(64 * W) void me_kernel_kcw(const double* __restrict__ mom, int64_t nevt,
                                                         double* __restrict__ out, double* __restrict__ out_hel,
                                                         const MeParams prm) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int KR = F64 ? P::KC_RE_F64 : P::KC_RE_F32, KC = F64 ? P::KC_CX_F64 : P::KC_CX_F32;
  constexpr int KE = F64 ? P::KC_EPS_F64 : P::KC_EPS_F32;
  constexpr int KM = F64 ? P::KC_MOM_F64 : P::KC_MOM_F32, KS = F64 ? P::KC_SP_F64 : P::KC_SP_F32;
  using DC = LdsKinCache<T, 64, true>;
  constexpr int NV = DC::NV;
  __shared__ T kre[(KR > 0 ? KR : 1) * 64];
  __shared__ cx<T> kcx[(KC > 0 ? KC : 1) * 64];
  __shared__ T keps[5 * (KE > 0 ? KE : 1) * 64];
  __shared__ typename DC::V kmo[NV * (KM > 0 ? KM : 1) * 64];
  __shared__ typename DC::V ksp[4 * NV * (KS > 0 ? KS : 1) * 64];
  __shared__ double part[W * 64];
  const int lane = threadIdx.x % 64;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / 64);
  const int64_t e = int64_t(blockIdx.x) * 64 + lane;
  const bool live = e < nevt;
  const int64_t ec = live ? e : nevt - 1;
  DC dc{kre, kcx, keps, lane, kmo, ksp};
  double p[P::NPAR][4];
  load_on_shell<P::MASSIVE>(mom + ec * (4 * P::NPAR), p, prm.mt);
  if (wave == 0) {
    if constexpr (F64) P::template den_fill_f64<T>(p, prm, dc);
    else P::template den_fill_f32<T>(p, prm, dc);
  }
  __syncthreads();
  double acc = 0.0;
  for (int ih = wave; ih < prm.nhel; ih += W) {
    asm volatile("" : "+v"(dc.off));
    const unsigned hel = prm.hel[ih];
    cx<T> jamp[P::NCOLOR];
    P::template amplitudes<T>(p, hel, prm, jamp, dc);
    const double q = double(P::template colour_sum<T>(jamp));
    if constexpr (F64) {
      if (out_hel && live) out_hel[e * P::NHEL + hel] = q * (P::coupling_factor(prm) / P::CDEN);
    }
    acc += q;
  }
  part[wave * 64 + lane] = acc;
  __syncthreads();
  if (wave == 0 && live && out) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += part[w * 64 + lane];
    store_me(prm, out, e, s * (P::coupling_factor(prm) / (P::CDEN * P::IDEN)));
  }
}

// Per-event light-cone cache of the FP64 form in LDS (128-thread blocks):
// the small light-cone component of each outgoing leg and the invariants of
// the pairs of massless outgoing legs, formed once per event and read where
// the propagator invariants are formed (slot s of thread t at s * 128 + t).
// The per-iteration offset passes through an empty asm statement so that the
// reads stay inside the helicity loop instead of being held in registers.
struct LdsLcCache {
  static constexpr bool kCached = false;
  static constexpr bool kMom = false;
  static constexpr bool kLc = true;
  double* base;
  int npair0;   // first pair slot (after the legs)
  int off;
  __device__ __forceinline__ double lcs(int k) const { return base[k * 128 + off]; }
  __device__ __forceinline__ double pair(int k) const { return base[(npair0 + k) * 128 + off]; }
  __device__ __forceinline__ void set_lcs(int k, double v) { base[k * 128 + off] = v; }
  __device__ __forceinline__ void set_pair(int k, double v) { base[(npair0 + k) * 128 + off] = v; }
};

// Jamps of one lane held in LDS instead of registers: element k of lane l at
// base[k * 64 + l], so a wave's 64 accesses to one jamp are contiguous.
template <class T>
struct LdsJamps {
  cx<T>* base;
  __device__ __forceinline__ cx<T>& operator[](int k) const { return base[k * 64]; }
};

// The jamps in LDS (frees 2 sizeof(T)/4 * NCOLOR registers per lane for the
// wavefunction schedule).  128-thread blocks: 2 waves x NCOLOR x 64 complex.
template <class P, class T>
__global__ __launch_bounds__(128) void me_kernel_ldsjamp(const double* __restrict__ mom, int64_t nevt,
                                                          double* __restrict__ out, double* __restrict__ out_hel,
                                                          const MeParams prm) {
  __shared__ cx<T> lds[2 * P::NCOLOR * 64];
  // the light-cone cache of the FP64 form (its light-cone invariants)
  constexpr int NLC = sizeof(T) == 8 ? P::LC_LEGS + P::LC_PAIRS : 1;
  __shared__ double lcb[NLC * 128];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  LdsJamps<T> jamp{lds + wave * P::NCOLOR * 64 + lane};
  double p[P::NPAR][4];
  load_on_shell<P::MASSIVE>(mom + e * (4 * P::NPAR), p, prm.mt);
  LdsLcCache lc{lcb, P::LC_LEGS, int(threadIdx.x)};
  if constexpr (sizeof(T) == 8) P::lc_fill(p, prm, lc);
  double acc = 0.0;
  for (int ih = 0; ih < prm.nhel; ++ih) {
#pragma unroll
    for (int i = 0; i < P::NPAR; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) asm volatile("" : "+v"(p[i][c]));
    const unsigned hel = prm.hel[ih];
    if constexpr (sizeof(T) == 8) {
      asm volatile("" : "+v"(lc.off));
      P::template amplitudes<T>(p, hel, prm, jamp, lc);
    } else {
      P::template amplitudes<T>(p, hel, prm, jamp);
    }
    const double q = double(P::template colour_sum<T>(jamp));
    if (out_hel) out_hel[e * P::NHEL + hel] = q * (P::coupling_factor(prm) / P::CDEN);
    acc += q;
  }
  if (out) store_me(prm, out, e, acc * (P::coupling_factor(prm) / (P::CDEN * P::IDEN)));
}

// Mixed form with the colour sum on MFMA.  Every lane of a wave stays active
// through the helicity loop (the MFMA needs the whole wave); lanes past the
// end of the batch evaluate the last event again and do not store.  The
// kinematic cache of the vector-ALU form (propagator factors and polarisation
// bases in LDS, once per event) is used when the process's FP32 schedule
// reads one: with the colour staging, 115 KB of LDS per 256-lane block for
// g g > t t~ g g.  OPS: the colour sum's operands, FP16 hi+lo jamps, FP32
// jamps or BF16 hi+lo jamps (colour_mfma.hpp).
enum { kMfmaF16HiLo = 0, kMfmaF32 = 1, kMfmaBf16HiLo = 2 };

template <class P, int OPS>
__device__ __forceinline__ void me_mfma_body(const double* __restrict__ mom, int64_t nevt, double* __restrict__ out,
                                             const MeParams& prm) {
  constexpr int kLds = OPS == kMfmaF32 ? kColourLds32Bytes : ColourTile<P::NCOLOR>::kLdsBytes;
  __shared__ __attribute__((aligned(16))) char lds_all[4 * kLds];
  // the mixed form's kinematic cache (propagator factors and polarisation
  // bases once per event), when the process's FP32 schedule reads one
  constexpr int KR = P::KC_RE_F32, KC = P::KC_CX_F32, KE = P::KC_EPS_F32;
  constexpr bool kCache = KR + KC + KE > 0;
  __shared__ float kre[(kCache && KR > 0 ? KR : 1) * 256];
  __shared__ cx<float> kcx[(kCache && KC > 0 ? KC : 1) * 256];
  __shared__ float keps[5 * (kCache && KE > 0 ? KE : 1) * 256];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t e0 = int64_t(blockIdx.x) * blockDim.x + 64 * wave;
  if (e0 >= nevt) return;   // whole wave past the end (wave-uniform)
  const int64_t e = e0 + lane;
  const int64_t ec = e < nevt ? e : nevt - 1;
  void* lds = lds_all + wave * kLds;
  const ColourA<P::NCOLOR> A = colour_a<P::NCOLOR>(P::cmat(), lane);
  const ColourA32<P::NCOLOR> A32 = colour_a32<P::NCOLOR>(P::cmat(), lane);
  const ColourA<P::NCOLOR, __bf16> Ab = colour_a<P::NCOLOR, __bf16>(P::cmat(), lane);
  double p[P::NPAR][4];
  load_on_shell<P::MASSIVE>(mom + ec * (4 * P::NPAR), p, prm.mt);
  LdsKinCache<float> dc{kre, kcx, keps, int(threadIdx.x)};
  if constexpr (kCache) P::template den_fill_f32<float>(p, prm, dc);
  double acc = 0.0;
  for (int ih = 0; ih < prm.nhel; ++ih) {
#pragma unroll
    for (int i = 0; i < P::NPAR; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) asm volatile("" : "+v"(p[i][c]));
    const unsigned hel = prm.hel[ih];
    cx<float> jamp[P::NCOLOR];
    if constexpr (kCache) {
      asm volatile("" : "+v"(dc.off));
      P::template amplitudes<float>(p, hel, prm, jamp, dc);
    } else {
      P::template amplitudes<float>(p, hel, prm, jamp);
    }
    if constexpr (OPS == kMfmaF32)
      acc += double(colour_sum_mfma32<P::NCOLOR>(jamp, A32, lds, lane));
    else if constexpr (OPS == kMfmaBf16HiLo)
      acc += double(colour_sum_mfma<P::NCOLOR, __bf16>(jamp, Ab, lds, lane));
    else
      acc += double(colour_sum_mfma<P::NCOLOR>(jamp, A, lds, lane));
  }
  if (e < nevt) store_me(prm, out, e, acc * (P::coupling_factor(prm) / (P::CDEN * P::IDEN)));
}

// The same with the full kinematic cache of me_kernel_kcw (momentum sums and
// spinors too): four waves share one block's 64 events, wave w evaluating
// the helicities w, w + 4, ...; each wave sums the colours of its 64 events
// for its helicity on MFMA as above, and the waves' helicity partial sums
// meet in LDS (wave order).  Every lane of every wave stays active.
template <class P, int OPS>
__device__ __forceinline__ void me_mfma_body_w(const double* __restrict__ mom, int64_t nevt,
                                               double* __restrict__ out, const MeParams& prm) {
  constexpr int W = 4;
  constexpr int kLds = OPS == kMfmaF32 ? kColourLds32Bytes : ColourTile<P::NCOLOR>::kLdsBytes;
  __shared__ __attribute__((aligned(16))) char lds_all[W * kLds];
  constexpr int KR = P::KC_RE_F32, KC = P::KC_CX_F32, KE = P::KC_EPS_F32;
  constexpr int KM = P::KC_MOM_F32, KS = P::KC_SP_F32;
  __shared__ float kre[(KR > 0 ? KR : 1) * 64];
  __shared__ cx<float> kcx[(KC > 0 ? KC : 1) * 64];
  __shared__ float keps[5 * (KE > 0 ? KE : 1) * 64];
  __shared__ float4 kmo[(KM > 0 ? KM : 1) * 64];
  __shared__ float4 ksp[4 * (KS > 0 ? KS : 1) * 64];
  __shared__ double part[W * 64];
  const int lane = threadIdx.x % 64;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / 64);
  const int64_t e = int64_t(blockIdx.x) * 64 + lane;
  const bool live = e < nevt;
  const int64_t ec = live ? e : nevt - 1;
  void* lds = lds_all + wave * kLds;
  const ColourA<P::NCOLOR> A = colour_a<P::NCOLOR>(P::cmat(), lane);
  const ColourA32<P::NCOLOR> A32 = colour_a32<P::NCOLOR>(P::cmat(), lane);
  const ColourA<P::NCOLOR, __bf16> Ab = colour_a<P::NCOLOR, __bf16>(P::cmat(), lane);
  LdsKinCache<float, 64, true> dc{kre, kcx, keps, lane, kmo, ksp};
  double p[P::NPAR][4];
  load_on_shell<P::MASSIVE>(mom + ec * (4 * P::NPAR), p, prm.mt);
  if (wave == 0) P::template den_fill_f32<float>(p, prm, dc);
  __syncthreads();
  double acc = 0.0;
  for (int ih = wave; ih < prm.nhel; ih += W) {
    asm volatile("" : "+v"(dc.off));
    const unsigned hel = prm.hel[ih];
    cx<float> jamp[P::NCOLOR];
    P::template amplitudes<float>(p, hel, prm, jamp, dc);
    if constexpr (OPS == kMfmaF32)
      acc += double(colour_sum_mfma32<P::NCOLOR>(jamp, A32, lds, lane));
    else if constexpr (OPS == kMfmaBf16HiLo)
      acc += double(colour_sum_mfma<P::NCOLOR, __bf16>(jamp, Ab, lds, lane));
    else
      acc += double(colour_sum_mfma<P::NCOLOR>(jamp, A, lds, lane));
  }
  part[wave * 64 + lane] = acc;
  __syncthreads();
  if (wave == 0 && live && out) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += part[w * 64 + lane];
    store_me(prm, out, e, s * (P::coupling_factor(prm) / (P::CDEN * P::IDEN)));
  }
}

// events per 256-lane block of the MFMA kernels
template <class P>
constexpr int mfma_block_events() {
  return P::KC_MOM_F32 + P::KC_SP_F32 > 0 ? 64 : 256;
}

// FP16 hi+lo (F32OPS false) or FP32 (true) colour-sum operands
template <class P, bool F32OPS>
__global__ __launch_bounds__(256) void me_kernel_mfma(const double* __restrict__ mom, int64_t nevt,
                                                      double* __restrict__ out, const MeParams prm) {
  if constexpr (mfma_block_events<P>() == 64)
    me_mfma_body_w<P, F32OPS ? kMfmaF32 : kMfmaF16HiLo>(mom, nevt, out, prm);
  else
    me_mfma_body<P, F32OPS ? kMfmaF32 : kMfmaF16HiLo>(mom, nevt, out, prm);
}

// BF16 hi+lo colour-sum operands
template <class P>
__global__ __launch_bounds__(256) void me_kernel_mfma_bf16(const double* __restrict__ mom, int64_t nevt,
                                                           double* __restrict__ out, const MeParams prm) {
  if constexpr (mfma_block_events<P>() == 64)
    me_mfma_body_w<P, kMfmaBf16HiLo>(mom, nevt, out, prm);
  else
    me_mfma_body<P, kMfmaBf16HiLo>(mom, nevt, out, prm);
}

// mode: ME_MODE_FP64; ME_MODE_MIXED (colour sum on the unit chosen for the
// process, P::MIXED_MFMA); ME_MODE_MIXED_VALU, ME_MODE_MIXED_MFMA16,
// ME_MODE_MIXED_MFMA32 or ME_MODE_MIXED_MFMABF16 (vector ALU, FP16 hi+lo, FP32
// or BF16 hi+lo MFMA; the MFMA forms for 6 to 32 colour flows, the vector ALU
// otherwise).  out_hel (FP64 only) receives the
// colour-summed |M_h|^2 of every listed helicity, [nevt][NHEL].
template <class P>
int launch(int mode, const double* mom, int64_t nevt, double* out, double* out_hel, const MeParams& prm,
           hipStream_t stream) {
  static_assert(!P::SPLIT, "split processes launch through launch_split");
  if (nevt <= 0) return 0;
  const int block = 256;
  const int64_t nblk = (nevt + block - 1) / block;
  if (nblk > 0x7fffffffLL) return -1;
  if (mode == ME_MODE_FP64) {
    // one FP64 kernel per process, chosen when the process is generated
    if constexpr (P::FP64_LDS_JAMPS) {
      const int64_t nb = (nevt + 127) / 128;
      hipLaunchKernelGGL((me_kernel_ldsjamp<P, double>), dim3(unsigned(nb)), dim3(128), 0, stream, mom, nevt,
                         out, out_hel, prm);
    } else if constexpr (P::KC_MOM_F64 + P::KC_SP_F64 > 0) {
      const int64_t nb = (nevt + 63) / 64;
      if (nb > 0x7fffffffLL) return -1;
      constexpr int W = P::F64_KCW_WAVES;
      hipLaunchKernelGGL((me_kernel_kcw<P, double, W>), dim3(unsigned(nb)), dim3(64 * W), 0, stream, mom, nevt,
                         out, out_hel, prm);
    } else if constexpr (P::KC_RE_F64 + P::KC_CX_F64 + P::KC_EPS_F64 > 0) {
      hipLaunchKernelGGL((me_kernel_kc<P, double>), dim3(unsigned(nblk)), dim3(block), 0, stream, mom, nevt, out,
                         out_hel, prm);
    } else {
      hipLaunchKernelGGL((me_kernel<P, double>), dim3(unsigned(nblk)), dim3(block), 0, stream, mom, nevt, out,
                         out_hel, prm);
    }
  } else if (((mode == ME_MODE_MIXED && P::MIXED_MFMA) || mode == ME_MODE_MIXED_MFMA16 ||
              mode == ME_MODE_MIXED_MFMA32 || mode == ME_MODE_MIXED_MFMABF16) && P::NCOLOR >= 6 &&
             P::NCOLOR <= 32) {
    if (out_hel || !out) return -1;
    constexpr int EB = mfma_block_events<P>();
    const int64_t nbm = (nevt + EB - 1) / EB;
    if (nbm > 0x7fffffffLL) return -1;
    if (mode == ME_MODE_MIXED_MFMA32)
      hipLaunchKernelGGL((me_kernel_mfma<P, true>), dim3(unsigned(nbm)), dim3(block), 0, stream, mom, nevt, out,
                         prm);
    else if (mode == ME_MODE_MIXED_MFMABF16)
      hipLaunchKernelGGL((me_kernel_mfma_bf16<P>), dim3(unsigned(nbm)), dim3(block), 0, stream, mom, nevt, out,
                         prm);
    else
      hipLaunchKernelGGL((me_kernel_mfma<P, false>), dim3(unsigned(nbm)), dim3(block), 0, stream, mom, nevt, out,
                         prm);
  } else if (mode == ME_MODE_MIXED || mode == ME_MODE_MIXED_VALU || mode == ME_MODE_MIXED_MFMA32 ||
             mode == ME_MODE_MIXED_MFMA16 || mode == ME_MODE_MIXED_MFMABF16) {
    if (out_hel) return -1;
    if constexpr (P::F32_LDS_JAMPS) {
      const int64_t nb = (nevt + 127) / 128;
      hipLaunchKernelGGL((me_kernel_ldsjamp<P, float>), dim3(unsigned(nb)), dim3(128), 0, stream, mom, nevt,
                         out, nullptr, prm);
    } else if constexpr (P::KC_MOM_F32 + P::KC_SP_F32 > 0) {
      const int64_t nb = (nevt + 63) / 64;
      if (nb > 0x7fffffffLL) return -1;
      constexpr int W = P::F32_KC_WAVES;
      hipLaunchKernelGGL((me_kernel_kcw<P, float, W>), dim3(unsigned(nb)), dim3(64 * W), 0, stream, mom, nevt,
                         out, nullptr, prm);
    } else if constexpr (P::KC_RE_F32 + P::KC_CX_F32 + P::KC_EPS_F32 > 0) {
      hipLaunchKernelGGL((me_kernel_kc<P, float>), dim3(unsigned(nblk)), dim3(block), 0, stream, mom, nevt, out,
                         nullptr, prm);
    } else {
      hipLaunchKernelGGL((me_kernel<P, float>), dim3(unsigned(nblk)), dim3(block), 0, stream, mom, nevt, out,
                         nullptr, prm);
    }
  } else {
    return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace me
