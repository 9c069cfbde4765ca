// Device-side phase-space generation: RAMBO (Kleiss, Stirling, Ellis 1986),
// the generator of the paper's standalone test-bed (Sec. 2), writing momenta
// straight into the [nevt][npar][4] layout me_compute reads, so a batch never
// crosses PCIe.  One event per lane; HBM-write bound (32 npar bytes per event).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds of  (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0))  with M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the key bumped by the
// Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.  Counter = (event
// low, event high, 2*particle + half, 0), key = seed; one block gives two
// 53-bit uniforms u in [0,1).  Draw order per particle: cos theta, phi, then
// the two factors of the energy; 1-u enters the logarithms.
//
// Kinematics in FP64 with the massless invariant mass formed as
// sum_{i<j} q0_i q0_j |n_i - n_j|^2 (no cancellation); a two-body final state
// is rebuilt back to back from RAMBO's direction; massive final states are
// rescaled with Newton's method (at most 30 steps).
#include <hip/hip_runtime.h>

#include "me.h"

namespace {

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const uint32_t lo0 = M0 * c.x, hi0 = __umulhi(M0, c.x);
    const uint32_t lo1 = M1 * c.z, hi1 = __umulhi(M1, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  return double((uint64_t(a >> 5) << 26) | uint64_t(b >> 6)) * (1.0 / 9007199254740992.0);
}

constexpr int kMaxFinal = 5;

struct RamboArgs {
  int32_t nfinal;
  double sqrt_s;
  double mass[kMaxFinal];
  uint32_t k0, k1;
};

// N = number of final-state particles (a compile-time constant, so the
// per-particle arrays live in registers)
template <int N>
__global__ __launch_bounds__(256) void rambo_kernel(int64_t nevt, RamboArgs a, double* __restrict__ out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  constexpr int n = N;
  const double pi = 3.14159265358979323846;
  double q0[N], nh[N][3];
  for (int i = 0; i < n; ++i) {
    const U4 r0 = philox4x32_10(U4{uint32_t(e), uint32_t(uint64_t(e) >> 32), uint32_t(2 * i), 0u}, a.k0, a.k1);
    const U4 r1 = philox4x32_10(U4{uint32_t(e), uint32_t(uint64_t(e) >> 32), uint32_t(2 * i + 1), 0u}, a.k0, a.k1);
    const double c = 2.0 * u53(r0.x, r0.y) - 1.0;
    const double phi = 2.0 * pi * u53(r0.z, r0.w);
    q0[i] = -log((1.0 - u53(r1.x, r1.y)) * (1.0 - u53(r1.z, r1.w)));
    const double st = sqrt(fmax(0.0, 1.0 - c * c));
    nh[i][0] = st * cos(phi);
    nh[i][1] = st * sin(phi);
    nh[i][2] = c;
  }
  double Q[4] = {0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    Q[0] += q0[i];
    for (int k = 0; k < 3; ++k) Q[k + 1] += q0[i] * nh[i][k];
  }
  double M2 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double d2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double d = nh[i][k] - nh[j][k];
        d2 += d * d;
      }
      M2 += q0[i] * q0[j] * d2;
    }
  const double M = sqrt(M2);
  const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
  const double gam = Q[0] / M, aa = 1.0 / (1.0 + gam), x = a.sqrt_s / M;
  double p[N][4];
  for (int i = 0; i < n; ++i) {
    double qv[3];
    for (int k = 0; k < 3; ++k) qv[k] = q0[i] * nh[i][k];
    const double bq = b[0] * qv[0] + b[1] * qv[1] + b[2] * qv[2];
    p[i][0] = x * (gam * q0[i] + bq);
    for (int k = 0; k < 3; ++k) p[i][k + 1] = x * (qv[k] + b[k] * q0[i] + aa * bq * b[k]);
  }
  if (n == 2) {
    // exact back-to-back pair along RAMBO's direction
    const double pn = sqrt(p[0][1] * p[0][1] + p[0][2] * p[0][2] + p[0][3] * p[0][3]);
    const double m1 = a.mass[0], m2 = a.mass[1], s = a.sqrt_s;
    const double e1 = (s * s + m1 * m1 - m2 * m2) / (2.0 * s);
    const double pa = sqrt(fmax(0.0, e1 * e1 - m1 * m1));
    double dir[3];
    for (int k = 0; k < 3; ++k) dir[k] = p[0][k + 1] / pn;
    p[0][0] = e1;
    p[1][0] = s - e1;
    for (int k = 0; k < 3; ++k) { p[0][k + 1] = pa * dir[k]; p[1][k + 1] = -pa * dir[k]; }
  } else {
    double msum = 0.0;
    for (int i = 0; i < n; ++i) msum += a.mass[i];
    if (msum > 0.0) {
      double xi = sqrt(1.0 - (msum / a.sqrt_s) * (msum / a.sqrt_s));
      for (int it = 0; it < 30; ++it) {
        double f = -a.sqrt_s, df = 0.0;
        for (int i = 0; i < n; ++i) {
          const double en = sqrt(a.mass[i] * a.mass[i] + xi * xi * p[i][0] * p[i][0]);
          f += en;
          df += xi * p[i][0] * p[i][0] / en;
        }
        if (fabs(f) <= 4e-16 * a.sqrt_s) break;
        xi -= f / df;
      }
      for (int i = 0; i < n; ++i) {
        p[i][0] = sqrt(a.mass[i] * a.mass[i] + xi * xi * p[i][0] * p[i][0]);
        for (int k = 1; k < 4; ++k) p[i][k] *= xi;
      }
    }
  }
  double* o = out + e * (4 * (n + 2));
  const double h = 0.5 * a.sqrt_s;
  o[0] = h; o[1] = 0.0; o[2] = 0.0; o[3] = h;
  o[4] = h; o[5] = 0.0; o[6] = 0.0; o[7] = -h;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 4; ++k) o[8 + 4 * i + k] = p[i][k];
}

// ----------------------------------------------- importance-sampled points
// A non-flat generator with the channel structure of madevent's phase-space
// mappings: sequential two-body splitting.  The centre-of-mass system emits
// final particle N-1, its remainder particle N-2, ..., and the last remainder
// decays into particles 0 and 1.  Per split k, Philox words (event,
// 0x10000 + 2k + half) give u0 (remainder mass), u1 (polar angle), u2
// (azimuth), angles taken in the decaying system's rest frame (pure boost)
// about the z axis:
//   M^2 = Mmin^2 + (1 - u0^2)(Mmax^2 - Mmin^2)         (soft splittings favoured;
//                                                       both ends of the range carried exactly)
//   c = sqrt(1+eps) tanh(y), y = (2 u1 - 1) Y, Y = atanh(1/sqrt(1+eps)), eps = 1/100
//                                                       (peaked along the beams)
//   phi = 2 pi u2.
// Weight = phase-space Jacobian for dPhi_n = (2pi)^4 delta^4 prod d^3p/((2pi)^3 2E):
//   prod_splits |p*|/(16 pi^2 M) * 2Y (1+eps-c^2)/sqrt(1+eps) * 2 pi
//     (the angular factor taken as 2Y sqrt(1+eps)/cosh^2(y), free of cancellation)
//   * prod_remainder-masses 2 u0 (Mmax^2 - Mmin^2)/(2 pi).
struct SampleArgs {
  double sqrt_s;
  double mass[kMaxFinal];
  uint32_t k0, k1;
};

// rest-frame four-momentum q of a system P of mass M, boosted to the lab
__device__ __forceinline__ void to_lab(const double (&P)[4], double M, double (&q)[4]) {
  const double e = (P[0] * q[0] + P[1] * q[1] + P[2] * q[2] + P[3] * q[3]) / M;
  const double f = (q[0] + e) / (P[0] + M);
  q[0] = e;
  q[1] += f * P[1];
  q[2] += f * P[2];
  q[3] += f * P[3];
}

template <int N>
__global__ __launch_bounds__(256) void sample_kernel(int64_t nevt, SampleArgs a, double* __restrict__ out,
                                                     double* __restrict__ weight) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  const double pi = 3.14159265358979323846, eps = 0.01;
  const double se = sqrt(1.0 + eps), Y = atanh(1.0 / se);
  double p[N][4];
  double P[4] = {a.sqrt_s, 0.0, 0.0, 0.0};
  double M = a.sqrt_s, W = 1.0, mrest = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) mrest += a.mass[i];
  double gap = a.sqrt_s - mrest;                  // M minus the masses it still holds
#pragma unroll
  for (int k = 0; k < N - 1; ++k) {
    const U4 r0 = philox4x32_10(U4{uint32_t(e), uint32_t(uint64_t(e) >> 32), uint32_t(0x10000 + 2 * k), 0u},
                                a.k0, a.k1);
    const U4 r1 = philox4x32_10(U4{uint32_t(e), uint32_t(uint64_t(e) >> 32), uint32_t(0x10000 + 2 * k + 1), 0u},
                                a.k0, a.k1);
    const double u0 = u53(r0.x, r0.y), u1 = u53(r0.z, r0.w), u2 = u53(r1.x, r1.y);
    const bool last = k == N - 2;
    const int ja = last ? 1 : N - 1 - k;          // particle split off here
    const double ma = a.mass[ja];
    mrest -= ma;
    double Mr, thr;                               // remainder mass, M - ma - Mr
    if (last) {
      Mr = a.mass[0];
      thr = gap;
    } else {
      // the distances to both ends of the mass range without cancellation
      const double lo = mrest, hi = M - ma, d2 = gap * (hi + lo), x = (1.0 - u0) * (1.0 + u0);
      Mr = sqrt(lo * lo + x * d2);
      thr = u0 * u0 * d2 / (hi + Mr);
      gap = x * d2 / (Mr + lo);
      W *= 2.0 * u0 * d2 / (2.0 * pi);
    }
    const double ps = sqrt(fmax(0.0, thr * (M + ma + Mr) * (M - ma + Mr) * (M + ma - Mr))) / (2.0 * M);
    const double y = (2.0 * u1 - 1.0) * Y, c = se * tanh(y), ch = cosh(y);
    const double st = sqrt(fmax(0.0, 1.0 - c * c)), phi = 2.0 * pi * u2;
    W *= ps / (16.0 * pi * pi * M) * (2.0 * Y * se / (ch * ch)) * (2.0 * pi);
    double qa[4] = {sqrt(ma * ma + ps * ps), ps * st * cos(phi), ps * st * sin(phi), ps * c};
    double qr[4] = {sqrt(Mr * Mr + ps * ps), -qa[1], -qa[2], -qa[3]};
    to_lab(P, M, qa);
    to_lab(P, M, qr);
#pragma unroll
    for (int q = 0; q < 4; ++q) p[ja][q] = qa[q];
    if (last) {
#pragma unroll
      for (int q = 0; q < 4; ++q) p[0][q] = qr[q];
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) P[q] = qr[q];
      M = Mr;
    }
  }
  double* o = out + e * (4 * (N + 2));
  const double h = 0.5 * a.sqrt_s;
  o[0] = h; o[1] = 0.0; o[2] = 0.0; o[3] = h;
  o[4] = h; o[5] = 0.0; o[6] = 0.0; o[7] = -h;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) o[8 + 4 * i + k] = p[i][k];
  weight[e] = W;
}

}  // namespace

extern "C" me_status me_sample(int64_t nevt, int32_t nfinal, const double* masses, double sqrt_s, uint64_t seed,
                               double* d_momenta, double* d_weight, void* hip_stream) {
  if (nevt < 0 || nfinal < 2 || nfinal > kMaxFinal || !masses || !(sqrt_s > 0) ||
      (nevt > 0 && (!d_momenta || !d_weight)))
    return ME_EINVAL;
  SampleArgs a;
  a.sqrt_s = sqrt_s;
  double msum = 0.0;
  for (int i = 0; i < kMaxFinal; ++i) a.mass[i] = i < nfinal ? masses[i] : 0.0;
  for (int i = 0; i < nfinal; ++i) {
    if (!(masses[i] >= 0)) return ME_EINVAL;
    msum += masses[i];
  }
  if (!(msum < sqrt_s)) return ME_EINVAL;
  a.k0 = uint32_t(seed);
  a.k1 = uint32_t(seed >> 32);
  if (nevt == 0) return ME_OK;
  const int64_t blocks = (nevt + 255) / 256;
  if (blocks > 0x7fffffffLL) return ME_EINVAL;
  const dim3 grid{unsigned(blocks)}, block{256};
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  switch (nfinal) {
    case 2: hipLaunchKernelGGL(sample_kernel<2>, grid, block, 0, s, nevt, a, d_momenta, d_weight); break;
    case 3: hipLaunchKernelGGL(sample_kernel<3>, grid, block, 0, s, nevt, a, d_momenta, d_weight); break;
    case 4: hipLaunchKernelGGL(sample_kernel<4>, grid, block, 0, s, nevt, a, d_momenta, d_weight); break;
    default: hipLaunchKernelGGL(sample_kernel<5>, grid, block, 0, s, nevt, a, d_momenta, d_weight); break;
  }
  return hipGetLastError() == hipSuccess ? ME_OK : ME_EHIP;
}

extern "C" me_status me_rambo(int64_t nevt, int32_t nfinal, const double* masses, double sqrt_s, uint64_t seed,
                              double* d_momenta, void* hip_stream) {
  if (nevt < 0 || nfinal < 2 || nfinal > kMaxFinal || !masses || !(sqrt_s > 0) || (nevt > 0 && !d_momenta))
    return ME_EINVAL;
  RamboArgs a;
  a.nfinal = nfinal;
  a.sqrt_s = sqrt_s;
  double msum = 0.0;
  for (int i = 0; i < kMaxFinal; ++i) a.mass[i] = i < nfinal ? masses[i] : 0.0;
  for (int i = 0; i < nfinal; ++i) {
    if (!(masses[i] >= 0)) return ME_EINVAL;
    msum += masses[i];
  }
  if (msum >= sqrt_s) return ME_EINVAL;
  a.k0 = uint32_t(seed);
  a.k1 = uint32_t(seed >> 32);
  if (nevt == 0) return ME_OK;
  const int64_t blocks = (nevt + 255) / 256;
  if (blocks > 0x7fffffffLL) return ME_EINVAL;
  const dim3 grid{unsigned(blocks)}, block{256};
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  switch (nfinal) {
    case 2: hipLaunchKernelGGL(rambo_kernel<2>, grid, block, 0, s, nevt, a, d_momenta); break;
    case 3: hipLaunchKernelGGL(rambo_kernel<3>, grid, block, 0, s, nevt, a, d_momenta); break;
    case 4: hipLaunchKernelGGL(rambo_kernel<4>, grid, block, 0, s, nevt, a, d_momenta); break;
    default: hipLaunchKernelGGL(rambo_kernel<5>, grid, block, 0, s, nevt, a, d_momenta); break;
  }
  return hipGetLastError() == hipSuccess ? ME_OK : ME_EHIP;
}
