// Split form of the matrix-element evaluation, for processes whose colour
// flows do not fit in a lane's registers (gg -> t tbar ggg: 120 flows).
//
// The amplitude program of one helicity is cut into parts (separate kernels,
// run in stream order).  A lane of a part kernel evaluates one event at one
// helicity, keeps a bounded set of jamp accumulators in registers and adds
// them into its row of a workspace X; the first part to touch a jamp stores
// it.  A second kernel then evaluates the colour sum q_h = Re(J^H C J) of
// every (event, helicity) row on MFMA and sums the helicities into |M|^2.
//
// Workspace layout (per chunk of events and helicities):
//   X[(hc * NCOLOR + k) * ne_pad + e]   complex, hc = helicity slot in the
//   chunk, k = colour flow, e = event in the chunk,
// so a wave's 64 lanes touch 64 consecutive entries of one colour flow.
//
// Colour sum on MFMA, D' = C X^T for a tile of 16 events (N = 16 events,
// M = colour rows in tiles of 16, K = colours).  The K slots of A (colour
// matrix) and B (jamps) may be assigned to colours in any common order; the
// order used here gives lane l = 16 g + n, as B operands, exactly the
// colours of event n whose rows of D' the lane receives (FP16 form:
// D[4 g + i][n] of m-tile mt, colours 16 mt + 4 g + i; FP64 form:
// D[g + 4 i][n], colours 16 mt + g + 4 i).  So each lane finishes
// sum_c x_c (C x)_c over its own 32 colours without any data exchange, and
// four lanes add their parts with two cross-lane moves.
#pragma once
#include <hip/hip_runtime.h>

#include "colour_mfma.hpp"
#include "epilogue.hpp"
#include "helas.hpp"

namespace me {

typedef double double4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double4v mfma16x16x4f64(double a, double b, double4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Write-back of a jamp accumulator into the lane's workspace row.  The
// address goes through an empty asm statement so that the compiler cannot
// forward an earlier store of the same jamp into a later read-add-store:
// that forwarding would keep every partial jamp in registers until its last
// write-back and undo the bounded accumulator set of the schedule.
template <class T>
__device__ __forceinline__ void jw_store(cx<T>* jw, int64_t off, cx<T> v) {
  cx<T>* q = jw + off;
  asm volatile("" : "+v"(q));
  *q = v;
}
template <class T>
__device__ __forceinline__ void jw_add(cx<T>* jw, int64_t off, cx<T> v) {
  cx<T>* q = jw + off;
  asm volatile("" : "+v"(q));
  *q = *q + v;
}

// One part of the amplitude program for one (event, helicity) per lane.
// grid.x covers the events of the chunk, grid.y its helicity slots.
template <class P, class T, int J>
__global__ __launch_bounds__(256) void me_part_kernel(const double* __restrict__ mom, int64_t ne, int h0,
                                                      cx<T>* __restrict__ X, int64_t ne_pad, const MeParams prm) {
  // jamp accumulators of the part when its schedule keeps them in LDS: lane
  // l's slots are a row of NQP (odd) complex values at qbuf[l * NQP], so
  // every slot is a small immediate offset from the lane's base, and eight
  // consecutive lanes' 16-byte accesses fall in distinct groups of banks
  constexpr int NQ = sizeof(T) == 8 ? P::QLDS_F64 : P::QLDS_F32;
  constexpr int NQP = NQ > 0 ? (NQ | 1) : 1;
  __shared__ cx<T> qbuf[NQP * 256];
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int hc = blockIdx.y;
  const unsigned hel = prm.hel[h0 + hc];
  double p[P::NPAR][4];
  load_on_shell<P::MASSIVE>(mom + e * (4 * P::NPAR), p, prm.mt);
  P::template part<T, J>(p, hel, prm, X + int64_t(hc) * P::NCOLOR * ne_pad + e, ne_pad, qbuf + threadIdx.x * NQP);
}

// Host launcher of one part kernel (each part is compiled in a translation
// unit of its own and reached through a table of these).
typedef void (*PartLaunchFn)(dim3 grid, hipStream_t s, const double* mom, int64_t ne, int h0, void* X,
                             int64_t ne_pad, const MeParams* prm);

template <class P, class T, int J>
void launch_part(dim3 grid, hipStream_t s, const double* mom, int64_t ne, int h0, void* X, int64_t ne_pad,
                 const MeParams* prm) {
  hipLaunchKernelGGL((me_part_kernel<P, T, J>), grid, dim3(256), 0, s, mom, ne, h0, static_cast<cx<T>*>(X),
                     ne_pad, *prm);
}

// Colour tiles: MT2 m-tiles of 16 colours (colours padded to 16 * MT2).
template <int NC>
struct SplitTiles {
  static constexpr int KS = (NC + 31) / 32;   // K steps of 32 (FP16 MFMA)
  static constexpr int MT2 = 2 * KS;          // m-tiles of 16 colours
  static constexpr int NCP = 16 * MT2;        // padded colour count
};

// Mixed form: jamps (FP32) split into FP16 hi + lo after a per-event
// power-of-two scale, colour matrix exact in FP16, FP32 accumulation on
// v_mfma_f32_16x16x32_f16; helicity sum in FP64.
// Block: 4 waves, 16 events per wave.  The helicity sum runs over passes
// (helicity slices of the workspace) in helicity order, one addition per
// helicity, so its rounding does not depend on how the helicities are
// sliced: the first pass starts from 0, later ones from out[e], which holds
// the unscaled partial sum; the last pass stores the sum times
// g^2n / (CDEN * IDEN).
template <class P>
__global__ __launch_bounds__(256) void me_colour_split_f16(const cx<float>* __restrict__ X, int64_t ne,
                                                           int64_t ne_pad, int nh, double* __restrict__ out,
                                                           int first, int last, const MeParams prm) {
  constexpr int NC = P::NCOLOR;
  using TL = SplitTiles<NC>;
  const int lane = threadIdx.x % 64, n = lane % 16, g = lane / 16;
  const int64_t e = (int64_t(blockIdx.x) * 4 + threadIdx.x / 64) * 16 + n;
  if (e - n >= ne) return;   // whole wave past the end (wave-uniform)
  const bool live = e < ne;
  const int* cm = P::cmat();
  // A operands: lane supplies C[16 mt + n][kappa(s, g, j)], kappa = 16 (2s + j/4) + 4 g + j%4
  half8 A[TL::MT2][TL::KS];
#pragma unroll
  for (int mt = 0; mt < TL::MT2; ++mt)
#pragma unroll
    for (int s = 0; s < TL::KS; ++s)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int row = 16 * mt + n, col = 16 * (2 * s + j / 4) + 4 * g + j % 4;
        A[mt][s][j] = (row < NC && col < NC) ? _Float16(float(cm[row * NC + col])) : _Float16(0.0f);
      }
  double acc = (!first && live && g == 0) ? out[e] : 0.0;
  for (int hc = 0; hc < nh; ++hc) {
    // this lane's colours 16 mt + 4 g + i of event e
    float xr[TL::MT2][4], xi[TL::MT2][4];
    const cx<float>* xrow = X + int64_t(hc) * NC * ne_pad + e;
    float m = 0.f;
#pragma unroll
    for (int mt = 0; mt < TL::MT2; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * mt + 4 * g + i;
        cx<float> v{0.f, 0.f};
        if (live && c < NC) v = xrow[int64_t(c) * ne_pad];
        xr[mt][i] = v.r;
        xi[mt][i] = v.i;
        m = fmaxf(m, fmaxf(fabsf(v.r), fabsf(v.i)));
      }
    m = fmaxf(m, __shfl_xor(m, 16, 64));
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    int ex = 0;
    (void)frexpf(m, &ex);
    float q = 0.f;
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      float v[TL::MT2][4];
#pragma unroll
      for (int mt = 0; mt < TL::MT2; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[mt][i] = ldexpf(ri ? xi[mt][i] : xr[mt][i], -ex);
      half8 bh[TL::KS], bl[TL::KS];
#pragma unroll
      for (int s = 0; s < TL::KS; ++s)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float x = v[2 * s + j / 4][j % 4];
          const _Float16 h = _Float16(x);
          bh[s][j] = h;
          bl[s][j] = _Float16(x - float(h));
        }
#pragma unroll
      for (int mt = 0; mt < TL::MT2; ++mt) {
        if (16 * mt >= NC) continue;
        float4v d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < TL::KS; ++s) {
          d = mfma16x16x32(A[mt][s], bh[s], d);
          d = mfma16x16x32(A[mt][s], bl[s], d);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) q += v[mt][i] * d[i];
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    q += __shfl_xor(q, 16, 64);
    q += __shfl_xor(q, 32, 64);
    acc += double(ldexpf(q, 2 * ex));
  }
  if (live && g == 0) {
    if (last) store_me(prm, out, e, acc * (P::coupling_factor(prm) / (P::CDEN * P::IDEN)));
    else out[e] = acc;
  }
}

// FP64 form on v_mfma_f64_16x16x4_f64.  Its result rows are interleaved:
// lane l = 16 g + n receives D[g + 4 r][n] in register r (measured on
// gfx950), so the lane's own colours are 16 mt + g + 4 r and K slot g of
// step s holds colour kappa(s, g) = 16 (s/4) + g + 4 (s%4).  The colour
// matrix sits in LDS as FP32 (exact integers), converted per step.  out_hel
// (optional) receives the colour-summed |M_h|^2 of every helicity,
// [nevt][NHEL].  The helicity sum over passes is accumulated as in the FP16
// form (first, last: see there).
template <class P>
__global__ __launch_bounds__(256) void me_colour_split_f64(const cx<double>* __restrict__ X, int64_t ne,
                                                           int64_t ne_pad, int nh, int h0,
                                                           double* __restrict__ out, double* __restrict__ out_hel,
                                                           int first, int last, const MeParams prm) {
  constexpr int NC = P::NCOLOR;
  using TL = SplitTiles<NC>;
  constexpr int LDW = TL::NCP + 1;
  __shared__ float cs[TL::NCP * LDW];
  const int* cm = P::cmat();
  for (int t = threadIdx.x; t < TL::NCP * TL::NCP; t += blockDim.x) {
    const int r = t / TL::NCP, c = t % TL::NCP;
    cs[r * LDW + c] = (r < NC && c < NC) ? float(cm[r * NC + c]) : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x % 64, n = lane % 16, g = lane / 16;
  const int64_t e = (int64_t(blockIdx.x) * 4 + threadIdx.x / 64) * 16 + n;
  if (e - n >= ne) return;   // whole wave past the end (wave-uniform)
  const bool live = e < ne;
  const double f = P::coupling_factor(prm) / P::CDEN;
  double acc = (!first && out && live && g == 0) ? out[e] : 0.0;
  for (int hc = 0; hc < nh; ++hc) {
    const cx<double>* xrow = X + int64_t(hc) * NC * ne_pad + e;
    double q = 0.0;
    for (int ri = 0; ri < 2; ++ri) {
      double x[TL::MT2][4];
#pragma unroll
      for (int mt = 0; mt < TL::MT2; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * mt + g + 4 * i;
          const double* src = reinterpret_cast<const double*>(xrow + int64_t(c) * ne_pad);
          x[mt][i] = (live && c < NC) ? src[ri] : 0.0;
        }
#pragma unroll
      for (int mt = 0; mt < TL::MT2; ++mt) {
        if (16 * mt >= NC) continue;
        double4v d = {0.0, 0.0, 0.0, 0.0};
        const float* crow = cs + (16 * mt + n) * LDW + g;
#pragma unroll
        for (int s4 = 0; s4 < TL::MT2; ++s4) {
#pragma unroll
          for (int i = 0; i < 4; ++i) d = mfma16x16x4f64(double(crow[16 * s4 + 4 * i]), x[s4][i], d);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) q += x[mt][i] * d[i];
        // keep the next tile's colour-matrix loads from being hoisted here
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    q += __shfl_xor(q, 16, 64);
    q += __shfl_xor(q, 32, 64);
    if (out_hel && live && g == 0) out_hel[e * P::NHEL + prm.hel[h0 + hc]] = q * f;
    acc += q;
  }
  if (out && live && g == 0) {
    if (last) store_me(prm, out, e, acc * (f / P::IDEN));
    else out[e] = acc;
  }
}

// Events per chunk and the default workspace cap per call.  Without a
// caller workspace the launch takes it from the stream-ordered allocator, so
// concurrent calls on different streams each get their own.  A slice of
// 2^14 events x the helicities that fit in 128 MiB (FP64: 4, 65536 lanes,
// one 256-lane block per CU; FP32: 8) stays resident in the 256 MB last-level
// cache while the parts read-add-store it one after another: measured on
// 2^17 events, FP64 321 -> 269 ms and mixed 170 -> 142 ms against chunks of
// 2^17 events and a 1 GiB workspace (256 MiB, or chunks of 2^15 and 2^16,
// in between; 64 MiB leaves half the CUs idle in FP64).
constexpr int64_t kSplitChunkEvents = int64_t(1) << 14;
constexpr int64_t kSplitWorkspaceBytes = int64_t(1) << 27;

// Bytes of one helicity slot of the jamp workspace for a chunk of nevt events.
template <class P, class T> int64_t split_row_bytes(int64_t nevt) {
  const int64_t ne_max = nevt < kSplitChunkEvents ? nevt : kSplitChunkEvents;
  const int64_t ne_pad = (ne_max + 255) / 256 * 256;
  return int64_t(P::NCOLOR) * int64_t(sizeof(cx<T>)) * ne_pad;
}
// Helicity slots a workspace of `bytes` holds (at most nhel, at least 1).
template <class P, class T> int64_t split_slots(int64_t nevt, int nhel, int64_t bytes) {
  int64_t nh = bytes / split_row_bytes<P, T>(nevt);
  if (nh > nhel && nhel > 0) nh = nhel;
  return nh < 1 ? 1 : nh;
}
// Workspace of a launch that may use at most cap bytes (cap <= 0: default).
template <class P>
int64_t split_workspace_bytes(int mode, int64_t nevt, int nhel, int64_t cap) {
  if (nevt <= 0) return 0;
  if (cap <= 0) cap = kSplitWorkspaceBytes;
  if (mode == ME_MODE_FP64) return split_row_bytes<P, double>(nevt) * split_slots<P, double>(nevt, nhel, cap);
  return split_row_bytes<P, float>(nevt) * split_slots<P, float>(nevt, nhel, cap);
}

template <class P, class T>
int run_split(const double* mom, int64_t nevt, double* out, double* out_hel, const MeParams& prm,
              hipStream_t stream, void* ws, int64_t ws_bytes, const PartLaunchFn* parts, int nparts) {
  const int64_t ne_max = nevt < kSplitChunkEvents ? nevt : kSplitChunkEvents;
  const int64_t ne_pad = (ne_max + 255) / 256 * 256;
  const int64_t row = split_row_bytes<P, T>(nevt);   // one helicity slot
  cx<T>* X = static_cast<cx<T>*>(ws);
  int64_t nh;
  if (X) {
    // the caller's workspace: as many helicity slots as it holds
    if (ws_bytes < row) return -3;
    nh = split_slots<P, T>(nevt, prm.nhel, ws_bytes);
  } else {
    nh = split_slots<P, T>(nevt, prm.nhel, kSplitWorkspaceBytes);
    if (hipMallocAsync(reinterpret_cast<void**>(&X), size_t(row) * size_t(nh), stream) != hipSuccess) return -3;
  }
  for (int64_t e0 = 0; e0 < nevt; e0 += kSplitChunkEvents) {
    const int64_t ne = nevt - e0 < kSplitChunkEvents ? nevt - e0 : kSplitChunkEvents;
    // with no helicity left the colour kernel still runs once and writes zeros
    for (int h0 = 0; h0 < (prm.nhel > 0 ? prm.nhel : 1); h0 += int(nh)) {
      const int nhc = prm.nhel - h0 < nh ? prm.nhel - h0 : int(nh);
      if (nhc > 0)
        for (int j = 0; j < nparts; ++j)
          parts[j](dim3(unsigned((ne + 255) / 256), unsigned(nhc)), stream, mom + e0 * 4 * P::NPAR, ne, h0, X,
                   ne_pad, &prm);
      const dim3 cgrid(unsigned((ne + 63) / 64));
      const int first = h0 == 0 ? 1 : 0, last = h0 + nhc >= prm.nhel ? 1 : 0;
      const MeParams cprm = epilogue_at(prm, e0);   // the last pass's epilogue sees this chunk
      if constexpr (sizeof(T) == 8)
        hipLaunchKernelGGL((me_colour_split_f64<P>), cgrid, dim3(256), 0, stream, X, ne, ne_pad, nhc, h0,
                           out ? out + e0 : nullptr, out_hel ? out_hel + e0 * P::NHEL : nullptr, first, last, cprm);
      else
        hipLaunchKernelGGL((me_colour_split_f16<P>), cgrid, dim3(256), 0, stream, X, ne, ne_pad, nhc, out + e0,
                           first, last, cprm);
    }
  }
  const hipError_t err = hipGetLastError();
  if (!ws) (void)hipFreeAsync(X, stream);
  return err == hipSuccess ? 0 : -2;
}

// mode: ME_MODE_FP64 (FP64 parts, colour sum on FP64 MFMA, out_hel allowed)
// or one of the mixed modes (FP32 parts, FP16 hi/lo MFMA colour sum).
template <class P>
int launch_split(int mode, const double* mom, int64_t nevt, double* out, double* out_hel, const MeParams& prm,
                 hipStream_t stream, void* ws, int64_t ws_bytes, const PartLaunchFn* parts64, int n64,
                 const PartLaunchFn* parts32, int n32) {
  if (nevt <= 0) return 0;
  if ((nevt + 255) / 256 > 0x7fffffffLL) return -1;
  if (mode == ME_MODE_FP64)
    return run_split<P, double>(mom, nevt, out, out_hel, prm, stream, ws, ws_bytes, parts64, n64);
  if (mode != ME_MODE_MIXED && mode != ME_MODE_MIXED_VALU && mode != ME_MODE_MIXED_MFMA32 &&
      mode != ME_MODE_MIXED_MFMA16 && mode != ME_MODE_MIXED_MFMABF16)
    return -1;
  if (out_hel || !out) return -1;
  return run_split<P, float>(mom, nevt, out, nullptr, prm, stream, ws, ws_bytes, parts32, n32);
}

}  // namespace me
