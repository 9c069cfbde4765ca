// Device-side channel partition, gather and rescaling scatter for
// multi-subprocess requests (see channels.hpp).  All kernels are plain
// vector-memory code: per-block LDS counters, one wave-level ballot per
// channel for the stable ranks, one block for the scan over blocks.
#include "channels.hpp"
#include "handle.hpp"

namespace me {
namespace chan {
namespace {

constexpr int kBlock = 256;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

__global__ __launch_bounds__(kBlock) void count_kernel(const int32_t* __restrict__ ch, int64_t n, int nch,
                                                       int32_t* __restrict__ counts, int32_t* __restrict__ bad) {
  __shared__ int32_t c[kMaxChannels];
  if (threadIdx.x < unsigned(nch)) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e < n) {
    const int k = ch[e];
    if (k >= 0 && k < nch) atomicAdd(&c[k], 1);
    else atomicOr(bad, 1);
  }
  __syncthreads();
  if (threadIdx.x < unsigned(nch)) counts[int64_t(blockIdx.x) * nch + threadIdx.x] = c[threadIdx.x];
}

// offs[c * nblk + b] = events before block b's events of channel c in the
// channel-major order; totals[c] = events of channel c.  One block.
__global__ __launch_bounds__(kBlock) void scan_kernel(const int32_t* __restrict__ counts, int64_t nblk, int nch,
                                                      int64_t* __restrict__ offs, int64_t* __restrict__ totals) {
  __shared__ int64_t part[kBlock];
  __shared__ int64_t tot;
  const int t = threadIdx.x;
  const int64_t chunk = (nblk + kBlock - 1) / kBlock;
  const int64_t b0 = t * chunk < nblk ? t * chunk : nblk;
  const int64_t b1 = b0 + chunk < nblk ? b0 + chunk : nblk;
  int64_t base = 0;
  for (int c = 0; c < nch; ++c) {
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += counts[b * nch + c];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
      int64_t a = 0;
      for (int i = 0; i < kBlock; ++i) {
        const int64_t v = part[i];
        part[i] = a;
        a += v;
      }
      tot = a;
      totals[c] = a;
    }
    __syncthreads();
    int64_t run = base + part[t];
    for (int64_t b = b0; b < b1; ++b) {
      offs[c * nblk + b] = run;
      run += counts[b * nch + c];
    }
    base += tot;
    __syncthreads();
  }
}

// perm[offs[c][b] + rank] = e, rank = position of e among its block's
// events of channel c (wave ballots, then the waves before it).
__global__ __launch_bounds__(kBlock) void perm_kernel(const int32_t* __restrict__ ch, int64_t n, int nch,
                                                      const int64_t* __restrict__ offs, int64_t nblk,
                                                      int64_t* __restrict__ perm) {
  __shared__ int32_t wcnt[kBlock / 64][kMaxChannels];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int k = e < n ? ch[e] : -1;
  const bool valid = k >= 0 && k < nch;
  int rank = 0;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int c = 0; c < nch; ++c) {
    const unsigned long long m = __ballot(valid && k == c);
    if (lane == 0) wcnt[w][c] = __popcll(m);
    if (valid && k == c) rank = __popcll(m & below);
  }
  __syncthreads();
  if (valid) {
    int before = 0;
    for (int v = 0; v < w; ++v) before += wcnt[v][k];
    perm[offs[int64_t(k) * nblk + blockIdx.x] + before + rank] = e;
  }
}

__global__ __launch_bounds__(kBlock) void gather_kernel(const double* __restrict__ mom,
                                                        const int64_t* __restrict__ perm, int64_t n, int width,
                                                        double* __restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n * width) return;
  const int64_t j = i / width, q = i % width;
  dst[i] = mom[perm[j] * width + q];
}

__global__ __launch_bounds__(kBlock) void scatter_kernel(const double* __restrict__ res,
                                                         const int64_t* __restrict__ perm,
                                                         const int32_t* __restrict__ ch,
                                                         const double* __restrict__ alphas, const Scale sc,
                                                         int64_t n, double* __restrict__ out) {
  const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= n) return;
  const int64_t e = perm[j];
  double v = res[j];
  if (alphas) {
    const int c = ch[e];
    const double r = alphas[e] / sc.aref[c];
    double f = 1.0;
    for (int q = 0; q < sc.power[c]; ++q) f *= r;
    v *= f;
  }
  out[e] = v;
}

__global__ void clear_flag(int32_t* flag) { *flag = 0; }

int64_t nblocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

size_t workspace_bytes(int64_t nevt, int nch, int npar) {
  const int64_t nb = nblocks(nevt);
  return align256(size_t(nevt) * 8) * 2 + align256(size_t(nevt) * 32 * npar) +
         align256(size_t(nb) * nch * 4) + align256(size_t(nb) * nch * 8) + align256(size_t(nch) * 8) + 256;
}

Workspace carve(void* base, int64_t nevt, int nch, int npar) {
  const int64_t nb = nblocks(nevt);
  char* p = static_cast<char*>(base);
  Workspace w;
  w.perm = reinterpret_cast<int64_t*>(p);
  p += align256(size_t(nevt) * 8);
  w.out = reinterpret_cast<double*>(p);
  p += align256(size_t(nevt) * 8);
  w.mom = reinterpret_cast<double*>(p);
  p += align256(size_t(nevt) * 32 * npar);
  w.counts = reinterpret_cast<int32_t*>(p);
  p += align256(size_t(nb) * nch * 4);
  w.offs = reinterpret_cast<int64_t*>(p);
  p += align256(size_t(nb) * nch * 8);
  w.totals = reinterpret_cast<int64_t*>(p);
  p += align256(size_t(nch) * 8);
  w.bad = reinterpret_cast<int32_t*>(p);
  return w;
}

hipError_t partition(const int32_t* d_channel, int64_t nevt, int nch, const Workspace& w, int64_t* h_totals,
                     int32_t* h_bad, hipStream_t s) {
  const int64_t nb = nblocks(nevt);
  if (nb > 0x7fffffffLL || nch < 1 || nch > kMaxChannels) return hipErrorInvalidValue;
  hipLaunchKernelGGL(clear_flag, dim3(1), dim3(1), 0, s, w.bad);
  hipLaunchKernelGGL(count_kernel, dim3(unsigned(nb)), dim3(kBlock), 0, s, d_channel, nevt, nch, w.counts, w.bad);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kBlock), 0, s, w.counts, nb, nch, w.offs, w.totals);
  hipLaunchKernelGGL(perm_kernel, dim3(unsigned(nb)), dim3(kBlock), 0, s, d_channel, nevt, nch, w.offs, nb, w.perm);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  err = hipMemcpyAsync(h_totals, w.totals, sizeof(int64_t) * nch, hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipMemcpyAsync(h_bad, w.bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  return err;
}

hipError_t gather(const double* mom, const int64_t* perm, int64_t n, int npar, double* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t total = n * 4 * npar;
  const int64_t nb = (total + kBlock - 1) / kBlock;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gather_kernel, dim3(unsigned(nb)), dim3(kBlock), 0, s, mom, perm, n, 4 * npar, dst);
  return hipGetLastError();
}

hipError_t scatter(const double* res, const int64_t* perm, const int32_t* channel, const double* alphas,
                   const Scale& sc, int64_t nevt, double* out, hipStream_t s) {
  if (nevt <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(unsigned(nblocks(nevt))), dim3(kBlock), 0, s, res, perm, channel, alphas,
                     sc, nevt, out);
  return hipGetLastError();
}

}  // namespace chan

namespace {
__global__ __launch_bounds__(256) void validate_kernel(const double* __restrict__ mom, int64_t n, int npar,
                                                       unsigned long long* __restrict__ bad) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= n) return;
  const double* p = mom + e * 4 * npar;
  double bal[4] = {0, 0, 0, 0};
  bool ok = true;
  for (int i = 0; i < npar; ++i) {
    for (int c = 0; c < 4; ++c) {
      const double v = p[4 * i + c];
      ok = ok && isfinite(v);
      bal[c] += i < 2 ? v : -v;
    }
    ok = ok && p[4 * i] >= 0.0;
  }
  const double scale = p[0] + p[4];
  for (int c = 0; c < 4; ++c) ok = ok && fabs(bal[c]) <= 1e-9 * scale;
  if (!ok) atomicAdd(bad, 1ull);
}
__global__ void clear_u64(unsigned long long* x) { *x = 0ull; }
}  // namespace

int64_t validate_momenta(const double* d_mom, int64_t nevt, int npar, hipStream_t s) {
  if (nevt <= 0) return 0;
  const int64_t nb = (nevt + 255) / 256;
  if (nb > 0x7fffffffLL) return -1;
  unsigned long long* d_bad = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&d_bad), sizeof(unsigned long long), s) != hipSuccess) return -1;
  hipLaunchKernelGGL(clear_u64, dim3(1), dim3(1), 0, s, d_bad);
  hipLaunchKernelGGL(validate_kernel, dim3(unsigned(nb)), dim3(256), 0, s, d_mom, nevt, npar, d_bad);
  unsigned long long h_bad = 0;
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) err = hipMemcpyAsync(&h_bad, d_bad, sizeof(h_bad), hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  (void)hipFreeAsync(d_bad, s);
  return err == hipSuccess ? int64_t(h_bad) : -1;
}

}  // namespace me
