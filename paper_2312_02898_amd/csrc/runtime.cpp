// Host runtime of the C ABI declared in include/me.h: process lookup,
// couplings, helicity filtering, argument validation and kernel launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "me.h"
#include "channels.hpp"
#include "handle.hpp"
#include "me_types.h"
#include "gen/process_table.inc"

namespace {

thread_local std::string g_err = "";

me_status fail(me_status code, const std::string& msg) {
  g_err = msg;
  return code;
}
me_status hip_fail(hipError_t e, const char* what) {
  return fail(ME_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

const me::ProcessEntry* find_process(const char* process) {
  if (!process) return nullptr;
  // normalise whitespace
  std::string want;
  bool sp = false;
  for (const char* c = process; *c; ++c) {
    if (*c == ' ' || *c == '\t') { sp = !want.empty(); continue; }
    if (sp) { want.push_back(' '); sp = false; }
    want.push_back(*c);
  }
  for (const auto& e : kProcessTable)
    if (want == e.process || want == e.name) return &e;
  return nullptr;
}

// ------------------------------------------------------------ host RAMBO
// Flat phase space (Kleiss, Stirling, Ellis 1986) for the helicity-filter
// sample, in the centre-of-mass frame with the beams on +-z.  Random numbers
// from splitmix64 (Steele, Lea, Flood 2014), 53-bit mantissa in (0, 1].
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double((next() >> 11) + 1)) * (1.0 / 9007199254740992.0); }
};

void rambo_event(SplitMix64& rng, double sqrt_s, const std::vector<double>& masses, double* out) {
  const int n = int(masses.size());
  const double pi = 3.14159265358979323846;
  std::vector<double> q(4 * n), p(4 * n);
  double Q[4] = {0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    double c = 2.0 * rng.uniform() - 1.0, phi = 2.0 * pi * rng.uniform();
    double q0 = -std::log(rng.uniform() * rng.uniform());
    double s = std::sqrt(std::max(0.0, 1.0 - c * c));
    q[4 * i] = q0; q[4 * i + 1] = q0 * s * std::cos(phi); q[4 * i + 2] = q0 * s * std::sin(phi);
    q[4 * i + 3] = q0 * c;
    for (int m = 0; m < 4; ++m) Q[m] += q[4 * i + m];
  }
  const double M = std::sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
  const double gam = Q[0] / M, a = 1.0 / (1.0 + gam), x = sqrt_s / M;
  for (int i = 0; i < n; ++i) {
    const double* qi = &q[4 * i];
    double bq = b[0] * qi[1] + b[1] * qi[2] + b[2] * qi[3];
    p[4 * i] = x * (gam * qi[0] + bq);
    for (int k = 0; k < 3; ++k) p[4 * i + 1 + k] = x * (qi[1 + k] + b[k] * qi[0] + a * bq * b[k]);
  }
  double msum = 0;
  for (double m : masses) msum += m;
  if (msum > 0) {
    double xi = std::sqrt(1.0 - (msum / sqrt_s) * (msum / sqrt_s));
    for (int it = 0; it < 50; ++it) {
      double f = -sqrt_s, df = 0;
      for (int i = 0; i < n; ++i) {
        double e = std::sqrt(masses[i] * masses[i] + xi * xi * p[4 * i] * p[4 * i]);
        f += e;
        df += xi * p[4 * i] * p[4 * i] / e;
      }
      if (std::fabs(f) <= 1e-14 * sqrt_s) break;
      xi -= f / df;
    }
    for (int i = 0; i < n; ++i) {
      double e = std::sqrt(masses[i] * masses[i] + xi * xi * p[4 * i] * p[4 * i]);
      p[4 * i] = e;
      for (int k = 1; k < 4; ++k) p[4 * i + k] *= xi;
    }
  }
  const double e = 0.5 * sqrt_s;
  const double in[8] = {e, 0, 0, e, e, 0, 0, -e};
  std::memcpy(out, in, sizeof(in));
  std::memcpy(out + 8, p.data(), sizeof(double) * 4 * n);
}

}  // namespace

namespace me {

me_status set_error(me_status code, const std::string& msg) { return fail(code, msg); }

me_status compute_on(me_handle h, const double* d_momenta, int64_t nevt, double* d_me, hipStream_t s, void* ws,
                     int64_t ws_bytes, const MeParams* kp) {
  if (!h) return fail(ME_EINVAL, "me_compute: null handle");
  if (nevt < 0) return fail(ME_EINVAL, "me_compute: nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!d_momenta || !d_me) return fail(ME_EINVAL, "me_compute: null pointer");
  if (h->debug) {
    const int64_t bad = validate_momenta(d_momenta, nevt, h->proc->npar, s);
    if (bad < 0) return fail(ME_EHIP, "me_compute: momentum validation failed to run");
    if (bad > 0)
      return fail(ME_EINVAL, "me_compute: " + std::to_string(bad) +
                                 " events with non-finite components, negative energy or unbalanced momentum");
  }
  const int rc = h->proc->launch(mode_of(h->params), d_momenta, nevt, d_me, nullptr, kp ? kp : &h->kp, s, ws,
                                 ws_bytes);
  if (rc == -3)
    return fail(ws ? ME_EINVAL : ME_ENOMEM,
                ws ? "me_compute: workspace too small" : "me_compute: no device memory for the workspace");
  if (rc != 0) {
    hipError_t le = hipGetLastError();
    return fail(ME_EHIP, std::string("me_compute: launch failed: ") + hipGetErrorString(le));
  }
  return ME_OK;
}

me_status compute_channels_on(const me_handle* handles, int32_t nchannels, const double* d_momenta,
                              const int32_t* d_channel, const double* d_alphas, int64_t nevt, double* d_me,
                              hipStream_t s, void* ws, int64_t ws_bytes, const char* who) {
  const std::string w_ = who;
  if (!handles || nchannels < 1 || nchannels > chan::kMaxChannels) return fail(ME_EINVAL, w_ + ": need 1..32 handles");
  for (int c = 0; c < nchannels; ++c)
    if (!handles[c]) return fail(ME_EINVAL, w_ + ": null handle");
  const int npar = handles[0]->proc->npar;
  for (int c = 1; c < nchannels; ++c)
    if (handles[c]->proc->npar != npar)
      return fail(ME_EINVAL, w_ + ": channels must have the same number of legs");
  if (nevt < 0) return fail(ME_EINVAL, w_ + ": nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!d_momenta || !d_channel || !d_me) return fail(ME_EINVAL, w_ + ": null pointer");
  const size_t need = chan::workspace_bytes(nevt, nchannels, npar);
  void* base = ws;
  if (ws) {
    // a caller workspace: nothing may allocate
    if (ws_bytes < 0 || size_t(ws_bytes) < need)
      return fail(ME_EINVAL, w_ + ": " + std::to_string(nevt) + " events need " + std::to_string(need) +
                                 " bytes of workspace, more than the " + std::to_string(ws_bytes) + " available");
    for (int c = 0; c < nchannels; ++c)
      if (handles[c]->proc->workspace(mode_of(handles[c]->params), 1, handles[c]->kp.nhel, 0) > 0)
        return fail(ME_ENOTSUP, w_ + ": process '" + handles[c]->proc->process +
                                    "' needs a workspace of its own (split form)");
  } else if (hipMallocAsync(&base, need, s) != hipSuccess) {
    return fail(ME_ENOMEM, w_ + ": no device memory for the workspace");
  }
  const chan::Workspace w = chan::carve(base, nevt, nchannels, npar);
  int64_t totals[chan::kMaxChannels];
  int32_t bad = 0;
  hipError_t err = chan::partition(d_channel, nevt, nchannels, w, totals, &bad, s);
  if (err != hipSuccess || bad) {
    if (!ws) (void)hipFreeAsync(base, s);
    if (err != hipSuccess) return hip_fail(err, (w_ + ": partition").c_str());
    return fail(ME_EINVAL, w_ + ": channel index out of range");
  }
  chan::Scale sc;
  int64_t off = 0;
  int rc = 0;
  for (int c = 0; c < nchannels; ++c) {
    sc.aref[c] = handles[c]->params.alpha_s;
    sc.power[c] = handles[c]->proc->alphas_power;
    if (totals[c] == 0) continue;
    err = chan::gather(d_momenta, w.perm + off, totals[c], npar, w.mom + off * 4 * npar, s);
    if (err != hipSuccess) break;
    const me_handle h = handles[c];
    rc = h->proc->launch(mode_of(h->params), w.mom + off * 4 * npar, totals[c], w.out + off, nullptr, &h->kp, s,
                         nullptr, 0);
    if (rc != 0) {
      err = hipGetLastError();
      if (err == hipSuccess) err = hipErrorLaunchFailure;
      break;
    }
    off += totals[c];
  }
  if (err == hipSuccess) err = chan::scatter(w.out, w.perm, d_channel, d_alphas, sc, nevt, d_me, s);
  if (!ws) (void)hipFreeAsync(base, s);
  if (rc == -3) return fail(ME_ENOMEM, w_ + ": no device memory for a channel's workspace");
  if (err != hipSuccess) return hip_fail(err, w_.c_str());
  return ME_OK;
}

}  // namespace me


extern "C" {

const char* me_last_error(void) { return g_err.c_str(); }

void me_default_params(me_sm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->alpha_em = 1.0 / 132.507;
  p->sin2_thetaw = 0.2222;
  p->mz = 91.188; p->wz = 2.441;
  p->mt = 173.0; p->wt = 1.49;
  p->alpha_s = 0.118;
  p->tchannel_zero_width = 1;
  p->precision = ME_FP64;
  p->filter_sqrt_s = 1500.0;
  p->filter_seed = 1;
  p->filter_nevt = 1024;
}

me_status me_create(const char* process, const me_sm_params* p, me_handle* out) {
  if (!process || !p || !out) return fail(ME_EINVAL, "me_create: null argument");
  const me::ProcessEntry* e = find_process(process);
  if (!e) return fail(ME_EPROCESS, std::string("me_create: unknown process '") + process + "'");
  if (p->precision != ME_FP64 && p->precision != ME_MIXED && p->precision != ME_MIXED_VALU &&
      p->precision != ME_MIXED_MFMA32 && p->precision != ME_MIXED_MFMA16 && p->precision != ME_MIXED_MFMABF16)
    return fail(ME_EINVAL, "me_create: bad precision");
  if (!(p->alpha_em > 0) || !(p->alpha_s > 0) || !(p->sin2_thetaw > 0 && p->sin2_thetaw < 1) || !(p->mz > 0) ||
      !(p->wz >= 0) || !(p->mt >= 0) || !(p->wt >= 0) || p->filter_nevt < 1 || !(p->filter_sqrt_s > 0))
    return fail(ME_EINVAL, "me_create: parameter out of range");
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_fail(he, "me_create: hipGetDevice");
  me_handle h = new (std::nothrow) me_handle_s();
  if (!h) return fail(ME_ENOMEM, "me_create: out of host memory");
  h->proc = e;
  h->params = *p;
  h->device = dev;
  h->filtered = 0;
  {
    const char* dbg = std::getenv("ME_DEBUG");
    h->debug = dbg && *dbg && std::strcmp(dbg, "0") != 0;
  }
  const double pi = 3.14159265358979323846;
  const double ee = std::sqrt(4.0 * pi * p->alpha_em);
  const double s2 = p->sin2_thetaw, sw = std::sqrt(s2), cw = std::sqrt(1.0 - s2);
  const double Q = -1.0, T3 = -0.5;
  const double cl = (T3 - Q * s2) / (sw * cw), cr = (-Q * s2) / (sw * cw);
  me::MeParams& k = h->kp;
  std::memset(&k, 0, sizeof(k));
  k.gs = std::sqrt(4.0 * pi * p->alpha_s);
  k.ea = -ee * Q;
  k.gzl = -ee * cl;
  k.gzr = -ee * cr;
  k.mz = p->mz; k.wz = p->wz;
  k.mt = p->mt; k.wt = p->wt;
  k.wt_tchan = p->tchannel_zero_width ? 0.0 : p->wt;
  k.nhel = e->nhel;
  for (int i = 0; i < e->nhel; ++i) k.hel[i] = uint8_t(i);
  *out = h;
  return ME_OK;
}

me_status me_helicity_filter(me_handle h) {
  if (!h) return fail(ME_EINVAL, "me_helicity_filter: null handle");
  if (h->filtered) return ME_OK;
  const me::ProcessEntry* e = h->proc;
  const int n = h->params.filter_nevt, npar = e->npar, nhel = e->nhel;
  std::vector<double> masses(npar - 2, 0.0);
  if (e->massive_top) masses[0] = masses[1] = h->params.mt;
  if (h->params.filter_sqrt_s <= 2.0 * h->params.mt && e->massive_top)
    return fail(ME_EINVAL, "me_helicity_filter: filter_sqrt_s below threshold");
  std::vector<double> mom(size_t(n) * npar * 4);
  SplitMix64 rng{h->params.filter_seed};
  for (int i = 0; i < n; ++i) rambo_event(rng, h->params.filter_sqrt_s, masses, &mom[size_t(i) * npar * 4]);
  double *d_mom = nullptr, *d_hel = nullptr;
  hipError_t he = hipMalloc(&d_mom, mom.size() * sizeof(double));
  if (he != hipSuccess) return hip_fail(he, "me_helicity_filter: hipMalloc");
  he = hipMalloc(&d_hel, size_t(n) * nhel * sizeof(double));
  if (he != hipSuccess) { (void)hipFree(d_mom); return hip_fail(he, "me_helicity_filter: hipMalloc"); }
  std::vector<double> mh(size_t(n) * nhel);
  me::MeParams all = h->kp;
  all.nhel = nhel;
  for (int i = 0; i < nhel; ++i) all.hel[i] = uint8_t(i);
  int rc = -1;
  he = hipMemcpy(d_mom, mom.data(), mom.size() * sizeof(double), hipMemcpyHostToDevice);
  if (he == hipSuccess) rc = e->launch(me::ME_MODE_FP64, d_mom, n, nullptr, d_hel, &all, nullptr, nullptr, 0);
  if (he == hipSuccess && rc == 0) he = hipMemcpy(mh.data(), d_hel, mh.size() * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d_mom);
  (void)hipFree(d_hel);
  if (he != hipSuccess) return hip_fail(he, "me_helicity_filter");
  if (rc != 0) return fail(ME_EHIP, "me_helicity_filter: kernel launch failed");
  // keep h iff max over events of |M_h|^2 / sum_h' |M_h'|^2 exceeds 1e-24
  std::vector<double> best(nhel, 0.0);
  for (int i = 0; i < n; ++i) {
    double tot = 0;
    for (int k = 0; k < nhel; ++k) tot += mh[size_t(i) * nhel + k];
    if (!(tot > 0) || !std::isfinite(tot)) continue;
    for (int k = 0; k < nhel; ++k) best[k] = std::max(best[k], mh[size_t(i) * nhel + k] / tot);
  }
  int ng = 0;
  for (int k = 0; k < nhel; ++k)
    if (best[k] > 1e-24) h->kp.hel[ng++] = uint8_t(k);
  if (ng == 0) return fail(ME_EINVAL, "me_helicity_filter: no helicity survived (bad filter sample?)");
  h->kp.nhel = ng;
  h->filtered = 1;
  return ME_OK;
}

me_status me_compute(me_handle h, const double* d_momenta, int64_t nevt, double* d_me, void* hip_stream) {
  return me::compute_on(h, d_momenta, nevt, d_me, static_cast<hipStream_t>(hip_stream), nullptr, 0);
}

namespace {
__global__ void weight_max_clear(unsigned long long* bits) { *bits = 0ull; }
}  // namespace

me_status me_compute_weighted(me_handle h, const double* d_momenta, int64_t nevt, const double* d_factor,
                              double* d_me, double* d_w, double* d_max, void* hip_stream) {
  if (!h) return fail(ME_EINVAL, "me_compute_weighted: null handle");
  if (nevt < 0) return fail(ME_EINVAL, "me_compute_weighted: nevt < 0");
  if (!d_max || (nevt > 0 && (!d_momenta || !d_factor || !d_me)))
    return fail(ME_EINVAL, "me_compute_weighted: null pointer");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  auto* bits = reinterpret_cast<unsigned long long*>(d_max);
  // a fill kernel, not a memset: the call stays safe to capture in a graph
  hipLaunchKernelGGL(weight_max_clear, dim3(1), dim3(1), 0, s, bits);
  if (hipGetLastError() != hipSuccess) return fail(ME_EHIP, "me_compute_weighted: launch failed");
  if (nevt == 0) return ME_OK;
  me::MeParams kp = h->kp;
  kp.w_fac = d_factor;
  kp.w_out = d_w;
  kp.w_max = bits;
  return me::compute_on(h, d_momenta, nevt, d_me, s, nullptr, 0, &kp);
}

me_status me_workspace_bytes(me_handle h, int64_t nevt, int64_t* bytes) {
  if (!h || !bytes || nevt < 0) return fail(ME_EINVAL, "me_workspace_bytes: bad argument");
  *bytes = h->proc->workspace(me::mode_of(h->params), nevt, h->kp.nhel, 0);
  return ME_OK;
}

me_status me_compute_channels(const me_handle* handles, int32_t nchannels, const double* d_momenta,
                              const int32_t* d_channel, const double* d_alphas, int64_t nevt, double* d_me,
                              void* hip_stream) {
  return me::compute_channels_on(handles, nchannels, d_momenta, d_channel, d_alphas, nevt, d_me,
                                 static_cast<hipStream_t>(hip_stream), nullptr, 0, "me_compute_channels");
}

me_status me_compute_helicities(me_handle h, const double* d_momenta, int64_t nevt, double* d_me_hel,
                                void* hip_stream) {
  if (!h) return fail(ME_EINVAL, "me_compute_helicities: null handle");
  if (nevt < 0) return fail(ME_EINVAL, "me_compute_helicities: nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!d_momenta || !d_me_hel) return fail(ME_EINVAL, "me_compute_helicities: null pointer");
  me::MeParams all = h->kp;
  all.nhel = h->proc->nhel;
  for (int i = 0; i < all.nhel; ++i) all.hel[i] = uint8_t(i);
  int rc = h->proc->launch(me::ME_MODE_FP64, d_momenta, nevt, nullptr, d_me_hel, &all,
                           static_cast<hipStream_t>(hip_stream), nullptr, 0);
  if (rc != 0) return fail(ME_EHIP, "me_compute_helicities: launch failed");
  return ME_OK;
}

me_status me_good_helicities(me_handle h, int32_t* hel, int32_t cap, int32_t* n) {
  if (!h || !n || (cap > 0 && !hel) || cap < 0) return fail(ME_EINVAL, "me_good_helicities: bad argument");
  *n = h->kp.nhel;
  for (int i = 0; i < h->kp.nhel && i < cap; ++i) hel[i] = h->kp.hel[i];
  return ME_OK;
}

me_status me_info(me_handle h, me_info_t* info) {
  if (!h || !info) return fail(ME_EINVAL, "me_info: null argument");
  const me::ProcessEntry* e = h->proc;
  info->npar = e->npar;
  info->nhel = e->nhel;
  info->nhel_good = h->kp.nhel;
  info->ndiagrams = e->ndiagrams;
  info->ncolor = e->ncolor;
  info->iden = e->iden;
  info->flops_per_event = int64_t(e->flops_per_hel) * h->kp.nhel;
  info->bytes_per_event = int64_t(32) * e->npar + 8;
  info->precision = h->params.precision;
  info->filtered = h->filtered;
  return ME_OK;
}

me_status me_destroy(me_handle h) {
  if (!h) return fail(ME_EINVAL, "me_destroy: null handle");
  delete h;
  return ME_OK;
}

}  // extern "C"
