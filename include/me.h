/*
 * me.h -- C ABI of the MI355X (gfx950) leading-order matrix-element engine.
 *
 * The engine evaluates, for a batch of phase-space points ("events"), the
 * spin- and colour-summed, initial-state averaged squared matrix element
 * |M|^2 of a fixed tree-level process: the quantity the paper (Sec. 2 and
 * Sec. 3) identifies as the most expensive part of event generation and
 * offloads to GPUs with event-level data parallelism.  Per event the device
 * computes external wavefunctions, HELAS-style vertex and propagator calls for
 * every Feynman diagram and helicity, the colour-flow amplitudes jamp, the
 * colour sum jamp^H C jamp and the helicity sum.
 *
 * Supported processes (Summary section of the paper: LO QED/QCD; the
 * processes validated there are e+e- -> mu+mu- and gg -> ttbar + 0..3 g,
 * and p p -> t tbar + jets is named as the next target):
 *     "e+ e- > mu+ mu-"
 *     "g g > t t~"  "g g > t t~ g"  "g g > t t~ g g"  "g g > t t~ g g g"
 *     "u u~ > t t~"  "u~ u > t t~"                      (p p > t t~, quark channels)
 *     "u u~ > t t~ g"  "u~ u > t t~ g"  "u g > t t~ u"  "g u > t t~ u"
 *     "u~ g > t t~ u~"  "g u~ > t t~ u~"               (p p > t t~ + 1 jet)
 *     "u u~ > t t~ g g"  "u~ u > t t~ g g"  "u g > t t~ u g"  "g u > t t~ u g"
 *     "u~ g > t t~ u~ g"  "g u~ > t t~ u~ g"  "g g > t t~ u u~"
 *     "u u~ > t t~ u u~"  "u u~ > t t~ d d~"  "u u > t t~ u u"
 *     "u d > t t~ u d"  "u~ u~ > t t~ u~ u~"          (p p > t t~ + 2 jets)
 * The short names "eemumu", "ggtt", "ggttg", "ggttgg", "ggttggg", "uutt",
 * "uxutt", "uuttg", "uxuttg", "ugttu", "guttu", "uxgttux", "guxttux",
 * "uuttgg", "uxuttgg", "ugttug", "guttug", "uxgttuxg", "guxttuxg", "ggttuux",
 * "uuttuux", "uuttddx", "uuttuu", "udttud", "uxuxttuxux" are accepted too.  "g g > t t~ g g g" runs in a split form whose jamp
 * workspace (me_workspace_bytes) comes from the stream-ordered allocator.
 *
 * Conventions
 *   momenta   const double mom[nevt][npar][4], (E, px, py, pz) in GeV, in
 *             DEVICE memory, legs in the order of the process string, legs 0
 *             and 1 incoming.  Events must be in the partonic centre-of-mass
 *             frame with the beams along +-z: the helicity filter's list of
 *             vanishing helicities is frame dependent for massive legs.
 *   output    double me[nevt] in device memory, in GeV^(4-2n) for 2 -> n.
 *   helicity  configuration h in [0, 2^npar): leg i has helicity +1 iff bit i
 *             of h is set.
 *   widths    fixed-width propagators; in the "zero-width t-channel mode" of
 *             the paper (Sec. 3, Tables 1-2) the top width is 0 in every
 *             propagator whose momentum is the sum of exactly one incoming
 *             leg and some outgoing legs.
 *
 * Ownership and threading
 *   A handle owns its device constants; the caller owns momenta, outputs and
 *   streams.  me_compute is asynchronous and stream-ordered: results are valid
 *   once the stream has been synchronised, and the inputs must stay alive until
 *   then.  After me_helicity_filter a handle is read-only, so me_compute may be
 *   called concurrently on several streams.  me_destroy must not race with
 *   work in flight.
 *
 * Errors
 *   Every function returns an me_status; 0 is success.  Null pointers and
 *   negative sizes give ME_EINVAL, an unknown process ME_EPROCESS, a failed
 *   allocation ME_ENOMEM, a failed HIP call ME_EHIP.  nevt == 0 is a no-op.
 *   me_last_error() returns a thread-local message for the last failure.
 *   Momentum values are not validated on the hot path.
 */
#ifndef ME_H
#define ME_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct me_handle_s* me_handle;
typedef int32_t me_status;

enum {
  ME_OK = 0,
  ME_EINVAL = -1,
  ME_EPROCESS = -2,
  ME_ENOMEM = -3,
  ME_EHIP = -4,
  ME_ENOTSUP = -5,
  ME_EBUSY = -6
};

typedef enum {
  ME_FP64 = 0,       /* all arithmetic in FP64 */
  ME_MIXED = 1,      /* FP32 wavefunctions and vertices; FP64 momenta, p^2,
                        propagator denominators and helicity-sum accumulation;
                        colour sum on the unit measured fastest for the
                        process (one of the three below; gg -> t t~ g g g
                        always uses FP16 hi+lo MFMA) */
  ME_MIXED_VALU = 2, /* as ME_MIXED with the colour sum on the FP32 vector
                        ALU (processes of up to 32 colour flows) */
  ME_MIXED_MFMA32 = 3, /* as ME_MIXED with the colour sum on MFMA with FP32
                        operands (exact FP32 jamps and colour matrix, no
                        hi+lo split) for 6..32 colour flows */
  ME_MIXED_MFMA16 = 4, /* as ME_MIXED with the colour sum on MFMA with FP16
                        hi+lo jamps, exact FP16 colour matrix and FP32
                        accumulation, for 6..32 colour flows and the split
                        form */
  ME_MIXED_MFMABF16 = 5 /* as ME_MIXED with the colour sum on MFMA with BF16
                        hi+lo jamps (16 significant bits), exact BF16 colour
                        matrix and FP32 accumulation, for 6..32 colour flows
                        (other processes: vector ALU; the split form keeps
                        FP16 hi+lo, its colour matrix needing 9 bits) */
} me_precision;

/* Standard-Model inputs.  me_default_params() fills the benchmark values
 * alpha = 1/132.507, sin^2 thetaW = 0.2222, MZ = 91.188, GZ = 2.441,
 * mt = 173, Gt = 1.49, alpha_s = 0.118, zero-width t-channel mode on, FP64,
 * helicity-filter sample of 1024 events at sqrt(s) = 1500 GeV, seed 1. */
typedef struct {
  double alpha_em;
  double sin2_thetaw;
  double mz, wz;
  double mt, wt;
  double alpha_s;
  int32_t tchannel_zero_width;
  int32_t precision;        /* me_precision */
  double filter_sqrt_s;     /* CM energy of the helicity-filter sample (GeV) */
  uint64_t filter_seed;
  int32_t filter_nevt;      /* number of filter events (>= 1) */
  int32_t reserved;
} me_sm_params;

typedef struct {
  int32_t npar;             /* external legs */
  int32_t nhel;             /* 2^npar helicity configurations */
  int32_t nhel_good;        /* configurations summed by me_compute */
  int32_t ndiagrams;        /* tree-level Feynman diagrams */
  int32_t ncolor;           /* colour flows (jamps) */
  int32_t iden;             /* averaging and symmetry denominator */
  int64_t flops_per_event;  /* algorithmic flops of one me_compute event */
  int64_t bytes_per_event;  /* HBM bytes one event needs: 32 npar in + 8 out */
  int32_t precision;
  int32_t filtered;         /* 1 after me_helicity_filter */
} me_info_t;

/* Fill *p with the benchmark Standard-Model inputs listed above. */
void me_default_params(me_sm_params* p);

/* Create a handle for `process` (one of the strings above) with inputs *p on
 * the current HIP device.  The quantity it will compute is the LO |M|^2 of
 * the process (paper, Sec. 2: the "matrix elements" that dominate madevent;
 * Summary: LO QED and QCD), at the couplings, masses and widths of *p.
 * Copies the constants the kernels need (they travel in each launch's
 * argument block; the colour matrix is compiled in); *out receives the
 * handle, which the caller releases with me_destroy.  ME_EPROCESS for an
 * unknown process string, ME_EINVAL for null arguments or inputs out of
 * range (non-positive couplings or masses of the Z, negative widths). */
me_status me_create(const char* process, const me_sm_params* p, me_handle* out);

/* Helicity filtering at initialisation.  The paper does not discuss
 * helicities; skipping configurations whose |M_h|^2 vanishes leaves the
 * |M|^2 of me_compute (paper, Sec. 2) unchanged and only removes work.
 * Evaluates |M_h|^2 for all 2^npar
 * helicity configurations on filter_nevt RAMBO events at filter_sqrt_s
 * (centre-of-mass frame, seed filter_seed) in FP64 and keeps configuration h
 * iff max_events |M_h|^2 / sum_h' |M_h'|^2 > 1e-24.  Synchronous, idempotent.
 * Without it me_compute sums all 2^npar configurations (correct, slower). */
me_status me_helicity_filter(me_handle h);

/* |M|^2 for nevt events (paper, Sec. 2: the same function evaluated for
 * every event of a batch, in parallel over events): d_momenta [nevt][npar][4]
 * and d_me [nevt] are device pointers owned by the caller, hip_stream a
 * hipStream_t (NULL: default stream).  Asynchronous and stream-ordered;
 * d_me holds 1/IDEN sum_helicities sum_colours |M|^2 (FP64, in every
 * precision) once the stream is synchronised.  ME_EINVAL for a null handle or
 * pointer or nevt < 0 (nothing is launched), ME_EHIP if a launch fails;
 * nevt == 0 is a no-op.  Only "g g > t t~ g g g" allocates (its jamp
 * workspace, stream-ordered: ME_ENOMEM if that fails). */
me_status me_compute(me_handle h, const double* d_momenta, int64_t nevt, double* d_me,
                     void* hip_stream);

/* me_compute with the unweighting step of the paper's Sec. 3 (Table 2: the
 * event weights and their batch maximum formed on the device) fused into the
 * kernel that produces |M|^2: besides d_me [nevt] it stores, when d_w is not
 * NULL, d_w[i] = max(d_me[i] * d_factor[i], 0) (NaN clamped to 0 as well),
 * and *d_max receives the maximum weight (0 for nevt == 0).  Bit for bit the
 * result of me_compute followed by me_max_weight(d_me, d_factor, nevt, d_w,
 * d_max).  All pointers are device pointers owned by the caller; d_factor
 * [nevt] holds each event's Jacobian x PDF factor.  Asynchronous on
 * hip_stream; *d_max is cleared on the stream by a kernel (no memset), so
 * the call may be captured in a graph except for "g g > t t~ g g g", whose
 * workspace is allocated as in me_compute.  ME_EINVAL for a null handle or
 * pointer or nevt < 0, ME_EHIP if a launch fails. */
me_status me_compute_weighted(me_handle h, const double* d_momenta, int64_t nevt, const double* d_factor,
                              double* d_me, double* d_w, double* d_max, void* hip_stream);

/* Multi-subprocess request: event e of the batch is evaluated with
 * handles[d_channel[e]] (e.g. the g g, u u~ and u~ u channels of
 * p p > t t~; the paper's Summary names p p -> t tbar + jets, whose
 * subprocesses share the final state and the momenta layout).
 *   handles      nchannels (1..32) handles with the same number of legs; each
 *                keeps its own precision and helicity selection.
 *   d_momenta    device [nevt][npar][4], as for me_compute.
 *   d_channel    device int32 [nevt], values in [0, nchannels).
 *   d_alphas     device [nevt] per-event strong coupling, or NULL.  Every
 *                diagram of these processes carries the same power of g_s, so
 *                |M|^2 = |M|^2(alpha_s of the handle) x (alpha_s(e) /
 *                alpha_s of the handle)^p exactly, p = 2 for 2 -> t t~ and one
 *                more per extra gluon (0 for e+ e- > mu+ mu-).
 *   d_me         device [nevt] output, FP64.
 * The events are partitioned by channel on the device (stable), gathered,
 * evaluated and scattered back.  Workspace (about 32 npar + 16 bytes per
 * event) comes from the stream-ordered allocator.  The call waits for the
 * per-channel counts (one short synchronisation of the stream); the
 * evaluation itself stays asynchronous.  ME_EINVAL for a channel index out of
 * range (nothing is written), mismatched legs or null pointers; ME_ENOMEM if
 * the workspace cannot be allocated. */
me_status me_compute_channels(const me_handle* handles, int32_t nchannels, const double* d_momenta,
                              const int32_t* d_channel, const double* d_alphas, int64_t nevt,
                              double* d_me, void* hip_stream);

/* Device workspace bytes that me_compute allocates (stream-ordered) for nevt
 * events of this handle: 0 for every process but "g g > t t~ g g g", whose
 * split form keeps its jamps in a workspace of up to 128 MiB per call.
 * ME_EINVAL for a null handle or pointer or nevt < 0. */
me_status me_workspace_bytes(me_handle h, int64_t nevt, int64_t* bytes);

/* Size of the fixed device workspace of me_compute_channels_noalloc. */
#define ME_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call and result as me_compute_channels, with its workspace (about
 * 32 npar + 16 bytes per event) in a fixed device array of
 * ME_NOALLOC_SCRATCH_BYTES per device instead of the stream-ordered
 * allocator.  Nothing is allocated: a batch whose workspace would exceed the
 * array gives ME_EINVAL (nothing is launched), a handle whose process needs
 * a workspace of its own ("g g > t t~ g g g") ME_ENOTSUP.  The array is
 * shared by every call on a device and keeps the last call's contents:
 * calls that overlap on one device (other streams or threads) race and
 * must be serialised by the caller.  Like me_compute_channels it waits once
 * for the per-channel counts. */
me_status me_compute_channels_noalloc(const me_handle* handles, int32_t nchannels, const double* d_momenta,
                                      const int32_t* d_channel, const double* d_alphas, int64_t nevt,
                                      double* d_me, void* hip_stream);

/* Debugging: with the environment variable ME_DEBUG set (not "0") when a
 * handle is created, me_compute first checks every event on the device
 * (finite components, E >= 0, incoming = outgoing four-momentum within 1e-9
 * of the incoming energy; this synchronises the stream) and returns
 * ME_EINVAL without computing if any event fails.  Off by default: the hot
 * path does not validate. */

/* Colour-summed (not averaged) |M_h|^2 of all 2^npar helicity configurations,
 * d_me_hel [nevt][2^npar], FP64.  Diagnostic; asynchronous. */
me_status me_compute_helicities(me_handle h, const double* d_momenta, int64_t nevt,
                                double* d_me_hel, void* hip_stream);

/* Good-helicity list after filtering: hel[0..*n) (capacity cap entries). */
me_status me_good_helicities(me_handle h, int32_t* hel, int32_t cap, int32_t* n);

/* Static data of the handle's process and current helicity selection. */
me_status me_info(me_handle h, me_info_t* info);

/* Release the handle.  No work on it may be in flight. */
me_status me_destroy(me_handle h);

/* Thread-local text of the last error (never NULL). */
const char* me_last_error(void);

/* GPU-assisted batch unweighting (paper, Sec. 3 and Table 2): event weights
 * w_i = d_me[i] * d_factor[i] (|M|^2 times the Jacobian x PDF factor) formed
 * on the device, and their maximum over the batch written to *d_max (device
 * memory, one double).  Negative or NaN products count as 0.  d_w [nevt]
 * receives the weights if non-NULL.  All pointers are device pointers;
 * asynchronous on hip_stream; nevt == 0 gives *d_max = 0.  The caller owns
 * every buffer; nothing is allocated. */
me_status me_max_weight(const double* d_me, const double* d_factor, int64_t nevt, double* d_w,
                        double* d_max, void* hip_stream);

/* Device-side phase-space generation: nevt RAMBO events (Kleiss, Stirling,
 * Ellis), the flat generator of the paper's standalone test-bed (Sec. 2),
 * written to d_momenta [nevt][nfinal+2][4] (device) in the layout me_compute
 * reads: two massless beams (sqrt_s/2)(1,0,0,+-1), then nfinal (2..5) final
 * particles with masses[0..nfinal) (host array, GeV).  Random numbers from
 * Philox4x32-10 with key = seed and counter = (event, 2*particle+half): the
 * batch is reproducible and any event range can be regenerated.  Asynchronous
 * on hip_stream; nothing is allocated.  ME_EINVAL for bad sizes or
 * sum(masses) >= sqrt_s. */
me_status me_rambo(int64_t nevt, int32_t nfinal, const double* masses, double sqrt_s, uint64_t seed,
                   double* d_momenta, void* hip_stream);

/* Device-side importance-sampled phase space (the structure of madevent's
 * mappings, which the paper's Sec. 3 profiles as the remaining host hotspot
 * once the matrix element runs on the GPU): sequential two-body splitting of
 * the centre-of-mass system (final particle nfinal-1 first, the last
 * remainder into particles 0 and 1), remainder masses favouring soft
 * splittings and polar angles peaked along the beams, Philox4x32-10
 * uniforms with key = seed and counter = (event, 0x10000 + 2 split + half).
 * Writes d_momenta [nevt][nfinal+2][4] (device; beams (sqrt_s/2)(1,0,0,+-1),
 * then the final particles with masses[0..nfinal) (host array, GeV)) and
 * d_weight [nevt] (device): each point's phase-space weight for
 * dPhi_n = (2pi)^4 delta^4 prod d^3p / ((2pi)^3 2E), so that the mean of
 * weight x f estimates the phase-space integral of f (feed weight / (2 s)
 * times PDFs to me_max_weight as its factor).  Asynchronous; nothing is
 * allocated.  ME_EINVAL for bad sizes, null pointers or sum(masses) >= sqrt_s. */
me_status me_sample(int64_t nevt, int32_t nfinal, const double* masses, double sqrt_s, uint64_t seed,
                    double* d_momenta, double* d_weight, void* hip_stream);

/* ------------------------------------------------------------ serving --
 * A persistent request loop for uneven |M|^2 batches of several processes,
 * as integration channels emit them (continuous batching).  A request's
 * device footprint is its momenta, its results and the workspace its
 * process needs ("g g > t t~ g g g": the jamp workspace, capped per request
 * at a quarter of budget_bytes and at most 128 MiB), all carved from one
 * device arena of budget_bytes allocated at creation; nothing is allocated
 * per request.  Requests are admitted in arrival order as stream slots and
 * arena memory free up; when the head of the queue waits for memory, at
 * most 16 later requests that fit may pass it before the queue is strictly
 * in order again.  Requests whose estimated work (flops of the process x
 * events) exceeds 2e10 are large: they may hold at most half of the slots,
 * small requests pass a large head that waits for such a slot, and a large
 * request above 2e11 runs in pieces of 16384 events with one piece's kernels
 * queued at a time, so a small request neither queues behind long ones nor
 * waits behind their whole kernel sequence on a shared hardware queue.
 * Admitted work on different slots overlaps on the device.
 * Host buffers: the server stages momenta to device memory and results
 * back.  Handles must be filtered before submission and stay alive while
 * their requests are in flight.
 */
typedef struct me_server_s* me_server;

typedef struct {
  int64_t submitted, completed, failed, rejected;
  int64_t events_completed;
  int64_t bytes_in_use, peak_bytes_in_use;
  int32_t active_slots, queued;
  int64_t bypassed;         /* admissions past a head that waited for memory */
  int64_t passed_large;     /* admissions past a large head that waited for a slot */
} me_server_stats_t;

/* n_slots HIP streams (1..64), budget_bytes of device memory for requests. */
me_status me_server_create(int64_t budget_bytes, int32_t n_slots, me_server* out);

/* Enqueue a request: h_momenta [nevt][npar][4] and h_out [nevt] are HOST
 * pointers that must stay valid until the ticket completes.  ME_EINVAL for
 * nevt <= 0; ME_ENOMEM if the request's footprint alone exceeds the budget.
 * *ticket
 * receives an id (monotonic from 1). */
me_status me_server_submit(me_server s, me_handle h, const double* h_momenta, int64_t nevt,
                           double* h_out, int64_t* ticket);

/* Non-blocking: *done = 1 when the ticket finished (status in *result),
 * *latency_s = time from submit to completion seen by the server loop. */
me_status me_server_poll(me_server s, int64_t ticket, int32_t* done, me_status* result,
                         double* latency_s);

/* Block until the ticket finished or timeout_s elapsed (ME_EBUSY then). */
me_status me_server_wait(me_server s, int64_t ticket, double timeout_s, me_status* result,
                         double* latency_s);

/* For a finished ticket: time from submit to admission (slot and arena
 * memory granted, queueing) and from admission to completion (service:
 * staging copies, kernels, copy back).  ME_EBUSY while it runs. */
me_status me_server_times(me_server s, int64_t ticket, double* queue_s, double* service_s);

me_status me_server_stats(me_server s, me_server_stats_t* st);

/* Drain in-flight work, stop the loop and free all resources. */
me_status me_server_destroy(me_server s);

#ifdef __cplusplus
}
#endif
#endif /* ME_H */
