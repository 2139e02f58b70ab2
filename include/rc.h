/*
 * rc.h -- C ABI of the MI355X (gfx950) Doppler and ionospheric correction library
 * (librc.so).  It implements the correction of sampled arbitrary waveforms of
 * Vickers, Mack & Osaretin (arXiv 2508.04951):
 *
 *   - Doppler dilation, Eq (1)-(2): S(alpha t) with alpha = (1 + v_r/c)/(1 - v_r/c),
 *     v_r positive when the target approaches, computed by windowed
 *     Whittaker-Shannon (sinc) resampling, Eq (17), Sec. III-B and App. C;
 *   - ionospheric dispersion, Eq (3), Eq (15) (distortion) and Eq (16) (correction):
 *     y = IDFT( DFT(x) * exp(-/+ i 4 pi K2 / (c f_k)) ), K2 = e^2 E / (8 pi^2 m_e eps0).
 *
 * Conventions shared by every entry point
 *   - Sample buffers are DEVICE pointers (HIP global memory) owned by the caller, holding
 *     interleaved complex64 samples (rc_c64, the layout of torch.complex64).  The library
 *     never frees or keeps them past the call's stream work.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Compute calls
 *     only enqueue work and return; results are ready when the stream reaches them.
 *   - Errors are status codes; no C++ exception crosses the ABI.  RC_ERR_INVALID_ARG is
 *     returned before any work is enqueued; rc_last_error() gives the reason.  A fault in
 *     enqueued work surfaces as RC_ERR_DEVICE from a later call or from rc_sync().
 *   - A context is bound to one HIP device.  Calls on one context are serialised by an
 *     internal mutex, so several host threads may share it.
 *   - Time is in input-sample units: output m samples the input at t = alpha * m, and
 *     x[n] = 0 outside [0, n_in).  The arithmetic is float32 with float64 sample
 *     positions alpha * m, float64 window coefficients and a float64 dispersive phase.
 */
#ifndef RC_H
#define RC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Interleaved complex64, identical to torch.complex64 / std::complex<float>. */
typedef struct {
    float re, im;
} rc_c64;

typedef enum {
    RC_OK = 0,
    RC_ERR_INVALID_ARG = 1,   /* bad pointer, size, parameter or overlap; nothing enqueued */
    RC_ERR_UNSUPPORTED = 2,   /* a valid request the library cannot serve */
    RC_ERR_OUT_OF_MEMORY = 3, /* workspace or table allocation failed */
    RC_ERR_DEVICE = 4,        /* a HIP runtime call or a kernel failed */
    RC_ERR_BUSY = 5           /* reserved for admission control */
} rc_status;

/* Sinc taper (rc_sinc.window). */
enum {
    RC_WIN_KAISER = 0, /* 2H taps n = floor(t)-H+1 .. floor(t)+H, weight sinc(t-n) K((t-n)/H),
                          K(x) = I0(beta sqrt(1-x^2)) / I0(beta) */
    RC_WIN_RECT = 1,   /* the same 2H taps, weight sinc(t-n) */
    RC_WIN_PAPER = 2   /* 2H+1 taps centred on the nearest input sample, no taper
                          (the odd N_window of App. C, Fig. 10) */
};

/* Ionospheric operator direction. */
enum {
    RC_CORRECT = 0, /* Eq (16): phase exp(-i 4 pi K2 / (c f)) removes the two-way delay */
    RC_DISTORT = 1  /* Eq (15): phase exp(+i 4 pi K2 / (c f)) applies it */
};

/* rc_pulse.flags */
enum {
    RC_DO_DOPPLER = 1u, /* resample to S(alpha t) first */
    RC_DO_IONO = 2u     /* then apply the ionospheric operator to the n_out samples */
};

typedef struct rc_context_s *rc_context;

/* Resampling kernel.  half_width H >= 1 selects 2H taps (2H+1 for RC_WIN_PAPER);
 * H = 0 selects the full, unwindowed Whittaker-Shannon sum over every input sample
 * (Eq 17 on the finite record).  kaiser_beta >= 0 is used by RC_WIN_KAISER only. */
typedef struct {
    int32_t half_width;
    int32_t window;
    double kaiser_beta;
} rc_sinc;

/* One pulse of a batch.  Offsets and lengths count complex samples inside the packed
 * input / output buffers passed to correct_pulse_batch.
 *   fs_hz          sample rate (Hz), > 0
 *   alpha          Doppler factor (> 0; use rc_alpha_from_vr); ignored without RC_DO_DOPPLER
 *   tec_el_per_m2  one-way path TEC E in electrons/m^2 (1 TECU = 1e16); >= 0
 *   carrier_hz     RF frequency of baseband 0 Hz (f_k = carrier + fs * fftfreq(n_out)[k])
 *   flags          RC_DO_DOPPLER | RC_DO_IONO; without RC_DO_DOPPLER n_out must equal n_in
 *   direction      RC_CORRECT or RC_DISTORT */
typedef struct {
    int64_t off_in, n_in, off_out, n_out;
    double fs_hz, alpha, tec_el_per_m2, carrier_hz;
    uint32_t flags;
    int32_t direction;
} rc_pulse;

/* Create a context on HIP device `hip_device` (device tables are built here).
 * *out receives the handle.  RC_ERR_INVALID_ARG for a NULL out or a bad device. */
rc_status rc_create(int hip_device, rc_context *out);

/* Synchronise the device, then free every table and workspace of the context. */
rc_status rc_destroy(rc_context ctx);

/* Static, human-readable name of a status code. */
const char *rc_status_string(rc_status status);

/* Text of the last error recorded on ctx ("" if none).  Valid until the next call on ctx. */
const char *rc_last_error(rc_context ctx);

/* Eq (1): alpha = (1 + v_r/c)/(1 - v_r/c) = 1 + 2 v_r / (c - v_r); NaN unless |v_r| < c. */
double rc_alpha_from_vr(double v_r_mps);

/* Eq (3): K2 / E = e^2 / (8 pi^2 m_e eps0) in m^3 s^-2 (CODATA 2022 constants). */
double rc_k2_per_tec(void);

/* Block the host until `stream` has drained; report any device error as RC_ERR_DEVICE. */
rc_status rc_sync(rc_context ctx, void *stream);

/* Doppler resampling, Eq (2) with Eq (17):
 *   y[m] = sum_n x[n] h(alpha m - n),  m = 0 .. n_out-1,
 * h the kernel selected by *k.  An output whose position alpha*m is an exact integer is
 * that input sample (zero past the end).  x: n_in samples, y: n_out samples, both device
 * pointers that must not overlap.  fs_hz (> 0) documents the time base; the result does
 * not depend on it.  alpha must be finite and > 0. */
rc_status correct_doppler(rc_context ctx, const rc_c64 *x, int64_t n_in, rc_c64 *y,
                          int64_t n_out, double fs_hz, double alpha, const rc_sinc *k,
                          void *stream);

/* Ionospheric operator, Eq (15) / Eq (16), on one pulse of n samples:
 *   y = IDFT_n( DFT_n(x) * exp(s i 4 pi K2 / (c f_k)) ),  s = -1 (RC_CORRECT) or +1,
 *   f_k = carrier_hz + fs_hz * fftfreq(n)[k]; bins with f_k == 0 keep their value.
 * DFT unnormalised, IDFT scaled by 1/n, both circular over the n given samples.
 * Any n >= 1: powers of two up to 2^24 run a multi-level FFT, other lengths up to 2^23 the
 * same N-point DFT by Bluestein's chirp convolution at the power of two >= 2n - 1 (its
 * workspace comes from the context); longer pulses give RC_ERR_UNSUPPORTED.  y may equal x
 * (in place) but must not partially overlap it. */
rc_status correct_ionosphere(rc_context ctx, const rc_c64 *x, rc_c64 *y, int64_t n,
                             double fs_hz, double carrier_hz, double tec_el_per_m2,
                             int32_t direction, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): correct_ionosphere with the same arguments, result
 * and kernels, that allocates nothing.  A length that is not a power of two takes its Bluestein
 * workspace (2 M complex values, M the power of two >= 2n - 1) from a static 32 MiB device array
 * of the library, one per GPU, held until the process ends; so such lengths are limited to
 * n <= 2^20 (larger: RC_ERR_UNSUPPORTED).  Powers of two up to 2^24 need no workspace.  Every
 * call on one GPU shares that array, whatever its context or stream: calls that overlap on one
 * GPU (different streams, contexts or threads, not ordered by the caller) race on it and give
 * undefined results.  The context must have been created by rc_create (which looks up the
 * array's device address); no FFT plan is cached and no profiling span is recorded. */
rc_status correct_ionosphere_noalloc(rc_context ctx, const rc_c64 *x, rc_c64 *y, int64_t n,
                                     double fs_hz, double carrier_hz, double tec_el_per_m2,
                                     int32_t direction, void *stream);

/* Pulse compression with the ionospheric operator in the same frequency-domain pass (Sec. II-B
 * bundles Eq (15)/(16) with other FFT work such as pulse compression; Sec. II-D times it).
 * Matched filtering is the circular cross-correlation with a replica r zero-padded to n:
 *   y = IDFT_n( DFT_n(x) * conj(DFT_n(r)) * exp(s i 4 pi K2 / (c f_k)) ),
 *   i.e. y[m] = sum_j xc[(j + m) mod n] conj(r[j]), xc the ionosphere-corrected x,
 * with f_k, s and the scaling as in correct_ionosphere, and the same lengths: powers of two up
 * to 2^24 in the multi-level FFT's row pass, other lengths up to 2^23 by Bluestein's chirp
 * convolution with the correlation folded into its middle step (workspace from the context);
 * longer pulses give RC_ERR_UNSUPPORTED.
 *
 * replica_spectrum writes DFT_n(r) (r: n_rep samples, 1 <= n_rep <= n) to spec, a caller-owned
 * device buffer of n samples, in the library's internal bin order: it is only for
 * compress_pulse at the same n, and one spectrum serves any number of pulses.  replica and
 * spec must not overlap.
 * compress_pulse reads x (n samples) and spec and writes y (n samples); y may equal x (in
 * place) but must not partially overlap it, and must not overlap spec. */
rc_status replica_spectrum(rc_context ctx, const rc_c64 *replica, int64_t n_rep, int64_t n,
                           rc_c64 *spec, void *stream);
rc_status compress_pulse(rc_context ctx, const rc_c64 *x, rc_c64 *y, int64_t n, const rc_c64 *spec,
                         double fs_hz, double carrier_hz, double tec_el_per_m2, int32_t direction,
                         void *stream);

/* A batch of pulses with their own alpha, TEC, carrier and lengths, in packed buffers:
 * pulse i reads x_packed[off_in .. off_in+n_in) and writes y_packed[off_out .. off_out+n_out),
 * Doppler first, then the ionosphere on the resampled samples (the order matters: the
 * two operators do not commute).  `pulses` is a HOST array of `count` descriptors, read
 * during the call only.  x_len / y_len are the buffer lengths in samples; every range must
 * lie inside its buffer, output ranges must not overlap each other, and the two buffers
 * must not overlap.  Every pulse uses the kernel *k.  The result of each pulse does not
 * depend on the other pulses of the batch. */
rc_status correct_pulse_batch(rc_context ctx, const rc_c64 *x_packed, int64_t x_len,
                              rc_c64 *y_packed, int64_t y_len, const rc_pulse *pulses,
                              int32_t count, const rc_sinc *k, void *stream);

/* Batch plans: one correct_pulse_batch call captured once in a HIP graph and replayed.  For a
 * caller that runs the same batch shape again and again (a pulse train, a fixed bank of channels):
 * the host work of a call (validation, grouping, descriptor upload, the matrix-core tile list) is
 * done at creation, and a launch is one hipGraphLaunch of the recorded kernels.
 *
 * rc_batch_plan_create takes correct_pulse_batch's arguments (count >= 1) and fixes them; the plan
 * owns device memory for the descriptors and workspace (not counted against rc_set_mem_budget).
 * rc_batch_plan_launch(plan, stream) then enqueues exactly the work of that correct_pulse_batch
 * call on `stream`, with bit-identical results.  rc_batch_plan_update(plan, pulses, count, stream)
 * replaces the pulses (same buffers) for later launches; it enqueues the new descriptors and tile
 * list on `stream`, so a launch on that stream after it sees them and one before it does not.
 * The new pulses must need the same launches: the same count, lengths and flags, the same
 * resampling engine per pulse (alpha within the same eligibility range), and pulses with neither
 * step at the same offsets; otherwise RC_ERR_UNSUPPORTED and the plan is unchanged.
 * rc_batch_plan_destroy synchronises the device and frees the plan; destroy every plan before its
 * context.  Launches of one plan share its buffers: launches on different streams that overlap
 * in time race on the outputs as two correct_pulse_batch calls would. */
typedef struct rc_batch_plan_s *rc_batch_plan;
rc_status rc_batch_plan_create(rc_context ctx, const rc_c64 *x_packed, int64_t x_len,
                               rc_c64 *y_packed, int64_t y_len, const rc_pulse *pulses,
                               int32_t count, const rc_sinc *k, rc_batch_plan *out);
rc_status rc_batch_plan_launch(rc_batch_plan plan, void *stream);
rc_status rc_batch_plan_update(rc_batch_plan plan, const rc_pulse *pulses, int32_t count,
                               void *stream);
rc_status rc_batch_plan_destroy(rc_batch_plan plan);

/* A bank of Doppler hypotheses on one pulse (many alpha on the same input):
 *   y[h * n_out + m] = sum_n x[n] h(alphas[h] m - n),  h < n_hyp, m < n_out,
 * each row the correct_doppler result for its alpha (the same Eq (17) sum; the exact-integer
 * rule is kept).  x: n device samples; y: n_hyp * n_out device samples, must not overlap x;
 * alphas: HOST array of n_hyp values, finite and > 0, read during the call only.
 *
 * The filter bank: each tap weight h(mu - j) is a degree-7 polynomial in the fractional position
 * mu, so the 2H-tap FIR of each of its 8 coefficients runs once per input position (a dense
 * contraction on the matrix cores) and every (hypothesis, output) then costs an 8-term sum.  It
 * needs a Kaiser or rectangular window, 1 <= H <= 256 and every alpha in (0, 2]; elsewhere the bank
 * runs every hypothesis as a pulse of correct_pulse_batch (see rc_set_bank_engine).
 *
 * precision selects the arithmetic of the filter bank's contraction (float32 accumulation in all
 * three; the per-output sums are float32):
 *   RC_BANK_FP16X3  samples and coefficients split into float16 hi + lo after power-of-two scaling,
 *                   hi*hi + hi*lo + lo*hi (+ lo*lo) products: ~3e-7 rel-L2 against the float64
 *                   direct sum at H = 64 and 128 (the default, and the fastest);
 *   RC_BANK_BF16X3  the same split in bfloat16 (float32's exponent range, 8-bit significands):
 *                   ~4e-6 rel-L2;
 *   RC_BANK_FP32    float32 products on the float32 matrix cores: ~3e-7 rel-L2.
 * The per-hypothesis engine ignores precision (float32-accurate resampling engines).
 * Every mode stays within 1e-5 rel-L2 of the float64 direct sum.  The filter bank's workspace
 * (8 complex values per input position) comes from the context.  This extends the paper (one
 * alpha per pulse) to the hypothesis search of a Doppler-ambiguous return; the operator per row
 * is Eq (2) with Eq (17). */
enum { RC_BANK_FP16X3 = 0, RC_BANK_BF16X3 = 1, RC_BANK_FP32 = 2 };
rc_status correct_doppler_bank(rc_context ctx, const rc_c64 *x, int64_t n, rc_c64 *y,
                               int64_t n_out, double fs_hz, const double *alphas, int32_t n_hyp,
                               const rc_sinc *k, int32_t precision, void *stream);

/* Engine of the context's later correct_doppler_bank calls:
 *   RC_BANK_ENGINE_AUTO            the filter bank where it applies, else per hypothesis (default);
 *   RC_BANK_ENGINE_FARROW          always the filter bank: RC_ERR_UNSUPPORTED where it does not apply;
 *   RC_BANK_ENGINE_PER_HYPOTHESIS  every hypothesis as a pulse of correct_pulse_batch.
 * RC_ERR_INVALID_ARG for an unknown engine. */
enum { RC_BANK_ENGINE_AUTO = 0, RC_BANK_ENGINE_FARROW = 1, RC_BANK_ENGINE_PER_HYPOTHESIS = 2 };
rc_status rc_set_bank_engine(rc_context ctx, int32_t engine);

/* Serving: a continuous-batching server over independent requests (the paper corrects one
 * pulse at a time; a radar front end sees a stream of them).  Each request is one pulse,
 * Doppler first and then the ionosphere as in correct_pulse_batch, on caller-owned device
 * buffers that must stay valid (and y untouched) until the request completes.  A launcher
 * thread takes everything queued (up to max_batch requests) as one batch on the server's own
 * stream whenever fewer than two earlier batches are still running on the device: a request
 * that arrives at an idle server starts at once, and under load the queue fills while the
 * device works, so one launch sequence serves many requests (ionospheric lengths that are not
 * powers of two share theirs by convolution length).  A completer thread times each batch's
 * completion.  Admission is by bytes: a request holds, until it completes,
 * 8 (n_in + n_out) + 1024 bytes, plus the Bluestein workspace of an ionospheric length that is
 * not a power of two (2 M complex values, M the power of two >= 2 n_out - 1), plus, for a
 * Doppler pulse on the matrix cores, its tile list (17 bytes per 2048 outputs and 516 bytes per
 * 256 tiles).  Those bound the context workspace of every batch in flight: with the context's
 * rc_set_mem_budget at the server's budget the workspace never exceeds it.
 * rc_server_submit returns RC_ERR_BUSY when the budget is full and
 * RC_ERR_UNSUPPORTED for a request that could never fit.  Every pulse uses the kernel *k
 * given at creation.  Output of a request does not depend on what it was batched with. */
typedef struct rc_server_s *rc_server;
typedef struct {
    const rc_c64 *x;        /* device input, n_in samples */
    rc_c64 *y;              /* device output, n_out samples (may equal x without RC_DO_DOPPLER) */
    int64_t n_in, n_out;
    double fs_hz, alpha, tec_el_per_m2, carrier_hz;
    uint32_t flags;         /* RC_DO_DOPPLER | RC_DO_IONO */
    int32_t direction;      /* RC_CORRECT | RC_DISTORT */
    void *stream;           /* hipStream_t: the work enqueued on it before rc_server_submit (such
                               as what fills x) completes before the request reads x; NULL is the
                               null stream */
} rc_request;
typedef struct {
    int64_t submitted, completed, rejected;   /* since creation or the last reset */
    int64_t batches;                          /* launches */
    double mean_batch;                        /* requests per launch */
    double latency_ms_p50, latency_ms_p99, latency_ms_max;  /* submit -> completion observed */
    double samples_per_s;   /* completed output samples / (last completion - first submission) */
} rc_server_stats_t;
rc_status rc_server_create(rc_context ctx, const rc_sinc *k, int64_t mem_budget_bytes,
                           int32_t max_batch, rc_server *out);
rc_status rc_server_submit(rc_server srv, const rc_request *req, int64_t *ticket);
/* The bytes rc_server_submit would charge this request against the budget (see above), or -1
 * for a NULL argument.  The request is not validated. */
int64_t rc_server_request_bytes(rc_server srv, const rc_request *req);
/* done = 1 once the request is complete; a completed ticket is then released (poll again:
 * RC_ERR_INVALID_ARG).  Returns the request's status when it reports done. */
rc_status rc_server_poll(rc_server srv, int64_t ticket, int32_t *done);
/* Block until the ticket (0: every request submitted so far) is complete, then release it. */
rc_status rc_server_wait(rc_server srv, int64_t ticket);
rc_status rc_server_stats(rc_server srv, rc_server_stats_t *out);
rc_status rc_server_reset_stats(rc_server srv);
/* Launch what is queued, wait for everything, free the server. */
rc_status rc_server_destroy(rc_server srv);

/* Tuning.  These set launch shapes that change speed: the grid and chunk settings give
 * bit-identical results; another FFT split changes the float32 rounding order only (results
 * within the same parity bar against the float64 definition).
 *   rc_set_fft_levels     the split of the n-point transform (n a power of two, 4096 < n <= 2^24)
 *                         into `count` (1..3) strided levels, each a power of two in [2, 256], run
 *                         before the 4096-point contiguous level; their product times 4096 is n.
 *                         count 0 restores the default split (levels of 256, then the rest);
 *   rc_set_sinc_grid      workgroups per CU of the matrix-core resampler's persistent grid at
 *                         half_width 64 or 128 (0: as many as fit, the default);
 *   rc_set_bluestein_chunk  workspace cap of one Bluestein launch sequence in a batch (0: 256 MiB).
 * rc_load_tuning applies a JSON file written by the autotuner (paper_2508_04951_amd/tune.py):
 *   {"fft_levels": {"<n>": [L0, ...], ...}, "sinc_grid": {"64": w, "128": w},
 *    "bluestein_chunk_bytes": b, ...}   (other keys are ignored).
 * rc_create loads the file named by the environment variable RC_TUNE_FILE when it is set and
 * fails with RC_ERR_INVALID_ARG if that file cannot be read or applied.  All three settings
 * are per context and apply to later calls. */
rc_status rc_set_fft_levels(rc_context ctx, int64_t n, const int32_t *levels, int32_t count);
rc_status rc_set_sinc_grid(rc_context ctx, int32_t half_width, int32_t wg_per_cu);
rc_status rc_set_bluestein_chunk(rc_context ctx, int64_t bytes);
rc_status rc_load_tuning(rc_context ctx, const char *path);

/* Resampling engine (rc_set_sinc_engine).  Every engine computes the same sum of Eq (17):
 *   RC_SINC_AUTO   matrix cores for the Kaiser taper at H = 64 or 128 and |alpha - 1| <= 6e-5,
 *                  else the vector tile kernel (Kaiser, H <= 256, |alpha - 1| <= 1e-4), else the
 *                  direct sum (float64 positions, float32 tap weights and accumulation);
 *   RC_SINC_VALU   never the matrix cores;
 *   RC_SINC_DIRECT always the direct sum (reference-speed path). */
enum { RC_SINC_AUTO = 0, RC_SINC_VALU = 1, RC_SINC_DIRECT = 2 };

/* Select the resampling engine of the context's later calls; RC_ERR_INVALID_ARG for an
 * unknown engine.  The default is RC_SINC_AUTO. */
rc_status rc_set_sinc_engine(rc_context ctx, int32_t engine);

/* Cap the context's device workspace at `bytes` (0: no cap, the default).  The workspace is
 * the scratch the calls stage lazily and keep for reuse: descriptor tables, the matrix-core
 * tile lists, Bluestein's convolution buffers and the filter bank's Z rows.  Twiddle tables,
 * FFT plans and kernel tables are not counted.  A call whose workspace would grow past the cap
 * fails with RC_ERR_OUT_OF_MEMORY; workspace already held is kept (a lower cap only stops
 * further growth).  bytes < 0 gives RC_ERR_INVALID_ARG. */
rc_status rc_set_mem_budget(rc_context ctx, int64_t bytes);

/* Kernel timing for benchmarks.  While enabled, every kernel the context launches is
 * bracketed by a pair of HIP events recorded on the launch stream.  rc_profile_read waits for
 * the recorded events, adds their spans to per-kernel totals, and returns (then clears) the
 * total milliseconds and launch count of one kernel: "k_sinc_mfma", "k_sinc_fast",
 * "k_sinc_direct", "k_fft_strided_fwd", "k_fft_rows_iono", "k_fft_strided_inv" or
 * "k_mf_tile_list" (the three small kernels that sort a batch's matrix-core tiles by phase,
 * timed together as one launch), "k_bluestein" (the pointwise chirp kernels of lengths that are
 * not powers of two), "k_farrow_z" or "k_farrow_bank".  Unknown names give
 * RC_ERR_INVALID_ARG.  Timing adds two event records per launch and no synchronisation. */
rc_status rc_profile_enable(rc_context ctx, int enable);
rc_status rc_profile_read(rc_context ctx, const char *kernel, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------------------------------
 * The paper's other Doppler resampling methods, as baselines beside correct_doppler.
 * Same conventions: device pointers, asynchronous on `stream`, x and y must not overlap
 * (except correct_doppler_tone, which may work in place), alpha finite and > 0, fs_hz > 0.
 * ------------------------------------------------------------------------------------- */

/* Variants of the paper's own GPU sinc kernel (App. C). */
enum {
    RC_PAPER_DIRECT = 0, /* Alg. 1: one thread per output, sinc computed per tap */
    RC_PAPER_TILED = 1,  /* Alg. 3: each block stages its inputs in LDS first ("tiling") */
    RC_PAPER_LUT = 2     /* Alg. 2: sinc from an LDS table of its positive half */
};

/* The paper's windowed Whittaker-Shannon kernel (App. C, Fig. 10): output m sums the
 * n_window (odd, >= 1) inputs centred on the nearest input c = floor(alpha m + 1/2),
 * y[m] = sum_{|n - c| <= (n_window-1)/2} x[n] sinc(alpha m - n), untapered, in the structure
 * of the paper's kernels: a grid-stride loop over outputs with `blocks` blocks of 256 threads
 * (0: one output per thread; the paper's H100 runs used 32).  RC_PAPER_DIRECT and
 * RC_PAPER_TILED compute the same sum (bit-identical) and equal correct_doppler with
 * RC_WIN_PAPER to float32 rounding.  RC_PAPER_LUT takes sinc from a table of lut_size
 * (2 .. 16384) values sinc(i dx), i = 0 .. lut_size-1, dx = (h + 1/2) / (lut_size - 1),
 * h = (n_window-1)/2: a tap at distance u = |alpha m - n| takes entry floor(u / dx + 1/2)
 * (the nearest); lut_size = 100 (h + 1/2) + 1 gives the dx = 1/100 of Sec. III-A, Fig. 5.
 * RC_PAPER_TILED needs (ceil(255 alpha) + n_window + 2) * 8 bytes of LDS, at most 64 KiB
 * (RC_ERR_UNSUPPORTED above). */
rc_status correct_doppler_paper(rc_context ctx, const rc_c64 *x, int64_t n_in, rc_c64 *y,
                                int64_t n_out, double fs_hz, double alpha, int32_t n_window,
                                int32_t variant, int32_t lut_size, int32_t blocks, void *stream);

/* Linear interpolation (Sec. I, Table I): y[m] = (1 - mu) x[f] + mu x[f + 1] at
 * t = alpha m, f = floor(t), mu = t - f; x = 0 outside [0, n_in). */
rc_status correct_doppler_linear(rc_context ctx, const rc_c64 *x, int64_t n_in, rc_c64 *y,
                                 int64_t n_out, double fs_hz, double alpha, void *stream);

/* Frequency conversion (Sec. I, Table I): the dilation replaced by the frequency shift it
 * causes at one reference frequency f_ref_hz (on the samples' own frequency axis):
 * y[m] = x[m] exp(2 pi i (alpha - 1) f_ref_hz m / fs_hz).  Exact for a tone at f_ref_hz only.
 * y may equal x. */
rc_status correct_doppler_tone(rc_context ctx, const rc_c64 *x, rc_c64 *y, int64_t n,
                               double fs_hz, double alpha, double f_ref_hz, void *stream);

/* Length of the FFT P/Q resampled record for a dilation alpha (Sec. III-A): the n_in / alpha
 * samples the dilated record spans, rounded so that an even number of samples is removed or
 * added: n_in - 2 round((n_in - n_in / alpha) / 2) (halves away from zero).  0 if alpha is not
 * finite and > 0 or n_in < 1. */
int64_t rc_pq_length(int64_t n_in, double alpha);

/* Doppler correction by FFT P/Q resampling (Sec. I, Sec. III-A): the DFT of x has bins removed
 * or zero bins added to reach n_i = rc_pq_length(n_in, alpha) bins, then the inverse DFT:
 *   y[m] = (1/n_in) sum_j Y_j exp(2 pi i j m / n_i),  m < min(n_i, n_out),  0 beyond,
 * the trigonometric interpolant of x at t = m n_in / n_i (exact dilation by n_in / n_i).
 * With K = min(n_in, n_i), signed bins |k| <= (K-1)/2 are copied; for even K the bin K/2 is
 * the sum of input bins +K/2 and -K/2 when removing, and half the input Nyquist bin at +K/2
 * and at -K/2 when adding.  With with_tone != 0 the remaining dilation alpha / alpha_eff
 * (alpha_eff = n_in / n_i) follows as frequency conversion at alpha_eff f_ref_hz ("P/Q with
 * frequency conversion").  n_i == n_in transforms nothing.  2 <= n_in, n_i <= 2^23; the
 * transforms run Bluestein's chirp convolution (workspace from the context). */
rc_status correct_doppler_fft_pq(rc_context ctx, const rc_c64 *x, int64_t n_in, rc_c64 *y,
                                 int64_t n_out, double fs_hz, double alpha, double f_ref_hz,
                                 int32_t with_tone, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RC_H */
