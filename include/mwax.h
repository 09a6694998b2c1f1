/*
 * mwax.h -- C ABI of the MI355X FX correlation hot path.
 *
 * Implements, for one GPU, the per-coarse-channel FX engine of Morrison et al.,
 * "MWAX: A New Correlator for the Murchison Widefield Array" (PASA 2023):
 *   - fine channelisation by FFT of complex int8 voltage streams (Sec. 2.5,
 *     Sec. 2.5.1), channels centre-symmetric with DC at c = L/2 (Sec. 2.6);
 *   - the transpose to channel-major order ahead of the X-engine (Sec. 2.5.1);
 *   - the X-engine: for every channel c and input pair n1 >= n2, autos
 *     included, V[c][n1,n2] += sum_m X_n1[m,c] conj(X_n2[m,c]) (Sec. 2.5.2);
 *   - time integration and output of the packed lower triangle
 *     (Sec. 2.5.2, Sec. 2.7).
 *
 * Conventions used throughout:
 *   inputs      n = 2*tile + pol (pol 0 = X, 1 = Y): the [tile][polarisation]
 *               order of Sec. 2.5.1.  n_inputs = 2 * n_tiles.
 *   FFT         unnormalised forward transform over contiguous, non-overlapping
 *               frames of L samples, rectangular window.
 *   channels    c = (k + L/2) mod L for FFT bin k; channel c is centred at
 *               (c - L/2) * coarse_bw / L from the coarse-channel centre.
 *   visibility  sums (not means) over the spectra of an integration.
 *   pair index  p(n1, n2) = n1 (n1 + 1) / 2 + n2 for n1 >= n2; P = n(n+1)/2.
 *
 * Memory: every pointer named d_* is device memory on the plan's device; h_*
 * is host memory.  The caller owns all buffers it passes; the plan owns its
 * workspace (allocated by mwax_plan_create, released by mwax_plan_destroy).
 *
 * Asynchrony: calls enqueue work on the plan's stream and return.  Argument
 * and call-order errors return at once and enqueue nothing.  Runtime errors
 * seen at launch return MWAX_E_DEVICE; faults raised while kernels run are
 * reported by the HIP runtime at the next synchronisation (mwax_sync).
 *
 * Threading: a plan must not be used from two threads at once.  Distinct plans
 * are independent.  No C++ exception crosses this interface.
 */
#ifndef MWAX_H
#define MWAX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mwax_plan_s *mwax_plan;

typedef enum {
    MWAX_OK = 0,
    MWAX_E_INVAL = 1,       /* bad argument or configuration; nothing enqueued       */
    MWAX_E_NOMEM = 2,       /* device allocation failed                               */
    MWAX_E_DEVICE = 3,      /* HIP runtime error                                      */
    MWAX_E_STATE = 4,       /* call out of order (see each call)                      */
    MWAX_E_UNSUPPORTED = 5  /* a valid request this library does not implement        */
} mwax_status;

/* Arithmetic of the X-engine (precision forms beyond the paper's FP32,
 * Sec. 2.5.1 and 2.5.2 use single precision throughout):
 *   FP32: spectra kept in FP32, X-engine on the vector ALUs in FP32, partial
 *         sums flushed to FP64 integrators every 2048 spectra.
 *   FP16: spectra scaled by 2^-e, e = ceil(log2(L)/2), rounded to binary16
 *         (ties to even); X-engine on FP16 matrix cores with FP32 accumulation,
 *         flushed to FP64 integrators; output scaled back by 2^(2e).
 *   INT8: spectra requantised per channel to q = clamp(rne(X * inv_s_c), -127,
 *         127); X-engine on int8 matrix cores with int32 accumulation flushed to
 *         integer integrators, exact: int32 pairs when an integration holds at
 *         most 65536 spectra, int64 pairs otherwise (the raw output is int64
 *         either way); output V = V_int * s_c^2. */
typedef enum { MWAX_X_FP32 = 0, MWAX_X_FP16 = 1, MWAX_X_INT8 = 2 } mwax_xprec;

/* Output orders of mwax_integrate:
 *   CHAN_TRI: [integration][channel][P] complex64, packed lower triangle.
 *   TILE_BL : [integration][baseline][channel][4] complex64, baselines a >= b
 *             at a(a+1)/2 + b, products XX, XY, YX, YY (pol of tile a first);
 *             the auto-tile XY is conj(YX).  Sec. 2.7 orders its output by
 *             baseline, channel and polarisation; its exact figure is not in
 *             the text, so this layout is not claimed to match it bit for bit. */
typedef enum { MWAX_ORDER_CHAN_TRI = 0, MWAX_ORDER_TILE_BL = 1 } mwax_order;

/* Plan configuration, following the paper's statement of the problem:
 * N tiles x 2 polarisations (Sec. 2.5), 1.28 MHz coarse channels sampled at
 * 1.28 Msps complex (Sec. 2.1, Sec. 2.5), a chosen fine-channel width and
 * integration time (Table 1, Sec. 2.5.2). */
typedef struct {
    int32_t n_tiles;       /* 1 .. 1024                                                   */
    int32_t n_pols;        /* must be 2                                                   */
    double coarse_bw_hz;   /* complex sample rate == coarse bandwidth (1.28e6 for MWA)     */
    double fine_chan_hz;   /* L = coarse_bw / fine_chan: a whole number; this library
                              implements powers of two 1 .. 1024 (others: UNSUPPORTED)  */
    double int_time_s;     /* T = int_time * coarse_bw / L must be an integer >= 1         */
    int32_t xprec;         /* mwax_xprec                                                  */
    int32_t reserved;      /* must be 0                                                   */
    int64_t max_samples;   /* largest n_samples of one channelise call; multiple of L     */
    uint64_t flags;        /* must be 0                                                   */
} mwax_config;

/* Quantities derived from a configuration (host arithmetic only). */
typedef struct {
    int32_t n_inputs;          /* 2 * n_tiles                                          */
    int32_t fft_len;           /* L                                                    */
    int64_t spectra_per_int;   /* T                                                    */
    int64_t n_pairs;           /* P = n_inputs (n_inputs + 1) / 2                      */
    int64_t n_baselines;       /* n_tiles (n_tiles + 1) / 2                            */
    int64_t max_spectra;       /* max_samples / L                                      */
    int32_t n_slots;           /* integrations the plan can hold on the device         */
    int32_t group;             /* spectra per 32-byte row of the channel-major layout  */
    int64_t vis_per_int;       /* L * P complex values per integration (CHAN_TRI)      */
    int64_t cal_spectra;       /* spectra used to calibrate an integration's scales    */
    uint64_t workspace_bytes;  /* device bytes a plan allocates                        */
    double sample_time_s;      /* 1 / coarse_bw                                        */
    double fine_chan_hz;       /* coarse_bw / L                                        */
    double int_time_s;         /* T * L / coarse_bw                                    */
} mwax_dims;

/* Validate a configuration and derive its dimensions.  Host only: touches no
 * GPU, so it can be called anywhere.  MWAX_E_INVAL with a message for any rule
 * the configuration breaks (see mwax_config); MWAX_E_UNSUPPORTED for a whole
 * FFT length that is not a power of two in 1..1024 (e.g. the 6,400-point
 * transform of Sec. 2.5.1). */
mwax_status mwax_plan_derive(const mwax_config *cfg, mwax_dims *out);

/* Create a plan on the current HIP device.  hip_stream is a hipStream_t (NULL
 * for the default stream) on which every later call of the plan enqueues.
 * Allocates the workspace (channel-major buffer for max_samples, integrators,
 * scales, twiddles) and generates the FFT twiddles on the device in FP64.
 * Errors: MWAX_E_INVAL (configuration), MWAX_E_NOMEM, MWAX_E_DEVICE. */
mwax_status mwax_plan_create(const mwax_config *cfg, void *hip_stream, mwax_plan *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): like
 * mwax_plan_create, but the plan's workspace is carved out of a static device
 * array of the library (64 MiB per device, held from library load until the
 * process ends) instead of being allocated; no device allocation routine is
 * called.  Every later call on the plan behaves as for mwax_plan_create.  At
 * most one such plan exists per device at a time (they would share the
 * array): MWAX_E_STATE while another lives; mwax_plan_destroy releases it.
 * The workspace is initialised here (integrators cleared, scales 1), so it
 * keeps nothing of the previous plan.  Errors: MWAX_E_INVAL for a
 * configuration, or a workspace (mwax_dims.workspace_bytes, each buffer
 * rounded up to 256 bytes) larger than 64 MiB; MWAX_E_DEVICE. */
mwax_status mwax_plan_create_noalloc(const mwax_config *cfg, void *hip_stream, mwax_plan *out);

/* Release the plan and its workspace (waits for its stream first).  NULL is
 * accepted and ignored. */
mwax_status mwax_plan_destroy(mwax_plan p);

/* The plan's dimensions (see mwax_dims). */
mwax_status mwax_plan_get_dims(mwax_plan p, mwax_dims *out);

/* F-engine (Sec. 2.5.1): channelise n_samples samples of every input.
 *   d_volts   : int8 [n_inputs][ld_samples][2] (re, im) complex samples; must be
 *               16-byte aligned, ld_samples a multiple of 8 and >= n_samples.
 *   n_samples : > 0, a multiple of L, <= max_samples.
 * The samples continue the stream of earlier calls: integration boundaries
 * fall every T spectra of the concatenated stream.  Transforms every frame,
 * requantises (INT8: with the scales of the integration each spectrum belongs
 * to; FP16: to binary16) and writes the channel-major buffer.  For INT8 plans
 * in automatic-scale mode, each integration that begins in this call first
 * has its per-channel scales calibrated from its first cal_spectra spectra
 * (or as many as this call holds): sigma_c^2 = sum of (re^2 + im^2) / (2 F)
 * over the F populated frames (frame m of input n is populated if any of its
 * L samples is nonzero: the capture stage of Sec. 2.4 zeroes lost packets, and
 * such frames are left out), s_c = 5 sigma_c / 127, inv_s_c = 127 / (5
 * sigma_c); a channel with zero power gets s_c = 1.  A window with no
 * populated frame keeps the scales of the plan's most recent calibrated
 * integration (1 if there is none; mwax_reset forgets them).
 * Errors: MWAX_E_INVAL (arguments); MWAX_E_STATE if the previous channelised
 * block has not been correlated, or if an integration this call would start
 * needs a device slot still held by a completed integration that
 * mwax_integrate has not emitted. */
mwax_status mwax_channelise(mwax_plan p, const int8_t *d_volts, int64_t n_samples,
                            int64_t ld_samples);

/* Load already channelised data in place of mwax_channelise, in the X-engine
 * input order of Sec. 2.5.1, [time][channel][tile][pol]:
 *   d_chan: [n_spectra][L][n_inputs][2] of the plan's element type: int8
 *           (values in -127..127; -128 is clamped to -127), binary16 bits
 *           (uint16), or float32.  INT8 plans apply their fixed scales (see
 *           mwax_set_scales) or 1.0 at output; FP16 values are taken as
 *           spectra times 2^-e like those mwax_channelise stores.
 * Same stream position and state rules as mwax_channelise. */
mwax_status mwax_load_channelised(mwax_plan p, const void *d_chan, int64_t n_spectra);

/* Copy out the channelised block last produced by mwax_channelise or
 * mwax_load_channelised, in the [time][channel][input][2] order above and the
 * plan's element type, spectra in stream order.  Needs d_out to hold
 * n_spectra * L * n_inputs * 2 elements with n_spectra <= max_spectra;
 * writes the count to *n_spectra.  MWAX_E_STATE if nothing was channelised. */
mwax_status mwax_read_channelised(mwax_plan p, void *d_out, int64_t max_spectra,
                                  int64_t *n_spectra);

/* Tied-array beamforming (Sec. 4.4) from the last channelised block (the
 * voltages the X-engine correlates: INT8 codes times the channel's scale s_c,
 * binary16 values times 2^e, or FP32 spectra), before or after mwax_correlate.
 *
 * mwax_beamform: coherent beams
 *   out[m][c][b] = sum_n w[c][b][n] X_n[m, c]
 * d_weights [L][n_beams][n_inputs] complex64 (e.g. the phase factors that
 * align every signal path for beam b's pointing, zeros for the paths a beam
 * leaves out); d_out [n_spectra][L][n_beams] complex64 with n_spectra =
 * the block's spectra (<= max_spectra), written to *n_spectra.  Sums on the
 * FP32 matrix cores.
 *
 * mwax_beamform_incoherent: the incoherent beam, detected power summed over
 * the inputs of each polarisation (input n = 2 tile + p), t_avg consecutive
 * spectra and f_avg consecutive channels:
 *   out[j][o][p] = sum_{m in j, c in o, n mod 2 = p} |X_n[m, c]|^2
 * d_out [n_spectra / t_avg][L / f_avg][2] float32 (FP64 sums), needing
 * max_bins >= (n_spectra / t_avg) (L / f_avg); *n_time_bins receives
 * n_spectra / t_avg.  t_avg must divide the block's spectra and f_avg divide L.
 *
 * Both: device pointers, 8-byte (weights, beams) / 4-byte (power) aligned,
 * caller-owned; enqueued on the plan's stream.  MWAX_E_STATE if nothing has
 * been channelised, MWAX_E_INVAL for bad arguments or too small an output. */
mwax_status mwax_beamform(mwax_plan p, const void *d_weights, int32_t n_beams, void *d_out, int64_t max_spectra,
                          int64_t *n_spectra);
mwax_status mwax_beamform_incoherent(mwax_plan p, int32_t t_avg, int32_t f_avg, float *d_out, int64_t max_bins,
                                     int64_t *n_time_bins);

/* X-engine (Sec. 2.5.2): accumulate the last channelised block into the
 * device integrators.  MWAX_E_STATE if there is no fresh channelised block. */
mwax_status mwax_correlate(mwax_plan p);

/* Emit up to max_ints completed integrations, oldest first, into d_vis
 * (complex64 in the given mwax_order; CHAN_TRI needs max_ints * L * P values,
 * TILE_BL max_ints * n_baselines * L * 4) and free their device slots (the
 * integrators are cleared, except in plans of a batch or stream whose next
 * X-engine work overwrites a slot anyway).  *n_emitted receives the count (0
 * if none is complete).  Integrations still in progress are kept. */
mwax_status mwax_integrate(mwax_plan p, void *d_vis, int32_t max_ints, int32_t *n_emitted,
                           int32_t order);

/* Like mwax_integrate in CHAN_TRI order, with the channel averaging of Sec. 2.6
 * (the rule of mwax_fscrunch: centre-symmetric output channels of F fine
 * channels, half-weight shared boundaries for even F, DC left out of the centre
 * channel) done in the same pass over the integrators: d_vis receives
 * [max_ints][L / fscrunch][P] complex64, means of the scaled sums in FP64
 * rounded once.  d_weights, if not NULL, is [max_ints][P] float32 occupancy
 * weights (mwax_vis_weights) of the emitted integrations, dividing each pair's
 * means where positive.  For L = 6400 this is the paper's output path: the
 * 6,400-channel visibilities are never written.  MWAX_E_INVAL if fscrunch does
 * not divide L. */
mwax_status mwax_integrate_averaged(mwax_plan p, int32_t fscrunch, const float *d_weights, void *d_vis,
                                    int32_t max_ints, int32_t *n_emitted);

/* Averaging inside the X-engine (Sec. 2.6 folded into Sec. 2.5.2): from the
 * next block on, the plan correlates its fine channels straight into
 * N = L / fscrunch output channels by the averaging rule of mwax_fscrunch
 * (offsets |d| <= fscrunch / 2 around each output channel's centre, the
 * outermost pair at weight 1/2 for even fscrunch, DC left out of the centre
 * channel; weighted means), so the fine-channel visibilities are never formed
 * (at L = 6400 and 250 ms integrations, 6.7 GB of integrator traffic per
 * integration is avoided).  mwax_integrate then emits N channels
 * ([max_ints][N][P] complex64, or the tile-baseline order over N channels);
 * mwax_integrate_raw_i64 and mwax_integrate_averaged are refused
 * (MWAX_E_STATE).  Arithmetic: each fine channel's partial sums over a
 * segment (INT8: the exact integer sums times s_c^2) are weighted and summed
 * in FP32, then accumulated across segments in FP64 integrators.  INT8 and
 * FP16 plans only (MWAX_E_UNSUPPORTED for FP32 plans and for batch or stream
 * instances); fscrunch must divide L (1 turns it off); allowed before the
 * first block and after mwax_reset only (MWAX_E_STATE), and kept by
 * mwax_reset. */
mwax_status mwax_set_averaging(mwax_plan p, int32_t fscrunch);

/* INT8 plans only: like mwax_integrate in CHAN_TRI order but emits the exact
 * int64 sums, d_vis = [max_ints][L][P][2] int64 (re, im), and, if d_scales is
 * not NULL, the per-channel scales s_c used, [max_ints][L] float32.
 * MWAX_E_UNSUPPORTED for other precisions. */
mwax_status mwax_integrate_raw_i64(mwax_plan p, int64_t *d_vis, float *d_scales,
                                   int32_t max_ints, int32_t *n_emitted);

/* INT8 plans: fix the per-channel scales s_c (h_scales: [L] host floats > 0)
 * for every integration that starts after this call; inv_s_c = 1/s_c in FP32.
 * mwax_auto_scales returns to per-integration calibration.  Both return
 * MWAX_E_STATE while an integration is partly accumulated and
 * MWAX_E_UNSUPPORTED for other precisions. */
mwax_status mwax_set_scales(mwax_plan p, const float *h_scales);
mwax_status mwax_auto_scales(mwax_plan p);

/* INT8 plans: copy the per-channel scales s_c (Sec. 2.5.1 keeps one data path
 * per fine channel; the requantiser gives each channel its own scale) of the
 * most recently begun integration into d_scales ([L] float32, device, 4-byte
 * aligned), enqueued on the plan's stream after that integration's
 * calibration.  MWAX_E_STATE if no integration has begun since the plan was
 * created or reset, MWAX_E_UNSUPPORTED for other precisions, MWAX_E_INVAL for
 * a null or misaligned pointer. */
mwax_status mwax_get_scales(mwax_plan p, float *d_scales);

/* Fractional delay and phase correction (Sec. 2.5.1, delay paragraph; Sec.
 * 4.3).  The capture stage shifts each signal path by whole samples; the
 * residual fractional delays, updated every step (5 ms in the paper), are
 * applied to the frequency-domain samples before they are requantised: every
 * sample of channel c of signal path n in a frame of step s is multiplied by
 *   exp(-2 pi i ((c - L/2) / L + sky_freq_hz / coarse_bw) d[n][s]),
 * a phase gradient across the channels (slope set by the delay alone) times a
 * phase offset set by the coarse channel's sky frequency (the delay theorem:
 * delaying by d samples multiplies the spectrum at sky frequency nu by
 * exp(-2 pi i nu d / coarse_bw)).  The phase offset is reduced in FP64, the
 * gains evaluated in FP32.
 *   d_delays     : [n_inputs][n_steps] float32, device, delays to apply in
 *                  samples (caller-owned; read by every later mwax_channelise
 *                  until replaced, so it must stay valid and unchanged while
 *                  that work runs).  NULL turns the correction off.
 *   step_samples : samples per step, a multiple of L (6400 = 5 ms).
 * Step 0 starts at the plan's current stream position; mwax_channelise
 * returns MWAX_E_INVAL if a call reaches past step n_steps - 1.  The INT8
 * calibration measures power, which the unit-modulus gains leave unchanged,
 * so it runs on the uncorrected spectra.  MWAX_E_STATE with a block pending
 * correlation; MWAX_E_UNSUPPORTED for instances of a batch (whose F-engine
 * runs from batch tables); MWAX_E_INVAL for bad arguments.  mwax_reset turns
 * the correction off. */
mwax_status mwax_set_delays(mwax_plan p, const float *d_delays, int64_t n_steps, int64_t step_samples,
                            double sky_freq_hz);

/* Discard every integration in progress or not yet emitted and any pending
 * channelised block; the stream position returns to zero and delay
 * correction is turned off. */
mwax_status mwax_reset(mwax_plan p);

/* Wait for the plan's stream.  MWAX_E_DEVICE if the runtime reports an error. */
mwax_status mwax_sync(mwax_plan p);

/* Kernel timing for measurement.  When enabled, the plan records HIP events on
 * its stream around each launch of the F-engine, X-engine and pack kernels.
 * mwax_kernel_time synchronises the stream and returns, for a kernel family
 * (0 = F-engine main pass, 1 = X-engine, 2 = pack, 3 = int8 scale
 * calibration: statistics pass and its reduction), the summed duration in
 * milliseconds and the launch count since the last read, then clears them. */
mwax_status mwax_set_timing(mwax_plan p, int32_t enable);
mwax_status mwax_kernel_time(mwax_plan p, int32_t family, double *total_ms, int64_t *launches);

/* ------------------------------------------------------------------------
 * Batches.  The cluster of Sec. 2.1 correlates up to 24 coarse channels, one
 * per server, each with the FX engine of Sec. 2.5.  A batch runs many such
 * per-coarse-channel plans ("instances", which may differ in tile count, FFT
 * length and integration time) on one GPU as one unit of device work per call:
 * the table-driven F-engine launches (one per distinct FFT length), the scale
 * calibration and a single persistent matrix-core X-engine launch that takes
 * 128 x 128 tiles of every instance from per-XCD work queues.  The sequence is
 * captured once in a HIP graph and replayed on every call; only its device
 * work tables change (uploaded from pinned host memory ahead of the replay).
 *
 * Each instance is a full plan (same workspace, stream position, integrators
 * and mwax_integrate / mwax_integrate_raw_i64 / mwax_plan_get_dims /
 * mwax_set_scales behaviour); the batch owns them.  Results are those of the
 * same plans driven one by one with mwax_channelise + mwax_correlate: bit for
 * bit for INT8, and for FP16 too (every integrator element is summed in the
 * same order).
 * ------------------------------------------------------------------------ */
typedef struct mwax_batch_s *mwax_batch;

/* Create a batch of n (1..64) instances from cfgs[n].  All instances must use
 * the same xprec, INT8 or FP16 (FP32 runs on the vector ALUs and is not
 * batched: MWAX_E_UNSUPPORTED).  hip_stream: the stream every batch call
 * enqueues on; NULL makes the batch create its own stream, which like the
 * default stream's other users synchronises with the legacy default stream.
 * Errors: MWAX_E_INVAL (a configuration, with its index in the message),
 * MWAX_E_UNSUPPORTED, MWAX_E_NOMEM, MWAX_E_DEVICE. */
mwax_status mwax_batch_create(const mwax_config *cfgs, int32_t n, void *hip_stream, mwax_batch *out);

/* Release the batch, its instances and its tables (waits for its stream). */
mwax_status mwax_batch_destroy(mwax_batch b);

/* Instance i's plan handle, for mwax_integrate and the other per-plan calls.
 * It stays owned by the batch: mwax_plan_destroy on it is refused. */
mwax_status mwax_batch_plan(mwax_batch b, int32_t i, mwax_plan *out);

/* One batch step: for every instance i with n_samples[i] > 0, the work of
 * mwax_channelise(plan_i, d_volts[i], n_samples[i], ld_samples[i]) followed by
 * mwax_correlate(plan_i); instances with n_samples[i] == 0 are left as they
 * are.  d_volts, n_samples and ld_samples are host arrays of n entries (the
 * voltage pointers are device pointers, rules as in mwax_channelise).  All
 * arguments and states are checked first: on any error nothing is enqueued
 * and no instance changes. */
mwax_status mwax_batch_run(mwax_batch b, const int8_t *const *d_volts, const int64_t *n_samples,
                           const int64_t *ld_samples);

/* Autotuner: on the given block (as for mwax_batch_run, every n_samples[i] >
 * 0), channelise once, then time the persistent X-engine on the device for
 * candidate work shapes: per instance shape (inputs, L), the MFMA tile edge
 * (128 x 128 tiles, four waves of 64 x 64; or 64 x 64 tiles, four waves of
 * 32 x 32, which waste less of the diagonal tiles on small instances) and the
 * number of row groups per work item (whole segments, or chunks of 4096 .. 128
 * row groups; INT8 only, chunks of one tile then flush with exact int64 atomic
 * adds), and the persistent grid size.  Each candidate is timed `trials` times
 * (median); the fastest is kept.  With a tuning cache set
 * (mwax_batch_set_tuning_cache), shape classes found in it take their cached
 * choice untimed (and, when every class and the batch's grid are cached, no
 * trial runs at all); the choices made are written back to it, keyed by
 * (architecture, inputs, L, precision).  Needs every instance at stream
 * position 0 with nothing accumulated (MWAX_E_STATE otherwise) and resets
 * every instance afterwards, except when everything came from the cache. */
mwax_status mwax_batch_autotune(mwax_batch b, const int8_t *const *d_volts, const int64_t *n_samples,
                                const int64_t *ld_samples, int32_t trials);

/* The tuning in force: kchunk[n] row groups per work item (0 = whole segment)
 * and the persistent X-engine grid.  set_tuning installs one (kchunk must be
 * 0, or >= 1 for INT8 batches; grid 0 = the device's resident maximum). */
mwax_status mwax_batch_get_tuning(mwax_batch b, int32_t *kchunk, int32_t *grid);
mwax_status mwax_batch_set_tuning(mwax_batch b, const int32_t *kchunk, int32_t grid);

/* The X-engine tile edge per instance (host arrays of n entries): 128 (the
 * default, as single plans) or 64.  set_tiles refuses other values and a 64
 * edge where an instance would need more than 256 tiles per channel
 * (MWAX_E_INVAL), and pending blocks (MWAX_E_STATE).  Any tiling computes the
 * same sums (INT8: bit-identical); only the work split changes. */
mwax_status mwax_batch_get_tiles(mwax_batch b, int32_t *tile);
mwax_status mwax_batch_set_tiles(mwax_batch b, const int32_t *tile);

/* The autotuner's on-disk cache: a text file (path, NUL-terminated host string,
 * copied) read before and rewritten after each mwax_batch_autotune; NULL or ""
 * turns it off (the default).  Entries: "shape <arch> <inputs> <L> <xprec>
 * <tile> <kchunk>" and "grid <arch> <classes> <xprec> <grid>".  A file that
 * cannot be written makes the autotuner return MWAX_E_INVAL after tuning. */
mwax_status mwax_batch_set_tuning_cache(mwax_batch b, const char *path);

/* Graph replay on (1, the default) or off (0: the same launches issued one by
 * one, which also allows per-kernel timing). */
mwax_status mwax_batch_set_graph(mwax_batch b, int32_t enable);

/* Timing as mwax_set_timing / mwax_kernel_time, per batch: families 0 =
 * F-engine main pass, 1 = X-engine, 3 = calibration (graph off only), 4 =
 * whole batch step (both modes). */
mwax_status mwax_batch_set_timing(mwax_batch b, int32_t enable);
mwax_status mwax_batch_kernel_time(mwax_batch b, int32_t family, double *total_ms, int64_t *launches);

/* Wait for the batch's stream. */
mwax_status mwax_batch_sync(mwax_batch b);

/* ------------------------------------------------------------------------
 * Real-time streaming.  Voltages reach a server as 8 s sub-observation blocks
 * per coarse channel (Sec. 2.4), which must be correlated as fast as they
 * arrive (Sec. 3.4: under 8 s per 8 s block).  A stream keeps one plan per
 * coarse channel (integrators stay on the device across blocks) and a pool of
 * device block buffers whose number is set by an HBM budget: admission
 * (mwax_stream_acquire) hands out a free buffer, or waits, or refuses when the
 * budget is exhausted.  Blocks are written into their buffer on the stream's
 * ingest stream (a copy from pinned host memory, mwax_stream_copy_in, or any
 * producer kernel), then submitted; the channel's lane stream (one of two,
 * channel mod 2) waits for the ingest, runs the channel's plan over the block
 * in calls of cfg.max_samples samples, and emits every completed integration
 * into the channel's device output ring; the compute stream then waits for
 * that lane, so blocks complete in submission order.
 * Block latency = ready time - arrival time, with the ready time taken from a
 * HIP event timestamp on the stream clock.
 * ------------------------------------------------------------------------ */
typedef struct mwax_stream_s *mwax_stream;

typedef struct {
    int32_t n_channels;         /* coarse channels, 1..64; channel k runs plan k         */
    int32_t out_depth;          /* integrations each channel's output ring holds (>= 1)   */
    mwax_config cfg;            /* every channel's plan; max_samples = samples per call    */
    int64_t block_samples;      /* samples per input per block; a multiple of
                                   cfg.max_samples                                         */
    uint64_t hbm_budget_bytes;  /* device bytes for resident voltage blocks; the pool holds
                                   budget / block_bytes buffers (at least 1 must fit)      */
} mwax_stream_config;

typedef struct {
    int32_t pool_slots;         /* block buffers (admission capacity)                      */
    int32_t n_inputs;
    uint64_t block_bytes;       /* n_inputs * block_samples * 2                            */
    int64_t block_ld;           /* samples between input rows of a buffer (block_samples)  */
    void *ingest_stream;        /* hipStream_t to write buffers on before submitting       */
    void *compute_stream;       /* hipStream_t ordered after each submitted block (plans run on two lane streams it joins) */
    uint64_t device_bytes;      /* device memory held: pool, plans, output rings           */
} mwax_stream_info;

typedef struct {
    int32_t channel;
    int32_t slot;
    int64_t block;              /* the channel's block sequence number                      */
    int64_t first_int;          /* first integration index emitted by this block            */
    int32_t n_ints;             /* integrations completed and emitted by this block         */
    int32_t reserved;
    double t_arrival_s;         /* as given to mwax_stream_submit (stream clock)            */
    double t_submit_s;          /* when mwax_stream_submit was called                        */
    double t_ready_s;           /* when its visibilities were in the output ring             */
} mwax_block_done;

/* Create a stream on the current device with its own ingest and compute
 * streams (default priority).  Errors: MWAX_E_INVAL (configuration, or a
 * budget that holds no block), MWAX_E_NOMEM, MWAX_E_DEVICE. */
mwax_status mwax_stream_create(const mwax_stream_config *cfg, mwax_stream *out);
/* Wait for all work, release everything. */
mwax_status mwax_stream_destroy(mwax_stream s);
mwax_status mwax_stream_get_info(mwax_stream s, mwax_stream_info *out);
/* Channel k's plan (owned by the stream). */
mwax_status mwax_stream_plan(mwax_stream s, int32_t channel, mwax_plan *out);
/* Seconds on the stream clock (steady host clock, zero at creation). */
mwax_status mwax_stream_now(mwax_stream s, double *t);

/* Admission: a free pool buffer (device int8 [n_inputs][block_ld][2]).  Waits
 * up to wait_ms milliseconds (0: do not wait; < 0: wait until one frees) for a
 * submitted block to finish; MWAX_E_STATE if the budget stays exhausted.  The
 * buffer keeps its previous contents until written. */
mwax_status mwax_stream_acquire(mwax_stream s, int32_t wait_ms, int32_t *slot, int8_t **d_block);
/* Enqueue on the ingest stream a copy of one block from host memory h_block
 * ([n_inputs][h_ld][2], h_ld >= block_samples; pinned for an asynchronous
 * copy) into an acquired buffer.  The host memory must stay valid until the
 * block is reported done. */
mwax_status mwax_stream_copy_in(mwax_stream s, int32_t slot, const int8_t *h_block, int64_t h_ld);
/* Submit an acquired buffer as channel's next block (arrival time t_arrival_s
 * on the stream clock).  Enqueues the channel's work after everything enqueued
 * so far on the ingest stream.  MWAX_E_STATE if the slot is not acquired, or
 * if the block could overwrite an output-ring entry (integration j takes the
 * entry of j - out_depth) of an integration that mwax_stream_poll has not yet
 * returned: poll first, or use a deeper ring. */
mwax_status mwax_stream_submit(mwax_stream s, int32_t slot, int32_t channel, double t_arrival_s);
/* Report finished blocks in submission order (their buffers return to the
 * pool): up to max records into out, count in *n.  wait_ms as in acquire, for
 * at least one record when blocks are in flight. */
mwax_status mwax_stream_poll(mwax_stream s, int32_t wait_ms, mwax_block_done *out, int32_t max, int32_t *n);
/* Device pointer of channel's integration j ([L][P] complex64, CHAN_TRI) once
 * mwax_stream_poll has returned its block, while it is still in the ring.  The
 * entry stays unchanged until the caller submits a block for that channel that
 * reaches it (integration j + out_depth), so reads of it, on any stream, must
 * be complete before such a submit.  MWAX_E_STATE if j is not (or no longer)
 * available. */
mwax_status mwax_stream_vis(mwax_stream s, int32_t channel, int64_t j, void **d_vis);

/* ---- visibility weights (Sec. 4.1; zeroing flags of Sec. 2.4; weight table
 * of Sec. 2.7) ----
 *
 * The capture stage zeroes the samples of lost or excised packets and flags,
 * per signal path, each 50 ms sub-block that was zeroed.  The weight of input
 * pair (n1, n2) in an integration is the fraction of its sub-blocks that are
 * populated in both inputs, one value per pair for all fine channels.  An
 * integration must span a whole number of sub-blocks (subs_per_int; 8 s = 160
 * sub-blocks).  Both calls enqueue on hip_stream (NULL = the null stream) and
 * need no plan and no workspace.
 *
 * mwax_vis_weights: d_flags = [n_inputs][n_ints * subs_per_int] uint8, device,
 * nonzero = that input's sub-block was zeroed (row n holds integration j's
 * sub-blocks at j * subs_per_int ..).  d_weights = [n_ints][P] float32, device,
 * packed like the visibilities: w = (populated-in-both count) / subs_per_int,
 * divided in FP32 (correctly rounded).  n_inputs 1..2048, subs_per_int >= 1;
 * n_ints == 0 enqueues nothing.  MWAX_E_INVAL on bad sizes, NULL or misaligned
 * pointers (weights 4-byte aligned). */
mwax_status mwax_vis_weights(const uint8_t *d_flags, int32_t n_inputs, int32_t subs_per_int, int32_t n_ints,
                             float *d_weights, void *hip_stream);
/* mwax_apply_weights: normalise CHAN_TRI visibilities in place, d_vis =
 * [n_ints][n_chan][P] complex64, device: V /= w[j][p] (FP32, correctly
 * rounded) where w > 0; where w == 0, V is left unchanged.  When the sub-block
 * length is a whole number of FFT frames (Sec. 2.5.1: 64,000-sample blocks of
 * 6,400-point frames), w == 0 means every product of the sum had a zeroed
 * sample, so V is 0 there; frames that straddle sub-blocks mix zeroed and live
 * samples, and V need not vanish (the weight counts sub-blocks, whatever L).
 * d_weights as written by mwax_vis_weights.  Sizes as above, n_chan >= 1;
 * d_vis 8-byte aligned. */
mwax_status mwax_apply_weights(void *d_vis, const float *d_weights, int32_t n_inputs, int32_t n_chan,
                               int32_t n_ints, void *hip_stream);

/* ---- channel averaging (Sec. 2.6) ----
 *
 * Average CHAN_TRI visibilities d_vis = [n_ints][n_chan][P] complex64 (DC at
 * channel n_chan/2) by F = fscrunch into d_out = [n_ints][n_chan/F][P]
 * complex64, both device memory, not overlapping.  Output channel o is centred
 * (o - N/2) * F channels from DC (N = n_chan/F, N/2 rounded down) and averages
 * the channels at offsets d around its centre: for odd F, |d| <= (F-1)/2 at
 * weight 1; for even F, |d| <= F/2 with the two outermost at weight 1/2, so
 * that a fine channel on a boundary is shared half and half.  The centre
 * output channel leaves the DC channel out and is divided by F - 1, every
 * other by F.  For even N the outermost output channel is the half channel at
 * the coarse-channel edges (its channels wrap round +-f_s/2) and is meant to be
 * ignored.  F = 1 copies.  If d_weights is not NULL ([n_ints][P] float32,
 * device, as written by mwax_vis_weights) each pair's means are also divided
 * by its weight where it is positive: the weighting Sec. 2.6 allows during
 * averaging, in the same pass.  Sums and divisions in FP64, one rounding to
 * FP32.  n_inputs 1..2048, n_chan >= 1, F >= 1 dividing n_chan; n_ints == 0
 * enqueues nothing.  MWAX_E_INVAL on bad sizes, NULL, misaligned (8 bytes;
 * weights 4) or overlapping buffers.  Enqueued on hip_stream (NULL = the null
 * stream); no workspace. */
mwax_status mwax_fscrunch(const void *d_vis, const float *d_weights, int32_t n_inputs, int32_t n_chan,
                          int32_t n_ints, int32_t fscrunch, void *d_out, void *hip_stream);

/* Message for the last error of the calling thread (empty if none). */
const char *mwax_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MWAX_H */
