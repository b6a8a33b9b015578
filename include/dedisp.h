/*
 * dedisp.h -- C ABI of the MI355X (gfx950) transient-search hot path.
 *
 * The library runs the detection chain of "Spotting Radio Transients with the
 * help of GPUs" (Barsdell, Bailes, Barnes & Fluke): brute-force incoherent
 * dedispersion of 2-bit filterbank data over many trial DMs (section 2.2),
 * boxcar matched filtering through a running sum (section 2.3) and peak
 * finding by a sigma-cut followed by gathering contiguous samples into events
 * (section 2.3).  Every step runs in hand-written HIP kernels; the caller owns
 * all data buffers.
 *
 * Conventions for every entry point:
 *   - Pointers documented as "device" must point to device memory of the
 *     current HIP device; "host" pointers to ordinary host memory.
 *   - Calls are asynchronous on `stream` unless documented as synchronising.
 *   - Arguments are validated synchronously; on any non-OK status no output
 *     buffer is written (except where a CAPACITY result says otherwise) and
 *     dedisp_last_error() describes the failure.  No call aborts the process
 *     and no C++ exception crosses this boundary.
 *   - A device fault raised by earlier asynchronous work is reported as
 *     DEDISP_ERR_HIP by the next call that synchronises.
 */
#ifndef DEDISP_H
#define DEDISP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque HIP stream (hipStream_t); NULL is the legacy default stream. */
typedef struct ihipStream_t* dedisp_stream;

typedef enum {
    DEDISP_OK = 0,
    DEDISP_ERR_INVALID_ARG = 1,
    DEDISP_ERR_TOO_FEW_SAMPLES = 2,
    DEDISP_ERR_OUT_OF_MEMORY = 3,
    DEDISP_ERR_CAPACITY = 4,
    DEDISP_ERR_HIP = 5,
    DEDISP_ERR_UNSUPPORTED = 6,
    DEDISP_ERR_BUSY = 7
} dedisp_status;

typedef enum { DEDISP_OUT_I32 = 0, DEDISP_OUT_U16 = 1 } dedisp_out_type;

/* One detected event (section 2.3: a contiguous above-threshold region of one
 * boxcar series).  40 bytes. */
typedef struct {
    int32_t width_idx; /* index into the widths list                            */
    int32_t dm_idx;    /* DM trial index                                        */
    int64_t t_start;   /* first sample of the run (boxcar start index)          */
    int64_t t_end;     /* last sample of the run, inclusive                     */
    int64_t t_peak;    /* first sample where the boxcar sum is largest          */
    int32_t b_peak;    /* boxcar sum at t_peak                                  */
    float snr;         /* (B - mean) / sigma at t_peak, population sigma        */
} dedisp_event;

/* One candidate: a cluster of events merged across DM trials and widths
 * (dedisp_cluster_events).  72 bytes. */
typedef struct {
    int64_t first;     /* lowest event index in the cluster (its identity)      */
    int64_t rep;       /* event of largest snr; ties to the lower index         */
    int64_t t_lo;      /* first sample any member covers (min t_start)          */
    int64_t t_hi;      /* last sample any member covers (max t_end + width - 1) */
    int64_t t_peak;    /* t_peak of the representative                          */
    int32_t n_members;
    int32_t dm_lo, dm_hi;   /* DM-trial range of the members                    */
    int32_t w_lo, w_hi;     /* width-index range of the members                 */
    int32_t dm_idx;    /* of the representative                                 */
    int32_t width_idx; /* of the representative                                 */
    float snr;         /* of the representative                                 */
} dedisp_cluster;

/* A window of raw input samples to dump from a baseband buffer
 * (dedisp_trigger_windows).  32 bytes. */
typedef struct {
    int64_t start;       /* first raw sample                                    */
    int64_t end;         /* one past the last raw sample                        */
    float snr;           /* largest cluster snr inside the window               */
    int32_t cluster;     /* index (into the clusters given) of that cluster     */
    int32_t n_clusters;  /* clusters merged into the window                     */
    int32_t reserved;
} dedisp_trigger;

typedef struct dedisp_plan_s* dedisp_plan;
typedef struct triage_model_s* triage_model;

/* ------------------------------------------------------------------------
 * Plan: the DM delay table (section 2.2).
 *
 * delay[d][c] = round(K * DM_d * (f_c^-2 - f_top^-2) / tsamp),
 *   K = 4.148808e3 s MHz^2 pc^-1 cm^3, f_c = f_top + c*df (MHz), tsamp in s,
 *   rounding half away from zero on the IEEE-double value evaluated as
 *   fc = f_top + c*df; a = 1/(fc*fc) - 1/(f_top*f_top); x = ((K*DM)*a)/tsamp.
 * max_delay = max over the table.
 *
 * nchans: number of channels, a multiple of 4, 4 <= nchans <= 21844.
 * f_top_mhz: frequency of channel 0 (the highest); df_mhz < 0 is the channel
 *   step; the lowest channel f_top + (nchans-1)*df must be > 0.
 * tsamp_s > 0: sampling interval.
 * dm_list: host, ndm finite values >= 0, non-decreasing.  Copied.
 * plan_out: host, receives the new plan.  The plan owns its device delay table
 *   and, per dedispersion tile shape, a table of LDS read offsets and shifts
 *   (ndm*nchans uint32).  The default shape's table is built here; another
 *   shape's is built, synchronously (host computation, device allocation and
 *   upload), by the first call that uses it -- make that call outside any
 *   stream capture.  Apart from that the plan is immutable: it may be used
 *   from several streams and threads at once as long as every call gets its
 *   own workspace.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP (device allocation / copy failed).
 * ------------------------------------------------------------------------ */
dedisp_status dedisp_plan_create(int32_t nchans, double f_top_mhz, double df_mhz,
                                 double tsamp_s, const double* dm_list, int32_t ndm,
                                 dedisp_plan* plan_out);
dedisp_status dedisp_plan_destroy(dedisp_plan plan);
/* Any of the output pointers may be NULL. */
dedisp_status dedisp_plan_info(dedisp_plan plan, int32_t* nchans, int32_t* ndm,
                               int64_t* max_delay);
/* host_out: host, ndm*nchans int32, row-major [d][c]. */
dedisp_status dedisp_plan_copy_delays(dedisp_plan plan, int32_t* host_out);

/* Bytes of device workspace dedisp_execute needs for nsamps samples (the
 * channel-major bit-plane copy of the input).  0 on invalid arguments. */
size_t dedisp_workspace_bytes(dedisp_plan plan, int64_t nsamps);

/* ------------------------------------------------------------------------
 * Dedispersion (section 2.2): out[d][t] = sum_c in[c][t + delay[d][c]] for
 * 0 <= t < nout = nsamps - max_delay.  Exact integer result.
 *
 * in_2bit: device, nsamps*nchans/4 bytes, time-major: channel c of sample t
 *   is the unsigned level in bits [2(c%4), 2(c%4)+1] of byte t*nchans/4 + c/4
 *   (section 1: 2 bits per sample); channel 0 = f_top.
 * out: device, [ndm][nout] row-major, int32 (DEDISP_OUT_I32) or uint16
 *   (DEDISP_OUT_U16, exact because 3*nchans <= 65535).
 * workspace: device, >= dedisp_workspace_bytes(plan, nsamps) bytes, 256-byte
 *   aligned; clobbered.
 * Errors: INVALID_ARG (NULL pointers, bad out_type), TOO_FEW_SAMPLES
 *   (nsamps <= max_delay), HIP (launch failure).  Asynchronous on stream.
 * ------------------------------------------------------------------------ */
dedisp_status dedisp_execute(dedisp_plan plan, const uint8_t* in_2bit, int64_t nsamps,
                             void* out, dedisp_out_type out_type, void* workspace,
                             dedisp_stream stream);

/* Tile shape of the dedispersion kernel: trials sharing one LDS tile
 * (4, 8, 16 or 32), 32-sample groups per lane (1 or 2; time tile = 2048 *
 * groups samples) and channels per LDS stage (multiple of 4; the LDS holds
 * two stages).  Every supported shape gives bit-identical output; they
 * differ only in speed. */
typedef struct {
    int32_t dms_per_block;
    int32_t groups;
    int32_t stage_chans;
} dedisp_tile;

/* Writes up to `cap` supported shapes to host array `out` (may be NULL when
 * cap == 0) and returns how many exist. */
int32_t dedisp_tile_candidates(dedisp_tile* out, int32_t cap);

/* The tile shape dedisp_execute uses for this plan. */
dedisp_status dedisp_default_tile(dedisp_plan plan, dedisp_tile* out);

/* dedisp_execute with an explicit tile shape (host pointer `tile`).  The
 * first call with a shape builds the plan's offset table for it (see
 * dedisp_plan_create).
 * Errors as dedisp_execute, plus INVALID_ARG for an unsupported shape,
 * UNSUPPORTED when its LDS tile does not fit for this plan and
 * OUT_OF_MEMORY when its offset table cannot be allocated. */
dedisp_status dedisp_execute_tile(dedisp_plan plan, const uint8_t* in_2bit, int64_t nsamps,
                                  void* out, dedisp_out_type out_type, void* workspace,
                                  const dedisp_tile* tile, dedisp_stream stream);

/* The two kernels of dedisp_execute, callable separately (timing, and
 * streaming callers that keep the bit-plane copy resident):
 *   dedisp_repack: in_2bit (device, layout as dedisp_execute) -> workspace
 *     (device, >= dedisp_workspace_bytes(plan, nsamps), 256-byte aligned),
 *     the channel-major bit-plane copy: for channel c, word j holds samples
 *     32j..32j+31 as two 32-bit planes (bit 0 and bit 1 of each level; bit b
 *     is sample 32j+b).  A channel's row is nwords = 2*ceil(nsamps/64) + 2
 *     words of 8 bytes, at word c*nwords of the workspace; words past the
 *     last sample, the two trailing ones included, are zero.
 *   dedisp_execute_repacked: dedispersion from that copy; `tile` (host) may
 *     be NULL for the default shape.
 * Errors and asynchrony as dedisp_execute. */
dedisp_status dedisp_repack(dedisp_plan plan, const uint8_t* in_2bit, int64_t nsamps,
                            void* workspace, dedisp_stream stream);
dedisp_status dedisp_execute_repacked(dedisp_plan plan, const void* workspace, int64_t nsamps,
                                      void* out, dedisp_out_type out_type,
                                      const dedisp_tile* tile, dedisp_stream stream);

/* ------------------------------------------------------------------------
 * Boxcar matched filter (section 2.3), materialised for a DM sub-range:
 *   P[0] = 0, P[t+1] = P[t] + s[t];  B_w[t] = P[t+w] - P[t],
 *   0 <= t < n_bx = nout - w_max + 1 (leading window; all widths share n_bx).
 *
 * in: device [ndm][nout] dedispersed series (int32 or uint16 per in_type).
 * widths: host, nwidths strictly increasing values >= 1, w_max <= nout,
 *   nwidths <= 32.
 * out: device int32 [nwidths][dm_count][n_bx] for DMs [dm_first,
 *   dm_first+dm_count) of the input.  Every B_w must be < 2^31 (true for
 *   dedispersed 2-bit data with nchans*3*w_max < 2^31).
 * Errors: INVALID_ARG, TOO_FEW_SAMPLES (n_bx < 1), HIP.  Asynchronous.
 * ------------------------------------------------------------------------ */
dedisp_status boxcar_filter(const void* in, dedisp_out_type in_type, int32_t ndm,
                            int64_t nout, const int32_t* widths, int32_t nwidths,
                            int32_t dm_first, int32_t dm_count, int32_t* out,
                            dedisp_stream stream);

/* ------------------------------------------------------------------------
 * Baseline (red-noise) removal by a running mean (section 2.3, first
 * paragraph), exact in integers:
 *   out[d][t] = in[d][t + R] - floor(sum_{j=t}^{t+2R} in[d][j] / (2R + 1)) + offset
 * for 0 <= t < nout - 2R (windows wholly inside the series).
 *
 * in: device [ndm][nout] series (int32 or uint16 per in_type; values >= 0
 *   and any 2R + 1 of them summing below 2^31 -- always so for uint16).
 * out: device [ndm][nout - 2R], int32 or uint16 per out_type, row stride
 *   nout - 2R.  The caller chooses offset so that the results fit out_type
 *   (for a dedispersed 2-bit series with values in [0, 3 nchans] and uint16
 *   output: offset = 3 nchans, needs 6 nchans <= 65535).  A constant offset
 *   changes no S/N: the result feeds boxcar_filter / find_peaks directly.
 * 0 <= radius <= 8192.  Errors: INVALID_ARG, TOO_FEW_SAMPLES, UNSUPPORTED,
 *   HIP.  Asynchronous.
 * ------------------------------------------------------------------------ */
dedisp_status baseline_remove(const void* in, dedisp_out_type in_type, int32_t ndm, int64_t nout,
                              int32_t radius, int32_t offset, void* out, dedisp_out_type out_type,
                              dedisp_stream stream);

/* Bytes of device workspace find_peaks needs. 0 on invalid arguments. */
size_t find_peaks_workspace_bytes(int32_t ndm, int64_t nout, const int32_t* widths,
                                  int32_t nwidths);

/* ------------------------------------------------------------------------
 * Peak finding (section 2.3): per (width, DM) series of B_w over its n_bx
 * samples, S1 = sum B, S2 = sum B^2, D = n*S2 - S1^2 (exact integers); a
 * sample is above the cut when S/N = (n*B - S1)/sqrt(D) > snr_thresh, decided
 * exactly as B >= ceil((S1 + isqrt(floor(k^2 D)) + 1)/n) with k the float
 * value of snr_thresh; D == 0 gives no events.  Maximal runs of consecutive
 * above-cut samples of one series become events, listed in (width_idx,
 * dm_idx, t_start) order; t_peak is the first maximum of the run and snr is
 * float((double)(n*B - S1) / sqrt((double)D)) at t_peak.
 *
 * in: device [ndm][nout] dedispersed series (int32 or uint16).
 * widths: host, as for boxcar_filter.  snr_thresh: finite, > 0.
 * events: device, capacity records.  n_events: host, receives the total
 *   number found.  If it exceeds capacity the first `capacity` events (in
 *   order) are written and DEDISP_ERR_CAPACITY is returned.
 * workspace: device, >= find_peaks_workspace_bytes(...) bytes; clobbered.
 * Synchronises `stream` (the event count is read back).
 * Errors: INVALID_ARG, TOO_FEW_SAMPLES, CAPACITY, HIP.
 * ------------------------------------------------------------------------ */
dedisp_status find_peaks(const void* in, dedisp_out_type in_type, int32_t ndm,
                         int64_t nout, const int32_t* widths, int32_t nwidths,
                         float snr_thresh, dedisp_event* events, int64_t capacity,
                         int64_t* n_events, void* workspace, dedisp_stream stream);

/* ------------------------------------------------------------------------
 * find_peaks without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as find_peaks,
 * minus `workspace`: the workspace is a static device array of 32 MiB, one
 * per GPU the library runs on, held until the process ends (its address is
 * looked up on the first call on each device).  Inputs needing more than
 * 32 MiB (find_peaks_workspace_bytes) fail with UNSUPPORTED; the survey
 * shape -- 1200 series of 503 812 samples, widths 1..512 -- needs 29.5 MiB.
 * Calls on one GPU share its array: calls that overlap in time on one GPU
 * (from several threads or streams) race and must be serialised by the
 * caller; sequential calls need no clearing (each call initialises what it
 * reads).  Synchronises `stream`.
 * ------------------------------------------------------------------------ */
dedisp_status find_peaks_noalloc(const void* in, dedisp_out_type in_type, int32_t ndm,
                                 int64_t nout, const int32_t* widths, int32_t nwidths,
                                 float snr_thresh, dedisp_event* events, int64_t capacity,
                                 int64_t* n_events, dedisp_stream stream);

/* Per-series statistics of the last find_peaks call that used `workspace`
 * with the same (ndm, nout, widths).  Host outputs of nwidths*ndm entries,
 * [w][d] order, any may be NULL: s1 = S1; s2_lo/s2_hi = low/high 64 bits of
 * S2; thr = B_thr, or -1 when D == 0 (no events), or INT64_MAX when no
 * value can pass.  Synchronises `stream`. */
dedisp_status find_peaks_read_stats(const void* workspace, int32_t ndm, int64_t nout,
                                    const int32_t* widths, int32_t nwidths, int64_t* s1,
                                    uint64_t* s2_lo, uint64_t* s2_hi, int64_t* thr,
                                    dedisp_stream stream);

/* ------------------------------------------------------------------------
 * Multibeam batch (the receiver has 13 beams, section 1; the plan of the
 * paper's discussion runs one beam per GPU -- here all beams share one GPU):
 * every beam's dedispersion runs in ONE persistent kernel that pops
 * (beam, time tile, DM block) work items, then each beam's boxcar /
 * sigma-cut / peak chain runs; the whole sequence is captured once in a HIP
 * graph and replayed, and re-captured when any beam's buffers, capacity or
 * length change.  Results are bit-identical to the single-beam calls.
 *
 * dedisp_batch_create: plans (host array of nbeams plans, same device, same
 *   counter width: all nchans <= 1365 or all > 1365; the plans must outlive
 *   the batch), widths / snr_thresh as find_peaks, out_type of every beam's
 *   series, tune_cache_path (NULL: the first plan's default tile shape; else
 *   the cached autotuned shape for the first plan when present).
 * dedisp_batch_execute: host arrays of nbeams entries: in_2bit (device
 *   inputs), nsamps, out (device series [ndm_b][nsamps_b - max_delay_b]),
 *   events (device, capacity_b records each), capacity, n_events (host
 *   outputs: events found per beam).  Synchronises `stream`.  CAPACITY when a
 *   beam found more events than its capacity (its first `capacity` written).
 *   Not thread-safe per batch object.
 * dedisp_batch_info: the tile shape, persistent grid size and number of
 *   graph captures so far (any output may be NULL).
 * ------------------------------------------------------------------------ */
typedef struct dedisp_batch_s* dedisp_batch;
dedisp_status dedisp_batch_create(const dedisp_plan* plans, int32_t nbeams,
                                  const int32_t* widths, int32_t nwidths, float snr_thresh,
                                  dedisp_out_type out_type, const char* tune_cache_path,
                                  dedisp_batch* out);
dedisp_status dedisp_batch_execute(dedisp_batch b, const uint8_t* const* in_2bit,
                                   const int64_t* nsamps, void* const* out,
                                   dedisp_event* const* events, const int64_t* capacity,
                                   int64_t* n_events, dedisp_stream stream);
dedisp_status dedisp_batch_info(dedisp_batch b, dedisp_tile* tile, int32_t* grid,
                                int32_t* captures);
dedisp_status dedisp_batch_destroy(dedisp_batch b);
/* Optional stages of the batch, in the order of the paper's pipeline
 * (section 2: interference mitigation, dedispersion, baseline removal,
 * matched filter, peak finding):
 *   rfi_k_sigma > 0: the multibeam coincidence mask of section 2.1 (as
 *     dedisp_rfi_mask with k_sigma and rfi_min_beams, over the samples every
 *     beam has: 0 <= t < min_b nsamps_b) is applied before dedispersion --
 *     flagged samples read as the mean level of every channel, as
 *     dedisp_rfi_apply writes them; the caller's inputs are not modified.
 *     Needs one channel count for all beams, 1 <= rfi_min_beams <= nbeams
 *     <= 64.  rfi_k_sigma == 0: no mask.
 *   baseline_radius R > 0 (<= 8192): baseline_remove of radius R (offset
 *     3 nchans, the batch's series type; uint16 needs 6 nchans <= 65535)
 *     runs between dedispersion and the search, which then covers the
 *     nout - 2R samples of the flattened series: event times count from the
 *     flattened series' first sample, dedispersed sample R.  0: none.
 * `out` still receives the dedispersed series.  Takes effect at the next
 * dedisp_batch_execute (the graph is captured again).  Errors: INVALID_ARG,
 * UNSUPPORTED. */
dedisp_status dedisp_batch_set_stages(dedisp_batch b, float rfi_k_sigma, int32_t rfi_min_beams,
                                      int32_t baseline_radius);

/* ------------------------------------------------------------------------
 * Autotuner of the dedispersion tile shape for one plan and input length.
 * Generates a deterministic pseudo-random input on the device, computes the
 * output with a reference shape, and times only candidates whose output is
 * bit-identical to it (others are counted in *n_rejected).  The fastest
 * shape becomes the plan's default for dedisp_execute and, when cache_path
 * is not NULL, is stored in that JSON file under the key
 * "<gfx arch>:nchans=<n>:ndm=<next power of two>:<u16|i32>".  Plans created
 * while the environment variable DEDISP_TUNE_CACHE names such a file start
 * from its u16 entry.  best_out / n_rejected (host) may be NULL.
 * Allocates about 2 output arrays + the input on the device; synchronous.
 * ------------------------------------------------------------------------ */
dedisp_status dedisp_autotune(dedisp_plan plan, int64_t nsamps, dedisp_out_type out_type,
                              const char* cache_path, dedisp_tile* best_out,
                              int32_t* n_rejected);

/* ------------------------------------------------------------------------
 * Streaming server (the paper's aim: search in real time as the telescope
 * observes, sections 1 and 3; 13 beams at ~4 MB/s each, section 1).
 *
 * Each beam delivers chunks of chunk_nsamps samples (packed as for
 * dedisp_execute).  The server keeps on the device, per beam, the last
 * H_b = max_delay_b + w_max - 1 input samples, so chunk k >= 1 of a beam
 * (contiguous after chunk k-1) is searched over the window of absolute
 * samples [k*C - H_b, (k+1)*C) and yields exactly C boxcar start positions;
 * the first chunk of a beam, or the first after a gap in seq, yields C - H_b.
 * The concatenated series / boxcars equal the one-shot result; the
 * sigma-cut statistics are those of each chunk's positions.
 *
 * Admission: the overlaps are resident; the rest of hbm_budget_bytes is cut
 * into chunk slots of dedisp_serve_slot_bytes() each (window, bit-planes,
 * uint16 series, peak workspace, 65536 event records).  Continuous batching:
 * whenever slots are free, every queued chunk of any beam joins the next
 * persistent launch; copies of one batch overlap the compute of the previous
 * one.  submit() copies the chunk to pinned staging and returns BUSY when the
 * staging is full (the caller retries).  Chunks of a beam must be submitted
 * in increasing seq; a smaller seq than already submitted is INVALID_ARG, a
 * jump marks the result GAP.  arrival_ns is the caller's CLOCK_MONOTONIC time
 * (steady clock) at which the chunk's last sample arrived; latency is
 * done_ns - arrival_ns and LATE marks results later than C * tsamp.
 * model: optional triage network (NULL: FALLBACK on every result, the plain
 * S/N detector's events are returned unscored).
 * poll(): up to cap results, waiting up to timeout_ms for the first; event
 * arrays stay valid until the next poll.  destroy() drains queued work.
 * ------------------------------------------------------------------------ */
typedef struct dedisp_server_s* dedisp_server;

enum {
    DEDISP_CHUNK_GAP = 1,       /* the chunk does not follow the previous one */
    DEDISP_CHUNK_LATE = 2,      /* result later than the chunk duration       */
    DEDISP_CHUNK_FALLBACK = 4,  /* no triage scores (no or invalid model)     */
    DEDISP_CHUNK_OVERFLOW = 8,  /* more than 65536 events: first 65536 kept   */
    DEDISP_CHUNK_CLUSTERED = 16 /* clusters of the kept events are attached   */
};

typedef struct {
    int32_t beam;
    int64_t seq;
    int64_t t_abs0;        /* absolute sample index of the window start = first position */
    int64_t n_bx;          /* boxcar start positions searched                            */
    int64_t n_events;      /* events found (may exceed the records when OVERFLOW)        */
    const dedisp_event* events;  /* host, min(n_events, 65536) records, t relative to t_abs0 */
    const float* scores;   /* host, per event: the triage score (0..1) of the candidates
                              dedisp_candidates_nms keeps (dm_half 32, t_half_per_width
                              128), -1 for the events it suppresses; NULL without a
                              network (FALLBACK)                                          */
    int64_t arrival_ns, done_ns;
    int32_t flags;
    int64_t n_clusters;    /* clusters of the kept events (CLUSTERED), else 0           */
    const dedisp_cluster* clusters;  /* host, n_clusters records, t relative to t_abs0,
                                        rep/first index the chunk's events, or NULL      */
    int64_t n_candidates;  /* events scored by the network (0 without scores)           */
} dedisp_chunk_result;

typedef struct {
    int64_t chunks_done;
    int64_t p50_ns, p99_ns, max_ns;   /* nearest-rank percentiles of latency */
    int64_t deadline_ns;              /* C * tsamp                           */
    int64_t deadline_misses;
    int64_t batches, max_batch;
    double mean_batch;
    int32_t slots;
} dedisp_serve_stats_t;

size_t dedisp_serve_slot_bytes(const dedisp_plan* plans, int32_t nbeams, int64_t chunk_nsamps,
                               const int32_t* widths, int32_t nwidths);
dedisp_status dedisp_serve_create(const dedisp_plan* plans, int32_t nbeams, int64_t chunk_nsamps,
                                  const int32_t* widths, int32_t nwidths, float snr_thresh,
                                  size_t hbm_budget_bytes, triage_model model,
                                  dedisp_server* out);
dedisp_status dedisp_serve_submit(dedisp_server s, int32_t beam, int64_t seq,
                                  const uint8_t* host_chunk, int64_t arrival_ns);
dedisp_status dedisp_serve_poll(dedisp_server s, dedisp_chunk_result* out, int32_t cap,
                                int32_t* n_out, int32_t timeout_ms);
dedisp_status dedisp_serve_stats(dedisp_server s, dedisp_serve_stats_t* stats);
/* Cluster every chunk's kept events across DM and width (the rule of
 * dedisp_cluster_events, same parameter ranges) before its result is
 * returned; results then carry CLUSTERED and their clusters.  Call before the
 * first submit (else BUSY).  Allocates, per chunk slot, a cluster workspace
 * and a 65536-record cluster buffer beyond the HBM budget given at create
 * (about 9 MB per slot at 1200 trials).  Errors: INVALID_ARG, BUSY,
 * OUT_OF_MEMORY. */
/* Optional stages of every chunk, in the order of the paper's pipeline
 * (section 2), set before the first submit (else BUSY):
 *   rfi_k_sigma > 0: the multibeam coincidence mask of section 2.1 over the
 *     round of chunks with one sequence number (as dedisp_rfi_mask with
 *     k_sigma and rfi_min_beams, over each chunk's C new samples), applied to
 *     those samples before dedispersion (dedisp_rfi_apply) -- the overlap a
 *     window reuses was masked with its own round.  A round waits until every
 *     beam has submitted that sequence number or a later one (a beam that
 *     skipped it sits the round out) and runs when a slot is free for each of
 *     its chunks, so the budget must hold a slot per beam.  rfi_k_sigma == 0:
 *     no mask.
 *   baseline_radius R > 0 (<= 8192, 6 nchans <= 65535): baseline_remove of
 *     radius R (offset 3 nchans) between dedispersion and the search; the
 *     overlap grows by 2R samples so that every chunk still yields C boxcar
 *     positions, and t_abs0 is the absolute sample of the first position of
 *     the flattened series (window start + R).  0: none.
 * The chunk slots are sized again for the stages (the budget given at create
 * still applies).  Errors: INVALID_ARG, UNSUPPORTED, BUSY, OUT_OF_MEMORY
 * (the budget holds too few slots; the previous stages stay in force). */
dedisp_status dedisp_serve_set_stages(dedisp_server s, float rfi_k_sigma, int32_t rfi_min_beams,
                                      int32_t baseline_radius);
dedisp_status dedisp_serve_set_clustering(dedisp_server s, int32_t dm_radius,
                                          int32_t width_radius, int64_t time_tol);
dedisp_status dedisp_serve_destroy(dedisp_server s);
/* Current time of the clock arrival_ns refers to. */
int64_t dedisp_now_ns(void);
/* Host-only helpers the server uses (no device needed):
 * nearest-rank percentile q in (0,1] of an ascending array (0 when n <= 0);
 * number of chunk slots a budget admits after the resident overlaps
 * (0 when not even one fits; at most 4096). */
int64_t dedisp_percentile_ns(const int64_t* sorted, int64_t n, double q);
int32_t dedisp_serve_admission(size_t budget, size_t resident, size_t slot_bytes);

/* ------------------------------------------------------------------------
 * Subband (two-stage) dedispersion: a cheaper approximation of the direct
 * method of section 2.2.  The band is split into nsub subbands of
 * S = nchans / nsub channels (subband s starts at channel c0 = s * S);
 * the plan's fine trials are grouped `group` at a time in list order, and
 * group q's coarse DM is the DM of its middle trial, q * group +
 * (size_q - 1) / 2.
 *   stage 1: sub[s][q][t] = sum_{c' < S} x[c0 + c'][t + dsub[s][q][c']],
 *     dsub the delay table of subband s as its own filterbank (top frequency
 *     f_top + c0 * df, same df and tsamp, the coarse DMs, the plan's law and
 *     rounding);
 *   stage 2: out[d][t] = sum_s sub[s][q(d)][t + delay[d][c0]].
 * Exact integers throughout; equal to direct dedispersion with the effective
 * delay delay[d][c0] + dsub[s][q(d)][c - c0].  nsub = 1 with group = 1
 * reproduces dedisp_execute exactly.
 *
 * create: plan = the fine-trial plan (must outlive the subband object);
 *   nchans / nsub a multiple of 4; group in [1, 16].  Builds one plan per
 *   subband.  UNSUPPORTED when a group's subband delays spread over more than
 *   31 728 samples.
 *   Stage 1 sums few channels per output, so create tunes its tile shape
 *   (dedisp_autotune, bit-exact candidates only) on the subband with the
 *   largest delays and uses it for every subband whose LDS tile it fits.
 * info: max_delay = nsamps - nout of the output; ncoarse = coarse trials;
 *   span = largest spread of a group's subband delays (samples); tile = the
 *   stage-1 tile shape of that subband.  Any output may be NULL.
 * workspace_bytes: device bytes for nsamps samples (0 when too few).
 * execute: in = device packed 2-bit input (time-major, as dedisp_execute);
 *   out = device [ndm][nsamps - max_delay] (int32 or uint16); workspace
 *   256-byte aligned, clobbered.  Asynchronous on `stream`.
 * Errors: INVALID_ARG, TOO_FEW_SAMPLES, UNSUPPORTED, OUT_OF_MEMORY, HIP.
 * ------------------------------------------------------------------------ */
typedef struct dedisp_subband_s* dedisp_subband;
dedisp_status dedisp_subband_create(dedisp_plan plan, int32_t nsub, int32_t group,
                                    dedisp_subband* out);
dedisp_status dedisp_subband_info(dedisp_subband b, int64_t* max_delay, int32_t* ncoarse,
                                  int32_t* span, dedisp_tile* tile);
size_t dedisp_subband_workspace_bytes(dedisp_subband b, int64_t nsamps);
dedisp_status dedisp_subband_execute(dedisp_subband b, const uint8_t* in, int64_t nsamps,
                                     void* out, dedisp_out_type out_type, void* workspace,
                                     dedisp_stream stream);
dedisp_status dedisp_subband_destroy(dedisp_subband b);

/* ------------------------------------------------------------------------
 * Event clustering across DM trials and widths.  Section 2.3 gathers the
 * above-cut samples of one series into events; one dispersed pulse crosses
 * the cut in many neighbouring trials and widths and so gives many events.
 * This merges them (friends of friends):
 *   * event e covers samples [t_start, t_end + W - 1], W = widths[width_idx];
 *   * a and b are friends when |dm_a - dm_b| <= dm_radius,
 *     |width_idx_a - width_idx_b| <= width_radius, and
 *     s_a <= e_b + time_tol and s_b <= e_a + time_tol (s, e: the spans);
 *   * a cluster is a connected component of that relation.  Clusters are
 *     listed in the order of their lowest-index member; the representative
 *     is the member of largest snr, ties to the lower index (-0 equals +0).
 *
 * events: device, n_events records in the order and form find_peaks writes
 *   (sorted by (width_idx, dm_idx, t_start); runs of one series disjoint and
 *   increasing; 0 <= dm_idx < ndm, 0 <= width_idx < nwidths; t_start >= 0;
 *   t_end >= t_start; snr not NaN).  Other input gives INVALID_ARG.
 * widths: host, nwidths (1..32) boxcar widths, each in [1, 2^30].
 * dm_radius in [0, 65535], width_radius in [0, 31], time_tol in [0, 2^40].
 *   The cost per event grows with (2 dm_radius + 1)(2 width_radius + 1).
 * clusters: device, capacity records; n_clusters: host, the number found.
 *   If it exceeds capacity the first `capacity` clusters are written and
 *   DEDISP_ERR_CAPACITY is returned.
 * labels: device, n_events int32 (may be NULL): the cluster index of each
 *   event (may exceed capacity).
 * workspace: device, dedisp_cluster_workspace_bytes(n_events, ndm, nwidths)
 *   bytes, 256-byte aligned; clobbered.  n_events <= 2^31 - 1.
 * Deterministic: the output does not depend on thread timing.
 * Synchronises `stream` (the count is read back).
 * Errors: INVALID_ARG, CAPACITY, HIP.
 * ------------------------------------------------------------------------ */
size_t dedisp_cluster_workspace_bytes(int64_t n_events, int32_t ndm, int32_t nwidths);
dedisp_status dedisp_cluster_events(const dedisp_event* events, int64_t n_events, int32_t ndm,
                                    const int32_t* widths, int32_t nwidths, int32_t dm_radius,
                                    int32_t width_radius, int64_t time_tol,
                                    dedisp_cluster* clusters, int64_t capacity,
                                    int64_t* n_clusters, int32_t* labels, void* workspace,
                                    dedisp_stream stream);

/* ------------------------------------------------------------------------
 * Candidate export and baseband-dump triggers (host code).  The introduction
 * motivates real-time processing by immediate follow-up of events and by
 * dumps of the full-resolution baseband data, held briefly in a buffer and
 * written out when an event merits it.
 *
 * dedisp_write_candidates: one text line per cluster (host array), after a
 *   '#' header naming the columns: snr (%.9g), t_peak + t_offset,
 *   (t_peak + t_offset) * tsamp, dm_list[dm_idx], dm_idx, widths[width_idx],
 *   width_idx, n_members, t_lo + t_offset, t_hi + t_offset, dm_lo, dm_hi, beam.
 *   Time and DM print with %.17g (they read back exactly).  Overwrites path.
 *   Errors: INVALID_ARG (NULL, bad sizes, an index outside the lists, I/O).
 *
 * dedisp_trigger_windows: for every cluster with snr >= snr_min and
 *   n_members >= min_members, the raw samples that fed its dedispersed span
 *   [t_lo, t_hi] in any channel at any trial of [dm_lo, dm_hi]:
 *     [t_lo + min delay - pad, t_hi + max delay + pad], both ends inclusive,
 *   min/max over those trials and all channels of delays (host, [ndm][nchans],
 *   as dedisp_plan_copy_delays gives), clipped to [0, nsamps).  Windows that
 *   overlap or touch are merged; the result is sorted by start and written to
 *   out (host, capacity records).  Samples are relative to the first input
 *   sample of the searched block.  *n_out receives the number of windows; if
 *   it exceeds capacity the first `capacity` are written and CAPACITY is
 *   returned.  Errors: INVALID_ARG, CAPACITY.
 * ------------------------------------------------------------------------ */
dedisp_status dedisp_write_candidates(const char* path, const dedisp_cluster* clusters, int64_t n,
                                      const double* dm_list, int32_t ndm, const int32_t* widths,
                                      int32_t nwidths, double tsamp, int64_t t_offset,
                                      int32_t beam);
dedisp_status dedisp_trigger_windows(const dedisp_cluster* clusters, int64_t n,
                                     const int32_t* delays, int32_t ndm, int32_t nchans,
                                     float snr_min, int32_t min_members, int64_t pad,
                                     int64_t nsamps, dedisp_trigger* out, int64_t capacity,
                                     int64_t* n_out);

/* ------------------------------------------------------------------------
 * Candidate selection for triage (host code).  Per boxcar width w, events
 * are visited from the highest snr down (ties: lower dm_idx, then earlier
 * t_peak, then lower index) and one is kept unless an already kept event of
 * the same width lies within dm_half trials and t_half_per_width * w samples
 * of it, both strictly (|d_a - d_b| < dm_half and |t_a - t_b| < t_half * w).
 * The triage network is trained on, and the server scores, the events this
 * keeps with dm_half = 32 and t_half_per_width = 128: one candidate per
 * 64-trial x 256 w-sample tile.
 * events: host, n >= 0 in any order; widths: host, nwidths values >= 1 that
 * width_idx indexes.  keep_out: host, room for n indices; receives the kept
 * indices in ascending order, *n_keep (host) their number.
 * Errors: INVALID_ARG (NULL, bad sizes, width_idx outside the list).
 * ------------------------------------------------------------------------ */
dedisp_status dedisp_candidates_nms(const dedisp_event* events, int64_t n, const int32_t* widths,
                                    int32_t nwidths, int32_t dm_half, int32_t t_half_per_width,
                                    int64_t* keep_out, int64_t* n_keep);

/* ------------------------------------------------------------------------
 * Multibeam coincidence RFI mask (section 2.1: interference is not localised,
 * so the beams of the multibeam receiver act as reference antennas for one
 * another; a sample where enough beams exceed a S/N threshold is flagged).
 *
 * For each beam b the zero-DM series z_b[t] = sum_c level_b(c, t) over
 * 0 <= t < nsamps (all beams cover the same samples), its exact sums
 * S1 = sum z, S2 = sum z^2, D = nsamps*S2 - S1^2, and the cut level
 * thr_b = ceil((S1 + isqrt(floor(k^2 D)) + 1) / nsamps) with k the float
 * value of k_sigma (z >= thr_b <=> (z - mean)/sigma > k, population sigma;
 * D == 0: the beam never exceeds).  mask[t] = 1 when at least min_beams
 * beams have z_b[t] >= thr_b, else 0.
 *
 * in_2bit: host array of nbeams device pointers, each nsamps*nchans/4 bytes
 *   laid out as for dedisp_execute.  1 <= nbeams <= 64; nchans a multiple of
 *   4 in [4, 21844]; 1 <= nsamps < 2^31.  k_sigma finite, > 0; min_beams >= 1.
 * mask: device, nsamps bytes (0 or 1).  n_masked: host, number of ones.
 * workspace: device, >= dedisp_rfi_mask_workspace_bytes(nbeams, nsamps)
 *   bytes, 256-byte aligned; it starts with the zero-DM series, int32
 *   [nbeams][nsamps], which dedisp_rfi_mask_read_stats copies out together
 *   with the cut levels (int64 [nbeams], -1 where D == 0).
 * Synchronises `stream`.  Errors: INVALID_ARG, HIP.
 * ------------------------------------------------------------------------ */
size_t dedisp_rfi_mask_workspace_bytes(int32_t nbeams, int64_t nsamps);
dedisp_status dedisp_rfi_mask(const uint8_t* const* in_2bit, int32_t nbeams, int32_t nchans,
                              int64_t nsamps, float k_sigma, int32_t min_beams, uint8_t* mask,
                              int64_t* n_masked, void* workspace, dedisp_stream stream);
dedisp_status dedisp_rfi_mask_read_stats(const void* workspace, int32_t nbeams, int64_t nsamps,
                                         int32_t* zero_dm, int64_t* thr, dedisp_stream stream);
/* Apply the mask (reading of section 2.1, which leaves the use of the mask
 * open): every flagged sample of every beam is replaced, in place, by the
 * mean level of the symmetric 2-bit quantiser in every channel -- level 1 in
 * even and level 2 in odd channels, so each channel pair sums to 3 and the
 * sample's zero-DM sum is exactly 1.5 * nchans.  beams_2bit: host array of
 * nbeams device pointers to packed time-major 2-bit data (modified); mask:
 * device, nsamps bytes (nonzero = flagged), as dedisp_rfi_mask writes it.
 * Asynchronous on `stream`.  Errors: INVALID_ARG, HIP. */
dedisp_status dedisp_rfi_apply(uint8_t* const* beams_2bit, int32_t nbeams, int32_t nchans,
                               int64_t nsamps, const uint8_t* mask, dedisp_stream stream);

/* ------------------------------------------------------------------------
 * Learned triage (section 2.1: interference can swamp detection with false
 * positives; a small network scores candidates so that the plain S/N
 * detector's events can be filtered).  Candidate tile of an event: 64 DM
 * rows [d_peak-32, d_peak+32) shifted into [0, ndm), 256 columns at stride w
 * (the event's width) from t0 = t_peak - 128 w clamped to
 * [0, n_bx - 255 w - 1], value (n B - S1)/sqrt(D) of that row's series, 0
 * outside the series or where D = 0, rounded to bfloat16.  Network: 4 x
 * [3x3 conv pad 1 + bias, ReLU, 2x2 max-pool] with 1->32->32->32->32
 * channels, global average, linear 32->1, logit; bfloat16 weights and
 * activations, float32 accumulation; binary cross-entropy with logits,
 * Adam (beta 0.9/0.999, eps 1e-8) on float32 master weights.  Reductions of
 * gradients are in a fixed order: a training run is reproducible.
 *
 * triage_create: weights_path NULL -> He-normal initial weights from seed;
 *   else a file written by triage_save (INVALID_ARG if missing, of another
 *   version or holding non-finite weights: callers fall back to the plain
 *   detector).
 * tiles_bf16: device [n][64][256] bfloat16 bit patterns.  labels: device
 *   float [n] in {0, 1}.  logits / scores (sigmoid): device float [n], may be
 *   NULL.  loss: host, may be NULL (then no synchronisation).
 * triage_tiles: tiles of n_events device events from a dedispersed uint16
 *   series block and the workspace of the find_peaks call that found them.
 * triage_score: the candidates' scores (sigmoid of the logit) only;
 *   triage_forward gives the logits and, optionally, the scores as well.
 * triage_set_params / triage_get_params: host float32 arrays of
 *   triage_num_params() values in the order w1[32][1][3][3], b1, w2, b2,
 *   w3, b3, w4, b4 ([32][32][3][3] and [32]), wf[32], bf[1]; grads (may be
 *   NULL) receives the gradient of the last backward pass.
 * ------------------------------------------------------------------------ */
dedisp_status triage_create(const char* weights_path, uint64_t seed, triage_model* out);
dedisp_status triage_destroy(triage_model m);
int32_t triage_num_params(void);
dedisp_status triage_set_params(triage_model m, const float* host_params, int32_t n);
dedisp_status triage_get_params(triage_model m, float* host_params, float* host_grads, int32_t n);
dedisp_status triage_tiles(const void* series_u16, int32_t ndm, int64_t nout, const int32_t* widths,
                           int32_t nwidths, const void* peaks_workspace, const dedisp_event* events,
                           int32_t n_events, uint16_t* tiles_out, dedisp_stream stream);
dedisp_status triage_forward(triage_model m, const uint16_t* tiles_bf16, int32_t n, float* logits,
                             float* scores, dedisp_stream stream);
dedisp_status triage_score(triage_model m, const uint16_t* tiles_bf16, int32_t n, float* scores,
                           dedisp_stream stream);
dedisp_status triage_forward_backward(triage_model m, const uint16_t* tiles_bf16,
                                      const float* labels, int32_t n, float* loss,
                                      dedisp_stream stream);
dedisp_status triage_train_step(triage_model m, const uint16_t* tiles_bf16, const float* labels,
                                int32_t n, float lr, float* loss, dedisp_stream stream);
dedisp_status triage_save(triage_model m, const char* path);

/* ------------------------------------------------------------------------
 * Device description, for relating measured rates to the chip's peaks
 * (compute units x 64 lanes x clock; HBM bandwidth).
 *
 * dedisp_device_info: hipGetDeviceProperties of the current device.
 *   Synchronous, host-only output.  Errors: INVALID_ARG (NULL), HIP.
 * dedisp_clock_probe: runs dependent 32-bit integer work on every SIMD (8
 *   waves each) for wall_us microseconds of wall time (100..2e6) and returns
 *   in *shader_ghz (host) the median over waves of the shader clock counter's
 *   rate against the constant-rate wall clock: the clock the shader runs at
 *   under full vector load.  Synchronous; allocates a small device buffer.
 *   Errors: INVALID_ARG, UNSUPPORTED (no wall clock), HIP.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t device;
    int32_t compute_units;
    int32_t max_clock_khz;       /* peak shader clock */
    int32_t memory_clock_khz;
    int32_t memory_bus_bits;
    int32_t l2_bytes;            /* per XCD as the runtime reports it */
    int32_t wall_clock_khz;      /* rate of the constant wall clock */
    int32_t reserved;
    int64_t lds_bytes_per_cu;
    int64_t total_memory_bytes;
    char arch[64];               /* e.g. "gfx950:sramecc+:xnack-" */
    char name[128];
} dedisp_device_props;

dedisp_status dedisp_device_info(dedisp_device_props* out);
dedisp_status dedisp_clock_probe(int32_t wall_us, double* shader_ghz);

/* Thread-local description of the last non-OK status ("" if none). */
const char* dedisp_last_error(void);

/* Library version string. */
const char* dedisp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DEDISP_H */
