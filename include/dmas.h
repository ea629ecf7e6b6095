/*
 * dmas.h -- C ABI of the MI355X (gfx950) DMAS-CF beamforming library.
 *
 * The library evaluates n-th order Delay-Multiply-and-Sum beamforming with
 * optional Coherence-Factor weighting and envelope detection, following
 * W. Jansen, W. Daems, J. Steckel, "Delay-Multiply-And-Sum Beamforming for
 * Real-Time In-Air Acoustic Imaging":
 *   - problem statement and pre-steering, Section II, eq. (1);
 *   - signed n-th root, eq. (4); DMAS-n as the n-th elementary symmetric
 *     polynomial of the roots, eqs. (5)/(6);
 *   - evaluation through the power sums of eq. (7) and the Newton-Girard
 *     identities, eqs. (8)-(12), in O(M) per output pixel;
 *   - coherence factor, eqs. (13)/(14);
 *   - envelope detection (|.| then low-pass filter), the pipeline of Section II.
 *
 * Conventions (M microphones, D directions or voxels, T samples per channel):
 *   - Recordings d_x: device memory, M x T row-major (channel i starts at
 *     element i*T), element type given by the plan's in_dtype.
 *   - Images d_y / d_env: device memory, D x T row-major FP32;
 *     element [p*T + t] is the output for direction p at sample t (the same
 *     time index as the input).
 *   - Steering delay (eq. (1)): x_i(t, p) = m_i(t + tau_{i,p}) with
 *       far field : tau = -(r_i . u_p) / c      (u_p unit vector toward the source)
 *       near field: tau = (|v_p - r_i| - |v_p|) / c   (v_p voxel centre)
 *     computed on the device in FP64 for every (direction, microphone). The
 *     NEAREST mode uses floor(fs*tau + 1/2) whole samples; the LINEAR mode
 *     interpolates between floor(fs*tau) and floor(fs*tau) + 1.
 *     Samples outside [0, T) are zero.
 *   - Signed root: sgn(0) = 0. With whole-sample delays every finite channel
 *     value, including values below the FP32 normal range (|x| < 2^-126),
 *     gets its root per eq. (4). With LINEAR delays an interpolated value
 *     below the normal range enters the root as zero.
 *   - Coherence factor: CF = (sum x_i)^2 / (M * sum x_i^2 + cf_eps) on the
 *     delayed samples; y = E_n * CF.
 *   - Envelope: env[t] = sum_k h[k] * |y[t + (L-1)/2 - k]|, y = 0 outside
 *     [0, T), odd L.
 *   - in_scale multiplies the result (S is homogeneous of degree 1 in x for a
 *     positive scale); it lets FP16/BF16 storage carry a per-frame scale.
 *
 * Ownership and threading:
 *   - A plan owns device copies of the geometry, taps and tiling tables; it is
 *     immutable after creation and may be used from several host threads and
 *     streams at once. The caller owns every I/O buffer and must make sure
 *     no work using a plan is in flight when it destroys the plan.
 *   - A plan is bound to the device that was current when it was created;
 *     calls must be made with that device current.
 *   - Launch functions are asynchronous on the given stream (a hipStream_t
 *     passed as void*; NULL is the default stream). They return after the
 *     launch, not after completion.
 *
 * Errors: every call returns a dmas_status_t. Argument and shape checks are
 * made on the host before anything is launched; a failed check launches
 * nothing. dmas_last_error() returns a message for the calling thread's most
 * recent failure. Data values are not checked: NaN and Inf propagate.
 */
#ifndef DMAS_H
#define DMAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmas_plan_s *dmas_plan_t;

typedef enum {
    DMAS_OK = 0,
    DMAS_ERR_INVALID_ARG = 1,   /* bad pointer, size, order or flag */
    DMAS_ERR_UNSUPPORTED = 2,   /* valid request the library does not serve */
    DMAS_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed */
    DMAS_ERR_DEVICE = 4,        /* a HIP call or kernel launch failed */
    DMAS_ERR_BUSY = 5,          /* serving: staging memory full, submit again later */
    DMAS_ERR_TIMEOUT = 6        /* serving: a wait ended before the frame was done */
} dmas_status_t;

typedef enum { DMAS_FARFIELD = 0, DMAS_NEARFIELD = 1 } dmas_geometry_t;
typedef enum { DMAS_F32 = 0, DMAS_F16 = 1, DMAS_BF16 = 2 } dmas_dtype_t;
typedef enum { DMAS_DELAY_NEAREST = 0, DMAS_DELAY_LINEAR = 1 } dmas_delay_mode_t;

/* Accumulation of the power sums P_k of eq. (7) and of the CF sums of
 * eq. (13). F32: plain FP32 sums. KAHAN: FP32 sums with one compensation term
 * each. F64: the signed root is taken in FP32, its powers and all sums are
 * formed in FP64, and eqs. (8)-(12) are evaluated in FP64. KAHAN and F64 are
 * built for the far field with CF and nearest delays. */
typedef enum { DMAS_ACCUM_F32 = 0, DMAS_ACCUM_KAHAN = 1, DMAS_ACCUM_F64 = 2 } dmas_accumulate_t;

/* Largest supported order n and envelope length L. */
#define DMAS_MAX_ORDER 8
#define DMAS_MAX_FIR_LEN 255
#define DMAS_MAX_MF_LEN 8192

/*
 * Plan description. Initialise with dmas_plan_desc_init() and then set the
 * fields that differ from the defaults. Host pointers are read during
 * dmas_plan_create() only.
 */
typedef struct {
    int32_t num_mics;      /* M >= 1 */
    int32_t num_samples;   /* T >= 1 */
    int32_t num_dirs;      /* D >= 1 */
    int32_t order;         /* n, 1 <= n <= min(M, DMAS_MAX_ORDER); eq. (5) */
    int32_t use_cf;        /* 0/1: coherence-factor weighting, eqs. (13)/(14) */
    int32_t geometry;      /* dmas_geometry_t */
    const double *mic_pos; /* host, M x 3 metres (x, y, z) */
    const double *dirs;    /* host, D x 3: unit vectors (far) or voxel centres in metres (near) */
    double fs;             /* sample rate, Hz, > 0 */
    double c;              /* speed of sound, m/s; 0 selects 343 */
    double cf_eps;         /* CF denominator guard; 0 selects 1e-20 */
    const float *fir_taps; /* host, fir_len taps; NULL selects the default low-pass */
    int32_t fir_len;       /* odd, 1..DMAS_MAX_FIR_LEN; 0 selects 63 */
    double fir_fc;         /* default low-pass cut-off in Hz; 0 selects 5000 */
    int32_t in_dtype;      /* dmas_dtype_t of d_x */
    int32_t ng_fp64;       /* 0/1: evaluate eqs. (8)-(12) in FP64 instead of FP32 */
    int32_t compensated;   /* dmas_accumulate_t: accumulation of the power sums (0 = FP32) */
    int32_t delay_mode;    /* dmas_delay_mode_t */
    int32_t env_decimation; /* envelope output keeps every k-th sample (k >= 1; 0 selects 1):
                               dmas_envelope writes D x ceil(T/k), element [p*ceil(T/k) + j]
                               = env[p][j*k] */
    const float *mf_pulse; /* host, mf_len samples of the emitted pulse for
                              dmas_matched_filter; NULL: no matched filter */
    int32_t mf_len;        /* 0..DMAS_MAX_MF_LEN */
} dmas_plan_desc_t;

/* Read-only facts about a created plan (tiling chosen for the device). */
typedef struct {
    int32_t num_mics, num_samples, num_dirs, order;
    int32_t dirs_per_tile;     /* directions sharing one staged channel window */
    int32_t num_tiles;
    int32_t samples_per_lane;  /* output samples each lane produces per chunk */
    int32_t chunk;             /* samples per direction per chunk */
    int32_t segment;           /* samples per direction per workgroup */
    int32_t num_segments;
    int32_t window_halo;       /* max |delay difference| to the tile's reference direction */
    int32_t mics_per_block;    /* microphones staged in LDS at once */
    int32_t lds_bytes;         /* dynamic LDS per workgroup */
    int32_t fir_len;
    int64_t workgroups;        /* per launch */
    int64_t delay_table_bytes; /* device memory of the plan's per-tile delay tables
                                  (0: delays are evaluated on the device) */
    int64_t device_bytes;      /* all device memory the plan holds (geometry, taps,
                                  tiling, delay tables); a server counts it against
                                  its HBM budget */
} dmas_plan_info_t;

/* Fill *desc with defaults: far field, FP32 input, CF on, nearest delays,
 * c = 343 m/s, cf_eps = 1e-20, default 63-tap 5 kHz low-pass. */
dmas_status_t dmas_plan_desc_init(dmas_plan_desc_t *desc);

/* Validate *desc, copy geometry and taps to the current device, choose the
 * tiling, and for whole-sample delays build per-tile delay tables on the
 * device (36 bytes per tile of 8 directions and microphone; skipped above
 * 2 GiB). Synchronises the null stream. On success *out receives the plan. n > M, an even fir_len and a
 * non-unit far-field direction (| |u| - 1 | > 1e-6) are DMAS_ERR_INVALID_ARG.
 * Environment overrides read here (tuning and tests only; results do not
 * depend on them beyond rounding order, which none of them changes):
 * DMAS_SEGMENT=s fixes the samples per workgroup (rounded up to 32),
 * DMAS_MIC_BLOCK=m the microphones per LDS block (clamped to the valid
 * range), DMAS_NO_DELAY_TABLE evaluates the delays on the device instead of
 * building tables, DMAS_BLOCK_TABLES=0/1 chooses how a kernel with at most
 * 64 microphones reads the tables (one microphone ahead, or a block of
 * offsets at a time), DMAS_RING_SHARING=0/1 whether a kernel reading a block
 * of offsets at a time keeps the envelope rings in the LDS region of the
 * channel windows, DMAS_LOG prints the plan's choices and errors to stderr. */
dmas_status_t dmas_plan_create(const dmas_plan_desc_t *desc, dmas_plan_t *out);

/* Release a plan and its device memory. NULL is a no-op. Work queued with
 * the plan must have completed (the caller synchronises its streams first). */
dmas_status_t dmas_plan_destroy(dmas_plan_t plan);

dmas_status_t dmas_plan_query(dmas_plan_t plan, dmas_plan_info_t *info);

/* DMAS-n (+CF) image, eqs. (1)-(14): writes d_y (D x T FP32, device).
 * d_x: M x T channels of the plan's in_dtype, device, row-major (channel i
 * at d_x + i*T). in_scale > 0 multiplies the result (the image is
 * homogeneous of degree 1 in x, so scaled FP16/BF16 storage is undone here).
 * Work is queued on `stream` (a hipStream_t; NULL = the null stream) and the
 * call returns without waiting. With whole-sample delays and n >= 2 the
 * call first takes every channel sample's signed root, eq. (4), into a
 * plane of M x T (root, sample) FP32 pairs, which the beamformer then reads
 * in place of d_x; the plane is allocated and freed in stream order from a
 * device memory pool that the library keeps per device (M*T*8 bytes per call
 * in flight), so one plan may be used on several streams at once. Errors:
 * DMAS_ERR_INVALID_ARG (NULL pointers, in_scale, plan of another device),
 * DMAS_ERR_OUT_OF_MEMORY (plane allocation), DMAS_ERR_DEVICE (launch). */
dmas_status_t dmas_beamform(dmas_plan_t plan, const void *d_x, float *d_y,
                            float in_scale, void *stream);

/* DMAS-n (+CF) image followed by envelope detection in the same kernel:
 * writes d_env (D x ceil(T/k) FP32, device; k = env_decimation). Arguments,
 * root plane and errors as for dmas_beamform. */
dmas_status_t dmas_envelope(dmas_plan_t plan, const void *d_x, float *d_env,
                            float in_scale, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): dmas_envelope
 * with the root plane taken from a fixed array of DMAS_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device until the process ends, instead of
 * the stream-ordered pool. The call allocates nothing (no hipMalloc, hipFree
 * or pool allocation); it computes the same kernels and gives the same bits
 * as dmas_envelope. Arguments as for dmas_envelope.
 * Limit: a plan whose root plane (M * T * 8 bytes; whole-sample delays and
 * n >= 2) exceeds DMAS_NOALLOC_SCRATCH_BYTES returns DMAS_ERR_UNSUPPORTED
 * and launches nothing; plans without a root plane (n = 1, LINEAR delays)
 * use no scratch.
 * Sharing: every call on a device uses that device's one array. Calls whose
 * work overlaps in time on one device (several streams or host threads
 * without ordering between them) race on it and give wrong results; calls
 * queued one after another on one stream are safe. The array keeps the last
 * call's roots; each call writes every element it later reads, so nothing
 * in it needs to start at zero.
 * Errors as for dmas_envelope, except that there is no allocation to fail. */
#define DMAS_NOALLOC_SCRATCH_BYTES (16u << 20)
dmas_status_t dmas_envelope_noalloc(dmas_plan_t plan, const void *d_x, float *d_env,
                                    float in_scale, void *stream);

/* Matched filter (pulse compression, the pipeline step before the
 * beamformer, Section II): d_x[i*T + t] = sum_{k < mf_len} d_raw[i*T + t + k]
 * * pulse[k], raw = 0 beyond the record. d_raw and d_x are M x T FP32 device
 * arrays (the plan must have in_dtype F32 and a pulse); d_x is then the input
 * of dmas_beamform / dmas_envelope. FP32 products and sums on the matrix
 * cores (four taps per step, steps in tap order), so each output is within
 * the usual dot-product bound of its exact value; a non-finite raw sample
 * also reaches up to 18 outputs before those that use it. */
dmas_status_t dmas_matched_filter(dmas_plan_t plan, const float *d_raw, float *d_x, void *stream);

/* The steering delays the beamformer uses, eq. (1), computed by the same
 * device code: d_whole (D x M int32, device) receives floor(fs*tau + 1/2) in
 * NEAREST mode and floor(fs*tau) in LINEAR mode; d_frac (D x M FP32, device,
 * may be NULL) receives fs*tau - floor(fs*tau) in LINEAR mode and 0 otherwise.
 * The plan's device must be current (DMAS_ERR_INVALID_ARG otherwise). */
dmas_status_t dmas_steering_delays(dmas_plan_t plan, int32_t *d_whole, float *d_frac,
                                   void *stream);

/* Default envelope low-pass design (host only): Hamming-windowed sinc of
 * odd length L and cut-off fc at sample rate fs, unit DC gain. */
dmas_status_t dmas_design_lowpass(int32_t fir_len, double fc, double fs, float *taps);

/* ------------------------------------------------------------------------
 * Serving runtime: continuous batching of heterogeneous frames.
 *
 * Not part of the paper's method (which images one frame at a time); it is
 * the request loop that keeps the GPU busy when frames of different arrays,
 * direction grids, orders and lengths arrive while others are running:
 *   - submit copies the frame's input into pinned staging memory and queues it;
 *   - a scheduler thread admits queued frames in arrival order while their
 *     device input, root plane (M*T*8 bytes, plans with whole-sample delays
 *     and n >= 2) and output fit in the HBM budget (an arena allocated once;
 *     while any frame of a plan holds device memory, an arena range of the
 *     plan's own device memory is reserved too, as accounting only: the
 *     plan's memory was allocated by dmas_plan_create, so the device holds
 *     the arena plus the plans, and the budget bounds the frames' memory
 *     together with that of the plans in use),
 *     copies the input and fills the root plane on a copy stream, and groups
 *     admitted frames into one
 *     multi-frame launch (frames with the same CF / envelope / geometry flags,
 *     nearest delays, plain sums; others are launched one by one) on the next
 *     free compute stream, so a new batch starts while earlier ones finish;
 *     launches go in arrival order, and a new one overlaps a running launch
 *     only in its last device round, except that a group of at most four
 *     device rounds of workgroups may start on an idle stream at once
 *     (DMAS_SMALL_LAUNCH_WGS, read at server creation, sets that limit in
 *     workgroups; 0 turns it off);
 *   - completion is observed from stream events and stamped per frame.
 * With `resident` set, frames of orders 3 and 5 whose plan reads its delays
 * from tables (nearest delays, plain sums) are served instead by a resident
 * worker: one persistent launch per kernel class whose workgroups take work
 * items (a frame's root-plane chunks, then its (tile, segment) workgroups) from
 * a queue of job descriptors that the scheduler writes into pinned host memory
 * while the launch runs, so frames start without a launch each; a resident
 * frame's input is read from the staging memory (coherent in this mode) and
 * takes no device copy. A worker serves
 * one class and plans created before its launch; a frame of another class or
 * a newer plan lets the worker finish its queue and exit, and the next worker is
 * launched for it (after DMAS_RESIDENT_SWITCH_US microseconds of waiting,
 * default 1000, read at server creation; at once when the worker is idle).
 * Workers exit after about 7 ms without work, and when the server is destroyed.
 * While a worker runs, the device memory of finished frames returns to the
 * budget in epochs (at least 2 ms apart, when frames wait for memory or a
 * drain waits), so hbm_in_use can include it for that long. While a worker runs it holds the compute units it was
 * launched on, so other kernels on the device (other frames' launches, plan
 * creation) start when it exits.
 * Each frame's pixels are computed by the same device code as
 * dmas_beamform / dmas_envelope, so a frame gives the same bits alone and
 * in a batch. Plans stay owned by the caller and must outlive their frames.
 * All times are seconds on dmas_server_clock().
 * ------------------------------------------------------------------------ */
typedef struct dmas_server_s *dmas_server_t;

typedef struct {
    int64_t hbm_budget_bytes;  /* arena for admitted frames' inputs, root planes and outputs, which
                                  also counts the device memory of the plans in use (> 0) */
    int64_t staging_bytes;     /* pinned host memory for queued inputs; 0 selects 256 MiB */
    int32_t num_streams;       /* launches in flight at once; 0 selects 2 */
    int32_t max_batch_frames;  /* frames per launch; 0 selects 64; 1 = one plain launch per frame */
    int32_t resident;          /* 1: serve the frames that have a resident worker through one (below); 0: launches only */
    int32_t reserved;          /* 0 */
} dmas_server_desc_t;

/* submit flags */
#define DMAS_SUBMIT_ENVELOPE 1     /* envelope image (else the RF image) */
#define DMAS_SUBMIT_AUTO_RELEASE 2 /* free the frame's device memory at completion; the
                                      frame's record is kept for dmas_server_completed */

typedef struct {
    uint64_t ticket;
    int32_t state;         /* 0 queued, 1 admitted, 2 launched, 3 done, -1 failed */
    int32_t batch_frames;  /* frames in the launch that carried this frame */
    double t_arrival;      /* caller-given arrival time (or submit time) */
    double t_admit;        /* device memory granted, input copy issued */
    double t_launch;       /* launch issued */
    double t_done;         /* completion observed */
    float *d_out;          /* device result, D x T FP32 (D x ceil(T/k) for an envelope with
                              env_decimation k); NULL until done and once released */
    int64_t pixels;        /* D * T, the beamformed pixels (before any decimation) */
} dmas_frame_info_t;

typedef struct {
    int64_t submitted, completed, failed, launches, batched_frames;
    int64_t queued, admitted_not_launched, in_flight;
    int64_t hbm_in_use, hbm_peak, hbm_budget;
    int64_t resident_launches;  /* resident worker launches */
    int64_t resident_frames;    /* frames served by resident workers */
} dmas_server_stats_t;

/* Seconds on the serving clock (monotonic). */
double dmas_server_clock(void);

/* Create a server on the current device: allocates the HBM arena
 * (hbm_budget_bytes) and pinned staging, creates the streams and starts the
 * scheduler thread. */
dmas_status_t dmas_server_create(const dmas_server_desc_t *desc, dmas_server_t *out);

/* Queue one frame. h_x: host memory, M x T of the plan's in_dtype, copied
 * before return. arrival: the request's arrival time for latency accounting
 * (< 0: now). A frame whose input + root plane + output, plus its plan's
 * device memory (dmas_plan_info_t.device_bytes), exceed the budget is
 * DMAS_ERR_INVALID_ARG; full staging is DMAS_ERR_BUSY (nothing queued). */
dmas_status_t dmas_server_submit(dmas_server_t srv, dmas_plan_t plan, const void *h_x, float in_scale,
                                 int32_t flags, double arrival, uint64_t *ticket);

/* Current record of a frame (not blocking). */
dmas_status_t dmas_server_query(dmas_server_t srv, uint64_t ticket, dmas_frame_info_t *info);

/* Block until the frame is done or failed, or timeout seconds pass
 * (DMAS_ERR_TIMEOUT). timeout >= 0 (NaN or negative: DMAS_ERR_INVALID_ARG);
 * values above 1e9, infinity included, wait 1e9 seconds. */
dmas_status_t dmas_server_wait(dmas_server_t srv, uint64_t ticket, double timeout, dmas_frame_info_t *info);

/* Return a done frame's device memory to the arena and forget the ticket. */
dmas_status_t dmas_server_release(dmas_server_t srv, uint64_t ticket);

/* Copy a done frame's result into host memory h_out (synchronous): D x T FP32,
 * or D x ceil(T/k) for an envelope of a plan with env_decimation k; h_out
 * must hold that many floats. */
dmas_status_t dmas_server_fetch(dmas_server_t srv, uint64_t ticket, float *h_out);

/* Move up to max records of auto-released, completed frames into out
 * (oldest first); *count receives how many. */
dmas_status_t dmas_server_completed(dmas_server_t srv, dmas_frame_info_t *out, int32_t max, int32_t *count);

/* Block until nothing is queued, admitted or in flight (or timeout, taken as
 * in dmas_server_wait). */
dmas_status_t dmas_server_drain(dmas_server_t srv, double timeout);

dmas_status_t dmas_server_stats(dmas_server_t srv, dmas_server_stats_t *stats);

/* Stop the scheduler after in-flight launches finish and free everything.
 * Unreleased results become invalid. NULL is a no-op. */
dmas_status_t dmas_server_destroy(dmas_server_t srv);

/* Message describing the calling thread's last failure ("" if none). */
const char *dmas_last_error(void);

/* Library version string. */
const char *dmas_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DMAS_H */
