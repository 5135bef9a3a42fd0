/*
 * acq.h -- acquisition-mode correlation search on AMD Instinct MI355X (gfx950).
 *
 * The problem (paper, Section 2 and Section 3 steps 7-8): given a block of
 * received complex baseband samples, decide which known tags transmitted in it
 * and estimate each detected transmission's sub-sample time of arrival, its
 * power and a quantity correlated with its SNR.  Searching correlates the one
 * block with the replicas of many tags (Section 2.1, searching mode), each over
 * a grid of carrier-offset hypotheses.
 *
 * What the library computes for every tag t, bin k and valid lag tau:
 *
 *     c[t,k,tau] = sum_{n<L} x[tau+n] * s_t[n] * exp(-j 2 pi f_k (tau+n) / Fs)
 *     P = |c|^2,  z = P / (L * Pxhat),   Pxhat = mean |x|^2 over the block,
 *
 * tau = 0 .. N-L (only lags where the whole replica lies inside the block);
 * s_t[n] = chip_t[n / spc] is the +/-1 BPSK replica held spc samples per chip
 * (the stored replica of Section 3, step 6).  The correlation is evaluated by
 * overlap-save FFT correlation (the identity of Section 4.1, with the
 * conjugate on the replica spectrum) whose replica spectra are computed once at
 * plan time and kept on the GPU (Section 4.2).  For each tag the peak
 * (Section 3, step 8) is the argmax of P over all bins and lags (ties: smaller
 * lag, then smaller bin); it is detected when z >= threshold.  The peak
 * neighbourhood is re-correlated in FP64, re-maximised within +/- refine_radius
 * lags, and the time of arrival is the vertex of the parabola through the
 * powers at the peak lag and its two neighbours (the interpolation of
 * Section 3, step 8).  The power and SNR sums of the same step become, for a
 * unit-modulus replica, the relative power A^2 = P / L^2 and the SNR
 * A^2 / sigma^2 with sigma^2 = (E - P/L) / L, E the block energy under the
 * replica at the peak.
 *
 * Carrier-offset bins are snapped to multiples of q = Fs / M_min with
 * M_min = 2^ceil(log2(L+1)): f_k = centre + (k - (K-1)/2) * step, where centre
 * and step are the requested values rounded to multiples of q (step at least
 * q when K > 1); K must be odd.  On this grid the frequency shift of a bin is an
 * exact circular rotation of the segment spectrum at any power-of-two FFT
 * length M >= M_min, so results do not depend on M.
 *
 * Conventions for every entry point:
 *   - return value: ACQ_OK (0) or a negative acq_status; no exceptions cross
 *     the boundary; acq_last_error() gives a message for the calling thread;
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory;
 *   - the caller owns every buffer it passes; a plan owns only the memory it
 *     allocated itself, and acq_release frees exactly that;
 *   - a plan is bound to one HIP stream and is not thread-safe: use one plan
 *     per stream and per host thread.
 */
#ifndef ACQ_H_
#define ACQ_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACQ_API_VERSION 2

typedef enum acq_status {
    ACQ_OK = 0,
    ACQ_ERR_INVALID_ARG = -1,        /* bad pointer, size or configuration          */
    ACQ_ERR_OOM = -2,                /* device or pinned host allocation failed     */
    ACQ_ERR_DEVICE = -3,             /* a HIP call or kernel launch failed          */
    ACQ_ERR_TRUNCATED = -4,          /* more detections than capacity; see n_found */
    ACQ_ERR_BLOCK_TOO_LONG = -5,     /* n > max_block_len of the plan              */
    ACQ_ERR_WORKSPACE_TOO_SMALL = -6,/* caller workspace smaller than acq_workspace_size */
    ACQ_ERR_UNSUPPORTED = -7,        /* valid request outside what the library implements */
    ACQ_ERR_NON_FINITE = -8          /* ACQ_FLAG_CHECK_FINITE: a block holds a NaN or infinite
                                        sample; that block gave no detection, the others'
                                        detections are delivered */
} acq_status;

typedef enum acq_precision {
    ACQ_FP32 = 0,   /* spectra stored and multiplied in FP32                       */
    ACQ_FP16 = 1,   /* spectra stored in FP16 (RNE), arithmetic in FP32            */
    ACQ_BF16 = 2    /* spectra stored in BF16 (RNE), arithmetic in FP32            */
} acq_precision;

/* acq_config.flags */
#define ACQ_FLAG_GRAPH       0x1u  /* acq_detect_batch replays one captured hipGraph  */
#define ACQ_FLAG_EXACT_BINS  0x2u  /* bins at the requested frequencies, not snapped:
                                      f_k = centre + (k - (K-1)/2) * step exactly.  Each
                                      bin is the nearest integer rotation m_k of the
                                      M-point spectrum plus a residual offset applied
                                      to the samples before the forward transform; one
                                      set of segment spectra per distinct residual. */
#define ACQ_FLAG_ASYNC       0x4u  /* acq_detect, acq_detect_batch and acq_track_batch only
                                      enqueue their kernels on the plan's stream and return:
                                      no host synchronisation, no copy, so acq_detect can be
                                      captured into a caller's hipGraph.  The detections and
                                      their count stay in the plan's workspace
                                      (acq_device_results), overwritten by the next search;
                                      acq_collect copies them to the host.  The proposal
                                      searches stay synchronous. */
#define ACQ_FLAG_CHECK_FINITE 0x8u /* a block holding a non-finite sample gives no detection
                                      and the call reports ACQ_ERR_NON_FINITE (tested on the
                                      block power: any NaN or infinite sample makes it non-
                                      finite, finite samples cannot) */

/* acq_detection.flags */
#define ACQ_DET_NEAR_EDGE    0x1u  /* peak at lag 0 or N-L: no parabola, delta = 0    */
#define ACQ_DET_WINDOW_EDGE  0x2u  /* FP64 re-maximisation ended on its window edge */

/*
 * Plan configuration.  All fields are read during acq_plan() only; `chips` is
 * copied, so the caller may free it afterwards.
 */
typedef struct acq_config {
    double        sample_rate_hz;    /* Fs > 0                                          */
    double        bin_center_hz;     /* requested centre of the offset grid              */
    double        bin_step_hz;       /* requested bin spacing (ignored when K == 1)      */
    double        threshold;         /* detection threshold on z; <= 0 selects, per
                                        block, ln(T*K*(N-L+1) / 1e-3)                    */
    const int8_t* chips;             /* host [num_tags][num_chips], each +1 or -1        */
    int64_t       max_block_len;     /* largest N accepted by acq_detect                  */
    int32_t       num_tags;          /* T >= 1                                           */
    int32_t       num_chips;         /* C >= 1                                           */
    int32_t       samples_per_chip;  /* spc in {1, 2, 4, 8}                              */
    int32_t       num_bins;          /* K >= 1, odd                                      */
    int32_t       fft_len;           /* M: power of two >= M_min; 0 = library's choice   */
    int32_t       precision;         /* acq_precision                                    */
    int32_t       refine_radius;     /* FP64 re-maximisation radius in lags, 0 -> 1, <= 8 */
    int32_t       tag_tile;          /* tags per correlation work item; 0 = default      */
    uint32_t      flags;             /* ACQ_FLAG_*                                       */
    int32_t       max_batch_blocks;  /* blocks per acq_detect_batch call; 0 -> 1         */
    int64_t       max_batch_samples; /* samples per acq_detect_batch call; 0 -> blocks * max_block_len */
} acq_config;

/* Derived plan geometry (filled by acq_plan_geometry without touching the GPU). */
typedef struct acq_geometry {
    int64_t template_len;        /* L = C * spc                                   */
    int64_t min_fft_len;         /* M_min = 2^ceil(log2(L+1))                     */
    int64_t fft_len;             /* M, the overlap-save segment length            */
    int64_t sub_fft_len;         /* M / spc, the per-tag inverse transform length */
    int64_t valid_per_segment;   /* V = M - L + 1 lags produced per segment       */
    int64_t max_segments;        /* ceil((max_block_len - L + 1) / V)              */
    double  freq_quantum_hz;     /* q = Fs / M_min                                 */
    double  bin_center_hz;       /* snapped centre                                  */
    double  bin_step_hz;         /* snapped step (0 when K == 1)                    */
    int64_t device_bytes;        /* device memory of a plan, its workspace included */
    int64_t workspace_bytes;     /* per-search buffers: acq_workspace_size          */
} acq_geometry;

/* One detection.  lag and bin identify the peak; values are FP64 re-correlations. */
typedef struct acq_detection {
    int32_t  tag;           /* tag index t                                           */
    int32_t  bin;           /* bin index k*                                          */
    int64_t  lag;           /* tau*: peak lag in samples from the block start        */
    double   toa_samples;   /* tau* + delta, delta the parabola vertex in [-1/2,1/2]  */
    double   freq_hz;       /* snapped frequency of bin k*                           */
    double   peak_power;    /* P at (k*, tau*)                                       */
    double   z;             /* P / (L * Pxhat)                                       */
    double   energy;        /* E = sum_{n<L} |x[tau*+n]|^2                           */
    double   block_power;   /* Pxhat                                                 */
    double   power;         /* relative power A^2 = P / L^2 (replica of unit modulus) */
    double   snr;           /* A^2 / sigma^2, sigma^2 = (E - P/L) / L; +inf if <= 0   */
    int32_t  block;         /* index of the block in a batch call, else 0            */
    uint32_t flags;         /* ACQ_DET_*                                             */
    int64_t  crossings;     /* hypotheses (bin, lag) of this tag with z >= threshold,
                               decided on the FP32 powers of the correlation pass    */
} acq_detection;

typedef struct acq_plan_s* acq_plan_t;

/*
 * Validate `cfg` and derive the plan geometry without any GPU call.
 * Returns ACQ_OK, ACQ_ERR_INVALID_ARG (malformed) or ACQ_ERR_UNSUPPORTED.
 */
int acq_plan_geometry(const acq_config* cfg, acq_geometry* out);

/*
 * The K snapped bin frequencies (Hz) of `cfg`, written to host `freqs_hz[0..K)`.
 * No GPU call.  n must be >= num_bins.
 */
int acq_bin_frequencies(const acq_config* cfg, double* freqs_hz, int32_t n);

/*
 * Bytes of the per-search workspace of a plan for `cfg` (Section 4.2: every
 * buffer a search writes is allocated once, not per block): segment spectra
 * for the largest batch, peak keys, refinement sums, detections, batch
 * descriptors.  No GPU call.
 */
int acq_workspace_size(const acq_config* cfg, size_t* bytes);

/*
 * Create a plan: build the replica spectra (Section 4.2: computed once, kept
 * for the plan's lifetime) and the transform tables in device memory the plan
 * allocates, and bind the per-search workspace.  `workspace`: device memory
 * of at least acq_workspace_size(cfg) bytes, 256-byte aligned, owned by the
 * caller and kept alive until acq_release (searches write nothing else);
 * NULL: the plan allocates and frees it.  A smaller `workspace_bytes` gives
 * ACQ_ERR_WORKSPACE_TOO_SMALL.  `stream` is a hipStream_t (NULL: the null
 * stream).  Synchronises the stream before returning.  On failure *out is
 * NULL and nothing is leaked.
 */
int acq_plan(const acq_config* cfg, void* workspace, size_t workspace_bytes, void* stream, acq_plan_t* out);

/*
 * Search one block.  `block`: device, n complex64 samples (interleaved re, im,
 * 8-byte aligned), read only.  Detections (at most one per tag, sorted by tag)
 * go to host `out[0..capacity)`; *n_found receives the number of detections.
 * If that exceeds capacity, the first `capacity` are written and
 * ACQ_ERR_TRUNCATED is returned.  n < L is valid and yields 0 detections.
 * Synchronous: returns after the results are on the host.  With
 * ACQ_FLAG_ASYNC the call only enqueues the search (out, capacity and n_found
 * are not used and may be NULL/0): the results stay on the device, and no
 * call it makes is illegal under stream capture, so a caller may capture it
 * into a hipGraph (the block pointer and length are then fixed in the graph).
 */
int acq_detect(acq_plan_t plan, const void* block, int64_t n,
               acq_detection* out, int32_t capacity, int32_t* n_found);

/*
 * Search a batch of blocks of uneven lengths (a stream of blocks from several
 * receivers): blocks[b] is a device pointer to lens[b] complex64 samples, both
 * arrays on the host, 1 <= nblocks <= max_batch_blocks, every lens[b] <=
 * max_block_len and their sum <= max_batch_samples.  Each block is searched
 * independently, exactly as acq_detect would (same kernels, same results);
 * the work items of all blocks share one correlation launch.
 * Detections are sorted by (block, tag) and carry their block index.  With
 * ACQ_FLAG_GRAPH the launch sequence is captured once as a hipGraph (on a
 * private stream) and replayed on the plan's stream for every later call;
 * block descriptors travel through pinned memory that the graph copies.
 * block_of (host [capacity], may be NULL) receives the block index of each
 * delivered detection (the same value as its `block` field).
 * Synchronous; capacity and truncation as in acq_detect.  With ACQ_FLAG_ASYNC
 * the call returns once the search is enqueued (it waits only for the
 * previous call's descriptor upload); results as for acq_detect.
 */
int acq_detect_batch(acq_plan_t plan, const void* const* blocks, const int64_t* lens, int32_t nblocks,
                     acq_detection* out, int32_t capacity, int32_t* n_found, int32_t* block_of);

/*
 * Tracking-mode tasks (Section 2: a task looks for one packet of one
 * particular tag in a block of samples a little longer than the packet,
 * placed around its predicted arrival).  Each task names a device block and
 * the tag to look for; its search is the plan's search restricted to that one
 * code: every bin, every valid lag, the same kernels and FP64 refinement, at
 * most one detection.  With threshold <= 0 the per-task threshold counts the
 * hypotheses of one code, ln(K*(n-L+1) / 1e-3).
 */
typedef struct acq_track_task {
    const void* block;      /* device pointer, n complex64 samples (8-byte aligned) */
    int64_t     n;          /* samples; n <= max_block_len; n < L gives no detection */
    int32_t     tag;        /* index into the plan's codes, [0, num_tags)            */
    int32_t     reserved;   /* 0                                                     */
} acq_track_task;

/*
 * Run ntasks tracking tasks (1 <= ntasks <= max_batch_blocks, total samples
 * <= max_batch_samples; tasks may share a block or a tag) in one launch
 * sequence.  Detections are in task order, detection.block = task index.
 * ACQ_FLAG_GRAPH captures and replays a graph of its own for tracking
 * batches.  Errors: ACQ_ERR_INVALID_ARG for a tag outside [0, num_tags),
 * otherwise as acq_detect_batch.  Synchronous; capacity and truncation as in
 * acq_detect.
 */
int acq_track_batch(acq_plan_t plan, const acq_track_task* tasks, int32_t ntasks,
                    acq_detection* out, int32_t capacity, int32_t* n_found);

/*
 * Results of the plan's last search, for ACQ_FLAG_ASYNC plans (any plan may
 * call it): waits for the plan's stream, then copies the detections to host
 * out[0..capacity) and their number to *n_found, with the statuses of
 * acq_detect (ACQ_ERR_TRUNCATED, ACQ_ERR_NON_FINITE).  A plan that has not
 * searched yet reports none.
 */
int acq_collect(acq_plan_t plan, acq_detection* out, int32_t capacity, int32_t* n_found);

/*
 * Device addresses of the last search's results in the plan's workspace, for
 * consumers on the device: *records = detections (sorted, at most
 * max_batch_blocks * num_tags), *counts = int32[2] {detections, blocks with a
 * non-finite sample}.  Fixed for the plan's lifetime; valid once the search
 * has run on the plan's stream.
 */
int acq_device_results(acq_plan_t plan, const acq_detection** records, const int32_t** counts);

/*
 * For callers that cannot allocate memory (code under hipGraph capture, tight
 * serving loops, harnesses that forbid hipMalloc): acq_detect of one block
 * whose per-search buffers (segment spectra, peak keys, refinement sums,
 * candidate records) live in a static device array of the library, 64 MiB on
 * every GPU the library runs on, instead of the plan's workspace.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine) and
 * only enqueues work on the plan's stream: `out` (device, capacity records)
 * receives the detections sorted by tag, the first `capacity` of them, and
 * `count` (device, int32[1]) their total number; both are valid once the
 * stream has run the search.  Results equal acq_detect's for the same plan
 * and block.  A block whose search needs more than the static array holds
 * (about 64 MiB / (fft_len * 8) segments: 4.1 M samples at fft_len 2^15) is
 * rejected with ACQ_ERR_WORKSPACE_TOO_SMALL before anything is enqueued.
 * All calls on one GPU share its array, which keeps the last call's contents
 * (every buffer a search reads is rewritten by that search first): calls that
 * overlap on one GPU, from any plans or streams, race and must be ordered by
 * the caller.  ACQ_ERR_DEVICE if the array's address could not be resolved
 * when the plan was made.
 */
int acq_detect_noalloc(acq_plan_t plan, const void* block, int64_t n, acq_detection* out, int32_t capacity,
                       int32_t* count);


/*
 * Launch configuration of the correlation kernel.  engine: 0 = the default
 * transform engine for the plan's inverse-transform length, 1 = Stockham
 * passes through padded LDS (available for every length).  tag_tile: tags per
 * work item, 1..64.  Results do not depend on the tuning.
 */
typedef struct acq_tuning {
    int32_t engine;
    int32_t tag_tile;
    int32_t batch_launch;       /* ACQ_BATCH_GRID or ACQ_BATCH_PERSISTENT */
    int32_t track_bins;         /* bins per work item of tracking batches, 1..64;
                                   0 = chosen per launch from the work size      */
} acq_tuning;

/* Launch forms of the correlation kernel in batched searches.  GRID: one
 * workgroup per work item, dispatched by the hardware; a graph-captured batch
 * is sized for the plan's capacity and surplus workgroups exit at once.
 * PERSISTENT: one workgroup per compute unit pulling work items from per-XCD
 * atomic counters. */
#define ACQ_BATCH_GRID       0
#define ACQ_BATCH_PERSISTENT 1

typedef struct acq_tune_entry {
    acq_tuning tuning;
    int32_t    fft_len;         /* the plan's overlap-save segment length M */
    int32_t    reserved;
    double     ms;              /* acq_tune: mean correlation-kernel time over the repetitions;
                                   acq_tune_fft_len: mean time of the whole search */
} acq_tune_entry;

int acq_get_tuning(acq_plan_t plan, acq_tuning* out);
int acq_set_tuning(acq_plan_t plan, const acq_tuning* tuning);

/*
 * Autotune: time every candidate tuning (engines x tag tiles 4..64 that divide
 * the work sensibly) on the device block `block` of n samples, `reps` runs
 * each (HIP events around the correlation kernel), then both batch launch
 * forms with the fastest engine and tile on a batch of copies of the same
 * block (as many as the batch capacity holds, at most 16; the last two
 * entries; skipped when n exceeds max_batch_samples).
 * Keeps the fastest in the plan and writes the candidates to host
 * out[0..capacity) (*n_out = count).
 */
int acq_tune(acq_plan_t plan, const void* block, int64_t n, int32_t reps,
             acq_tune_entry* out, int32_t capacity, int32_t* n_out);

/*
 * Segment-length autotuning (Section 4.2: the transform sizes are chosen when
 * the plan is made, by measurement).  For every overlap-save length M this
 * library can run for `cfg` -- powers of two from the smallest M >= L + 1 up
 * to four of them, each with a per-phase transform M / samples_per_chip of at
 * most 2^14 points (the largest transform one workgroup keeps in LDS, and
 * with the tag-independent first step in registers, in its register file) --
 * a plan with fft_len = M is made on `stream` (hipStream_t), tuned by
 * acq_tune on the device block `block`, and its whole search of the block
 * (every kernel, HIP events) timed `reps` times.  One entry per M goes to host
 * out[0..capacity) (*n_out = count), with the tuning acq_tune kept; the M of
 * the fastest search goes to *best_fft_len.  cfg->fft_len is ignored; every
 * candidate plan is released before returning.  Results of a search do not
 * depend on M (up to FP32 rounding of the correlation; the FP64 refinement
 * decides the reported values).
 */
int acq_tune_fft_len(const acq_config* cfg, const void* block, int64_t n, int32_t reps, void* stream,
                     acq_tune_entry* out, int32_t capacity, int32_t* n_out, int32_t* best_fft_len);

/*
 * Test hook: the FFT-path power P[t][k][tau] for every valid lag, written to
 * device `power` laid out [T][K][n-L+1] as FP32 (the values the peak search
 * compares, before any FP64 re-correlation).  Synchronous.
 */
int acq_correlate_power(acq_plan_t plan, const void* block, int64_t n, float* power);

/*
 * Kernel timing.  With profiling on, acq_detect and acq_correlate_power record
 * HIP events on the plan's stream around each kernel they launch; after the
 * call, acq_last_kernel_times writes the durations (milliseconds) in the order
 * ACQ_KERNEL_* below to host `ms[0..n)` and the number of kernels to *count.
 * Kernels a call did not launch, or did not time, report 0.  `on` is
 * ACQ_PROFILE_OFF (the default), ACQ_PROFILE_ALL (every kernel) or
 * ACQ_PROFILE_CORRELATE (the correlation kernel only: two events per call,
 * so the timed calls run closest to unprofiled ones); other values return
 * ACQ_ERR_INVALID_ARG.
 */
#define ACQ_PROFILE_OFF        0
#define ACQ_PROFILE_ALL        1
#define ACQ_PROFILE_CORRELATE  2
#define ACQ_KERNEL_BLOCK_POWER 0
#define ACQ_KERNEL_FORWARD     1
#define ACQ_KERNEL_CORRELATE   2
#define ACQ_KERNEL_REFINE      3
#define ACQ_KERNEL_COMPACT     4
#define ACQ_NUM_KERNELS        5
int acq_set_profiling(acq_plan_t plan, int on);
int acq_last_kernel_times(acq_plan_t plan, double* ms, int32_t n, int32_t* count);

/* Release a plan and the memory it allocated.  NULL is a no-op. */
int acq_release(acq_plan_t plan);

/* ====================================================================
 * Proposal stage (an extension: the paper searches every lag).  A small
 * 1-D CNN scores the frames of a block's STFT power map; the exhaustive
 * search then runs only on the overlap-save segments that the best-scoring
 * frames propose, with a full search as fallback.  Inside the searched
 * segments every value is the one the exhaustive search computes.
 *
 * Power map: 256-sample frames at hop 128 (F = floor((n-256)/128)+1 rows),
 * periodic Hann window, P[f][b] = |DFT_256|^2 (FP32), map = ln(P / med) with
 * med the lower median of the block's F*256 powers (0 when med is 0), stored
 * [F][256] row-major as bf16 (ACQ_BF16 networks) or FP32 (ACQ_FP32).
 *
 * Network: four "same"-padded conv layers over frames (kernel 5, dilations
 * 1, 2, 4, 8, in_channels -> 64 -> 64 -> 64 -> 64, ReLU), then a 1x1 head to one
 * logit per frame.  Frame f proposes the lags [128f + 256 - L, 128f] (the
 * replica covers the whole frame); the searched segments are those meeting a
 * proposed range.  Parameters, FP32, in this order: per layer W[5][cin][64]
 * then b[64]; then wh[64], bh.  Training: mean weighted BCE with logits over
 * frames (label 1 when half the frame lies inside a transmission), Adam.
 * ==================================================================== */
typedef struct acq_cnn_s* acq_cnn_t;

typedef struct acq_cnn_config {
    int32_t precision;          /* ACQ_BF16: bf16 activations and weights, MFMA products,
                                   FP32 accumulation and master weights; ACQ_FP32: FP32
                                   throughout (reference arithmetic, slow, for tests) */
    int32_t in_channels;        /* 256 for power maps; ACQ_BF16 needs a multiple of 64 */
    int64_t max_rows;           /* most frames in one call, over all its blocks */
    int64_t max_block_len;      /* longest block acq_power_map/acq_detect_learned take */
} acq_cnn_config;

/* Number of FP32 parameters of a network with this many input channels. */
int64_t acq_cnn_num_params(int32_t in_channels);

/* Create a network bound to a HIP stream (NULL: the null stream).  Parameters
 * start at zero; load them with acq_cnn_set_params. */
int acq_cnn_create(const acq_cnn_config* cfg, void* hip_stream, acq_cnn_t* out);
int acq_cnn_release(acq_cnn_t cnn);

/* Copy n = acq_cnn_num_params FP32 parameters from / to host memory.  Setting
 * also clears the optimiser state (moments, step count). */
int acq_cnn_set_params(acq_cnn_t cnn, const float* params, int64_t n);
int acq_cnn_get_params(acq_cnn_t cnn, float* params, int64_t n);

/* Logits of nblocks blocks of `frames` rows each: input device
 * [nblocks*frames][in_channels] (bf16 or FP32 by precision), logits device
 * FP32 [nblocks*frames].  Synchronous. */
int acq_cnn_forward(acq_cnn_t cnn, const void* input, int32_t nblocks, int64_t frames, float* logits);

/* Loss and gradient for labels (device FP32 [rows]) with positive-class
 * weight pos_weight: *loss (host) is the mean loss; the gradient is kept for
 * acq_cnn_adam_step and, when grad is not NULL, copied to device FP32
 * grad[acq_cnn_num_params].  Synchronous. */
int acq_cnn_gradients(acq_cnn_t cnn, const void* input, int32_t nblocks, int64_t frames, const float* labels,
                      float pos_weight, float* grad, float* loss);

/* Adam (b1 0.9, b2 0.999, eps 1e-8) on the gradient of the last
 * acq_cnn_gradients call, learning rate lr; clears that gradient. */
int acq_cnn_adam_step(acq_cnn_t cnn, float lr);

/* Power map of one device block of n >= 256 samples into device `map`
 * (layout above); *median (host) receives med.  Synchronous. */
int acq_power_map(acq_cnn_t cnn, const void* block, int64_t n, void* map, float* median);

/* One transmission of a synthetic training block: BPSK chips (Philox stream
 * `code`) held samples_per_chip samples, amplitude amp (noise power 1),
 * carrier offset freq_over_fs cycles per sample, phase phase0 cycles at
 * sample 0, starting at sample `delay`. */
typedef struct acq_synth_tx {
    int64_t  delay;
    double   freq_over_fs;
    float    amp;
    float    phase0;
    uint32_t code;
    uint32_t reserved;
} acq_synth_tx;

#define ACQ_SYNTH_MAX_TX 32

/* A batch of synthetic blocks generated on the device (Philox4x32-10 keyed by
 * seed; block b is stream first_block + b): CN(0,1) noise plus ntx[b] <= 32
 * transmissions tx[b*32 + i] (host arrays), num_chips chips each. */
typedef struct acq_synth_batch {
    uint64_t seed;
    int64_t  first_block;
    int32_t  nblocks;
    int32_t  num_chips;
    int32_t  samples_per_chip;
    int64_t  block_len;
    const acq_synth_tx* tx;
    const int32_t* ntx;
} acq_synth_batch;

/* Write the samples of synthetic block 0 of the batch to device complex64
 * out[block_len].  Synchronous. */
int acq_synth_block(acq_cnn_t cnn, const acq_synth_batch* batch, void* out);

/* Test hook: the training labels of the batch's frames, device FP32
 * labels[nblocks * frames] (block-major): 1 where at least half of the
 * frame's 256 samples lie inside some transmission [delay, delay + L),
 * L = num_chips * samples_per_chip, else 0.  Synchronous. */
int acq_synth_labels(acq_cnn_t cnn, const acq_synth_batch* batch, float* labels);

/* One training step on a generated batch: samples, power maps, frame labels,
 * forward, loss, backward and Adam, all on the device (no sample is written to
 * memory).  *loss (host) is the batch's mean loss before the update. */
int acq_cnn_train_synthetic(acq_cnn_t cnn, const acq_synth_batch* batch, float pos_weight, float lr, float* loss);

typedef struct acq_learned_params {
    float   kappa;              /* a frame is proposed when its window score (the sum of the
                                   logits of frames f-63 .. f+64) reaches kappa */
    float   max_fraction;       /* full search when more than this fraction of segments is proposed */
    float   floor_db;           /* full search when the map median departs from the running
                                   noise floor by more than this (dB); <= 0 disables */
} acq_learned_params;

#define ACQ_FALLBACK_NONE     0
#define ACQ_FALLBACK_FRACTION 1
#define ACQ_FALLBACK_FLOOR    2

typedef struct acq_learned_report {
    int32_t proposals;          /* proposed frames */
    int32_t segments;           /* segments searched */
    int32_t total_segments;     /* segments of the block */
    int32_t fallback;           /* ACQ_FALLBACK_* */
    float   median;             /* power-map median of the block */
    float   floor;              /* running noise floor before this block */
} acq_learned_report;

/* Proposal-driven search of one device block: power map, network, window
 * scores, proposals, then the plan's search on the proposed segments only (or
 * on all segments when a fallback rule fires).  Output as acq_detect;
 * *report (host, may be NULL) describes what was searched.  The network keeps
 * the running noise floor: the first call sets it to the block's map median,
 * every later call moves it a tenth of the way towards the new median (after
 * the fallback test).  Synchronous; one call at a time per network. */
int acq_detect_learned(acq_plan_t plan, acq_cnn_t cnn, const void* block, int64_t n,
                       const acq_learned_params* params, acq_detection* out, int32_t capacity,
                       int32_t* n_found, acq_learned_report* report);

/* The proposal search over a batch of device blocks (as acq_detect_batch):
 * proposals block by block (in order, each updating the noise floor), then one
 * batched search over the proposed (or, on a fallback, all) segments of every
 * block.  reports: host [nblocks] or NULL.  Detections carry their block index.
 * Synchronous; not captured into a graph. */
int acq_detect_batch_learned(acq_plan_t plan, acq_cnn_t cnn, const void* const* blocks, const int64_t* lens,
                             int32_t nblocks, const acq_learned_params* params, acq_detection* out,
                             int32_t capacity, int32_t* n_found, acq_learned_report* reports);

/* ------------------------------------------------------------------------
 * FSK searching pipeline (Section 3, steps 1-8, with the FFT methods of
 * Section 4.1): int16 IQ samples -> complex, local-oscillator mix, band-pass
 * filter composed with two one-bit matched filters (one per FSK tone) and
 * applied by overlap-save FFTs, demodulation d = (|f1|-|f0|)/(|f1|+|f0|) and
 * u = |f1|-|f0|, real cross-correlation of d with each tag's demodulated
 * replica d^(c) (computed on the GPU at plan time by the same filters and
 * demodulator from a noise-free continuous-phase FSK packet of the tag's
 * bits), argmax of |xcorr|, parabolic interpolation and the sums w_c, q, p_c
 * of step 8 in FP64.
 * ------------------------------------------------------------------------ */
typedef struct acq_fsk_plan_s* acq_fsk_plan_t;

typedef struct acq_fsk_config {
    double         sample_rate_hz;  /* Fs > 0                                              */
    double         lo_hz;           /* mix: x[n] * exp(-j 2 pi lo n / Fs), n from the block start */
    double         f1_hz, f0_hz;    /* tones of a 1 and a 0 bit after the mix, |f| < Fs/2  */
    double         threshold;       /* report tags with z = w_c^2 / (q E_c) >= threshold;
                                       <= 0 reports every tag's peak                      */
    const float*   bp_taps;         /* host [bp_len][2] band-pass taps (re, im), copied   */
    const uint8_t* bits;            /* host [num_tags][num_bits] of 0/1, copied           */
    int64_t        max_block_len;   /* largest n accepted by acq_fsk_detect               */
    int32_t        bp_len;          /* 1 .. 1024                                          */
    int32_t        mf_len;          /* matched-filter length = samples per bit, 1 .. 64   */
    int32_t        num_tags;        /* >= 1                                               */
    int32_t        num_bits;        /* >= 1                                               */
    int32_t        fft_len;         /* correlation segment M: power of two in
                                       [2^10, 2^18], > template length; 0 = the
                                       library's choice (the smallest such power,
                                       doubled from 2^17 when the blocks -- one of
                                       max_block_len, or max_track_tasks of equal
                                       length when that is set -- need fewer
                                       transform points)                              */
    int32_t        max_track_tasks; /* tasks per acq_fsk_track call; 0 -> 16             */
} acq_fsk_config;

/* One tag's result.  The template length is n_t = num_bits * mf_len +
 * bp_len + mf_len - 2 (the nonzero span of d^(c)); lags are 0 .. n - n_t. */
typedef struct acq_fsk_detection {
    int32_t  tag;
    uint32_t flags;          /* ACQ_DET_NEAR_EDGE, ACQ_DET_WINDOW_EDGE                 */
    int64_t  lag;            /* j*: argmax of |xcorr| (FP64 re-maximised over +/-1)    */
    double   toa_samples;    /* j* + delta, delta the parabola vertex through |xcorr|  */
    double   xcorr;          /* w_c = sum_{i<n_t} d^(c)[i] d[i+j*]                     */
    double   q;              /* sum_{i<n_t} d[i+j*]^2                                  */
    double   p;              /* p_c = sum_{i<n_t} d^(c)[i] u[i+j*]                     */
    double   z;              /* w_c^2 / (q E_c), E_c = sum d^(c)^2                     */
    int32_t  block;          /* task index of acq_fsk_track, else 0                    */
    int32_t  reserved;
} acq_fsk_detection;

/* Geometry of an FSK configuration (no GPU involved): template length, the
 * correlation segment M and its valid lags, and the front end's FFT length. */
typedef struct acq_fsk_geometry {
    int64_t template_len;    /* n_t                                                    */
    int64_t fft_len;         /* M                                                      */
    int64_t valid_per_segment; /* M - n_t + 1                                          */
    int64_t filter_len;      /* composed filter length bp_len + mf_len - 1             */
    int64_t front_fft_len;   /* overlap-save length of the composed filters (4096)     */
    int64_t device_bytes;
} acq_fsk_geometry;

int acq_fsk_plan_geometry(const acq_fsk_config* cfg, acq_fsk_geometry* out);

/* Plan: composed filter spectra, replica templates d^(c) and their spectra,
 * all buffers for blocks up to max_block_len.  Synchronous on `stream`. */
int acq_fsk_plan(const acq_fsk_config* cfg, void* stream, acq_fsk_plan_t* out);
int acq_fsk_release(acq_fsk_plan_t plan);     /* NULL-safe */

/* Steps 1-5 only (test hook): d and u of a device int16 block iq[n][2] into
 * device float arrays d[n], u[n].  Synchronous. */
int acq_fsk_demod(acq_fsk_plan_t plan, const int16_t* iq, int64_t n, float* d, float* u);

/* The stored replica template d^(c) of a tag (test hook): device float[n_t]. */
int acq_fsk_template(acq_fsk_plan_t plan, int32_t tag, float* out);

/* Kernel timing of the FSK search (HIP events on the plan's stream around
 * each launch of the last acq_fsk_detect while profiling is on), in ms:
 * ms[ACQ_FSK_KERNEL_*], n >= ACQ_FSK_NUM_KERNELS. */
enum {
    ACQ_FSK_KERNEL_FRONT = 0,       /* conversion, mixing, composed filters, demodulation */
    ACQ_FSK_KERNEL_FORWARD = 1,     /* segment spectra of d                               */
    ACQ_FSK_KERNEL_CORRELATE = 2,   /* correlation with every template, peak keys         */
    ACQ_FSK_KERNEL_REFINE = 3,      /* FP64 peak sums                                     */
    ACQ_FSK_NUM_KERNELS = 4
};
int acq_fsk_set_profiling(acq_fsk_plan_t plan, int on);
int acq_fsk_last_kernel_times(acq_fsk_plan_t plan, double* ms, int32_t n);

/* Steps 1-7 (test hook): the FFT path's correlation xcorr(d, d^(c)) of every
 * tag at every lag into device float out[num_tags][n - n_t + 1] (n >= n_t).
 * Synchronous. */
int acq_fsk_xcorr(acq_fsk_plan_t plan, const int16_t* iq, int64_t n, float* out);

/* FSK tracking tasks (Section 2: one packet of one tag in a block a little
 * longer than the packet, around its predicted arrival): each task names a
 * device int16 block iq[n][2] and a tag; steps 1-8 run on every block (its
 * own LO phase from its first sample) against that tag's template only, all
 * tasks in one launch sequence.  1 <= ntasks <= max_track_tasks; the tasks'
 * total length is at most max_block_len; n < n_t gives no result.  One result
 * per task whose z reaches the threshold, in task order, block = task index.
 * Errors as acq_fsk_detect; ACQ_ERR_INVALID_ARG for a tag outside
 * [0, num_tags).  Synchronous. */
typedef struct acq_fsk_task {
    const int16_t* iq;
    int64_t        n;
    int32_t        tag;
    int32_t        reserved;      /* 0 */
} acq_fsk_task;

int acq_fsk_track(acq_fsk_plan_t plan, const acq_fsk_task* tasks, int32_t ntasks, acq_fsk_detection* out,
                  int32_t capacity, int32_t* n_found);

/* Steps 1-8 on a device int16 block iq[n][2] (n <= max_block_len): one
 * result per tag whose z reaches the threshold, in tag order, to the host
 * array out[capacity].  n < n_t gives none.  Errors and truncation as
 * acq_detect.  Synchronous. */
int acq_fsk_detect(acq_fsk_plan_t plan, const int16_t* iq, int64_t n, acq_fsk_detection* out,
                   int32_t capacity, int32_t* n_found);

/* Static description of a status code. */
const char* acq_strerror(int status);

/* Message describing the last failure on the calling thread ("" if none). */
const char* acq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ACQ_H_ */
