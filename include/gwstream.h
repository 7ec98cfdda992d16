/*
 * gwstream.h - C ABI of libgwstream.so: streaming 1-D CNN inference and
 * training kernels for gravitational-wave time series on MI355X (gfx950).
 *
 * The calls follow the paper's framing of online inference (Gunny et al.,
 * "Hardware-accelerated Inference for Real-Time Gravitational-Wave
 * Astronomy"):
 *   - a stateful "snapshotter" holds each stream's previous input snapshot on
 *     the device; a request carries floor(f_s/r) strictly new samples that
 *     update it to the next snapshot (App. B.1)            -> snapshot_update
 *   - the updated snapshot feeds the static models: a DeepClean-shaped 1-D
 *     convolutional autoencoder that predicts witness-coupled noise (main
 *     text, DeepClean paragraph)                           -> deepclean_forward
 *     and a BBHnet-shaped 1-D CNN that scores binary-black-hole likelihood
 *     (main text, BBHnet paragraph; App. B.5 ensemble)     -> bbhnet_forward
 *   - time-series outputs are used "fully online": only the most recent
 *     floor(f_s/r) predicted samples of each window are kept (App. B.2) and
 *     subtracted from the strain (App. B.4, client pipeline)
 *   - DeepClean is retrained on recent data on a single GPU (main text,
 *     retraining paragraph)                                -> deepclean_backward
 *
 * Conventions (all calls):
 *   - Layout is channel-major, time-contiguous: a window is [C][W] float32,
 *     a batch is [n][C][W].  Parameters are one flat float32 vector in the
 *     order documented at gw_model_create.
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory read before the call returns.
 *   - Work is enqueued asynchronously on `hip_stream` (a hipStream_t, NULL =
 *     the default stream).  Device buffers must stay valid until that work
 *     completes.  Calls on one pool or one model must be serialised by the
 *     caller (one host thread, or external locking).
 *   - Every call validates all of its arguments before enqueueing anything;
 *     an invalid call returns a nonzero status and leaves all state
 *     untouched.  No C++ exception crosses the ABI.  gw_last_error() returns
 *     a thread-local message describing the last failure.
 *   - The library never allocates device memory after gw_pool_init: ring
 *     state lives in a caller-provided arena, packed weights in a
 *     caller-provided buffer and temporaries in caller-provided workspaces
 *     whose sizes the *_workspace queries return.
 */
#ifndef GWSTREAM_H
#define GWSTREAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GW_OK 0
#define GW_EINVAL 1        /* null pointer, bad shape/stride/size, duplicate slot */
#define GW_ENOMEM 2        /* arena or slot table full (admission control)       */
#define GW_ESTATE 3        /* closed slot, wrong model kind, mismatched state    */
#define GW_EHIP 4          /* a HIP runtime error; message from the runtime      */
#define GW_EUNSUPPORTED 5  /* precision or shape without a compiled kernel       */

/* ---- enums ------------------------------------------------------------- */
#define GW_FP32 0          /* FP32 direct convolution on the vector ALUs        */
#define GW_BF16 1          /* BF16 MFMA implicit GEMM, FP32 accumulate/epilogue */
#define GW_FP16 2          /* FP16 operands in the fused DeepClean kernel (the
                              reference network's inference only; the precision
                              the paper served DeepClean in); else
                              GW_EUNSUPPORTED */

#define GW_MODEL_DEEPCLEAN 1
#define GW_MODEL_BBHNET 2

#define GW_TRAIN 1u        /* deepclean_forward: batch-statistics normalisation,
                              save what deepclean_backward needs into ws      */
#define GW_RECOMPUTE 2u    /* with GW_TRAIN: save only checkpoints, recompute
                              the rest in deepclean_backward                   */
#define GW_LAYERWISE 8u    /* deepclean_forward BF16 inference: run one kernel per
                              layer instead of the fused whole-network kernel  */
#define GW_CACHE_FULL 16u  /* deepclean_forward_cached: recompute every position of
                              every cache (the from-scratch reference)          */
#define GW_CAUSAL 4u       /* deepclean_forward inference: compute only what the
                              fully-online output needs (the newest s samples
                              depend on a band of about s + 93 input samples at
                              the end of the window, the network's receptive
                              field); clean is bitwise equal to the full-window
                              result; noise must be NULL                      */

#define GW_LAYER_CONV 0
#define GW_LAYER_CONVT 1
#define GW_LAYER_BN_TANH 1 /* layer flag: BatchNorm then tanh after the conv */

typedef struct gw_pool gw_pool;
typedef struct gw_model gw_model;

/* Thread-local description of the last failed call ("" if none). */
const char* gw_last_error(void);

/* ---- snapshot pool ---------------------------------------------------- */
/*
 * gw_pool_init: create a pool of per-stream snapshot rings inside the
 * caller-owned device arena `dev_arena` of `bytes` bytes (256-byte aligned).
 * `max_slots` bounds the number of concurrently open streams and
 * `max_items` the number of items one batched call may carry.  The pool keeps
 * a small part of the arena for per-call item tables and allocates a pinned
 * host staging area of its own (released by gw_pool_free).  The arena must
 * outlive the pool.  Returns GW_EINVAL on null/misaligned/too-small input.
 */
int gw_pool_init(void* dev_arena, size_t bytes, int32_t max_slots, int32_t max_items,
                 gw_pool** out);
int gw_pool_free(gw_pool* pool);

/*
 * gw_stream_open: admit one stream of C channels and window W samples.
 * Reserves C*W float32 ring samples plus a C*W bfloat16 shadow copy (6*C*W
 * bytes, rounded up to 256) and zero-fills them on `hip_stream` (the snapshot
 * before any request is all zeros).  Writes the slot id to *slot.  Returns
 * GW_ENOMEM, with no state change, when the arena or the slot table has no
 * room: the caller's admission control queues the stream and retries after a
 * gw_stream_close.
 */
int gw_stream_open(gw_pool* pool, int32_t C, int32_t W, void* hip_stream, int32_t* slot);
/* Release a slot; its memory is reused by later opens (after pending work). */
int gw_stream_close(gw_pool* pool, int32_t slot);
/* Query a slot: channels, window, samples received so far (host-side state). */
int gw_stream_info(const gw_pool* pool, int32_t slot, int32_t* C, int32_t* W, int64_t* n_seen);
/*
 * gw_stream_window (window fetch): copy the slot's current snapshot, oldest
 * sample first, into out (device [C][W] float32, exact) and/or out_bf16
 * (device [C][W] uint16 bit patterns of the bfloat16 shadow).  Either may be
 * NULL.  Used to export stream state and by tests.
 */
int gw_stream_window(gw_pool* pool, int32_t slot, float* out, uint16_t* out_bf16, void* hip_stream);
/*
 * gw_stream_load (App. B.1, the snapshotter's state): restore a slot from an
 * exported snapshot, e.g. to move a stream to another pool or process.
 *   window  device [C][W] float32, oldest sample first (the layout that
 *           gw_stream_window writes), read on hip_stream
 *   n_seen  samples the stream had received (gw_stream_info of the source)
 * The slot's ring becomes that window (its BF16 shadow re-derived by round
 * to nearest even, so both equal the exported ones bitwise), its head 0 and
 * its received count n_seen; an attached activation cache is invalidated
 * (the next cached forward recomputes every position).  Later updates and
 * forwards continue exactly as on the source slot.  Ordering with other work
 * on the slot is as for snapshot_update.  Errors: GW_EINVAL (bad slot, null
 * window, negative n_seen), GW_EHIP.
 */
int gw_stream_load(gw_pool* pool, int32_t slot, const float* window, int64_t n_seen, void* hip_stream);
/* Pool occupancy: bytes in use by rings and bytes still free for rings. */
int gw_pool_usage(const gw_pool* pool, size_t* used, size_t* free_bytes);

/*
 * snapshot_update (App. B.1): for each item i < n, append the strictly new
 * samples of stream slots[i] to its snapshot so that it holds the most recent
 * W samples:  S <- last W samples of (S ++ X_i).
 *   slots   host [n]  open slot ids, each at most once per call
 *   strides host [n]  s_i = number of new samples, 1 <= s_i <= W_i
 *   samples device    float32; item i's block is [C_i][s_i] (channel-major)
 *                     starting at element offsets[i]
 *   offsets host [n]  element offsets into `samples`
 * Updates of one stream are applied in call order (requests of a stream are
 * sequential); items of different streams in one call run in parallel.  The
 * FP32 ring is an exact copy; the BF16 shadow holds round-to-nearest-even
 * copies for the BF16 path.  All items are validated before any launch.
 */
int snapshot_update(gw_pool* pool, int32_t n, const int32_t* slots, const int32_t* strides,
                    const float* samples, const int64_t* offsets, void* hip_stream);

/* ---- models ------------------------------------------------------------ */
/*
 * Network description `desc` (host int32):
 *   GW_MODEL_DEEPCLEAN: desc[0] = L (number of layers), then 8 ints per layer:
 *       {type (GW_LAYER_CONV|GW_LAYER_CONVT), C_in, C_out, k, stride, pad,
 *        out_pad, flags (GW_LAYER_BN_TANH or 0)}
 *     with C_in of layer l+1 == C_out of layer l, 1 <= k <= 7, stride 1 or 2,
 *     0 <= pad < k, the last layer C_out == 1 and without BN.  The reference
 *     network is 21->8->16->32->64 strided convs (k7 s2 p3, BN+tanh), then
 *     64->32->16->8->8 transposed convs (k7 s2 p3 op1, BN+tanh), then an 8->1
 *     k7 s1 p3 linear conv.  Conv weights are [C_out][C_in][k] and transposed
 *     weights [C_in][C_out][k] (cross-correlation, PyTorch layouts).
 *     Parameter order per layer: weight, bias, then with BN: gamma, beta,
 *     running mean, running variance (eps = 1e-5).
 *   GW_MODEL_BBHNET: desc[0] = number of stages S, desc[1] = input channels,
 *     desc[2..S+1] = output channels of each stage.  Stage = conv_a (k7 s2 p3)
 *     + ReLU, conv_b (k7 s1 p3), 1x1 stride-2 projection shortcut, add, ReLU;
 *     then global average pooling and Linear(C_last -> 1).  Parameter order:
 *     per stage wa, ba, wb, bb, ws, bs (conv layouts), then head w [C_last], b.
 *
 * gw_model_packed_bytes: bytes of the caller-owned device buffer that
 * gw_model_create fills with derived data (folded normalisation, BF16 weight
 * tiles).  gw_model_create validates `desc` and `n_params`, keeps pointers to
 * `dev_params` (which must outlive the model) and enqueues the packing
 * kernels on `hip_stream`.  After the caller changes dev_params (a training
 * step), gw_model_refresh re-derives the packed data; activation caches
 * computed with the previous weights are then recomputed in full by their
 * next deepclean_forward_cached.
 */
int gw_model_packed_bytes(int32_t kind, const int32_t* desc, int32_t desc_len, size_t* bytes);
int gw_model_create(int32_t kind, const int32_t* desc, int32_t desc_len, const float* dev_params,
                    int64_t n_params, void* dev_packed, size_t packed_bytes, void* hip_stream,
                    gw_model** out);
int gw_model_refresh(gw_model* model, void* hip_stream);
int gw_model_free(gw_model* model);
/* Compute-unit budget of a model's persistent kernels (the fused DeepClean
 * forward, which otherwise keeps every CU busy for its whole run): their grid
 * is sized for min(ncu, CUs of the device) CUs, so kernels of another model
 * group on a second HIP stream find CUs free while it runs.  0 (the default)
 * means every CU.  Outputs do not depend on the budget.  The setting is read
 * at each launch; changing it while a forward of this model is being enqueued
 * on another host thread races.  Errors: GW_EINVAL for a null model or
 * ncu < 0. */
int gw_model_set_cu_budget(gw_model* model, int32_t ncu);
/* gw_model_set_layerwise: for a BBHnet model of the reference shape (2 input
 * channels, stages of 32, 64 and 128 channels), BF16 forwards run by default
 * as one fused kernel that keeps every intermediate activation on chip and
 * reads ring windows in place; on != 0 selects the per-layer kernels instead
 * (the same results within the BF16 tolerance).  DeepClean takes GW_LAYERWISE
 * per call instead (GW_EINVAL here).  Same threading rule as the CU budget. */
int gw_model_set_layerwise(gw_model* model, int32_t on);
/* Number of float32 parameters a description implies. */
int gw_model_n_params(int32_t kind, const int32_t* desc, int32_t desc_len, int64_t* n_params);

/* ---- DeepClean ------------------------------------------------------- */
/*
 * deepclean_workspace: bytes of workspace deepclean_forward needs for a batch
 * of n windows of W samples at `precision` with `flags`.  With GW_TRAIN the
 * same workspace carries the saved state into deepclean_backward.
 */
int deepclean_workspace(const gw_model* model, int32_t n, int32_t W, int32_t precision,
                        uint32_t flags, size_t* bytes);

/*
 * deepclean_forward: predicted noise for n witness windows, and the
 * fully-online cleaned strain.
 * Input, one of:
 *   pool != NULL: slots host [n], open slots with C == model C_in and window
 *                 W (all equal); the windows are the current snapshots;
 *   x    != NULL: device [n][C_in][W] float32 (offline or training use).
 * Outputs (any may be NULL):
 *   noise  device [n][W] float32: the full predicted-noise window;
 *   clean  device, packed float32: item i's block [s_i] starts at the prefix
 *          sum of strides[0..i) and holds strain - noise[W - s_i .. W) (App.
 *          B.2 causal selection, App. B.4 subtraction); needs strides (host
 *          [n], 1 <= s_i <= W) and strain (device, same packing: the s_i
 *          newest strain samples of each item).
 *   delays host [n] or NULL (all 0), with clean only: aggregation latency
 *          d_i in [0, W - s_i] samples (App. B "Aggregation latency": the
 *          prediction's noisy newest edge is dropped and the output waits
 *          d_i samples).  Item i's clean block is then strain - noise[W - s_i
 *          - d_i .. W - d_i), and its strain block holds the s_i strain
 *          samples that end d_i samples before the window's newest sample.
 * precision GW_FP32, GW_BF16, or GW_FP16 (reference network, inference,
 * fused kernel only; GW_EUNSUPPORTED otherwise).  flags: 0 (inference, running statistics),
 * GW_TRAIN (batch statistics over n*time per channel; requires x),
 * GW_TRAIN|GW_RECOMPUTE, or GW_CAUSAL (inference, clean output only; the
 * band is chosen from the largest s_i + d_i and aligned to the network's total
 * stride so every layer's sample grid coincides with the full window's).
 * Returns GW_EINVAL if ws_bytes is too small (the size deepclean_workspace
 * returns for the same n, W, precision and flags always suffices).
 * W must be a multiple of 16 (four stride-2 stages).  For the reference
 * network shape, GW_BF16 inference runs one fused kernel that keeps every
 * intermediate activation on chip (unless GW_LAYERWISE is given); both
 * variants agree within the BF16 tolerance and each is bitwise reproducible.
 */
int deepclean_forward(const gw_model* model, gw_pool* pool, const int32_t* slots, const float* x,
                      int32_t n, int32_t W, const int32_t* strides, const int32_t* delays,
                      const float* strain, float* noise, float* clean, int32_t precision, uint32_t flags,
                      void* ws, size_t ws_bytes, void* hip_stream);

/*
 * deepclean_update_forward (App. B.1, then the DeepClean forward of the main
 * text): one request per stream, i.e. snapshot_update(pool, n, slots,
 * strides, samples, offsets) followed by deepclean_forward(model, pool,
 * slots, NULL, n, W, strides, delays, strain, noise, clean, precision, flags,
 * ws, ws_bytes), with the same arguments, results and errors as those two
 * calls: each stream's new samples are also its clean stride.  For BF16
 * inference on the fused network (precision GW_BF16, flags 0; noise, clean
 * or both as for deepclean_forward) it is one launch with one staged item
 * table: each tile
 * writes the new samples its input rows hold to the ring and its shadow
 * (rounded as snapshot_update rounds them) before reading its rows, and no
 * tile reads the ring positions those samples replace; outputs, rings and
 * host state are bitwise those of the two calls.  Otherwise it makes the two
 * calls.  On the one-launch path every argument is checked before any
 * launch; on the other, an error from the forward's checks comes after the
 * update has been enqueued.
 */
int deepclean_update_forward(const gw_model* model, gw_pool* pool, int32_t n, const int32_t* slots,
                             const int32_t* strides, const float* samples, const int64_t* offsets, int32_t W,
                             const int32_t* delays, const float* strain, float* noise, float* clean,
                             int32_t precision, uint32_t flags, void* ws, size_t ws_bytes, void* hip_stream);

/*
 * Incremental DeepClean forward over per-stream activation caches.  The
 * stateful model hands each request's full window to the static model
 * (App. B.1), whose update step the paper names as the online bottleneck
 * (main text, online results).  Between two requests the window only slides:
 * with a per-stream cache of every layer's activations of the last window,
 * a request recomputes only the positions whose receptive field reaches the
 * new samples or the window's left edge, and the full predicted-noise window
 * comes out as if recomputed.
 *
 * deepclean_cache_bytes: device bytes of one stream's cache for windows of W
 * samples: every layer's activations as a ring, C_out x L_out BF16 (FP32 for
 * the output conv).  W must be a multiple of 16; at most 16 layers.
 *
 * gw_stream_attach_cache: attach a caller-owned cache (device, 256-byte
 * aligned, at least deepclean_cache_bytes for the slot's W) to an open slot,
 * or detach it (cache NULL).  The memory must stay valid until it is
 * detached, replaced or the slot is closed and the work that uses it has
 * completed.  Attaching invalidates the cache (the next call recomputes it).
 *
 * deepclean_cache_bands: for the DeepClean network `desc` (as for
 * gw_model_create), the dirty positions [0, zl[l]) and [zr[l], L_l) of every
 * layer l (host [layers] each) after the window advanced by `shift` samples
 * (a multiple of 16 below W; -1: everything).  Host only (no device work).
 *
 * deepclean_forward_cached: for n slots (host [n], distinct, C == model C_in,
 * window W, each with a cache attached) whose snapshots are current on
 * hip_stream, bring every cache to the current window and write the outputs.
 * A cache that holds the window from `a` samples ago, a a multiple of 16
 * below W, is updated incrementally (its dirty bands only); any other cache
 * (never computed, attached anew, computed by another model or before this
 * model's last gw_model_refresh, a not a multiple of 16 or a >= W), and
 * every cache under GW_CACHE_FULL, is recomputed at every position.  Each
 * value is the same function of its inputs either way, so the two are
 * bitwise equal.  Arithmetic: BF16 activations (the snapshot's BF16 shadow
 * for the first layer) and BF16-rounded weights, FP32 accumulation in a
 * fixed order, FP32 folded normalisation and tanh (running statistics).
 * Outputs, as deepclean_forward's (either may be NULL): noise device [n][W]
 * float32; clean packed by strides (host [n]) with strain, and delays (host
 * [n] or NULL).  flags: 0 or GW_CACHE_FULL.  Errors: GW_EINVAL (shapes,
 * strides, delays, missing or small cache, duplicate slot), GW_ESTATE (closed
 * slot, wrong model kind), GW_EUNSUPPORTED (more than 16 layers).  Calls on
 * one pool are serialised by the caller; the caches' contents are undefined
 * if a call fails.
 */
int deepclean_cache_bytes(const gw_model* model, int32_t W, size_t* bytes);
int gw_stream_attach_cache(gw_pool* pool, int32_t slot, void* cache, size_t bytes);
int deepclean_cache_bands(const int32_t* desc, int32_t desc_len, int32_t W, int32_t shift, int32_t* zl, int32_t* zr);
int deepclean_forward_cached(const gw_model* model, gw_pool* pool, const int32_t* slots, int32_t n, int32_t W,
                             const int32_t* strides, const int32_t* delays, const float* strain, float* noise,
                             float* clean, uint32_t flags, void* hip_stream);

/*
 * gw_decimate2: streaming decimation by 2 with a causal FIR, the step of the
 * end-to-end ensemble (main text, second offline workflow; its figure of the
 * ensemble) that takes the two detectors' cleaned 4096 Hz strain to BBHnet's
 * 2048 Hz input: y[m] = sum_j taps[j] x[2m + 1 - j] over each channel's
 * stream of samples (zero before the first).  n items (streams) with C
 * channels, all with the same even stride s (new input samples per call):
 *   taps  device [ntaps] float32, 1 <= ntaps <= 257;
 *   x     device [C][n][s] float32: channel c of item i at (c n + i) s (two
 *         deepclean_forward clean outputs of equal strides, one after the
 *         other, are this layout for C = 2);
 *   hist  device [n][C][ntaps - 1] float32, caller-owned: the inputs before
 *         this call's, oldest first; zero at a stream's start; advanced by
 *         the call;
 *   y     device [n][C][s / 2] float32: the s / 2 new outputs, item by item
 *         in the [C][s/2] block layout snapshot_update reads.
 * Errors: GW_EINVAL for sizes or null pointers.
 */
int gw_decimate2(int32_t n, int32_t C, int32_t s, int32_t ntaps, const float* taps, const float* x, float* hist,
                 float* y, void* hip_stream);

/*
 * deepclean_overlap_average: aggregation of overlapping predictions (App.
 * B.2: the output segments of successive windows overlap and, unlike the
 * inputs, differ; averaging them trades latency for quality).  With depth N,
 * request k of a stream with stride s outputs the s samples that lie
 * (N - 1) s to N s samples before its newest sample, averaged over the
 * predictions of windows k - N + 1 .. k (of those that exist: min(N, k + 1)
 * windows), i.e. the mean of noise_{k-i}[W - (N - i) s + t], i = 0..N-1.
 * N = 1 is the fully-online output.  Latency grows by (N - 1) s samples.
 *   n, W, strides host [n] (1 <= s_i, N s_i <= W), counts host [n]: k_i,
 *   the number of earlier requests of item i's stream passed through this
 *   call (0 for its first request);
 *   noise  device [n][W] float32: this request's predicted windows (the
 *          noise output of deepclean_forward);
 *   state  device float32, caller-owned, packed per item: item i's block
 *          of N s_i floats starts at the prefix sum of N s_j over j < i; it
 *          must be zero before a stream's first request and is carried from
 *          one request of the stream to the next (same N and s);
 *   strain device packed [s_i] (with clean): the strain samples of the
 *          output span; clean device packed [s_i] = strain - average; avg
 *          device packed [s_i] = the averaged noise.  Either may be NULL,
 *          not both.
 * Errors: GW_EINVAL (null pointers, sizes), GW_ESTATE (not a DeepClean
 * model; the model's staging ring carries the item table).
 */
int deepclean_overlap_average(const gw_model* model, int32_t n, int32_t W, const int32_t* strides, int32_t depth,
                              const int64_t* counts, const float* noise, float* state, const float* strain,
                              float* clean, float* avg, void* hip_stream);

/*
 * deepclean_backward (retraining): gradient of a scalar loss with respect to
 * the flat parameter vector, given dnoise = dL/dnoise (device [n][W] float32)
 * for the batch-statistics forward that filled `saved` (the ws of a
 * deepclean_forward call with GW_TRAIN and the same n, W, x, flags and
 * precision).  dparams (device, n_params float32) is overwritten, not
 * accumulated; running-statistics entries get 0.  With GW_RECOMPUTE the
 * activations are recomputed from checkpoints; the result is bitwise equal
 * to the stored-activation path.  `scratch` needs deepclean_backward_scratch
 * bytes.  All reductions have a fixed order (deterministic).  precision must
 * equal the forward's: GW_BF16 runs the forward (and recomputed) convolutions
 * on BF16 matrix cores with FP32 activations, statistics and gradients.
 */
int deepclean_backward_scratch(const gw_model* model, int32_t n, int32_t W, uint32_t flags,
                               size_t* bytes);
int deepclean_backward(const gw_model* model, int32_t n, int32_t W, const float* x,
                       const float* dnoise, const void* saved, float* dparams, uint32_t flags,
                       int32_t precision, void* scratch, size_t scratch_bytes, void* hip_stream);

/*
 * gw_bandpass_mse: band-passed mean-squared-error training loss,
 *   L = 1/(n W) sum_i || P (strain_i - noise_i) ||^2,
 * where P projects each length-W row onto its DFT bins k with
 * f_lo <= k f_s / W <= f_hi, and dL/dnoise = -2/(n W) P (strain - noise).
 * strain, noise: device [n][W] float32; loss: device float32 scalar;
 * dnoise: device [n][W] float32 or NULL.  ws: gw_bandpass_workspace bytes.
 */
int gw_bandpass_workspace(int32_t n, int32_t W, float fs, float f_lo, float f_hi, size_t* bytes);
int gw_bandpass_mse(int32_t n, int32_t W, float fs, float f_lo, float f_hi, const float* strain,
                    const float* noise, float* loss, float* dnoise, void* ws, size_t ws_bytes,
                    void* hip_stream);

/*
 * gw_bandpass_mse_noalloc: gw_bandpass_mse for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training loops,
 * harnesses that forbid hipMalloc).  Same arguments and results as
 * gw_bandpass_mse (the same kernels, so bitwise the same outputs) without the
 * workspace: the projection scratch is a library-owned static device array of
 * 1 MiB per GPU, held until the process ends, so n x (number of band bins)
 * must not exceed 131072 (else GW_EINVAL, nothing enqueued).  The call
 * allocates nothing; the first call on a device looks up that device's copy
 * of the array.  Calls that overlap on one GPU (concurrent streams, or
 * threads) share that array and race: serialise them.
 */
int gw_bandpass_mse_noalloc(int32_t n, int32_t W, float fs, float f_lo, float f_hi, const float* strain,
                            const float* noise, float* loss, float* dnoise, void* hip_stream);

/* ---- BBHnet ---------------------------------------------------------- */
/*
 * bbhnet_forward: one logit (event likelihood score) per window.
 * Input, one of: pool slots (host [n], C == model C_in, window W) or dense
 * x device [n][C_in][W].  logits: device [n] float32.  W must be a multiple
 * of 2^S (S stride-2 stages).  ws: bbhnet_workspace bytes.
 */
int bbhnet_workspace(const gw_model* model, int32_t n, int32_t W, int32_t precision, size_t* bytes);
int bbhnet_forward(const gw_model* model, gw_pool* pool, const int32_t* slots, const float* x,
                   int32_t n, int32_t W, float* logits, int32_t precision, void* ws,
                   size_t ws_bytes, void* hip_stream);

/* ---- host staging --------------------------------------------------- */
/*
 * gw_host_copy_batch: n host-memory copies, dst[i] <- src[i] (bytes[i]
 * bytes), spread over up to `threads` host threads (the calling thread and
 * a pool the library starts on first use and keeps until the process ends).
 * This is the ingest step's host side (App. B.4: requests of many streams
 * packaged into pinned staging memory before the host-to-device copy): the
 * serving loop packs client arrays with it, and clients receiving straight
 * into handed-out staging buffers may use it too.  Plain host pointers;
 * regions must not overlap.  Returns GW_EINVAL for n < 0, threads < 1 or a
 * NULL pointer with bytes > 0; nothing is copied then.  The call returns when
 * every copy is complete.  Thread-safe (concurrent calls are serialised).
 */
int gw_host_copy_batch(void* const* dst, const void* const* src, const size_t* bytes, int32_t n, int32_t threads);

/* ---- measurement ------------------------------------------------------ */
/*
 * Kernel timing for benchmarks.  Between gw_profile_begin and gw_profile_end
 * every kernel launch the library makes is bracketed by two HIP events
 * recorded on the stream it is launched on.  gw_profile_end waits for those
 * events and writes one line per launch name, "name count total_ms\n", into
 * buf (NUL-terminated, truncated to len bytes), then stops recording.  Names
 * are "<kernel>.<layer>", e.g. "dc_conv_fp32.L3".  Process-wide; not for use
 * while another thread makes library calls.
 */
int gw_profile_begin(void);
int gw_profile_end(char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* GWSTREAM_H */
