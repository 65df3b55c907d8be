/*
 * ffv.h — C ABI of the MI355X view-interpolation library (libffv.so).
 *
 * The library evaluates the forward pass of the view-interpolation network of
 * "A Multi-user Oriented Live Free-viewpoint Video Streaming System Based On
 * View Interpolation" (section 3.1, Eq. 1 and Eq. 2; supplementary layer
 * table): given two neighbouring camera images it synthesises the virtual
 * view at phase t between them. Every step runs in the library's own HIP
 * kernels for gfx950.
 *
 * Conventions for every entry point:
 *   - Each call returns an ffv_status; nothing throws or aborts across the
 *     ABI. On failure ffv_last_error() describes the cause.
 *   - Image pointers are DEVICE pointers to planar float32 [3][H][W] RGB in
 *     [0, 1], contiguous, owned by the caller.
 *   - The library owns the net, its packed weights, its workspace, resident
 *     camera data and tickets.
 */
#ifndef FFV_H
#define FFV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFV_ABI_VERSION 1

typedef struct ffv_net ffv_net; /* opaque, library-owned */

typedef enum {
  FFV_OK = 0,
  FFV_PENDING = 1,       /* request admitted or queued, not finished */
  FFV_ERR_ARG = -1,      /* invalid argument (null, size, t out of [0,1], NaN) */
  FFV_ERR_OOM = -2,      /* device allocation failed */
  FFV_ERR_BUDGET = -3,   /* request can never fit the admission budget */
  FFV_ERR_DEVICE = -4,   /* HIP runtime error (launch, copy, sync) */
  FFV_ERR_WEIGHTS = -5,  /* weights file missing, malformed, checksum or shape mismatch */
  FFV_ERR_TICKET = -6,   /* unknown or already collected ticket */
  FFV_ERR_STATE = -7     /* call not valid in the net's current state */
} ffv_status;

typedef enum {
  FFV_FP32 = 0,      /* convolutions on fp32 MFMA, fp32 activations */
  FFV_BF16 = 1,      /* convolutions on bf16 MFMA with fp32 accumulation */
  FFV_FP8_E4M3 = 2   /* VIBlock 128/256-channel convs in fp8 e4m3 (per-channel activation
                        scales folded into per-output-channel weight scales, fp32
                        accumulation); other convs bf16. Needs ffv_calibrate. */
} ffv_precision;

typedef struct {
  int32_t abi_version;          /* must be FFV_ABI_VERSION */
  int32_t precision;            /* ffv_precision */
  int32_t device;               /* HIP device ordinal */
  int32_t graphs;               /* 1 (default): ffv_interpolate replays its launches as one
                                   hipGraph per call shape, captured on first use; 0: eager */
  void* stream;                 /* hipStream_t to order against; NULL = library stream */
  uint64_t workspace_bytes;     /* cap on the per-call workspace; 0 = 16 GiB */
  uint64_t hbm_budget_bytes;    /* serving admission budget; 0 = serving off */
  float tick_ms;                /* serving tick; <= 0 means 5 ms */
  int32_t max_batch_views;      /* views per launch in serving; 0 = 64 */
} ffv_opts;

/* Fills *opts with the defaults (FP32, device 0, library stream, graphs on,
 * 16 GiB workspace cap, serving off). */
void ffv_default_opts(ffv_opts* opts);

/*
 * Load a .ffvw weights file (layout: magic "FFVW", version 1, text header
 * with base width, t-plane flag and per-layer shapes/offsets, SHA-256 of the
 * float32 payload) and build a net for opts->precision on opts->device.
 * Weights are checked against the network definition (section 3.1 and the
 * supplementary layer table) and packed for the chosen precision.
 * Errors: FFV_ERR_ARG (null args, ABI version), FFV_ERR_WEIGHTS (file),
 * FFV_ERR_DEVICE / FFV_ERR_OOM (device).
 */
ffv_status ffv_create_net(const char* weights_path, const ffv_opts* opts, ffv_net** out);

/* Release everything the net owns. Waits for its in-flight work. NULL is a no-op. */
void ffv_destroy_net(ffv_net* net);

typedef struct {
  const float* left;   /* device, planar [3][H][W] float32 */
  const float* right;  /* device, planar [3][H][W] float32 */
  int32_t height, width;
} ffv_pair;

/*
 * Synthesise n_t virtual views for each of n_pairs camera pairs: the view at
 * phase t[j] between pair i's left (t = 0) and right (t = 1) image, per the
 * network of section 3.1 (Eq. 1, Eq. 2). All pairs share one height and
 * width (>= 2 each). Pairs that share an image pointer share its per-camera
 * work (image pyramid, context features).
 *   t:   HOST array of n_t phases, each in [0, 1].
 *   out: DEVICE float32 [n_pairs][n_t][3][H][W], caller-owned.
 * Work is ordered on opts->stream (or the library stream); the call returns
 * after the output is written. Calls on one net are serialised. With
 * opts->graphs the first call of a shape (H, W, number of distinct images,
 * number of views) captures the whole launch sequence into a hipGraph and
 * every later call of that shape replays it after writing the per-call
 * tables (image pointers, t, output pointers) to device memory; the results
 * are the same as eager launches (same kernels, same order).
 * Errors: FFV_ERR_ARG (nulls, n <= 0, mixed sizes, t outside [0,1] or NaN),
 * FFV_ERR_OOM, FFV_ERR_DEVICE.
 */
ffv_status ffv_interpolate(ffv_net* net, const ffv_pair* views, int32_t n_pairs,
                           const float* t, int32_t n_t, float* out);

/*
 * The flow-and-mask blend alone (Eq. 1: I = sigma(M) W_l + (1 - sigma(M)) W_r
 * with the coarse-to-fine flow and mask of Eq. 2): the paper's "w/o Refine"
 * variant of its ablation (Table 1), with no context features, U-Net or
 * residual. Arguments, layout and errors as ffv_interpolate.
 */
ffv_status ffv_interpolate_blend(ffv_net* net, const ffv_pair* views, int32_t n_pairs,
                                 const float* t, int32_t n_t, float* out);

/*
 * Dense views by recursive midpoints (the paper's dense-view scheme,
 * section 4, Fig. 6): level 1 synthesises the middle view of each pair, and
 * every further level the middle view of each adjacent pair of the views so
 * far, all at t = 1/2. levels = n in [1, 10] gives 2^n - 1 views per pair:
 *   out: DEVICE float32 [n_pairs][2^n - 1][3][H][W], view k-1 at t = k/2^n.
 * One batched launch sequence per level (level l holds n_pairs * 2^(l-1)
 * views); a view's two neighbours are read back from `out`. Errors as
 * ffv_interpolate, plus FFV_ERR_ARG for levels outside [1, 10].
 */
ffv_status ffv_interpolate_recursive(ffv_net* net, const ffv_pair* views, int32_t n_pairs,
                                     int32_t levels, float* out);

/*
 * Conv tile autotuning (the conv kernel is instantiated for 256-pixel M tiles
 * with 256/128/64/32-channel N tiles, halo variants with 256/128/32
 * channels, resident-weight variants with 64/32 and stride-2 resident
 * variants with 128/64/32; the 256 pixels form a tile_w-wide 2-D block). Runs the call exactly as ffv_interpolate does (same arguments, same
 * result in *out*), then re-launches each convolution of that call with
 * every candidate (N tile at most twice the real channel count rounded to
 * 32; pixel-block widths 8, 16, 32, 64 within 10 % of the least padding),
 * timed with HIP events on the net's stream, and keeps the fastest per
 * (layer, fp8 or not, output grid, images per launch). Later calls whose
 * launches match use those choices; captured graphs are dropped.
 * *n_tuned (nullable) = launch shapes tuned. Takes seconds at 1080p batch
 * sizes. Errors as ffv_interpolate.
 */
ffv_status ffv_autotune(ffv_net* net, const ffv_pair* views, int32_t n_pairs, const float* t,
                        int32_t n_t, float* out, int32_t* n_tuned);

/*
 * Tuning table as text, one line per launch shape:
 * "layer fp8 Ho Wo n_img n_tile tile_w" ('#' starts a comment line); n_tile
 * is 256, 128, 64, 32, or h256, h128, h32 for the halo variants, r64, r32
 * for the resident-weight variants, s128, s64, s32 for the few-channel ones,
 * q256 for the 2 x 4-wave halo tile, p256 for the halo tile whose two wave
 * groups alternate MFMA and memory phases.
 * ffv_save_tuning writes the net's table; ffv_load_tuning merges a file's
 * entries into it (*n_loaded, nullable, = entries read) and rejects the
 * whole file on a malformed line, an unknown layer or a tile that does not
 * fit its layer (FFV_ERR_ARG).
 */
ffv_status ffv_save_tuning(ffv_net* net, const char* path);
ffv_status ffv_load_tuning(ffv_net* net, const char* path, int32_t* n_loaded);

/* Last error message of the calling thread (valid until its next call). */
const char* ffv_last_error(void);

/*
 * FP8 nets only: run the view at phase t of `pair` once in bf16, record the
 * range of every VIBlock activation channel (|value| max), and quantise the
 * VIBlock layers that read those activations to fp8 e4m3: the producer's
 * per-channel scale (max / 448) is folded into the weights, each output
 * channel then gets its own weight scale, and activations are stored as
 * value / scale, saturated to +-448. Must be called (with representative
 * content) before ffv_interpolate or ffv_submit on an FP8 net; may be called
 * again to recalibrate. Errors: FFV_ERR_ARG, FFV_ERR_STATE (not an FP8 net),
 * FFV_ERR_OOM, FFV_ERR_DEVICE.
 */
ffv_status ffv_calibrate(ffv_net* net, const ffv_pair* pair, float t);

/* ---------------------------------------------------------------------- */
/* Serving (enabled when ffv_opts.hbm_budget_bytes > 0)                     */
/* ---------------------------------------------------------------------- */
/*
 * While serving is on, ffv_autotune, ffv_load_tuning, ffv_calibrate and
 * ffv_set_profiling pause admission and wait for the batches in flight
 * before they change the net, and resume it when done.
 *
 * Many users each ask for their own viewpoint between neighbouring cameras
 * (the paper's multi-user setting, section 2; one network evaluation per
 * view, section 3.1). Cameras are registered once; the library keeps each
 * camera's padded image, its image pyramid and its context features
 * resident in device memory, and every request reuses them. Requests are
 * admitted in FIFO order once per tick (opts.tick_ms) or when a running
 * batch finishes, into batches of at most opts.max_batch_views that span
 * at most four camera sizes (a request of a fifth size waits for a later
 * batch), while the bytes of resident cameras plus the workspaces of
 * batches in flight stay within opts.hbm_budget_bytes. A batch's workspace
 * is sized for its largest height and width, and every layer of a batch is
 * one launch over all its views whatever their sizes. Each batch runs on
 * its own stream, so batches overlap on the device. A view's result does
 * not depend on the batch it runs in.
 */

/* Copy a DEVICE planar [3][H][W] float32 image in [0,1] as camera cam_id
 * and build its resident data (synchronous). Re-registering an id with an
 * image of the same size replaces the camera after the batches in flight
 * finish (queued requests then read the new image); a different size is
 * FFV_ERR_ARG. If rebuilding a replaced camera fails, the id is
 * unregistered. Errors: FFV_ERR_ARG, FFV_ERR_BUDGET (cameras alone exceed
 * the budget), FFV_ERR_STATE (serving off), FFV_ERR_OOM, FFV_ERR_DEVICE. */
ffv_status ffv_register_camera(ffv_net* net, int32_t cam_id, const float* image, int32_t height,
                               int32_t width);

typedef struct {
  int32_t cam_left, cam_right; /* registered ids, equal sizes */
  float t;                     /* phase in [0,1]: 0 = cam_left, 1 = cam_right */
  float* out;                  /* DEVICE planar [3][H][W] float32, caller-owned,
                                  valid until ffv_poll returns FFV_OK */
  uint64_t user_tag;
} ffv_request;

typedef struct {
  double t_submit, t_admit, t_launch, t_done; /* seconds, steady clock */
} ffv_timing;

/* Queue a request (non-blocking, thread-safe). `out` must hold [3][H][W]
 * floats of the cameras' size (the library cannot check a raw pointer).
 * Errors: FFV_ERR_ARG (unknown camera, sizes differ, t outside [0,1], null
 * out), FFV_ERR_BUDGET (one view can never fit the budget), FFV_ERR_STATE
 * (serving off, or an FP8 net not yet calibrated). */
ffv_status ffv_submit(ffv_net* net, const ffv_request* req, uint64_t* ticket);

/* Queue n requests (HOST array) at once, tickets[i] for reqs[i] (HOST
 * array of n): every request is checked as in ffv_submit before any is
 * queued, so on an error none is (ffv_last_error names the first bad
 * index). The scheduler sees them together, so a burst lands in as few
 * batches as max_batch_views and the four-size limit allow. n = 0 is a
 * no-op. Thread-safe. */
ffv_status ffv_submit_many(ffv_net* net, const ffv_request* reqs, int32_t n, uint64_t* tickets);

/* FFV_PENDING while queued or running; FFV_OK once the output is written
 * (fills *timing if non-NULL; the ticket is then collected). If the
 * request's batch failed, the batch's error: FFV_ERR_DEVICE (a launch could
 * not be queued) or FFV_ERR_OOM (no workspace could be allocated while
 * nothing else was running); the output is then undefined and the ticket
 * is collected. FFV_ERR_TICKET for unknown or collected tickets.
 * Thread-safe. */
ffv_status ffv_poll(ffv_net* net, uint64_t ticket, ffv_timing* timing);

/* Requests admitted and completed so far, requests queued now, and device
 * bytes held by resident cameras plus batch workspaces. */
ffv_status ffv_serving_stats(ffv_net* net, int64_t* admitted, int64_t* completed, int64_t* queued,
                             uint64_t* bytes_in_use);

/* ---------------------------------------------------------------------- */
/* Instrumentation (used by tests and the benchmark)                       */
/* ---------------------------------------------------------------------- */

/*
 * Copy an intermediate tensor of view 0 of the last ffv_interpolate call to
 * the DEVICE buffer dst as float32 [C][Hs][Ws] (C, Hs, Ws written to dims),
 * at the padded size (multiples of 16) and its 2^-k levels. Names:
 *   "F0" "F1" "F2"  flow + mask logit of Eq. 2 (5 channels) at stage s
 *   "I2"            the Eq. 1 blend (3 channels)
 *   "x0"            the refinement U-Net's input [X_l, X_r, W_l, W_r, M, F]
 *   "d1".."d4"      U-Net encoder outputs (B, 2B, 4B, 8B channels at 2^-k)
 *   "u1".."u4"      U-Net decoder outputs (4B, 2B, B, B/2 channels at 2^(k-4))
 *   "cl1".."cl4", "cr1".."cr4"    context features of the left / right view
 *   "wcl1".."wcl4", "wcr1".."wcr4" the same, warped to the virtual view
 * (section 3.1, "Refinement Network"). The U-Net names describe the last
 * chunk of views, which holds view 0 when debug taps are on.
 * Only available when the net was created with debug taps enabled
 * (ffv_set_debug). Errors: FFV_ERR_ARG (unknown name, capacity too small),
 * FFV_ERR_STATE (no taps recorded).
 */
ffv_status ffv_debug_tap(ffv_net* net, const char* name, float* dst, size_t capacity_floats,
                         int32_t dims[3]);
ffv_status ffv_set_debug(ffv_net* net, int32_t enable);

/*
 * Per-kernel-class timing with HIP events recorded on the work stream.
 * ffv_set_profiling(net, 1) clears and starts collection; ffv_kernel_stats
 * returns, for the class named `name`, the number of launches, the summed
 * device time in milliseconds and the summed algorithmic work (flops for
 * convolution classes, bytes for per-pixel classes). Class names:
 * "conv256" (3x3 stride-1 convs with 256 in/out channels), "conv" (other
 * convolutions), "convT" (transposed convs), "pixel" (warp/resample/blend
 * passes), "head" (output head).
 */
ffv_status ffv_set_profiling(ffv_net* net, int32_t enable);
ffv_status ffv_kernel_stats(ffv_net* net, const char* name, int64_t* launches, double* ms,
                            double* work);

/*
 * Fault injection for tests of the error paths: the N-th device allocation
 * ("alloc:N") or the N-th serving batch launch ("launch:N") after this call
 * fails with FFV_ERR_OOM / FFV_ERR_DEVICE before any device work is issued
 * for it; entries may be joined with ','. NULL or "" disarms. The
 * environment variable FFV_FAULT sets the same spec for a whole process
 * (read once, unless this call came first).
 */
ffv_status ffv_debug_fault(const char* spec);

/*
 * Multi-view cluster frame (the Multiview Organizer of section 3.2; the
 * supplement's clusters of 16 views per side, 33 views in all): the real
 * view of a camera at full resolution between two blocks of its
 * neighbouring views, each downscaled by g = sqrt(n_per_side) in both
 * directions (g x g box mean) and tiled g x g in raster order, so each side
 * fills one H x W block:
 *   out[3][H][3W] = [left block | real view | right block]
 * real_view: DEVICE planar [3][H][W]; left, right: HOST arrays of
 * n_per_side DEVICE planar [3][H][W] views (left: far to near, right: near
 * to far); out: DEVICE planar [3][H][3W]. n_per_side in {1, 4, 16, 64};
 * H and W multiples of g; views 16-byte aligned when g = 4. Enqueued on
 * `stream` (NULL = default stream), asynchronous. Errors: FFV_ERR_ARG,
 * FFV_ERR_DEVICE.
 */
ffv_status ffv_stitch_cluster(const float* real_view, const float* const* left,
                              const float* const* right, int32_t n_per_side, int32_t height,
                              int32_t width, float* out, void* stream);

/* Flag for ffv_op_conv's precision argument (see there). */
#define FFV_OP_ACT_OUT 0x100

/*
 * One convolution layer through the library's implicit-GEMM kernel (kernel
 * unit tests). 3x3 conv, padding 1, stride 1 or 2 (transposed = 0), or 4x4
 * stride-2 padding-1 transposed conv (transposed = 1); optional ReLU.
 *   x:      DEVICE float32 planar [n][cin][h][w]
 *   weight: HOST float32, [cout][cin][3][3] (conv) or [cin][cout][4][4] (transposed)
 *   bias:   HOST float32 [cout]
 *   y:      DEVICE float32 planar [n][cout][ho][wo], ho = (h-1)/stride+1
 *           (conv) or 2h (transposed)
 * precision: FFV_FP32 or FFV_BF16 (inputs and weights rounded to bf16, fp32
 * accumulation and output), optionally or'ed with FFV_OP_ACT_OUT: the layer
 * writes its output in the activation dtype (bf16 for FFV_BF16), as the
 * network's layers do, and y receives those values widened to float32. n_tile (0 = the layer's default, else 256, 128,
 * 64 or 32 output channels per workgroup, or 1 = the halo-reuse kernel:
 * 32 channels of a 16x16 pixel block, for stride-1 convs whose input
 * channels are a multiple of the K step; 2 and 3 = the 128- and 256-channel
 * tiles reading each channel slice's input halo once, for stride-1 and
 * transposed convs whose input channels are a multiple of the K step, with
 * tile_w 8, 16 or 32; 4 and 5 = the persistent kernel with the layer's
 * weights resident in LDS, 32 or 64 GEMM columns, for stride-1 and
 * phase-merged transposed convs with few output channels; 6, 7, 8 = the
 * persistent stride-2 kernel for 8 to 32 input channels with 32, 64 or 128
 * columns, weights resident, bf16 outputs in 16-byte channel runs only; 9 =
 * the 256-column halo tile with 2 x 4 waves (all four phases of a
 * transposed conv with at most 64 outputs in one workgroup); 10 = the
 * 256-column halo tile (as 3) with its eight waves in two groups whose
 * MFMA and memory phases alternate; a variant that
 * cannot run the layer gives FFV_ERR_DEVICE) and tile_w (0 =
 * default, else the
 * width of the 256-pixel block of a workgroup, a divisor of 256) pick the
 * kernel variant, as autotuning does; every choice gives the same result.
 * Allocates temporaries; synchronises `stream`.
 */
ffv_status ffv_op_conv(int32_t precision, const float* x, int32_t n, int32_t cin, int32_t h,
                       int32_t w, const float* weight, const float* bias, int32_t cout,
                       int32_t stride, int32_t transposed, int32_t relu, int32_t n_tile,
                       int32_t tile_w, float* y, void* stream);

/*
 * Laplacian-pyramid colour loss of the training objective (section 3.1,
 * "Loss functions", Eq. 3) and, optionally, its gradient with respect to the
 * synthesised images:
 *   loss[i] = sum_{k=1..5} 2^(k-1) * mean |L^k(x_i) - L^k(gt_i)|
 * where L^k is the k-th band-pass level of a Laplacian pyramid. The paper
 * does not define the pyramid; the library's reading: the separable
 * binomial filter [1, 4, 6, 4, 1] / 16 with mirror padding (edge sample not
 * repeated), reduce = even samples of the blurred level, expand = the
 * zero-inserted coarser level blurred with gain 2 per axis, band
 * L^k = G^k - expand(G^(k+1)) (the low-pass residual is not a term), and the
 * mean taken over all 3 * h_k * w_k values of a level.
 *   x, gt: DEVICE float32 planar [n][3][H][W] (synthesised view, ground truth)
 *   loss:  DEVICE float32 [n]
 *   grad:  DEVICE float32 [n][3][H][W] = d loss[i] / d x_i, or NULL; at a
 *          sample where a band is exactly 0 the sign is taken as 0
 * H, W >= 33 (five levels of mirror padding need 3 samples at the coarsest).
 * Allocates its workspace, orders its work on `stream` (NULL = default
 * stream) and synchronises it. Per-workgroup sums are combined in a fixed
 * order in double precision, so repeated calls give identical results.
 * Errors: FFV_ERR_ARG, FFV_ERR_OOM, FFV_ERR_DEVICE.
 */
ffv_status ffv_lap_loss(const float* x, const float* gt, int32_t n, int32_t height, int32_t width,
                        float* loss, float* grad, void* stream);

/* Bytes of the per-device scratch array behind ffv_op_conv_noalloc. */
#define FFV_OP_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * ffv_op_conv without device allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc). Arguments, layout, result and errors are those of
 * ffv_op_conv, and it runs the same kernels, so the two give the same
 * values bit for bit. Its device buffers (NHWC input copy, packed weights,
 * bias, NHWC output, zero block, each rounded up to 256 bytes) live in one
 * array of FFV_OP_NOALLOC_SCRATCH_BYTES per device, which the library holds
 * from the first call on that device until the process ends. A layer whose
 * buffers do not fit is rejected with FFV_ERR_ARG before any device work.
 * The call works on the current device, orders its work on `stream`
 * (NULL = default stream) and synchronises it before returning. Every call
 * on a device shares that device's array, so calls that overlap in time on
 * one device (other host threads, other streams) race; callers serialise
 * them.
 */
ffv_status ffv_op_conv_noalloc(int32_t precision, const float* x, int32_t n, int32_t cin,
                               int32_t h, int32_t w, const float* weight, const float* bias,
                               int32_t cout, int32_t stride, int32_t transposed, int32_t relu,
                               int32_t n_tile, int32_t tile_w, float* y, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FFV_H */
