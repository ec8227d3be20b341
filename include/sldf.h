/*
 * sldf.h -- C ABI of the MI355X (gfx950) stereo-LiDAR depth-fusion library
 * libsldf.so.
 *
 * The library computes, per frame, the method of "Stereo-LiDAR Fusion by
 * Semi-Global Matching with Discrete Disparity-Matching Cost and
 * Semidensification" (Yao, Ishikawa, Oishi, IEEE RA-L 2025):
 *   inputs   a rectified uint8 stereo pair (left image = base) and a sparse
 *            LiDAR disparity map D-bar aligned with the left image
 *            (Sec. IV, definition of D-bar: values in N or "invalid");
 *   steps    semidensification (Sec. IV-B, Eq. 5; SDSGM variant only),
 *            census Hamming cost + discrete disparity-matching cost
 *            (Sec. IV-A, Eq. 4), multi-path SGM aggregation (Sec. III,
 *            Eq. 2), winner-takes-all (Eq. 3) with parabola subpixel fit,
 *            the right-view SGM pass and the stereo-LiDAR consistency check
 *            (Sec. IV-C, Eq. 6);
 *   output   a dense float32 disparity map with invalid pixels (-1.0f) and a
 *            uint8 validity mask (the consistent map D^{c*} of Eq. 6).
 *
 * Conventions
 *   - Every function returns an sldf_status and never aborts or throws.
 *   - "device" pointers are HIP device memory on the device that was current
 *     when the context was created; "host" pointers are ordinary memory.
 *   - Pitches are in ELEMENTS of the array's own type (bytes for uint8).
 *   - All GPU work is enqueued on the caller's HIP stream (hipStream_t passed
 *     as void*; NULL = the null stream).  No call synchronises the host and
 *     no call allocates device memory after sldf_create: the workspace is
 *     caller-owned and sldf_workspace_size() is the exact HBM cost.
 *   - A context may be used by one stream at a time; separate contexts may run
 *     concurrently on separate streams.
 *
 * Readings of the paper fixed by this ABI (the CPU oracle uses the same):
 *   alpha = alpha_num / alpha_den is applied exactly by scaling every cost
 *   term by alpha_den: C' = (den - num) H + num DDC, P1' = den P1,
 *   P2' = den P2 (argmin and subpixel offset are scale invariant); census
 *   is the centre-symmetric census with bit k = [I(p+o_k) > I(p-o_k)] over
 *   the raster-order first half of the window, 0 where the window leaves the
 *   image; the Hamming cost is n (all bits) where the matching pixel leaves
 *   the image; ties in WTA and semidensification go to the smallest d; the
 *   right-view disparity d' is a full right-base SGM without prior; the
 *   check uses the integer d* and the raw LiDAR map.
 */
#ifndef SLDF_H
#define SLDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SLDF_ABI_VERSION 1

typedef enum {
    SLDF_OK = 0,
    SLDF_EINVAL = -1,    /* invalid argument or parameter value */
    SLDF_ESHAPE = -2,    /* width / height / disparity range out of range */
    SLDF_EALIGN = -3,    /* pointer or pitch alignment violated */
    SLDF_EOVERFLOW = -4, /* parameters could overflow the 16-bit cost sums */
    SLDF_ENOMEM = -5,    /* workspace too small / host allocation failed */
    SLDF_EDEVICE = -6,   /* a HIP call or kernel launch failed */
    SLDF_ESTATE = -7     /* context used in a state that does not allow it */
} sldf_status;

/* Method parameters.  Tab. II values are the defaults (sldf_params_default). */
typedef struct {
    int32_t struct_size;   /* sizeof(sldf_params): ABI check */
    int32_t width;         /* W, 16 <= W <= 4096 */
    int32_t height;        /* H, 16 <= H <= 4096 */
    int32_t max_disp;      /* D, disparities 0..D-1; D in {64, 128, 256};
                              W * H * D <= 2^31 (one frame's cost volume is
                              addressed with 32-bit byte offsets) */
    int32_t census_w;      /* odd census window width  (<= 15) */
    int32_t census_h;      /* odd census window height (<= 15); at most 32
                              code bits (see census_kind) */
    int32_t num_paths;     /* 4 (horizontal + vertical) or 8 (+ diagonals),
                              Sec. III; 1 = left-to-right only (debug) */
    int32_t p1, p2;        /* SGM penalties, Eq. 1-2 (Tab. II: 10, 120) */
    int32_t q1, q2;        /* DDC penalties, Eq. 4 (Tab. II: 5, 160), q1 <= q2 */
    int32_t alpha_num;     /* alpha = alpha_num / alpha_den (Tab. II: 7/10) */
    int32_t alpha_den;
    int32_t blend_mode;    /* 0: Eq. 4 at every pixel, DDC = 0 without prior
                              (cost (1-alpha) H); 1: cost H at full weight
                              where there is no prior */
    int32_t semidense;     /* 0 = DSGM, 1 = SDSGM (Tab. I) */
    int32_t ts, rs;        /* semidensification threshold / window radius,
                              Eq. 5 (Tab. II: 2, 6); 0 <= rs <= 15 */
    int32_t tc, rc;        /* consistency threshold / window radius, Eq. 6
                              (Tab. II: 2, 20); 0 <= rc <= 31 */
    int32_t check_mode;    /* 0 none, 1 stereo only, 2 LiDAR only,
                              3 stereo OR LiDAR (Eq. 6; Tab. V variants) */
    int32_t check_impl;    /* 0: plain check with the right-view SGM pass;
                              1: learned check (needs check_mode 3 and weights,
                              see sldf_surrogate_set_weights): a small CNN on
                              left-view cost features replaces the stereo
                              half of Eq. 6, the right-view pass is skipped
                              unless the fallback triggers */
    int32_t subpixel;      /* 1: parabola fit (Sec. III end), 0: integer */
    int32_t batch;         /* max frames per sldf_run_batch call (>= 1) */
    float fallback_tau;    /* learned check: when more than tau * W * H pixels
                              of a frame are undecided by LiDAR and have
                              |logit| < uncertain_margin, that frame falls
                              back to the plain check (decided on the device,
                              no host synchronisation); in [0, 1] */
    float uncertain_margin;  /* >= 0 */
    int32_t prior_cost;    /* LiDAR term of the joint cost: 0 = DDC (Eq. 4,
                              the paper's method); the terms it is compared
                              with (Sec. IV-A, V-B), capped at q2 so that the
                              16-bit bound holds: 1 = quadratic
                              min(q1 t^2, q2), 2 = Huber min(q1 h_k(t), q2)
                              with h_k(t) = t^2 (t <= k), k (2t - k) beyond;
                              t = |d - prior| */
    int32_t huber_k;       /* Huber threshold k >= 1 (prior_cost 2) */
    int32_t schedule;      /* order of the path passes (results identical):
                              0 = automatic (two sweeps for runs of 16 or
                              more frames, split for single frames, paired
                              otherwise);
                              1 = paired: both directions of a pair on one
                              line, S read and written once per pair;
                              2 = split: the two directions of a pair as
                              separate lines into two cost terms, then one WTA
                              pass (shortest critical path, more S traffic;
                              runs of more than one frame fall back to paired);
                              3 = two sweeps: rows walk the image top to
                              bottom with four directions (S written once),
                              then bottom to top with the other four and the
                              WTA (S read once); rows are handed from one
                              band of rows to the next through a workspace
                              buffer.  Single-frame contexts (batch 1) with
                              8 paths and schedule 0 or 2 run the split
                              schedule on two streams: the caller's and one
                              the context creates (default priority),
                              forked from and joined back into the caller's
                              stream with events, so a call stays ordered
                              on the caller's stream and can be captured
                              into a graph */
    int32_t census_kind;   /* census of the matching cost (Sec. IV-A):
                              0 = centre-symmetric census (default): bit k =
                              [I(p + o_k) > I(p - o_k)] over the first
                              (w h - 1) / 2 window offsets in raster order;
                              1 = full census: bit k = [I(p + o_k) < I(p)]
                              over every offset but the centre in raster
                              order, w h - 1 bits, which must be <= 32
                              (e.g. 5 x 5: 24 bits; 9 x 7 is refused) */
} sldf_params;

/* Optional debug taps: device pointers, any may be NULL.  Written for frame
   0 of each run.  Dense layouts, row pitch = width:
     census_l, census_r  uint32 [H][W]
     prior               int16  [H][W]   D-hat (SDSGM) or D-bar (DSGM)
     cost_sum            uint16 [H][W][D] aggregated left cost S (Eq. 3 sum)
     dstar               int16  [H][W]   integer left disparity d*
     dright              int16  [H][W]   right-view disparity d'
     dsub                float  [H][W]   subpixel d* before the check
     rho                 uint16 [H][W]   LiDAR residual: min |d* - v| over the
                                         valid raw sparse values v in the check
                                         window (65535 = none); the LiDAR half
                                         of Eq. 6 is rho <= Tc
     features            uint16 [H][W][8] bf16 inputs of the learned check:
                                         S(d*), second minimum of S over
                                         |d - d*| >= 2, curvature
                                         S(d*-1) - 2 S(d*) + S(d*+1), each times
                                         1 / (num_paths P2'); d* / D;
                                         min(rho, 32) / 32; three zeros
     sweep_errors        int32  [1]      two-sweep schedule: nonzero if a wait
                                         for the row band above timed out (the
                                         results are then not valid); written
                                         by every run of that schedule
     cost                uint16 [H][W][D] joint cost C'(p, d) of the left view
                                         (Eq. 4 scaled by alpha_den: (den - num)
                                         H + num DDC), which the path passes
                                         otherwise never store
     path_cost           uint16 [H][W][D] L_r(p, d) of the left view for the one
                                         direction path_dir (Eq. 2): 0 (+1, 0),
                                         1 (-1, 0), 2 (0, +1), 3 (0, -1),
                                         4 (+1, +1), 5 (-1, +1), 6 (+1, -1),
                                         7 (-1, -1), as steps (dx, dy) from a
                                         pixel's predecessor
     path_dir            the direction of path_cost (0..7) */
typedef struct {
    uint32_t* census_l;
    uint32_t* census_r;
    int16_t* prior;
    uint16_t* cost_sum;
    int16_t* dstar;
    int16_t* dright;
    float* dsub;
    uint16_t* rho;
    uint16_t* features;
    int32_t* sweep_errors;
    uint16_t* cost;
    uint16_t* path_cost;
    int32_t path_dir;
} sldf_taps;

typedef struct sldf_ctx sldf_ctx;

/* Human-readable name of a status code (static string, never NULL). */
const char* sldf_status_string(sldf_status s);

/* ABI version of the loaded library (SLDF_ABI_VERSION). */
int32_t sldf_abi_version(void);

/* Fill *p with Tab. II parameters for a 1242x375, D=128, 9x7 census, 8-path
   SDSGM frame with the stereo-LiDAR check.  p must be non-NULL. */
void sldf_params_default(sldf_params* p);

/* Validate p (shape ranges, odd census window, D, num_paths, q1 <= q2,
   alpha in [0, 1], the 16-bit bound
     num_paths * (C'max + P2') < 65536 and C'max + P2' + max(P1', P2') <
     0x7c00 (the recurrence compares its terms as fp16 bit patterns),
   with C'max the largest joint cost) and return the exact device workspace
   size for p->batch frames in *bytes.  Host only.
   Errors: EINVAL, ESHAPE, EOVERFLOW. */
sldf_status sldf_workspace_size(const sldf_params* p, size_t* bytes);

/* Create a context on the current HIP device.  dev_workspace: caller-owned
   device buffer of at least sldf_workspace_size() bytes, 256-byte aligned,
   which must outlive the context.  *out receives a host-allocated handle.
   Single-frame contexts (batch 1) with 8 paths and schedule 0 or 2 also
   create a HIP stream (default priority, non-blocking) and two events for
   the two-stream schedule; sldf_destroy releases them.
   Errors: as sldf_workspace_size, EALIGN (workspace), ENOMEM (ws_bytes too
   small or host allocation failed), EDEVICE (no HIP device, or the stream or
   events could not be created). */
sldf_status sldf_create(const sldf_params* p, void* dev_workspace, size_t ws_bytes,
                        sldf_ctx** out);

/* Release the handle (not the workspace) and the stream and events the
   context created (after waiting for the work on that stream).  NULL is
   accepted.  The caller must have synchronised the stream of the last run
   first. */
sldf_status sldf_destroy(sldf_ctx* ctx);

/* Set the debug taps written by subsequent runs (copied; NULL clears).
   Errors: EINVAL (path_cost with path_dir outside 0..7). */
sldf_status sldf_set_taps(sldf_ctx* ctx, const sldf_taps* taps);

/* Process one frame (the whole method, Fig. 1 flow).  All pointers device:
     left, right  uint8 [H][img_pitch], 16-byte aligned, img_pitch % 16 == 0
     lidar        int16 [H][lidar_pitch], lidar_pitch >= W, D-bar:
                  0..D-1 or -1 (= invalid), as written by sldf_lidar_quantize;
                  other values are outside the contract (memory-safe, result
                  unspecified)
     disp_out     float [H][out_pitch]: subpixel disparity, -1.0f if invalid
     valid_out    uint8 [H][out_pitch]: 1 = consistent (Eq. 6), 0 = invalid
   Enqueue-only on hip_stream.  Errors: EINVAL (NULL pointer / pitch < W),
   EALIGN, EDEVICE (launch failure). */
sldf_status sldf_run(sldf_ctx* ctx, const uint8_t* left, const uint8_t* right,
                     int32_t img_pitch, const int16_t* lidar, int32_t lidar_pitch,
                     float* disp_out, uint8_t* valid_out, int32_t out_pitch,
                     void* hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid allocation): sldf_run without a
   context or a caller workspace.  The workspace is a static device array of
   SLDF_NOALLOC_SCRATCH_BYTES per GPU, held by the library until the process
   ends and shared by every call on that GPU: calls that overlap on one GPU
   (several streams or threads) race and must be serialised by the caller.
   One frame, plain check only (params->check_impl 0; batch is taken as 1),
   run on the caller's stream with the paired schedule (schedule 0 and 2 run
   as 1, 3 stays; results are the same for every schedule).  Pointers and
   layouts as for sldf_run.  No hipMalloc / hipFree or other allocation.
   Errors: as sldf_workspace_size and sldf_run; EINVAL (check_impl != 0);
   ENOMEM when the frame's workspace (sldf_workspace_size with batch 1 and
   that schedule) exceeds SLDF_NOALLOC_SCRATCH_BYTES: 320 x 96 and 640 x 480
   at D = 64 fit, 1242 x 375 at D = 128 does not. */
#define SLDF_NOALLOC_SCRATCH_BYTES (128u << 20)
sldf_status sldf_run_noalloc(const sldf_params* params, const uint8_t* left,
                             const uint8_t* right, int32_t img_pitch, const int16_t* lidar,
                             int32_t lidar_pitch, float* disp_out, uint8_t* valid_out,
                             int32_t out_pitch, void* hip_stream);

/* Process n_frames (1 <= n_frames <= p.batch) frames of the context's shape
   in one pass; frame i of each array starts at base + i * (its frame stride,
   in elements; image strides must keep 16-byte alignment).  Same layouts and
   errors as sldf_run. */
sldf_status sldf_run_batch(sldf_ctx* ctx, int32_t n_frames, const uint8_t* left,
                           const uint8_t* right, int32_t img_pitch,
                           int64_t img_frame_stride, const int16_t* lidar,
                           int32_t lidar_pitch, int64_t lidar_frame_stride,
                           float* disp_out, uint8_t* valid_out, int32_t out_pitch,
                           int64_t out_frame_stride, void* hip_stream);

/* Ingest: quantise projected LiDAR disparities to D-bar on the device.
   in float [H][in_pitch] (NaN or negative = no return), out int16
   [H][out_pitch]: round to nearest, ties to even; NaN, negative and values
   rounding to >= max_disp become -1.  Errors: EINVAL, EDEVICE. */
sldf_status sldf_lidar_quantize(const float* in, int32_t width, int32_t height,
                                int32_t in_pitch, int32_t max_disp, int16_t* out,
                                int32_t out_pitch, void* hip_stream);

/* Stage timing with HIP events recorded on the run's stream (for roofline
   measurements inside a timed region).  sldf_timing_enable(ctx, n) creates
   events for up to n runs (host-side HIP events, no device memory) and
   starts recording; n = 0 stops and frees them.  Stages:
     0 census, 1 semidensification, 2 SGM path passes (all directions, both
     views; left view only for the learned check), 3 check, 4 fallback.
   sldf_timing_read waits for the recorded events, writes the summed
   milliseconds per stage into ms[5] and the number of SGM-pass / other
   kernel launches per stage into launches[5] (host arrays), and resets
   the counters.
   Errors: EINVAL, ESTATE (not enabled / more runs than events), EDEVICE.
   Stage 3 holds the LiDAR window pass and the plain check, or the CNN and
   the learned mask; stage 4 the gated fallback (right-view SGM + plain
   check) of the learned check (empty for the plain check). */
#define SLDF_NUM_STAGES 5
sldf_status sldf_timing_enable(sldf_ctx* ctx, int32_t max_runs);
sldf_status sldf_timing_read(sldf_ctx* ctx, double* ms, int64_t* launches);

/* ---- Learned consistency check (an extension beside the paper's method;
   the plain check of Eq. 6 stays the reference and the fallback) ----
   Network: 3x3 convolutions with dilations 1, 3, 9, 27 (an 81 x 81 receptive
   field covered without gaps); channels
   6 (+2 zero) -> 32 -> 32 -> 32 -> 1; ReLU after the first three; bf16
   weights and activations, fp32 accumulation; logit > 0 means "consistent".
   Parameter blob (device, caller-owned, may be shared by contexts):
     weights: bf16 (uint16 bit patterns), sldf_surrogate_num_weights() of
              them: layer l stored as [9 taps][out][in] with taps in raster
              order of the 3x3 grid and (out, in) = (32, 8), (32, 32),
              (32, 32), (16, 32) (padding rows / columns zero);
     biases:  float, 32 + 32 + 32 + 1. */
int32_t sldf_surrogate_num_weights(void);
int32_t sldf_surrogate_num_biases(void);

/* Attach the surrogate parameters used when check_impl = 1 (pointers are
   kept, not copied; NULL detaches).  Errors: EINVAL. */
sldf_status sldf_surrogate_set_weights(sldf_ctx* ctx, const uint16_t* weights,
                                       const float* biases);

/* The same from one device blob of sldf_surrogate_blob_bytes() bytes: the
   bf16 weights, zero padding to a 256-byte boundary, then the float biases.
   The blob is referenced, not copied (caller-owned; it may be shared by
   contexts).  Errors: EINVAL (null ctx or blob, bytes other than
   sldf_surrogate_blob_bytes(), blob not 256-byte aligned). */
size_t sldf_surrogate_blob_bytes(void);
sldf_status sldf_surrogate_load(sldf_ctx* ctx, const void* blob, size_t bytes);

/* Monitoring (host-synchronous: call after the stream of the last run has
   completed): copies the per-frame count of uncertain pixels of the last
   learned-check run into counts[n] (host) and the fallback limit
   (tau * W * H) into *limit; frame f fell back iff counts[f] > *limit.
   Errors: EINVAL, ESTATE (context without the learned check), EDEVICE. */
sldf_status sldf_fallback_read(sldf_ctx* ctx, int32_t* counts, int32_t n, int32_t* limit);

/* Forward pass on given inputs (device): x0 bf16 [F][H][W][8] (the
   `features` tap layout) -> logits float [F][H][W]; act1..act3 bf16
   [F][H][W][32] receive the hidden activations (all three required).
   Errors: EINVAL, EDEVICE. */
sldf_status sldf_surrogate_forward(const uint16_t* x0, int32_t width, int32_t height,
                                   int32_t n_frames, const uint16_t* weights,
                                   const float* biases, uint16_t* act1, uint16_t* act2,
                                   uint16_t* act3, float* logits, void* hip_stream);

/* Working parameters from fp32 master parameters (device, num_weights +
   num_biases floats, weights first): weights <- bf16 of the master weights
   (round to nearest even), biases <- the master biases.  Enqueue-only.
   Errors: EINVAL, EDEVICE. */
sldf_status sldf_surrogate_sync_weights(const float* master, uint16_t* weights, float* biases,
                                        void* hip_stream);

/* Device workspace bytes of sldf_surrogate_train_step for F frames. */
sldf_status sldf_surrogate_train_workspace_size(int32_t width, int32_t height,
                                                int32_t n_frames, size_t* bytes);

/* One training step on F frames (all device pointers): forward, binary
   cross-entropy on the pixels the LiDAR test leaves undecided (rho > tc)
   against labels (the plain check's mask, uint8 [F][H][W]), backward
   (dgrad + wgrad on the matrix cores, deterministic reductions) and, when
   apply_update != 0, one Adam step (bias-corrected, step >= 1) on the fp32
   master parameters (master, adam_m, adam_v: num_weights + num_biases
   floats, weights first), rewriting weights (bf16) and biases in place.
   grads_out (optional, same layout as master) receives the gradient;
   stats_out (optional, 3 floats) the mean loss, the number of undecided
   pixels and the number of pixels whose learned mask equals the label.
   Errors: EINVAL, ENOMEM (workspace too small), EDEVICE. */
sldf_status sldf_surrogate_train_step(const uint16_t* x0, const uint8_t* labels,
                                      const uint16_t* rho, int32_t tc, int32_t width,
                                      int32_t height, int32_t n_frames, float* master,
                                      float* adam_m, float* adam_v, uint16_t* weights,
                                      float* biases, float lr, float beta1, float beta2,
                                      float eps, int32_t step, int32_t apply_update,
                                      void* workspace, size_t ws_bytes, float* grads_out,
                                      float* stats_out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SLDF_H */
