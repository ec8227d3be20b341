// Internal declarations shared by the HIP sources of libsldf.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sldf {

// Workspace segments of one context (segment-major: every segment holds all
// batch frames back to back with the stated frame stride, in elements).
// Census rows are padded by D codes on both sides so that every matching
// pixel x -+ d of a disparity range lies inside the allocation, and one guard
// row lies before frame 0 and after the last frame (rows -1 and H of every
// frame are inside the allocation); census_l and census_r point at pixel
// (0, 0) of frame 0 (pad included before it) and pixel (x, y) of frame f sits
// at f * census_fstride + y * census_pitch + x.  Pads and guard rows are
// never written: the passes read them only where the cost is masked.
struct Buffers {
    uint32_t* census_l;
    uint32_t* census_r;
    int32_t census_pitch;     // W + 2 D
    int64_t census_fstride;   // H * census_pitch
    // prior words of the joint cost (see prior_word): the left view's per
    // frame, [F][H + 2][W + 2] from D-hat (SDSGM) or D-bar (DSGM), and one
    // [H + 2][W + 2] map shared by all frames of the right view (no prior);
    // each points at the guard corner (-1, -1) of frame 0
    uint32_t* pword[2];
    int32_t pword_pitch;      // W + 2
    int64_t pword_fstride;    // (H + 2) * (W + 2), left view
    int16_t* dstar;       // [F][H][W]
    int16_t* dright;      // [F][H][W]
    float* dsub;          // [F][H][W]
    uint16_t* S_left;     // [F][H][W][D]
    uint16_t* S_right;    // [F][H][W][D] (only when the stereo check is on)
    uint16_t* S2[2];      // split schedule (single frames): second cost term per view,
                          // [min(F, kSplitFrames)][H][W][D]
    uint16_t* S3[2];      // split schedule, 8 paths: the cost term of the pairs run on the
                          // second stream, [min(F, kSplitFrames)][H][W][D]
    uint32_t* ckpt;       // paired-pass checkpoints, [F * views][lines][segs][D / 2] u32
    uint32_t* ckpt2;      // checkpoints of the pairs on the second stream (split schedule)
    uint32_t* wmask;      // LiDAR window masks computed on the second stream (split
                          // schedule), [min(F, kSplitFrames)][H][W][D / 32]
    uint32_t* rowbits;    // [F][H][W][D / 32] LiDAR row-window masks
    uint16_t* rho;        // [F][H][W] LiDAR residual
    uint32_t* feat;       // [F][H][W][2] surrogate cost features
    uint16_t* x0;         // [F][H][W][8] bf16 surrogate inputs
    uint16_t* act[2];     // [F][H][W][32] bf16 CNN activations (learned check)
    float* logits;        // [F][H][W] (learned check)
    int32_t* counter;     // [F] uncertain pixels per frame (learned check)
    uint32_t* hand;       // two-sweep schedule: row-band handoff, [F * 2][bands - 1][W][chunks]
    int32_t* sync;        // two-sweep schedule: ticket, done, error words
    size_t hand_bytes;
    int64_t px_stride;    // W * H
    int64_t S_stride;     // W * H * D
};

struct CensusArgs {
    const uint8_t* left;
    const uint8_t* right;
    int32_t pitch;
    int64_t img_fstride;
    uint32_t* out_l;
    uint32_t* out_r;
    int32_t out_pitch;
    int64_t out_fstride;
    int32_t W, H, cw, ch;
    int32_t kind;            // 0 centre-symmetric census, 1 full census
};

// Prior word of a pixel: what the path passes need of the prior e_p of the
// joint cost (Eq. 4), precomputed once per pixel so that a step does not
// derive it per lane.  Bits 0-15: the census weight of the pixel's cost,
// (den - num) with a prior, (den - num) or den (blend mode 1) without, and 0
// on the guard ring around each map (the virtual positions before a line
// start read the ring and get cost 0).  Bits 16-31: byte offset, in the LDS
// prior-term table (build_pattern), of the first of the four packed entries
// lane 0 (disparities 0..7) reads; lane g reads 16 g bytes further.  The
// table holds P[k] = num * q(|k - D|) for k in [0, 2 D + 16) as pairs
// (P[2 i], P[2 i + 1]) at word i and pairs (P[2 i + 1], P[2 i + 2]) at word
// D + 8 + i, then a run of D / 2 zero words for pixels without prior.
__host__ __device__ constexpr int pattern_words(int D) { return 2 * (D + 8) + D / 2; }
__host__ __device__ inline uint32_t prior_word(int e, int D, uint32_t w_prior,
                                               uint32_t w_noprior)
{
    // lane 0, disparity 0: entry k = 0 - e + D; odd entries sit in the second half
    if ((unsigned)e >= (unsigned)D) return ((uint32_t)(2 * (D + 8)) * 4u << 16) | w_noprior;
    const int k = D - e;
    const uint32_t word = (uint32_t)(k >> 1) + ((k & 1) ? (uint32_t)(D + 8) : 0u);
    return (word * 4u << 16) | w_prior;
}
__host__ __device__ constexpr uint32_t guard_word(int D)
{
    return (uint32_t)(2 * (D + 8)) * 4u << 16;
}

// Destination of the prior words of the left view (and the debug tap of
// the prior disparities of frame 0).
struct PriorOut {
    uint32_t* words;            // guard corner (-1, -1) of frame 0
    int32_t pitch;              // W + 2
    int64_t fstride;
    uint32_t w_prior, w_noprior;
    int16_t* tap;               // [H][W] e_p of frame 0, or null
};

struct SemiArgs {
    const uint32_t* census_l;
    const uint32_t* census_r;
    int32_t census_pitch;
    int64_t census_fstride;
    const int16_t* lidar;
    int32_t lidar_pitch;
    int64_t lidar_fstride;
    PriorOut out;
    int32_t W, H, D, n, ts, rs;
};

struct SgmArgs {
    const uint32_t* cbase[2];   // base-view census per view (left, right)
    const uint32_t* cmatch[2];  // matching-view census per view
    int32_t census_pitch;
    int64_t census_fstride;
    const uint32_t* pword[2];   // prior words per view, guard corner of frame 0
    int32_t pword_pitch;
    int64_t pword_fstride[2];   // the right view's map is shared (stride 0)
    uint16_t* S[2];             // aggregated cost per view
    uint16_t* S2[2];            // split schedule: the term of the opposite directions
    int16_t* wta[2];            // integer WTA output per view (d*, d')
    float* dsub;                // left-view subpixel output
    int64_t px_stride;
    int64_t S_stride;
    int32_t W, H;
    int32_t n;                  // census bits (cost where the match leaves)
    int32_t dx, dy;             // path step r
    int32_t nlines;
    uint32_t q1s, q2s;          // num * Q1, num * Q2
    int32_t prior_cost;         // 0 DDC, 1 quadratic, 2 Huber (table in build_pattern)
    int32_t huber_k;
    uint32_t p1s, p2s;          // den * P1, den * P2
    int32_t subpixel;
    int32_t store_sum;          // last pass also stores S (debug tap)
    uint32_t* feat;             // last left pass: surrogate cost features, or null
    uint32_t* ckpt;             // paired passes: forward-state checkpoints (scratch)
    int32_t ckpt_segs;          // checkpoints per line (filled by launch_sgm_pair)
    // fallback gate: when non-null, frame f runs only if gate[f] > gate_limit
    const int32_t* gate;
    int32_t gate_limit;
    int32_t view_base;          // first view of the launch (1 = right view only)
    // two-sweep schedule: per-pixel handoff between row bands (zero between
    // launches) and the ticket / done / error words of the launch
    uint32_t* hand;
    int32_t* sync;
    int32_t npaths;
    int32_t rows_per_band;      // filled by launch_sgm_sweep
    // launch geometry (filled by launch_sgm_dir)
    int32_t blocks_per_fv;      // blocks per (frame, view)
    int32_t nviews;
    int32_t n_fv;               // frames * views
};

struct LidarArgs {
    const int16_t* lidar;       // raw sparse map D-bar
    int32_t lidar_pitch;
    int64_t lidar_fstride;
    uint32_t* rowbits;          // [F][H][W][D / 32] row-pass masks
    const int16_t* dstar;       // [F][H][W]
    uint16_t* rho;              // [F][H][W] LiDAR residual (65535 = none)
    const uint32_t* feat;       // [F][H][W][2] (S(d*) | S2nd << 16, curvature)
    uint16_t* x0;               // [F][H][W][8] bf16 surrogate inputs, or null
    uint32_t* wmask;            // when set: the column pass stores the window masks
                                // [F][H][W][D / 32] here instead of the residual
    int64_t px_stride;
    int32_t W, H, D, rc, nframes;
    float sS, sD, sR;           // feature scales
};

struct CheckArgs {
    const int32_t* gate;        // when non-null, frame f runs only if gate[f] > gate_limit
    int32_t gate_limit;
    const int16_t* dstar;
    const int16_t* dright;
    const float* dsub;
    const uint16_t* rho;        // LiDAR residual (Eq. 6 LiDAR test: rho <= Tc)
    float* disp_out;
    uint8_t* valid_out;
    int32_t out_pitch;
    int64_t out_fstride;
    int64_t px_stride;
    int32_t W, H, tc, rc, mode;
};

// ---- learned consistency surrogate ----
// Packed parameters: bf16 weights [tap][out][in] per layer, then fp32 biases.
constexpr int kSurCh = 32;
constexpr int kSurW1 = 9 * 32 * 8, kSurW2 = 9 * 32 * 32, kSurW3 = 9 * 32 * 32, kSurW4 = 9 * 16 * 32;
constexpr int kSurOffW1 = 0, kSurOffW2 = kSurW1, kSurOffW3 = kSurOffW2 + kSurW2,
              kSurOffW4 = kSurOffW3 + kSurW3, kSurNW = kSurOffW4 + kSurW4;
constexpr int kSurNB = 32 + 32 + 32 + 1;
constexpr int kSurOffB1 = 0, kSurOffB2 = 32, kSurOffB3 = 64, kSurOffB4 = 96;
// dilations 1, 3, 9, 27: the composite offsets sum_l k_l 3^l (k_l in -1..1)
// cover every offset in [-40, 40] exactly once (an 81 x 81 receptive field)
constexpr int kSurDil[4] = {1, 3, 9, 27};

struct ConvArgs {
    const uint16_t* x;        // NHWC bf16 input [F][H][W][cin]
    const uint16_t* w;        // [9][cout_pad][cin] bf16
    const float* bias;        // [cout] or null
    uint16_t* y;              // NHWC bf16 output [F][H][W][32] or null
    float* yf;                // channel-0 fp32 output [F][H][W] or null
    const uint16_t* gate;     // NHWC bf16 [F][H][W][32]: keep output where gate > 0
    int64_t px_stride;
    int32_t W, H, dil, relu, cout;
};

struct WgradArgs {
    const uint16_t* x;        // layer input NHWC [F][H][W][cin]
    const uint16_t* g;        // output gradient NHWC [F][H][W][gc]
    float* partial_w;         // [F * blocks][9][32][32]
    float* partial_b;         // [F * blocks][32]
    int64_t px_stride;
    int32_t W, H, dil, rows;
};

struct LossArgs {
    const float* z;           // logits [F][H][W]
    const uint8_t* labels;    // plain-check mask [F][H][W]
    const uint16_t* rho;      // LiDAR residual [F][H][W]
    uint16_t* dz;             // [F][H][W][8] bf16, channel 0 = dLoss/dz
    float* partial_loss;
    int32_t* partial_cnt;
    int32_t* partial_agree;
    float* stats;             // [3]: mean loss, decided pixels, agreeing pixels
    int64_t px_stride;
    int32_t tc;
    float inv_n;
};

struct AdamArgs {
    float* master;
    float* m;
    float* v;
    const float* grad;
    uint16_t* w_bf16;
    float* bias;
    int32_t n, n_w;
    float b1, b2, eps, lr_t;
};

struct MaskArgs {
    const float* logits;
    const uint16_t* rho;
    const float* dsub;
    float* disp_out;
    uint8_t* valid_out;
    int32_t* counter;         // [F] uncertain pixels per frame
    int64_t px_stride;
    int32_t out_pitch;
    int64_t out_fstride;
    int32_t W, H, tc;
    float margin;
};

hipError_t launch_conv(const ConvArgs& a, int cin, int cout_pad, int nframes, hipStream_t s);
hipError_t launch_wtrans(const uint16_t* w, int oc_src, int ic_src, int oc_valid, uint16_t* wt,
                         int oc_dst, int ic_dst, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs& a, int cin, int gc, int nframes, hipStream_t s);
hipError_t launch_reduce_wgrad(const float* pw, const float* pb, int nblocks, int oc_pad, int ic_n,
                               int oc_valid, float* gw, float* gb, hipStream_t s);
hipError_t launch_bce(const LossArgs& a, int nframes, hipStream_t s);
hipError_t launch_adam(const AdamArgs& a, hipStream_t s);
hipError_t launch_sync_weights(const float* master, uint16_t* w_bf16, float* bias, hipStream_t s);
hipError_t launch_learned_mask(const MaskArgs& a, int nframes, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int v, hipStream_t s);

// path pass roles: the first pass stores S, middle ones add into it, the
// last takes the WTA; kMiddle2 also adds the second term S2 of a split pass
enum SgmMode { kFirst = 0, kMiddle = 1, kLast = 2, kSingle = 3, kMiddle2 = 4 };

hipError_t launch_census(const CensusArgs& a, int nframes, hipStream_t s);
hipError_t launch_semidense(const SemiArgs& a, int nframes, hipStream_t s);
// D-bar int16 (caller's pitch) -> prior words (DSGM)
hipError_t launch_prior_words(const int16_t* in, int32_t in_pitch, int64_t in_fstride,
                              const PriorOut& out, int32_t W, int32_t H, int32_t D,
                              int nframes, hipStream_t s);
// guard rings of the left-view maps and the right view's shared map
hipError_t launch_prior_guards(const PriorOut& out, uint32_t* right, uint32_t w_right,
                               int32_t W, int32_t H, int32_t D, int nframes, hipStream_t s);
hipError_t launch_sgm_dir(const SgmArgs& a, int D, int mode, int nviews, int nframes,
                          hipStream_t s);
// split schedule: direction (dx, dy) into S and (-dx, -dy) into S2, one
// launch; k disparities per lane (8, or 4 for D <= 128)
hipError_t launch_sgm_dual(const SgmArgs& a, int D, int mode, int nviews, int nframes,
                           hipStream_t s, int k = 8);
// split schedule: winner-takes-all (+ subpixel) on S + S2 of every pixel
hipError_t launch_sgm_wta(const SgmArgs& a, int D, int nviews, int nframes, hipStream_t s);
// debug tap: C'(p, d) of frame 0, left view, [H][W][D]
hipError_t launch_cost_tap(const SgmArgs& a, int D, uint16_t* out, hipStream_t s);
// runs of at most this many frames use the split schedule
constexpr int kSplitFrames = 1;

// Two-sweep schedule (k_sgm_sweep.hip): sweep A (pass 0) stores the first
// four directions' share of S, sweep B (pass 1) adds the other four and
// takes the WTA.  a.npaths is 4 or 8; a.hand / a.sync as in SgmArgs.
hipError_t launch_sgm_sweep(const SgmArgs& a, int D, int pass, int nviews, int nframes,
                            hipStream_t s);
// row bands per frame-view and rows per band of the two-sweep schedule
struct SweepPlan {
    int bands;
    int rows_per_band;
};
SweepPlan sweep_plan(int H, int D);
int64_t sweep_hand_bytes_per_fv(int W, int H, int D);
// runs of at least this many frames take the two-sweep schedule by default
// (smaller runs leave the machine idle along the sweeps' row skew and are
// faster with the paired passes)
constexpr int kSweepMinFrames = 16;
// two opposite directions (dx, dy) and (-dx, -dy) in one launch
hipError_t launch_sgm_pair(const SgmArgs& a, int D, int mode, int nviews, int nframes,
                           hipStream_t s);
int64_t sgm_pair_ckpt_segs(int W, int H, int dx, int dy);
hipError_t launch_check(const CheckArgs& a, int nframes, hipStream_t s);
hipError_t launch_lidar_bits(const LidarArgs& a, int nframes, hipStream_t s);
// residual + surrogate inputs from a.wmask (masks of launch_lidar_bits with wmask)
hipError_t launch_lidar_rho(const LidarArgs& a, int nframes, hipStream_t s);
// sixth learned-check input (occlusion margin of d*) into x0 channel 5
hipError_t launch_occlusion(const int16_t* dstar, uint16_t* x0, int W, int H, int64_t px_stride,
                            int nframes, hipStream_t s);
hipError_t launch_quantize(const float* in, int W, int H, int in_pitch, int D,
                           int16_t* out, int out_pitch, hipStream_t s);

// number of independent path lines of direction (dx, dy)
inline int num_lines(int W, int H, int dx, int dy)
{
    if (dy == 0) return H;
    if (dx == 0) return W;
    return W + H - 1;
}

}  // namespace sldf
