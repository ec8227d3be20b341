// Internal declarations shared by the HIP sources of libsldf.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sldf {

// Workspace segments of one context (segment-major: every segment holds all
// batch frames back to back with the stated frame stride, in elements).
// Census rows are padded by D codes on both sides so that every matching
// pixel x -+ d of a disparity range lies inside the allocation; census_l and
// census_r point at pixel (0, 0) of frame 0 (pad included before it) and
// pixel (x, y) of frame f sits at f * census_fstride + y * census_pitch + x.
struct Buffers {
    uint32_t* census_l;
    uint32_t* census_r;
    int32_t census_pitch;     // W + 2 D
    int64_t census_fstride;   // H * census_pitch
    int16_t* prior;       // [F][H][W]  semidense map (SDSGM only)
    int16_t* dstar;       // [F][H][W]
    int16_t* dright;      // [F][H][W]
    float* dsub;          // [F][H][W]
    uint16_t* S_left;     // [F][H][W][D]
    uint16_t* S_right;    // [F][H][W][D] (only when the stereo check is on)
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
};

struct SemiArgs {
    const uint32_t* census_l;
    const uint32_t* census_r;
    int32_t census_pitch;
    int64_t census_fstride;
    const int16_t* lidar;
    int32_t lidar_pitch;
    int64_t lidar_fstride;
    int16_t* out;
    int64_t px_stride;
    int32_t W, H, n, ts, rs;
};

struct SgmArgs {
    const uint32_t* cbase[2];   // base-view census per view (left, right)
    const uint32_t* cmatch[2];  // matching-view census per view
    int32_t census_pitch;
    int64_t census_fstride;
    const int16_t* prior;       // left-view prior (D-hat / D-bar)
    int32_t prior_pitch;
    int64_t prior_fstride;
    uint16_t* S[2];             // aggregated cost per view
    int16_t* wta[2];            // integer WTA output per view (d*, d')
    float* dsub;                // left-view subpixel output
    int64_t px_stride;
    int64_t S_stride;
    int32_t W, H;
    int32_t n;                  // census bits (cost where the match leaves)
    int32_t dx, dy;             // path step r
    int32_t nlines;
    uint32_t mulh_prior;        // (den - num)
    uint32_t mulh_noprior;      // (den - num) or den (blend mode 1)
    uint32_t q1s, q2s;          // num * Q1, num * Q2
    uint32_t p1s, p2s;          // den * P1, den * P2
    int32_t subpixel;
    int32_t store_sum;          // last pass also stores S (debug tap)
    // launch geometry (filled by launch_sgm_dir)
    int32_t blocks_per_fv;      // blocks per (frame, view)
    int32_t nviews;
    int32_t n_fv;               // frames * views
};

struct CheckArgs {
    const int16_t* dstar;
    const int16_t* dright;
    const float* dsub;
    const int16_t* lidar;
    int32_t lidar_pitch;
    int64_t lidar_fstride;
    float* disp_out;
    uint8_t* valid_out;
    int32_t out_pitch;
    int64_t out_fstride;
    int64_t px_stride;
    int32_t W, H, tc, rc, mode;
};

enum SgmMode { kFirst = 0, kMiddle = 1, kLast = 2, kSingle = 3 };

hipError_t launch_census(const CensusArgs& a, int nframes, hipStream_t s);
hipError_t launch_semidense(const SemiArgs& a, int nframes, hipStream_t s);
hipError_t launch_sgm_dir(const SgmArgs& a, int D, int mode, int nviews, int nframes,
                          hipStream_t s);
hipError_t launch_check(const CheckArgs& a, int nframes, hipStream_t s);
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
