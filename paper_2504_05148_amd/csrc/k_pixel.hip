// Per-pixel kernels: LiDAR ingest, census transform, semidensification and
// the stereo-LiDAR consistency check.
#include "sldf_internal.h"

namespace sldf {

// ---------------------------------------------------------------------------
// Ingest: real LiDAR disparities -> D-bar (values in N or invalid, Sec. IV).
// Round to nearest, ties to even; NaN, negative and >= D become -1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void quantize_kernel(const float* in, int W, int H,
                                                       int in_pitch, int D, int16_t* out,
                                                       int out_pitch)
{
    int x = blockIdx.x * 64 + (threadIdx.x & 63);
    int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    float v = in[(int64_t)y * in_pitch + x];
    int16_t q = -1;
    if (v >= 0.0f) {                    // false for NaN
        float r = __builtin_rintf(v);   // current rounding mode: nearest even
        if (r < (float)D) q = (int16_t)r;
    }
    out[(int64_t)y * out_pitch + x] = q;
}

hipError_t launch_quantize(const float* in, int W, int H, int in_pitch, int D,
                           int16_t* out, int out_pitch, hipStream_t s)
{
    dim3 grid((W + 63) / 64, (H + 3) / 4);
    hipLaunchKernelGGL(quantize_kernel, grid, dim3(256), 0, s, in, W, H, in_pitch, D, out,
                       out_pitch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Census transform (Sec. IV-A: Hamming distance of census-transformed images,
// centre-symmetric variant).  Bit k of the code is [I(p+o_k) > I(p-o_k)] for
// the first n = (w h - 1) / 2 window offsets in raster order; 0 where the
// window leaves the image.
//
// Tile: 64 x 16 output pixels per 256-thread block, both images of every
// frame in one launch (blockIdx.z = 2 * frame + view).  Image rows are
// staged in LDS with 16-byte (128-bit) coalesced loads: each tile row spans
// [x0 - 16, x0 + 80), 16-byte aligned because the pitch is a multiple of 16.
// ---------------------------------------------------------------------------
constexpr int kCensusTW = 64, kCensusTH = 16, kCensusMaxR = 7;
constexpr int kCensusLW = kCensusTW + 32;
constexpr int kCensusLH = kCensusTH + 2 * kCensusMaxR;

template <int CWT, int CHT>
__global__ __launch_bounds__(256) void census_kernel(CensusArgs a)
{
    const int cw = CWT ? CWT : a.cw, ch = CHT ? CHT : a.ch;
    const int rx = (cw - 1) / 2, ry = (ch - 1) / 2;
    const int n = a.kind == 1 ? cw * ch - 1 : (cw * ch - 1) / 2;
    __shared__ __align__(16) uint8_t tile[kCensusLH][kCensusLW];
    const int view = blockIdx.z & 1, frame = blockIdx.z >> 1;
    const uint8_t* img = (view ? a.right : a.left) + (int64_t)frame * a.img_fstride;
    const int x0 = blockIdx.x * kCensusTW, y0 = blockIdx.y * kCensusTH;
    const int lh = kCensusTH + 2 * ry;
    constexpr int chunks = kCensusLW / 16;
    for (int c = threadIdx.x; c < lh * chunks; c += 256) {
        int r = c / chunks, cc = c - r * chunks;
        int gy = y0 - ry + r, gx = x0 - 16 + cc * 16;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.pitch)
            v = *reinterpret_cast<const uint4*>(img + (int64_t)gy * a.pitch + gx);
        *reinterpret_cast<uint4*>(&tile[r][cc * 16]) = v;
    }
    __syncthreads();
    uint32_t* out = (view ? a.out_r : a.out_l) + (int64_t)frame * a.out_fstride;
    if constexpr (CWT != 0) {
        // a thread takes 4 consecutive pixels of one row (16 threads per
        // 64-pixel row, 16 rows): bytes x - 4 .. x + 7 of each window row are
        // three aligned LDS words, and every comparison takes its two bytes
        // from those registers
        constexpr int RX = (CWT - 1) / 2, RY = (CHT - 1) / 2, N = (CWT * CHT - 1) / 2;
        static_assert(RX <= 4, "the register window covers offsets up to 4");
        const int t = threadIdx.x & 15, ty = threadIdx.x >> 4;
        const int x = x0 + 4 * t, y = y0 + ty;
        if (y >= a.H) return;
        uint32_t R[2 * RY + 1][3];
#pragma unroll
        for (int r = 0; r <= 2 * RY; ++r) {
            const uint32_t* w = reinterpret_cast<const uint32_t*>(&tile[ty + r][12 + 4 * t]);
            R[r][0] = w[0];
            R[r][1] = w[1];
            R[r][2] = w[2];
        }
        const bool yin = y >= RY && y < a.H - RY;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // bit k = [I(p + o_k) > I(p - o_k)], offsets in raster order:
            // shifted in from the last offset to the first
            uint32_t code = 0;
#pragma unroll
            for (int k = N - 1; k >= 0; --k) {
                const int dy = k / CWT - RY, dx = k % CWT - RX;
                const int bp = i + dx + 4, bq = i - dx + 4;
                const uint32_t pv = (R[RY + dy][bp >> 2] >> (8 * (bp & 3))) & 0xffu;
                const uint32_t qv = (R[RY - dy][bq >> 2] >> (8 * (bq & 3))) & 0xffu;
                // qv - pv wraps (bit 31 set) exactly when pv > qv; shift
                // that bit in below the code's previous bits
                code = __builtin_amdgcn_alignbit(code, qv - pv, 31);
            }
            const int xi = x + i;
            if (xi < a.W)
                out[(int64_t)y * a.out_pitch + xi] = yin && xi >= RX && xi < a.W - RX ? code : 0u;
        }
        return;
    }
    const int lx = threadIdx.x & 63;
    for (int ty = threadIdx.x >> 6; ty < kCensusTH; ty += 4) {
        const int x = x0 + lx, y = y0 + ty;
        if (x >= a.W || y >= a.H) continue;
        uint32_t code = 0;
        if (x >= rx && x < a.W - rx && y >= ry && y < a.H - ry) {
            const int cy = ry + ty, cx = 16 + lx;
            int k = 0;
            if (a.kind == 1) {
                // full census: every offset but the centre, raster order,
                // bit k = [I(p + o_k) < I(p)]
                const uint32_t c = tile[cy][cx];
                for (int dy = -ry; dy <= ry; ++dy) {
                    for (int dx = -rx; dx <= rx; ++dx) {
                        if (dx == 0 && dy == 0) continue;
                        code |= (uint32_t)(tile[cy + dy][cx + dx] < c) << k;
                        ++k;
                    }
                }
            } else {
#pragma unroll
                for (int dy = -ry; dy <= ry; ++dy) {
#pragma unroll
                    for (int dx = -rx; dx <= rx; ++dx) {
                        if (k < n) {
                            uint32_t p = tile[cy + dy][cx + dx];
                            uint32_t q = tile[cy - dy][cx - dx];
                            code |= (uint32_t)(p > q) << k;
                        }
                        ++k;
                    }
                }
            }
        }
        out[(int64_t)y * a.out_pitch + x] = code;
    }
}

hipError_t launch_census(const CensusArgs& a, int nframes, hipStream_t s)
{
    dim3 grid((a.W + kCensusTW - 1) / kCensusTW, (a.H + kCensusTH - 1) / kCensusTH,
              2 * nframes);
    if (a.kind == 1)
        hipLaunchKernelGGL((census_kernel<0, 0>), grid, dim3(256), 0, s, a);
    else if (a.cw == 9 && a.ch == 7)
        hipLaunchKernelGGL((census_kernel<9, 7>), grid, dim3(256), 0, s, a);
    else if (a.cw == 5 && a.ch == 5)
        hipLaunchKernelGGL((census_kernel<5, 5>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((census_kernel<0, 0>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Semidensification, Eq. 5 (Sec. IV-B).  For every pixel p: among the valid
// sparse disparities in the (2 rs + 1)^2 window (clipped), take the one with
// the smallest Hamming cost H(p, d) (ties -> smallest d); keep it if that
// cost is below Ts, otherwise keep the sparse value of p.
// Block: 16 x 16 pixels.  The LiDAR window tile is staged in LDS and its
// valid points are compacted into a list (the map is sparse, so a pixel
// visits a few dozen points instead of every window tap); the right-view
// census of the columns a match can reach (x0 - D + 1 .. x0 + 15) is staged
// too.  The minimum over (H, d) does not depend on the visiting order.
// ---------------------------------------------------------------------------
constexpr int kSemiT = 16, kSemiMaxR = 15, kSemiLT = kSemiT + 2 * kSemiMaxR, kSemiMaxD = 256;

// Prior e of pixel (x, y) of frame f: its word for the path passes and, for
// frame 0, the debug tap.
__device__ __forceinline__ void emit_prior(const PriorOut& o, int f, int x, int y, int16_t e,
                                           int D)
{
    o.words[f * o.fstride + (int64_t)(y + 1) * o.pitch + x + 1] =
        prior_word(e, D, o.w_prior, o.w_noprior);
    if (o.tap && f == 0) o.tap[(int64_t)y * (o.pitch - 2) + x] = e;
}

__global__ __launch_bounds__(256) void semidense_kernel(SemiArgs a)
{
    // LDS sized for this D and rs (so that more blocks fit a CU): the right
    // census of the reachable columns [kSemiT][D + kSemiT], the candidate
    // list [lt * lt] ((row << 16) | (col << 8) | d), the LiDAR tile [lt][lt]
    extern __shared__ uint32_t smem[];
    __shared__ int ncand;
    const int frame = blockIdx.z;
    const int16_t* lid = a.lidar + (int64_t)frame * a.lidar_fstride;
    const int rs = a.rs, lt = kSemiT + 2 * rs, D = a.D;
    const int cp = D + kSemiT;
    uint32_t* crow = smem;
    uint32_t* cand = smem + kSemiT * cp;
    int16_t* tile = reinterpret_cast<int16_t*>(cand + lt * lt);
    const int x0 = blockIdx.x * kSemiT, y0 = blockIdx.y * kSemiT;
    if (threadIdx.x == 0) ncand = 0;
    // all staging loads of a thread are issued before its LDS writes, so
    // that they are in flight together
    constexpr int kTileK = (kSemiLT * kSemiLT + 255) / 256;
    constexpr int kRowK = (kSemiT * (kSemiMaxD + kSemiT) + 255) / 256;
    int16_t tv[kTileK];
#pragma unroll
    for (int k = 0; k < kTileK; ++k) {
        const int i = threadIdx.x + 256 * k;
        const int r = i / lt, c = i - r * lt;
        const int gy = y0 - rs + r, gx = x0 - rs + c;
        tv[k] = (i < lt * lt && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
                    ? lid[(int64_t)gy * a.lidar_pitch + gx]
                    : (int16_t)-1;
    }
    // census rows are padded by D codes on each side: columns down to -D are
    // inside the buffer
    const uint32_t* crb = a.census_r + (int64_t)frame * a.census_fstride;
    const int cw = D + kSemiT - 1;
    uint32_t cv[kRowK];
#pragma unroll
    for (int k = 0; k < kRowK; ++k) {
        const int i = threadIdx.x + 256 * k;
        const int r = i / cw, q = i - r * cw, gy = y0 + r;
        cv[k] = (i < kSemiT * cw && gy < a.H)
                    ? crb[(int64_t)gy * a.census_pitch + x0 - D + 1 + q]
                    : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTileK; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i >= lt * lt) break;
        const int r = i / lt, c = i - r * lt;
        const int16_t v = tv[k];
        tile[r * lt + c] = v;
        // values outside [0, D) are no candidates (the ABI admits only -1)
        if ((unsigned)v < (unsigned)D) cand[atomicAdd(&ncand, 1)] = (r << 16) | (c << 8) | v;
    }
#pragma unroll
    for (int k = 0; k < kRowK; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i >= kSemiT * cw) break;
        crow[(i / cw) * cp + i % cw] = cv[k];
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= a.W || y >= a.H) return;
    const uint32_t c = a.census_l[(int64_t)frame * a.census_fstride + (int64_t)y * a.census_pitch + x];
    uint32_t best = 0xffffffffu;   // (H << 16) | d, lexicographic minimum
    auto visit = [&](int d) {
        // matching pixel x - d: staged column tx - d + D - 1 (in [0, cw) for
        // 0 <= d < D)
        const uint32_t h = x - d >= 0 ? (uint32_t)__builtin_popcount(c ^ crow[ty * cp + tx - d + D - 1])
                                      : (uint32_t)a.n;
        const uint32_t key = (h << 16) | (uint32_t)d;
        best = key < best ? key : best;
    };
    const int n = ncand, w = 2 * rs + 1;
    if (n < w * w) {
        for (int k = 0; k < n; ++k) {
            const uint32_t e = cand[k];
            const int r = (int)(e >> 16), cc = (int)((e >> 8) & 0xff);
            if ((unsigned)(r - ty) < (unsigned)w && (unsigned)(cc - tx) < (unsigned)w)
                visit((int)(e & 0xff));
        }
    } else {
        for (int r = 0; r < w; ++r)
            for (int q = 0; q < w; ++q) {
                const int d = tile[(ty + r) * lt + tx + q];
                if ((unsigned)d < (unsigned)D) visit(d);
            }
    }
    int16_t outv = lid[(int64_t)y * a.lidar_pitch + x];
    if ((best >> 16) < (uint32_t)a.ts) outv = (int16_t)(best & 0xffffu);
    emit_prior(a.out, frame, x, y, outv, D);
}

// DSGM: the prior is D-bar itself.
__global__ void prior_words_kernel(const int16_t* in, int32_t in_pitch, int64_t in_fstride,
                                   PriorOut out, int32_t W, int32_t D)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, f = blockIdx.z;
    if (x >= W) return;
    emit_prior(out, f, x, y, in[(int64_t)f * in_fstride + (int64_t)y * in_pitch + x], D);
}

hipError_t launch_prior_words(const int16_t* in, int32_t in_pitch, int64_t in_fstride,
                              const PriorOut& out, int32_t W, int32_t H, int32_t D,
                              int nframes, hipStream_t s)
{
    hipLaunchKernelGGL(prior_words_kernel, dim3((W + 255) / 256, H, nframes), dim3(256), 0, s,
                       in, in_pitch, in_fstride, out, W, D);
    return hipGetLastError();
}

// Guard rings (cost weight 0) of the left-view maps, blockIdx.y = frame:
// the top and bottom rows, then the two side columns.
__global__ void prior_rings_kernel(PriorOut out, int32_t W, int32_t H, int32_t D)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int P = W + 2, f = blockIdx.y;
    if (i >= 2 * P + 2 * H) return;
    int gx, gy;
    if (i < 2 * P) {
        gx = i % P;
        gy = i < P ? 0 : H + 1;
    } else {
        const int k = i - 2 * P;
        gx = k < H ? 0 : W + 1;
        gy = 1 + (k < H ? k : k - H);
    }
    out.words[f * out.fstride + (int64_t)gy * P + gx] = guard_word(D);
}

// The right view's shared map: no prior anywhere, weight w inside, 0 on the
// ring.
__global__ void prior_right_kernel(uint32_t* right, uint32_t w, int32_t W, int32_t H, int32_t D)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int P = W + 2;
    if (i >= P * (H + 2)) return;
    const int gx = i % P, gy = i / P;
    const bool ring = gx == 0 || gx == W + 1 || gy == 0 || gy == H + 1;
    right[i] = ring ? guard_word(D) : prior_word(-1, D, w, w);
}

hipError_t launch_prior_guards(const PriorOut& out, uint32_t* right, uint32_t w_right,
                               int32_t W, int32_t H, int32_t D, int nframes, hipStream_t s)
{
    const int ring = 2 * (W + 2) + 2 * H, n = (W + 2) * (H + 2);
    hipLaunchKernelGGL(prior_rings_kernel, dim3((ring + 255) / 256, nframes), dim3(256), 0, s,
                       out, W, H, D);
    if (right)
        hipLaunchKernelGGL(prior_right_kernel, dim3((n + 255) / 256), dim3(256), 0, s, right,
                           w_right, W, H, D);
    return hipGetLastError();
}

hipError_t launch_semidense(const SemiArgs& a, int nframes, hipStream_t s)
{
    dim3 grid((a.W + kSemiT - 1) / kSemiT, (a.H + kSemiT - 1) / kSemiT, nframes);
    const int lt = kSemiT + 2 * a.rs;
    const size_t lds = ((size_t)kSemiT * (a.D + kSemiT) + (size_t)lt * lt) * 4 + (size_t)lt * lt * 2;
    hipLaunchKernelGGL(semidense_kernel, grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stereo-LiDAR consistency check, Eq. 6 (Sec. IV-C).  A pixel with integer
// disparity d keeps its (subpixel) disparity if
//   stereo: the matched right pixel (x - d, y) exists and |d - d'| <= 1, or
//   LiDAR:  some valid raw sparse value in the (2 rc + 1)^2 window (clipped)
//           is within Tc of d, i.e. the residual rho (window bitset pass) is
//           <= Tc;
// mode selects stereo only (1), LiDAR only (2), both (3) or no check (0).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void check_kernel(CheckArgs a)
{
    const int frame = blockIdx.z;
    if (a.gate && a.gate[frame] <= a.gate_limit) return;   // fallback not needed
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    const int64_t p = (int64_t)frame * a.px_stride + (int64_t)y * a.W + x;
    const int d = a.dstar[p];
    bool valid = a.mode == 0;
    if (a.mode & 1) {
        int xm = x - d;
        if (xm >= 0) {
            int diff = d - a.dright[p - x + xm];
            valid = diff >= -1 && diff <= 1;
        }
    }
    if ((a.mode & 2) && !valid) valid = (int)a.rho[p] <= a.tc;
    const int64_t o = (int64_t)frame * a.out_fstride + (int64_t)y * a.out_pitch + x;
    a.valid_out[o] = valid ? 1 : 0;
    a.disp_out[o] = valid ? a.dsub[p] : -1.0f;
}

hipError_t launch_check(const CheckArgs& a, int nframes, hipStream_t s)
{
    dim3 grid((a.W + 63) / 64, (a.H + 3) / 4, nframes);
    hipLaunchKernelGGL(check_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sldf
