// Learned consistency surrogate: a 4-layer 3x3 CNN (6 -> 32 -> 32 -> 32 -> 1
// channels, dilations 1, 3, 9, 27, ReLU between layers) that predicts the
// validity mask of the stereo-LiDAR check (Eq. 6) from left-view cost
// features, so that the right-view SGM pass can be skipped.  BF16 weights and
// activations, FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16), FP32 master weights for training.
//
// Convolution = implicit GEMM per 16-pixel row tile:
//   D[oc][px] += W[oc][k] * X[k][px],  k = (tap, input channel)
// A operand (16 output channels x 32 k): the weights, held in registers for
// a whole block; B operand (32 k x 16 pixels): one 16-byte LDS read of 8
// input channels of one neighbour pixel (NHWC).  With 32 input channels one k-step
// is one tap; with 8 input channels one k-step covers four taps.
// Backward: dgrad is the same convolution with tap-flipped, channel-
// transposed weights and the ReLU gate of the layer input; wgrad is an MFMA
// GEMM over pixels with transposed tiles staged in LDS, reduced across
// blocks in a fixed order (deterministic).
#include "sldf_internal.h"

namespace sldf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f32(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

__device__ __forceinline__ f32x4 mfma16(uint4 a, uint4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// 3x3 dilated convolution, NHWC bf16 in, bf16 (32 ch) or fp32 (1 ch) out. A
// block owns TW = 64 TPW output columns of one dilation lattice (the rows r, r
// + d, r + 2d, ... of a residue r) and walks down up to kConvRowsMax of its
// rows (8 in single-frame calls).  Output row i reads the input rows y - d, y,
// y + d, so consecutive output rows share two of their three input rows: the
// input rows (columns x0 - d .. x0 + TW - 1 + d, zero outside the image) pass
// through a ring of kConvSlots LDS slots, each read from memory once per
// block, and are fetched kConvAhead rows ahead into registers so that their
// latency overlaps the matrix work of the rows before.  Wave w computes the
// 16-pixel tiles w, w + 4, .. of every output row; the weights (A operand)
// stay in registers for the whole block.  Blocks go to the XCDs in contiguous
// ranges, so neighbouring column tiles share the halo through one L2.  Every
// output pixel sums its k-steps in order, whatever the tiling.
// ---------------------------------------------------------------------------
constexpr int kConvMaxDil = 29;      // largest dilation (LDS budget of the ring)
constexpr int kConvSlots = 4;        // three input rows in use, one being filled
constexpr int kConvAhead = 3;        // input rows in flight in registers
constexpr int kConvRowsMax = 32;     // output rows per block, at most
constexpr int kConvMaxLds = 65536;

// 16-byte chunk c of pixel q (CIN = 32: 4 chunks) is stored at chunk
// position c ^ ((q >> 2) & 3): the 16 lanes of one LDS read pass (16
// consecutive q, same c) then cover all 64 banks.
template <int C16>
__device__ __forceinline__ int swz(int q, int c)
{
    return C16 == 4 ? q * 4 + (c ^ ((q >> 2) & 3)) : q * C16 + c;
}

template <int CIN, int NMT, int TPW>
__global__ __launch_bounds__(256) void conv3x3_kernel(ConvArgs a, int ntx, int qblocks,
                                                      int rows_blk, int nframes)
{
    constexpr int OC = NMT * 16;                 // padded output channels
    constexpr int KSTEPS = CIN == 32 ? 9 : 3;
    constexpr int C16 = CIN / 8;                 // 16-byte chunks per pixel
    constexpr int TW = 64 * TPW;                 // output columns per block
    constexpr int PPASS = 256 / C16;             // pixels staged per pass
    constexpr int PASSES = (TW + 2 * kConvMaxDil + PPASS - 1) / PPASS;
    extern __shared__ uint4 xin[];               // [kConvSlots][tw][C16], swizzled
    const int d = a.dil;
    const int tw = TW + 2 * d;
    // block -> (frame, lattice residue r, lattice block qb, column tile tx)
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const int logical = (b % 8) * (nb / 8) + b / 8;
    const int per_frame = ntx * d * qblocks;
    const int frame = logical / per_frame;
    if (frame >= nframes) return;
    const int rem = logical - frame * per_frame;
    const int yb = rem / ntx, tx = rem - yb * ntx;
    const int r = yb / qblocks, qb = yb - r * qblocks;
    const int x0 = tx * TW;
    const int nrows = min(rows_blk, (a.H - r + d - 1) / d - qb * rows_blk);
    if (nrows <= 0) return;                      // uniform over the block
    const uint16_t* x = a.x + (int64_t)frame * a.px_stride * CIN;
    const int ybase = r + d * (qb * rows_blk - 1);   // input row k is ybase + d k

    // input row k (0 .. nrows + 1) into registers; rows past the block's
    // last one repeat it (cache hits, never used), rows outside the image
    // load a clamped row and are stored as zeros
    const int c = threadIdx.x % C16, pxo = threadIdx.x / C16;
    auto load_row = [&](int k, uint4(&v)[PASSES]) {
        const int sy = ybase + d * min(k, nrows + 1);
        const int syc = min(max(sy, 0), a.H - 1);
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            // lanes past the tile row (px >= tw) repeat its last pixel, so
            // their requests merge with that lane's instead of fetching more
            const int sx = x0 - d + min(ps * PPASS + pxo, tw - 1);
            const int sxc = min(max(sx, 0), a.W - 1);
            v[ps] = *reinterpret_cast<const uint4*>(x + ((int64_t)syc * a.W + sxc) * CIN + 8 * c);
        }
    };
    auto store_row = [&](int k, const uint4(&v)[PASSES]) {
        const int sy = ybase + d * k;
        const bool rin = sy >= 0 && sy < a.H;
        uint4* slot = xin + (k % kConvSlots) * tw * C16;
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int px = ps * PPASS + pxo;
            const int sx = x0 - d + px;
            const bool in = rin && sx >= 0 && sx < a.W;
            if (px < tw) slot[swz<C16>(px, c)] = in ? v[ps] : make_uint4(0, 0, 0, 0);
        }
    };

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    // weights: A operand of every k-step and output-channel tile
    uint4 av[KSTEPS][NMT];
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        const int tap = CIN == 32 ? ks : 4 * ks + g;
        const int ch0 = CIN == 32 ? 8 * g : 0;
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt)
            av[ks][mt] = tap < 9 ? *reinterpret_cast<const uint4*>(a.w + (tap * OC + 16 * mt + j) * CIN + ch0)
                                 : make_uint4(0, 0, 0, 0);
    }
    // bias of the lane's output channels, held for the whole block (a load
    // inside the row loop would wait for every input row in flight)
    float bias[NMT][4];
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int oc = 16 * mt + 4 * g + e;
            bias[mt][e] = a.bias && oc < a.cout ? a.bias[oc] : 0.f;
        }
    {
        uint4 v[3][PASSES];
#pragma unroll
        for (int k = 0; k < 3; ++k) load_row(k, v[k]);
#pragma unroll
        for (int k = 0; k < 3; ++k) store_row(k, v[k]);
    }
    uint4 q[kConvAhead][PASSES];
#pragma unroll
    for (int k = 0; k < kConvAhead; ++k) load_row(3 + k, q[k]);
    __syncthreads();

    // output row i: input rows i, i + 1, i + 2 are in their slots; the slot
    // of row i + 3 held row i - 1, whose readers all passed the last barrier
    for (int i0 = 0; i0 < nrows; i0 += kConvAhead) {
#pragma unroll
        for (int jj = 0; jj < kConvAhead; ++jj) {
            const int i = i0 + jj;
            store_row(i + 3, q[jj]);
            load_row(i + 3 + kConvAhead, q[jj]);
            f32x4 acc[TPW][NMT];
#pragma unroll
            for (int t = 0; t < TPW; ++t)
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt) acc[t][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KSTEPS; ++ks) {
                const int tap = CIN == 32 ? ks : 4 * ks + g;
                const int ky = tap / 3, kx = tap % 3;
                const uint4* slot = xin + ((i + ky) % kConvSlots) * tw * C16;
#pragma unroll
                for (int t = 0; t < TPW; ++t) {
                    const int xt = wave + 4 * t;
                    uint4 bv = make_uint4(0, 0, 0, 0);
                    if (tap < 9) bv = slot[swz<C16>(xt * 16 + j + kx * d, CIN == 32 ? g : 0)];
#pragma unroll
                    for (int mt = 0; mt < NMT; ++mt) acc[t][mt] = mfma16(av[ks][mt], bv, acc[t][mt]);
                }
            }
            // rows past nrows (the last group's padding) are computed but not stored
            const int y = r + d * (qb * rows_blk + i);
            const int64_t prow = (int64_t)frame * a.px_stride + (int64_t)y * a.W;
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int pxt = x0 + (wave + 4 * t) * 16;    // first pixel of the tile
                const int px = pxt + j;
                const bool keep = i < nrows && px < a.W;
                const int64_t p = prow + px;
                // lane holds pixel j, output channels 16 mt + 4 g + e
                float v[NMT][4];
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        v[mt][e] = acc[t][mt][e] + bias[mt][e];
                        if (a.relu) v[mt][e] = v[mt][e] > 0.f ? v[mt][e] : 0.f;
                    }
                    if (a.gate && keep) {
                        const uint2 gv = *reinterpret_cast<const uint2*>(a.gate + p * 32 + 16 * mt + 4 * g);
                        const uint16_t gs[4] = {(uint16_t)(gv.x & 0xffff), (uint16_t)(gv.x >> 16),
                                                (uint16_t)(gv.y & 0xffff), (uint16_t)(gv.y >> 16)};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            v[mt][e] = (gs[e] != 0 && !(gs[e] & 0x8000)) ? v[mt][e] : 0.f;   // gate > 0
                    }
                }
                if (a.yf && g == 0 && keep) a.yf[p] = v[0][0];
                if (NMT == 2 && a.y) {
                    // lane (j, g) holds channels 4g..4g+3 (A) and 16+4g..
                    // 16+4g+3 (B) of pixel j, rows of 16 lanes being g.  One
                    // swap of the odd rows of A with the even rows of B gives
                    // row 0 channels 0-7, row 1 16-23, row 2 8-15, row 3
                    // 24-31: each lane then stores 16 contiguous bytes and a
                    // wave the tile's 16 whole pixels (1 KB).  Channels at
                    // or above cout hold bias 0 and zero weights: they are 0.
                    const uint32_t A0 = bf16_rne(v[0][0]) | ((uint32_t)bf16_rne(v[0][1]) << 16);
                    const uint32_t A1 = bf16_rne(v[0][2]) | ((uint32_t)bf16_rne(v[0][3]) << 16);
                    const uint32_t B0 = bf16_rne(v[1][0]) | ((uint32_t)bf16_rne(v[1][1]) << 16);
                    const uint32_t B1 = bf16_rne(v[1][2]) | ((uint32_t)bf16_rne(v[1][3]) << 16);
                    const auto s0 = __builtin_amdgcn_permlane16_swap(A0, B0, false, false);
                    const auto s1 = __builtin_amdgcn_permlane16_swap(A1, B1, false, false);
                    const uint4 o = make_uint4(s0[0], s1[0], s0[1], s1[1]);
                    const int chunk = ((g & 1) << 1) | (g >> 1);
                    if (keep) *reinterpret_cast<uint4*>(a.y + p * 32 + 8 * chunk) = o;
                }
            }
            __syncthreads();
        }
    }
}

template <int CIN, int NMT, int TPW>
static hipError_t launch_conv_tw(const ConvArgs& a, int nframes, hipStream_t s)
{
    const int d = a.dil;
    const size_t lds = (size_t)kConvSlots * (64 * TPW + 2 * d) * CIN * 2;
    if (d < 1 || d > kConvMaxDil || lds > (size_t)kConvMaxLds) return hipErrorInvalidValue;
    const int ntx = (a.W + 64 * TPW - 1) / (64 * TPW);
    const int lattice_rows = (a.H + d - 1) / d;                  // rows per residue, at most
    // single frames: shorter walks, more blocks (one frame alone fills about
    // one block per CU at 32 rows, and a block's rows run one after another)
    const int rows_max = nframes == 1 ? 8 : kConvRowsMax;
    const int qblocks = (lattice_rows + rows_max - 1) / rows_max;
    const int rows_blk = (lattice_rows + qblocks - 1) / qblocks;
    const int64_t nb = (int64_t)ntx * d * qblocks * nframes;
    dim3 grid((unsigned)((nb + 7) / 8 * 8));
    hipLaunchKernelGGL((conv3x3_kernel<CIN, NMT, TPW>), grid, dim3(256), lds, s, a, ntx, qblocks,
                       rows_blk, nframes);
    return hipGetLastError();
}

// wide dilations take 128-column tiles (the 2d halo columns are read once
// per tile, so wider tiles read fewer of them per output pixel)
template <int CIN, int NMT>
static hipError_t launch_conv_t(const ConvArgs& a, int nframes, hipStream_t s)
{
    return a.dil >= 9 ? launch_conv_tw<CIN, NMT, 2>(a, nframes, s)
                      : launch_conv_tw<CIN, NMT, 1>(a, nframes, s);
}

hipError_t launch_conv(const ConvArgs& a, int cin, int cout_pad, int nframes, hipStream_t s)
{
    if (cin == 32 && cout_pad == 32) return launch_conv_t<32, 2>(a, nframes, s);
    if (cin == 8 && cout_pad == 32) return launch_conv_t<8, 2>(a, nframes, s);
    // 16 padded output channels: channel 0 as fp32 only
    if (cin == 32 && cout_pad == 16 && !a.y) return launch_conv_t<32, 1>(a, nframes, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// dgrad weights: Wt[tap][i][o] = W[8 - tap][o][i]  (the flipped tap set is
// the mirrored 3x3 offset grid), zero-padded to the target shape.
// ---------------------------------------------------------------------------
__global__ void wtrans_kernel(const uint16_t* w, int oc_src, int ic_src, int oc_valid,
                              uint16_t* wt, int oc_dst, int ic_dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * oc_dst * ic_dst) return;
    const int tap = i / (oc_dst * ic_dst), r = i % (oc_dst * ic_dst);
    const int o = r / ic_dst, in = r % ic_dst;   // o: input ch of the source layer
    uint16_t v = 0;
    if (in < oc_valid && o < ic_src) v = w[((8 - tap) * oc_src + in) * ic_src + o];
    wt[i] = v;
}

hipError_t launch_wtrans(const uint16_t* w, int oc_src, int ic_src, int oc_valid, uint16_t* wt,
                         int oc_dst, int ic_dst, hipStream_t s)
{
    const int n = 9 * oc_dst * ic_dst;
    hipLaunchKernelGGL(wtrans_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, oc_src, ic_src,
                       oc_valid, wt, oc_dst, ic_dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// wgrad: dW[tap][co][ci] = sum_p G[p][co] * X[p + off(tap)][ci], db[co] =
// sum_p G[p][co], over the rows [y0, y0 + rows) of one frame; one partial
// [9][32][32] + [32] per block, summed in a fixed order afterwards.
// G^T and the shifted X^T tiles (64 pixels) are staged in LDS with padded
// rows; wave w computes output tile (co-tile w / 2, ci-tile w % 2).
// ---------------------------------------------------------------------------
constexpr int kWgPx = 64, kWgLd = kWgPx + 8;

template <int CIN, int GC>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a)
{
    __shared__ __align__(16) uint16_t gT[32][kWgLd];
    __shared__ __align__(16) uint16_t xT[32][kWgLd];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    const int mt = wave >> 1, nt = wave & 1;
    const int frame = blockIdx.y;
    const int y0 = blockIdx.x * a.rows;
    const uint16_t* X = a.x + (int64_t)frame * a.px_stride * CIN;
    const uint16_t* G = a.g + (int64_t)frame * a.px_stride * GC;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const bool active = (16 * mt < GC) && (16 * nt < CIN);
    for (int y = y0; y < y0 + a.rows && y < a.H; ++y) {
        for (int xb = 0; xb < a.W; xb += kWgPx) {
            __syncthreads();
            // stage G^T: 64 px x GC channels, 8 channels per 16-byte load
            for (int i = threadIdx.x; i < kWgPx * (GC / 8); i += 256) {
                const int pp = i / (GC / 8), c8 = i % (GC / 8);
                uint4 v = make_uint4(0, 0, 0, 0);
                if (xb + pp < a.W)
                    v = *reinterpret_cast<const uint4*>(G + ((int64_t)y * a.W + xb + pp) * GC + 8 * c8);
                const uint16_t e[8] = {(uint16_t)(v.x & 0xffff), (uint16_t)(v.x >> 16),
                                       (uint16_t)(v.y & 0xffff), (uint16_t)(v.y >> 16),
                                       (uint16_t)(v.z & 0xffff), (uint16_t)(v.z >> 16),
                                       (uint16_t)(v.w & 0xffff), (uint16_t)(v.w >> 16)};
#pragma unroll
                for (int k = 0; k < 8; ++k) gT[8 * c8 + k][pp] = e[k];
            }
            __syncthreads();
            if (threadIdx.x < GC) {
                for (int pp = 0; pp < kWgPx; ++pp) bsum += bf16_f32(gT[threadIdx.x][pp]);
            }
            for (int tap = 0; tap < 9; ++tap) {
                const int dx = (tap % 3 - 1) * a.dil, dy = (tap / 3 - 1) * a.dil;
                const int sy = y + dy;
                for (int i = threadIdx.x; i < kWgPx * (CIN / 8); i += 256) {
                    const int pp = i / (CIN / 8), c8 = i % (CIN / 8);
                    const int sx = xb + pp + dx;
                    uint4 v = make_uint4(0, 0, 0, 0);
                    if (xb + pp < a.W && sx >= 0 && sx < a.W && sy >= 0 && sy < a.H)
                        v = *reinterpret_cast<const uint4*>(X + ((int64_t)sy * a.W + sx) * CIN + 8 * c8);
                    const uint16_t e[8] = {(uint16_t)(v.x & 0xffff), (uint16_t)(v.x >> 16),
                                           (uint16_t)(v.y & 0xffff), (uint16_t)(v.y >> 16),
                                           (uint16_t)(v.z & 0xffff), (uint16_t)(v.z >> 16),
                                           (uint16_t)(v.w & 0xffff), (uint16_t)(v.w >> 16)};
#pragma unroll
                    for (int k = 0; k < 8; ++k) xT[8 * c8 + k][pp] = e[k];
                }
                __syncthreads();
                if (active) {
#pragma unroll
                    for (int ks = 0; ks < kWgPx / 32; ++ks) {
                        const int co = 16 * mt + j, ci = 16 * nt + j;
                        uint4 av = make_uint4(0, 0, 0, 0), bv = make_uint4(0, 0, 0, 0);
                        if (co < GC) av = *reinterpret_cast<const uint4*>(&gT[co][32 * ks + 8 * g]);
                        if (ci < CIN) bv = *reinterpret_cast<const uint4*>(&xT[ci][32 * ks + 8 * g]);
                        acc[tap] = mfma16(av, bv, acc[tap]);
                    }
                }
                __syncthreads();
            }
        }
    }
    // partial of this block: lane holds D[co = 16 mt + 4 g + e][ci = 16 nt + j]
    float* pw = a.partial_w + (int64_t)(frame * gridDim.x + blockIdx.x) * 9 * 32 * 32;
    if (active) {
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                pw[(t * 32 + 16 * mt + 4 * g + e) * 32 + 16 * nt + j] = acc[t][e];
    } else {
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                pw[(t * 32 + 16 * mt + 4 * g + e) * 32 + 16 * nt + j] = 0.f;
    }
    if (threadIdx.x < 32)
        a.partial_b[(int64_t)(frame * gridDim.x + blockIdx.x) * 32 + threadIdx.x] =
            threadIdx.x < GC ? bsum : 0.f;
}

hipError_t launch_wgrad(const WgradArgs& a, int cin, int gc, int nframes, hipStream_t s)
{
    dim3 grid((a.H + a.rows - 1) / a.rows, nframes);
    if (cin == 32 && gc == 32) hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, dim3(256), 0, s, a);
    else if (cin == 8 && gc == 32) hipLaunchKernelGGL((wgrad_kernel<8, 32>), grid, dim3(256), 0, s, a);
    else if (cin == 32 && gc == 8) hipLaunchKernelGGL((wgrad_kernel<32, 8>), grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// Fixed-order sum of the per-block partials into the packed gradient of one
// layer: gw[tap][oc][ic] (oc < oc_pad, ic < ic_n), gb[oc] (oc < oc_valid).
__global__ void reduce_wgrad_kernel(const float* pw, const float* pb, int nblocks, int oc_pad,
                                    int ic_n, int oc_valid, float* gw, float* gb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = 9 * oc_pad * ic_n;
    if (i < nw) {
        const int tap = i / (oc_pad * ic_n), r = i % (oc_pad * ic_n);
        const int oc = r / ic_n, ic = r % ic_n;
        float s = 0.f;
        if (oc < 32)
            for (int b = 0; b < nblocks; ++b) s += pw[((int64_t)b * 9 + tap) * 1024 + oc * 32 + ic];
        gw[i] = oc < oc_valid ? s : 0.f;
    } else if (i < nw + oc_valid) {
        const int oc = i - nw;
        float s = 0.f;
        for (int b = 0; b < nblocks; ++b) s += pb[(int64_t)b * 32 + oc];
        gb[oc] = s;
    }
}

hipError_t launch_reduce_wgrad(const float* pw, const float* pb, int nblocks, int oc_pad, int ic_n,
                               int oc_valid, float* gw, float* gb, hipStream_t s)
{
    const int n = 9 * oc_pad * ic_n + oc_valid;
    hipLaunchKernelGGL(reduce_wgrad_kernel, dim3((n + 255) / 256), dim3(256), 0, s, pw, pb, nblocks,
                       oc_pad, ic_n, oc_valid, gw, gb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Loss: binary cross-entropy with logits over the pixels the LiDAR test does
// not decide (rho > Tc); the label is the plain check's mask.  Writes the
// logit gradient (sigma(z) - y) * inv_n as the channel-0 of a bf16 [px][8]
// map, and per-block partial sums (loss, count, agreement) in a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void bce_kernel(LossArgs a)
{
    __shared__ float sl[256];
    __shared__ int sc[256], sa[256];
    const int frame = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    int c = 0, agree = 0;
    if (i < a.px_stride) {
        const int64_t p = (int64_t)frame * a.px_stride + i;
        const float z = a.z[p];
        const int lab = a.labels[p] ? 1 : 0;
        const bool m = (int)a.rho[p] > a.tc;
        float dz = 0.f;
        if (m) {
            const float sg = 1.f / (1.f + __expf(-z));
            dz = (sg - (float)lab) * a.inv_n;
            const float az = fabsf(z);
            l = (z > 0.f ? z : 0.f) - z * (float)lab + log1pf(__expf(-az));
            c = 1;
            agree = ((z > 0.f) ? 1 : 0) == lab;
        } else {
            agree = lab;   // the LiDAR test decides; plain mask is valid too
        }
        uint4 o = make_uint4(bf16_rne(dz), 0, 0, 0);
        *reinterpret_cast<uint4*>(a.dz + p * 8) = o;
    }
    sl[threadIdx.x] = l;
    sc[threadIdx.x] = c;
    sa[threadIdx.x] = i < a.px_stride ? agree : 0;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sl[threadIdx.x] += sl[threadIdx.x + st];
            sc[threadIdx.x] += sc[threadIdx.x + st];
            sa[threadIdx.x] += sa[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t b = (int64_t)frame * gridDim.x + blockIdx.x;
        a.partial_loss[b] = sl[0];
        a.partial_cnt[b] = sc[0];
        a.partial_agree[b] = sa[0];
    }
}

__global__ void bce_reduce_kernel(const float* pl, const int* pc, const int* pa, int n, float* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float l = 0.f;
    long long c = 0, ag = 0;
    for (int i = 0; i < n; ++i) {
        l += pl[i];
        c += pc[i];
        ag += pa[i];
    }
    out[0] = c ? l / (float)c : 0.f;   // mean loss over decided pixels
    out[1] = (float)c;
    out[2] = (float)ag;                // pixels where (z > 0 or LiDAR) == label
}

hipError_t launch_bce(const LossArgs& a, int nframes, hipStream_t s)
{
    const int nb = (int)((a.px_stride + 255) / 256);
    hipLaunchKernelGGL(bce_kernel, dim3(nb, nframes), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.stats)
        hipLaunchKernelGGL(bce_reduce_kernel, dim3(1), dim3(64), 0, s, a.partial_loss, a.partial_cnt,
                           a.partial_agree, nb * nframes, a.stats);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adam on the fp32 master parameters; writes the bf16 weights and fp32 biases
// used by the kernels.  lr_t already carries the bias correction.
// ---------------------------------------------------------------------------
__global__ void adam_kernel(AdamArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float gr = a.grad[i];
    const float m = a.b1 * a.m[i] + (1.f - a.b1) * gr;
    const float v = a.b2 * a.v[i] + (1.f - a.b2) * gr * gr;
    a.m[i] = m;
    a.v[i] = v;
    const float p = a.master[i] - a.lr_t * m / (sqrtf(v) + a.eps);
    a.master[i] = p;
    if (i < a.n_w)
        a.w_bf16[i] = bf16_rne(p);
    else
        a.bias[i - a.n_w] = p;
}

// Working parameters from the fp32 master copy: bf16 weights (RNE) and fp32
// biases, the form the convolutions read.
__global__ void sync_weights_kernel(const float* master, int n_w, int n, uint16_t* w_bf16,
                                    float* bias)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i < n_w)
        w_bf16[i] = bf16_rne(master[i]);
    else
        bias[i - n_w] = master[i];
}

hipError_t launch_sync_weights(const float* master, uint16_t* w_bf16, float* bias, hipStream_t s)
{
    const int n = kSurNW + kSurNB;
    hipLaunchKernelGGL(sync_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, s, master, kSurNW,
                       n, w_bf16, bias);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Learned check output: valid = (logit > 0) or (rho <= Tc); counts the
// undecided-and-uncertain pixels (rho > Tc, |logit| < margin) per frame for
// the device-side fallback to the plain check.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void learned_mask_kernel(MaskArgs a)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int frame = blockIdx.z;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x < a.W && y < a.H) {
        const int64_t p = (int64_t)frame * a.px_stride + (int64_t)y * a.W + x;
        const float z = a.logits[p];
        const bool lid = (int)a.rho[p] <= a.tc;
        const bool valid = lid || z > 0.f;
        const int64_t o = (int64_t)frame * a.out_fstride + (int64_t)y * a.out_pitch + x;
        a.valid_out[o] = valid ? 1 : 0;
        a.disp_out[o] = valid ? a.dsub[p] : -1.0f;
        if (!lid && fabsf(z) < a.margin) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(&a.counter[frame], cnt);
}

hipError_t launch_learned_mask(const MaskArgs& a, int nframes, hipStream_t s)
{
    dim3 grid((a.W + 63) / 64, (a.H + 3) / 4, nframes);
    hipLaunchKernelGGL(learned_mask_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256),
                       0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace sldf
