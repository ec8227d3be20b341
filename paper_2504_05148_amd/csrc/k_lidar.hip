// LiDAR window test of Eq. 6 (Sec. IV-C) as an exact separable bitset OR,
// and the learned-surrogate input features.
//
// For every pixel the set of valid raw sparse disparities inside the
// (2 rc + 1)^2 window K_p is a D-bit mask (D / 32 words).  The row pass ORs
// the single-bit masks of the 2 rc + 1 pixels of each row segment, the
// column pass ORs 2 rc + 1 row masks as a sliding window (a constant number
// of word ORs per pixel), so the window test costs O(rc) operations per
// pixel instead of (2 rc + 1)^2 compares.  From the mask
// and d* the column pass derives rho_p = min |d* - v| over the set (65535 if
// empty); the LiDAR half of Eq. 6 is then exactly rho_p <= Tc.
#include "sldf_internal.h"

namespace sldf {

constexpr int kRowSeg = 256, kMaxRc = 31;

template <int NW>
__global__ __launch_bounds__(256) void lidar_rowbits_kernel(LidarArgs a)
{
    __shared__ int16_t seg[kRowSeg + 2 * kMaxRc];
    const int frame = blockIdx.z, y = blockIdx.y, x0 = blockIdx.x * kRowSeg;
    const int16_t* lid = a.lidar + (int64_t)frame * a.lidar_fstride + (int64_t)y * a.lidar_pitch;
    const int rc = a.rc;
    for (int i = threadIdx.x; i < kRowSeg + 2 * rc; i += 256) {
        const int gx = x0 - rc + i;
        seg[i] = (gx >= 0 && gx < a.W) ? lid[gx] : (int16_t)-1;
    }
    __syncthreads();
    const int x = x0 + threadIdx.x;
    if (x >= a.W) return;
    uint32_t w[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) w[j] = 0u;
    for (int k = 0; k <= 2 * rc; ++k) {
        const int v = seg[threadIdx.x + k];
        if ((unsigned)v < (unsigned)a.D) {
            const uint32_t bit = 1u << (v & 31);
#pragma unroll
            for (int j = 0; j < NW; ++j) w[j] |= (v >> 5) == j ? bit : 0u;
        }
    }
    uint32_t* out = a.rowbits + (((int64_t)frame * a.H + y) * a.W + x) * NW;
#pragma unroll
    for (int j = 0; j < NW; j += 2) *reinterpret_cast<uint2*>(out + j) = make_uint2(w[j], w[j + 1]);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// rho_p = min |d - v| over the set bits v of the pixel's window mask m
// (NW lanes per pixel, lane w holding word w; 65535 if empty), written by
// the owner lane (w == 0) with the surrogate inputs when requested.
template <int NW>
__device__ __forceinline__ void emit_rho(const LidarArgs& a, uint32_t m, int d, int w, bool owner,
                                         int64_t px, uint32_t s01, uint32_t cv)
{
    const int lo = 32 * w;
    // this word's nearest set bits at index >= d and <= d
    const uint32_t mu = d < lo ? m : (d - lo < 32 ? m & (0xffffffffu << (d - lo)) : 0u);
    const uint32_t md =
        d < lo ? 0u : (d - lo < 32 ? m & (0xffffffffu >> (31 - (d - lo))) : m);
    const int up = mu ? lo + __builtin_ctz(mu) - d : 0xffff;
    const int dn = md ? d - (lo + 31 - __builtin_clz(md)) : 0xffff;
    int rho = up < dn ? up : dn;
#pragma unroll
    for (int q = 1; q < NW; q <<= 1) {
        const int o = __shfl_xor(rho, q, NW);
        rho = o < rho ? o : rho;
    }
    if (!owner) return;
    a.rho[px] = (uint16_t)rho;
    if (a.x0) {
        // surrogate inputs: S(d*), second minimum, curvature, d*,
        // residual, each an integer times a float32 scale, stored as
        // bf16 (RNE)
        const int r = rho < 32 ? rho : 32;
        uint16_t f[5];
        f[0] = f32_to_bf16_rne((float)(s01 & 0xffffu) * a.sS);
        f[1] = f32_to_bf16_rne((float)(s01 >> 16) * a.sS);
        f[2] = f32_to_bf16_rne((float)(int)cv * a.sS);
        f[3] = f32_to_bf16_rne((float)d * a.sD);
        f[4] = f32_to_bf16_rne((float)r * a.sR);
        uint4 o;
        o.x = f[0] | ((uint32_t)f[1] << 16);
        o.y = f[2] | ((uint32_t)f[3] << 16);
        o.z = f[4];
        o.w = 0;
        *reinterpret_cast<uint4*>(a.x0 + 8 * px) = o;
    }
}

// Column pass: the window mask of pixel (x, y) is the OR of the row masks of
// rows y - rc .. y + rc.  Sliding-window OR by the van Herk / Gil-Werman
// scheme: with L = 2 rc + 1, a block takes a band of L output rows; the
// window of output row t (band rows t .. t + L - 1 of the input rows
// y0 - rc ..) is the OR of the suffix of the first L input rows from t and
// the prefix of the next L rows up to t + L - 1.  Each input row is read
// twice per band (suffix scan and prefix scan) instead of L times.
// Thread = (column, mask word): lane c NW + w holds word w of column c; the
// nearest-set-bit search runs per word and is reduced over the NW lanes.
constexpr int kColT = 128;   // threads per column-pass block (small: many blocks per CU)

template <int NW>
__global__ __launch_bounds__(kColT) void lidar_colbits_kernel(LidarArgs a)
{
    extern __shared__ uint32_t hbuf[];   // [L][kColT] suffix ORs of the first L rows
    constexpr int TC = kColT / NW;
    const int rc = a.rc, L = 2 * rc + 1;
    const int w = threadIdx.x % NW, c = threadIdx.x / NW;
    const int x = blockIdx.x * TC + c, y0 = blockIdx.y * L, frame = blockIdx.z;
    const bool xin = x < a.W;
    const uint32_t* rb = a.rowbits + (int64_t)frame * a.H * a.W * NW + w;
    auto row = [&](int r) -> uint32_t {
        const int gy = y0 - rc + r;
        return (xin && gy >= 0 && gy < a.H) ? rb[((int64_t)gy * a.W + x) * NW] : 0u;
    };
    // loads in chunks of kC rows, so that a chunk's loads are in flight
    // together instead of one dependent load per row
    constexpr int kC = 48;
    uint32_t h = 0u;
    for (int base = L - 1; base >= 0; base -= kC) {
        uint32_t v[kC];
#pragma unroll
        for (int k = 0; k < kC; ++k) v[k] = base - k >= 0 ? row(base - k) : 0u;
#pragma unroll
        for (int k = 0; k < kC; ++k) {
            if (base - k < 0) break;
            h |= v[k];
            hbuf[(base - k) * kColT + threadIdx.x] = h;
        }
    }
    uint32_t g = 0u;
    const bool owner = xin && w == 0;
    const int64_t px0 = (int64_t)frame * a.px_stride + (int64_t)y0 * a.W + x;
    constexpr int kF = 16;
    for (int t0 = 0; t0 < L; t0 += kF) {
        uint32_t v[kF], s01[kF], cv[kF];
        int dv[kF];
#pragma unroll
        for (int k = 0; k < kF; ++k) {
            const int t = t0 + k;
            // (mask mode reads neither d* nor the features: they are being
            // written by the path passes meanwhile)
            const bool in = t < L && y0 + t < a.H && xin && !a.wmask;
            const int64_t px = px0 + (int64_t)t * a.W;
            v[k] = t > 0 && t < L ? row(t + L - 1) : 0u;
            dv[k] = in ? a.dstar[px] : 0;
            s01[k] = in && w == 0 && a.x0 ? a.feat[2 * px] : 0u;
            cv[k] = in && w == 0 && a.x0 ? a.feat[2 * px + 1] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kF; ++k) {
            const int t = t0 + k;
            if (t >= L || y0 + t >= a.H) break;
            g |= v[k];
            const uint32_t m = hbuf[t * kColT + threadIdx.x] | g;
            const int64_t px = px0 + (int64_t)t * a.W;
            if (a.wmask) {
                // masks only (the residual follows once d* exists)
                if (xin) a.wmask[px * NW + w] = m;
                continue;
            }
            emit_rho<NW>(a, m, dv[k], w, owner, px, s01[k], cv[k]);
        }
    }
}

// Residual and surrogate inputs from window masks computed before d*
// existed (lidar_colbits_kernel with wmask): the same lane layout, one
// pixel per NW lanes.
template <int NW>
__global__ __launch_bounds__(256) void lidar_rho_kernel(LidarArgs a)
{
    const int w = threadIdx.x % NW;
    const int64_t q = (int64_t)blockIdx.x * (256 / NW) + threadIdx.x / NW;   // pixel of the batch
    const int64_t npx = (int64_t)a.W * a.H;
    const int frame = (int)(q / npx);
    const bool in = frame < a.nframes;
    const int64_t px = in ? (int64_t)frame * a.px_stride + (q - (int64_t)frame * npx) : 0;
    const uint32_t m = in ? a.wmask[px * NW + w] : 0u;
    const int d = in ? a.dstar[px] : 0;
    const bool owner = in && w == 0;
    const uint32_t s01 = owner && a.x0 ? a.feat[2 * px] : 0u;
    const uint32_t cv = owner && a.x0 ? a.feat[2 * px + 1] : 0u;
    emit_rho<NW>(a, m, d, w, owner, px, s01, cv);
}

hipError_t launch_lidar_bits(const LidarArgs& a, int nframes, hipStream_t s)
{
    const int NW = a.D / 32;
    dim3 g1((a.W + kRowSeg - 1) / kRowSeg, a.H, nframes);
    if (NW == 2) hipLaunchKernelGGL(lidar_rowbits_kernel<2>, g1, dim3(256), 0, s, a);
    else if (NW == 4) hipLaunchKernelGGL(lidar_rowbits_kernel<4>, g1, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(lidar_rowbits_kernel<8>, g1, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // a band of L = 2 rc + 1 rows per block, kColT / NW columns
    const int L = 2 * a.rc + 1;
    auto col = [&](auto kern) {
        const int TC = kColT / NW;
        dim3 g2((a.W + TC - 1) / TC, (a.H + L - 1) / L, nframes);
        hipLaunchKernelGGL(kern, g2, dim3(kColT), (size_t)L * kColT * 4, s, a);
    };
    if (NW == 2) col(lidar_colbits_kernel<2>);
    else if (NW == 4) col(lidar_colbits_kernel<4>);
    else col(lidar_colbits_kernel<8>);
    return hipGetLastError();
}

// Occlusion margin of the left disparity map, the sixth learned-check input:
// for pixel (x, y) with d = d*, m = min over x' > x of x' - d*(x', y) (the
// leftmost right-image pixel that the pixels to its right map to) and
// v = (x - d) - m, clamped to [-16, 16] (16 where x - d < 0: no matching
// pixel; -16 at the row end); the input is v / 16.  v >= 0 means that a
// pixel further right lands on or left of this pixel's match, as around
// occlusions.  One wave per row: each lane takes a run of pixels, the runs'
// minima are combined right to left across the wave, then each lane walks
// its run from right to left.
__global__ __launch_bounds__(256) void occlusion_kernel(const int16_t* dstar, uint16_t* x0, int W,
                                                        int H, int64_t px_stride)
{
    // per wave: the row's d* and the margins, staged in LDS so that the
    // global reads and writes go pixel by pixel across the lanes
    extern __shared__ int16_t occ_lds[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int y = blockIdx.x * 4 + wv;
    const bool live = y < H;                     // uniform over the wave
    int16_t* sd = occ_lds + (size_t)wv * 2 * W;  // d*, then v in place
    const int64_t row = (int64_t)blockIdx.y * px_stride + (int64_t)min(y, H - 1) * W;
    if (live)
        for (int x = lane; x < W; x += 64) sd[x] = dstar[row + x];
    __syncthreads();
    if (live) {
        const int seg = (W + 63) / 64;
        const int lo = min(lane * seg, W), hi = min(lo + seg, W);
        constexpr int kNone = 1 << 20;           // no pixel to the right
        int run_min = kNone;
        for (int x = lo; x < hi; ++x) run_min = min(run_min, x - (int)sd[x]);
        // minimum over the runs of the lanes to the right (exclusive)
        int incl = run_min;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_down(incl, o, 64);
            incl = lane + o < 64 ? min(incl, v) : incl;
        }
        const int excl = __shfl_down(incl, 1, 64);
        int m = lane < 63 ? excl : kNone;
        int16_t* sv = sd + W;
        for (int x = hi - 1; x >= lo; --x) {
            const int q = x - (int)sd[x];
            sv[x] = (int16_t)(q < 0 ? 16 : max(-16, min(16, q - m)));
            m = min(m, q);
        }
    }
    __syncthreads();
    if (live) {
        const int16_t* sv = sd + W;
        for (int x = lane; x < W; x += 64)
            x0[(row + x) * 8 + 5] = f32_to_bf16_rne((float)sv[x] * (1.0f / 16.0f));
    }
}

hipError_t launch_occlusion(const int16_t* dstar, uint16_t* x0, int W, int H, int64_t px_stride,
                            int nframes, hipStream_t s)
{
    const size_t lds = (size_t)4 * 2 * W * sizeof(int16_t);
    hipLaunchKernelGGL(occlusion_kernel, dim3((H + 3) / 4, nframes), dim3(256), lds, s, dstar, x0,
                       W, H, px_stride);
    return hipGetLastError();
}

hipError_t launch_lidar_rho(const LidarArgs& a0, int nframes, hipStream_t s)
{
    if (!a0.wmask || !a0.dstar || !a0.rho || (a0.x0 && !a0.feat)) return hipErrorInvalidValue;
    const int NW = a0.D / 32;
    LidarArgs a = a0;
    a.nframes = nframes;
    const int64_t lanes = (int64_t)a.W * a.H * nframes * NW;
    dim3 g((unsigned)((lanes + 255) / 256));
    if (NW == 2) hipLaunchKernelGGL(lidar_rho_kernel<2>, g, dim3(256), 0, s, a);
    else if (NW == 4) hipLaunchKernelGGL(lidar_rho_kernel<4>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(lidar_rho_kernel<8>, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sldf
