// SGM path aggregation, one direction per launch, with the joint census + DDC
// cost fused in (Sec. III Eq. 2, Sec. IV-A Eq. 4) and the winner-takes-all +
// subpixel step fused into the last direction (Eq. 3).  Used for the
// one-path debug mode and, two directions per launch, for the split schedule
// of small batches; larger batches run the paired kernel (k_sgm_pair.hip),
// which handles two opposite directions per line.
//
// Every line of the direction is an independent recurrence owned by G = D / 8
// lanes (see sgm_common.h).  The aggregated sum S = sum_r L_r is kept as u16
// in HBM: the first direction stores it, the middle ones add into it and the
// last one adds its own L_r in registers and takes the WTA directly.  All
// values are bounded by the 16-bit limit the host checks, so the modular u16
// arithmetic is exact.
#include "sgm_common.h"

namespace sldf {

template <int G, int MODE, int VIEW>
__device__ __forceinline__ void run_line(const SgmArgs& a, const uint32_t* pat, int line,
                                         int g, int frame, int dx, int dy, uint16_t* S)
{
    constexpr int D = G * 8;
    constexpr bool kLoadS = MODE == kMiddle || MODE == kLast;
    int x0, y0, len;
    line_start(line, a.W, a.H, dx, dy, x0, y0, len);
    const int d0 = g * 8;
    const LineAddr la = line_addr<D, VIEW>(a, frame, x0, y0, d0, dx, dy, S);
    const uint32_t p1x2 = a.p1s * 0x10001u, p2x2 = a.p2s * 0x10001u;
    const bool gfirst = g == 0, glast = g == G - 1;
    uint32_t L[4] = {0, 0, 0, 0};   // zero state: the first step yields L = C
    Edge edge;
    uint32_t m = 0;
    auto step = [&](const StepIn<4>& in, const u32x4& s_in, int t) {
        uint32_t C[4];
        cost_lane<D, VIEW>(a, reinterpret_cast<const char*>(pat) + 2 * d0, in, x0 + t * dx, d0, C);
        rec_lane<G>(L, m, C, p1x2, p2x2, gfirst, glast, edge);
        const PixOff o = la.at(t);
        if (MODE == kFirst) {
            store_s(la, o, L);
        } else if (MODE == kMiddle) {
            uint32_t v[4] = {pk_add(s_in.x, L[0]), pk_add(s_in.y, L[1]), pk_add(s_in.z, L[2]),
                             pk_add(s_in.w, L[3])};
            store_s(la, o, v);
        } else {
            uint32_t St[4];
            if (MODE == kLast) {
                St[0] = pk_add(s_in.x, L[0]); St[1] = pk_add(s_in.y, L[1]);
                St[2] = pk_add(s_in.z, L[2]); St[3] = pk_add(s_in.w, L[3]);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) St[i] = L[i];
            }
            if (a.store_sum) store_s(la, o, St);
            const uint32_t px = (uint32_t)((y0 + t * dy) * a.W + x0 + t * dx);
            wta_emit<G, VIEW>(a, St, d0, (size_t)frame * a.px_stride + px);
        }
    };
    // three steps in flight: the loads of step t+3 are issued once step t
    // has consumed its buffer
    StepIn<4> b0, b1, b2;
    u32x4 s0 = {}, s1 = {}, s2 = {};
    auto load = [&](StepIn<4>& b, u32x4& sv, int t) {
        const PixOff o = la.at(t);
        load_pixel<VIEW>(la, o, b);
        if (kLoadS) sv = load_s(la, o);
    };
    load(b0, s0, 0);
    if (len > 1) load(b1, s1, 1);
    if (len > 2) load(b2, s2, 2);
    for (int t = 0; t < len; t += 3) {
        step(b0, s0, t);
        if (t + 3 < len) load(b0, s0, t + 3);
        if (t + 1 >= len) break;
        step(b1, s1, t + 1);
        if (t + 4 < len) load(b1, s1, t + 4);
        if (t + 2 >= len) break;
        step(b2, s2, t + 2);
        if (t + 5 < len) load(b2, s2, t + 5);
    }
}

// One direction of the split schedule (MODE kFirst: S = L_r, kMiddle:
// S += L_r).  As in the paired pass, the line is padded at its start to a
// whole number of kRing positions with virtual positions that read the
// guard position before the line start (cost 0: the state stays zero and
// their S update is a no-op on pixel 0, stored before pixel 0's own), so
// every step loads, computes and stores unconditionally and the inputs and
// S of kRing positions ahead are in flight.
template <int G, int MODE, int VIEW, int NR>
__device__ __forceinline__ void run_line_split(const SgmArgs& a, const uint32_t* pat, int line,
                                               int g, int frame, int dx, int dy, uint16_t* S)
{
    constexpr int K = 2 * NR, D = G * K;   // K disparities per lane
    constexpr bool kLoadS = MODE == kMiddle;
    constexpr int kRing = 8;
    int x0, y0, len;
    line_start(line, a.W, a.H, dx, dy, x0, y0, len);
    const int d0 = g * K;
    const LineAddr la = line_addr<D, VIEW, K>(a, frame, x0, y0, d0, dx, dy, S);
    const uint32_t p1x2 = a.p1s * 0x10001u, p2x2 = a.p2s * 0x10001u;
    const bool gfirst = g == 0, glast = g == G - 1;
    const char* patl = reinterpret_cast<const char*>(pat) + 2 * d0;
    const int pad = (len + kRing - 1) / kRing * kRing - len;
    const int nu = len + pad;
    uint32_t L[NR] = {};
    uint32_t m = 0;
    Edge edge;
    StepIn<NR> R[kRing];
    vecT<NR> SR[kRing];
    auto load = [&](int i, int u) {
        load_pixel<VIEW>(la, la.at(max(u - pad, -1)), R[i]);
        if (kLoadS) SR[i] = load_s<NR>(la, la.at(min(max(u - pad, 0), len - 1)));
    };
    // issued in slot order (the loop's waits assume slot 0 is the oldest)
#pragma unroll
    for (int i = 0; i < kRing; ++i) {
        load(i, i);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int u0 = 0; u0 < nu; u0 += kRing) {
#pragma unroll
        for (int i = 0; i < kRing; ++i) {
            const int u = u0 + i;
            uint32_t C[NR];
            cost_lane<D, VIEW, NR>(a, patl, R[i], x0 + (u - pad) * dx, d0, C);
            rec_lane<G, NR>(L, m, C, p1x2, p2x2, gfirst, glast, edge);
            uint32_t v[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) v[q] = kLoadS ? pk_add(L[q], SR[i][q]) : L[q];
            store_s<NR>(la, la.at(max(u - pad, 0)), v);
            load(i, min(u + kRing, nu - 1));
        }
    }
}

template <int G, int MODE, int NR>
__global__ __launch_bounds__(256) void sgm_dir_kernel(SgmArgs a)
{
    // raised issue priority: on single frames this pass heads the longer of
    // the two concurrent chains and shares its SIMDs with the other chain's
    // pairs (measured: graph-replay p99 0.85 -> 0.82 ms; raising the pair
    // after it too starves the other chain and is slower)
    __builtin_amdgcn_s_setprio(3);
    constexpr int D = G * 2 * NR;
    __shared__ uint32_t pat[pattern_words(D)];
    build_pattern<D>(a, pat);
    __syncthreads();
    // XCD-aware mapping: blocks are dispatched round-robin over the 8 XCDs
    // (physical block b runs on XCD b % 8).  Give each XCD a contiguous range
    // of logical blocks, so the lines of one frame-view share one L2 and its
    // copy of that view's census rows.
    const int nb = gridDim.x;                 // a multiple of kXcds
    const int b = blockIdx.x;
    const int logical = (b % kXcds) * (nb / kXcds) + b / kXcds;
    const int fv = logical / a.blocks_per_fv;
    if (fv >= a.n_fv) return;
    const int view = a.view_base + fv % a.nviews, frame = fv / a.nviews;
    if (a.gate && a.gate[frame] <= a.gate_limit) return;   // fallback not needed
    const int g = threadIdx.x % G;
    const int line = (logical - fv * a.blocks_per_fv) * (256 / G) + threadIdx.x / G;
    if (line >= a.nlines) return;
    // blockIdx.y = 1 (split schedule): the opposite direction, into S2
    const int sg = blockIdx.y ? -1 : 1;
    uint16_t* S = blockIdx.y ? a.S2[view] : a.S[view];
    if constexpr (MODE == kFirst || MODE == kMiddle) {
        if (view == 0)
            run_line_split<G, MODE, 0, NR>(a, pat, line, g, frame, sg * a.dx, sg * a.dy, S);
        else
            run_line_split<G, MODE, 1, NR>(a, pat, line, g, frame, sg * a.dx, sg * a.dy, S);
    } else {
        if (view == 0)
            run_line<G, MODE, 0>(a, pat, line, g, frame, a.dx, a.dy, S);
        else
            run_line<G, MODE, 1>(a, pat, line, g, frame, a.dx, a.dy, S);
    }
}

template <int G>
static void launch_g(const SgmArgs& a, int mode, dim3 grid, hipStream_t s)
{
    switch (mode) {
    case kFirst: hipLaunchKernelGGL((sgm_dir_kernel<G, kFirst, 4>), grid, dim3(256), 0, s, a); break;
    case kMiddle: hipLaunchKernelGGL((sgm_dir_kernel<G, kMiddle, 4>), grid, dim3(256), 0, s, a); break;
    case kLast: hipLaunchKernelGGL((sgm_dir_kernel<G, kLast, 4>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((sgm_dir_kernel<G, kSingle, 4>), grid, dim3(256), 0, s, a); break;
    }
}

// four disparities per lane: the split passes of single-frame runs
template <int G>
static void launch_g2(const SgmArgs& a, int mode, dim3 grid, hipStream_t s)
{
    if (mode == kFirst)
        hipLaunchKernelGGL((sgm_dir_kernel<G, kFirst, 2>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((sgm_dir_kernel<G, kMiddle, 2>), grid, dim3(256), 0, s, a);
}

static hipError_t launch_dir(const SgmArgs& a0, int D, int mode, int nviews, int nframes,
                             int ndirs, hipStream_t s, int k = 8)
{
    if (k == 4 && (D > 128 || (mode != kFirst && mode != kMiddle))) return hipErrorInvalidValue;
    const int G = D / k;
    const int lines_per_block = 256 / G;
    SgmArgs a = a0;
    a.blocks_per_fv = (a.nlines + lines_per_block - 1) / lines_per_block;
    a.nviews = nviews;
    a.n_fv = nviews * nframes;
    const int64_t nb = (int64_t)a.blocks_per_fv * a.n_fv;
    dim3 grid((unsigned)((nb + kXcds - 1) / kXcds * kXcds), ndirs);
    if (k == 4) {
        if (G == 16) launch_g2<16>(a, mode, grid, s);
        else launch_g2<32>(a, mode, grid, s);
    } else if (G == 8) {
        launch_g<8>(a, mode, grid, s);
    } else if (G == 16) {
        launch_g<16>(a, mode, grid, s);
    } else {
        launch_g<32>(a, mode, grid, s);
    }
    return hipGetLastError();
}

// Joint cost tap: C'(p, d) of frame 0's left view for every pixel, computed
// as the path passes compute it (cost_lane) and stored as [H][W][D] u16.
// G lanes per pixel, each with 8 disparities.
template <int G>
__global__ __launch_bounds__(256) void cost_tap_kernel(SgmArgs a, uint16_t* out)
{
    constexpr int D = G * 8;
    __shared__ uint32_t pat[pattern_words(D)];
    build_pattern<D>(a, pat);
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    if (q >= (int64_t)a.W * a.H) return;
    const int g = threadIdx.x % G, d0 = 8 * g;
    const int y = (int)(q / a.W), x = (int)(q - (int64_t)y * a.W);
    const LineAddr la = line_addr<D, 0>(a, 0, 0, y, d0, 1, 0, a.S[0]);
    StepIn<4> in;
    load_pixel<0>(la, la.at(x), in);
    uint32_t C[4];
    cost_lane<D, 0>(a, reinterpret_cast<const char*>(pat) + 2 * d0, in, x, d0, C);
    *reinterpret_cast<u32x4*>(out + q * D + d0) = pack_v<4>(C);
}

hipError_t launch_cost_tap(const SgmArgs& a, int D, uint16_t* out, hipStream_t s)
{
    const int G = D / 8;
    const int64_t n = (int64_t)a.W * a.H;
    dim3 grid((unsigned)((n + 256 / G - 1) / (256 / G)));
    if (G == 8) hipLaunchKernelGGL(cost_tap_kernel<8>, grid, dim3(256), 0, s, a, out);
    else if (G == 16) hipLaunchKernelGGL(cost_tap_kernel<16>, grid, dim3(256), 0, s, a, out);
    else hipLaunchKernelGGL(cost_tap_kernel<32>, grid, dim3(256), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_sgm_dir(const SgmArgs& a, int D, int mode, int nviews, int nframes,
                          hipStream_t s)
{
    return launch_dir(a, D, mode, nviews, nframes, 1, s);
}

// Split schedule (small batches): the two directions of a pair run as
// independent lines, r into S and -r into S2, so a line is one pass of
// its length instead of three (forward, recompute, backward) and the two
// run side by side; S + S2 is taken by sgm_wta_kernel after the last pair.
hipError_t launch_sgm_dual(const SgmArgs& a, int D, int mode, int nviews, int nframes,
                           hipStream_t s, int k)
{
    return launch_dir(a, D, mode, nviews, nframes, 2, s, k);
}

// Winner-takes-all (+ subpixel, cost features) on S + S2: G lanes per pixel,
// each with its 8 disparities; the pixel's summed costs are staged in LDS
// for the parabola neighbours.  With store_sum the sum is written back to S
// (the cost-sum tap).
template <int G>
__global__ __launch_bounds__(256) void sgm_wta_kernel(SgmArgs a, int64_t npx_fv)
{
    constexpr int D = G * 8;
    __shared__ u32x4 simg[256];
    const int64_t q = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;   // pixel-view
    const int g = threadIdx.x % G;
    const int fv = (int)(q / npx_fv);
    if (fv >= a.n_fv) return;
    const int view = a.view_base + fv % a.nviews, frame = fv / a.nviews;
    if (a.gate && a.gate[frame] <= a.gate_limit) return;
    const int64_t p = q - (int64_t)fv * npx_fv;
    const size_t off = (size_t)frame * a.S_stride + (size_t)p * D + 8 * g;
    const u32x4 s1 = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(a.S[view] + off));
    const u32x4 s2 = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(a.S2[view] + off));
    const uint32_t St[4] = {pk_add(s1.x, s2.x), pk_add(s1.y, s2.y), pk_add(s1.z, s2.z),
                            pk_add(s1.w, s2.w)};
    const size_t px = (size_t)frame * a.px_stride + (size_t)p;
    if (view == 0) {
        if (a.store_sum)
            *reinterpret_cast<u32x4*>(a.S[0] + off) = u32x4{St[0], St[1], St[2], St[3]};
        simg[threadIdx.x] = u32x4{St[0], St[1], St[2], St[3]};
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        wta_emit<G, 0>(a, St, 8 * g, px,
                       reinterpret_cast<const uint16_t*>(&simg[threadIdx.x - g]));
    } else {
        wta_emit<G, 1>(a, St, 8 * g, px);
    }
}

hipError_t launch_sgm_wta(const SgmArgs& a0, int D, int nviews, int nframes, hipStream_t s)
{
    const int G = D / 8;
    SgmArgs a = a0;
    a.nviews = nviews;
    a.n_fv = nviews * nframes;
    const int64_t npx = (int64_t)a.W * a.H;
    const int64_t nb = (npx * a.n_fv + 256 / G - 1) / (256 / G);
    dim3 grid((unsigned)nb);
    if (G == 8) hipLaunchKernelGGL(sgm_wta_kernel<8>, grid, dim3(256), 0, s, a, npx);
    else if (G == 16) hipLaunchKernelGGL(sgm_wta_kernel<16>, grid, dim3(256), 0, s, a, npx);
    else hipLaunchKernelGGL(sgm_wta_kernel<32>, grid, dim3(256), 0, s, a, npx);
    return hipGetLastError();
}

}  // namespace sldf
