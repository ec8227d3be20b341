// SGM path aggregation, one direction per launch, with the joint census + DDC
// cost fused in (Sec. III Eq. 2, Sec. IV-A Eq. 4) and the winner-takes-all +
// subpixel step fused into the last direction (Eq. 3).  Used for the
// one-path debug mode; the 4- and 8-path sets run the paired kernel
// (k_sgm_pair.hip), which handles two opposite directions per launch.
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
                                         int g, int frame)
{
    constexpr int D = G * 8;
    constexpr bool kLoadS = MODE == kMiddle || MODE == kLast;
    int x0, y0, len;
    line_start(line, a.W, a.H, a.dx, a.dy, x0, y0, len);
    const int d0 = g * 8;
    const LineAddr la = line_addr<D, VIEW>(a, frame, x0, y0, d0);
    const uint32_t p1x2 = a.p1s * 0x10001u, p2x2 = a.p2s * 0x10001u;
    const bool gfirst = g == 0, glast = g == G - 1;
    uint32_t L[4] = {0, 0, 0, 0};   // zero state: the first step yields L = C
    Edge edge;
    uint32_t m = 0;
    auto step = [&](const StepIn& in, const u32x4& s_in, int t) {
        uint32_t C[4];
        cost8<D, VIEW>(a, reinterpret_cast<const char*>(pat) + 2 * d0, in, x0 + t * a.dx, d0, C);
        rec8<G>(L, m, C, p1x2, p2x2, gfirst, glast, edge);
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
            const uint32_t px = (uint32_t)((y0 + t * a.dy) * a.W + x0 + t * a.dx);
            wta_emit<G, VIEW>(a, St, d0, (size_t)frame * a.px_stride + px);
        }
    };
    // three steps in flight: the loads of step t+3 are issued once step t
    // has consumed its buffer
    StepIn b0, b1, b2;
    u32x4 s0 = {}, s1 = {}, s2 = {};
    auto load = [&](StepIn& b, u32x4& sv, int t) {
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

template <int G, int MODE>
__global__ __launch_bounds__(256) void sgm_dir_kernel(SgmArgs a)
{
    constexpr int D = G * 8;
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
    if (view == 0)
        run_line<G, MODE, 0>(a, pat, line, g, frame);
    else
        run_line<G, MODE, 1>(a, pat, line, g, frame);
}

template <int G>
static void launch_g(const SgmArgs& a, int mode, dim3 grid, hipStream_t s)
{
    switch (mode) {
    case kFirst: hipLaunchKernelGGL((sgm_dir_kernel<G, kFirst>), grid, dim3(256), 0, s, a); break;
    case kMiddle: hipLaunchKernelGGL((sgm_dir_kernel<G, kMiddle>), grid, dim3(256), 0, s, a); break;
    case kLast: hipLaunchKernelGGL((sgm_dir_kernel<G, kLast>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((sgm_dir_kernel<G, kSingle>), grid, dim3(256), 0, s, a); break;
    }
}

hipError_t launch_sgm_dir(const SgmArgs& a0, int D, int mode, int nviews, int nframes,
                          hipStream_t s)
{
    const int G = D / 8;
    const int lines_per_block = 256 / G;
    SgmArgs a = a0;
    a.blocks_per_fv = (a.nlines + lines_per_block - 1) / lines_per_block;
    a.nviews = nviews;
    a.n_fv = nviews * nframes;
    const int64_t nb = (int64_t)a.blocks_per_fv * a.n_fv;
    dim3 grid((unsigned)((nb + kXcds - 1) / kXcds * kXcds));
    if (G == 8) launch_g<8>(a, mode, grid, s);
    else if (G == 16) launch_g<16>(a, mode, grid, s);
    else launch_g<32>(a, mode, grid, s);
    return hipGetLastError();
}

}  // namespace sldf
