// SGM path aggregation for a pair of opposite directions r and -r in one
// launch (Sec. III, Eq. 2), with the joint cost fused in (Eq. 4) and, for
// the last pair, the winner-takes-all + subpixel step (Eq. 3).
//
// Opposite directions walk the same lines in opposite orders.  For each line
// (owned by G = D / 8 lanes, see sgm_common.h):
//   1. the forward direction r runs over the line and stores its state L_r
//      every kSeg pixels (a checkpoint per segment, 1 / kSeg of the cost
//      volume) in a scratch buffer;
//   2. the segments are then visited from the last to the first: the
//      forward states of the segment are recomputed from the checkpoint into
//      registers (with the joint costs of its pixels), and the backward
//      direction -r, whose state runs on continuously, walks the segment in
//      reverse and adds L_r + L_-r into S (or takes the WTA).
// S is therefore read and written once per pair instead of once per
// direction; the price is one extra forward recurrence per pixel (the
// costs are computed twice, as in two separate passes).
#include "sgm_common.h"

namespace sldf {

constexpr int kSeg = 8;   // checkpoint interval (pixels per segment)
// depth of the census / prior prefetch ring: 4 positions, 2 in the last pair
// (whose WTA needs the registers; the census rows mostly come from L2)
template <int MODE, int NR>
constexpr int ring_depth() { return MODE == kLast ? 2 : 4; }

template <int G, int MODE, int VIEW, int NR>
__device__ __forceinline__ void run_pair(const SgmArgs& a, const uint32_t* pat, vecT<NR>* cw,
                                         int line, int g, int frame, int fv)
{
    constexpr int K = 2 * NR, D = G * K;   // K disparities per lane
    constexpr bool kLoadS2 = MODE == kMiddle2;
    constexpr bool kLoadS = MODE == kMiddle || MODE == kLast || kLoadS2;
    constexpr bool kStoreS = MODE == kFirst || MODE == kMiddle || kLoadS2;
    constexpr int kRing = ring_depth<MODE, NR>();
    // slot j % kRing of a segment must be slot j % kRing of the next one
    static_assert(kSeg % kRing == 0, "the ring depth must divide the segment length");
    int x0, y0, len;
    line_start(line, a.W, a.H, a.dx, a.dy, x0, y0, len);
    const int d0 = g * K;
    const LineAddr la = line_addr<D, VIEW, K>(a, frame, x0, y0, d0, a.dx, a.dy, a.S[VIEW]);
    // kMiddle2: the second term S2 of the split first pass, folded into S here
    const LineAddr la2 =
        kLoadS2 ? line_addr<D, VIEW, K>(a, frame, x0, y0, d0, a.dx, a.dy, a.S2[VIEW]) : la;
    uint32_t* __restrict__ ck =
        a.ckpt + (((size_t)fv * a.nlines + line) * a.ckpt_segs * G + g) * NR;
    const uint32_t p1x2 = a.p1s * 0x10001u, p2x2 = a.p2s * 0x10001u;
    const bool gfirst = g == 0, glast = g == G - 1;
    Edge edge;

    // The line is cut into nseg segments of kSeg positions; `pad` virtual
    // positions before pixel 0 fill the first one.  Position u maps to pixel
    // t = u - pad.  Virtual positions (and prefetches before the line) read
    // the position t = -1 before the line start, whose cost is 0 (see
    // cost_lane), so every step below runs unconditionally; only S stores and
    // the WTA are skipped for them.
    const int nseg = (len + kSeg - 1) / kSeg;
    const int pad = nseg * kSeg - len;
    const char* patl = reinterpret_cast<const char*>(pat) + 2 * d0;
    auto load = [&](StepIn<NR>& b, int u) { load_pixel<VIEW>(la, la.at(max(u - pad, -1)), b); };
    auto sat = [&](int u) { return la.at(max(u - pad, 0)); };
    auto cost = [&](const StepIn<NR>& in, int u, uint32_t C[NR]) {
        cost_lane<D, VIEW, NR>(a, patl, in, x0 + (u - pad) * a.dx, d0, C);
    };
    auto ckpt = [&](int q) { return reinterpret_cast<vecT<NR>*>(ck + (size_t)q * G * NR); };

    // ---- 1. forward direction r over segments 0 .. nseg-2, checkpoints ----
    // R[j % kRing] holds the inputs of position u = kSeg q + j; each slot is
    // reloaded with position u + kRing as soon as it has been used.
    StepIn<NR> R[kRing];
#pragma unroll
    for (int j = 0; j < kRing; ++j) load(R[j], j);
    {
        uint32_t L[NR] = {};
        uint32_t m = 0;
        for (int q = 0; q < nseg - 1; ++q) {
#pragma unroll
            for (int j = 0; j < kSeg; ++j) {
                uint32_t C[NR];
                cost(R[j % kRing], q * kSeg + j, C);
                load(R[j % kRing], q * kSeg + j + kRing);
                rec_lane<G, NR>(L, m, C, p1x2, p2x2, gfirst, glast, edge);
            }
            *ckpt(q) = pack_v<NR>(L);
        }
    }

    // ---- 2. segments from the last to the first ----
    // The forward states of a segment are recomputed from its checkpoint;
    // the backward direction -r then walks the segment in reverse and adds
    // L_r + L_-r into S (or takes the WTA).  While segment s is walked, the
    // inputs, checkpoint and S of segment s - 1 are already in flight.
    vecT<NR> Sin[kSeg], Sin2[kLoadS2 ? kSeg : 1];
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        Sin[j] = kLoadS ? load_s<NR>(la, sat((nseg - 1) * kSeg + j)) : vecT<NR>{};
        if (kLoadS2) Sin2[j] = load_s<NR>(la2, sat((nseg - 1) * kSeg + j));
    }
    // forward state entering a segment: its checkpoint (zero for the first
    // segment), with the group minimum; prepared one iteration ahead
    uint32_t Ln[NR], mn;
    auto enter = [&](const vecT<NR>& c, bool zero) {
#pragma unroll
        for (int i = 0; i < NR; ++i) Ln[i] = zero ? 0u : c[i];
        mn = group_min<G>(lane_min<NR>(Ln));
    };
    enter(*ckpt(max(nseg - 2, 0)), nseg == 1);
    uint32_t Lb[NR] = {};
    uint32_t mb = 0;
    for (int s = nseg - 1; s >= 0; --s) {
        const int u0 = s * kSeg;
        // issued first in the iteration (and kept there), so that every load
        // after it may still be in flight when it is consumed at the end
        const vecT<NR> cin = *ckpt(max(s - 2, 0));
        __builtin_amdgcn_sched_barrier(0);
        uint32_t Lf[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) Lf[i] = Ln[i];
        uint32_t mf = mn;
        // the joint costs of the segment go to this lane's slots in LDS
        // (cw[j * 64]), the forward states stay in registers
        uint32_t Lbuf[kSeg][NR];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            uint32_t C[NR];
            cost(R[j % kRing], u0 + j, C);
            // the slot moves on to position j + kRing of this segment, or past
            // its end to the start of segment s - 1
            load(R[j % kRing], j + kRing < kSeg ? u0 + j + kRing : u0 + j + kRing - 2 * kSeg);
            cw[j * 64] = pack_v<NR>(C);
            rec_lane<G, NR>(Lf, mf, C, p1x2, p2x2, gfirst, glast, edge);
#pragma unroll
            for (int i = 0; i < NR; ++i) Lbuf[j][i] = Lf[i];
        }
#pragma unroll
        for (int j = kSeg - 1; j >= 0; --j) {
            const vecT<NR> cv = cw[j * 64];
            uint32_t C[NR];
#pragma unroll
            for (int i = 0; i < NR; ++i) C[i] = cv[i];
            rec_lane<G, NR>(Lb, mb, C, p1x2, p2x2, gfirst, glast, edge);
            uint32_t St[NR];
#pragma unroll
            for (int i = 0; i < NR; ++i) St[i] = pk_add(Lbuf[j][i], Lb[i]);
            if (kLoadS) {
#pragma unroll
                for (int i = 0; i < NR; ++i) St[i] = pk_add(St[i], Sin[j][i]);
            }
            if (kLoadS2) {
#pragma unroll
                for (int i = 0; i < NR; ++i) St[i] = pk_add(St[i], Sin2[j][i]);
            }
            const int u = u0 + j;
            if (u >= pad) {
                const PixOff o = la.at(u - pad);
                if (kStoreS) {
                    store_s<NR>(la, o, St);
                } else {
                    if (a.store_sum) store_s<NR>(la, o, St);
                    const int t = u - pad;
                    const uint32_t px = (uint32_t)((y0 + t * a.dy) * a.W + x0 + t * a.dx);
                    // the segment cost slot j is free now: it takes S(p, .)
                    // so that the WTA reads the neighbours of d* from LDS
                    const uint16_t* simg = nullptr;
                    if (VIEW == 0) {
                        cw[j * 64] = pack_v<NR>(St);
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        simg = reinterpret_cast<const uint16_t*>(cw + j * 64 - g);
                    }
                    wta_emit<G, VIEW, NR>(a, St, d0, (size_t)frame * a.px_stride + px, simg);
                }
            }
            if (kLoadS) Sin[j] = load_s<NR>(la, sat(u - kSeg));
            if (kLoadS2) Sin2[j] = load_s<NR>(la2, sat(u - kSeg));
        }
        enter(cin, s == 1);
    }
}

template <int G, int MODE, int NR>
__global__ __launch_bounds__(256) void sgm_pair_kernel(SgmArgs a)
{
    constexpr int D = G * 2 * NR;
    __shared__ uint32_t pat[pattern_words(D)];
    __shared__ vecT<NR> cbuf[256 / 64][kSeg][64];   // per wave: segment costs
    build_pattern<D>(a, pat);
    __syncthreads();
    // XCD-aware mapping (blocks are dispatched round-robin over the XCDs):
    // each XCD takes a contiguous range of logical blocks, i.e. the lines of
    // one frame-view, which share its L2 copy of the census rows
    const int nb = gridDim.x;
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
        run_pair<G, MODE, 0, NR>(a, pat, &cbuf[threadIdx.x / 64][0][threadIdx.x % 64], line, g,
                                 frame, fv);
    else
        run_pair<G, MODE, 1, NR>(a, pat, &cbuf[threadIdx.x / 64][0][threadIdx.x % 64], line, g,
                                 frame, fv);
}

template <int G>
static void launch_pg(const SgmArgs& a, int mode, dim3 grid, hipStream_t s)
{
    switch (mode) {
    case kFirst: hipLaunchKernelGGL((sgm_pair_kernel<G, kFirst, 4>), grid, dim3(256), 0, s, a); break;
    case kMiddle: hipLaunchKernelGGL((sgm_pair_kernel<G, kMiddle, 4>), grid, dim3(256), 0, s, a); break;
    case kMiddle2: hipLaunchKernelGGL((sgm_pair_kernel<G, kMiddle2, 4>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((sgm_pair_kernel<G, kLast, 4>), grid, dim3(256), 0, s, a); break;
    }
}

int64_t sgm_pair_ckpt_segs(int W, int H, int dx, int dy)
{
    const int maxlen = dy == 0 ? W : dx == 0 ? H : (W < H ? W : H);
    return (maxlen + kSeg - 1) / kSeg;
}

hipError_t launch_sgm_pair(const SgmArgs& a0, int D, int mode, int nviews, int nframes,
                           hipStream_t s)
{
    const int G = D / 8;
    const int lines_per_block = 256 / G;
    SgmArgs a = a0;
    a.blocks_per_fv = (a.nlines + lines_per_block - 1) / lines_per_block;
    a.nviews = nviews;
    a.n_fv = nviews * nframes;
    a.ckpt_segs = (int32_t)sgm_pair_ckpt_segs(a.W, a.H, a.dx, a.dy);
    const int64_t nb = (int64_t)a.blocks_per_fv * a.n_fv;
    dim3 grid((unsigned)((nb + kXcds - 1) / kXcds * kXcds));
    if (G == 8) launch_pg<8>(a, mode, grid, s);
    else if (G == 16) launch_pg<16>(a, mode, grid, s);
    else launch_pg<32>(a, mode, grid, s);
    return hipGetLastError();
}

}  // namespace sldf
