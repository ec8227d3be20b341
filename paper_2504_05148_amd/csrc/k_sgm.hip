// SGM path aggregation with the joint census + DDC cost fused in, and the
// winner-takes-all + subpixel step fused into the last path.
//
// One launch handles one path direction r = (dx, dy) for both views and all
// frames of a batch.  Every line of that direction (a row, a column or a
// diagonal) is an independent recurrence (Sec. III, Eq. 2):
//   L_r(p,d) = C(p,d) + min(L_r(p-r,d), L_r(p-r,d+-1) + P1, m + P2) - m,
//   m = min_k L_r(p-r,k),   L_r = C at the start of the line.
// A line is owned by a group of G = D / 8 lanes of one wavefront; lane g of
// the group holds disparities [8g, 8g + 8) as four packed 2 x u16 registers,
// so one VALU instruction (v_pk_*_u16) advances two disparities.  The d +- 1
// neighbours across lane boundaries come from one wave_shr / wave_shl DPP
// move each, and the running minimum over d is an in-lane packed minimum
// followed by a DPP butterfly inside the group (quad_perm, half-row mirror,
// row mirror and, for 32-lane groups, a permlane16 swap).  No MFMA: the path
// is integer min-plus arithmetic.
//
// The joint cost C'(p,d) = (den - num) H(p,d) + num DDC(d, prior_p)
// (Sec. IV-A, Eq. 4, scaled by den = alpha denominator so every term is an
// integer) is rebuilt at every step from the census codes (xor + popcount)
// and a per-block LDS table of the DDC pattern, so the cost volume is never
// materialised.  The aggregated sum S = sum_r L_r (Eq. 3) is kept as u16 in
// HBM: the first direction stores it, the middle ones add into it, and the
// last one adds its own L_r in registers and takes the WTA (ties -> smallest
// d) and the parabola fit through S(d*-1), S(d*), S(d*+1) directly.
// All values are bounded by the 16-bit limit that the host checks, so the
// modular u16 arithmetic is exact.
#include "sldf_internal.h"

namespace sldf {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u16x2 v2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t u1(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b)
{
    return u1(__builtin_elementwise_min(v2(a), v2(b)));
}
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) { return u1(v2(a) + v2(b)); }
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) { return u1(v2(a) - v2(b)); }
__device__ __forceinline__ uint32_t pk_mad(uint32_t a, uint32_t b, uint32_t c)
{
    return u1(v2(a) * v2(b) + v2(c));
}

// DPP controls (GFX9 encoding)
constexpr int kQuadXor1 = 0xB1;        // quad_perm:[1,0,3,2]
constexpr int kQuadXor2 = 0x4E;        // quad_perm:[2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kWaveShr1 = 0x138;       // lane i <- lane i-1
constexpr int kWaveShl1 = 0x130;       // lane i <- lane i+1

constexpr int kXcds = 8;               // MI355X: 8 XCDs, one L2 each

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return __builtin_amdgcn_update_dpp(0u, v, CTRL, 0xf, 0xf, true);
}

// Minimum over the G lanes of a group, broadcast to all of them.
template <int G>
__device__ __forceinline__ uint32_t group_min(uint32_t v)
{
    v = min(v, dpp<kQuadXor1>(v));
    v = min(v, dpp<kQuadXor2>(v));
    v = min(v, dpp<kRowHalfMirror>(v));
    if (G >= 16) v = min(v, dpp<kRowMirror>(v));
    if (G >= 32) {
        auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = min(sw[0], sw[1]);
    }
    return v;
}

__device__ __forceinline__ void line_start(int line, int W, int H, int dx, int dy, int& x,
                                           int& y, int& len)
{
    if (dy == 0) {
        y = line;
        x = dx > 0 ? 0 : W - 1;
        len = W;
    } else if (dx == 0) {
        x = line;
        y = dy > 0 ? 0 : H - 1;
        len = H;
    } else {
        if (line < W) {
            x = line;
            y = dy > 0 ? 0 : H - 1;
        } else {
            int k = line - W + 1;
            x = dx > 0 ? 0 : W - 1;
            y = dy > 0 ? k : H - 1 - k;
        }
        int nx = dx > 0 ? W - x : x + 1;
        int ny = dy > 0 ? H - y : y + 1;
        len = nx < ny ? nx : ny;
    }
}

// Inputs of one step (one pixel of the line) for one lane, loaded a few
// steps ahead of their use.
struct StepIn {
    uint32_t cb;        // census of the base pixel
    u32x4a4 m0, m1;     // census of 8 consecutive matching pixels
    int32_t e;          // prior disparity (-1 = none)
    u32x4 s;            // partial S of the lane's 8 d (middle / last passes)
};

// Offsets of the current pixel, advanced by a constant per step.
struct Cursor {
    int x, y;
    uint32_t oc;    // census offset  y * census_pitch + x + D (padded row)
    uint32_t op;    // prior offset   y * prior_pitch + x
    uint32_t opx;   // pixel offset   y * W + x
};

template <int D, int VIEW, bool LOAD_S>
__device__ __forceinline__ void load_step(const uint32_t* __restrict__ cbase,
                                          const uint32_t* __restrict__ cmatch,
                                          const int16_t* __restrict__ prior,
                                          const uint16_t* __restrict__ S, const Cursor& c,
                                          int d0, StepIn& st)
{
    st.cb = cbase[c.oc];
    // matching pixels: x - d (left base, descending) or x + d (right base)
    // for d = d0 .. d0+7; the census pad keeps both runs inside the buffer
    const uint32_t om = VIEW == 0 ? c.oc - (uint32_t)(d0 + 7) : c.oc + (uint32_t)d0;
    st.m0 = *reinterpret_cast<const u32x4a4*>(cmatch + om);
    st.m1 = *reinterpret_cast<const u32x4a4*>(cmatch + om + 4);
    if (VIEW == 0) st.e = prior ? (int32_t)prior[c.op] : -1;
    // S streams through once per pass: non-temporal, so it does not evict
    // the census rows that neighbouring lines re-read from L2
    if (LOAD_S) st.s = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(S + (size_t)c.opx * D + d0));
}

template <int G, int MODE, int VIEW>
__device__ __forceinline__ void run_line(const SgmArgs& a, const uint32_t* pat, int line,
                                         int g, int frame)
{
    constexpr int D = G * 8;
    constexpr bool kLoadS = MODE == kMiddle || MODE == kLast;
    int x0, y0, len;
    line_start(line, a.W, a.H, a.dx, a.dy, x0, y0, len);
    const int d0 = g * 8;
    // census rows are addressed from their padded start (pixel x at x + D),
    // so every offset below is non-negative
    const uint32_t* __restrict__ cbase = a.cbase[VIEW] - D + (int64_t)frame * a.census_fstride;
    const uint32_t* __restrict__ cmatch = a.cmatch[VIEW] - D + (int64_t)frame * a.census_fstride;
    const int16_t* __restrict__ prior =
        VIEW == 0 && a.prior ? a.prior + (int64_t)frame * a.prior_fstride : nullptr;
    uint16_t* __restrict__ S = a.S[VIEW] + (int64_t)frame * a.S_stride;
    const uint32_t p1x2 = a.p1s * 0x10001u;
    const uint32_t nfill = (uint32_t)a.n;
    const bool gfirst = g == 0, glast = g == G - 1;
    const int W = a.W;
    // per-step offset increments
    const uint32_t dc = (uint32_t)(a.dy * a.census_pitch + a.dx);
    const uint32_t dp = (uint32_t)(a.dy * a.prior_pitch + a.dx);
    const uint32_t dpx = (uint32_t)(a.dy * W + a.dx);

    Cursor cl;   // cursor of the next load
    cl.x = x0;
    cl.y = y0;
    cl.oc = (uint32_t)(y0 * a.census_pitch + x0 + D);
    cl.op = (uint32_t)(y0 * a.prior_pitch + x0);
    cl.opx = (uint32_t)(y0 * W + x0);
    Cursor cc = cl;   // cursor of the step being computed
    auto advance = [&](Cursor& c) {
        c.x += a.dx;
        c.y += a.dy;
        c.oc += dc;
        c.op += dp;
        c.opx += dpx;
    };

    uint32_t L[4] = {0, 0, 0, 0};
    uint32_t m = 0;

    auto step = [&](const StepIn& in, int t) {
        // ---- joint cost C'(p, d), d = d0 .. d0+7 (Eq. 4, scaled) ----
        uint32_t mc[8];
        if (VIEW == 0) {
            mc[0] = in.m1.w; mc[1] = in.m1.z; mc[2] = in.m1.y; mc[3] = in.m1.x;
            mc[4] = in.m0.w; mc[5] = in.m0.z; mc[6] = in.m0.y; mc[7] = in.m0.x;
        } else {
            mc[0] = in.m0.x; mc[1] = in.m0.y; mc[2] = in.m0.z; mc[3] = in.m0.w;
            mc[4] = in.m1.x; mc[5] = in.m1.y; mc[6] = in.m1.z; mc[7] = in.m1.w;
        }
        uint32_t h[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) h[j] = __builtin_popcount(in.cb ^ mc[j]);
        // matching pixel outside the image: all n bits differ
        if (VIEW == 0 ? cc.x < d0 + 7 : cc.x + d0 + 7 >= W) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool out = VIEW == 0 ? cc.x - d0 - j < 0 : cc.x + d0 + j >= W;
                h[j] = out ? nfill : h[j];
            }
        }
        uint32_t C[4];
        if (VIEW == 0) {
            // values outside [0, D) carry no prior (the ABI only admits -1)
            const bool has = (unsigned)in.e < (unsigned)D;
            const uint32_t mulh = (has ? a.mulh_prior : a.mulh_noprior) * 0x10001u;
            // DDC of disparity d sits at pattern entry d - e + D; no prior
            // reads the zero run at the end of the table
            const int sidx = d0 - in.e + D;
            const int base = has ? ((sidx & 1) ? (D + 8) + ((sidx - 1) >> 1) : (sidx >> 1))
                                 : 2 * (D + 8);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                C[i] = pk_mad(h[2 * i] | (h[2 * i + 1] << 16), mulh, pat[base + i]);
        } else {
            const uint32_t mulh = a.mulh_noprior * 0x10001u;
#pragma unroll
            for (int i = 0; i < 4; ++i) C[i] = pk_mad(h[2 * i] | (h[2 * i + 1] << 16), mulh, 0u);
        }

        // ---- path recurrence, Eq. 2 ----
        if (t == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) L[i] = C[i];
        } else {
            uint32_t pv = dpp<kWaveShr1>(L[3]);   // hi half: cell d0-1
            uint32_t nx = dpp<kWaveShl1>(L[0]);   // lo half: cell d0+8
            // ends of the disparity range: reuse the cell itself, which is
            // already a candidate of the minimum (= leaving the term out)
            pv = gfirst ? (L[0] << 16) : pv;
            nx = glast ? (L[3] >> 16) : nx;
            uint32_t Dm[5];
            Dm[0] = __builtin_amdgcn_alignbit(L[0], pv, 16);
            Dm[1] = __builtin_amdgcn_alignbit(L[1], L[0], 16);
            Dm[2] = __builtin_amdgcn_alignbit(L[2], L[1], 16);
            Dm[3] = __builtin_amdgcn_alignbit(L[3], L[2], 16);
            Dm[4] = __builtin_amdgcn_alignbit(nx, L[3], 16);
            const uint32_t mp2 = (m + a.p2s) * 0x10001u;
            const uint32_t mm = m * 0x10001u;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint32_t nb = pk_add(pk_min(Dm[i], Dm[i + 1]), p1x2);
                uint32_t best = pk_min(pk_min(L[i], nb), mp2);
                L[i] = pk_add(best, pk_sub(C[i], mm));
            }
        }
        {
            uint32_t mn = pk_min(pk_min(L[0], L[1]), pk_min(L[2], L[3]));
            m = group_min<G>(min(mn & 0xffffu, mn >> 16));
        }

        // ---- aggregated sum S (Eq. 3) ----
        uint16_t* sp = S + (size_t)cc.opx * D + d0;
        if (MODE == kFirst) {
            __builtin_nontemporal_store(u32x4{L[0], L[1], L[2], L[3]},
                                        reinterpret_cast<u32x4*>(sp));
        } else if (MODE == kMiddle) {
            __builtin_nontemporal_store(
                u32x4{pk_add(in.s.x, L[0]), pk_add(in.s.y, L[1]), pk_add(in.s.z, L[2]),
                      pk_add(in.s.w, L[3])},
                reinterpret_cast<u32x4*>(sp));
        } else {
            uint32_t St[4];
            if (MODE == kLast) {
                St[0] = pk_add(in.s.x, L[0]); St[1] = pk_add(in.s.y, L[1]);
                St[2] = pk_add(in.s.z, L[2]); St[3] = pk_add(in.s.w, L[3]);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) St[i] = L[i];
            }
            if (a.store_sum) *reinterpret_cast<uint4*>(sp) = make_uint4(St[0], St[1], St[2], St[3]);
            // ---- WTA, Eq. 3: lexicographic minimum of (S, d) ----
            uint32_t best = 0xffffffffu;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint32_t k0 = ((St[i] & 0xffffu) << 9) | (uint32_t)(d0 + 2 * i);
                uint32_t k1 = ((St[i] >> 16) << 9) | (uint32_t)(d0 + 2 * i + 1);
                best = min(best, min(k0, k1));
            }
            best = group_min<G>(best);
            const int db = (int)(best & 511u);
            const uint32_t spv = dpp<kWaveShr1>(St[3]);
            const uint32_t snx = dpp<kWaveShl1>(St[0]);
            // surrogate cost feature: second minimum of S over |d - d*| >= 2
            uint32_t second = 0xffffu;
            if (VIEW == 0 && a.feat) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int d_lo = d0 + 2 * i, d_hi = d_lo + 1;
                    const uint32_t s_lo = St[i] & 0xffffu, s_hi = St[i] >> 16;
                    second = (d_lo - db >= 2 || db - d_lo >= 2) ? min(second, s_lo) : second;
                    second = (d_hi - db >= 2 || db - d_hi >= 2) ? min(second, s_hi) : second;
                }
                second = group_min<G>(second);
            }
            if (db >= d0 && db < d0 + 8) {
                const size_t px = (size_t)frame * a.px_stride + cc.opx;
                a.wta[VIEW][px] = (int16_t)db;
                if (VIEW == 0) {
                    // cells d0-1 .. d0+8 of S
                    uint32_t c[10];
                    c[0] = spv >> 16;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        c[1 + 2 * i] = St[i] & 0xffffu;
                        c[2 + 2 * i] = St[i] >> 16;
                    }
                    c[9] = snx & 0xffffu;
                    const int j = db - d0 + 1;
                    uint32_t A = 0, B = 0, Cc = 0;
#pragma unroll
                    for (int k = 1; k <= 8; ++k) {
                        if (k == j) {
                            A = c[k - 1];
                            B = c[k];
                            Cc = c[k + 1];
                        }
                    }
                    float v = (float)db;
                    const int den = (int)A - 2 * (int)B + (int)Cc;
                    if (a.subpixel && db > 0 && db < D - 1 && den > 0)
                        v = (float)db + __fdiv_rn((float)((int)A - (int)Cc), (float)(2 * den));
                    a.dsub[px] = v;
                    if (a.feat) {
                        a.feat[2 * px] = B | (second << 16);
                        a.feat[2 * px + 1] = (db > 0 && db < D - 1) ? (uint32_t)den : 0u;
                    }
                }
            }
        }
        advance(cc);
    };

    // three steps in flight: the loads of step t+3 are issued once step t
    // has consumed its buffer
    StepIn b0, b1, b2;
    load_step<D, VIEW, kLoadS>(cbase, cmatch, prior, S, cl, d0, b0);
    advance(cl);
    if (len > 1) load_step<D, VIEW, kLoadS>(cbase, cmatch, prior, S, cl, d0, b1);
    advance(cl);
    if (len > 2) load_step<D, VIEW, kLoadS>(cbase, cmatch, prior, S, cl, d0, b2);
    advance(cl);
    for (int t = 0; t < len; t += 3) {
        step(b0, t);
        if (t + 3 < len) load_step<D, VIEW, kLoadS>(cbase, cmatch, prior, S, cl, d0, b0);
        advance(cl);
        if (t + 1 >= len) break;
        step(b1, t + 1);
        if (t + 4 < len) load_step<D, VIEW, kLoadS>(cbase, cmatch, prior, S, cl, d0, b1);
        advance(cl);
        if (t + 2 >= len) break;
        step(b2, t + 2);
        if (t + 5 < len) load_step<D, VIEW, kLoadS>(cbase, cmatch, prior, S, cl, d0, b2);
        advance(cl);
    }
}

template <int G, int MODE>
__global__ __launch_bounds__(256) void sgm_dir_kernel(SgmArgs a)
{
    constexpr int D = G * 8;
    // DDC pattern (the Eq. 4 term: 0 at the prior, Q1 at +-1, Q2 beyond), as
    // pairs of u16 starting at even (first half) and odd (second half)
    // entries of P[k] = ddc(k - D), k in [0, 2D + 16), followed by a run of
    // zeros used where a pixel has no prior.
    __shared__ uint32_t pat[2 * (D + 8) + 4];
    for (int i = threadIdx.x; i < 2 * (D + 8) + 4; i += 256) {
        uint32_t v[2] = {0u, 0u};
        if (i < 2 * (D + 8)) {
            const int half = i >= D + 8;
            const int k0 = 2 * (i - half * (D + 8)) + half;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                int diff = k0 + j - D;
                diff = diff < 0 ? -diff : diff;
                v[j] = diff == 0 ? 0u : (diff == 1 ? a.q1s : a.q2s);
            }
        }
        pat[i] = v[0] | (v[1] << 16);
    }
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
