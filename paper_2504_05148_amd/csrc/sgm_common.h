// Building blocks of the SGM path passes (Sec. III, Eq. 2-3 with the joint
// cost of Sec. IV-A, Eq. 4): packed 2 x u16 arithmetic, DPP group
// reductions, line geometry, per-step loads, the fused cost, one recurrence
// step and the winner-takes-all + parabola emit.
//
// A line of a path direction is owned by G = D / K lanes of a wavefront;
// lane g holds disparities [K g, K g + K) as NR = K / 2 packed 2 x u16
// registers.  K = 8 (four registers) is the throughput layout; K = 4 (two
// registers, twice the lanes per line) halves the work of a lane per step
// and serves single frames, whose few lines leave the SIMDs idle otherwise.
// Memory layouts (S, census, prior words) do not depend on K.
#pragma once

#include "sldf_internal.h"

namespace sldf {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// NR packed registers as one vector (16 or 8 bytes per lane)
template <int NR> struct VecT;
template <> struct VecT<4> { typedef u32x4 type; };
template <> struct VecT<2> { typedef u32x2 type; };
template <int NR> using vecT = typename VecT<NR>::type;
template <int NR>
__device__ __forceinline__ vecT<NR> pack_v(const uint32_t v[NR])
{
    vecT<NR> x;
#pragma unroll
    for (int i = 0; i < NR; ++i) x[i] = v[i];
    return x;
}

__device__ __forceinline__ u16x2 v2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t u1(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b)
{
    return u1(__builtin_elementwise_min(v2(a), v2(b)));
}
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) { return u1(v2(a) + v2(b)); }
// a + b + c as one instruction (the compiler would otherwise split it into a
// subtract it can start early and an add)
__device__ __forceinline__ uint32_t add3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
// |a - b| + c in one instruction (both operands below 2^31 here, so the
// signed and unsigned readings of the difference agree)
__device__ __forceinline__ uint32_t sad(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) { return u1(v2(a) - v2(b)); }
// Three-way packed minimum of u16 values below 0x7c00: such bit patterns
// are positive finite fp16 numbers (denormals included, which the kernels
// preserve) ordered as the integers, so the fp16 minimum instruction
// (v_pk_minimum3_f16) returns the u16 minimum.  The host bound keeps every
// operand of the recurrence below 0x7c00.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_min3(uint32_t a, uint32_t b, uint32_t c)
{
    const f16x2 x = __builtin_bit_cast(f16x2, a), y = __builtin_bit_cast(f16x2, b),
                z = __builtin_bit_cast(f16x2, c);
    return __builtin_bit_cast(uint32_t,
                              __builtin_elementwise_minimum(__builtin_elementwise_minimum(x, y), z));
}
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
constexpr int kRowShr1 = 0x111;        // lane i <- lane i-1 within a row of 16
constexpr int kRowShl1 = 0x101;        // lane i <- lane i+1 within a row of 16

constexpr int kXcds = 8;               // MI355X: 8 XCDs, one L2 each
constexpr int kCus = 256;              // compute units

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

// First pixel and length of line `line` of direction (dx, dy): rows for
// horizontal steps, columns for vertical ones, W + H - 1 diagonals otherwise
// (first the ones starting on the top / bottom row, then the side column).
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

// Global-memory pointers (address space 1): loads through them are global
// loads; a base that is the same in every lane sits in scalar registers.
typedef __attribute__((address_space(1))) const char* gcptr;
typedef __attribute__((address_space(1))) char* gptr;

template <typename P>
__device__ __forceinline__ P uniform_ptr(const void* p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P)(((uint64_t)hi << 32) | lo);
}

// Inputs of one step (one pixel of the line) for one lane.
template <int NR>
struct StepIn {
    uint32_t cb;        // census of the base pixel
    u32x4a4 m[NR / 2];  // census of K = 2 NR consecutive matching pixels
    uint32_t w;         // prior word of the pixel (sldf_internal.h)
};

// Byte offsets of one pixel for one lane: census of the base pixel, census
// of the lane's first matching pixel, prior, the lane's 8 cells of S.
struct PixOff {
    uint32_t oc, om, op, os;
};

// Addressing of one line for one lane.  The bases are uniform over the
// workgroup (one frame-view), the offsets 32-bit byte offsets, so every load
// is a scalar base plus a vector offset.  Pixel t of the line sits at
// offset0 + t * step; the steps are small signed values (24-bit products).
// Census and prior words may be read at t = -1, the position before the
// line start: it lies in the census row pads / guard rows and on the guard
// ring of the prior words (cost weight 0); S only at t >= 0.
struct LineAddr {
    gcptr cbase;            // census of the base view, guard row, padded row starts
    gcptr cmatch;           // census of the matching view
    gcptr prior;            // prior words, guard corner
    gptr S;                 // aggregated cost
    uint32_t oc0, om0, op0, os0;
    int32_t dc, dp, ds;

    __device__ __forceinline__ PixOff at(int t) const
    {
        const uint32_t c = (uint32_t)__mul24(t, dc);
        return PixOff{oc0 + c, om0 + c, op0 + (uint32_t)__mul24(t, dp),
                      os0 + (uint32_t)__mul24(t, ds)};
    }
};


// frame and view are uniform over a workgroup, so the bases are too; the
// line steps by (dx, dy) and its S term is the view's buffer S; the lane
// owns disparities d0 .. d0 + K - 1
template <int D, int VIEW, int K = 8>
__device__ __forceinline__ LineAddr line_addr(const SgmArgs& a, int frame, int x0, int y0,
                                              int d0, int dx, int dy, uint16_t* S)
{
    LineAddr la;
    // census rows are addressed from the padded start of the row before
    // (pixel (x, y) at row y + 1, column x + D), so every offset down to
    // t = -1 is non-negative
    const int64_t crow = D + (int64_t)a.census_pitch;
    la.cbase = uniform_ptr<gcptr>(a.cbase[VIEW] - crow + (int64_t)frame * a.census_fstride);
    la.cmatch = uniform_ptr<gcptr>(a.cmatch[VIEW] - crow + (int64_t)frame * a.census_fstride);
    la.prior = uniform_ptr<gcptr>(a.pword[VIEW] + (int64_t)frame * a.pword_fstride[VIEW]);
    la.S = uniform_ptr<gptr>(S + (int64_t)frame * a.S_stride);
    la.oc0 = (uint32_t)((y0 + 1) * a.census_pitch + x0 + D) * 4u;
    // matching pixels: x - d (left base, descending) or x + d (right base)
    // for d = d0 .. d0+K-1; the census pad keeps both runs inside the buffer
    la.om0 = VIEW == 0 ? la.oc0 - (uint32_t)(d0 + K - 1) * 4u : la.oc0 + (uint32_t)d0 * 4u;
    la.op0 = (uint32_t)((y0 + 1) * a.pword_pitch + x0 + 1) * 4u;
    la.os0 = ((uint32_t)(y0 * a.W + x0) * D + (uint32_t)d0) * 2u;
    la.dc = (dy * a.census_pitch + dx) * 4;
    la.dp = (dy * a.pword_pitch + dx) * 4;
    la.ds = (dy * a.W + dx) * D * 2;
    return la;
}

template <int VIEW, int NR>
__device__ __forceinline__ void load_pixel(const LineAddr& la, const PixOff& o, StepIn<NR>& st)
{
    typedef __attribute__((address_space(1))) const uint32_t* gu32;
    typedef __attribute__((address_space(1))) const u32x4a4* gu32x4;
    st.cb = *reinterpret_cast<gu32>(la.cbase + o.oc);
    const gcptr pm = la.cmatch + o.om;
#pragma unroll
    for (int i = 0; i < NR / 2; ++i) st.m[i] = *reinterpret_cast<gu32x4>(pm + 16 * i);
    st.w = *reinterpret_cast<gu32>(la.prior + o.op);
}

// S streams through once per pass: non-temporal loads / stores, so it does not
// evict the census rows that neighbouring lines re-read from L2.  The lane's
// NR registers are its K cells of the pixel's D (contiguous, 2 NR x 2 bytes).
template <int NR = 4>
__device__ __forceinline__ vecT<NR> load_s(const LineAddr& la, const PixOff& o)
{
    typedef __attribute__((address_space(1))) const vecT<NR>* gcv;
    return __builtin_nontemporal_load(reinterpret_cast<gcv>(la.S + o.os));
}
template <int NR = 4>
__device__ __forceinline__ void store_s(const LineAddr& la, const PixOff& o, const uint32_t v[NR])
{
    typedef __attribute__((address_space(1))) vecT<NR>* gv;
    __builtin_nontemporal_store(pack_v<NR>(v), reinterpret_cast<gv>(la.S + o.os));
}

// Joint cost C'(p, d) for the lane's d = d0 .. d0+K-1 (Eq. 4 scaled by the
// alpha denominator): w H + num DDC with H = popcount of the census xor (n
// where the matching pixel leaves the image), the weight w and the DDC table
// entry from the pixel's prior word (sldf_internal.h).  The prior term is
// read from the LDS table at patl (the lane's first entry, pattern + 2 d0
// bytes) plus the word's offset; the right view has no prior term.  On the
// guard ring the weight is 0 and the entry a zero run, so the virtual
// positions before a line start cost 0: from a zero state L = 0, m = 0 such a
// step leaves the state at zero, and the first real pixel then yields L = C
// as Eq. 2 starts a path.  Inputs: the base pixel's code cb, the lane's K
// matching codes in ascending address order (asc[e] is the code at the
// lane's first matching address + e) and the pixel's prior word w.
template <int D, int VIEW, int NR = 4>
__device__ __forceinline__ void cost_codes(const SgmArgs& a, const char* patl, uint32_t cb,
                                           const uint32_t asc[2 * NR], uint32_t w, int x, int d0,
                                           uint32_t C[NR])
{
    constexpr int K = 2 * NR;
    // x - d descends with d for the left base, x + d ascends for the right base
    uint32_t h[K];
#pragma unroll
    for (int j = 0; j < K; ++j) h[j] = __builtin_popcount(cb ^ asc[VIEW == 0 ? K - 1 - j : j]);
    if (VIEW == 0 ? x < d0 + K - 1 : x + d0 + K - 1 >= a.W) {
        // distance of the lane's first matching pixel from the image edge;
        // opaque, so that the compiler derives the K tests here instead of
        // carrying K induction variables through every step
        int k = VIEW == 0 ? x - d0 : a.W - 1 - x - d0;
        asm volatile("" : "+v"(k));
#pragma unroll
        for (int j = 0; j < K; ++j) h[j] = k < j ? (uint32_t)a.n : h[j];
    }
    // the weight (low half of the word) multiplies both halves
    const u16x2 wt = __builtin_shufflevector(v2(w), v2(w), 0, 0);
    if (VIEW == 0) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(patl + (w >> 16));
#pragma unroll
        for (int i = 0; i < NR; ++i)
            C[i] = u1(v2(h[2 * i] | (h[2 * i + 1] << 16)) * wt + v2(p[i]));
    } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) C[i] = u1(v2(h[2 * i] | (h[2 * i + 1] << 16)) * wt);
    }
}

// The same from one pixel's loads (load_pixel); in.m holds the K matching
// codes in ascending address order.
template <int D, int VIEW, int NR = 4>
__device__ __forceinline__ void cost_lane(const SgmArgs& a, const char* patl,
                                          const StepIn<NR>& in, int x, int d0, uint32_t C[NR])
{
    uint32_t asc[2 * NR];
#pragma unroll
    for (int e = 0; e < 2 * NR; ++e) asc[e] = in.m[e / 4][e % 4];
    cost_codes<D, VIEW, NR>(a, patl, in.cb, asc, in.w, x, d0, C);
}

// Minimum of the lane's K cells, in both halves of the result.
template <int NR = 4>
__device__ __forceinline__ uint32_t lane_min(const uint32_t L[NR])
{
    if (NR == 4) {
        // t = min(L0, L1, L2) per half; u adds L3 and the other half of t; the
        // last minimum with the halves swapped covers all eight cells
        const f16x2 t = __builtin_bit_cast(f16x2, pk_min3(L[0], L[1], L[2]));
        const f16x2 l3 = __builtin_bit_cast(f16x2, L[NR - 1]);
        const f16x2 u = __builtin_elementwise_minimum(__builtin_elementwise_minimum(t, l3),
                                                      __builtin_shufflevector(t, t, 1, 0));
        return __builtin_bit_cast(
            uint32_t, __builtin_elementwise_minimum(u, __builtin_shufflevector(u, u, 1, 0)));
    } else {
        // t = min(L0, L1, L0 swapped), then with L1 swapped: all four cells
        const f16x2 l0 = __builtin_bit_cast(f16x2, L[0]), l1 = __builtin_bit_cast(f16x2, L[1]);
        const f16x2 t = __builtin_elementwise_minimum(__builtin_elementwise_minimum(l0, l1),
                                                      __builtin_shufflevector(l0, l0, 1, 0));
        return __builtin_bit_cast(
            uint32_t, __builtin_elementwise_minimum(t, __builtin_shufflevector(l1, l1, 1, 0)));
    }
}

// One step of Eq. 2 on the lane's K disparities.  L holds L_r(p - r, .) on
// entry and L_r(p, .) on exit; m is the group minimum of L_r(p - r, .) on
// entry and of L_r(p, .) on exit, held in both u16 halves.  A path starts
// from L = 0, m = 0: the first step then yields L = C.
// Neighbour exchange registers of the recurrence when a group is one DPP
// row (16 lanes): a row shift leaves the lane at the row end unwritten, so a
// register that starts as 0xffffffff keeps that value there for good and can
// serve every step of every chain.
struct Edge {
    uint32_t pv = 0xffffffffu, nx = 0xffffffffu;
};

template <int G, int NR = 4>
__device__ __forceinline__ void rec_lane(uint32_t L[NR], uint32_t& m, const uint32_t C[NR],
                                         uint32_t p1x2, uint32_t p2x2, bool gfirst, bool glast,
                                         Edge& edge)
{
    // neighbour cells d0-1 (hi half of pv) and d0+K (lo half of nx); at the
    // ends of the disparity range the term is left out of the minimum
    uint32_t pv, nx;
    if (G == 16) {
        // lanes at the row ends read 0xffff, which never wins the neighbour
        // minimum (the other neighbour is in range)
        edge.pv = __builtin_amdgcn_update_dpp(edge.pv, L[NR - 1], kRowShr1, 0xf, 0xf, false);
        edge.nx = __builtin_amdgcn_update_dpp(edge.nx, L[0], kRowShl1, 0xf, 0xf, false);
        pv = edge.pv;
        nx = edge.nx;
    } else {
        pv = dpp<kWaveShr1>(L[NR - 1]);
        nx = dpp<kWaveShl1>(L[0]);
        // reuse the cell itself, already a candidate of the minimum
        pv = gfirst ? (L[0] << 16) : pv;
        nx = glast ? (L[NR - 1] >> 16) : nx;
    }
    uint32_t Dm[NR + 1];
    Dm[0] = __builtin_amdgcn_alignbit(L[0], pv, 16);
#pragma unroll
    for (int i = 1; i < NR; ++i) Dm[i] = __builtin_amdgcn_alignbit(L[i], L[i - 1], 16);
    Dm[NR] = __builtin_amdgcn_alignbit(nx, L[NR - 1], 16);
    const uint32_t mp2 = pk_add(m, p2x2);
    // best - m + C in one 32-bit instruction |best - m| + C: in each half
    // best >= m (every term of the minimum is at least m), so the 32-bit
    // difference borrows nothing across the halves, and the result lies in
    // [0, 0xffff] per half: it equals the packed one
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        uint32_t nb = pk_add(pk_min(Dm[i], Dm[i + 1]), p1x2);
        uint32_t best = pk_min3(L[i], nb, mp2);
        L[i] = sad(best, m, C[i]);
    }
    m = group_min<G>(lane_min<NR>(L));
}

// Where wta_emit puts the owner lane's outputs of a pixel: with on false, to
// global memory at px; otherwise to these LDS slots, which the caller writes
// out later with other pixels of the row in whole cache lines, taking the
// parabola there: d*, S(d*-1) | S(d*+1) << 16 and S(d*) | second << 16 (the
// first cost-feature word; left view only).
struct WtaStage {
    bool on = false;
    bool feat = false;      // with on: the cost features are wanted (a.feat not null)
    __attribute__((address_space(3))) int16_t* d = nullptr;
    __attribute__((address_space(3))) uint32_t* ac = nullptr;
    __attribute__((address_space(3))) uint32_t* bs = nullptr;
};

// Subpixel disparity of the parabola through S(d*-1), S(d*), S(d*+1):
// d* + num / (2 den) with num = S(d*-1) - S(d*+1) and den = S(d*-1) - 2 S(d*)
// + S(d*+1), passed as 0 at the ends of the disparity range; no refinement
// there or for a flat parabola (den is never negative at the minimum).  One
// correctly rounded float division of exact integers, then one float add.
__device__ __forceinline__ float subpixel_value(int subpixel, int db, int num, int den)
{
    float v = (float)db;
    if (subpixel && den > 0) v = (float)db + __fdiv_rn((float)num, (float)(2 * den));
    return v;
}

// The left view's outputs of a pixel from d* = db and its staged words ac =
// S(d*-1) | S(d*+1) << 16 (either half arbitrary at its end of the range) and
// bs = S(d*) | second << 16: the subpixel disparity and the two cost-feature
// words (bs itself and the parabola's denominator, 0 at the range ends).
template <int D>
__device__ __forceinline__ void parabola_outputs(int subpixel, int db, uint32_t ac, uint32_t bs,
                                                 float& v, uint32_t& f1)
{
    const int A = (int)(ac & 0xffffu), Cc = (int)(ac >> 16), B = (int)(bs & 0xffffu);
    const int den = A - 2 * B + Cc;
    f1 = (db > 0 && db < D - 1) ? (uint32_t)den : 0u;
    v = subpixel_value(subpixel, db, A - Cc, (int)f1);
}

// Winner-takes-all on the aggregated cost St (Eq. 3; lexicographic minimum
// of (S, d), ties -> smallest d) and the parabola fit through S(d*-1),
// S(d*), S(d*+1); the owning lane writes d* (and for the left view the
// subpixel disparity and the learned-check cost features).  simg, when not
// null, is the line's S(p, .) as D u16 in LDS (written by the group before
// the call), from which the owner reads the two neighbours of d*.  With
// kPadded, simg is never null and one u16 before and after the line is
// readable, so the owner reads both neighbours without range tests (what
// they hold at the range ends is not used).
template <int G, int VIEW, int NR = 4, bool kPadded = false>
__device__ __forceinline__ void wta_emit(const SgmArgs& a, const uint32_t St[NR], int d0,
                                         size_t px, const uint16_t* simg = nullptr,
                                         const WtaStage& stage = WtaStage{})
{
    constexpr int K = 2 * NR, D = G * K;
    // keys S << 16 | e over the lane's cells e, then d0 added to the lane's
    // minimum: the smallest key is the smallest S and, among equal S, the
    // smallest d = d0 + e
    uint32_t best = 0xffffffffu;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const uint32_t k0 = (St[i] << 16) | (uint32_t)(2 * i);
        const uint32_t k1 = (St[i] & 0xffff0000u) | (uint32_t)(2 * i + 1);
        best = min(best, min(k0, k1));
    }
    best = group_min<G>(best + (uint32_t)d0);
    const int db = (int)(best & 0xffffu);
    const bool lds_row = kPadded || simg != nullptr;
    const uint32_t spv = lds_row ? 0u : dpp<kWaveShr1>(St[NR - 1]);
    const uint32_t snx = lds_row ? 0u : dpp<kWaveShl1>(St[0]);
    // learned-check cost feature: second minimum of S over |d - d*| >= 2.  The
    // lane's cells d* - 1 .. d* + 1 (local indices e - 1 .. e + 1, e = d* - d0)
    // are set to 0xffff in packed form before a packed minimum: bits of the
    // 3-bit window shifted into place, two bits per register spread to the
    // two u16 halves.  An S of 0xffff elsewhere gives the same minimum.
    uint32_t second = 0xffffu;
    if (VIEW == 0 && (stage.on ? stage.feat : a.feat != nullptr)) {
        const int e = db - d0;
        const uint32_t win = (e >= -1 && e <= K) ? ((0x7u << (e + 7)) >> 8) : 0u;
        uint32_t mn = 0xffffffffu;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            // bits 2i and 2i + 1 sign-extended to 0 / all ones, their low
            // halves packed into one word
            const uint32_t lo = (uint32_t)__builtin_amdgcn_sbfe((int)win, 2 * i, 1);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_sbfe((int)win, 2 * i + 1, 1);
            const uint32_t gate = __builtin_amdgcn_perm(hi, lo, 0x05040100u);
            mn = pk_min(mn, St[i] | gate);
        }
        second = group_min<G>(min(mn & 0xffffu, mn >> 16));
    }
    if (db >= d0 && db < d0 + K) {
        if (stage.on) stage.d[0] = (int16_t)db;
        else a.wta[VIEW][px] = (int16_t)db;
        if (VIEW == 0) {
            uint32_t A = 0, B = best >> 16, Cc = 0;  // S(d*) is the minimum itself
            if (kPadded) {
                A = simg[db - 1];
                Cc = simg[db + 1];
            } else if (simg) {
                A = db > 0 ? simg[db - 1] : 0u;
                Cc = db < D - 1 ? simg[db + 1] : 0u;
            } else {
                // cells d0-1 .. d0+K of S
                uint32_t c[K + 2];
                c[0] = spv >> 16;
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    c[1 + 2 * i] = St[i] & 0xffffu;
                    c[2 + 2 * i] = St[i] >> 16;
                }
                c[K + 1] = snx & 0xffffu;
                const int j = db - d0 + 1;
#pragma unroll
                for (int k = 1; k <= K; ++k) {
                    if (k == j) {
                        A = c[k - 1];
                        Cc = c[k + 1];
                    }
                }
            }
            const uint32_t ac = A | (Cc << 16), f0 = B | (second << 16);
            if (stage.on) {
                stage.ac[0] = ac;
                stage.bs[0] = f0;
            } else {
                float v;
                uint32_t f1;
                parabola_outputs<D>(a.subpixel, db, ac, f0, v, f1);
                a.dsub[px] = v;
                if (a.feat) {
                    a.feat[2 * px] = f0;
                    a.feat[2 * px + 1] = f1;
                }
            }
        }
    }
}

// Prior-term table in LDS, P[k] = alpha_num * q(|k - D|), k in [0, 2D + 16):
// the DDC of Eq. 4 (0 at the prior, Q1 at +-1, Q2 beyond) or, by
// prior_cost, the quadratic min(Q1 t^2, Q2) or Huber min(Q1 h_k(t), Q2)
// terms; stored as pairs of u16 starting at even (first half) and odd
// (second half) entries, followed by a run of D / 2 zero words used where a
// pixel has no prior (the layout prior_word addresses).
template <int D>
__device__ __forceinline__ void build_pattern(const SgmArgs& a, uint32_t* pat)
{
    for (int i = threadIdx.x; i < pattern_words(D); i += blockDim.x) {
        uint32_t v[2] = {0u, 0u};
        if (i < 2 * (D + 8)) {
            const int half = i >= D + 8;
            const int k0 = 2 * (i - half * (D + 8)) + half;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                int diff = k0 + j - D;
                diff = diff < 0 ? -diff : diff;
                if (a.prior_cost == 0) {
                    v[j] = diff == 0 ? 0u : (diff == 1 ? a.q1s : a.q2s);
                } else {
                    const uint64_t t = (uint64_t)diff, k = (uint64_t)a.huber_k;
                    const uint64_t r = (a.prior_cost == 1 || t <= k) ? t * t : k * (2 * t - k);
                    const uint64_t q = r * a.q1s;   // num * Q1 * r, capped at num * Q2
                    v[j] = q < a.q2s ? (uint32_t)q : a.q2s;
                }
            }
        }
        pat[i] = v[0] | (v[1] << 16);
    }
}

}  // namespace sldf
