// SGM aggregation in two sweeps over the image (Sec. III, Eq. 2-3, with the
// joint cost of Sec. IV-A, Eq. 4 fused in): the cost sum S is written once
// and read once per view, instead of once per pair of directions.
//
// The eight directions split into two sets whose dependencies all point one
// way in a row-by-row walk:
//   sweep A, rows top to bottom, each row left to right:
//     h (+1, 0), dr (+1, +1), dn (0, +1), dl (-1, +1)
//   sweep B, the same on the image turned by 180 degrees:
//     (-1, 0), (-1, -1), (0, -1), (+1, -1)
// (the 4-path set keeps h and dn).  A row is owned by G = D / 8 lanes (lane
// g holds disparities 8 g .. 8 g + 7 as four packed u16 registers, see
// sgm_common.h) and walks its pixels one per step; the row below walks two
// pixels behind it (pixel x of row y is processed at step x + 2 y).  At step
// t the pixel (x, y) takes its h state from its own previous step and the
// states of (x + 1, y - 1), (x, y - 1), (x - 1, y - 1) for dl, dn, dr, which
// the row above produced at steps t - 1, t - 2, t - 3: each row passes its
// dl, dn, dr results to the row below through LDS after every step, and the
// row below keeps dn for one and dr for two more steps in registers.  So S
// gets the four terms of the set in one pass: sweep A stores them, sweep B
// adds its four and takes the winner-takes-all + parabola directly.
//
// A workgroup of 16 waves holds 15 waves of rows (60 rows at D = 128) in
// lock step (one barrier per step) and one loader wave.  The rows of a frame
// are cut into bands of workgroups; the first row of a band needs the last
// row of the band above, which another workgroup computes: the loader of the
// upper band writes that row's dl, dn, dr per pixel to a handoff buffer in
// global memory, the loader of the lower band reads them a few pixels ahead
// into the LDS slot of a virtual row -1.  Every handoff dword carries a tag
// bit (bit 31; the states are below 0x7c00 in both halves, so it is free),
// stored and loaded with agent-scope atomics: a dword is valid once its tag
// is set, with no ordering between dwords needed.  The reader clears what it
// consumed, so the buffer is all zero between launches.  Workgroups take
// their band from an atomic ticket in start order (bands of every frame
// before the next band), so the band a workgroup waits for has always
// started; every wait is bounded and reports a timeout in an error word.
//
// Virtual positions: a row walks W + 2 (rows - 1) + 2 steps, from two steps
// before its first pixel to past its last.  Positions before the row read
// the guard position (cost 0), so all states of the directions that enter
// from the left or the top stay zero there and each path starts with L = C
// as Eq. 2 starts a path; dl states leaving past the right end are replaced
// by zero (the dl path starts at the last pixel of the next row).
#include <type_traits>

#include "sgm_common.h"

namespace sldf {

constexpr int kSwWaves = 16;            // waves per workgroup: all but one of rows, 1 loader
constexpr int kSwAhead = 8;             // handoff pixels in flight in the loader
constexpr uint32_t kSwTag = 0x80000000u;
constexpr int kSwSpinMax = 1 << 20;     // bounded wait for a handoff dword (about 2 s)

template <int G, int NW = kSwWaves>
__host__ __device__ constexpr int sweep_rows() { return (NW - 1) * (64 / G); }
// 16-byte chunks of one handoff pixel: dl, dn, dr states of G lanes + the three minima
template <int G> __host__ __device__ constexpr int sweep_chunks() { return 3 * G + 1; }
// A pixel's record in the handoff buffer is dword-major, [4][RECP] with the
// chunk count padded to a multiple of 64: the loader lanes' stores and loads
// of dword e of their chunks then cover whole cache lines.
template <int G> __host__ __device__ constexpr int sweep_rec_pad()
{
    return (sweep_chunks<G>() + 63) / 64 * 64;
}

enum { kDirDL = 0, kDirDN = 1, kDirDR = 2 };

template <int G, int NP, int NW = kSwWaves>
struct SweepLds {
    static constexpr int ROWS = sweep_rows<G, NW>();
    static constexpr int NX = NP == 8 ? 3 : 1;     // directions handed to the row below
    // xch[slot][dir][row + 1][lane]: outputs of row r at step t in slot t & 1;
    // index 0 is the virtual row above the band (written by the loader)
    u32x4 xch[2][NX][ROWS + 1][G];
    uint32_t xm[2][NX][ROWS + 1];
    uint32_t pat[pattern_words(G * 8)];
    int ticket;
};

// A step's loads in sweep A: the base pixel's code, the matching code that
// enters the lane's run, the prior word
struct SweepWinIn {
    uint32_t cb, mnew, w;
};

// pass-coordinate position u of row j at step t
__device__ __forceinline__ int sw_pos(int t, int j) { return t - 2 * j; }

// The outputs of the last 2G pixels of a row in the second sweep (LDS),
// written to global memory 2G at a time (whole lines instead of one scattered
// 2- or 4-byte store per pixel); the subpixel division is taken there too,
// two pixels per lane, instead of once per step by the whole wave for its
// owner lanes
template <int G>
struct SweepStage {
    int16_t d[2 * G];
    uint32_t ac[2 * G];     // S(d*-1) | S(d*+1) << 16
    uint32_t bs[2 * G];     // S(d*) | second minimum << 16 (the first cost-feature word)
};

template <int G, int PASS, int NP, int VIEW, int NW>
__device__ __forceinline__ void sweep_compute(const SgmArgs& a, SweepLds<G, NP, NW>& sm, int j,
                                              int g, int frame, int band, int rpb, int T,
                                              uint32_t* sbuf, SweepStage<G>* ostage)
{
    constexpr int NR = 4, K = 8, D = G * K;
    constexpr int RPW = 64 / G;                 // rows per wave
    constexpr int kRing = PASS == 0 ? 4 : 2;   // steps of loads in flight
    constexpr bool kLast = PASS == 1;
    const int yp = band * rpb + j;              // row in pass coordinates
    const bool live = j < rpb && yp < a.H;
    const int ypc = min(yp, a.H - 1);
    const int y = PASS == 0 ? ypc : a.H - 1 - ypc;
    const int x0 = PASS == 0 ? 0 : a.W - 1, dx = PASS == 0 ? 1 : -1;
    const int d0 = g * K;
    const LineAddr la = line_addr<D, VIEW, K>(a, frame, x0, y, d0, dx, 0, a.S[VIEW]);
    const char* patl = reinterpret_cast<const char*>(sm.pat) + 2 * d0;
    const uint32_t p1x2 = a.p1s * 0x10001u, p2x2 = a.p2s * 0x10001u;
    const bool gfirst = g == 0, glast = g == G - 1;
    const int W = a.W;
    // the feature switch as a scalar (the compiler otherwise rebuilds it from
    // a lane mask in every step)
    const bool want_feat = __builtin_amdgcn_readfirstlane(a.feat != nullptr ? 1 : 0) != 0;
    // the wave's first and last rows: a step where all of them are before
    // their row (u < 0), past it by more than one pixel, or outside the band
    // / image is skipped as a whole (states stay zero before the row; the dl
    // output at u = W, the last one the row below reads, is still written)
    const int j0 = j - j % RPW;
    const bool wave_dead = j0 >= rpb || band * rpb + j0 >= a.H;
    Edge edge;

    uint32_t Lh[NR] = {}, mh = 0;
    uint32_t dnq[NR] = {}, mdnq = 0;            // dn input of this step (read one step ago)
    uint32_t drq1[NR] = {}, mdrq1 = 0;          // dr inputs of the next two steps
    uint32_t drq2[NR] = {}, mdrq2 = 0;

    // Sweep A: the lane's K matching codes move by one address per step (dx),
    // so a step loads only the code that enters the run.  The codes live in a
    // register window: at step t the code of ascending index e (the lane's
    // first matching address + e) is in slot (e + (t - t0) dx) mod K, the
    // entering code (e = K - 1 for dx = 1, e = 0 for dx = -1) takes the slot
    // of the one that leaves, and with the step loop unrolled by K every slot
    // index is a constant.  The entering codes are read unclamped from K
    // positions before the row (the census rows' pads and guard rows hold
    // them), so the window is exact from the row's first pixel on; positions
    // before that cost 0 whatever their codes (guard weight 0).  Sweep B,
    // short of registers and instruction-bound, loads the whole run per step.
    constexpr bool kWin = PASS == 0;
    constexpr int U = kWin ? K : kRing;         // steps per loop iteration
    // T + 2 is a multiple of the loader's unroll: every wave runs the same
    // number of steps, so of barriers
    static_assert(kSwAhead % U == 0 && U % kRing == 0, "step unrolls must divide kSwAhead");
    typename std::conditional<kWin, SweepWinIn, StepIn<NR>>::type R[kRing];
    vecT<NR> SA[kRing];
    uint32_t win[K];
    typedef __attribute__((address_space(1))) const uint32_t* gu32;
    const uint32_t mnew_off = dx > 0 ? 4u * (K - 1) : 0u;
    auto load = [&](int i, int u) {
        const int uc = min(max(u, -1), W);
        if constexpr (kWin) {
            // offsets summed in 32 bits before they meet the base (a step
            // before the row start is a negative product that the sum wraps
            // back into the row's pads)
            const int um = min(max(u, -K), W);
            const PixOff o = la.at(uc);
            const uint32_t om = la.om0 + (uint32_t)__mul24(um, la.dc) + mnew_off;
            R[i].cb = *reinterpret_cast<gu32>(la.cbase + o.oc);
            R[i].mnew = *reinterpret_cast<gu32>(la.cmatch + om);
            R[i].w = *reinterpret_cast<gu32>(la.prior + o.op);
        } else {
            load_pixel<VIEW>(la, la.at(uc), R[i]);
        }
        if (kLast) SA[i] = load_s<NR>(la, la.at(min(max(u, 0), W - 1)));
    };
    // joint cost of position u from ring slot i, s = (t - t0) mod K of its
    // step t (0 at virtual positions: they read the guard position)
    auto cost_at = [&](int i, int s, int u, uint32_t C[NR]) {
        const int uc = min(max(u, -1), W);
        if constexpr (kWin) {
            uint32_t asc[K];
#pragma unroll
            for (int e = 0; e < K; ++e) asc[e] = win[(e + s * dx + 8 * K) % K];
            cost_codes<D, VIEW, NR>(a, patl, R[i].cb, asc, R[i].w, x0 + uc * dx, d0, C);
        } else {
            cost_lane<D, VIEW, NR>(a, patl, R[i], x0 + uc * dx, d0, C);
        }
    };
    // the entering code of the step with window index s, then its cost
    auto cost = [&](int i, int s, int u, uint32_t C[NR]) {
        if constexpr (kWin) win[((dx > 0 ? K - 1 : 0) + s * dx + 8 * K) % K] = R[i].mnew;
        cost_at(i, s, u, C);
    };
    const int t0 = -2;
#pragma unroll
    for (int i = 0; i < kRing; ++i) load(i, sw_pos(t0 + i, j));
    if constexpr (kWin) {
        // the whole run of the first step (window index 0: slot e = index e)
        const int um = min(max(sw_pos(t0, j), -K), W);
        typedef __attribute__((address_space(1))) const u32x4a4* gu32x4;
        const gcptr pm = la.cmatch + (la.om0 + (uint32_t)__mul24(um, la.dc));
        const u32x4a4 lo = *reinterpret_cast<gu32x4>(pm), hi = *reinterpret_cast<gu32x4>(pm + 16);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            win[e] = lo[e];
            win[4 + e] = hi[e];
        }
    }
    // the cost of a step is computed at the end of the step before
    uint32_t C[NR];
    cost_at(0, 0, sw_pos(t0, j), C);

    for (int tb = t0; tb < T; tb += U) {
#pragma unroll
        for (int ii = 0; ii < U; ++ii) {
            const int i = ii % kRing;
            const int t = tb + ii;
            const int u = sw_pos(t, j);
            const int si = (t - 1) & 1, so = t & 1;
            const bool skip =
                wave_dead || sw_pos(t, j0) < 0 || sw_pos(t, j0 + RPW - 1) > W;
            // the row above (index j) wrote its outputs of step t - 1
            uint32_t dln[NR], mdln = 0, dnn[NR], mdnn, drn[NR], mdrn = 0;
            {
                const u32x4 v = sm.xch[si][NP == 8 ? kDirDN : 0][j][g];
#pragma unroll
                for (int q = 0; q < NR; ++q) dnn[q] = v[q];
                mdnn = sm.xm[si][NP == 8 ? kDirDN : 0][j];
            }
            if (NP == 8) {
                const u32x4 vl = sm.xch[si][kDirDL][j][g];
                const u32x4 vr = sm.xch[si][kDirDR][j][g];
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    dln[q] = vl[q];
                    drn[q] = vr[q];
                }
                mdln = sm.xm[si][kDirDL][j];
                mdrn = sm.xm[si][kDirDR][j];
            }
            const vecT<NR> sa = SA[i];
            const int inext = (i + 1) % kRing;
            const int snext = (ii + 1) % K;           // window index of step t + 1
            // sweep A: ring slot i (this step's inputs, consumed at the end of
            // the step before) takes those of step t + kRing, issued before this
            // step's S store, so that waiting for them never waits for that store
            // (loads and stores share one counter); sweep B, short of registers,
            // loads at the end of the step
            if (!kLast) load(i, sw_pos(t + kRing, j));
            if (!skip) {
                // Eq. 2 for each direction of the set: h, dn and dr first (their
                // inputs are in registers), dl last (it needs this step's read)
                rec_lane<G, NR>(Lh, mh, C, p1x2, p2x2, gfirst, glast, edge);
                uint32_t Ldn[NR], mdn = mdnq;
#pragma unroll
                for (int q = 0; q < NR; ++q) Ldn[q] = dnq[q];
                rec_lane<G, NR>(Ldn, mdn, C, p1x2, p2x2, gfirst, glast, edge);
                uint32_t Ldl[NR], mdl = mdln, Ldr[NR], mdr = mdrq2;
                if (NP == 8) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        Ldl[q] = dln[q];
                        Ldr[q] = drq2[q];
                    }
                    rec_lane<G, NR>(Ldr, mdr, C, p1x2, p2x2, gfirst, glast, edge);
                    rec_lane<G, NR>(Ldl, mdl, C, p1x2, p2x2, gfirst, glast, edge);
                }
                // the set's share of S (Eq. 3); every partial sum of paths fits
                // its u16 half (the host bounds |R| (C' + P2) below 2^16), so
                // 32-bit adds of the packed words are exact
                uint32_t St[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    if (NP == 8) {
                        St[q] = add3(Lh[q], Ldn[q], Ldl[q]);
                        St[q] = kLast ? add3(St[q], Ldr[q], sa[q]) : St[q] + Ldr[q];
                    } else {
                        St[q] = kLast ? add3(Lh[q], Ldn[q], sa[q]) : Lh[q] + Ldn[q];
                    }
                }
                // cost of the next step (its inputs were loaded a step ago)
                cost(inext, snext, u + 1, C);
                if (live && u >= 0 && u < W) {
                    const PixOff o = la.at(u);
                    if (!kLast) {
                        store_s<NR>(la, o, St);
                    } else {
                        if (a.store_sum) store_s<NR>(la, o, St);
                        const int x = x0 + u * dx;
                        // the row's S(p, .) in LDS: the owner of d* reads its neighbours
                        // (one u32x4 of padding before the first and after the last row)
                        u32x4* srow = reinterpret_cast<u32x4*>(sbuf) + 1 + j * G;
                        srow[g] = pack_v<NR>(St);
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        // the pixel's outputs wait in the row's stage (slot x mod 2G)
                        // until the row has walked down to a multiple of 2G
                        SweepStage<G>& rs = ostage[j];
                        const int slot = (int)((uint32_t)x % (2u * G));   // x >= 0 here
                        typedef __attribute__((address_space(3))) int16_t li16;
                        typedef __attribute__((address_space(3))) uint32_t lu32;
                        const WtaStage ws{true, want_feat, (li16*)&rs.d[slot], (lu32*)&rs.ac[slot],
                                          (lu32*)&rs.bs[slot]};
                        wta_emit<G, VIEW, NR, true>(a, St, d0, 0,
                                                    reinterpret_cast<const uint16_t*>(srow), ws);
                        if (slot == 0) {
                            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                            const size_t rowp = (size_t)frame * a.px_stride + (size_t)y * W;
#pragma unroll
                            for (int k = 0; k < 2; ++k) {
                                const int i = g + k * G;
                                if (x + i < W) {
                                    const size_t p = rowp + x + i;
                                    const int db = rs.d[i];
                                    a.wta[VIEW][p] = (int16_t)db;
                                    if (VIEW == 0) {
                                        float v;
                                        uint32_t f1;
                                        parabola_outputs<D>(a.subpixel, db, rs.ac[i], rs.bs[i], v,
                                                            f1);
                                        a.dsub[p] = v;
                                        if (want_feat) {
                                            a.feat[2 * p] = rs.bs[i];
                                            a.feat[2 * p + 1] = f1;
                                        }
                                    }
                                }
                            }
                        }
                    }
                }
                // outputs for the row below; a dl path leaving past the row end
                // starts afresh at the last pixel of the next row
                if (NP == 8 && u >= W) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) Ldl[q] = 0;
                    mdl = 0;
                }
                sm.xch[so][NP == 8 ? kDirDN : 0][j + 1][g] = pack_v<NR>(Ldn);
                if (NP == 8) {
                    sm.xch[so][kDirDL][j + 1][g] = pack_v<NR>(Ldl);
                    sm.xch[so][kDirDR][j + 1][g] = pack_v<NR>(Ldr);
                }
                if (g == 0) {
                    sm.xm[so][NP == 8 ? kDirDN : 0][j + 1] = mdn;
                    if (NP == 8) {
                        sm.xm[so][kDirDL][j + 1] = mdl;
                        sm.xm[so][kDirDR][j + 1] = mdr;
                    }
                }
            } else if (!wave_dead) {
                // the wave's rows have not started: the next step's cost
                cost(inext, snext, u + 1, C);
            }
            // delay lines: dn of the row above for the next step, dr for the one after
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                dnq[q] = dnn[q];
                if (NP == 8) {
                    drq2[q] = drq1[q];
                    drq1[q] = drn[q];
                }
            }
            mdnq = mdnn;
            if (NP == 8) {
                mdrq2 = mdrq1;
                mdrq1 = mdrn;
            }
            if (kLast) load(i, sw_pos(t + kRing, j));
            __syncthreads();
        }
    }
}

// The loader wave: hands the band's last row to the band below (producer)
// and the band above's last row to this band's first row (consumer).
template <int G, int NP, int NW>
__device__ __forceinline__ void sweep_loader(const SgmArgs& a, SweepLds<G, NP, NW>& sm, int lane,
                                             int fv, int band, int nbands, int rpb, int T)
{
    constexpr int NX = SweepLds<G, NP, NW>::NX;
    constexpr int NCH = NX * G + 1;              // chunks per pixel in use
    constexpr int CPL = (NCH + 63) / 64;         // chunks per loader lane
    constexpr int kRing = kSwAhead;
    const int W = a.W;
    constexpr int RECP = sweep_rec_pad<G>();
    constexpr int64_t rec = 4 * RECP;            // dwords per pixel in the buffer
    // buffer of the boundary below this band and of the one above it
    uint32_t* const out = band + 1 < nbands
                              ? a.hand + (((int64_t)fv * (nbands - 1) + band) * W) * rec
                              : nullptr;
    uint32_t* const in = band > 0
                             ? a.hand + (((int64_t)fv * (nbands - 1) + band - 1) * W) * rec
                             : nullptr;
    // chunk c of a pixel: c < NX G is lane c % G of direction c / G, chunk
    // NX G the NX minima
    u32x4 ring[kRing][CPL];
    auto fetch = [&](int k, int col) {
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
            const int c = lane + 64 * h;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (in && c < NCH && col < W) {
                uint32_t* p = in + (int64_t)col * rec + c;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    v[e] = __hip_atomic_load(p + e * RECP, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            ring[k][h] = v;
        }
    };
    bool dead = false;                           // a wait timed out: no further waits
    const int t0 = -2;
    // the first row reads, at step t, the pixel t + 1 of the row above (the
    // loader's slot of step t - 1): the loader writes pixel t + 2 at step t
#pragma unroll
    for (int k = 0; k < kRing; ++k) fetch(k, t0 + 2 + k);
    for (int tb = t0; tb < T; tb += kRing) {
#pragma unroll
        for (int k = 0; k < kRing; ++k) {
            const int t = tb + k;
            const int col = t + 2;
            // consumer: pixel col of the row above into slot t & 1, row index 0
#pragma unroll
            for (int h = 0; h < CPL; ++h) {
                const int c = lane + 64 * h;
                u32x4 v = ring[k][h];
                const bool need = in && c < NCH && col >= 0 && col < W;
                bool ok = !need || dead || ((v[0] & v[1] & v[2] & v[3]) & kSwTag);
                if (__builtin_amdgcn_ballot_w64(!ok)) {
                    // the upper band has not produced this pixel yet: wait
                    for (int it = 0; it < kSwSpinMax && __builtin_amdgcn_ballot_w64(!ok); ++it) {
                        __builtin_amdgcn_s_sleep(2);
                        if (!ok) {
                            uint32_t* p = in + (int64_t)col * rec + c;
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                v[e] = __hip_atomic_load(p + e * RECP, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                            ok = (v[0] & v[1] & v[2] & v[3]) & kSwTag;
                        }
                    }
                    if (!ok) {
                        __hip_atomic_fetch_or(a.sync + 2, 1, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                        v = u32x4{0u, 0u, 0u, 0u};
                    }
                    dead = dead || __builtin_amdgcn_ballot_w64(!ok);
                }
                if (need) {
                    // clear what was consumed: the buffer is zero between launches
                    uint32_t* p = in + (int64_t)col * rec + c;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        __hip_atomic_store(p + e * RECP, 0u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] &= ~kSwTag;
                if (c < NX * G) {
                    sm.xch[t & 1][c / G][0][c % G] = v;
                } else if (c == NX * G) {
#pragma unroll
                    for (int e = 0; e < NX; ++e) sm.xm[t & 1][e][0] = v[e];
                }
            }
            fetch(k, col + kRing);
            // producer: the band's last row wrote its outputs of step t - 1
            // (pixel (t - 1) - 2 (rpb - 1)) into slot (t - 1) & 1
            const int xp = t - 1 - 2 * (rpb - 1);
            if (out && xp >= 0 && xp < W) {
#pragma unroll
                for (int h = 0; h < CPL; ++h) {
                    const int c = lane + 64 * h;
                    if (c >= NCH) continue;
                    u32x4 v;
                    if (c < NX * G) {
                        v = sm.xch[(t - 1) & 1][c / G][rpb][c % G];
                    } else {
                        v = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
                        for (int e = 0; e < NX; ++e) v[e] = sm.xm[(t - 1) & 1][e][rpb];
                    }
                    uint32_t* p = out + (int64_t)xp * rec + c;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        __hip_atomic_store(p + e * RECP, v[e] | kSwTag, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
        }
    }
}

template <int G, int PASS, int NP, int NW>
__global__ __launch_bounds__(NW * 64, 4) void sgm_sweep_kernel(SgmArgs a)
{
    constexpr int ROWS = sweep_rows<G, NW>();
    constexpr int D = G * 8;
    __shared__ SweepLds<G, NP, NW> sm;
    __shared__ u32x4 sbuf[PASS == 1 ? ROWS * G + 2 : 1];
    __shared__ SweepStage<G> ostage[PASS == 1 ? ROWS : 1];
    const int tid = threadIdx.x;
    if (tid == 0)
        sm.ticket = __hip_atomic_fetch_add(a.sync, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // zero exchange slots: the states above the image and before the rows
    {
        uint32_t* z = reinterpret_cast<uint32_t*>(&sm.xch[0][0][0][0]);
        constexpr int nz = (int)(sizeof(sm.xch) + sizeof(sm.xm)) / 4;
        for (int i = tid; i < nz; i += NW * 64) z[i] = 0u;
    }
    build_pattern<D>(a, sm.pat);
    __syncthreads();
    // workgroups take (band, frame-view) items from the ticket in start order
    const int logical = sm.ticket;
    const int fv = logical % a.n_fv, band = logical / a.n_fv;
    const int rpb = a.rows_per_band;
    const int view = a.view_base + fv % a.nviews, frame = fv / a.nviews;
    const bool run = band < a.blocks_per_fv && !(a.gate && a.gate[frame] <= a.gate_limit);
    if (run) {
        // steps -2 .. T - 1: the last row's last pixel at step W - 1 + 2 (rpb - 1),
        // handed on by the loader one step later; a whole number of both unrolls
        const int T = -2 + (a.W + 2 * (rpb - 1) + 3 + kSwAhead - 1) / kSwAhead * kSwAhead;
        const int wave = tid >> 6;
        if (wave == NW - 1) {
            sweep_loader<G, NP, NW>(a, sm, tid & 63, fv, band, a.blocks_per_fv, rpb, T);
        } else {
            const int j = tid / G, g = tid % G;
            uint32_t* sb = reinterpret_cast<uint32_t*>(sbuf);
            if (view == 0)
                sweep_compute<G, PASS, NP, 0, NW>(a, sm, j, g, frame, band, rpb, T, sb, ostage);
            else
                sweep_compute<G, PASS, NP, 1, NW>(a, sm, j, g, frame, band, rpb, T, sb, ostage);
        }
    }
    // the last workgroup to finish resets the ticket counters for the next launch
    __syncthreads();
    if (tid == 0) {
        const int done =
            __hip_atomic_fetch_add(a.sync + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == (int)gridDim.x - 1) {
            __hip_atomic_store(a.sync, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(a.sync + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int G, int NP, int NW>
static hipError_t launch_sweep_g(const SgmArgs& a, int pass, dim3 grid, hipStream_t s)
{
    if (pass == 0)
        hipLaunchKernelGGL((sgm_sweep_kernel<G, 0, NP, NW>), grid, dim3(NW * 64), 0, s, a);
    else
        hipLaunchKernelGGL((sgm_sweep_kernel<G, 1, NP, NW>), grid, dim3(NW * 64), 0, s, a);
    return hipGetLastError();
}

static int rows_of(int D, int nw)
{
    return (nw - 1) * (64 / (D / 8));
}

// Bands of a frame-view: 16-wave workgroups (15 waves of rows, one
// workgroup per compute unit: they fill its LDS), the rows spread evenly over
// the fewest bands.  (Two 8-wave workgroups per unit, whose barriers do not
// run in step, measured no faster.)
SweepPlan sweep_plan(int H, int D)
{
    const int rpw = 64 / (D / 8);
    const int bands = (H + rows_of(D, kSwWaves) - 1) / rows_of(D, kSwWaves);
    const int per = (H + bands - 1) / bands;
    return SweepPlan{bands, (per + rpw - 1) / rpw * rpw};
}

int64_t sweep_hand_bytes_per_fv(int W, int H, int D)
{
    const int nb = sweep_plan(H, D).bands;
    const int recp = D == 64 ? sweep_rec_pad<8>() : D == 128 ? sweep_rec_pad<16>() : sweep_rec_pad<32>();
    return (int64_t)(nb - 1) * W * recp * 16;
}

hipError_t launch_sgm_sweep(const SgmArgs& a0, int D, int pass, int nviews, int nframes,
                            hipStream_t s)
{
    SgmArgs a = a0;
    a.nviews = nviews;
    a.n_fv = nviews * nframes;
    const SweepPlan pl = sweep_plan(a.H, D);
    a.blocks_per_fv = pl.bands;                  // bands per frame-view
    a.rows_per_band = pl.rows_per_band;
    const int np = a.npaths;                     // 4 or 8
    dim3 grid((unsigned)(a.n_fv * a.blocks_per_fv));
    if (D == 64)
        return np == 8 ? launch_sweep_g<8, 8, kSwWaves>(a, pass, grid, s)
                       : launch_sweep_g<8, 4, kSwWaves>(a, pass, grid, s);
    if (D == 128)
        return np == 8 ? launch_sweep_g<16, 8, kSwWaves>(a, pass, grid, s)
                       : launch_sweep_g<16, 4, kSwWaves>(a, pass, grid, s);
    return np == 8 ? launch_sweep_g<32, 8, kSwWaves>(a, pass, grid, s)
                   : launch_sweep_g<32, 4, kSwWaves>(a, pass, grid, s);
}

}  // namespace sldf
