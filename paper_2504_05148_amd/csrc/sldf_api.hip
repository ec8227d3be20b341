// C ABI of libsldf.so: parameter validation, workspace plan and the launch
// sequence of one frame batch (Fig. 1 flow of the paper).
#include <math.h>
#include <mutex>
#include <new>
#include <string.h>

#include "../../include/sldf.h"
#include "sldf_internal.h"

using namespace sldf;

// Per-run stage markers: events[k] of one run are recorded before census,
// after census, after semidensification, after the last SGM pass and after
// the check.
constexpr int kMarks = SLDF_NUM_STAGES + 1;

struct sldf_ctx {
    sldf_params p;
    int device;
    Buffers buf;
    sldf_taps taps;
    int need_right;   // right-view pass needed (stereo half of the check)
    int n;            // census bits
    int sweep_ready;  // handoff buffer and sync words of the two-sweep schedule zeroed
    const uint16_t* sur_w;  // learned-check parameters (caller-owned)
    const float* sur_b;
    // split schedule with 8 paths: a second stream for the pairs that run
    // beside the main stream's passes, and the events that fork and join it
    hipStream_t side;
    hipEvent_t fork_ev, join_ev;
    // timing
    hipEvent_t* events;
    int32_t timing_cap;     // runs that fit in events
    int32_t timing_runs;    // runs recorded since the last read
    int64_t launches[SLDF_NUM_STAGES];
};

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bits of a census code: (w h - 1) / 2 centre-symmetric pairs, or w h - 1
// for the full census.
int census_bits(const sldf_params* p)
{
    const int wh = p->census_w * p->census_h;
    return p->census_kind == 1 ? wh - 1 : (wh - 1) / 2;
}

// Largest joint cost C' = (den - num) H + num DDC, or den H without prior in
// blend mode 1 (Eq. 4 scaled by den).
int64_t max_cost(const sldf_params* p, int n)
{
    int64_t with_prior = (int64_t)(p->alpha_den - p->alpha_num) * n +
                         (int64_t)p->alpha_num * (p->q2 > p->q1 ? p->q2 : p->q1);
    int64_t without = (int64_t)(p->blend_mode ? p->alpha_den : p->alpha_den - p->alpha_num) * n;
    return with_prior > without ? with_prior : without;
}

sldf_status validate(const sldf_params* p)
{
    if (!p || p->struct_size != (int32_t)sizeof(sldf_params)) return SLDF_EINVAL;
    if (p->width < 16 || p->width > 4096 || p->height < 16 || p->height > 4096)
        return SLDF_ESHAPE;
    if (p->max_disp != 64 && p->max_disp != 128 && p->max_disp != 256) return SLDF_ESHAPE;
    // the path passes address one frame's cost volume with 32-bit byte offsets
    if ((int64_t)p->width * p->height * p->max_disp > ((int64_t)1 << 31)) return SLDF_ESHAPE;
    if (p->census_w < 1 || p->census_h < 1 || !(p->census_w & 1) || !(p->census_h & 1) ||
        p->census_w > 15 || p->census_h > 15)
        return SLDF_EINVAL;
    if (p->census_kind != 0 && p->census_kind != 1) return SLDF_EINVAL;
    int n = census_bits(p);
    if (n < 1 || n > 32) return SLDF_EINVAL;
    if (p->num_paths != 1 && p->num_paths != 4 && p->num_paths != 8) return SLDF_EINVAL;
    if (p->p1 < 0 || p->p2 < p->p1 || p->q1 < 0 || p->q2 < p->q1) return SLDF_EINVAL;
    if (p->alpha_den < 1 || p->alpha_num < 0 || p->alpha_num > p->alpha_den) return SLDF_EINVAL;
    if (p->blend_mode != 0 && p->blend_mode != 1) return SLDF_EINVAL;
    if (p->semidense != 0 && p->semidense != 1) return SLDF_EINVAL;
    if (p->ts < 0 || p->ts > 64 || p->rs < 0 || p->rs > 15) return SLDF_EINVAL;
    if (p->tc < 0 || p->tc > 4096 || p->rc < 0 || p->rc > 31) return SLDF_EINVAL;
    if (p->check_mode < 0 || p->check_mode > 3) return SLDF_EINVAL;
    if (p->check_impl != 0 && p->check_impl != 1) return SLDF_EINVAL;
    if (p->check_impl == 1 &&
        (p->check_mode != 3 || !(p->fallback_tau >= 0.f && p->fallback_tau <= 1.f) ||
         !(p->uncertain_margin >= 0.f)))
        return SLDF_EINVAL;
    if (p->subpixel != 0 && p->subpixel != 1) return SLDF_EINVAL;
    if (p->schedule < 0 || p->schedule > 3) return SLDF_EINVAL;
    if (p->prior_cost < 0 || p->prior_cost > 2 || p->huber_k < 1 || p->huber_k > 4096)
        return SLDF_EINVAL;
    if (p->batch < 1 || p->batch > 4096) return SLDF_EINVAL;
    // 16-bit bound: every L_r lies in [C', C' + P2'] (Eq. 2), the sum of the
    // paths in [|R| C', |R| (C' + P2')], and the largest intermediate of the
    // recurrence is C' + P2' + P1' (neighbour term) or m + P2' <= C' + 2 P2'.
    // The recurrence compares its terms as fp16 bit patterns (a three-way
    // packed minimum), exact while they stay below 0x7c00 (the fp16
    // infinity): C' + P2' + max(P1', P2') < 0x7c00.
    int64_t cmax = max_cost(p, n);
    int64_t P1 = (int64_t)p->alpha_den * p->p1, P2 = (int64_t)p->alpha_den * p->p2;
    if ((int64_t)p->num_paths * (cmax + P2) >= 65536) return SLDF_EOVERFLOW;
    if (cmax + P2 + (P1 > P2 ? P1 : P2) >= 0x7c00) return SLDF_EOVERFLOW;
    if ((int64_t)p->alpha_num * p->q2 >= 65536) return SLDF_EOVERFLOW;
    return SLDF_OK;
}

// right-view S volume: the plain stereo check, or the fallback of the
// learned check
bool needs_right(const sldf_params* p) { return p->check_mode == 1 || p->check_mode == 3; }

// Path directions: horizontal and vertical first (4-path set), then the
// diagonals (8-path set); the 1-path debug mode is left-to-right only.
const int kDirs[8][2] = {{+1, 0}, {-1, 0}, {0, +1}, {0, -1},
                         {+1, +1}, {-1, +1}, {+1, -1}, {-1, -1}};
// The same sets as pairs of opposite directions (forward of each pair).
const int kPairDirs[4][2] = {{+1, 0}, {0, +1}, {+1, +1}, {-1, +1}};

// Workspace plan: one 256-byte aligned segment per array, each holding all
// batch frames.  Returns the total size; fills b when base != NULL.
size_t plan(const sldf_params* p, char* base, Buffers* b)
{
    const size_t F = (size_t)p->batch;
    const size_t px = (size_t)p->width * p->height;
    const size_t cells = px * (size_t)p->max_disp;
    size_t off = 0;
    auto seg = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return base ? (void*)(base + o) : nullptr;
    };
    const size_t cpitch = (size_t)p->width + 2 * (size_t)p->max_disp;
    const size_t cframe = cpitch * (size_t)p->height;
    // census: one guard row before frame 0 and after the last frame
    void* cl = seg((F * cframe + 2 * cpitch) * 4);
    void* cr = seg((F * cframe + 2 * cpitch) * 4);
    // prior words with a one-pixel guard ring; the right view's map is shared
    const size_t pwf = ((size_t)p->width + 2) * ((size_t)p->height + 2);
    void* pr = seg(F * pwf * 4);
    void* prr = needs_right(p) ? seg(pwf * 4) : nullptr;
    void* ds = seg(F * px * 2);
    void* dr = seg(F * px * 2);
    void* dsub = seg(F * px * 4);
    void* sl = seg(F * cells * 2);
    void* sr = needs_right(p) ? seg(F * cells * 2) : nullptr;
    // second cost term of the split schedule (runs of up to kSplitFrames frames)
    const size_t Fs = F < (size_t)kSplitFrames ? F : (size_t)kSplitFrames;
    const bool split = p->num_paths >= 4 && p->schedule != 1;
    void* s2l = split ? seg(Fs * cells * 2) : nullptr;
    void* s2r = split && needs_right(p) ? seg(Fs * cells * 2) : nullptr;
    // 8 paths, single-frame contexts: a third term and checkpoints for the
    // pairs of the second stream (batch contexts run single frames on one
    // stream: a stream per context would share the few hardware queues with
    // the caller's streams)
    const bool split3 = split && p->num_paths == 8 && F <= (size_t)kSplitFrames;
    void* s3l = split3 ? seg(Fs * cells * 2) : nullptr;
    void* s3r = split3 && needs_right(p) ? seg(Fs * cells * 2) : nullptr;
    // checkpoints of the paired passes: the largest direction pair in use
    size_t ck_per_fv = 0;
    for (int k = 0; k < (p->num_paths >= 4 ? p->num_paths / 2 : 0); ++k) {
        const int dx = kPairDirs[k][0], dy = kPairDirs[k][1];
        const size_t n = (size_t)num_lines(p->width, p->height, dx, dy) *
                         (size_t)sgm_pair_ckpt_segs(p->width, p->height, dx, dy) *
                         (size_t)p->max_disp * 2;
        ck_per_fv = n > ck_per_fv ? n : ck_per_fv;
    }
    void* ck = ck_per_fv ? seg(F * 2 * ck_per_fv) : nullptr;
    void* ck2 = split3 ? seg(Fs * 2 * ck_per_fv) : nullptr;
    void* wm = split3 ? seg(Fs * px * (size_t)(p->max_disp / 32) * 4) : nullptr;
    void* rb = seg(F * px * (size_t)(p->max_disp / 32) * 4);
    void* rho = seg(F * px * 2);
    void* feat = seg(F * px * 8);
    void* x0 = seg(F * px * 16);
    const bool learned = p->check_impl == 1;
    void* act0 = learned ? seg(F * px * 64) : nullptr;
    void* act1 = learned ? seg(F * px * 64) : nullptr;
    void* logits = learned ? seg(F * px * 4) : nullptr;
    void* counter = learned ? seg(F * 4) : nullptr;
    // two-sweep schedule (runs of kSweepMinFrames or more frames, or schedule 3)
    const bool sweep = p->num_paths >= 4 &&
                       (p->schedule == 3 || (p->schedule == 0 && F >= (size_t)kSweepMinFrames));
    void* hand = sweep ? seg(F * 2 * (size_t)sweep_hand_bytes_per_fv(p->width, p->height,
                                                                      p->max_disp))
                       : nullptr;
    void* sync = sweep ? seg(16) : nullptr;
    if (b) {
        b->census_l = base ? (uint32_t*)cl + cpitch + p->max_disp : nullptr;
        b->census_r = base ? (uint32_t*)cr + cpitch + p->max_disp : nullptr;
        b->census_pitch = (int32_t)cpitch;
        b->census_fstride = (int64_t)cframe;
        b->pword[0] = (uint32_t*)pr;
        b->pword[1] = (uint32_t*)prr;
        b->pword_pitch = p->width + 2;
        b->pword_fstride = (int64_t)pwf;
        b->dstar = (int16_t*)ds;
        b->dright = (int16_t*)dr;
        b->dsub = (float*)dsub;
        b->S_left = (uint16_t*)sl;
        b->S_right = (uint16_t*)sr;
        b->S2[0] = (uint16_t*)s2l;
        b->S2[1] = (uint16_t*)s2r;
        b->S3[0] = (uint16_t*)s3l;
        b->S3[1] = (uint16_t*)s3r;
        b->ckpt = (uint32_t*)ck;
        b->ckpt2 = (uint32_t*)ck2;
        b->wmask = (uint32_t*)wm;
        b->rowbits = (uint32_t*)rb;
        b->rho = (uint16_t*)rho;
        b->feat = (uint32_t*)feat;
        b->x0 = (uint16_t*)x0;
        b->act[0] = (uint16_t*)act0;
        b->act[1] = (uint16_t*)act1;
        b->logits = (float*)logits;
        b->counter = (int32_t*)counter;
        b->hand = (uint32_t*)hand;
        b->sync = (int32_t*)sync;
        b->hand_bytes = sweep ? F * 2 * (size_t)sweep_hand_bytes_per_fv(p->width, p->height,
                                                                         p->max_disp)
                              : 0;
        b->px_stride = (int64_t)px;
        b->S_stride = (int64_t)cells;
    }
    return off;
}



}  // namespace

extern "C" {

const char* sldf_status_string(sldf_status s)
{
    switch (s) {
    case SLDF_OK: return "ok";
    case SLDF_EINVAL: return "invalid argument";
    case SLDF_ESHAPE: return "shape out of range";
    case SLDF_EALIGN: return "alignment violated";
    case SLDF_EOVERFLOW: return "parameters overflow the 16-bit cost bound";
    case SLDF_ENOMEM: return "workspace too small or out of host memory";
    case SLDF_EDEVICE: return "HIP device error";
    case SLDF_ESTATE: return "invalid context state";
    }
    return "unknown status";
}

int32_t sldf_abi_version(void) { return SLDF_ABI_VERSION; }

void sldf_params_default(sldf_params* p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->struct_size = (int32_t)sizeof(sldf_params);
    p->width = 1242;
    p->height = 375;
    p->max_disp = 128;
    p->census_w = 9;
    p->census_h = 7;
    p->num_paths = 8;
    p->p1 = 10;           // Tab. II
    p->p2 = 120;
    p->q1 = 5;
    p->q2 = 160;
    p->alpha_num = 7;     // alpha = 0.7
    p->alpha_den = 10;
    p->blend_mode = 0;
    p->semidense = 1;     // SDSGM
    p->ts = 2;
    p->rs = 6;
    p->tc = 2;
    p->rc = 20;
    p->check_mode = 3;    // stereo OR LiDAR (Eq. 6)
    p->check_impl = 0;
    p->subpixel = 1;
    p->batch = 1;
    p->fallback_tau = 0.05f;
    p->uncertain_margin = 0.5f;
    p->prior_cost = 0;    // DDC
    p->huber_k = 1;
    p->schedule = 0;      // automatic
    p->census_kind = 0;   // centre-symmetric census
}

sldf_status sldf_workspace_size(const sldf_params* p, size_t* bytes)
{
    if (!bytes) return SLDF_EINVAL;
    sldf_status st = validate(p);
    if (st != SLDF_OK) return st;
    *bytes = plan(p, nullptr, nullptr);
    return SLDF_OK;
}

sldf_status sldf_create(const sldf_params* p, void* dev_workspace, size_t ws_bytes,
                        sldf_ctx** out)
{
    if (!out) return SLDF_EINVAL;
    *out = nullptr;
    sldf_status st = validate(p);
    if (st != SLDF_OK) return st;
    if (!dev_workspace) return SLDF_EINVAL;
    if (((uintptr_t)dev_workspace & 255) != 0) return SLDF_EALIGN;
    size_t need = plan(p, nullptr, nullptr);
    if (ws_bytes < need) return SLDF_ENOMEM;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SLDF_EDEVICE;
    sldf_ctx* c = new (std::nothrow) sldf_ctx;
    if (!c) return SLDF_ENOMEM;
    memset(c, 0, sizeof(*c));
    c->p = *p;
    c->device = dev;
    plan(p, (char*)dev_workspace, &c->buf);
    c->need_right = needs_right(p);
    c->n = census_bits(p);
    if (c->buf.S3[0]) {
        // default priority; non-blocking w.r.t. the null stream (the events
        // order it against the caller's stream)
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return SLDF_EDEVICE;
        }
        if (hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess) {
            if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
            (void)hipStreamDestroy(c->side);
            delete c;
            return SLDF_EDEVICE;
        }
    }
    *out = c;
    return SLDF_OK;
}

static void free_events(sldf_ctx* ctx)
{
    if (!ctx->events) return;
    for (int64_t i = 0; i < (int64_t)ctx->timing_cap * kMarks; ++i) (void)hipEventDestroy(ctx->events[i]);
    delete[] ctx->events;
    ctx->events = nullptr;
    ctx->timing_cap = ctx->timing_runs = 0;
}

sldf_status sldf_destroy(sldf_ctx* ctx)
{
    if (!ctx) return SLDF_OK;
    free_events(ctx);
    if (ctx->side) {
        // release paths: failures here leave nothing for the caller to do
        (void)hipStreamSynchronize(ctx->side);
        (void)hipEventDestroy(ctx->fork_ev);
        (void)hipEventDestroy(ctx->join_ev);
        (void)hipStreamDestroy(ctx->side);
    }
    delete ctx;
    return SLDF_OK;
}

sldf_status sldf_timing_enable(sldf_ctx* ctx, int32_t max_runs)
{
    if (!ctx || max_runs < 0 || max_runs > (1 << 20)) return SLDF_EINVAL;
    free_events(ctx);
    memset(ctx->launches, 0, sizeof(ctx->launches));
    if (max_runs == 0) return SLDF_OK;
    const int64_t n = (int64_t)max_runs * kMarks;
    ctx->events = new (std::nothrow) hipEvent_t[n];
    if (!ctx->events) return SLDF_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        if (hipEventCreate(&ctx->events[i]) != hipSuccess) {
            for (int64_t j = 0; j < i; ++j) (void)hipEventDestroy(ctx->events[j]);
            delete[] ctx->events;
            ctx->events = nullptr;
            return SLDF_EDEVICE;
        }
    }
    ctx->timing_cap = max_runs;
    ctx->timing_runs = 0;
    return SLDF_OK;
}

sldf_status sldf_timing_read(sldf_ctx* ctx, double* ms, int64_t* launches)
{
    if (!ctx || !ms || !launches) return SLDF_EINVAL;
    if (!ctx->events) return SLDF_ESTATE;
    for (int k = 0; k < SLDF_NUM_STAGES; ++k) ms[k] = 0.0;
    for (int r = 0; r < ctx->timing_runs; ++r) {
        hipEvent_t* m = ctx->events + (size_t)r * kMarks;
        if (hipEventSynchronize(m[kMarks - 1]) != hipSuccess) return SLDF_EDEVICE;
        for (int k = 0; k < SLDF_NUM_STAGES; ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, m[k], m[k + 1]) != hipSuccess) return SLDF_EDEVICE;
            ms[k] += t;
        }
    }
    for (int k = 0; k < SLDF_NUM_STAGES; ++k) launches[k] = ctx->launches[k];
    memset(ctx->launches, 0, sizeof(ctx->launches));
    ctx->timing_runs = 0;
    return SLDF_OK;
}

sldf_status sldf_set_taps(sldf_ctx* ctx, const sldf_taps* taps)
{
    if (!ctx) return SLDF_EINVAL;
    if (taps && taps->path_cost && (taps->path_dir < 0 || taps->path_dir > 7)) return SLDF_EINVAL;
    if (taps)
        ctx->taps = *taps;
    else
        memset(&ctx->taps, 0, sizeof(ctx->taps));
    return SLDF_OK;
}

sldf_status sldf_run_batch(sldf_ctx* ctx, int32_t n_frames, const uint8_t* left,
                           const uint8_t* right, int32_t img_pitch,
                           int64_t img_frame_stride, const int16_t* lidar,
                           int32_t lidar_pitch, int64_t lidar_frame_stride,
                           float* disp_out, uint8_t* valid_out, int32_t out_pitch,
                           int64_t out_frame_stride, void* hip_stream)
{
    if (!ctx) return SLDF_EINVAL;
    const sldf_params& p = ctx->p;
    if (n_frames < 1 || n_frames > p.batch) return SLDF_EINVAL;
    if (!left || !right || !lidar || !disp_out || !valid_out) return SLDF_EINVAL;
    if (img_pitch < p.width || lidar_pitch < p.width || out_pitch < p.width)
        return SLDF_EINVAL;
    if (n_frames > 1) {
        if (img_frame_stride < (int64_t)img_pitch * p.height ||
            lidar_frame_stride < (int64_t)lidar_pitch * p.height ||
            out_frame_stride < (int64_t)out_pitch * p.height)
            return SLDF_EINVAL;
    }
    if ((((uintptr_t)left | (uintptr_t)right) & 15) != 0 || (img_pitch & 15) != 0 ||
        (n_frames > 1 && (img_frame_stride & 15) != 0))
        return SLDF_EALIGN;
    if (((uintptr_t)lidar & 1) != 0 || ((uintptr_t)disp_out & 3) != 0) return SLDF_EALIGN;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) return SLDF_ESTATE;
    const bool learned = p.check_impl == 1;
    if (learned && (!ctx->sur_w || !ctx->sur_b)) return SLDF_ESTATE;
    hipStream_t s = (hipStream_t)hip_stream;
    const Buffers& b = ctx->buf;
    const int W = p.width, H = p.height, D = p.max_disp;
    hipError_t e;
    hipEvent_t* marks = nullptr;
    if (ctx->events) {
        if (ctx->timing_runs >= ctx->timing_cap) return SLDF_ESTATE;
        marks = ctx->events + (size_t)ctx->timing_runs * kMarks;
        ctx->timing_runs++;
    }
    auto mark = [&](int k) {
        return marks ? hipEventRecord(marks[k], s) : hipSuccess;
    };
    if (mark(0) != hipSuccess) return SLDF_EDEVICE;
    if (learned && launch_fill_i32(b.counter, n_frames, 0, s) != hipSuccess) return SLDF_EDEVICE;

    // census of both images (Sec. IV-A)
    CensusArgs ca;
    ca.left = left;
    ca.right = right;
    ca.pitch = img_pitch;
    ca.img_fstride = img_frame_stride;
    ca.out_l = b.census_l;
    ca.out_r = b.census_r;
    ca.out_pitch = b.census_pitch;
    ca.out_fstride = b.census_fstride;
    ca.W = W;
    ca.H = H;
    ca.cw = p.census_w;
    ca.ch = p.census_h;
    ca.kind = p.census_kind;
    if ((e = launch_census(ca, n_frames, s)) != hipSuccess) return SLDF_EDEVICE;
    if (mark(1) != hipSuccess) return SLDF_EDEVICE;
    ctx->launches[0] += 1;

    // prior words: semidensification (Sec. IV-B, SDSGM only) or D-bar
    // itself (DSGM), guard rings, the right view's shared map
    PriorOut po;
    po.words = b.pword[0];
    po.pitch = b.pword_pitch;
    po.fstride = b.pword_fstride;
    po.w_prior = (uint32_t)(p.alpha_den - p.alpha_num);
    po.w_noprior = (uint32_t)(p.blend_mode ? p.alpha_den : p.alpha_den - p.alpha_num);
    po.tap = (int16_t*)ctx->taps.prior;
    if (launch_prior_guards(po, b.pword[1], po.w_noprior, W, H, D, n_frames, s) != hipSuccess)
        return SLDF_EDEVICE;
    if (p.semidense) {
        SemiArgs sa;
        sa.census_l = b.census_l;
        sa.census_r = b.census_r;
        sa.census_pitch = b.census_pitch;
        sa.census_fstride = b.census_fstride;
        sa.lidar = lidar;
        sa.lidar_pitch = lidar_pitch;
        sa.lidar_fstride = lidar_frame_stride;
        sa.out = po;
        sa.W = W;
        sa.H = H;
        sa.D = D;
        sa.n = ctx->n;
        sa.ts = p.ts;
        sa.rs = p.rs;
        if ((e = launch_semidense(sa, n_frames, s)) != hipSuccess) return SLDF_EDEVICE;
        ctx->launches[1] += 1;
    } else if ((e = launch_prior_words(lidar, lidar_pitch, lidar_frame_stride, po, W, H, D,
                                       n_frames, s)) != hipSuccess) {
        return SLDF_EDEVICE;
    }
    if (mark(2) != hipSuccess) return SLDF_EDEVICE;

    // path aggregation with fused cost, WTA + subpixel in the last path
    SgmArgs ga;
    memset(&ga, 0, sizeof(ga));
    ga.cbase[0] = b.census_l;
    ga.cmatch[0] = b.census_r;
    ga.cbase[1] = b.census_r;
    ga.cmatch[1] = b.census_l;
    ga.census_pitch = b.census_pitch;
    ga.census_fstride = b.census_fstride;
    ga.pword[0] = b.pword[0];
    ga.pword[1] = b.pword[1];
    ga.pword_pitch = b.pword_pitch;
    ga.pword_fstride[0] = b.pword_fstride;
    ga.pword_fstride[1] = 0;
    ga.S[0] = b.S_left;
    ga.S[1] = b.S_right;
    ga.wta[0] = b.dstar;
    ga.wta[1] = b.dright;
    ga.dsub = b.dsub;
    ga.px_stride = b.px_stride;
    ga.S_stride = b.S_stride;
    ga.W = W;
    ga.H = H;
    ga.n = ctx->n;
    ga.prior_cost = p.prior_cost;
    ga.huber_k = p.huber_k;
    ga.q1s = (uint32_t)(p.alpha_num * p.q1);
    ga.q2s = (uint32_t)(p.alpha_num * p.q2);
    ga.p1s = (uint32_t)(p.alpha_den * p.p1);
    ga.p2s = (uint32_t)(p.alpha_den * p.p2);
    ga.subpixel = p.subpixel;
    ga.store_sum = ctx->taps.cost_sum != nullptr;
    const bool want_features = learned || ctx->taps.features != nullptr;
    ga.feat = want_features ? b.feat : nullptr;
    // plain check: both views in every launch; learned check: left view
    // here, right view only in the gated fallback below
    const int nviews = ctx->need_right && !learned ? 2 : 1;
    ga.ckpt = b.ckpt;
    // LiDAR window test arguments (used after the path passes, or for the
    // masks on the second stream)
    LidarArgs la;
    la.lidar = lidar;
    la.lidar_pitch = lidar_pitch;
    la.lidar_fstride = lidar_frame_stride;
    la.rowbits = b.rowbits;
    la.dstar = b.dstar;
    la.rho = b.rho;
    la.feat = b.feat;
    la.x0 = want_features ? b.x0 : nullptr;
    la.px_stride = b.px_stride;
    la.W = W;
    la.H = H;
    la.D = D;
    la.rc = p.rc;
    la.sS = 1.0f / (float)(p.num_paths * p.alpha_den * p.p2);
    la.sD = 1.0f / (float)D;
    la.sR = 1.0f / 32.0f;
    la.wmask = nullptr;
    la.nframes = n_frames;
    bool masks_done = false;
    auto sgm_passes = [&](int view_base, int nv, int stage) {
        ga.view_base = view_base;
        if (p.num_paths == 1) {
            ga.dx = kDirs[0][0];
            ga.dy = kDirs[0][1];
            ga.nlines = num_lines(W, H, ga.dx, ga.dy);
            if (launch_sgm_dir(ga, D, kSingle, nv, n_frames, s) != hipSuccess) return false;
            ctx->launches[stage] += 1;
            return true;
        }
        if (b.hand && (p.schedule == 3 || (p.schedule == 0 && n_frames >= kSweepMinFrames))) {
            // two sweeps: S written once (sweep A, four directions) and read
            // once (sweep B, the other four, WTA); the handoff buffer and the
            // launch words start at zero (then every launch leaves them so)
            if (!ctx->sweep_ready) {
                if (launch_fill_i32((int32_t*)b.hand, (int64_t)(b.hand_bytes / 4), 0, s) != hipSuccess ||
                    launch_fill_i32(b.sync, 4, 0, s) != hipSuccess)
                    return false;
                ctx->sweep_ready = 1;
            }
            ga.hand = b.hand;
            ga.sync = b.sync;
            ga.npaths = p.num_paths;
            for (int pass = 0; pass < 2; ++pass) {
                if (launch_sgm_sweep(ga, D, pass, nv, n_frames, s) != hipSuccess) return false;
                ctx->launches[stage] += 1;
            }
            return true;
        }
        const int npairs = p.num_paths / 2;
        // single frames: the split schedule.  The horizontal pair (the
        // longest lines, and the fewest) runs its two directions as separate
        // line passes, r into S and -r into S2, so one pass of a row's
        // length is on its critical path instead of three; the next pair
        // folds S2 into S (8 paths), or both pairs are split and one WTA pass
        // takes S + S2 (4 paths).  The price is the S2 traffic.
        const bool split = p.schedule != 1 && n_frames <= kSplitFrames && b.S2[view_base] &&
                           (nv == 1 || b.S2[view_base + 1]);
        if (split && npairs == 4 && ctx->side) {
            // 8 paths on two streams: the main stream runs the split
            // horizontal pair (r into S, -r into S2) and then the -x+y
            // diagonal pair, which folds S2 into S; the second stream runs
            // the vertical pair into S3 and then the +x+y diagonal pair on
            // S3, with checkpoints of its own.  After the join one WTA pass
            // takes S + S3.  Each line pass is as in the other schedules, so
            // the results are identical; the two chains fill a machine that
            // one single-frame pass leaves mostly idle.
            ga.S2[0] = b.S2[0];
            ga.S2[1] = b.S2[1];
            SgmArgs gs = ga;
            gs.S[0] = b.S3[0];
            gs.S[1] = b.S3[1];
            gs.ckpt = b.ckpt2;
            // the split pass heads the longer chain: it is enqueued first (the
            // host's launch work for the other chain then overlaps it)
            if (hipEventRecord(ctx->fork_ev, s) != hipSuccess) return false;
            const int kd = D <= 128 ? 4 : 8;
            ga.dx = kPairDirs[0][0];
            ga.dy = kPairDirs[0][1];
            ga.nlines = num_lines(W, H, ga.dx, ga.dy);
            if (launch_sgm_dual(ga, D, kFirst, nv, n_frames, s, kd) != hipSuccess) return false;
            if (hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0) != hipSuccess) return false;
            if (view_base == 0 && b.wmask) {
                // the LiDAR window masks first: the second stream's chain is
                // the shorter one
                LidarArgs lm = la;
                lm.wmask = b.wmask;
                if (launch_lidar_bits(lm, n_frames, ctx->side) != hipSuccess) return false;
                masks_done = true;
            }
            for (int k = 1; k <= 2; ++k) {
                gs.dx = kPairDirs[k][0];
                gs.dy = kPairDirs[k][1];
                gs.nlines = num_lines(W, H, gs.dx, gs.dy);
                if (launch_sgm_pair(gs, D, k == 1 ? kFirst : kMiddle, nv, n_frames, ctx->side) !=
                    hipSuccess)
                    return false;
                ctx->launches[stage] += 1;
            }
            if (hipEventRecord(ctx->join_ev, ctx->side) != hipSuccess) return false;
            ga.dx = kPairDirs[3][0];
            ga.dy = kPairDirs[3][1];
            ga.nlines = num_lines(W, H, ga.dx, ga.dy);
            if (launch_sgm_pair(ga, D, kMiddle2, nv, n_frames, s) != hipSuccess) return false;
            if (hipStreamWaitEvent(s, ctx->join_ev, 0) != hipSuccess) return false;
            SgmArgs gw = ga;
            gw.S2[0] = b.S3[0];
            gw.S2[1] = b.S3[1];
            if (launch_sgm_wta(gw, D, nv, n_frames, s) != hipSuccess) return false;
            ctx->launches[stage] += 3;
            return true;
        }
        if (split) {
            ga.S2[0] = b.S2[0];
            ga.S2[1] = b.S2[1];
            // the split passes take four disparities per lane (twice the
            // lanes per line: a line step is half the instructions) up to
            // D = 128; the pairs keep eight (measured: their step time does
            // not shrink with four)
            const int kd = D <= 128 ? 4 : 8;
            for (int k = 0; k < npairs; ++k) {
                ga.dx = kPairDirs[k][0];
                ga.dy = kPairDirs[k][1];
                ga.nlines = num_lines(W, H, ga.dx, ga.dy);
                hipError_t e2;
                if (k == 0 || npairs == 2)
                    e2 = launch_sgm_dual(ga, D, k == 0 ? kFirst : kMiddle, nv, n_frames, s, kd);
                else
                    e2 = launch_sgm_pair(ga, D, k == 1 ? kMiddle2 : k == npairs - 1 ? kLast : kMiddle,
                                         nv, n_frames, s);
                if (e2 != hipSuccess) return false;
                ctx->launches[stage] += 1;
            }
            if (npairs == 2) {
                if (launch_sgm_wta(ga, D, nv, n_frames, s) != hipSuccess) return false;
                ctx->launches[stage] += 1;
            }
            return true;
        }
        // opposite directions in pairs: S is read-modified-written once per pair
        for (int k = 0; k < npairs; ++k) {
            ga.dx = kPairDirs[k][0];
            ga.dy = kPairDirs[k][1];
            ga.nlines = num_lines(W, H, ga.dx, ga.dy);
            const int mode = k == 0 ? kFirst : k == npairs - 1 ? kLast : kMiddle;
            if (launch_sgm_pair(ga, D, mode, nv, n_frames, s) != hipSuccess) return false;
            ctx->launches[stage] += 1;
        }
        return true;
    };
    if (!sgm_passes(0, nviews, 2)) return SLDF_EDEVICE;
    if (mark(3) != hipSuccess) return SLDF_EDEVICE;

    // LiDAR window masks and residual (the LiDAR half of Eq. 6), surrogate
    // inputs when requested; on two streams the masks (which do not need d*)
    // were computed on the second stream beside the path passes
    if (masks_done) {
        LidarArgs lr = la;
        lr.wmask = b.wmask;
        if ((e = launch_lidar_rho(lr, n_frames, s)) != hipSuccess) return SLDF_EDEVICE;
    } else if ((e = launch_lidar_bits(la, n_frames, s)) != hipSuccess) {
        return SLDF_EDEVICE;
    }
    if (la.x0 && launch_occlusion(b.dstar, b.x0, W, H, b.px_stride, n_frames, s) != hipSuccess)
        return SLDF_EDEVICE;

    // stereo-LiDAR consistency check (Sec. IV-C, Eq. 6)
    CheckArgs ka;
    ka.gate = nullptr;
    ka.gate_limit = 0;
    ka.dstar = b.dstar;
    ka.dright = b.dright;
    ka.dsub = b.dsub;
    ka.rho = b.rho;
    ka.disp_out = disp_out;
    ka.valid_out = valid_out;
    ka.out_pitch = out_pitch;
    ka.out_fstride = out_frame_stride;
    ka.px_stride = b.px_stride;
    ka.W = W;
    ka.H = H;
    ka.tc = p.tc;
    ka.rc = p.rc;
    ka.mode = p.check_mode;
    if (!learned) {
        if ((e = launch_check(ka, n_frames, s)) != hipSuccess) return SLDF_EDEVICE;
        ctx->launches[3] += 1;
        if (mark(4) != hipSuccess || mark(5) != hipSuccess) return SLDF_EDEVICE;
    } else {
        // learned check: CNN on the surrogate inputs, then the mask
        const uint16_t* w = ctx->sur_w;
        const float* bb = ctx->sur_b;
        const uint16_t* in = b.x0;
        for (int l = 0; l < 4; ++l) {
            ConvArgs cv;
            cv.x = in;
            cv.w = w + (l == 0 ? kSurOffW1 : l == 1 ? kSurOffW2 : l == 2 ? kSurOffW3 : kSurOffW4);
            cv.bias = bb + (l == 0 ? kSurOffB1 : l == 1 ? kSurOffB2 : l == 2 ? kSurOffB3 : kSurOffB4);
            cv.y = l < 3 ? b.act[l & 1] : nullptr;
            cv.yf = l == 3 ? b.logits : nullptr;
            cv.gate = nullptr;
            cv.px_stride = b.px_stride;
            cv.W = W;
            cv.H = H;
            cv.dil = kSurDil[l];
            cv.relu = l < 3;
            cv.cout = l < 3 ? 32 : 1;
            if (launch_conv(cv, l == 0 ? 8 : 32, l < 3 ? 32 : 16, n_frames, s) != hipSuccess)
                return SLDF_EDEVICE;
            in = b.act[l & 1];
        }
        MaskArgs ma;
        ma.logits = b.logits;
        ma.rho = b.rho;
        ma.dsub = b.dsub;
        ma.disp_out = disp_out;
        ma.valid_out = valid_out;
        ma.counter = b.counter;
        ma.px_stride = b.px_stride;
        ma.out_pitch = out_pitch;
        ma.out_fstride = out_frame_stride;
        ma.W = W;
        ma.H = H;
        ma.tc = p.tc;
        ma.margin = p.uncertain_margin;
        if (launch_learned_mask(ma, n_frames, s) != hipSuccess) return SLDF_EDEVICE;
        ctx->launches[3] += 5;
        if (mark(4) != hipSuccess) return SLDF_EDEVICE;
        // fallback: frames with too many uncertain pixels run the right-view
        // SGM and the plain check (every block tests the device counter)
        const int32_t limit = (int32_t)(p.fallback_tau * (float)W * (float)H);
        ga.gate = b.counter;
        ga.gate_limit = limit;
        ga.feat = nullptr;
        ga.store_sum = 0;
        if (!sgm_passes(1, 1, 4)) return SLDF_EDEVICE;
        ka.gate = b.counter;
        ka.gate_limit = limit;
        if ((e = launch_check(ka, n_frames, s)) != hipSuccess) return SLDF_EDEVICE;
        ctx->launches[4] += 1;
        if (mark(5) != hipSuccess) return SLDF_EDEVICE;
    }

    // debug taps of frame 0
    const sldf_taps& t = ctx->taps;
    const size_t px = (size_t)W * H;
    auto cp = [&](void* dst, const void* src, size_t bytes) {
        return dst && src ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s) : hipSuccess;
    };
    auto cp_census = [&](void* dst, const uint32_t* src) {
        return dst ? hipMemcpy2DAsync(dst, (size_t)W * 4, src, (size_t)b.census_pitch * 4,
                                      (size_t)W * 4, H, hipMemcpyDeviceToDevice, s)
                   : hipSuccess;
    };
    if (cp_census(t.census_l, b.census_l) != hipSuccess ||
        cp_census(t.census_r, b.census_r) != hipSuccess ||
        cp(t.dstar, b.dstar, px * 2) != hipSuccess ||
        cp(t.dsub, b.dsub, px * 4) != hipSuccess ||
        cp(t.cost_sum, b.S_left, px * D * 2) != hipSuccess)
        return SLDF_EDEVICE;
    if (t.dright && ctx->need_right && cp(t.dright, b.dright, px * 2) != hipSuccess)
        return SLDF_EDEVICE;
    if (cp(t.rho, b.rho, px * 2) != hipSuccess || cp(t.features, b.x0, px * 16) != hipSuccess)
        return SLDF_EDEVICE;
    if (b.sync && cp(t.sweep_errors, b.sync + 2, 4) != hipSuccess) return SLDF_EDEVICE;
    // joint cost and one direction's path cost of frame 0 (left view): the
    // passes never store them, so they are recomputed here from the census
    // and prior words of the run
    if (t.cost || t.path_cost) {
        SgmArgs gt = ga;
        gt.gate = nullptr;
        gt.feat = nullptr;
        gt.store_sum = 0;
        gt.view_base = 0;
        if (t.cost && launch_cost_tap(gt, D, t.cost, s) != hipSuccess) return SLDF_EDEVICE;
        if (t.path_cost) {
            gt.S[0] = t.path_cost;
            gt.dx = kDirs[t.path_dir][0];
            gt.dy = kDirs[t.path_dir][1];
            gt.nlines = num_lines(W, H, gt.dx, gt.dy);
            if (launch_sgm_dir(gt, D, kFirst, 1, 1, s) != hipSuccess) return SLDF_EDEVICE;
        }
    }
    return SLDF_OK;
}

sldf_status sldf_run(sldf_ctx* ctx, const uint8_t* left, const uint8_t* right,
                     int32_t img_pitch, const int16_t* lidar, int32_t lidar_pitch,
                     float* disp_out, uint8_t* valid_out, int32_t out_pitch,
                     void* hip_stream)
{
    return sldf_run_batch(ctx, 1, left, right, img_pitch, 0, lidar, lidar_pitch, 0,
                          disp_out, valid_out, out_pitch, 0, hip_stream);
}

}  // extern "C"

// Workspace of sldf_run_noalloc: one static device array per GPU, fixed size.
// In host code `scratch` names a host-side stand-in, not a device address:
// its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is handed to the kernels.
static __device__ __align__(256) unsigned char scratch[SLDF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch[kMaxDevices] = {};

// device address of this device's scratch array (dev is current), or null
void* scratch_ptr(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" {

sldf_status sldf_run_noalloc(const sldf_params* params, const uint8_t* left,
                             const uint8_t* right, int32_t img_pitch, const int16_t* lidar,
                             int32_t lidar_pitch, float* disp_out, uint8_t* valid_out,
                             int32_t out_pitch, void* hip_stream)
{
    if (!params) return SLDF_EINVAL;
    sldf_params p = *params;
    sldf_status st = validate(&p);
    if (st != SLDF_OK) return st;
    if (p.check_impl != 0) return SLDF_EINVAL;     // no surrogate weights here
    // one frame on the caller's stream only: the paired schedule (no second
    // stream, no split cost terms; the results are the same for every schedule)
    p.batch = 1;
    if (p.schedule != 3) p.schedule = 1;
    const size_t need = plan(&p, nullptr, nullptr);
    if (need > (size_t)SLDF_NOALLOC_SCRATCH_BYTES) return SLDF_ENOMEM;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SLDF_EDEVICE;
    char* ws = (char*)scratch_ptr(dev);
    if (!ws) return SLDF_EDEVICE;
    // a context on the stack over the static workspace: no host or device
    // allocation; everything the passes read is written earlier in the call
    sldf_ctx c;
    memset(&c, 0, sizeof(c));
    c.p = p;
    c.device = dev;
    plan(&p, ws, &c.buf);
    c.need_right = needs_right(&p);
    c.n = census_bits(&p);
    return sldf_run_batch(&c, 1, left, right, img_pitch, 0, lidar, lidar_pitch, 0, disp_out,
                          valid_out, out_pitch, 0, hip_stream);
}

int32_t sldf_surrogate_num_weights(void) { return kSurNW; }
int32_t sldf_surrogate_num_biases(void) { return kSurNB; }

sldf_status sldf_surrogate_set_weights(sldf_ctx* ctx, const uint16_t* weights,
                                       const float* biases)
{
    if (!ctx || (!weights) != (!biases)) return SLDF_EINVAL;
    ctx->sur_w = weights;
    ctx->sur_b = biases;
    return SLDF_OK;
}

static size_t surrogate_bias_offset()
{
    return align_up((size_t)sldf_surrogate_num_weights() * 2, 256);
}

size_t sldf_surrogate_blob_bytes(void)
{
    return surrogate_bias_offset() + (size_t)sldf_surrogate_num_biases() * 4;
}

sldf_status sldf_surrogate_load(sldf_ctx* ctx, const void* blob, size_t bytes)
{
    if (!ctx || !blob || bytes != sldf_surrogate_blob_bytes() || ((uintptr_t)blob & 255))
        return SLDF_EINVAL;
    const char* b = static_cast<const char*>(blob);
    return sldf_surrogate_set_weights(ctx, reinterpret_cast<const uint16_t*>(b),
                                      reinterpret_cast<const float*>(b + surrogate_bias_offset()));
}

sldf_status sldf_fallback_read(sldf_ctx* ctx, int32_t* counts, int32_t n, int32_t* limit)
{
    if (!ctx || !counts || !limit || n < 1 || n > ctx->p.batch) return SLDF_EINVAL;
    if (ctx->p.check_impl != 1) return SLDF_ESTATE;
    if (hipMemcpy(counts, ctx->buf.counter, (size_t)n * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return SLDF_EDEVICE;
    *limit = (int32_t)(ctx->p.fallback_tau * (float)ctx->p.width * (float)ctx->p.height);
    return SLDF_OK;
}

namespace {

hipError_t surrogate_forward(const uint16_t* x0, int W, int H, int F, const uint16_t* w,
                             const float* bb, uint16_t* const act[3], float* logits,
                             hipStream_t s)
{
    const uint16_t* in = x0;
    for (int l = 0; l < 4; ++l) {
        ConvArgs cv;
        cv.x = in;
        cv.w = w + (l == 0 ? kSurOffW1 : l == 1 ? kSurOffW2 : l == 2 ? kSurOffW3 : kSurOffW4);
        cv.bias = bb + (l == 0 ? kSurOffB1 : l == 1 ? kSurOffB2 : l == 2 ? kSurOffB3 : kSurOffB4);
        cv.y = l < 3 ? act[l] : nullptr;
        cv.yf = l == 3 ? logits : nullptr;
        cv.gate = nullptr;
        cv.px_stride = (int64_t)W * H;
        cv.W = W;
        cv.H = H;
        cv.dil = kSurDil[l];
        cv.relu = l < 3;
        cv.cout = l < 3 ? 32 : 1;
        hipError_t e = launch_conv(cv, l == 0 ? 8 : 32, l < 3 ? 32 : 16, F, s);
        if (e != hipSuccess) return e;
        if (l < 3) in = act[l];
    }
    return hipSuccess;
}

constexpr int kWgRows = 8;

// training workspace plan (byte offsets, 256-aligned)
struct TrainPlan {
    size_t a1, a2, a3, z, dz, d3, d2, d1, wt4, wt3, wt2, pw, pb, grads, pl, pc, pa, stats, total;
};

TrainPlan train_plan(int W, int H, int F)
{
    TrainPlan t;
    const size_t px = (size_t)W * H * F;
    const size_t wblocks = (size_t)F * ((H + kWgRows - 1) / kWgRows);
    const size_t lblocks = (size_t)F * (((size_t)W * H + 255) / 256);
    size_t off = 0;
    auto seg = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    t.a1 = seg(px * 64);
    t.a2 = seg(px * 64);
    t.a3 = seg(px * 64);
    t.z = seg(px * 4);
    t.dz = seg(px * 16);
    t.d3 = seg(px * 64);
    t.d2 = seg(px * 64);
    t.d1 = seg(px * 64);
    t.wt4 = seg(9 * 32 * 8 * 2);
    t.wt3 = seg(9 * 32 * 32 * 2);
    t.wt2 = seg(9 * 32 * 32 * 2);
    t.pw = seg(wblocks * 9 * 32 * 32 * 4);
    t.pb = seg(wblocks * 32 * 4);
    t.grads = seg((size_t)(kSurNW + kSurNB) * 4);
    t.pl = seg(lblocks * 4);
    t.pc = seg(lblocks * 4);
    t.pa = seg(lblocks * 4);
    t.stats = seg(16);
    t.total = off;
    return t;
}

}  // namespace

sldf_status sldf_surrogate_forward(const uint16_t* x0, int32_t width, int32_t height,
                                   int32_t n_frames, const uint16_t* weights,
                                   const float* biases, uint16_t* act1, uint16_t* act2,
                                   uint16_t* act3, float* logits, void* hip_stream)
{
    if (!x0 || !weights || !biases || !act1 || !act2 || !act3 || !logits || width < 1 ||
        height < 1 || n_frames < 1)
        return SLDF_EINVAL;
    if ((((uintptr_t)x0 | (uintptr_t)act1 | (uintptr_t)act2 | (uintptr_t)act3 |
          (uintptr_t)weights) & 15) != 0)
        return SLDF_EALIGN;
    uint16_t* const act[3] = {act1, act2, act3};
    return surrogate_forward(x0, width, height, n_frames, weights, biases, act, logits,
                             (hipStream_t)hip_stream) == hipSuccess
               ? SLDF_OK
               : SLDF_EDEVICE;
}

sldf_status sldf_surrogate_sync_weights(const float* master, uint16_t* weights, float* biases,
                                        void* hip_stream)
{
    if (!master || !weights || !biases) return SLDF_EINVAL;
    return launch_sync_weights(master, weights, biases, (hipStream_t)hip_stream) == hipSuccess
               ? SLDF_OK
               : SLDF_EDEVICE;
}

sldf_status sldf_surrogate_train_workspace_size(int32_t width, int32_t height,
                                                int32_t n_frames, size_t* bytes)
{
    if (!bytes || width < 1 || height < 1 || n_frames < 1) return SLDF_EINVAL;
    *bytes = train_plan(width, height, n_frames).total;
    return SLDF_OK;
}

sldf_status sldf_surrogate_train_step(const uint16_t* x0, const uint8_t* labels,
                                      const uint16_t* rho, int32_t tc, int32_t width,
                                      int32_t height, int32_t n_frames, float* master,
                                      float* adam_m, float* adam_v, uint16_t* weights,
                                      float* biases, float lr, float beta1, float beta2,
                                      float eps, int32_t step, int32_t apply_update,
                                      void* workspace, size_t ws_bytes, float* grads_out,
                                      float* stats_out, void* hip_stream)
{
    if (!x0 || !labels || !rho || !master || !adam_m || !adam_v || !weights || !biases ||
        !workspace || width < 1 || height < 1 || n_frames < 1 || step < 1)
        return SLDF_EINVAL;
    if ((((uintptr_t)x0 | (uintptr_t)weights | (uintptr_t)workspace) & 15) != 0)
        return SLDF_EALIGN;
    const int W = width, H = height, F = n_frames;
    const TrainPlan tp = train_plan(W, H, F);
    if (ws_bytes < tp.total) return SLDF_ENOMEM;
    hipStream_t s = (hipStream_t)hip_stream;
    char* ws = (char*)workspace;
    uint16_t* a1 = (uint16_t*)(ws + tp.a1);
    uint16_t* a2 = (uint16_t*)(ws + tp.a2);
    uint16_t* a3 = (uint16_t*)(ws + tp.a3);
    float* z = (float*)(ws + tp.z);
    uint16_t* dz = (uint16_t*)(ws + tp.dz);
    uint16_t* d3 = (uint16_t*)(ws + tp.d3);
    uint16_t* d2 = (uint16_t*)(ws + tp.d2);
    uint16_t* d1 = (uint16_t*)(ws + tp.d1);
    uint16_t* wt4 = (uint16_t*)(ws + tp.wt4);
    uint16_t* wt3 = (uint16_t*)(ws + tp.wt3);
    uint16_t* wt2 = (uint16_t*)(ws + tp.wt2);
    float* pw = (float*)(ws + tp.pw);
    float* pb = (float*)(ws + tp.pb);
    float* grads = (float*)(ws + tp.grads);
    const int64_t pxs = (int64_t)W * H;
    uint16_t* const act[3] = {a1, a2, a3};
    if (surrogate_forward(x0, W, H, F, weights, biases, act, z, s) != hipSuccess)
        return SLDF_EDEVICE;

    LossArgs la;
    la.z = z;
    la.labels = labels;
    la.rho = rho;
    la.dz = dz;
    la.partial_loss = (float*)(ws + tp.pl);
    la.partial_cnt = (int32_t*)(ws + tp.pc);
    la.partial_agree = (int32_t*)(ws + tp.pa);
    la.stats = stats_out;
    la.px_stride = pxs;
    la.tc = tc;
    la.inv_n = 1.0f / (float)(pxs * F);
    if (launch_bce(la, F, s) != hipSuccess) return SLDF_EDEVICE;

    // dgrad weights from the current (bf16) weights
    if (launch_wtrans(weights + kSurOffW4, 16, 32, 1, wt4, 32, 8, s) != hipSuccess ||
        launch_wtrans(weights + kSurOffW3, 32, 32, 32, wt3, 32, 32, s) != hipSuccess ||
        launch_wtrans(weights + kSurOffW2, 32, 32, 32, wt2, 32, 32, s) != hipSuccess)
        return SLDF_EDEVICE;

    const int nwb = (H + kWgRows - 1) / kWgRows;
    auto wgrad = [&](const uint16_t* xin, int cin, const uint16_t* g, int gc, int dil,
                     int oc_pad, int oc_valid, int woff, int boff) {
        WgradArgs wa;
        wa.x = xin;
        wa.g = g;
        wa.partial_w = pw;
        wa.partial_b = pb;
        wa.px_stride = pxs;
        wa.W = W;
        wa.H = H;
        wa.dil = dil;
        wa.rows = kWgRows;
        if (launch_wgrad(wa, cin, gc, F, s) != hipSuccess) return false;
        return launch_reduce_wgrad(pw, pb, nwb * F, oc_pad, cin, oc_valid, grads + woff,
                                   grads + kSurNW + boff, s) == hipSuccess;
    };
    auto dgrad = [&](const uint16_t* g, int gc, const uint16_t* wt, const uint16_t* gate,
                     int dil, uint16_t* out) {
        ConvArgs cv;
        cv.x = g;
        cv.w = wt;
        cv.bias = nullptr;
        cv.y = out;
        cv.yf = nullptr;
        cv.gate = gate;
        cv.px_stride = pxs;
        cv.W = W;
        cv.H = H;
        cv.dil = dil;
        cv.relu = 0;
        cv.cout = 32;
        return launch_conv(cv, gc, 32, F, s) == hipSuccess;
    };
    // layer 4 (32 -> 1, dilation 27), layer 3, layer 2, layer 1
    if (!wgrad(a3, 32, dz, 8, kSurDil[3], 16, 1, kSurOffW4, kSurOffB4) ||
        !dgrad(dz, 8, wt4, a3, kSurDil[3], d3) ||
        !wgrad(a2, 32, d3, 32, kSurDil[2], 32, 32, kSurOffW3, kSurOffB3) ||
        !dgrad(d3, 32, wt3, a2, kSurDil[2], d2) ||
        !wgrad(a1, 32, d2, 32, kSurDil[1], 32, 32, kSurOffW2, kSurOffB2) ||
        !dgrad(d2, 32, wt2, a1, kSurDil[1], d1) ||
        !wgrad(x0, 8, d1, 32, kSurDil[0], 32, 32, kSurOffW1, kSurOffB1))
        return SLDF_EDEVICE;
    if (grads_out &&
        hipMemcpyAsync(grads_out, grads, (size_t)(kSurNW + kSurNB) * 4, hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
        return SLDF_EDEVICE;
    if (apply_update) {
        AdamArgs aa;
        aa.master = master;
        aa.m = adam_m;
        aa.v = adam_v;
        aa.grad = grads;
        aa.w_bf16 = weights;
        aa.bias = biases;
        aa.n = kSurNW + kSurNB;
        aa.n_w = kSurNW;
        aa.b1 = beta1;
        aa.b2 = beta2;
        aa.eps = eps;
        const double bc1 = 1.0 - pow((double)beta1, (double)step);
        const double bc2 = 1.0 - pow((double)beta2, (double)step);
        aa.lr_t = (float)((double)lr * sqrt(bc2) / bc1);
        if (launch_adam(aa, s) != hipSuccess) return SLDF_EDEVICE;
    }
    return SLDF_OK;
}

sldf_status sldf_lidar_quantize(const float* in, int32_t width, int32_t height,
                                int32_t in_pitch, int32_t max_disp, int16_t* out,
                                int32_t out_pitch, void* hip_stream)
{
    if (!in || !out || width < 1 || height < 1 || in_pitch < width || out_pitch < width ||
        max_disp < 1 || max_disp > 32767)
        return SLDF_EINVAL;
    if (launch_quantize(in, width, height, in_pitch, max_disp, out, out_pitch,
                        (hipStream_t)hip_stream) != hipSuccess)
        return SLDF_EDEVICE;
    return SLDF_OK;
}

}  // extern "C"
