// C ABI of libsldf.so: parameter validation, workspace plan and the launch
// sequence of one frame batch (Fig. 1 flow of the paper).
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
    // timing
    hipEvent_t* events;
    int32_t timing_cap;     // runs that fit in events
    int32_t timing_runs;    // runs recorded since the last read
    int64_t launches[SLDF_NUM_STAGES];
};

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

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
    if (p->census_w < 1 || p->census_h < 1 || !(p->census_w & 1) || !(p->census_h & 1) ||
        p->census_w > 15 || p->census_h > 15)
        return SLDF_EINVAL;
    int n = (p->census_w * p->census_h - 1) / 2;
    if (n < 1 || n > 32) return SLDF_EINVAL;
    if (p->num_paths != 1 && p->num_paths != 4 && p->num_paths != 8) return SLDF_EINVAL;
    if (p->p1 < 0 || p->p2 < p->p1 || p->q1 < 0 || p->q2 < p->q1) return SLDF_EINVAL;
    if (p->alpha_den < 1 || p->alpha_num < 0 || p->alpha_num > p->alpha_den) return SLDF_EINVAL;
    if (p->blend_mode != 0 && p->blend_mode != 1) return SLDF_EINVAL;
    if (p->semidense != 0 && p->semidense != 1) return SLDF_EINVAL;
    if (p->ts < 0 || p->ts > 64 || p->rs < 0 || p->rs > 15) return SLDF_EINVAL;
    if (p->tc < 0 || p->tc > 4096 || p->rc < 0 || p->rc > 31) return SLDF_EINVAL;
    if (p->check_mode < 0 || p->check_mode > 3) return SLDF_EINVAL;
    if (p->check_impl != 0) return SLDF_EINVAL;
    if (p->subpixel != 0 && p->subpixel != 1) return SLDF_EINVAL;
    if (p->batch < 1 || p->batch > 4096) return SLDF_EINVAL;
    // 16-bit bound: every L_r lies in [C', C' + P2'] (Eq. 2), the sum of the
    // paths in [|R| C', |R| (C' + P2')], and the largest intermediate of the
    // recurrence is C' + P2' + P1' (neighbour term) or m + P2' <= C' + 2 P2'.
    int64_t cmax = max_cost(p, n);
    int64_t P1 = (int64_t)p->alpha_den * p->p1, P2 = (int64_t)p->alpha_den * p->p2;
    if ((int64_t)p->num_paths * (cmax + P2) >= 65536) return SLDF_EOVERFLOW;
    if (cmax + P2 + (P1 > P2 ? P1 : P2) >= 65536) return SLDF_EOVERFLOW;
    if ((int64_t)p->alpha_num * p->q2 >= 65536) return SLDF_EOVERFLOW;
    return SLDF_OK;
}

bool needs_right(const sldf_params* p) { return p->check_mode == 1 || p->check_mode == 3; }

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
    void* cl = seg(F * cframe * 4);
    void* cr = seg(F * cframe * 4);
    void* pr = p->semidense ? seg(F * px * 2) : nullptr;
    void* ds = seg(F * px * 2);
    void* dr = seg(F * px * 2);
    void* dsub = seg(F * px * 4);
    void* sl = seg(F * cells * 2);
    void* sr = needs_right(p) ? seg(F * cells * 2) : nullptr;
    if (b) {
        b->census_l = base ? (uint32_t*)cl + p->max_disp : nullptr;
        b->census_r = base ? (uint32_t*)cr + p->max_disp : nullptr;
        b->census_pitch = (int32_t)cpitch;
        b->census_fstride = (int64_t)cframe;
        b->prior = (int16_t*)pr;
        b->dstar = (int16_t*)ds;
        b->dright = (int16_t*)dr;
        b->dsub = (float*)dsub;
        b->S_left = (uint16_t*)sl;
        b->S_right = (uint16_t*)sr;
        b->px_stride = (int64_t)px;
        b->S_stride = (int64_t)cells;
    }
    return off;
}

// Path directions: horizontal and vertical first (4-path set), then the
// diagonals (8-path set); the 1-path debug mode is left-to-right only.
const int kDirs[8][2] = {{+1, 0}, {-1, 0}, {0, +1}, {0, -1},
                         {+1, +1}, {-1, +1}, {+1, -1}, {-1, -1}};

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
    c->n = (p->census_w * p->census_h - 1) / 2;
    *out = c;
    return SLDF_OK;
}

static void free_events(sldf_ctx* ctx)
{
    if (!ctx->events) return;
    for (int64_t i = 0; i < (int64_t)ctx->timing_cap * kMarks; ++i) hipEventDestroy(ctx->events[i]);
    delete[] ctx->events;
    ctx->events = nullptr;
    ctx->timing_cap = ctx->timing_runs = 0;
}

sldf_status sldf_destroy(sldf_ctx* ctx)
{
    if (!ctx) return SLDF_OK;
    free_events(ctx);
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
            for (int64_t j = 0; j < i; ++j) hipEventDestroy(ctx->events[j]);
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
    if ((e = launch_census(ca, n_frames, s)) != hipSuccess) return SLDF_EDEVICE;
    if (mark(1) != hipSuccess) return SLDF_EDEVICE;
    ctx->launches[0] += 1;

    // semidensification (Sec. IV-B, SDSGM only)
    const int16_t* prior = lidar;
    int32_t prior_pitch = lidar_pitch;
    int64_t prior_fstride = lidar_frame_stride;
    if (p.semidense) {
        SemiArgs sa;
        sa.census_l = b.census_l;
        sa.census_r = b.census_r;
        sa.census_pitch = b.census_pitch;
        sa.census_fstride = b.census_fstride;
        sa.lidar = lidar;
        sa.lidar_pitch = lidar_pitch;
        sa.lidar_fstride = lidar_frame_stride;
        sa.out = b.prior;
        sa.px_stride = b.px_stride;
        sa.W = W;
        sa.H = H;
        sa.n = ctx->n;
        sa.ts = p.ts;
        sa.rs = p.rs;
        if ((e = launch_semidense(sa, n_frames, s)) != hipSuccess) return SLDF_EDEVICE;
        prior = b.prior;
        prior_pitch = W;
        prior_fstride = b.px_stride;
        ctx->launches[1] += 1;
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
    ga.prior = prior;
    ga.prior_pitch = prior_pitch;
    ga.prior_fstride = prior_fstride;
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
    ga.mulh_prior = (uint32_t)(p.alpha_den - p.alpha_num);
    ga.mulh_noprior = (uint32_t)(p.blend_mode ? p.alpha_den : p.alpha_den - p.alpha_num);
    ga.q1s = (uint32_t)(p.alpha_num * p.q1);
    ga.q2s = (uint32_t)(p.alpha_num * p.q2);
    ga.p1s = (uint32_t)(p.alpha_den * p.p1);
    ga.p2s = (uint32_t)(p.alpha_den * p.p2);
    ga.subpixel = p.subpixel;
    ga.store_sum = ctx->taps.cost_sum != nullptr;
    const int nviews = ctx->need_right ? 2 : 1;
    for (int r = 0; r < p.num_paths; ++r) {
        ga.dx = kDirs[r][0];
        ga.dy = kDirs[r][1];
        ga.nlines = num_lines(W, H, ga.dx, ga.dy);
        int mode = p.num_paths == 1 ? kSingle
                   : r == 0          ? kFirst
                   : r == p.num_paths - 1 ? kLast
                                     : kMiddle;
        if ((e = launch_sgm_dir(ga, D, mode, nviews, n_frames, s)) != hipSuccess)
            return SLDF_EDEVICE;
        ctx->launches[2] += 1;
    }
    if (mark(3) != hipSuccess) return SLDF_EDEVICE;

    // stereo-LiDAR consistency check (Sec. IV-C, Eq. 6)
    CheckArgs ka;
    ka.dstar = b.dstar;
    ka.dright = b.dright;
    ka.dsub = b.dsub;
    ka.lidar = lidar;
    ka.lidar_pitch = lidar_pitch;
    ka.lidar_fstride = lidar_frame_stride;
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
    if ((e = launch_check(ka, n_frames, s)) != hipSuccess) return SLDF_EDEVICE;
    if (mark(4) != hipSuccess) return SLDF_EDEVICE;
    ctx->launches[3] += 1;

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
    if (t.prior) {
        if (p.semidense) {
            if (cp(t.prior, b.prior, px * 2) != hipSuccess) return SLDF_EDEVICE;
        } else if (hipMemcpy2DAsync(t.prior, (size_t)W * 2, lidar, (size_t)lidar_pitch * 2,
                                    (size_t)W * 2, H, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            return SLDF_EDEVICE;
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
