/*
 * Plain CPU oracle for the stereo-LiDAR SGM method (SGM with a discrete
 * disparity-matching cost, semidensification and a stereo-LiDAR consistency
 * check).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the GPU library; the two see the same seeded inputs and nothing
 * else.
 *
 * Every step is written as the straight loop of its definition, single
 * threaded, int32 arithmetic, and cites the passage of the paper it follows.
 * Section / equation numbers refer to the paper's LaTeX numbering:
 *   Sec. III     stereo SGM (Eq. 1 energy, Eq. 2 path recurrence, Eq. 3 WTA,
 *                parabola subpixel fit at the end of the section)
 *   Sec. IV-A    DDC and the joint cost (Eq. 4)
 *   Sec. IV-B    semidensification (Eq. 5)
 *   Sec. IV-C    stereo-LiDAR consistency check (Eq. 6)
 *   Tab. II      parameter values
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes):
 *   - alpha = a/b is applied exactly by scaling every cost term by b:
 *     C'(p,d) = (b-a) H + a q,  P1' = b P1,  P2' = b P2.  The argmin and the
 *     parabola offset are invariant under this positive scaling.
 *   - census: centre-symmetric census (CS-CT) with the first (w*h-1)/2
 *     window offsets in raster order, bit k set when I(p+o_k) > I(p-o_k);
 *     zero code where the window leaves the image.
 *   - Hamming cost where the matching pixel leaves the image: n (all bits).
 *   - no prior at a pixel: DDC term is 0 (blend mode 0: C' = (b-a) H) or the
 *     stereo cost alone at full weight (blend mode 1: C' = b H).
 *   - WTA and semidensification ties: smallest disparity.
 *   - subpixel: one float32 division of integers, then one float32 add.
 *   - right-view disparity d': full right-base SGM without a prior.
 *   - the check uses the integer disparity d* and the raw sparse map.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -5

/* ------------------------------------------------------------------------ */
/* Ingest: sparse LiDAR disparity map D-bar with values in N or "invalid"   */
/* (Sec. IV, definition of D-bar).  Real projections are rounded to the     */
/* nearest integer, ties to even; NaN, negative and >= D become -1.         */
/* ------------------------------------------------------------------------ */
int orc_quantize_lidar(const float* in, int W, int H, int D, int16_t* out)
{
    for (int i = 0; i < W * H; ++i) {
        float x = in[i];
        if (!(x >= 0.0f)) { out[i] = -1; continue; }   /* NaN or negative */
        float r = rintf(x);                              /* ties to even */
        if (r >= (float)D) { out[i] = -1; continue; }
        out[i] = (int16_t)r;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Census transform (Sec. IV-A: stereo cost is the Hamming distance of      */
/* census-transformed images, centre-symmetric variant).                    */
/* ------------------------------------------------------------------------ */
int orc_census_bits(int cw, int ch) { return (cw * ch - 1) / 2; }

/* Census codes (Sec. IV-A cites the census of its matching cost).  kind 0:
   the centre-symmetric census: the first n = (w h - 1) / 2 offsets o_k of
   the window in raster order (the ones before the centre), bit k =
   [I(p + o_k) > I(p - o_k)].  kind 1: the full census: every offset of the
   window but the centre, in raster order, bit k = [I(p + o_k) < I(p)]
   (w h - 1 bits, at most 32 here).  LSB first; 0 where the window leaves
   the image. */
int orc_census_kind(const uint8_t* img, int W, int H, int pitch, int cw, int ch, int kind,
                    uint32_t* out)
{
    if (cw < 1 || ch < 1 || (cw % 2) == 0 || (ch % 2) == 0 || kind < 0 || kind > 1)
        return ORC_EINVAL;
    int n = kind == 0 ? orc_census_bits(cw, ch) : cw * ch - 1;
    if (n > 32) return ORC_EINVAL;
    int rx = (cw - 1) / 2, ry = (ch - 1) / 2;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            uint32_t code = 0;
            if (x >= rx && x < W - rx && y >= ry && y < H - ry) {
                int k = 0;
                for (int dy = -ry; dy <= ry && k < n; ++dy) {
                    for (int dx = -rx; dx <= rx && k < n; ++dx) {
                        int a = img[(y + dy) * pitch + (x + dx)];
                        if (kind == 0) {
                            /* raster order over the window; the first n
                               offsets are the ones before the centre */
                            int b = img[(y - dy) * pitch + (x - dx)];
                            if (a > b) code |= (1u << k);
                            ++k;
                        } else {
                            if (dx == 0 && dy == 0) continue;
                            if (a < img[y * pitch + x]) code |= (1u << k);
                            ++k;
                        }
                    }
                }
            }
            out[y * W + x] = code;
        }
    }
    return ORC_OK;
}

int orc_census(const uint8_t* img, int W, int H, int pitch, int cw, int ch, uint32_t* out)
{
    return orc_census_kind(img, W, H, pitch, cw, ch, 0, out);
}

static int popcount32(uint32_t v)
{
    int c = 0;
    while (v) { c += (int)(v & 1u); v >>= 1; }
    return c;
}

/* Hamming cost with the left image as base: census of p against census of
   the matching pixel (x-d, y) in the right image; n where that pixel is
   outside the image. */
int orc_hamming_left(const uint32_t* cL, const uint32_t* cR, int W, int x, int y,
                     int d, int n)
{
    if (x - d < 0) return n;
    return popcount32(cL[y * W + x] ^ cR[y * W + (x - d)]);
}

/* Hamming cost with the right image as base: matching pixel (x+d, y) in the
   left image. */
int orc_hamming_right(const uint32_t* cL, const uint32_t* cR, int W, int x,
                      int y, int d, int n)
{
    if (x + d >= W) return n;
    return popcount32(cR[y * W + x] ^ cL[y * W + (x + d)]);
}

/* ------------------------------------------------------------------------ */
/* Semidensification, Eq. 5 (Sec. IV-B).                                    */
/* For each pixel p: candidates are the valid sparse disparities in the     */
/* (2 rs + 1)^2 window M_p clipped to the image.  If the smallest Hamming   */
/* cost over the candidates is below Ts, the (smallest) minimising          */
/* candidate is taken; otherwise the sparse value itself (possibly invalid) */
/* is kept.                                                                  */
/* ------------------------------------------------------------------------ */
int orc_semidense(const uint32_t* cL, const uint32_t* cR, const int16_t* lidar,
                  int W, int H, int n, int ts, int rs, int16_t* out)
{
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int best_h = 1 << 30, best_d = -1;
            for (int qy = y - rs; qy <= y + rs; ++qy) {
                if (qy < 0 || qy >= H) continue;
                for (int qx = x - rs; qx <= x + rs; ++qx) {
                    if (qx < 0 || qx >= W) continue;
                    int d = lidar[qy * W + qx];
                    if (d < 0) continue;
                    int h = orc_hamming_left(cL, cR, W, x, y, d, n);
                    if (h < best_h || (h == best_h && d < best_d)) {
                        best_h = h;
                        best_d = d;
                    }
                }
            }
            if (best_d >= 0 && best_h < ts)
                out[y * W + x] = (int16_t)best_d;
            else
                out[y * W + x] = lidar[y * W + x];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Penalty of a disparity that is adiff = |d - prior| away from the prior.   */
/* prior_cost 0: the DDC of Eq. 4 (Sec. IV-A): 0, Q1 at distance 1, Q2       */
/* beyond.  The other two are the LiDAR cost terms the paper compares DDC    */
/* with (Sec. IV-A, Sec. V-B), in the reading used here, capped at Q2 so     */
/* that the 16-bit bound of the DDC still holds:                             */
/*   1: quadratic (the LiDAR-SGM term): min(Q1 adiff^2, Q2);                 */
/*   2: Huber with threshold k: twice the Huber function, adiff^2 up to k,   */
/*      k (2 adiff - k) beyond, times Q1, capped at Q2.                      */
/* ------------------------------------------------------------------------ */
int orc_prior_penalty(int adiff, int q1, int q2, int prior_cost, int huber_k)
{
    long long r;
    if (prior_cost == 0) return adiff == 0 ? 0 : (adiff == 1 ? q1 : q2);
    if (prior_cost == 1 || adiff <= huber_k)
        r = (long long)adiff * adiff;
    else
        r = (long long)huber_k * (2LL * adiff - huber_k);
    r *= q1;
    return r < q2 ? (int)r : q2;
}

/* ------------------------------------------------------------------------ */
/* Joint matching cost, Eq. 4 (Sec. IV-A), scaled by b:                     */
/*   C'(p,d) = (b - a) H(p,d) + a * q(|d - prior_p|)                         */
/* with q the DDC (0 if d == prior, Q1 if |d - prior| == 1, Q2 otherwise)   */
/* or one of the alternative terms of orc_prior_penalty.                    */
/* prior may be NULL (no prior anywhere, as in the right-view pass).        */
/* view 0: left image is base; view 1: right image is base.                 */
/* Output layout: cost[(y * W + x) * D + d].                                */
/* ------------------------------------------------------------------------ */
int orc_joint_cost(const uint32_t* cL, const uint32_t* cR, const int16_t* prior,
                   int W, int H, int D, int n, int view, int a, int b, int q1,
                   int q2, int blend_mode, int prior_cost, int huber_k,
                   int32_t* cost)
{
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int e = prior ? prior[y * W + x] : -1;
            for (int d = 0; d < D; ++d) {
                int h = view == 0 ? orc_hamming_left(cL, cR, W, x, y, d, n)
                                  : orc_hamming_right(cL, cR, W, x, y, d, n);
                int c;
                if (e < 0) {
                    /* no sparse value here: DDC does not apply */
                    c = blend_mode == 0 ? (b - a) * h : b * h;
                } else {
                    int diff = d - e;
                    if (diff < 0) diff = -diff;
                    int q = orc_prior_penalty(diff, q1, q2, prior_cost, huber_k);
                    c = (b - a) * h + a * q;
                }
                cost[((size_t)y * W + x) * D + d] = c;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One SGM path, Eq. 2 (Sec. III).  r = (dx, dy) is the step: the           */
/* predecessor of p is p - r.  Where p - r is outside the image the path    */
/* starts: L_r(p,d) = C(p,d).  Otherwise, with m = min_k L_r(p - r, k):     */
/*   L_r(p,d) = C(p,d) + min(L_r(p-r,d), L_r(p-r,d-1) + P1,                 */
/*                           L_r(p-r,d+1) + P1, m + P2) - m                 */
/* where the d-1 / d+1 terms outside [0, D-1] are left out.                 */
/* Pixels are visited in an order where every predecessor comes first:      */
/* rows in the direction of dy (top-down if dy >= 0), columns in the        */
/* direction of dx.                                                          */
/* ------------------------------------------------------------------------ */
int orc_path(const int32_t* cost, int W, int H, int D, int dx, int dy, int P1,
             int P2, int32_t* L)
{
    if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || (dx == 0 && dy == 0))
        return ORC_EINVAL;
    for (int iy = 0; iy < H; ++iy) {
        int y = dy >= 0 ? iy : H - 1 - iy;
        for (int ix = 0; ix < W; ++ix) {
            int x = dx >= 0 ? ix : W - 1 - ix;
            const int32_t* c = cost + ((size_t)y * W + x) * D;
            int32_t* l = L + ((size_t)y * W + x) * D;
            int px = x - dx, py = y - dy;
            if (px < 0 || px >= W || py < 0 || py >= H) {
                for (int d = 0; d < D; ++d) l[d] = c[d];
                continue;
            }
            const int32_t* lp = L + ((size_t)py * W + px) * D;
            int m = lp[0];
            for (int k = 1; k < D; ++k)
                if (lp[k] < m) m = lp[k];
            for (int d = 0; d < D; ++d) {
                int best = lp[d];
                if (d - 1 >= 0 && lp[d - 1] + P1 < best) best = lp[d - 1] + P1;
                if (d + 1 < D && lp[d + 1] + P1 < best) best = lp[d + 1] + P1;
                if (m + P2 < best) best = m + P2;
                l[d] = c[d] + best - m;
            }
        }
    }
    return ORC_OK;
}

/* The path set R: 4 paths are the horizontal and vertical directions, 8 add
   the diagonals (Sec. III uses vertical, horizontal and diagonal paths).  A
   single path (num_paths == 1) is a debug mode: left-to-right only. */
static const int k_dirs[8][2] = {
    {+1, 0}, {-1, 0}, {0, +1}, {0, -1}, {+1, +1}, {-1, +1}, {+1, -1}, {-1, -1}};

int orc_direction(int i, int* dx, int* dy)
{
    if (i < 0 || i >= 8) return ORC_EINVAL;
    *dx = k_dirs[i][0];
    *dy = k_dirs[i][1];
    return ORC_OK;
}

/* Aggregated cost S(p,d) = sum over r in R of L_r(p,d) (the sum inside
   Eq. 3). */
int orc_aggregate(const int32_t* cost, int W, int H, int D, int num_paths, int P1,
                  int P2, int32_t* S)
{
    if (num_paths != 1 && num_paths != 4 && num_paths != 8) return ORC_EINVAL;
    size_t cells = (size_t)W * H * D;
    int32_t* L = (int32_t*)malloc(cells * sizeof(int32_t));
    if (!L) return ORC_ENOMEM;
    memset(S, 0, cells * sizeof(int32_t));
    for (int r = 0; r < num_paths; ++r) {
        orc_path(cost, W, H, D, k_dirs[r][0], k_dirs[r][1], P1, P2, L);
        for (size_t i = 0; i < cells; ++i) S[i] += L[i];
    }
    free(L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Winner takes all, Eq. 3, ties to the smallest d, then the parabola fit    */
/* through S(d*-1), S(d*), S(d*+1) (end of Sec. III).  At d* = 0 or D-1, or  */
/* a flat parabola, no refinement.                                           */
/* ------------------------------------------------------------------------ */
int orc_wta(const int32_t* S, int W, int H, int D, int subpixel, int32_t* dstar,
            float* dsub)
{
    for (int i = 0; i < W * H; ++i) {
        const int32_t* s = S + (size_t)i * D;
        int best = 0;
        for (int d = 1; d < D; ++d)
            if (s[d] < s[best]) best = d;
        dstar[i] = best;
        if (dsub) {
            float v = (float)best;
            if (subpixel && best > 0 && best < D - 1) {
                int A = s[best - 1], B = s[best], C = s[best + 1];
                int den = A - 2 * B + C;
                if (den > 0) {
                    float delta = (float)(A - C) / (float)(2 * den);
                    v = (float)best + delta;
                }
            }
            dsub[i] = v;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Stereo-LiDAR consistency check, Eq. 6 (Sec. IV-C).                       */
/*   stereo:  q_m = (x - d*, y) inside the image and |d* - d'(q_m)| <= 1    */
/*   LiDAR:   some valid raw sparse value in the (2 rc + 1)^2 window K_p     */
/*            (clipped) with |d* - dbar_q| <= Tc                             */
/*   mode 0: no check, 1: stereo only, 2: LiDAR only, 3: stereo OR LiDAR.   */
/* dright may be NULL when mode does not use it.                            */
/* ------------------------------------------------------------------------ */
int orc_check(const int32_t* dstar, const int32_t* dright, const int16_t* lidar,
              const float* dsub, int W, int H, int tc, int rc, int mode,
              float* disp_out, uint8_t* valid_out)
{
    if (mode < 0 || mode > 3) return ORC_EINVAL;
    if ((mode == 1 || mode == 3) && !dright) return ORC_EINVAL;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int d = dstar[y * W + x];
            int stereo_ok = 0, lidar_ok = 0;
            if (mode == 1 || mode == 3) {
                int xm = x - d;
                if (xm >= 0) {
                    int diff = d - dright[y * W + xm];
                    if (diff < 0) diff = -diff;
                    stereo_ok = diff <= 1;
                }
            }
            if (mode == 2 || mode == 3) {
                for (int qy = y - rc; qy <= y + rc && !lidar_ok; ++qy) {
                    if (qy < 0 || qy >= H) continue;
                    for (int qx = x - rc; qx <= x + rc; ++qx) {
                        if (qx < 0 || qx >= W) continue;
                        int v = lidar[qy * W + qx];
                        if (v < 0) continue;
                        int diff = d - v;
                        if (diff < 0) diff = -diff;
                        if (diff <= tc) { lidar_ok = 1; break; }
                    }
                }
            }
            int valid = mode == 0 ? 1 : (stereo_ok || lidar_ok);
            valid_out[y * W + x] = (uint8_t)valid;
            disp_out[y * W + x] = valid ? (dsub ? dsub[y * W + x] : (float)d) : -1.0f;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* LiDAR residual: rho_p = min over valid raw sparse values v in the         */
/* (2 rc + 1)^2 window K_p (clipped) of |d*_p - v|; 65535 where the window   */
/* holds none.  The LiDAR half of Eq. 6 is exactly rho_p <= Tc.              */
/* ------------------------------------------------------------------------ */
int orc_lidar_residual(const int32_t* dstar, const int16_t* lidar, int W, int H,
                       int D, int rc, uint16_t* rho)
{
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int d = dstar[y * W + x];
            int best = 65535;
            for (int qy = y - rc; qy <= y + rc; ++qy) {
                if (qy < 0 || qy >= H) continue;
                for (int qx = x - rc; qx <= x + rc; ++qx) {
                    if (qx < 0 || qx >= W) continue;
                    int v = lidar[qy * W + qx];
                    if (v < 0 || v >= D) continue;
                    int diff = d - v;
                    if (diff < 0) diff = -diff;
                    if (diff < best) best = diff;
                }
            }
            rho[y * W + x] = (uint16_t)best;
        }
    }
    return ORC_OK;
}

/* Input features of the learned consistency surrogate (an extension beside
   the paper's method; the plain check of Eq. 6 stays the reference).  Per
   pixel, from the aggregated left cost S and d*:
     f0 = S(d*)                          * sS
     f1 = min_{|d - d*| >= 2} S(d)       * sS
     f2 = S(d*-1) - 2 S(d*) + S(d*+1)    * sS   (0 at d* = 0 or D-1)
     f3 = d*                             * (1 / D)
     f4 = min(rho, 32)                   * (1 / 32)
     f5 = v                              * (1 / 16), the occlusion margin of
          the left disparity map: with q(x) = x - d*(x, y) the right-image
          pixel that (x, y) matches and m = min of q(x') over the pixels
          x' > x of the same row, v = q(x) - m clamped to [-16, 16]; v = 16
          where q(x) < 0 (no matching pixel), v = -16 at the row end (no
          pixel to the right)
   with sS = 1 / (num_paths * P2'); each product is one float32 multiply of
   the integer by the float32 scale.  out is float [H][W][6]. */
int orc_surrogate_features(const int32_t* S, const int32_t* dstar, const uint16_t* rho,
                           int W, int H, int D, int num_paths, int P2s, float* out)
{
    const float sS = 1.0f / (float)(num_paths * P2s);
    const float sD = 1.0f / (float)D;
    const float sR = 1.0f / 32.0f;
    for (int i = 0; i < W * H; ++i) {
        const int32_t* s = S + (size_t)i * D;
        int d = dstar[i];
        int second = 1 << 30;
        for (int k = 0; k < D; ++k) {
            int diff = k - d;
            if (diff < 0) diff = -diff;
            if (diff >= 2 && s[k] < second) second = s[k];
        }
        int curv = 0;
        if (d > 0 && d < D - 1) curv = s[d - 1] - 2 * s[d] + s[d + 1];
        int r = rho[i] < 32 ? rho[i] : 32;
        out[(size_t)i * 6 + 0] = (float)s[d] * sS;
        out[(size_t)i * 6 + 1] = (float)second * sS;
        out[(size_t)i * 6 + 2] = (float)curv * sS;
        out[(size_t)i * 6 + 3] = (float)d * sD;
        out[(size_t)i * 6 + 4] = (float)r * sR;
    }
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int q = x - dstar[y * W + x];
            int m = 1 << 20;                 /* no pixel to the right */
            for (int x2 = x + 1; x2 < W; ++x2) {
                const int q2 = x2 - dstar[y * W + x2];
                if (q2 < m) m = q2;
            }
            int v = q - m;
            if (v < -16) v = -16;
            if (v > 16) v = 16;
            if (q < 0) v = 16;
            out[((size_t)y * W + x) * 6 + 5] = (float)v * (1.0f / 16.0f);
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole pipeline for one frame (Fig. 1 flow): semidensification (SDSGM     */
/* only), joint cost, path aggregation, WTA + subpixel on the left view,    */
/* the same SGM with the right image as base and no prior, and the check.   */
/* Optional taps (any may be NULL): census codes, semidense map, the        */
/* aggregated left cost S, integer d*, right-view d', subpixel d_sub.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int W, H, D;
    int cw, ch;
    int num_paths;
    int p1, p2, q1, q2;
    int a, b;
    int blend_mode;
    int semidense;
    int ts, rs, tc, rc;
    int check_mode;
    int subpixel;
    int prior_cost;     /* 0 DDC, 1 quadratic, 2 Huber (orc_prior_penalty) */
    int huber_k;
    int census_kind;    /* 0 centre-symmetric, 1 full census (orc_census_kind) */
} orc_params;

int orc_run(const orc_params* P, const uint8_t* left, const uint8_t* right,
            int img_pitch, const int16_t* lidar, float* disp_out,
            uint8_t* valid_out, uint32_t* tap_census_l, uint32_t* tap_census_r,
            int16_t* tap_prior, int32_t* tap_S, int32_t* tap_dstar,
            int32_t* tap_dright, float* tap_dsub)
{
    int W = P->W, H = P->H, D = P->D;
    size_t px = (size_t)W * H, cells = px * (size_t)D;
    int n = P->census_kind == 1 ? P->cw * P->ch - 1 : orc_census_bits(P->cw, P->ch);
    int st = ORC_OK;
    uint32_t* cL = (uint32_t*)malloc(px * 4);
    uint32_t* cR = (uint32_t*)malloc(px * 4);
    int16_t* prior = (int16_t*)malloc(px * 2);
    int32_t* cost = (int32_t*)malloc(cells * 4);
    int32_t* S = (int32_t*)malloc(cells * 4);
    int32_t* dstar = (int32_t*)malloc(px * 4);
    int32_t* dright = (int32_t*)malloc(px * 4);
    float* dsub = (float*)malloc(px * 4);
    if (!cL || !cR || !prior || !cost || !S || !dstar || !dright || !dsub) {
        st = ORC_ENOMEM;
        goto done;
    }
    if ((st = orc_census_kind(left, W, H, img_pitch, P->cw, P->ch, P->census_kind, cL)))
        goto done;
    if ((st = orc_census_kind(right, W, H, img_pitch, P->cw, P->ch, P->census_kind, cR)))
        goto done;
    if (P->semidense)
        orc_semidense(cL, cR, lidar, W, H, n, P->ts, P->rs, prior);
    else
        memcpy(prior, lidar, px * 2);
    orc_joint_cost(cL, cR, prior, W, H, D, n, 0, P->a, P->b, P->q1, P->q2,
                   P->blend_mode, P->prior_cost, P->huber_k, cost);
    if ((st = orc_aggregate(cost, W, H, D, P->num_paths, P->b * P->p1,
                            P->b * P->p2, S)))
        goto done;
    orc_wta(S, W, H, D, P->subpixel, dstar, dsub);
    if (tap_S) memcpy(tap_S, S, cells * 4);
    if (P->check_mode == 1 || P->check_mode == 3) {
        orc_joint_cost(cL, cR, NULL, W, H, D, n, 1, P->a, P->b, P->q1, P->q2,
                       P->blend_mode, P->prior_cost, P->huber_k, cost);
        if ((st = orc_aggregate(cost, W, H, D, P->num_paths, P->b * P->p1,
                                P->b * P->p2, S)))
            goto done;
        orc_wta(S, W, H, D, 0, dright, NULL);
    } else {
        for (size_t i = 0; i < px; ++i) dright[i] = -1;
    }
    if ((st = orc_check(dstar, (P->check_mode & 1) ? dright : NULL, lidar, dsub,
                        W, H, P->tc, P->rc, P->check_mode, disp_out, valid_out)))
        goto done;
    if (tap_census_l) memcpy(tap_census_l, cL, px * 4);
    if (tap_census_r) memcpy(tap_census_r, cR, px * 4);
    if (tap_prior) memcpy(tap_prior, prior, px * 2);
    if (tap_dstar) memcpy(tap_dstar, dstar, px * 4);
    if (tap_dright) memcpy(tap_dright, dright, px * 4);
    if (tap_dsub) memcpy(tap_dsub, dsub, px * 4);
done:
    free(cL); free(cR); free(prior); free(cost); free(S);
    free(dstar); free(dright); free(dsub);
    return st;
}
