"""Seeded synthetic stereo + LiDAR frames: the input generator shared by the
tests, the benchmark and the smoke check.

This module holds none of the method's arithmetic.  It only draws scenes,
renders a rectified stereo pair with exact correspondences, and samples a
sparse LiDAR-like disparity map (float32, NaN = no return).  It stands in for
the paper's datasets (KITTI 141 with a 64-line LiDAR, its 32- and 16-line
subsamples, CARLA clear and rain scenes, Middlebury indoor scenes with a 1 %
sampled prior), none of which are used here.

Every frame is a pure function of ``(config_id, frame_idx)`` through
``numpy.random.default_rng([config_id, frame_idx])`` (PCG64).

Workloads:
  small   320x96, D=64: 3-6 fronto-parallel planes with integer disparities
          in [4, 60], i.i.d. uniform texels, 16 LiDAR rows at a 4 px pitch,
          thinned, noise sigma 0.5, 3 % outliers.
  kitti   1242x375, D=128: slanted planes (|b|,|c| <= 0.05) over a road-like
          background, random dots (+-48) over gradients, 20 % textureless
          patches, 64 LiDAR rows in the lower 2/3 covering ~5 % of pixels,
          noise sigma 0.3, 1 % misprojections next to occluding edges.
  robust  the kitti generator at 1242x375 or 640x480, D in {64, 128}, LiDAR
          density 0.5-10 % over 16-128 rows, optional degradation (noise
          sigma 8, contrast x0.5, rain-like streaks on 30 % of pixels), and an
          indoor variant 640x480, D=256, disparities in [40, 250], with a 1 %
          uniform sample of ground truth as the prior.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

CONFIG_IDS = {"small": 1, "kitti": 2, "robust": 3, "surrogate": 4, "serving": 5}


@dataclass(frozen=True)
class SceneSpec:
    W: int
    H: int
    D: int
    slanted: bool = True
    n_planes: tuple = (4, 8)          # inclusive range, background included
    disp_range: tuple = (0, 127)      # GT disparities are kept in this range
    integer_disp: bool = False        # fronto-parallel integer planes (small)
    textureless_frac: float = 0.2
    # LiDAR sampling
    lidar_kind: str = "lines"         # "lines", "lines_thin" or "uniform"
    lidar_lines: int = 64
    lidar_density: float = 0.05       # fraction of all pixels
    lidar_row0_frac: float = 1.0 / 3  # rows above this fraction are skipped
    lidar_sigma: float = 0.3
    lidar_outlier_frac: float = 0.0
    lidar_misproj_frac: float = 0.01
    lidar_pitch: float = 4.0          # lines_thin only
    lidar_keep: float = 0.3125        # lines_thin only
    degrade: str = "none"             # none | noise | contrast | rain


SMALL = SceneSpec(W=320, H=96, D=64, slanted=False, n_planes=(3, 6),
                  disp_range=(4, 60), integer_disp=True, textureless_frac=0.0,
                  lidar_kind="lines_thin", lidar_lines=16, lidar_row0_frac=0.0,
                  lidar_sigma=0.5, lidar_outlier_frac=0.03, lidar_misproj_frac=0.0)
KITTI = SceneSpec(W=1242, H=375, D=128)
INDOOR = SceneSpec(W=640, H=480, D=256, disp_range=(40, 250), lidar_kind="uniform",
                   lidar_density=0.01, lidar_sigma=0.0, lidar_misproj_frac=0.0)


def robust_spec(W=1242, H=375, D=128, density=0.05, lines=64, degrade="none"):
    """One cell of the robustness sweep (resolution x D x density x degradation)."""
    return replace(KITTI, W=W, H=H, D=D, disp_range=(0, D - 1), lidar_density=density,
                   lidar_lines=lines, degrade=degrade)


# Serving mix: six rigs, two per frame type, LiDAR density per rig.
SERVING_RIGS = [
    dict(rig=0, W=640, H=480, D=64, density=0.02),
    dict(rig=1, W=640, H=480, D=64, density=0.03),
    dict(rig=2, W=1242, H=375, D=128, density=0.04),
    dict(rig=3, W=1242, H=375, D=128, density=0.05),
    dict(rig=4, W=1920, H=1080, D=256, density=0.025),
    dict(rig=5, W=1920, H=1080, D=256, density=0.035),
]


def serving_spec(rig: int) -> SceneSpec:
    r = SERVING_RIGS[rig]
    return robust_spec(W=r["W"], H=r["H"], D=r["D"], density=r["density"],
                       lines=64 if r["H"] < 1000 else 128)


@dataclass
class _Plane:
    a: float
    b: float
    c: float
    region: np.ndarray       # bool [H, W] in left-image coordinates (None = all)
    tex: np.ndarray          # uint8 [H, TW] indexed by left-image x
    ellipse: tuple = None
    rect: tuple = None


def _region_mask(rng, W, H, shape_kind):
    cx, cy = rng.uniform(0.05 * W, 0.95 * W), rng.uniform(0.1 * H, 0.95 * H)
    hw, hh = rng.uniform(0.05 * W, 0.22 * W), rng.uniform(0.12 * H, 0.4 * H)
    yy, xx = np.mgrid[0:H, 0:W]
    if shape_kind == 0:
        m = (np.abs(xx - cx) <= hw) & (np.abs(yy - cy) <= hh)
    else:
        m = ((xx - cx) / hw) ** 2 + ((yy - cy) / hh) ** 2 <= 1.0
    return m


def _texture(rng, H, TW, spec: SceneSpec):
    if spec.integer_disp:
        return rng.integers(0, 256, size=(H, TW), dtype=np.int32).astype(np.uint8)
    base = rng.uniform(70, 180)
    gu, gy = rng.uniform(-0.04, 0.04), rng.uniform(-0.15, 0.15)
    yy, uu = np.mgrid[0:H, 0:TW]
    t = base + gu * uu + gy * (yy - H / 2)
    t = t + rng.integers(-48, 49, size=(H, TW))
    # textureless patches: constant-intensity rectangles attached to the plane
    if spec.textureless_frac > 0:
        covered = np.zeros((H, TW), bool)
        target = spec.textureless_frac * H * TW
        while covered.sum() < target:
            w, h = rng.integers(20, 81, size=2)
            x0, y0 = rng.integers(0, TW - 1), rng.integers(0, H - 1)
            t[y0:y0 + h, x0:x0 + w] = rng.uniform(40, 220)
            covered[y0:y0 + h, x0:x0 + w] = True
    return np.clip(np.rint(t), 0, 255).astype(np.uint8)


def _draw_planes(rng, spec: SceneSpec):
    W, H = spec.W, spec.H
    lo, hi = spec.disp_range
    TW = W + hi + 8
    n = int(rng.integers(spec.n_planes[0], spec.n_planes[1] + 1))
    planes = []
    if spec.integer_disp:
        ds = np.sort(rng.choice(np.arange(lo, hi + 1), size=n, replace=False))
        for k, d in enumerate(ds):
            region = None if k == 0 else _region_mask(rng, W, H, int(rng.integers(0, 2)))
            planes.append(_Plane(float(d), 0.0, 0.0, region, _texture(rng, H, TW, spec)))
        return planes
    # background: road-like slant, disparity rising towards the bottom rows
    span = hi - lo
    c_bg = rng.uniform(0.45, 0.6) * span / H
    b_bg = rng.uniform(-0.01, 0.01)
    a_bg = lo + rng.uniform(0.0, 0.05) * span + max(0.0, -b_bg * W)
    planes.append(_Plane(a_bg, b_bg, c_bg, None, _texture(rng, H, TW, spec)))
    for _ in range(n - 1):
        region = _region_mask(rng, W, H, int(rng.integers(0, 2)))
        b, c = rng.uniform(-0.05, 0.05, size=2)
        yy, xx = np.nonzero(region)
        # plane sits in front of the background over its region
        dmid = rng.uniform(lo + 0.35 * span, hi - 0.05 * span)
        a = dmid - b * xx.mean() - c * yy.mean()
        dv = a + b * xx + c * yy
        shift = 0.0
        if dv.max() > hi:
            shift = dv.max() - hi
        if dv.min() - shift < lo:
            shift = dv.min() - lo
        a -= shift
        planes.append(_Plane(a, b, c, region, _texture(rng, H, TW, spec)))
    return planes


def _render(planes, spec: SceneSpec):
    """Left view, right view, GT disparity of the left view and its occlusion
    mask, with exact correspondences: left pixel x shows plane texture at x,
    right pixel x_r shows the front-most plane whose left coordinate
    x_l = x_r + d(x_l, y) falls in its region."""
    W, H = spec.W, spec.H
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    best_d = np.full((H, W), -np.inf)
    best_k = np.zeros((H, W), np.int32)
    for k, p in enumerate(planes):
        d = p.a + p.b * xx + p.c * yy
        m = np.ones((H, W), bool) if p.region is None else p.region
        upd = m & (d > best_d)
        best_d[upd] = d[upd]
        best_k[upd] = k
    left = np.zeros((H, W), np.uint8)
    rows = np.arange(H)[:, None].repeat(W, 1)
    for k, p in enumerate(planes):
        m = best_k == k
        left[m] = p.tex[rows[m], xx.astype(np.int64)[m]]
    # right view
    rbest_d = np.full((H, W), -np.inf)
    rbest_k = np.full((H, W), -1, np.int32)
    rbest_xl = np.zeros((H, W))
    for k, p in enumerate(planes):
        xl = (xx + p.a + p.c * yy) / (1.0 - p.b)
        d = xl - xx
        if p.region is None:
            m = np.ones((H, W), bool)
        else:
            xi = np.rint(xl).astype(np.int64)
            inside = (xi >= 0) & (xi < W)
            m = np.zeros((H, W), bool)
            m[inside] = p.region[rows[inside], xi[inside]]
        upd = m & (d > rbest_d)
        rbest_d[upd] = d[upd]
        rbest_k[upd] = k
        rbest_xl[upd] = xl[upd]
    right = np.zeros((H, W), np.uint8)
    for k, p in enumerate(planes):
        m = rbest_k == k
        if not m.any():
            continue
        xl = rbest_xl[m]
        r = rows[m]
        if spec.integer_disp:
            right[m] = p.tex[r, np.rint(xl).astype(np.int64)]
        else:
            x0 = np.floor(xl).astype(np.int64)
            f = xl - x0
            t0 = p.tex[r, x0].astype(np.float64)
            t1 = p.tex[r, np.minimum(x0 + 1, p.tex.shape[1] - 1)].astype(np.float64)
            right[m] = np.clip(np.rint((1 - f) * t0 + f * t1), 0, 255).astype(np.uint8)
    gt = best_d.astype(np.float32)
    xr = np.rint(xx - best_d).astype(np.int64)
    occ = (xr < 0) | (xr >= W)
    ok = ~occ
    occ[ok] = rbest_k[rows[ok], xr[ok]] != best_k[ok]
    return left, right, gt, occ


def _lidar(rng, spec: SceneSpec, gt):
    W, H = spec.W, spec.H
    lid = np.full((H, W), np.nan, np.float32)
    if spec.lidar_kind == "uniform":
        n = int(round(spec.lidar_density * W * H))
        idx = rng.choice(W * H, size=n, replace=False)
        ys, xs = np.unravel_index(idx, (H, W))
    elif spec.lidar_kind == "lines_thin":
        rows = np.rint(np.linspace(0, H - 1, spec.lidar_lines + 2)[1:-1]).astype(np.int64)
        ys_l, xs_l = [], []
        for r in rows:
            phase = rng.integers(0, int(spec.lidar_pitch))
            xs_r = np.arange(phase, W, spec.lidar_pitch).astype(np.int64)
            keep = rng.random(xs_r.size) < spec.lidar_keep
            xs_l.append(xs_r[keep])
            ys_l.append(np.full(keep.sum(), r))
        ys, xs = np.concatenate(ys_l), np.concatenate(xs_l)
    else:
        row0 = int(np.ceil(spec.lidar_row0_frac * H))
        rows = np.unique(np.rint(np.linspace(row0, H - 1, spec.lidar_lines)).astype(np.int64))
        per_line = spec.lidar_density * W * H / len(rows)
        pitch = max(W / per_line, 1.0)
        ys_l, xs_l = [], []
        for r in rows:
            phase = rng.uniform(0, pitch)
            xs_r = np.unique(np.floor(np.arange(phase, W, pitch)).astype(np.int64))
            xs_l.append(xs_r)
            ys_l.append(np.full(xs_r.size, r))
        ys, xs = np.concatenate(ys_l), np.concatenate(xs_l)
    vals = gt[ys, xs].astype(np.float64)
    if spec.lidar_sigma > 0:
        vals = vals + rng.normal(0.0, spec.lidar_sigma, size=vals.size)
    if spec.lidar_outlier_frac > 0:
        out = rng.random(vals.size) < spec.lidar_outlier_frac
        vals[out] = rng.uniform(0, spec.D - 1, size=int(out.sum()))
    if spec.lidar_misproj_frac > 0:
        # foreground points 1-6 px from an occluding edge (GT jump > 2) take
        # the background disparity behind that edge
        cand, bgv = [], []
        for i, (y, x) in enumerate(zip(ys, xs)):
            for k in range(1, 7):
                hit = False
                for xn in (x + k, x - k):
                    if 0 <= xn < W and gt[y, xn] < gt[y, x] - 2:
                        cand.append(i)
                        bgv.append(gt[y, xn])
                        hit = True
                        break
                if hit:
                    break
        n_mis = int(round(spec.lidar_misproj_frac * vals.size))
        if cand and n_mis > 0:
            pick = rng.choice(len(cand), size=min(n_mis, len(cand)), replace=False)
            for j in pick:
                vals[cand[j]] = bgv[j] + rng.normal(0.0, spec.lidar_sigma)
    lid[ys, xs] = vals.astype(np.float32)
    return lid


def _degrade(rng, img, kind):
    if kind == "none":
        return img
    if kind == "noise":
        return np.clip(np.rint(img + rng.normal(0, 8, img.shape)), 0, 255).astype(np.uint8)
    if kind == "contrast":
        return np.clip(np.rint(128 + 0.5 * (img.astype(np.float64) - 128)), 0, 255).astype(np.uint8)
    if kind == "rain":
        H, W = img.shape
        out = img.astype(np.int32)
        mask = np.zeros((H, W), bool)
        target = 0.3 * H * W
        while mask.sum() < target:
            n = 2000
            x0 = rng.uniform(0, W, n)
            y0 = rng.uniform(0, H, n)
            ln = rng.integers(8, 33, n)
            ang = np.deg2rad(rng.uniform(-10, 10, n))
            br = rng.integers(50, 101, n)
            for i in range(n):
                t = np.arange(ln[i])
                xs = np.rint(x0[i] + t * np.sin(ang[i])).astype(np.int64)
                ys = np.rint(y0[i] + t * np.cos(ang[i])).astype(np.int64)
                ok = (xs >= 0) & (xs < W) & (ys >= 0) & (ys < H)
                xs, ys = xs[ok], ys[ok]
                fresh = ~mask[ys, xs]
                out[ys[fresh], xs[fresh]] += br[i]
                mask[ys, xs] = True
                if mask.sum() >= target:
                    break
        return np.clip(out, 0, 255).astype(np.uint8)
    raise ValueError(kind)


def make_frame(spec: SceneSpec, config_id: int, frame_idx: int) -> dict:
    """One frame: left/right uint8 [H, W], lidar float32 [H, W] (NaN = no
    return), gt float32 [H, W], occ bool [H, W]."""
    rng = np.random.default_rng([config_id, frame_idx])
    planes = _draw_planes(rng, spec)
    left, right, gt, occ = _render(planes, spec)
    if spec.lidar_kind == "uniform":
        # indoor protocol: a uniform random sample of ground truth
        lid = _lidar(rng, spec, gt)
    else:
        lid = _lidar(rng, spec, gt)
    if spec.degrade != "none":
        left = _degrade(rng, left, spec.degrade)
        right = _degrade(rng, right, spec.degrade)
    return dict(left=left, right=right, lidar=lid, gt=gt, occ=occ,
                W=spec.W, H=spec.H, D=spec.D)


def small_frame(idx: int = 0) -> dict:
    return make_frame(SMALL, CONFIG_IDS["small"], idx)


def kitti_frame(idx: int = 0) -> dict:
    return make_frame(KITTI, CONFIG_IDS["kitti"], idx)


def fronto_single_plane(W, H, d0, seed=0):
    """Random-dot pair of one fronto-parallel plane at integer disparity d0
    (right pixel x shows the left texel at x + d0)."""
    rng = np.random.default_rng([97, seed])
    tex = rng.integers(0, 256, size=(H, W + d0), dtype=np.int32).astype(np.uint8)
    left = tex[:, :W].copy()
    right = tex[:, d0:d0 + W].copy()
    return left, right
