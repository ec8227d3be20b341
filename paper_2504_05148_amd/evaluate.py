"""Accuracy of a disparity map against ground truth, in the form the paper
reports it (Sec. V, the KITTI-style evaluation): coverage, covered error and
total error at a 3-pixel threshold.

- coverage: fraction of the evaluated pixels (ground truth present) that
  carry a valid estimate;
- covered error: among evaluated pixels with a valid estimate, the fraction
  whose estimate differs from the ground truth by the threshold or more;
- total error: the same fraction over all evaluated pixels, after the
  invalid estimates are filled by background interpolation.

Background interpolation (the left-right-check fill of Hirschmueller's SGM
paper, which the evaluation cites): along each row, a run of invalid pixels
between two valid ones takes the smaller (farther) of the two disparities; a
run touching the left or right image border takes the value of its single
valid neighbour.  Rows without any valid pixel are then filled column-wise
from the nearest row above or below that has one.  A map without any valid
pixel fills with 0.

Readings: an estimate counts as an error when it is three pixels or more
off the ground truth, so |d - gt| >= 3 is an error (inclusive); ground truth
is present where it is finite and not occluded in the left view.

Host-side numpy; used by the ablation runner and the benchmark's accuracy
line on the synthetic frames.
"""
from __future__ import annotations

import numpy as np

THRESHOLD = 3.0


def background_fill(disp: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """Fill invalid pixels of `disp` (float [H, W]) by background
    interpolation; `valid` is a bool or 0/1 mask of the same shape."""
    d = np.asarray(disp, np.float32)
    v = np.asarray(valid).astype(bool)
    H, W = d.shape
    out = np.where(v, d, np.nan).astype(np.float32)
    cols = np.arange(W)
    row_has = v.any(axis=1)
    for y in np.nonzero(row_has)[0]:
        vx = cols[v[y]]
        vd = d[y, vx]
        # index of the nearest valid pixel to the left / right of every x
        k = np.searchsorted(vx, cols, side="right") - 1        # last valid <= x
        left = np.where(k >= 0, vd[np.clip(k, 0, None)], np.nan)
        kr = np.searchsorted(vx, cols, side="left")             # first valid >= x
        right = np.where(kr < vx.size, vd[np.clip(kr, None, vx.size - 1)], np.nan)
        fill = np.fmin(left, right)                             # one side missing -> other
        out[y] = np.where(v[y], d[y], fill)
    if not row_has.all():
        if not row_has.any():
            return np.zeros_like(d)
        rows = np.nonzero(row_has)[0]
        ys = np.arange(H)
        k = np.searchsorted(rows, ys, side="right") - 1
        above = np.where(k >= 0, rows[np.clip(k, 0, None)], -1)
        kr = np.searchsorted(rows, ys, side="left")
        below = np.where(kr < rows.size, rows[np.clip(kr, None, rows.size - 1)], -1)
        for y in np.nonzero(~row_has)[0]:
            # nearest filled row; ties go to the row above
            a, b = above[y], below[y]
            src = a if b < 0 or (a >= 0 and y - a <= b - y) else b
            out[y] = out[src]
    return out


def counts(disp: np.ndarray, valid: np.ndarray, gt: np.ndarray,
           gt_mask: np.ndarray | None = None, threshold: float = THRESHOLD):
    """(evaluated pixels, covered pixels, covered errors, total errors) of
    one map; `gt_mask` selects the evaluated pixels (default: finite gt)."""
    d = np.asarray(disp, np.float32)
    v = np.asarray(valid).astype(bool)
    g = np.asarray(gt, np.float32)
    fin = np.isfinite(g)
    m = fin if gt_mask is None else (np.asarray(gt_mask).astype(bool) & fin)
    cov = m & v
    bad_cov = int((np.abs(d[cov] - g[cov]) >= threshold).sum())
    filled = background_fill(d, v)
    bad_tot = int((np.abs(filled[m] - g[m]) >= threshold).sum())
    return int(m.sum()), int(cov.sum()), bad_cov, bad_tot


def _fractions(n, ncov, bad_cov, bad_tot):
    return dict(pixels=n, coverage=ncov / n if n else 0.0,
                covered_error=bad_cov / ncov if ncov else 0.0,
                total_error=bad_tot / n if n else 0.0)


def evaluate(disp: np.ndarray, valid: np.ndarray, gt: np.ndarray,
             gt_mask: np.ndarray | None = None, threshold: float = THRESHOLD) -> dict:
    """Coverage, covered error and total error (fractions in [0, 1]) of one
    map."""
    return _fractions(*counts(disp, valid, gt, gt_mask, threshold))


def evaluate_frames(results, frames, threshold: float = THRESHOLD) -> dict:
    """Pooled coverage / errors of several (disp, valid) results against
    synthetic frames (dicts with `gt` and `occ`; the evaluated pixels are the
    non-occluded ones)."""
    tot = np.zeros(4, np.int64)
    for (disp, valid), f in zip(results, frames):
        m = ~np.asarray(f["occ"]).astype(bool)
        tot += np.array(counts(disp, valid, f["gt"], m, threshold))
    out = _fractions(*(int(t) for t in tot))
    out["frames"] = len(frames)
    return out
