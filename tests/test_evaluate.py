"""Evaluation layer (coverage, covered / total error, background fill) on
hand-made maps whose metrics follow from the definitions by counting."""
import numpy as np

from paper_2504_05148_amd import evaluate as ev


def test_background_fill_takes_the_farther_neighbour_and_extends_borders():
    d = np.array([[0, 10, 0, 0, 4, 0]], np.float32)
    v = np.array([[0, 1, 0, 0, 1, 0]], bool)
    f = ev.background_fill(d, v)
    # left border <- 10, gap between 10 and 4 <- min = 4, right border <- 4
    assert f.tolist() == [[10, 10, 4, 4, 4, 4]]


def test_background_fill_rows_without_estimates_copy_the_nearest_row():
    d = np.array([[5, 5], [0, 0], [0, 0], [0, 0], [7, 7]], np.float32)
    v = np.array([[1, 1], [0, 0], [0, 0], [0, 0], [1, 1]], bool)
    f = ev.background_fill(d, v)
    assert f[:, 0].tolist() == [5, 5, 5, 7, 7]   # row 2 is equidistant: the row above


def test_background_fill_of_an_empty_map_is_zero():
    f = ev.background_fill(np.full((3, 4), 9, np.float32), np.zeros((3, 4), bool))
    assert (f == 0).all()


def test_valid_pixels_are_kept_exactly():
    rng = np.random.default_rng(0)
    d = rng.uniform(0, 60, (20, 30)).astype(np.float32)
    v = rng.random((20, 30)) < 0.3
    f = ev.background_fill(d, v)
    assert (f[v] == d[v]).all() and np.isfinite(f).all()


def test_metrics_by_counting():
    gt = np.full((2, 5), 10.0, np.float32)
    disp = np.array([[10, 12.9, 13, 0, 0], [7, 10.5, 0, 0, 10]], np.float32)
    valid = np.array([[1, 1, 1, 0, 0], [1, 1, 0, 0, 1]], bool)
    e = ev.evaluate(disp, valid, gt)
    assert e["pixels"] == 10
    assert e["coverage"] == 0.6
    # covered: |13 - 10| = 3 and |7 - 10| = 3 count (three pixels or more)
    assert abs(e["covered_error"] - 2 / 6) < 1e-12
    # fill row 0: [10, 12.9, 13, 13, 13] -> errors at 13, 13, 13
    # fill row 1: [7, 10.5, 10, 10, 10]  -> error at 7
    assert abs(e["total_error"] - 4 / 10) < 1e-12


def test_gt_mask_and_nonfinite_gt_are_excluded():
    gt = np.array([[10, np.nan, 10]], np.float32)
    disp = np.array([[30, 30, 10]], np.float32)
    valid = np.ones((1, 3), bool)
    e = ev.evaluate(disp, valid, gt, gt_mask=np.array([[0, 1, 1]], bool))
    assert e["pixels"] == 1 and e["covered_error"] == 0.0 and e["total_error"] == 0.0


def test_perfect_map_and_empty_map():
    gt = np.arange(12, dtype=np.float32).reshape(3, 4)
    e = ev.evaluate(gt, np.ones_like(gt, bool), gt)
    assert e == dict(pixels=12, coverage=1.0, covered_error=0.0, total_error=0.0)
    e = ev.evaluate(gt, np.zeros_like(gt, bool), gt + 100)
    assert e["coverage"] == 0.0 and e["covered_error"] == 0.0 and e["total_error"] == 1.0


def test_pooled_frames_equal_the_concatenated_map():
    rng = np.random.default_rng(1)
    frames, res = [], []
    for i in range(3):
        gt = rng.uniform(0, 50, (8, 9)).astype(np.float32)
        occ = rng.random((8, 9)) < 0.1
        d = gt + rng.normal(0, 3, gt.shape).astype(np.float32)
        v = rng.random(gt.shape) < 0.7
        frames.append(dict(gt=gt, occ=occ))
        res.append((d, v))
    pooled = ev.evaluate_frames(res, frames)
    n = sum(ev.counts(d, v, f["gt"], ~f["occ"])[0] for (d, v), f in zip(res, frames))
    assert pooled["pixels"] == n and pooled["frames"] == 3
    tot = [sum(ev.counts(d, v, f["gt"], ~f["occ"])[k] for (d, v), f in zip(res, frames))
           for k in range(4)]
    assert abs(pooled["total_error"] - tot[3] / tot[0]) < 1e-12
    assert abs(pooled["covered_error"] - tot[2] / tot[1]) < 1e-12
