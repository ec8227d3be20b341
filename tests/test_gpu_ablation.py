"""Ablation runner (check modes, prior maps, variants) on paper-scale
synthetic frames through the C ABI: relations the definitions fix exactly."""
import numpy as np
import pytest

from paper_2504_05148_amd import ablation, evaluate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frames():
    return ablation._frames(2, first=7000)


def test_check_modes_are_the_or_of_the_two_tests(frames):
    print("case ablation check modes, 2 frames 1242x375", flush=True)
    res = {m: ablation.run_frames(frames, check_mode=m) for m in (0, 1, 2, 3)}
    for i in range(len(frames)):
        v = {m: res[m][i][1].astype(bool) for m in res}
        d = {m: res[m][i][0] for m in res}
        assert v[0].all()
        # Eq. 6: stereo-LiDAR = stereo OR camera-LiDAR, on the same d*
        assert (v[3] == (v[1] | v[2])).all()
        for m in (1, 2, 3):
            assert (d[m][v[m]] == d[0][v[m]]).all() and (d[m][~v[m]] == -1.0).all()
    e = {m: evaluate.evaluate_frames(res[m], frames) for m in res}
    assert e[0]["coverage"] == 1.0
    assert e[3]["coverage"] >= max(e[1]["coverage"], e[2]["coverage"])


def test_semidense_prior_keeps_every_sparse_point(frames):
    _, priors = ablation.run_frames(frames, taps_prior=True, semidense=1)
    for sparse, semi in priors:
        assert ((sparse >= 0) <= (semi >= 0)).all()
    rows = ablation.prior_maps(frames)
    assert rows["semidense map"]["coverage"] >= rows["input sparse map"]["coverage"]


def test_variants_and_table(frames):
    rows = ablation.variants(frames, ablation._load_surrogate())
    assert set(ablation.VARIANTS) <= set(rows)
    for e in rows.values():
        assert 0.0 <= e["covered_error"] <= 1.0 and 0.0 < e["coverage"] <= 1.0
    t = ablation.table("variants", rows)
    assert t.count("\n") == len(rows) + 3


def test_prior_terms_rows(frames):
    rows = ablation.prior_terms(frames[:1])
    assert len(rows) == 2 * len(ablation.PRIOR_TERMS)
    for e in rows.values():
        assert 0.0 < e["coverage"] <= 1.0


def test_robustness_and_density_rows():
    rows = ablation.robustness(1, degradations=("rain",))
    assert len(rows) == len(ablation.ROBUST_METHODS)
    rows = ablation.density_sweep(1, densities=((0.02, 32),))
    assert len(rows) == 2
    for e in rows.values():
        assert 0.0 < e["coverage"] <= 1.0
