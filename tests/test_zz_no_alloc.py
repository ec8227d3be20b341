"""sldf_run_noalloc (the entry point for callers that cannot allocate)
against sldf_run on the same frames, through the C ABI: two calls in a row,
the second on a smaller frame, each bit for bit equal to the context run."""
import numpy as np
import pytest
import torch

from paper_2504_05148_amd import sldf, synth

pytestmark = pytest.mark.gpu


def _inputs(f):
    D = int(f["D"])
    return (sldf.device_image(f["left"]), sldf.device_image(f["right"]),
            sldf.quantize_lidar(torch.from_numpy(np.ascontiguousarray(f["lidar"])).cuda(), D))


def test_noalloc_equals_run_two_calls_second_smaller():
    cases = [
        (synth.make_frame(synth.robust_spec(W=640, H=480, D=64, density=0.03), 3, 640064),
         dict(width=640, height=480, max_disp=64)),
        (synth.small_frame(3), dict(width=320, height=96, max_disp=64, census_w=5,
                                    census_h=5, num_paths=4)),
    ]
    for f, kw in cases:
        print(f"case noalloc {kw}", flush=True)
        p = sldf.default_params(**kw)
        L, R, lq = _inputs(f)
        d0, v0 = sldf.Context(p).run(L, R, lq)
        d1 = torch.full_like(d0, 7.0)
        v1 = torch.full_like(v0, 7)
        sldf.run_noalloc(p, L, R, lq, d1, v1)
        torch.cuda.synchronize()
        assert torch.equal(v1, v0), kw
        assert torch.equal(d1, d0), kw


def test_noalloc_rejects_what_does_not_fit_and_the_learned_check():
    p = sldf.default_params()                 # 1242 x 375, D = 128: beyond the scratch
    H, W = 375, 1242
    img = torch.zeros((H, 1248), dtype=torch.uint8, device="cuda")[:, :W]
    lid = torch.full((H, W), -1, dtype=torch.int16, device="cuda")
    d = torch.empty((H, W), dtype=torch.float32, device="cuda")
    v = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    with pytest.raises(sldf.SldfError) as ei:
        sldf.run_noalloc(p, img, img, lid, d, v)
    assert ei.value.status == sldf.ENOMEM
    p = sldf.default_params(width=320, height=96, max_disp=64, check_impl=1)
    with pytest.raises(sldf.SldfError) as ei:
        sldf.run_noalloc(p, img[:96, :320], img[:96, :320], lid[:96, :320], d[:96, :320],
                         v[:96, :320])
    assert ei.value.status == sldf.EINVAL
