"""Serving loop on the GPU: the six-rig mix (640x480 D=64, 1242x375 D=128,
1920x1080 D=256) under Poisson load; every result equals the same frame run
alone on an idle GPU, bit for bit, and one served result per frame shape
equals the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_05148_amd import serving, sldf, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pools():
    return serving.make_pools(6, 2, workers=8)


def _alone(pools, rig, frame, check_impl=0, surrogate=None):
    r = synth.SERVING_RIGS[rig]
    p = sldf.default_params(width=r["W"], height=r["H"], max_disp=r["D"], check_impl=check_impl)
    ctx = sldf.Context(p)
    if check_impl:
        ctx.set_surrogate(*surrogate)
    L = sldf.device_image(pools[rig]["left"][frame].numpy())
    R = sldf.device_image(pools[rig]["right"][frame].numpy())
    lq = sldf.quantize_lidar(pools[rig]["lidar"][frame].cuda(), r["D"])
    d, v = ctx.run(L, R, lq)
    torch.cuda.synchronize()
    return d.cpu(), v.cpu()


_SERVED = {}


def _serve(pools, check_impl):
    # one mixed serving run per form, shared by the tests of this module
    if check_impl not in _SERVED:
        sur = None
        if check_impl:
            from paper_2504_05148_amd.train_surrogate import load_weights
            sur = load_weights()[:2]
        print(f"case serving mix check_impl={check_impl}", flush=True)
        _SERVED[check_impl] = sur, serving.run_serving(
            duration=1.5, pool_size=2, max_batch=4, hbm_budget=64 << 30,
            check_impl=check_impl, surrogate=sur, pools=pools, keep_outputs=True)
    return _SERVED[check_impl]


@pytest.mark.parametrize("check_impl", [0, 1])
def test_mix_equals_alone(pools, check_impl):
    sur, (summ, be, fin) = _serve(pools, check_impl)
    assert summ["failed"] == 0 and summ["completed"] == summ["requests"] > 300
    assert summ["peak_slot_bytes"] <= summ["budget_bytes"]
    assert summ["p99_ms"] is not None and summ["p99_ms"] >= summ["p50_ms"] > 0
    checked = 0
    for (rig, frame), outs in be.outputs.items():
        d0, v0 = _alone(pools, rig, frame, check_impl, sur)
        for d, v in outs:
            assert torch.equal(v, v0), (rig, frame)
            assert torch.equal(d, d0), (rig, frame)
            checked += 1
    assert checked == summ["completed"]


def test_small_budget_queues_but_completes(pools):
    # budget for about one slot per rig: requests wait for slots, none fail
    be_probe = serving.SldfBackend([dict(W=r["W"], H=r["H"], D=r["D"])
                                    for r in synth.SERVING_RIGS], pools, 2)
    budget = sum(be_probe.slot_bytes(r) for r in range(6)) + (1 << 20)
    summ, _, _ = serving.run_serving(duration=1.0, pool_size=2, max_batch=2, hbm_budget=budget,
                                     pools=pools)
    assert summ["failed"] == 0 and summ["completed"] == summ["requests"]
    assert all(v == 1 for v in summ["slots"].values())


@pytest.mark.parametrize("rig", [0, 2, 4])
def test_served_result_equals_oracle(pools, rig):
    """One result served in the mix per frame shape (640x480 D=64, 1242x375
    D=128, 1920x1080 D=256) against the CPU oracle: mask bit for bit, the
    disparity within 1e-4 px."""
    _, (summ, be, fin) = _serve(pools, 0)
    served = sorted(k for k in be.outputs if k[0] == rig)
    assert served, f"rig {rig} served nothing"
    frame = served[0][1]
    d, v = be.outputs[served[0]][0]
    r = synth.SERVING_RIGS[rig]
    print(f"case served rig {rig} frame {frame} vs oracle", flush=True)
    op = oracle.OracleParams(W=r["W"], H=r["H"], D=r["D"])
    lid = oracle.quantize_lidar(pools[rig]["lidar"][frame].numpy(), r["D"])
    od, ov = oracle.run(op, pools[rig]["left"][frame].numpy(),
                        pools[rig]["right"][frame].numpy(), lid)
    assert (v.numpy() == ov).all(), np.argwhere(v.numpy() != ov)[:5]
    assert np.abs(d.numpy() - od).max() <= 1e-4
