"""Learned consistency surrogate on the GPU (MFMA kernels through the C ABI):
forward and backward against a plain PyTorch fp32 CPU reference of the same
network, the learned sldf_run against its definition, and the fallback to
the plain check."""
import numpy as np
import pytest
import torch

import oracle
from oracle import surrogate_ref as ref
from paper_2504_05148_amd import sldf, synth

pytestmark = pytest.mark.gpu


def _features(f, pkw):
    """Run the plain path with the features / rho taps; return device tensors."""
    p = sldf.default_params(**pkw)
    W, H, D = p.width, p.height, p.max_disp
    ctx = sldf.Context(p)
    left, right = sldf.device_image(f["left"]), sldf.device_image(f["right"])
    lid = sldf.quantize_lidar(torch.from_numpy(f["lidar"]).cuda(), D)
    feats = torch.empty((H, W, 8), dtype=torch.int16, device="cuda")
    rho = torch.empty((H, W), dtype=torch.int16, device="cuda")
    ctx.set_taps(features=feats, rho=rho)
    disp, valid = ctx.run(left, right, lid)
    torch.cuda.synchronize()
    return dict(x0=feats, rho=rho, disp=disp, valid=valid, left=left, right=right, lid=lid,
                params=p)


def _params_bits(seed=0, bias_scale=0.1):
    master = ref.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    master[ref.N_W:] = rng.normal(0, bias_scale, ref.N_B).astype(np.float32)
    wbits = ref.f32_to_bf16_bits(master[:ref.N_W])
    return master, wbits, master[ref.N_W:].copy()


def _random_x0(F, H, W, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((F, H, W, 8), np.float32)
    x[..., :5] = rng.uniform(0, 1, size=(F, H, W, 5))
    return ref.f32_to_bf16_bits(x)


# sizes: ragged row blocks and column tiles of every dilation; H = 200 gives
# seven row blocks per lattice at dilation 1; 16 x 16 (the smallest frame) is
# narrower than a tile and shorter than the largest dilation
@pytest.mark.parametrize("F,H,W", [(1, 37, 70), (2, 64, 129), (1, 200, 300), (1, 16, 16),
                                   (3, 16, 17)])
def test_forward_matches_reference(F, H, W):
    """Activations within one bf16 rounding step, logits within a tolerance
    derived from fp32 accumulation of bf16 products."""
    _, wbits, b = _params_bits(1)
    x0 = _random_x0(F, H, W, 3)
    z, acts = sldf.surrogate_forward(torch.from_numpy(x0.view(np.int16)).cuda(),
                                     torch.from_numpy(wbits.view(np.int16)).cuda(),
                                     torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    zr, ar, _ = ref.forward(x0, wbits, b)
    zr = zr.numpy()
    for l in range(3):
        g = ref.bf16_bits_to_f32(acts[l].cpu().numpy().view(np.uint16))
        r = ar[l].permute(0, 2, 3, 1).numpy()
        # rounding boundaries may differ by one bf16 step (2^-8 relative)
        assert np.abs(g - r).max() <= 2 ** -7 * max(1.0, np.abs(r).max()), l
        assert (np.abs(g - r) <= 2 ** -7 * np.maximum(np.abs(r), 1e-2)).mean() > 0.999, l
    zg = z.cpu().numpy()
    scale = np.abs(zr).max()
    assert np.abs(zg - zr).max() <= 2e-2 * scale
    assert np.abs(zg - zr).mean() <= 1e-3 * scale


def test_backward_matches_reference():
    """Gradients of the masked BCE loss against autograd on the CPU."""
    F, H, W = 2, 48, 96
    master, wbits, b = _params_bits(2)
    x0 = _random_x0(F, H, W, 5)
    rng = np.random.default_rng(6)
    labels = (rng.random((F, H, W)) < 0.8).astype(np.uint8)
    rho = rng.integers(0, 6, size=(F, H, W)).astype(np.uint16)
    tc = 2
    trainer = sldf.SurrogateTrainer(W, H, F, torch.from_numpy(master))
    g = torch.zeros(ref.N_W + ref.N_B, dtype=torch.float32, device="cuda")
    trainer.step(torch.from_numpy(x0.view(np.int16)).cuda(), torch.from_numpy(labels).cuda(),
                 torch.from_numpy(rho.view(np.int16)).cuda(), tc, update=False, grads_out=g)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    # reference loss: mean over all pixels of the masked BCE
    z, _, params = ref.forward(x0, wbits, b, straight_through=True)
    m = torch.from_numpy((rho > tc).astype(np.float32))
    y = torch.from_numpy(labels.astype(np.float32))
    loss = (m * (torch.nn.functional.softplus(z) - y * z)).sum() / (F * H * W)
    loss.backward()
    off, boff = 0, 0
    for li, ((oc, ic, _), cout) in enumerate(zip(ref.LAYERS, ref.COUT)):
        gw = g[off:off + 9 * oc * ic].reshape(3, 3, oc, ic).transpose(2, 3, 0, 1)[:cout]
        rw = params[li][0].grad.numpy()
        err = np.linalg.norm(gw - rw) / np.linalg.norm(rw)
        assert err < 2e-2, (li, err)
        gb = g[ref.N_W + boff:ref.N_W + boff + cout]
        rb = params[li][1].grad.numpy()
        assert np.linalg.norm(gb - rb) / max(np.linalg.norm(rb), 1e-12) < 2e-2, li
        # padding entries carry no gradient
        pad = g[off:off + 9 * oc * ic].reshape(9, oc, ic)
        assert (pad[:, cout:, :] == 0).all()
        if li == 0:
            assert (pad[:, :, 5:] == 0).all()
        off += 9 * oc * ic
        boff += cout


def test_train_step_deterministic_and_descends():
    F, H, W = 2, 40, 80
    master, _, _ = _params_bits(3)
    x0 = torch.from_numpy(_random_x0(F, H, W, 7).view(np.int16)).cuda()
    rng = np.random.default_rng(8)
    labels = torch.from_numpy((rng.random((F, H, W)) < 0.7).astype(np.uint8)).cuda()
    rho = torch.from_numpy(np.full((F, H, W), 100, np.uint16).view(np.int16)).cuda()
    g1 = torch.zeros(ref.N_W + ref.N_B, device="cuda")
    g2 = torch.zeros_like(g1)
    t = sldf.SurrogateTrainer(W, H, F, torch.from_numpy(master), lr=3e-3)
    t.step(x0, labels, rho, 2, update=False, grads_out=g1)
    t.step(x0, labels, rho, 2, update=False, grads_out=g2)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    losses = []
    for _ in range(30):
        st = t.step(x0, labels, rho, 2)
        losses.append(float(st[0].cpu()))
    assert losses[-1] < 0.8 * losses[0], losses


# both path pass schedules (1 paired, 2 split), 4 and 8 paths
SCHED_PATHS = [(1, 4), (2, 4), (1, 8), (2, 8)]


@pytest.mark.parametrize("schedule,paths", SCHED_PATHS)
def test_learned_run_matches_definition(schedule, paths):
    """sldf_run with check_impl = 1 (fallback off) equals
    (CNN logit > 0) or (rho <= Tc) on the features of the same frame."""
    f = synth.small_frame(3)
    pkw = dict(width=f["W"], height=f["H"], max_disp=f["D"], census_w=5, census_h=5,
               num_paths=paths, schedule=schedule)
    base = _features(f, pkw)
    _, wbits, b = _params_bits(4)
    wt = torch.from_numpy(wbits.view(np.int16)).cuda()
    bt = torch.from_numpy(b).cuda()
    z, _ = sldf.surrogate_forward(base["x0"][None].contiguous(), wt, bt)
    p = sldf.default_params(check_impl=1, fallback_tau=1.0, uncertain_margin=0.0, **pkw)
    ctx = sldf.Context(p)
    ctx.set_surrogate(wt, bt)
    disp, valid = ctx.run(base["left"], base["right"], base["lid"])
    torch.cuda.synchronize()
    exp = (z[0] > 0) | (base["rho"].to(torch.int32) <= p.tc)
    assert torch.equal(valid.bool(), exp)
    # valid pixels carry the same subpixel disparity as the plain run
    both = valid.bool() & base["valid"].bool()
    assert torch.equal(disp[both], base["disp"][both])
    assert (disp[~valid.bool()] == -1).all()


@pytest.mark.parametrize("schedule,paths", SCHED_PATHS)
def test_fallback_forced_equals_plain_check(schedule, paths):
    """tau = 0 with a margin no logit reaches: every frame falls back to the
    right-view pass and the plain check, bit-exactly."""
    f = synth.small_frame(4)
    pkw = dict(width=f["W"], height=f["H"], max_disp=f["D"], census_w=5, census_h=5,
               num_paths=paths, schedule=schedule)
    base = _features(f, pkw)
    _, wbits, b = _params_bits(5)
    wt = torch.from_numpy(wbits.view(np.int16)).cuda()
    bt = torch.from_numpy(b).cuda()
    p = sldf.default_params(check_impl=1, fallback_tau=0.0, uncertain_margin=1e30, **pkw)
    ctx = sldf.Context(p)
    ctx.set_surrogate(wt, bt)
    disp, valid = ctx.run(base["left"], base["right"], base["lid"])
    torch.cuda.synchronize()
    assert torch.equal(valid, base["valid"])
    assert torch.equal(disp, base["disp"])


def test_learned_requires_weights():
    f = synth.small_frame(0)
    p = sldf.default_params(width=f["W"], height=f["H"], max_disp=f["D"], census_w=5,
                            census_h=5, num_paths=4, check_impl=1)
    ctx = sldf.Context(p)
    img = sldf.device_image(f["left"])
    lid = torch.full((f["H"], f["W"]), -1, dtype=torch.int16, device="cuda")
    with pytest.raises(sldf.SldfError) as ei:
        ctx.run(img, img, lid)
    assert ei.value.status == sldf.ESTATE
