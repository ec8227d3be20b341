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
    x[..., :ref.N_IN] = rng.uniform(0, 1, size=(F, H, W, ref.N_IN))
    return ref.f32_to_bf16_bits(x)


U32 = 2.0 ** -24          # fp32 unit roundoff


def _nchw(bits_nhwc):
    """bf16 bits [F, H, W, C] -> float32 torch [F, C, H, W]."""
    return torch.from_numpy(ref.bf16_bits_to_f32(bits_nhwc)).permute(0, 3, 1, 2).contiguous()


def _layer(x, w, b, dil):
    """One convolution of the reference in fp32 (value) and on |x|, |w| (the
    sum of the absolute terms, for the accumulation error bound)."""
    y = torch.nn.functional.conv2d(x, w, b, padding=dil, dilation=dil)
    a = torch.nn.functional.conv2d(x.abs(), w.abs(), b.abs(), padding=dil, dilation=dil)
    return y, a


def _bf16(t):
    return ref.f32_to_bf16_bits(t.numpy())


def _check_layer_output(g_bits, y, a, n_terms, relu, what):
    """GPU bf16 output vs the fp32 reference value y of the same inputs: the
    two sums differ only in their order, by at most gamma_n * sum|terms|
    (gamma_n = n u / (1 - n u)); so the GPU value must be the bf16 rounding
    of some value in [y - tol, y + tol]: rounding is monotonic, so it lies
    between the roundings of the two interval ends (where the terms cancel,
    the interval can span several bf16 steps), and it equals the rounding
    of y wherever the interval holds no rounding boundary."""
    gam = n_terms * U32 / (1 - n_terms * U32)
    tol = gam * a
    lo, hi = y - tol, y + tol
    if relu:
        lo, hi, y = torch.relu(lo), torch.relu(hi), torch.relu(y)
    rl, rh = _bf16(lo.permute(0, 2, 3, 1)), _bf16(hi.permute(0, 2, 3, 1))
    g = g_bits[..., :y.shape[1]]
    gv, lv, hv = (ref.bf16_bits_to_f32(t) for t in (g, rl, rh))
    ok = (gv >= lv) & (gv <= hv)
    assert ok.all(), (what, np.argwhere(~ok)[:5])
    # most values sit far from a boundary: there the roundings agree and the
    # GPU value must be that rounding exactly (random weights cancel often,
    # so a few per cent of the intervals hold a boundary)
    exact = rl == rh
    assert (g[exact] == rl[exact]).all(), what
    assert exact.mean() > 0.9, (what, exact.mean())


# sizes: ragged row blocks and column tiles of every dilation; H = 200 gives
# seven row blocks per lattice at dilation 1; 16 x 16 (the smallest frame) is
# narrower than a tile and shorter than the largest dilation; 1242 x 375 is
# the benchmark's frame, one at a time (8-row lattice walks) and sixteen per
# call (32-row walks, the learned check of a batch)
@pytest.mark.parametrize("F,H,W", [(1, 37, 70), (2, 64, 129), (1, 200, 300), (1, 16, 16),
                                   (3, 16, 17), (1, 375, 1242), (16, 375, 1242)])
def test_forward_matches_reference(F, H, W):
    """Layer by layer on the GPU's own inputs: each bf16 activation is the
    rounding of the fp32 reference value within the accumulation error
    bound, and the logits are within that bound element by element.  End to
    end (the reference's own activations): the learned mask differs only
    where the reference logit is within one bf16 step of the last layer's
    terms of zero."""
    print(f"case forward F={F} {H}x{W}", flush=True)
    _, wbits, b = _params_bits(1)
    x0 = _random_x0(F, H, W, 3)
    z, acts = sldf.surrogate_forward(torch.from_numpy(x0.view(np.int16)).cuda(),
                                     torch.from_numpy(wbits.view(np.int16)).cuda(),
                                     torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    params = ref.unpack(ref.bf16_bits_to_f32(wbits), b)
    g_acts = [a.cpu().numpy().view(np.uint16) for a in acts]
    inputs = [_nchw(x0)] + [_nchw(g) for g in g_acts]
    with torch.no_grad():
        for l in range(3):
            w, bb, dil = params[l]
            y, a = _layer(inputs[l], w, bb, dil)
            _check_layer_output(g_acts[l], y, a, 9 * w.shape[1] + 1, True, f"layer {l + 1}")
        w, bb, dil = params[3]
        y, a = _layer(inputs[3], w, bb, dil)
        n = 9 * w.shape[1] + 1
        tol = (n * U32 / (1 - n * U32)) * a[:, 0]
        zg = z.cpu()
        assert ((zg - y[:, 0]).abs() <= tol).all(), "logits"
        # end to end: rounding boundaries taken differently upstream move a
        # logit by about one bf16 step of the last layer's terms at most
        ze, _, _ = ref.forward(x0, wbits, b)
        flip = (zg > 0) != (ze > 0)
        tau = 2.0 ** -7 * a[:, 0]
        assert (ze[flip].abs() <= tau[flip]).all(), "mask flips away from zero"
        assert ((zg - ze).abs() <= tau).float().mean() > 0.999


def _rne_interval(v, delta):
    """bf16 rounding of every value in [v - delta, v + delta]: the rounding
    of v, and how far the roundings of the interval ends are from it."""
    mid = ref.round_bf16(v)
    lo, hi = ref.round_bf16(v - delta), ref.round_bf16(v + delta)
    return mid, torch.maximum((hi - mid).abs(), (mid - lo).abs())


def test_backward_matches_reference():
    """Gradients of the masked BCE loss, element by element, against an fp32
    CPU backward pass on the GPU's own forward activations (both sides take
    the same ReLU masks) that stores the logit gradient and each hidden
    gradient map as bf16 (round to nearest even), as the kernels do.

    The two sides then differ only in fp32 summation order, and where a
    stored map value lies so close to a bf16 rounding boundary that the two
    orders round it to neighbouring values.  The test carries that through
    by interval arithmetic: at each map, the GPU value is a rounding of some
    value within gamma_n sum|terms| (n terms, gamma_n = n u / (1 - n u),
    u = 2^-24) plus the propagated bound of the input map's differences,
    and its difference from the reference's rounding is bounded by the
    roundings of the interval ends.  Each weight and bias gradient is then
    within gamma_N sum|terms| of its N = F H W terms plus the propagated
    bound of its gradient map.  A wrong tap, channel, transposition or gate
    in dgrad or wgrad is off by the order of the gradient itself; dgrad is
    covered through the weight gradients of the layers below it."""
    F, H, W = 2, 48, 96
    master, wbits, b = _params_bits(2)
    x0 = _random_x0(F, H, W, 5)
    rng = np.random.default_rng(6)
    labels = (rng.random((F, H, W)) < 0.8).astype(np.uint8)
    rho = rng.integers(0, 6, size=(F, H, W)).astype(np.uint16)
    tc = 2
    trainer = sldf.SurrogateTrainer(W, H, F, torch.from_numpy(master))
    g = torch.zeros(ref.N_W + ref.N_B, dtype=torch.float32, device="cuda")
    x0_d = torch.from_numpy(x0.view(np.int16)).cuda()
    trainer.step(x0_d, torch.from_numpy(labels).cuda(), torch.from_numpy(rho.view(np.int16)).cuda(),
                 tc, update=False, grads_out=g)
    zg, acts = sldf.surrogate_forward(x0_d, torch.from_numpy(wbits.view(np.int16)).cuda(),
                                      torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    params = ref.unpack(ref.bf16_bits_to_f32(wbits), b)
    ins = [_nchw(x0)] + [_nchw(a.cpu().numpy().view(np.uint16)) for a in acts]
    m = torch.from_numpy((rho > tc).astype(np.float32))
    y = torch.from_numpy(labels.astype(np.float32))
    gam = lambda n: n * U32 / (1 - n * U32)
    # logit gradient m (sigma(z) - y) / (F H W); the GPU's sigmoid (fast exp
    # and division) is taken as good to 2^-16 relative, far below a bf16 step
    sg = torch.sigmoid(zg.cpu())
    inv_n = 1.0 / (F * H * W)
    gcur, err = _rne_interval((m * (sg - y) * inv_n)[:, None], (m * sg * 2.0 ** -16 * inv_n)[:, None])
    gout, eout = [None] * 4, [None] * 4
    for li in (3, 2, 1, 0):
        w, _, dil = params[li]
        gout[li], eout[li] = gcur, err
        if li > 0:
            mask = (ins[li] > 0).float()
            back = lambda t, ww: torch.nn.grad.conv2d_input(ins[li].shape, ww, t, padding=dil,
                                                            dilation=dil) * mask
            v = back(gcur, w)
            delta = gam(9 * w.shape[0]) * back(gcur.abs(), w.abs()) + back(err, w.abs())
            gcur, err = _rne_interval(v, delta)
    N = F * H * W
    off, boff = 0, 0
    for li, ((oc, ic, dil), cout) in enumerate(zip(ref.LAYERS, ref.COUT)):
        w = params[li][0]
        wg = lambda a, t: torch.nn.grad.conv2d_weight(a, w.shape, t, padding=dil,
                                                      dilation=dil).numpy()
        rw = wg(ins[li], gout[li])
        bound = gam(N) * wg(ins[li].abs(), gout[li].abs()) + wg(ins[li].abs(), eout[li])
        gw = g[off:off + 9 * oc * ic].reshape(3, 3, oc, ic).transpose(2, 3, 0, 1)[:cout]
        bad = np.abs(gw - rw) > bound + 1e-12
        assert not bad.any(), (li, np.argwhere(bad)[:5], np.abs(gw - rw).max())
        # the bound is not vacuous: it is a small fraction of the gradient
        assert bound.sum() < 0.25 * np.abs(rw).sum(), (li, bound.sum() / np.abs(rw).sum())
        gb = g[ref.N_W + boff:ref.N_W + boff + cout]
        rb = gout[li].sum(dim=(0, 2, 3)).numpy()
        bb = (gam(N) * gout[li].abs() + eout[li]).sum(dim=(0, 2, 3)).numpy()
        assert (np.abs(gb - rb) <= bb + 1e-12).all(), li
        # padding entries carry no gradient
        pad = g[off:off + 9 * oc * ic].reshape(9, oc, ic)
        assert (pad[:, cout:, :] == 0).all()
        if li == 0:
            assert (pad[:, :, ref.N_IN:] == 0).all()
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
    # the labels are random: below the entropy of their frequency (the best
    # constant predictor) only by fitting the inputs pixel by pixel
    p1 = float(labels.float().mean())
    entropy = -(p1 * np.log(p1) + (1 - p1) * np.log(1 - p1))
    assert losses[-1] < 0.9 * losses[0] and losses[-1] < entropy, (losses, entropy)


# every path pass schedule (1 paired, 2 split, 3 two sweeps), 4 and 8 paths
SCHED_PATHS = [(1, 4), (2, 4), (3, 4), (1, 8), (2, 8), (3, 8)]


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


def test_surrogate_blob_load_equals_attached_pointers():
    """sldf_surrogate_load (one blob) runs the same network as
    sldf_surrogate_set_weights; blobs of the wrong size or alignment are
    rejected."""
    f = synth.small_frame(2)
    pkw = dict(width=f["W"], height=f["H"], max_disp=f["D"], census_w=5, census_h=5,
               num_paths=8)
    base = _features(f, pkw)
    _, wbits, b = _params_bits(6)
    wt = torch.from_numpy(wbits.view(np.int16)).cuda()
    bt = torch.from_numpy(b).cuda()
    p = sldf.default_params(check_impl=1, fallback_tau=1.0, uncertain_margin=0.0, **pkw)
    outs = []
    for use_blob in (False, True):
        ctx = sldf.Context(p)
        if use_blob:
            blob = sldf.surrogate_blob(wt, bt)
            ctx.load_surrogate(blob)
            with pytest.raises(sldf.SldfError):
                ctx.load_surrogate(blob[:-4])
            with pytest.raises(sldf.SldfError):
                ctx.load_surrogate(torch.zeros(blob.numel() + 16, dtype=torch.uint8,
                                               device="cuda")[16:])
            ctx.load_surrogate(blob)
        else:
            ctx.set_surrogate(wt, bt)
        disp, valid = ctx.run(base["left"], base["right"], base["lid"])
        torch.cuda.synchronize()
        outs.append((disp.clone(), valid.clone()))
        ctx.close()
    assert torch.equal(outs[0][1], outs[1][1])
    assert torch.equal(outs[0][0], outs[1][0])


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


def test_committed_weights_agree_with_plain_check_on_heldout_frames():
    """The committed learned-check weights on held-out frames of the
    surrogate workload (paper-scale synthetic frames 2000..2007, never seen
    in training): the learned sldf_run_batch with its default fallback
    setting agrees with the plain check (Eq. 6) on at least 99 % of pixels."""
    from paper_2504_05148_amd.train_surrogate import load_weights
    w, b, meta = load_weights()
    frames = [synth.make_frame(synth.KITTI, synth.CONFIG_IDS["surrogate"], 2000 + i)
              for i in range(8)]
    F, D = len(frames), 128
    left = sldf.device_images(np.stack([f["left"] for f in frames]))
    right = sldf.device_images(np.stack([f["right"] for f in frames]))
    lid = torch.stack([sldf.quantize_lidar(torch.from_numpy(f["lidar"]).cuda(), D)
                       for f in frames])
    _, vp = sldf.Context(sldf.default_params(batch=F)).run_batch(left, right, lid)
    cl = sldf.Context(sldf.default_params(batch=F, check_impl=1))
    cl.set_surrogate(w, b)
    _, vl = cl.run_batch(left, right, lid)
    torch.cuda.synchronize()
    agree = float((vl == vp).float().mean())
    print(f"held-out agreement {agree:.5f}", flush=True)
    assert agree >= 0.99


def test_learned_bench_launch_configuration(bench_frames):
    """The learned check in the benchmark's launch configuration at 1242 x 375,
    D = 128: one 128-frame call, and two contexts of 64 frames on two streams
    (twice), bit for bit equal; sampled frames equal single-frame learned
    runs (the convolutions sum in a fixed order whatever their tiling)."""
    from paper_2504_05148_amd.train_surrogate import load_weights
    w, b, _ = load_weights()
    frames = bench_frames
    B, D = len(frames), 128
    left = sldf.device_images(np.stack([f["left"] for f in frames]))
    right = sldf.device_images(np.stack([f["right"] for f in frames]))
    lid = torch.stack([sldf.quantize_lidar(torch.from_numpy(f["lidar"]).cuda(), D)
                       for f in frames])
    print("case learned one 128-frame call", flush=True)
    c = sldf.Context(sldf.default_params(batch=B, check_impl=1))
    c.set_surrogate(w, b)
    d_all, v_all = c.run_batch(left, right, lid)
    torch.cuda.synchronize()
    del c
    print("case learned 2 streams x 64 frames", flush=True)
    n = B // 2
    streams = (torch.cuda.current_stream(), torch.cuda.Stream())
    ctxs = []
    for _ in range(2):
        ci = sldf.Context(sldf.default_params(batch=n, check_impl=1))
        ci.set_surrogate(w, b)
        ctxs.append(ci)
    outs = [ci.new_outputs(n) for ci in ctxs]
    torch.cuda.synchronize()
    for rep in range(2):
        for i, st in enumerate(streams):
            sl = slice(i * n, (i + 1) * n)
            ctxs[i].run_batch(left[sl], right[sl], lid[sl], outs[i][0], outs[i][1], stream=st)
        torch.cuda.synchronize()
        for i in range(2):
            sl = slice(i * n, (i + 1) * n)
            assert torch.equal(outs[i][1], v_all[sl]), (rep, i)
            assert torch.equal(outs[i][0], d_all[sl]), (rep, i)
    del ctxs, outs
    print("case learned single frames", flush=True)
    c1 = sldf.Context(sldf.default_params(batch=1, check_impl=1))
    c1.set_surrogate(w, b)
    for i in (0, 63, 64, B - 1):
        d1, v1 = c1.run(left[i], right[i], lid[i])
        torch.cuda.synchronize()
        assert torch.equal(v1, v_all[i]) and torch.equal(d1, d_all[i]), i
