"""Pins for the surrogate reference (CPU): the packed [tap][out][in] layout
and the dilated tap offsets, by a one-hot weight that must shift the input."""
import numpy as np
import torch

from oracle import surrogate_ref as ref


def test_one_hot_tap_shifts_input():
    F, H, W = 1, 20, 30
    rng = np.random.default_rng(0)
    x = np.zeros((F, H, W, 8), np.float32)
    x[..., 2] = rng.integers(1, 9, size=(F, H, W))          # exact in bf16
    xb = ref.f32_to_bf16_bits(x)
    w = np.zeros(ref.N_W, np.float32)
    b = np.zeros(ref.N_B, np.float32)
    # layer 1: tap (ky, kx) = (0, 2) -> offset (dy, dx) = (-1, +1) * dilation 1,
    # output channel 3 <- input channel 2
    tap = 0 * 3 + 2
    w[(tap * 32 + 3) * 8 + 2] = 1.0
    # layers 2-3: identity on channel 3 at the centre tap; layer 4 reads ch 3
    off2 = 9 * 32 * 8
    off3 = off2 + 9 * 32 * 32
    off4 = off3 + 9 * 32 * 32
    w[off2 + (4 * 32 + 3) * 32 + 3] = 1.0
    w[off3 + (4 * 32 + 3) * 32 + 3] = 1.0
    w[off4 + (4 * 16 + 0) * 32 + 3] = 1.0
    z, acts, _ = ref.forward(xb, ref.f32_to_bf16_bits(w), b)
    a1 = acts[0][0, 3].numpy()
    exp = np.zeros((H, W), np.float32)
    exp[1:, :-1] = x[0, :-1, 1:, 2]                           # a1[y, x] = x[y-1, x+1]
    assert np.array_equal(a1, exp)
    assert np.array_equal(z[0].numpy(), exp)


def test_init_params_padding_is_zero():
    m = ref.init_params(3)
    w1 = m[:9 * 32 * 8].reshape(9, 32, 8)
    assert (w1[:, :, ref.N_IN:] == 0).all() and (w1[:, :, :ref.N_IN] != 0).all(axis=(0, 1)).all()
    w4 = m[ref.N_W - 9 * 16 * 32:ref.N_W].reshape(9, 16, 32)
    assert (w4[:, 1:, :] == 0).all()
    assert m.size == ref.N_W + ref.N_B == 25344 + 97


def test_bf16_bits_are_the_oracle_rounding():
    """The reference rounds with the oracle's pinned bf16 rounding: ties to
    even, values just off a tie, and the sign."""
    import oracle
    x = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, 1.01171875, -2.5, -1.00390625,
                  3.0e-5, 65504.0], np.float32)
    bits = ref.f32_to_bf16_bits(x)
    assert (bits == oracle.bf16_round(x)).all()
    # 1 + 2^-8 ties to 1.0 (even), 1 + 3 * 2^-8 ties to 1 + 2^-6 (even)
    assert ref.bf16_bits_to_f32(bits).tolist()[:5] == [1.0, 1.0, 1.0078125, 1.0078125, 1.015625]


def test_reference_gradient_matches_finite_differences():
    """The reference loss (masked BCE of the logits, mean over all pixels)
    and its autograd gradient, pinned by central differences in float64 on
    the network without activation rounding, for weights of every layer,
    both sides of the 3 x 3 grid and a bias."""
    F, H, W = 1, 20, 36
    master = ref.init_params(9)
    rng0 = np.random.default_rng(109)
    master[ref.N_W:] = rng0.normal(0, 0.1, ref.N_B).astype(np.float32)
    x = np.zeros((F, H, W, 8))
    x[..., :ref.N_IN] = rng0.uniform(0, 1, size=(F, H, W, ref.N_IN))
    x = torch.from_numpy(x).permute(0, 3, 1, 2).contiguous()
    rng = np.random.default_rng(12)
    y = torch.from_numpy((rng.random((F, H, W)) < 0.7).astype(np.float64))
    m = torch.from_numpy((rng.integers(0, 5, size=(F, H, W)) > 2).astype(np.float64))
    params = [(w.double().clone().requires_grad_(True), bb.double().clone().requires_grad_(True),
               d) for w, bb, d in ref.unpack(master[:ref.N_W], master[ref.N_W:])]

    def loss_of(ps):
        h = x
        for li, (w, bb, d) in enumerate(ps):
            h = torch.nn.functional.conv2d(h, w, bb, padding=d, dilation=d)
            if li < 3:
                h = torch.relu(h)
        z = h[:, 0]
        return (m * (torch.nn.functional.softplus(z) - y * z)).sum() / (F * H * W)

    loss_of(params).backward()
    eps = 1e-6
    picks = [(0, (3, 2, 0, 0)), (0, (7, 5, 2, 2)), (1, (11, 30, 1, 0)), (2, (0, 4, 2, 1)),
             (3, (0, 17, 0, 2)), (3, (0, 3, 1, 1))]
    for li, idx in picks:
        w = params[li][0]
        with torch.no_grad():
            old = w[idx].item()
            w[idx] = old + eps
            lp = loss_of(params).item()
            w[idx] = old - eps
            lm = loss_of(params).item()
            w[idx] = old
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - w.grad[idx].item()) <= 1e-6 * max(1.0, abs(fd)), (li, idx, fd)
    bb = params[2][1]
    with torch.no_grad():
        old = bb[5].item()
        bb[5] = old + eps
        lp = loss_of(params).item()
        bb[5] = old - eps
        lm = loss_of(params).item()
        bb[5] = old
    assert abs((lp - lm) / (2 * eps) - bb.grad[5].item()) <= 1e-6
