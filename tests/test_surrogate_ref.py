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
    assert (w1[:, :, 5:] == 0).all() and (w1[:, :, :5] != 0).any()
    w4 = m[ref.N_W - 9 * 16 * 32:ref.N_W].reshape(9, 16, 32)
    assert (w4[:, 1:, :] == 0).all()
    assert m.size == ref.N_W + ref.N_B == 25344 + 97
