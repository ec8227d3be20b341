"""Reference of the learned consistency surrogate: plain PyTorch fp32 on the
CPU.  Test infrastructure only (like the rest of this package): the HIP
kernels are checked against it, never the other way round.

The network is the one the library runs for check_impl = 1: four 3x3
convolutions with dilations 1, 3, 9, 27 and channels 8 (6 used) -> 32 -> 32
-> 32 -> 1, ReLU after the first three.  Inputs and weights are bf16 values;
accumulation is fp32; the stored hidden activations are rounded to bf16 (round
to nearest even), as the kernels store them.
"""
from __future__ import annotations

import numpy as np
import torch

# packed weight layout per layer: [9 taps][out][in], taps in raster order
LAYERS = [(32, 8, 1), (32, 32, 3), (32, 32, 9), (16, 32, 27)]   # (out_pad, in, dilation)
COUT = [32, 32, 32, 1]
N_W = sum(9 * o * i for o, i, _ in LAYERS)
N_B = 32 + 32 + 32 + 1
N_IN = 6            # input channels in use (of 8): the six features of the library


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16).view(np.float32)


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bf16 bit patterns (round to nearest even): the oracle's
    pinned rounding."""
    from oracle import bf16_round
    return bf16_round(x)


def round_bf16(t: torch.Tensor) -> torch.Tensor:
    """Round float32 values to the nearest bf16 (ties to even)."""
    return torch.from_numpy(bf16_bits_to_f32(f32_to_bf16_bits(t.detach().numpy())))


def unpack(weights_f32: np.ndarray, biases: np.ndarray):
    """Packed parameter blob -> list of (torch weight [out, in, 3, 3], bias)."""
    out, off, boff = [], 0, 0
    for (oc, ic, dil), cout in zip(LAYERS, COUT):
        w = weights_f32[off:off + 9 * oc * ic].reshape(3, 3, oc, ic)
        w = np.transpose(w, (2, 3, 0, 1))[:cout]          # [out, in, ky, kx]
        out.append((torch.tensor(np.ascontiguousarray(w)), torch.tensor(biases[boff:boff + cout]),
                    dil))
        off += 9 * oc * ic
        boff += cout
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform fp32 master parameters (weights then biases), padding zero."""
    rng = np.random.default_rng(seed)
    w = np.zeros(N_W, np.float32)
    off = 0
    for (oc, ic, _), cout, cin_used in zip(LAYERS, COUT, [N_IN, 32, 32, 32]):
        blk = np.zeros((9, oc, ic), np.float32)
        bound = np.sqrt(6.0 / (9 * cin_used))
        blk[:, :cout, :cin_used] = rng.uniform(-bound, bound, size=(9, cout, cin_used))
        w[off:off + blk.size] = blk.ravel()
        off += blk.size
    b = np.zeros(N_B, np.float32)
    return np.concatenate([w, b])


def forward(x0_bits: np.ndarray, weight_bits: np.ndarray, biases: np.ndarray,
            straight_through: bool = False):
    """x0_bits uint16 [F, H, W, 8] -> (logits [F, H, W], [a1, a2, a3] NHWC)
    as torch tensors.  With straight_through the bf16 rounding of the hidden
    activations is an identity for autograd."""
    params = unpack(bf16_bits_to_f32(weight_bits), biases)
    x = torch.from_numpy(bf16_bits_to_f32(x0_bits)).permute(0, 3, 1, 2).contiguous()
    acts = []
    for li, (w, b, dil) in enumerate(params):
        if straight_through:
            w.requires_grad_(True)
            b.requires_grad_(True)
        y = torch.nn.functional.conv2d(x, w, b, padding=dil, dilation=dil)
        if li < 3:
            y = torch.relu(y)
            y = y + (round_bf16(y) - y).detach()
            acts.append(y)
        x = y
    return x[:, 0], acts, params
