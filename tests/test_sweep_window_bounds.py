"""Host model of the first sweep's census-window reads: every byte offset the
kernel forms (summed in 32 bits, then added to the frame's base) stays inside
the census allocation, for every view, row, lane and clamped step position.

Layout modelled (as the library allocates it): rows of W + 2D codes (D pad
codes on each side), frames back to back, one guard row before the first and
after the last frame; the kernel addresses a frame from the padded start of
the row before its row 0.  The window reads the entering matching code at
positions clamped to [-8, W], the whole run of the first step from the same
clamped position, and the base code at positions clamped to [-1, W]."""
import numpy as np
import pytest


def _reads(W, H, D, F=2):
    K = 8
    G = D // 8
    cpitch = W + 2 * D
    cframe = cpitch * H
    alloc = (F * cframe + 2 * cpitch) * 4
    lo, hi = alloc, 0
    # every offset is linear in the row, so its first and last rows bound it
    y0 = np.array([0, H - 1], dtype=np.int64)[:, None, None]
    d0 = (8 * np.arange(G, dtype=np.int64))[None, :, None]
    um = np.arange(-K, W + 1, dtype=np.int64)[None, None, :]
    uc = np.arange(-1, W + 1, dtype=np.int64)[None, None, :]
    for frame in (0, F - 1):
        base = frame * cframe * 4
        oc0 = ((y0 + 1) * cpitch + D) * 4
        for view in (0, 1):
            om0 = oc0 - (d0 + K - 1) * 4 if view == 0 else oc0 + d0 * 4
            wrap = lambda v: (v.astype(np.int64) % (1 << 32))
            ent = base + wrap(om0 + um * 4 + 4 * (K - 1))          # entering code, 4 B
            run = base + wrap(om0 + um * 4)                          # first step's run, 32 B
            cb = base + wrap(oc0 + uc * 4 + 0 * d0)                  # base code, 4 B
            lo = min(lo, int(ent.min()), int(run.min()), int(cb.min()))
            hi = max(hi, int(ent.max()) + 4, int(run.max()) + 32, int(cb.max()) + 4)
    return lo, hi, alloc


@pytest.mark.parametrize("W,H,D", [(320, 96, 64), (16, 16, 64), (17, 16, 256), (333, 77, 128),
                                   (1242, 375, 128), (640, 480, 256), (1920, 1080, 256)])
def test_window_reads_stay_in_the_census_allocation(W, H, D):
    lo, hi, alloc = _reads(W, H, D)
    assert 0 <= lo and hi <= alloc


def test_offsets_added_one_by_one_would_leave_the_buffer():
    """The pitfall the model guards: a negative step product added to the
    pointer on its own is zero-extended, 4 GiB past the row."""
    W, D = 320, 64
    oc0 = ((0 + 1) * (W + 2 * D) + D) * 4
    separate = oc0 + ((-1 * 4) % (1 << 32))
    summed = (oc0 - 4) % (1 << 32)
    assert separate > 1 << 32 and summed < 4 * (W + 2 * D) * 2
