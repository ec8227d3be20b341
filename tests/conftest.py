import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def bench_frames():
    """The benchmark's 128 paper-scale frames of one step as parity inputs:
    16 synthetic 1242 x 375 frames, each in eight copies whose views and LiDAR
    map are rolled together by 7 k columns, so that every frame of the batch
    differs (parity needs distinct inputs, not real scenes)."""
    import numpy as np
    from paper_2504_05148_amd import synth
    base = [synth.kitti_frame(i) for i in range(16)]
    return [dict(base[i % 16], **{c: np.roll(base[i % 16][c], 7 * (i // 16), axis=1)
                                  for c in ("left", "right", "lidar")}) for i in range(128)]
