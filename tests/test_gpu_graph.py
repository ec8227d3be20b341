"""sldf_run captured into a HIP graph (through torch's graph capture on the
caller's stream) and replayed: every replay must equal the eager run bit for
bit.  Between replays the program does eager work of its own (another context
on another frame, plain torch kernels) and synchronizes, and the outputs are
overwritten before each replay, so a replay that skipped or reordered work
would show.  The single-frame 8-path case runs the two-stream schedule
(forked and joined with events inside the captured call)."""
import numpy as np
import pytest
import torch

from paper_2504_05148_amd import sldf, synth

pytestmark = pytest.mark.gpu


def _inputs(f, D):
    left = sldf.device_image(f["left"])
    right = sldf.device_image(f["right"])
    lid = sldf.quantize_lidar(torch.from_numpy(np.ascontiguousarray(f["lidar"])).cuda(), D)
    return left, right, lid


@pytest.mark.parametrize("paths,schedule", [(8, 0), (8, 1), (4, 0)])
def test_graph_replays_equal_eager(paths, schedule):
    f = synth.small_frame(5)
    g_frame = synth.small_frame(6)
    pkw = dict(width=f["W"], height=f["H"], max_disp=f["D"], census_w=5, census_h=5,
               num_paths=paths, schedule=schedule)
    p = sldf.default_params(**pkw)
    ctx = sldf.Context(p)
    other = sldf.Context(p)
    left, right, lid = _inputs(f, p.max_disp)
    l2, r2, lid2 = _inputs(g_frame, p.max_disp)
    disp, valid = ctx.new_outputs()
    ctx.run(left, right, lid, disp, valid)
    torch.cuda.synchronize()
    d_ref, v_ref = disp.clone(), valid.clone()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ctx.run(left, right, lid, disp, valid)
    torch.cuda.synchronize()
    for k in range(4):
        # eager work between replays, then wipe the outputs
        d_o, v_o = other.run(l2, r2, lid2)
        x = torch.randn(1 << 20, device="cuda").sum()
        disp.fill_(-123.0)
        valid.fill_(7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(disp, d_ref), k
        assert torch.equal(valid, v_ref), k
        assert bool(torch.isfinite(x))
        assert d_o.shape == disp.shape
