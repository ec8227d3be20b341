"""sldf_run captured into a HIP graph (through torch's graph capture on the
caller's stream) and replayed: every replay must equal the eager run bit for
bit.  Between replays the program does eager work of its own (another context
on another frame, plain torch kernels) and synchronizes, and the outputs are
overwritten before each replay, so a replay that skipped or reordered work
would show.  The single-frame 8-path case runs the two-stream schedule
(forked and joined with events inside the captured call); the learned case
captures the surrogate, its uncertainty counter and the gated fallback."""
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


def _surrogate(seed=4):
    from oracle import surrogate_ref as ref
    master = ref.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    master[ref.N_W:] = rng.normal(0, 0.1, ref.N_B).astype(np.float32)
    wbits = ref.f32_to_bf16_bits(master[:ref.N_W])
    return (torch.from_numpy(wbits.view(np.int16)).cuda(),
            torch.from_numpy(master[ref.N_W:].copy()).cuda())


@pytest.mark.parametrize("paths,schedule,learned", [(8, 0, 0), (8, 1, 0), (4, 0, 0), (8, 0, 1)])
def test_graph_replays_equal_eager(paths, schedule, learned):
    f = synth.small_frame(5)
    g_frame = synth.small_frame(6)
    pkw = dict(width=f["W"], height=f["H"], max_disp=f["D"], census_w=5, census_h=5,
               num_paths=paths, schedule=schedule)
    if learned:
        # learned check with the device-side fallback counter in the graph
        pkw.update(check_impl=1, fallback_tau=0.5)
    p = sldf.default_params(**pkw)
    ctx = sldf.Context(p)
    other = sldf.Context(p)
    if learned:
        sur = _surrogate()
        ctx.set_surrogate(*sur)
        other.set_surrogate(*sur)
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
