"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by
element on the same seeded inputs: bit-exact for census codes, the prior
map, the aggregated cost S, integer disparities and masks; the subpixel
disparity within 1e-4 px (expected bit-exact)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_05148_amd import sldf, synth

pytestmark = pytest.mark.gpu

SUB_TOL = 1e-4


def _params(W, H, D, **kw):
    base = dict(width=W, height=H, max_disp=D)
    base.update(kw)
    return base


def _oracle_params(p: dict) -> oracle.OracleParams:
    return oracle.OracleParams(
        W=p["width"], H=p["height"], D=p["max_disp"], cw=p.get("census_w", 9),
        ch=p.get("census_h", 7), num_paths=p.get("num_paths", 8), p1=p.get("p1", 10),
        p2=p.get("p2", 120), q1=p.get("q1", 5), q2=p.get("q2", 160),
        a=p.get("alpha_num", 7), b=p.get("alpha_den", 10), blend_mode=p.get("blend_mode", 0),
        semidense=p.get("semidense", 1), ts=p.get("ts", 2), rs=p.get("rs", 6),
        tc=p.get("tc", 2), rc=p.get("rc", 20), check_mode=p.get("check_mode", 3),
        subpixel=p.get("subpixel", 1), prior_cost=p.get("prior_cost", 0),
        huber_k=p.get("huber_k", 1), census_kind=p.get("census_kind", 0))


def run_gpu(frame, pkw, taps=True):
    p = sldf.default_params(**pkw)
    W, H, D = p.width, p.height, p.max_disp
    ctx = sldf.Context(p)
    left = sldf.device_image(frame["left"])
    right = sldf.device_image(frame["right"])
    lid_f = torch.from_numpy(np.ascontiguousarray(frame["lidar"])).cuda()
    lid_q = sldf.quantize_lidar(lid_f, D)
    out = {}
    if taps:
        dev = "cuda"
        t = dict(census_l=torch.empty((H, W), dtype=torch.int32, device=dev),
                 census_r=torch.empty((H, W), dtype=torch.int32, device=dev),
                 prior=torch.empty((H, W), dtype=torch.int16, device=dev),
                 cost_sum=torch.empty((H, W, D), dtype=torch.int16, device=dev),
                 dstar=torch.empty((H, W), dtype=torch.int16, device=dev),
                 dright=torch.full((H, W), -7, dtype=torch.int16, device=dev),
                 dsub=torch.empty((H, W), dtype=torch.float32, device=dev),
                 rho=torch.empty((H, W), dtype=torch.int16, device=dev),
                 features=torch.empty((H, W, 8), dtype=torch.int16, device=dev))
        ctx.set_taps(**t)
    disp, valid = ctx.run(left, right, lid_q)
    torch.cuda.synchronize()
    out["disp"] = disp.cpu().numpy()
    out["valid"] = valid.cpu().numpy()
    out["lidar_q"] = lid_q.cpu().numpy()
    if taps:
        out["census_l"] = t["census_l"].cpu().numpy().view(np.uint32)
        out["census_r"] = t["census_r"].cpu().numpy().view(np.uint32)
        out["prior"] = t["prior"].cpu().numpy()
        out["S"] = t["cost_sum"].cpu().numpy().view(np.uint16)
        out["dstar"] = t["dstar"].cpu().numpy()
        out["dright"] = t["dright"].cpu().numpy()
        out["dsub"] = t["dsub"].cpu().numpy()
        out["rho"] = t["rho"].cpu().numpy().view(np.uint16)
        out["features"] = t["features"].cpu().numpy().view(np.uint16)
    ctx.close()
    return out


def run_oracle(frame, pkw):
    op = _oracle_params(sldf.default_params(**pkw).as_dict() | pkw)
    lid = oracle.quantize_lidar(frame["lidar"], op.D)
    r = oracle.run(op, frame["left"], frame["right"], lid, taps=True)
    r["lidar_q"] = lid
    r["rho"] = oracle.lidar_residual(r["dstar"], lid, op.D, op.rc)
    f = oracle.surrogate_features(r["S"], r["dstar"], r["rho"], op.num_paths, op.b * op.p2)
    feats = np.zeros(f.shape[:2] + (8,), np.uint16)
    feats[..., :6] = oracle.bf16_round(f)
    r["features"] = feats
    return r


def assert_parity(g, o, pkw, taps=True):
    assert (g["lidar_q"] == o["lidar_q"]).all(), "lidar quantisation"
    if taps:
        assert (g["census_l"] == o["census_l"]).all(), "census left"
        assert (g["census_r"] == o["census_r"]).all(), "census right"
        assert (g["prior"] == o["prior"]).all(), "prior map"
        bad = g["S"].astype(np.int64) != o["S"]
        assert not bad.any(), f"S mismatch at {np.argwhere(bad)[:5]}"
        assert (g["dstar"] == o["dstar"]).all(), "d*"
        if pkw.get("check_mode", 3) in (1, 3):
            assert (g["dright"] == o["dright"]).all(), "d'"
        diff = np.abs(g["dsub"] - o["dsub"])
        assert diff.max() <= SUB_TOL, f"dsub max diff {diff.max()}"
        assert (g["rho"] == o["rho"]).all(), "LiDAR residual"
        bad = g["features"] != o["features"]
        assert not bad.any(), f"surrogate features differ at {np.argwhere(bad)[:5]}"
    assert (g["valid"] == o["valid"]).all(), f"mask mismatch {np.argwhere(g['valid'] != o['valid'])[:5]}"
    assert (g["disp"][g["valid"] == 0] == -1.0).all()
    d = np.abs(g["disp"] - o["disp"])
    assert d.max() <= SUB_TOL, f"disp max diff {d.max()}"


SMALL = dict(census_w=5, census_h=5, num_paths=4)


# path pass schedules (identical results): 1 = paired directions on one
# line, 2 = split (each direction its own line pass, then one WTA pass),
# 3 = two sweeps (four directions per walk over the rows, bands of rows
# handed on through the workspace)
SCHEDULES = [1, 2, 3]


@pytest.mark.parametrize("idx", [0, 1])
@pytest.mark.parametrize("semi", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("schedule", SCHEDULES)
def test_small_workload(idx, semi, mode, schedule):
    f = synth.small_frame(idx)
    pkw = _params(f["W"], f["H"], f["D"], semidense=semi, check_mode=mode, schedule=schedule,
                  **SMALL)
    print(f"case small idx={idx} semi={semi} mode={mode} schedule={schedule}", flush=True)
    assert_parity(run_gpu(f, pkw), run_oracle(f, pkw), pkw)


def test_small_bit_exact_subpixel():
    f = synth.small_frame(2)
    pkw = _params(f["W"], f["H"], f["D"], **SMALL)
    g, o = run_gpu(f, pkw), run_oracle(f, pkw)
    assert (g["dsub"].view(np.uint32) == o["dsub"].view(np.uint32)).all()


def test_paper_scale_frame():
    """1242 x 375, D = 128, 9x7 census, 8 paths, SDSGM, stereo-LiDAR check,
    under both path pass schedules."""
    f = synth.kitti_frame(0)
    pkw = _params(1242, 375, 128)
    o = run_oracle(f, pkw)
    for schedule in SCHEDULES:
        print(f"case kitti frame 0 schedule={schedule}", flush=True)
        g = run_gpu(f, dict(pkw, schedule=schedule))
        assert_parity(g, o, pkw)
        assert (g["dsub"].view(np.uint32) == o["dsub"].view(np.uint32)).all()


@pytest.mark.parametrize("prior_cost,huber_k", [(1, 1), (2, 2)])
def test_paper_scale_alternative_prior_terms(prior_cost, huber_k):
    """The quadratic and Huber LiDAR terms through the same aggregation."""
    f = synth.kitti_frame(3)
    pkw = _params(1242, 375, 128, prior_cost=prior_cost, huber_k=huber_k, q2=980)
    print(f"case kitti prior_cost={prior_cost} k={huber_k}", flush=True)
    assert_parity(run_gpu(f, pkw), run_oracle(f, pkw), pkw)


def test_paper_scale_dsgm():
    f = synth.kitti_frame(1)
    pkw = _params(1242, 375, 128, semidense=0)
    o = run_oracle(f, pkw)
    for schedule in SCHEDULES:
        print(f"case kitti dsgm schedule={schedule}", flush=True)
        assert_parity(run_gpu(f, dict(pkw, schedule=schedule)), o, pkw)


@pytest.mark.parametrize("W,H,D,paths", [(333, 77, 128, 8), (130, 19, 64, 8), (301, 40, 256, 8),
                                         (300, 45, 256, 4), (97, 130, 64, 4),
                                         # the smallest frame, and a disparity range wider
                                         # than the image
                                         (16, 16, 64, 8), (16, 16, 64, 4), (17, 16, 256, 8)])
def test_ragged_shapes(W, H, D, paths):
    """Shapes that are not multiples of any tile, every disparity range."""
    spec = synth.robust_spec(W=W, H=H, D=D, density=0.05, lines=16)
    f = synth.make_frame(spec, 3, W * 7 + H)
    pkw = _params(W, H, D, num_paths=paths)
    o = run_oracle(f, pkw)
    for schedule in SCHEDULES:
        print(f"case ragged {W}x{H} D={D} paths={paths} schedule={schedule}", flush=True)
        assert_parity(run_gpu(f, dict(pkw, schedule=schedule)), o, pkw)


@pytest.mark.parametrize("extra", [
    dict(blend_mode=1), dict(subpixel=0), dict(num_paths=1), dict(rs=0, rc=0, tc=0),
    dict(rs=15, rc=31, ts=9), dict(alpha_num=0), dict(alpha_num=10, q1=0, q2=5),
    dict(census_w=7, census_h=7), dict(census_w=3, census_h=9), dict(p1=0, p2=0),
    dict(prior_cost=1), dict(prior_cost=1, q2=980), dict(prior_cost=2, huber_k=1),
    dict(prior_cost=2, huber_k=3, q2=980),
    # the full census (24 and 26 bits)
    dict(census_kind=1), dict(census_kind=1, census_w=3, census_h=9),
])
def test_parameter_variants(extra):
    f = synth.small_frame(4)
    pkw = _params(f["W"], f["H"], f["D"], **SMALL)
    pkw.update(extra)
    o = run_oracle(f, pkw)
    for schedule in SCHEDULES:
        print(f"case variant {extra} schedule={schedule}", flush=True)
        assert_parity(run_gpu(f, dict(pkw, schedule=schedule)), o, pkw)


@pytest.mark.parametrize("density", [0.0, 0.3])
def test_lidar_empty_and_dense(density):
    f = dict(synth.small_frame(5))
    rng = np.random.default_rng(5)
    lid = np.full(f["lidar"].shape, np.nan, np.float32)
    m = rng.random(lid.shape) < density
    lid[m] = (f["gt"][m] + rng.normal(0, 0.4, m.sum())).astype(np.float32)
    f["lidar"] = lid
    pkw = _params(f["W"], f["H"], f["D"], **SMALL)
    assert_parity(run_gpu(f, pkw), run_oracle(f, pkw), pkw)


def test_lidar_quantise_edge_values():
    vals = np.array([[np.nan, -0.3, 0.4, 2.5, 3.5, 62.5, 63.49, 63.5, 100.0, -np.inf, np.inf,
                      0.5, 1.5, 127.5, 126.5, 0.0]], np.float32)
    vals = np.repeat(vals, 3, axis=0)
    g = sldf.quantize_lidar(torch.from_numpy(vals).cuda(), 64).cpu().numpy()
    assert (g == oracle.quantize_lidar(vals, 64)).all()


def test_batch_matches_single_frames():
    """run_batch over 3 frames equals three single-frame runs and the oracle."""
    frames = [synth.small_frame(i) for i in (6, 7, 8)]
    W, H, D = frames[0]["W"], frames[0]["H"], frames[0]["D"]
    p = sldf.default_params(width=W, height=H, max_disp=D, batch=3, **SMALL)
    ctx = sldf.Context(p)
    left = sldf.device_images(np.stack([f["left"] for f in frames]))
    right = sldf.device_images(np.stack([f["right"] for f in frames]))
    lid = torch.stack([sldf.quantize_lidar(torch.from_numpy(f["lidar"]).cuda(), D)
                       for f in frames])
    disp, valid = ctx.run_batch(left, right, lid)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        pkw = _params(W, H, D, **SMALL)
        o = run_oracle(f, pkw)
        assert (valid[i].cpu().numpy() == o["valid"]).all()
        assert np.abs(disp[i].cpu().numpy() - o["disp"]).max() <= SUB_TOL


def test_paper_scale_batch_launch_configuration(bench_frames):
    """The benchmark's launch configuration at 1242 x 375, D = 128: 128 frames
    per step, timed as one 128-frame call on one stream and as two contexts of
    64 frames on two streams.  The 128-frame call: first and last frame
    against the oracle, sampled frames against single-frame runs; the two
    streams' outputs equal it bit for bit, twice in a row."""
    frames = bench_frames
    B = len(frames)
    p = sldf.default_params(batch=B)
    ctx = sldf.Context(p)
    left = sldf.device_images(np.stack([f["left"] for f in frames]))
    right = sldf.device_images(np.stack([f["right"] for f in frames]))
    lid = torch.stack([sldf.quantize_lidar(torch.from_numpy(f["lidar"]).cuda(), 128)
                       for f in frames])
    print("case kitti one 128-frame call", flush=True)
    disp, valid = ctx.run_batch(left, right, lid)
    torch.cuda.synchronize()
    disp, valid = disp.cpu().numpy(), valid.cpu().numpy()
    del ctx
    pkw = _params(1242, 375, 128)
    for i in (0, B - 1):
        print(f"case kitti batch frame {i}", flush=True)
        o = run_oracle(frames[i], pkw)
        assert (valid[i] == o["valid"]).all()
        assert np.abs(disp[i] - o["disp"]).max() <= SUB_TOL
    for i in (1, 40, 64, 100, B - 2):
        g = run_gpu(frames[i], pkw, taps=False)
        assert (g["valid"] == valid[i]).all() and (g["disp"] == disp[i]).all(), i
    print("case kitti 2 streams x 64 frames", flush=True)
    n = B // 2
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    ctxs = [sldf.Context(sldf.default_params(batch=n)) for _ in range(2)]
    outs = [c.new_outputs(n) for c in ctxs]
    torch.cuda.synchronize()
    for rep in range(2):
        for i, st in enumerate((main, side)):
            sl = slice(i * n, (i + 1) * n)
            ctxs[i].run_batch(left[sl], right[sl], lid[sl], outs[i][0], outs[i][1], stream=st)
        torch.cuda.synchronize()
        for i in range(2):
            sl = slice(i * n, (i + 1) * n)
            assert (outs[i][1].cpu().numpy() == valid[sl]).all(), (rep, i)
            assert (outs[i][0].cpu().numpy() == disp[sl]).all(), (rep, i)


def test_deterministic_repeat():
    f = synth.small_frame(9)
    pkw = _params(f["W"], f["H"], f["D"], **SMALL)
    a, b = run_gpu(f, pkw), run_gpu(f, pkw)
    for k in ("disp", "valid", "S", "dstar", "dright", "dsub"):
        assert (a[k] == b[k]).all()


def test_run_rejects_misaligned_pitch():
    p = sldf.default_params(width=64, height=32, max_disp=64, **SMALL)
    ctx = sldf.Context(p)
    img = torch.zeros((32, 72), dtype=torch.uint8, device="cuda")[:, :64]   # pitch 72
    lid = torch.full((32, 64), -1, dtype=torch.int16, device="cuda")
    with pytest.raises(sldf.SldfError) as ei:
        ctx.run(img, img, lid)
    assert ei.value.status == sldf.EALIGN


# The other workload shapes at full size, one frame each, every tap compared:
# the 640 x 480 robustness frames at D = 64 and 128, the indoor variant
# (640 x 480, D = 256, disparities 40-250, 1 % uniform LiDAR sample) and the
# 1920 x 1080, D = 256 serving frame (long lines, 256-wide disparity vectors).
WORKLOADS = {
    "640x480_D64": lambda: synth.make_frame(synth.robust_spec(W=640, H=480, D=64, density=0.05),
                                            synth.CONFIG_IDS["robust"], 640064),
    "640x480_D128": lambda: synth.make_frame(synth.robust_spec(W=640, H=480, D=128,
                                                               density=0.02, lines=32),
                                             synth.CONFIG_IDS["robust"], 640128),
    "indoor_640x480_D256": lambda: synth.make_frame(synth.INDOOR, synth.CONFIG_IDS["robust"],
                                                    640256),
    "1920x1080_D256": lambda: synth.make_frame(synth.serving_spec(4),
                                               synth.CONFIG_IDS["serving"], 4),
}


_WORKLOAD_ORACLE = {}


def _workload_case(name):
    # one oracle run per workload, shared by both schedules' tests (the
    # 1920 x 1080 x 256 oracle takes about a minute on one core)
    if name not in _WORKLOAD_ORACLE:
        f = WORKLOADS[name]()
        H, W = f["left"].shape
        pkw = _params(W, H, int(f["D"]))
        _WORKLOAD_ORACLE.clear()
        _WORKLOAD_ORACLE[name] = (f, pkw, run_oracle(f, pkw))
    return _WORKLOAD_ORACLE[name]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_workload_shapes(name, schedule):
    f, pkw, o = _workload_case(name)
    print(f"case workload {name} schedule={schedule}", flush=True)
    assert_parity(run_gpu(f, dict(pkw, schedule=schedule)), o, pkw)


def _cost_path_taps(f, pkw, dirs):
    """Run with the C' and L_r taps; return the GPU volumes and the oracle's
    (from the oracle's own census codes and prior map)."""
    p = sldf.default_params(**pkw)
    W, H, D = p.width, p.height, p.max_disp
    op = _oracle_params(p.as_dict() | pkw)
    o = run_oracle(f, pkw)
    n = oracle.census_bits(op.cw, op.ch, op.census_kind)
    prior = o["prior"]
    cost = oracle.joint_cost(o["census_l"], o["census_r"], prior, D, n, 0, op.a, op.b, op.q1,
                             op.q2, op.blend_mode, op.prior_cost, op.huber_k)
    ctx = sldf.Context(p)
    left = sldf.device_image(f["left"])
    right = sldf.device_image(f["right"])
    lid_q = sldf.quantize_lidar(torch.from_numpy(np.ascontiguousarray(f["lidar"])).cuda(), D)
    results = []
    for k in dirs:
        tc = torch.empty((H, W, D), dtype=torch.int16, device="cuda")
        tl = torch.empty((H, W, D), dtype=torch.int16, device="cuda")
        ctx.set_taps(cost=tc, path_cost=tl, path_dir=k)
        ctx.run(left, right, lid_q)
        torch.cuda.synchronize()
        dx, dy = oracle.direction(k)
        exp_l = oracle.path(cost, dx, dy, op.b * op.p1, op.b * op.p2)
        results.append((k, tc.cpu().numpy().view(np.uint16), tl.cpu().numpy().view(np.uint16),
                        exp_l))
    ctx.close()
    return cost, results


@pytest.mark.parametrize("extra", [dict(), dict(census_kind=1), dict(prior_cost=2, huber_k=2),
                                   dict(blend_mode=1, schedule=3)])
def test_cost_and_single_path_taps_small(extra):
    """C'(p, d) (Eq. 4) and L_r(p, d) (Eq. 2) of each of the eight
    directions, bit-exact against the oracle."""
    f = synth.small_frame(1)
    pkw = _params(f["W"], f["H"], f["D"], **SMALL)
    pkw.update(extra)
    print(f"case cost/path taps small {extra}", flush=True)
    cost, res = _cost_path_taps(f, pkw, range(8))
    for k, gc, gl, el in res:
        assert (gc.astype(np.int64) == cost).all(), f"C' mismatch at {np.argwhere(gc != cost)[:5]}"
        bad = gl.astype(np.int64) != el
        assert not bad.any(), f"L_r dir {k} mismatch at {np.argwhere(bad)[:5]}"


@pytest.mark.parametrize("W,H,D", [(1242, 375, 128), (301, 40, 256), (97, 31, 64)])
def test_cost_and_single_path_taps_shapes(W, H, D):
    if W == 1242:
        f = synth.kitti_frame(2)
    else:
        f = synth.make_frame(synth.robust_spec(W=W, H=H, D=D, density=0.05, lines=16), 3, W + H)
    pkw = _params(W, H, D)
    dirs = [0, 5] if W == 1242 else [1, 2, 7]
    print(f"case cost/path taps {W}x{H} D={D} dirs={dirs}", flush=True)
    cost, res = _cost_path_taps(f, pkw, dirs)
    for k, gc, gl, el in res:
        assert (gc.astype(np.int64) == cost).all(), "C' mismatch"
        assert (gl.astype(np.int64) == el).all(), f"L_r dir {k} mismatch"


def test_path_tap_direction_out_of_range_is_rejected():
    p = sldf.default_params(width=64, height=16, max_disp=64)
    ctx = sldf.Context(p)
    t = torch.empty((16, 64, 64), dtype=torch.int16, device="cuda")
    for bad in (-1, 8):
        with pytest.raises(sldf.SldfError):
            ctx.set_taps(path_cost=t, path_dir=bad)
    ctx.set_taps(path_cost=t, path_dir=7)
    ctx.close()
