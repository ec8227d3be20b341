"""Ablations of the method on seeded synthetic frames, in the shapes of the
paper's studies, scored with coverage / covered error / total error
(evaluate.py) against the synthetic ground truth:

- prior maps (Tab. IV): the quantised sparse LiDAR map D-bar and the
  semidense map D-hat (Sec. IV-B) taken as disparity maps;
- consistency checks (Tab. V): stereo only, camera-LiDAR only and the
  stereo-LiDAR check of Eq. 6 (plus no check) on the SDSGM output;
- method variants (Tab. I): SGM with census only (alpha = 0), DSGM, SDSGM,
  and SDSGM with the learned check;
- LiDAR cost terms (Tab. III): the DDC against the quadratic (LiDAR-SGM)
  and Huber terms, on the sparse and on the semidense prior;
- robustness: image noise, contrast loss and rain-like streaks, and LiDAR
  density / scan-line sweeps (the CARLA rain and density studies), with
  T_s = 9 as the paper uses for rain;
- parameter sweeps: any sldf_params field (T_s, r_s, Q1, Q2, T_c, r_c, ...)
  through --sweep name=v1,v2,...

Every run goes through the C ABI on the GPU; the scores are computed on the
host.  The synthetic frames stand in for the paper's datasets (KITTI 141,
CARLA, Middlebury), which are not used: the numbers follow the shape of the
paper's tables, not their values.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np
import torch

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2504_05148_amd import evaluate, sldf, synth  # noqa: E402

CHECK_MODES = {"none": 0, "stereo": 1, "camera-lidar": 2, "stereo-lidar": 3}
VARIANTS = {
    "SGM (census, alpha 0)": dict(alpha_num=0, semidense=0),
    "DSGM": dict(semidense=0),
    "SDSGM": dict(semidense=1),
}


def _frames(n: int, spec=None, config_id: int | None = None, first: int = 0):
    spec = synth.KITTI if spec is None else spec
    cid = synth.CONFIG_IDS["kitti"] if config_id is None else config_id
    return [synth.make_frame(spec, cid, first + i) for i in range(n)]


def run_frames(frames, surrogate=None, taps_prior: bool = False, **params):
    """Run the method on each frame (one frame per call).  Returns a list of
    (disp, valid) numpy pairs, and with taps_prior the D-bar / D-hat maps."""
    f0 = frames[0]
    H, W = f0["left"].shape
    D = params.pop("max_disp", f0.get("D", 128))
    p = sldf.default_params(width=W, height=H, max_disp=D, batch=1, **params)
    ctx = sldf.Context(p)
    if surrogate is not None:
        ctx.set_surrogate(*surrogate)
    prior = torch.empty((H, W), dtype=torch.int16, device="cuda") if taps_prior else None
    if taps_prior:
        ctx.set_taps(prior=prior)
    out, priors = [], []
    for f in frames:
        left = sldf.device_image(f["left"])
        right = sldf.device_image(f["right"])
        lid = sldf.quantize_lidar(torch.from_numpy(np.ascontiguousarray(f["lidar"])).cuda(), D)
        disp, valid = ctx.run(left, right, lid)
        torch.cuda.synchronize()
        out.append((disp.cpu().numpy(), valid.cpu().numpy()))
        if taps_prior:
            priors.append((lid.cpu().numpy(), prior.cpu().numpy()))
    ctx.close()
    return (out, priors) if taps_prior else out


def _score_map(m: np.ndarray):
    """A prior map (int16, -1 invalid) as a (disp, valid) pair."""
    return m.astype(np.float32), m >= 0


def prior_maps(frames) -> dict:
    """Tab. IV shape: the sparse and the semidense prior as disparity maps."""
    _, priors = run_frames(frames, taps_prior=True, semidense=1)
    sparse = evaluate.evaluate_frames([_score_map(a) for a, _ in priors], frames)
    semi = evaluate.evaluate_frames([_score_map(b) for _, b in priors], frames)
    return {"input sparse map": sparse, "semidense map": semi}


def check_modes(frames) -> dict:
    """Tab. V shape: the consistency checks on the SDSGM output."""
    return {name: evaluate.evaluate_frames(run_frames(frames, check_mode=m), frames)
            for name, m in CHECK_MODES.items()}


def variants(frames, surrogate=None) -> dict:
    """Tab. I variants (plus census-only SGM and the learned check)."""
    out = {name: evaluate.evaluate_frames(run_frames(frames, **kw), frames)
           for name, kw in VARIANTS.items()}
    if surrogate is not None:
        out["SDSGM, learned check"] = evaluate.evaluate_frames(
            run_frames(frames, surrogate=surrogate, semidense=1, check_impl=1), frames)
    return out


# the LiDAR cost terms DDC is compared with (Sec. IV-A, Tab. III), on the
# raw sparse map (as LiDAR-SGM uses it) and on the semidense one; the cap
# q2 = 980 is the largest the 16-bit bound admits at Tab. II otherwise
PRIOR_TERMS = {
    "DDC (Eq. 4)": dict(prior_cost=0),
    "quadratic": dict(prior_cost=1, q2=980),
    "Huber, k = 2": dict(prior_cost=2, huber_k=2, q2=980),
}


def prior_terms(frames) -> dict:
    """Tab. III shape: DDC against the quadratic and Huber LiDAR terms."""
    out = {}
    for semi, tag in ((0, "D-bar"), (1, "D-hat")):
        for name, kw in PRIOR_TERMS.items():
            out[f"{name}, {tag}"] = evaluate.evaluate_frames(
                run_frames(frames, semidense=semi, **kw), frames)
    return out


# robustness workloads (the shapes of the paper's CARLA rain and density
# studies): degraded images and LiDAR density / scan-line sweeps
DEGRADATIONS = ("none", "noise", "contrast", "rain")
DENSITIES = ((0.005, 16), (0.02, 32), (0.05, 64), (0.10, 128))
ROBUST_METHODS = {
    "SGM (census, stereo check)": dict(alpha_num=0, semidense=0, check_mode=1),
    "DSGM": dict(semidense=0),
    "SDSGM": dict(semidense=1),
    "SDSGM, Ts = 9": dict(semidense=1, ts=9),
}


def robustness(n: int, first: int = 9000, degradations=DEGRADATIONS) -> dict:
    """Methods under image degradations (noise, contrast, rain streaks)."""
    rows = {}
    for deg in degradations:
        spec = synth.robust_spec(degrade=deg)
        frames = [synth.make_frame(spec, synth.CONFIG_IDS["robust"], first + i) for i in range(n)]
        for name, kw in ROBUST_METHODS.items():
            rows[f"{deg}: {name}"] = evaluate.evaluate_frames(run_frames(frames, **kw), frames)
    return rows


def density_sweep(n: int, first: int = 9500, densities=DENSITIES) -> dict:
    """DSGM and SDSGM against the LiDAR density and scan-line count."""
    rows = {}
    for dens, lines in densities:
        spec = synth.robust_spec(density=dens, lines=lines)
        frames = [synth.make_frame(spec, synth.CONFIG_IDS["robust"], first + i) for i in range(n)]
        for name in ("DSGM", "SDSGM"):
            rows[f"{100 * dens:g} %, {lines} lines: {name}"] = evaluate.evaluate_frames(
                run_frames(frames, **ROBUST_METHODS[name]), frames)
    return rows


def sweep(frames, name: str, values) -> dict:
    return {f"{name}={v}": evaluate.evaluate_frames(run_frames(frames, **{name: v}), frames)
            for v in values}


def table(title: str, rows: dict) -> str:
    lines = [f"### {title}", "", "| | Coverage [%] | Covered error [%] | Total error [%] |",
             "|---|---|---|---|"]
    for k, e in rows.items():
        lines.append(f"| {k} | {100 * e['coverage']:.1f} | {100 * e['covered_error']:.2f} | "
                     f"{100 * e['total_error']:.2f} |")
    return "\n".join(lines)


def _load_surrogate():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                        "surrogate_synthetic_1242x375.npz")
    if not os.path.exists(path):
        return None
    from paper_2504_05148_amd.train_surrogate import load_weights
    w, b, _ = load_weights(path)
    return w, b


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--first", type=int, default=5000, help="first frame seed index")
    ap.add_argument("--sweep", action="append", default=[], metavar="NAME=V1,V2,...")
    ap.add_argument("--robust-frames", type=int, default=0,
                    help="frames per cell of the robustness and density tables (0 = skip)")
    args = ap.parse_args(argv)
    frames = _frames(args.frames, first=args.first)
    print(f"{args.frames} synthetic 1242x375 D=128 frames (seeds {args.first}..)\n")
    print(table("Prior maps (Tab. IV shape)", prior_maps(frames)), "\n")
    print(table("Consistency checks on SDSGM (Tab. V shape)", check_modes(frames)), "\n")
    print(table("Method variants (Tab. I)", variants(frames, _load_surrogate())), "\n")
    print(table("LiDAR cost terms (Tab. III shape)", prior_terms(frames)), "\n")
    if args.robust_frames > 0:
        print(table("Robustness to image degradations", robustness(args.robust_frames)), "\n")
        print(table("LiDAR density and scan lines", density_sweep(args.robust_frames)), "\n")
    for s in args.sweep:
        name, vals = s.split("=")
        print(table(f"Sweep of {name}", sweep(frames, name, [int(v) for v in vals.split(",")])),
              "\n")


if __name__ == "__main__":
    main()
