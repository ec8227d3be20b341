"""Pins for the CPU oracle: each test fixes a part of the oracle against
something other than the oracle itself -- hand-derived worked examples,
exhaustive minimisation, exact rational arithmetic, synthetic ground truth
and special cases that reduce to a textbook result.  CPU only."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2504_05148_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _popcount_np(a):
    a = np.ascontiguousarray(a, np.uint32)
    return np.unpackbits(a.view(np.uint8).reshape(a.shape + (4,)), axis=-1).sum(-1)


# ---------------------------------------------------------------- census --
def _ramp(name, W, H):
    yy, xx = np.mgrid[0:H, 0:W]
    return {"x_up": 2 * xx + 10, "x_down": 250 - 2 * xx, "y_up": 2 * yy + 10,
            "y_down": 250 - 2 * yy, "const": np.full((H, W), 77)}[name].astype(np.uint8)


def test_census_worked_examples():
    """Sec. IV-A census (CS-CT): hand-derived codes on ramps."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "census_ramps.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 10
    W, H = 40, 30
    for name, cw, ch, code in rows:
        cw, ch, code = int(cw), int(ch), int(code)
        c = oracle.census(_ramp(name, W, H), cw, ch)
        rx, ry = (cw - 1) // 2, (ch - 1) // 2
        inner = c[ry:H - ry, rx:W - rx]
        assert (inner == code).all(), (name, cw, ch, np.unique(inner))
        border = np.ones((H, W), bool)
        border[ry:H - ry, rx:W - rx] = False
        assert (c[border] == 0).all()


def test_census_bit_count():
    assert oracle.census_bits(5, 5) == 12 and oracle.census_bits(9, 7) == 31


def test_hamming_zero_at_true_shift():
    """Right view = left view shifted by d0: H(p, d0) = 0 wherever both census
    windows are inside the image (Sec. IV-A cost, matching pixel x - d)."""
    d0, W, H = 9, 80, 24
    left, right = synth.fronto_single_plane(W, H, d0, seed=3)
    cl, cr = oracle.census(left, 9, 7), oracle.census(right, 9, 7)
    cost = oracle.joint_cost(cl, cr, None, 32, 31, 0, 0, 1, 5, 160)  # a=0,b=1 -> H
    x0 = d0 + 4
    assert (cost[3:H - 3, x0:W - 4, d0] == 0).all()
    # every other disparity costs something on random dots in the interior
    others = np.delete(cost[3:H - 3, x0 + 32:W - 4, :], d0, axis=-1)
    assert (others > 0).mean() > 0.99
    # independent popcount for the raw Hamming volume
    for d in (0, 5, 17):
        ref = _popcount_np(cl[:, d:] ^ cr[:, :W - d])
        assert (cost[:, d:, d] == ref).all()
        assert (cost[:, :d, d] == 31).all()   # matching pixel outside: n


# ------------------------------------------------------------------- DDC --
def test_ddc_invariants():
    """Eq. 4: DDC is 0 at the prior, Q1 at +-1, Q2 beyond; no prior -> stereo
    cost only; alpha = 0 -> plain census cost."""
    rng = np.random.default_rng(0)
    W, H, D, n = 50, 12, 32, 12
    cl = rng.integers(0, 1 << 12, size=(H, W)).astype(np.uint32)
    cr = rng.integers(0, 1 << 12, size=(H, W)).astype(np.uint32)
    prior = rng.integers(-1, D, size=(H, W)).astype(np.int16)
    hv = oracle.joint_cost(cl, cr, None, D, n, 0, 0, 1, 5, 160)
    a, b, q1, q2 = 7, 10, 5, 160
    c = oracle.joint_cost(cl, cr, prior, D, n, 0, a, b, q1, q2, blend_mode=0)
    dd = np.arange(D)[None, None, :] - prior[:, :, None].astype(int)
    has = (prior >= 0)[:, :, None]
    ddc = c - (b - a) * hv
    assert (ddc[(dd == 0) & has] == 0).all()
    assert (ddc[(np.abs(dd) == 1) & has] == a * q1).all()
    assert (ddc[(np.abs(dd) > 1) & has] == a * q2).all()
    assert (ddc[~np.broadcast_to(has, ddc.shape)] == 0).all()
    c2 = oracle.joint_cost(cl, cr, prior, D, n, 0, a, b, q1, q2, blend_mode=1)
    nop = ~np.broadcast_to(has, c2.shape)
    assert (c2[nop] == b * hv[nop]).all()
    assert (c2[~nop] == c[~nop]).all()
    c0 = oracle.joint_cost(cl, cr, prior, D, n, 0, 0, b, q1, q2)
    assert (c0 == b * hv).all()


def test_alternative_prior_terms():
    """The LiDAR cost terms DDC is compared with (quadratic, Huber; capped at
    Q2), checked against what their definitions imply: a parabola has
    constant second differences; Huber equals the parabola up to k and then
    continues with the parabola's slope at k; Huber lies below the parabola;
    a cap of Q1 reduces both to the DDC with Q1 = Q2."""
    q1, big, D = 3, 10 ** 6, 256
    quad = [oracle.prior_penalty(t, q1, big, 1) for t in range(D)]
    assert quad[0] == 0
    assert all(quad[t + 1] - 2 * quad[t] + quad[t - 1] == 2 * q1 for t in range(1, D - 1))
    # Huber with k beyond the disparity range has no linear part
    assert [oracle.prior_penalty(t, q1, big, 2, D) for t in range(D)] == quad
    for k in (1, 3, 8):
        hub = [oracle.prior_penalty(t, q1, big, 2, k) for t in range(D)]
        assert hub[:k + 1] == quad[:k + 1]
        # straight tail whose slope, 2 q1 k, is the parabola's derivative at k
        assert all(hub[t + 1] - hub[t] == 2 * q1 * k for t in range(k, D - 1))
        assert all(0 <= h <= qd for h, qd in zip(hub, quad))
    for mode in (1, 2):
        assert [oracle.prior_penalty(t, 7, 7, mode, 2) for t in range(D)] == \
            [oracle.prior_penalty(t, 7, 7, 0) for t in range(D)]
    capped = [oracle.prior_penalty(t, 5, 160, 1) for t in range(D)]
    assert max(capped) == 160 and all(b >= a for a, b in zip(capped, capped[1:]))
    assert capped[:6] == [0, 5, 20, 45, 80, 125]
    # in the joint cost, mode 0 is the DDC of Eq. 4 unchanged
    rng = np.random.default_rng(4)
    W, H, Dd, n = 30, 6, 32, 12
    cl = rng.integers(0, 1 << 12, size=(H, W)).astype(np.uint32)
    cr = rng.integers(0, 1 << 12, size=(H, W)).astype(np.uint32)
    prior = rng.integers(-1, Dd, size=(H, W)).astype(np.int16)
    c0 = oracle.joint_cost(cl, cr, prior, Dd, n, 0, 7, 10, 5, 160)
    c1 = oracle.joint_cost(cl, cr, prior, Dd, n, 0, 7, 10, 5, 160, prior_cost=0, huber_k=4)
    assert (c0 == c1).all()
    # with alpha = 1 the cost is the prior term alone: its minimum over d sits
    # at the prior in every mode
    for mode in (0, 1, 2):
        c = oracle.joint_cost(cl, cr, prior, Dd, n, 0, 10, 10, 5, 160, prior_cost=mode,
                              huber_k=2)
        has = prior >= 0
        assert (c.argmin(axis=2)[has] == prior[has]).all()


# -------------------------------------------------------- path recurrence --
def _line_pixels(W, H, dx, dy):
    """All maximal lines of direction (dx, dy), each in traversal order."""
    lines = []
    for y in range(H):
        for x in range(W):
            px, py = x - dx, y - dy
            if 0 <= px < W and 0 <= py < H:
                continue  # not a start
            line, cx, cy = [], x, y
            while 0 <= cx < W and 0 <= cy < H:
                line.append((cx, cy))
                cx += dx
                cy += dy
            lines.append(line)
    return lines


def _pen(d1, d2, P1, P2):
    diff = abs(d1 - d2)
    return 0 if diff == 0 else (P1 if diff == 1 else P2)


@pytest.mark.parametrize("dir_idx", range(8))
def test_path_matches_exhaustive_minimisation(dir_idx):
    """Eq. 2 against Eq. 1 restricted to one line: the unnormalised path cost
    Lt(p_k, d) is the minimum of sum C + sum penalties over every disparity
    sequence on p_0..p_k ending in d, and the normalised recurrence equals
    Lt(p_k, d) - min_i Lt(p_{k-1}, i)."""
    dx, dy = oracle.direction(dir_idx)
    rng = np.random.default_rng(100 + dir_idx)
    for trial in range(12):
        W, H = int(rng.integers(2, 6)), int(rng.integers(2, 5))
        D = int(rng.integers(2, 5))
        P1 = int(rng.integers(0, 8))
        P2 = int(rng.integers(P1, 25))
        cost = rng.integers(0, 30, size=(H, W, D)).astype(np.int32)
        L = oracle.path(cost, dx, dy, P1, P2)
        for line in _line_pixels(W, H, dx, dy):
            n = len(line)
            Lt = np.full((n, D), 1 << 30)
            for seq in itertools.product(range(D), repeat=n):
                e = 0
                for k in range(n):
                    x, y = line[k]
                    e += int(cost[y, x, seq[k]])
                    if k:
                        e += _pen(seq[k - 1], seq[k], P1, P2)
                    Lt[k, seq[k]] = min(Lt[k, seq[k]], e)
            for k, (x, y) in enumerate(line):
                expect = Lt[k] - (Lt[k - 1].min() if k else 0)
                assert (L[y, x] == expect).all(), (dir_idx, trial, k)


def test_path_p2_bound():
    """C'(p,d) <= L_r(p,d) <= C'(p,d) + P2 for every direction."""
    rng = np.random.default_rng(7)
    cost = rng.integers(0, 1300, size=(9, 17, 24)).astype(np.int32)
    for i in range(8):
        dx, dy = oracle.direction(i)
        L = oracle.path(cost, dx, dy, 100, 1200)
        assert (L >= cost).all() and (L <= cost + 1200).all()


def test_zero_penalties_reduce_to_local_wta():
    """P1 = P2 = 0: L_r = C, S = |R| C, d* = local WTA of the cost."""
    rng = np.random.default_rng(8)
    cost = rng.integers(0, 90, size=(7, 11, 16)).astype(np.int32)
    for npaths in (4, 8):
        S = oracle.aggregate(cost, npaths, 0, 0)
        assert (S == npaths * cost).all()
        dstar, _ = oracle.wta(S, 0)
        assert (dstar == cost.argmin(-1)).all()   # argmin returns the first


def test_aggregate_is_sum_of_directions():
    """S is the sum of the per-direction path costs over the path set: 4
    paths = horizontal and vertical, 8 adds the diagonals."""
    rng = np.random.default_rng(9)
    cost = rng.integers(0, 200, size=(6, 9, 10)).astype(np.int32)
    dirs = [oracle.direction(i) for i in range(8)]
    assert set(dirs[:4]) == {(1, 0), (-1, 0), (0, 1), (0, -1)}
    assert set(dirs[4:]) == {(1, 1), (-1, 1), (1, -1), (-1, -1)}
    for npaths in (4, 8):
        S = oracle.aggregate(cost, npaths, 10, 120)
        ref = sum(oracle.path(cost, dx, dy, 10, 120) for dx, dy in dirs[:npaths])
        assert (S == ref).all()


# ------------------------------------------------------- WTA + subpixel --
def test_wta_ties_to_smallest_disparity():
    S = np.array([[[5, 3, 3, 9], [2, 2, 2, 2], [9, 8, 7, 7]]], np.int32)
    dstar, dsub = oracle.wta(S, 1)
    assert dstar.tolist() == [[1, 0, 2]]


def _exact_float32_ok(val32, exact: Fraction):
    """val32 is the float32 nearest to exact (within half an ulp)."""
    v = Fraction(float(val32))
    ulp = Fraction(float(np.spacing(np.float32(abs(float(val32)) or 1e-30))))
    return abs(v - exact) <= ulp / 2


def test_subpixel_against_exact_rationals():
    """Parabola through S(d*-1), S(d*), S(d*+1): offset (A - C) / (2 (A - 2B + C)),
    |offset| <= 1/2, zero for symmetric neighbours, none at the range ends."""
    rng = np.random.default_rng(11)
    D = 16
    S = rng.integers(0, 20000, size=(40, 50, D)).astype(np.int32)
    dstar, dsub = oracle.wta(S, 1)
    for y in range(40):
        for x in range(50):
            d = int(dstar[y, x])
            s = S[y, x]
            if d in (0, D - 1):
                assert dsub[y, x] == np.float32(d)
                continue
            A, B, C = int(s[d - 1]), int(s[d]), int(s[d + 1])
            den = A - 2 * B + C
            assert den > 0
            delta_exact = Fraction(A - C, 2 * den)
            assert abs(delta_exact) <= Fraction(1, 2)
            delta32 = np.float32(dsub[y, x]) - np.float32(d)
            # one rounding for the division, one for the add
            assert abs(Fraction(float(dsub[y, x])) - (d + delta_exact)) <= Fraction(1, 2 ** 18)
            assert _exact_float32_ok(np.float32(float(dsub[y, x])),
                                     Fraction(float(np.float32(d) + np.float32(
                                         float(delta_exact)))))
    sym = np.array([[[9, 4, 1, 4, 9]]], np.int32)
    _, dsub = oracle.wta(sym, 1)
    assert dsub[0, 0] == np.float32(2.0)
    _, dsub = oracle.wta(sym, 0)
    assert dsub[0, 0] == np.float32(2.0)


def test_subpixel_division_rounding():
    """The offset is the correctly rounded float32 quotient of two integers."""
    S = np.zeros((1, 1, 3), np.int32)
    for A, B, C in [(10, 3, 4), (7, 0, 1), (1000, 1, 998), (4, 1, 2), (19303, 0, 5)]:
        S[0, 0] = (A, B, C)
        _, dsub = oracle.wta(S, 1)
        exact = Fraction(A - C, 2 * (A - 2 * B + C))
        q = np.float32(float(dsub[0, 0])) - np.float32(1.0)
        assert _exact_float32_ok(q, exact) or abs(Fraction(float(q)) - exact) < Fraction(1, 2 ** 23)


# ----------------------------------------------------- end-to-end recovery --
def _params(W, H, D, **kw):
    base = dict(W=W, H=H, D=D, cw=5, ch=5, num_paths=4, semidense=0, check_mode=0)
    base.update(kw)
    return oracle.OracleParams(**base)


@pytest.mark.parametrize("d0,cw,ch,npaths", [(7, 5, 5, 4), (23, 9, 7, 8), (40, 5, 5, 8)])
def test_single_plane_exact_recovery(d0, cw, ch, npaths):
    """A fronto-parallel random-dot plane at integer disparity d0: d* = d0 on
    every interior pixel (left view) and d' = d0 (right view)."""
    W, H, D = 160, 40, 64
    left, right = synth.fronto_single_plane(W, H, d0, seed=d0)
    lid = np.full((H, W), -1, np.int16)
    t = oracle.run(_params(W, H, D, cw=cw, ch=ch, num_paths=npaths, check_mode=3),
                   left, right, lid, taps=True)
    rx, ry = (cw - 1) // 2, (ch - 1) // 2
    assert (t["dstar"][ry:H - ry, d0 + rx + 2:W - rx] == d0).all()
    assert (t["dright"][ry:H - ry, rx:W - rx - d0 - 2] == d0).all()
    # consistency: every interior pixel passes the stereo check
    assert t["valid"][ry:H - ry, d0 + rx + 2:W - rx].all()


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_multiplane_recovery_small_workload(idx):
    """320x96 fronto-parallel planes with integer disparities.  With exact
    LiDAR values (no noise) the full SDSGM recovers GT on >= 99 % of the
    non-occluded pixels away from discontinuities and the left border; plain
    census SGM (alpha = 0, no LiDAR) on >= 95 % (its P2 smooths small
    planes)."""
    from scipy.ndimage import binary_dilation
    f = synth.small_frame(idx)
    W, H, D = f["W"], f["H"], f["D"]
    gt = f["gt"].astype(int)
    exact = np.where(np.isfinite(f["lidar"]), f["gt"], np.nan).astype(np.float32)
    jump = np.zeros((H, W), bool)
    jump[:, 1:] |= gt[:, 1:] != gt[:, :-1]
    jump[:, :-1] |= gt[:, 1:] != gt[:, :-1]
    jump[1:, :] |= gt[1:, :] != gt[:-1, :]
    jump[:-1, :] |= gt[1:, :] != gt[:-1, :]
    near = binary_dilation(jump | f["occ"], iterations=4)
    m = ~f["occ"] & ~near
    m[:, :D] = False
    m[:2, :] = m[-2:, :] = False
    assert m.sum() > 5000
    t = oracle.run(_params(W, H, D, semidense=1), f["left"], f["right"],
                   oracle.quantize_lidar(exact, D), taps=True)
    assert (t["dstar"][m] == gt[m]).mean() >= 0.99
    t = oracle.run(_params(W, H, D, a=0), f["left"], f["right"],
                   np.full((H, W), -1, np.int16), taps=True)
    assert (t["dstar"][m] == gt[m]).mean() >= 0.95


def test_aggregate_bound_full_pipeline():
    """|R| C' <= S <= |R| (C' + P2') on a real frame (uint16 bound)."""
    f = synth.small_frame(1)
    W, H, D = f["W"], f["H"], f["D"]
    lid = oracle.quantize_lidar(f["lidar"], D)
    P = _params(W, H, D, semidense=1)
    t = oracle.run(P, f["left"], f["right"], lid, taps=True)
    cost = oracle.joint_cost(t["census_l"], t["census_r"], t["prior"], D, 12, 0,
                             P.a, P.b, P.q1, P.q2)
    S = t["S"]
    assert (S >= 4 * cost).all() and (S <= 4 * (cost + P.b * P.p2)).all()
    assert S.max() < 65536


# ---------------------------------------------------------- semidensify --
def test_semidense_special_cases():
    """Eq. 5: rs = 0 or Ts = 0 leave the sparse map unchanged; an empty map
    stays empty."""
    f = synth.small_frame(2)
    D = f["D"]
    cl, cr = oracle.census(f["left"], 5, 5), oracle.census(f["right"], 5, 5)
    lid = oracle.quantize_lidar(f["lidar"], D)
    assert (oracle.semidense(cl, cr, lid, 12, 2, 0) == lid).all()
    assert (oracle.semidense(cl, cr, lid, 12, 0, 6) == lid).all()
    empty = np.full_like(lid, -1)
    assert (oracle.semidense(cl, cr, empty, 12, 2, 6) == -1).all()
    # densifies: more valid pixels than the sparse map
    sd = oracle.semidense(cl, cr, lid, 12, 2, 6)
    assert (sd >= 0).sum() > 3 * (lid >= 0).sum()


def test_semidense_replaces_misprojection():
    """A wrong sparse value next to a correct one is replaced when the correct
    one matches (H < Ts), as the paper notes for occlusion misprojections."""
    d0, W, H = 11, 90, 30
    left, right = synth.fronto_single_plane(W, H, d0, seed=5)
    cl, cr = oracle.census(left, 5, 5), oracle.census(right, 5, 5)
    lid = np.full((H, W), -1, np.int16)
    lid[15, 50] = 30          # misprojected
    lid[15, 53] = d0          # correct, 3 px away
    sd = oracle.semidense(cl, cr, lid, 12, 2, 6)
    assert sd[15, 50] == d0
    # window reach: pixels within 6 of (53, 15) get d0, farther ones keep -1
    assert (sd[9:22, 47:60] == d0).all()
    assert sd[15, 40] == -1
    # raising nothing: with Ts = 0 the wrong value stays
    assert oracle.semidense(cl, cr, lid, 12, 0, 6)[15, 50] == 30


def test_semidense_strict_threshold_and_ties():
    """min H must be strictly below Ts; equal minima take the smallest d."""
    W, H = 60, 20
    flat = np.full((H, W), 100, np.uint8)
    c = oracle.census(flat, 5, 5)   # all zero codes: H = 0 wherever x - d >= 0
    lid = np.full((H, W), -1, np.int16)
    lid[10, 40] = 9
    lid[10, 42] = 5
    sd = oracle.semidense(c, c, lid, 12, 1, 6)
    assert sd[10, 41] == 5
    assert sd[10, 40] == 5            # replaces its own value: tie -> smaller d
    # H = 0 is not < Ts = 0
    assert oracle.semidense(c, c, lid, 12, 0, 6)[10, 41] == -1
    # near the left border x - d < 0 costs n = 12 -> not below Ts = 2
    lid2 = np.full((H, W), -1, np.int16)
    lid2[10, 3] = 9
    sd2 = oracle.semidense(c, c, lid2, 12, 2, 6)
    assert sd2[10, 4] == -1 and sd2[10, 9] == 9


def test_semidense_brute_force_numpy():
    """Independent vectorised restatement of Eq. 5 on a small frame."""
    f = synth.small_frame(3)
    D, H, W = f["D"], f["H"], f["W"]
    cl, cr = oracle.census(f["left"], 5, 5), oracle.census(f["right"], 5, 5)
    lid = oracle.quantize_lidar(f["lidar"], D)
    sd = oracle.semidense(cl, cr, lid, 12, 2, 6)
    # H volume from an independent popcount
    Hv = np.full((H, W, D), 12)
    for d in range(D):
        Hv[:, d:, d] = _popcount_np(cl[:, d:] ^ cr[:, :W - d])
    ys, xs = np.nonzero(lid >= 0)
    best_h = np.full((H, W), 1 << 20)
    best_d = np.full((H, W), -1)
    for y, x in zip(ys, xs):
        d = int(lid[y, x])
        y0, y1, x0, x1 = max(0, y - 6), min(H, y + 7), max(0, x - 6), min(W, x + 7)
        h = Hv[y0:y1, x0:x1, d]
        bh, bd = best_h[y0:y1, x0:x1], best_d[y0:y1, x0:x1]
        better = (h < bh) | ((h == bh) & (d < bd))
        bh[better] = h[better]
        bd[better] = d
    ref = np.where((best_d >= 0) & (best_h < 2), best_d, lid)
    assert (sd == ref).all()


# ------------------------------------------------------------------ check --
def test_check_reduces_to_lr_check_without_lidar():
    """No LiDAR: Eq. 6 is the classic left-right check |d* - d'(x - d*)| <= 1."""
    rng = np.random.default_rng(12)
    H, W = 20, 70
    dstar = rng.integers(0, 30, size=(H, W)).astype(np.int32)
    dright = (dstar + rng.integers(-3, 4, size=(H, W))).clip(0, 63).astype(np.int32)
    lid = np.full((H, W), -1, np.int16)
    dsub = dstar.astype(np.float32) + 0.25
    disp, valid = oracle.check(dstar, dright, lid, dsub, 2, 20, 3)
    for y in range(H):
        for x in range(W):
            d = dstar[y, x]
            ok = x - d >= 0 and abs(d - dright[y, x - d]) <= 1
            assert valid[y, x] == ok
            assert disp[y, x] == (dsub[y, x] if ok else -1.0)


def test_check_lidar_window_special_case():
    """rc = 0, Tc = 0: the LiDAR test passes iff the sparse value at p equals d*."""
    rng = np.random.default_rng(13)
    H, W = 15, 40
    dstar = rng.integers(0, 8, size=(H, W)).astype(np.int32)
    lid = rng.integers(-1, 8, size=(H, W)).astype(np.int16)
    _, valid = oracle.check(dstar, None, lid, None, 0, 0, 2)
    assert (valid == (lid == dstar)).all()


def test_check_brute_force_numpy():
    rng = np.random.default_rng(14)
    H, W = 50, 80
    dstar = rng.integers(0, 40, size=(H, W)).astype(np.int32)
    dright = rng.integers(0, 40, size=(H, W)).astype(np.int32)
    lid = np.where(rng.random((H, W)) < 0.02, rng.integers(0, 40, size=(H, W)), -1).astype(np.int16)
    for mode in range(4):
        _, valid = oracle.check(dstar, dright, lid, None, 2, 5, mode)
        for y in range(0, H, 3):
            for x in range(0, W, 3):
                d = int(dstar[y, x])
                st = x - d >= 0 and abs(d - int(dright[y, x - d])) <= 1
                win = lid[max(0, y - 5):y + 6, max(0, x - 5):x + 6].astype(int)
                li = bool(((win >= 0) & (np.abs(win - d) <= 2)).any())
                exp = [True, st, li, st or li][mode]
                assert valid[y, x] == exp


# ----------------------------------------------------------------- ingest --
def test_lidar_quantisation():
    vals = np.array([[np.nan, -0.3, 0.4, 2.5, 3.5, 62.5, 63.49, 63.5, 100.0]], np.float32)
    q = oracle.quantize_lidar(vals, 64)
    assert q.tolist() == [[-1, -1, 0, 2, 4, 62, 63, -1, -1]]


def test_tab2_defaults():
    rows = dict(l.split() for l in open(os.path.join(GOLDEN, "tab2_params.txt"))
                if l.strip() and not l.startswith("#"))
    P = oracle.OracleParams()
    assert (P.ts, P.rs, P.p1, P.p2, P.q1, P.q2, P.tc, P.rc) == tuple(
        int(rows[k]) for k in ("Ts", "rs", "P1", "P2", "Q1", "Q2", "Tc", "rc"))
    assert Fraction(P.a, P.b) == Fraction(rows["alpha"])


# ------------------------------------------------- LiDAR residual, features --
def test_lidar_residual_matches_check_and_special_cases():
    """rho <= Tc reproduces the LiDAR half of Eq. 6 (pinned above by brute
    force); rc = 0 gives |d* - D-bar_p| at the pixel itself; no LiDAR gives
    65535."""
    rng = np.random.default_rng(21)
    H, W, D = 40, 70, 64
    dstar = rng.integers(0, D, size=(H, W)).astype(np.int32)
    lid = np.where(rng.random((H, W)) < 0.03, rng.integers(0, D, size=(H, W)), -1).astype(np.int16)
    for rc in (0, 3, 9):
        rho = oracle.lidar_residual(dstar, lid, D, rc)
        for tc in (0, 1, 2, 5):
            _, valid = oracle.check(dstar, None, lid, None, tc, rc, 2)
            assert ((rho <= tc) == (valid == 1)).all()
    rho0 = oracle.lidar_residual(dstar, lid, D, 0)
    has = lid >= 0
    assert (rho0[has] == np.abs(dstar[has] - lid[has])).all()
    assert (rho0[~has] == 65535).all()
    assert (oracle.lidar_residual(dstar, np.full_like(lid, -1), D, 20) == 65535).all()


def test_surrogate_features_worked_example():
    """A parabolic cost curve S(d) = (d - 5)^2 + 100 (D = 16): d* = 5,
    S(d*) = 100, second minimum over |d - 5| >= 2 is S(3) = S(7) = 104,
    curvature S(4) - 2 S(5) + S(6) = 2."""
    D = 16
    S = np.array([[[(d - 5) ** 2 + 100 for d in range(D)]]], np.int32)
    dstar = np.array([[5]], np.int32)
    rho = np.array([[7]], np.uint16)
    f = oracle.surrogate_features(S, dstar, rho, 8, 1200)
    sS = np.float32(1) / np.float32(8 * 1200)
    exp = [np.float32(100) * sS, np.float32(104) * sS, np.float32(2) * sS,
           np.float32(5) * (np.float32(1) / np.float32(D)), np.float32(7) / np.float32(32),
           1.0]    # pixel x = 0 with d* = 5 has no matching pixel: margin 16 / 16
    assert f[0, 0].tolist() == [float(v) for v in exp]
    # range ends: no curvature; residual clipped at 32
    dstar = np.array([[0]], np.int32)
    f = oracle.surrogate_features(S, dstar, np.array([[65535]], np.uint16), 8, 1200)
    assert f[0, 0, 2] == 0.0 and f[0, 0, 4] == 1.0
    assert f[0, 0, 1] == np.float32(min((d - 5) ** 2 + 100 for d in range(2, D))) * sS


def _occlusion_brute(dstar):
    """The occlusion margin written out per pixel with Python loops."""
    H, W = dstar.shape
    out = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            q = x - int(dstar[y, x])
            right = [x2 - int(dstar[y, x2]) for x2 in range(x + 1, W)]
            if q < 0:
                v = 16
            elif not right:
                v = -16
            else:
                v = max(-16, min(16, q - min(right)))
            out[y, x] = v / 16
    return out


def test_occlusion_margin_worked_example_and_brute_force():
    """Sixth surrogate input: d* = [0, 0, 3, 0, 0] matches the right-image
    pixels q = [0, 1, -1, 3, 4]: pixel 2 has no match (16); pixels 0 and 1
    are overtaken by pixel 2's match q = -1 (margins 1 and 2); pixel 3 is
    visible (q = 3 < 4: -1); the last pixel has nothing to its right (-16)."""
    dstar = np.array([[0, 0, 3, 0, 0]], np.int32)
    S = np.zeros((1, 5, 8), np.int32)
    rho = np.zeros((1, 5), np.uint16)
    f = oracle.surrogate_features(S, dstar, rho, 8, 1200)[..., 5]
    assert (f[0] * 16).tolist() == [1.0, 2.0, 16.0, -1.0, -16.0]
    # a fronto-parallel row: every pixel visible by exactly one pixel, except
    # the first c pixels (no match) and the last one
    c = 3
    f = oracle.surrogate_features(np.zeros((1, 12, 8), np.int32),
                                  np.full((1, 12), c, np.int32), np.zeros((1, 12), np.uint16),
                                  8, 1200)[..., 5]
    assert (f[0] * 16).tolist() == [16.0] * c + [-1.0] * (12 - c - 1) + [-16.0]
    rng = np.random.default_rng(11)
    for W in (1, 2, 7, 40):
        dstar = rng.integers(0, 24, size=(3, W)).astype(np.int32)
        f = oracle.surrogate_features(np.zeros((3, W, 24), np.int32), dstar,
                                      np.zeros((3, W), np.uint16), 8, 1200)[..., 5]
        assert (f == _occlusion_brute(dstar)).all(), W


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, -2.5, 3.0e-5], np.float32)
    b = oracle.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1.0); 1 + 1.5 * 2^-8
    # rounds up to 1 + 2^-7
    assert oracle.bf16_to_f32(b).tolist()[:4] == [1.0, 1.0, 1.0078125, -2.5]
    # against PyTorch's float32 -> bfloat16 conversion (round to nearest even) on
    # random values of every magnitude and on exact ties
    import torch
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000)).astype(np.float32)
    ties = ((rng.integers(0, 1 << 16, 2000).astype(np.uint32) << 16) | 0x8000).view(np.float32)
    x = np.concatenate([x, ties[np.isfinite(ties)]])
    ref_bits = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert (oracle.bf16_round(x) == ref_bits).all()


def test_full_census_worked_examples():
    """Full census (census_kind 1), 5 x 5: every offset but the centre in
    raster order, bit k = [I(p + o_k) < I(p)], LSB first.  Horizontal ramp
    I = x: the bits of the offsets with dx < 0, i.e. the first two of each
    window row (bits 0, 1 | 5, 6 | 10, 11 | 14, 15 | 19, 20: the centre row
    has four offsets).  Vertical ramp I = y: the two rows above, bits 0..9.
    Decreasing ramp I = -x: dx > 0, bits 3, 4 | 8, 9 | 12, 13 | 17, 18 |
    22, 23.  Constant image: 0.  Border pixels: 0."""
    H, W = 9, 12
    ramp_x = np.tile(np.arange(W, dtype=np.uint8) * 7, (H, 1))
    ramp_y = np.tile((np.arange(H, dtype=np.uint8) * 9)[:, None], (1, W))
    ramp_nx = np.tile((200 - np.arange(W) * 7).astype(np.uint8), (H, 1))
    bits = lambda ks: sum(1 << k for k in ks)
    cases = [(ramp_x, bits([0, 1, 5, 6, 10, 11, 14, 15, 19, 20])),
             (ramp_y, bits(range(10))),
             (ramp_nx, bits([3, 4, 8, 9, 12, 13, 17, 18, 22, 23])),
             (np.full((H, W), 77, np.uint8), 0)]
    for img, code in cases:
        c = oracle.census(img, 5, 5, kind=1)
        assert (c[2:H - 2, 2:W - 2] == code).all()
        inner = np.zeros((H, W), bool)
        inner[2:H - 2, 2:W - 2] = True
        assert (c[~inner] == 0).all()
    assert oracle.census_bits(5, 5, 1) == 24 and oracle.census_bits(9, 7, 1) == 62


def test_full_census_brute_force():
    """Against a numpy brute force written from the definition."""
    rng = np.random.default_rng(21)
    img = rng.integers(0, 256, size=(14, 19)).astype(np.uint8)
    for cw, ch in ((3, 3), (5, 5), (3, 9), (7, 3)):
        c = oracle.census(img, cw, ch, kind=1)
        rx, ry = cw // 2, ch // 2
        H, W = img.shape
        for y in range(H):
            for x in range(W):
                exp = 0
                if rx <= x < W - rx and ry <= y < H - ry:
                    k = 0
                    for dy in range(-ry, ry + 1):
                        for dx in range(-rx, rx + 1):
                            if dx == 0 and dy == 0:
                                continue
                            if img[y + dy, x + dx] < img[y, x]:
                                exp |= 1 << k
                            k += 1
                assert c[y, x] == exp, (cw, ch, y, x)
