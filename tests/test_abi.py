"""The C ABI library loads and exports every symbol include/sldf.h declares;
host-only entry points (defaults, validation, workspace plan) behave as
documented.  No GPU work is launched here."""
import ctypes
import os
import re

import pytest

from paper_2504_05148_amd import sldf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sldf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(sldf_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for n in ("sldf_create", "sldf_run", "sldf_run_batch", "sldf_workspace_size",
              "sldf_destroy", "sldf_set_taps", "sldf_lidar_quantize", "sldf_status_string",
              "sldf_params_default", "sldf_abi_version"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = sldf.lib()
    for n in _declared():
        assert hasattr(L, n), n


def test_params_default_is_tab2():
    p = sldf.default_params()
    assert p.struct_size == ctypes.sizeof(sldf.Params)
    assert (p.ts, p.rs, p.p1, p.p2, p.q1, p.q2, p.tc, p.rc) == (2, 6, 10, 120, 5, 160, 2, 20)
    assert (p.alpha_num, p.alpha_den) == (7, 10)
    assert (p.width, p.height, p.max_disp, p.census_w, p.census_h, p.num_paths) == (
        1242, 375, 128, 9, 7, 8)
    assert p.semidense == 1 and p.check_mode == 3 and p.subpixel == 1
    assert p.prior_cost == 0 and p.huber_k == 1            # DDC (Eq. 4)
    assert sldf.lib().sldf_abi_version() == 1


def test_workspace_size_plan():
    p = sldf.default_params()
    n1 = sldf.workspace_size(p)
    W, H, D = 1242, 375, 128
    px, cells = W * H, W * H * D
    census = 2 * (W + 2 * D) * H * 4            # padded census rows, both views
    # prior words (u32, one-pixel guard ring), d*, d' (i16), dsub (f32), S left +
    # right (u16), LiDAR row masks (D/32 words), rho (u16), cost features
    # (2 u32), surrogate inputs (8 bf16)
    # paired-direction checkpoints: every 8 pixels of each line, D u16 per
    # checkpoint, both views; the largest pair is the diagonal one
    segs = lambda n: (n + 7) // 8
    ck = max(H * segs(W), W * segs(H), (W + H - 1) * segs(min(W, H))) * D * 2 * 2
    pw = (W + 2) * (H + 2) * 4
    per_frame = (census + pw + px * (2 + 2 + 4) + 2 * cells * 2 + ck +
                 px * (D // 32 * 4 + 2 + 8 + 16))
    # once per context: a guard row before and after the census of each view,
    # the right view's prior words; the split schedule's second cost term
    # for one frame, both views
    fixed = 2 * 2 * (W + 2 * D) * 4 + pw
    split = lambda F: min(F, 1) * 2 * cells * 2
    # single-frame contexts with 8 paths: the second stream's cost term,
    # checkpoints and LiDAR window masks
    split3 = lambda F: (2 * cells * 2 + ck + px * (D // 32) * 4) if F == 1 else 0
    exact = per_frame + fixed + split(1) + split3(1)
    assert exact <= n1 < exact + 20 * 256
    p.batch = 4
    exact4 = 4 * per_frame + fixed + split(4) + split3(4)
    assert exact4 <= sldf.workspace_size(p) < exact4 + 20 * 256
    p = sldf.default_params(check_mode=2)      # no right-view pass: one S volume
    assert sldf.workspace_size(p) < n1 - cells
    # the paired schedule needs no second cost term
    p = sldf.default_params(schedule=1)
    n_paired = n1 - split(1) - split3(1)     # (each left-out segment also drops its padding)
    assert n_paired - 20 * 256 <= sldf.workspace_size(p) < n_paired + 20 * 256


@pytest.mark.parametrize("field,value,status", [
    ("struct_size", 4, sldf.EINVAL),
    ("width", 8, sldf.ESHAPE),
    ("height", 5000, sldf.ESHAPE),
    ("max_disp", 96, sldf.ESHAPE),
    ("census_w", 8, sldf.EINVAL),
    ("census_h", 17, sldf.EINVAL),
    ("num_paths", 2, sldf.EINVAL),
    ("q2", 4, sldf.EINVAL),            # Q1 <= Q2 (Sec. IV-A)
    ("alpha_num", 11, sldf.EINVAL),
    ("rs", 16, sldf.EINVAL),
    ("rc", 32, sldf.EINVAL),
    ("check_mode", 4, sldf.EINVAL),
    ("check_impl", 2, sldf.EINVAL),
    ("batch", 0, sldf.EINVAL),
    ("prior_cost", 3, sldf.EINVAL),
    ("schedule", 4, sldf.EINVAL),
    ("huber_k", 0, sldf.EINVAL),
    ("census_kind", 2, sldf.EINVAL),
    ("census_kind", 1, sldf.EINVAL),   # full census of the default 9 x 7 window: 62 bits
    ("p2", 2000, sldf.EOVERFLOW),       # 8 paths * (C' + P2') >= 65536
])
def test_validation(field, value, status):
    p = sldf.default_params(**{field: value})
    with pytest.raises(sldf.SldfError) as ei:
        sldf.workspace_size(p)
    assert ei.value.status == status


def test_cost_volume_offset_limit():
    # one frame's cost volume is addressed with 32-bit byte offsets
    assert sldf.workspace_size(sldf.default_params(width=4096, height=4096, max_disp=128,
                                                   batch=1)) > 0
    with pytest.raises(sldf.SldfError) as ei:
        sldf.workspace_size(sldf.default_params(width=4096, height=4096, max_disp=256))
    assert ei.value.status == sldf.ESHAPE


def test_learned_check_needs_full_check_mode():
    for mode in (0, 1, 2):
        with pytest.raises(sldf.SldfError) as ei:
            sldf.workspace_size(sldf.default_params(check_impl=1, check_mode=mode))
        assert ei.value.status == sldf.EINVAL
    with pytest.raises(sldf.SldfError):
        sldf.workspace_size(sldf.default_params(check_impl=1, fallback_tau=1.5))
    # learned check adds activations, logits and counters to the workspace
    assert sldf.workspace_size(sldf.default_params(check_impl=1)) > \
        sldf.workspace_size(sldf.default_params()) + 2 * 1242 * 375 * 64


def test_surrogate_sizes():
    assert sldf.surrogate_sizes() == (25344, 97)


def test_overflow_bound_is_tight():
    # C'max = 3*31 + 7*160 = 1213; 8 * (1213 + 10*P2) < 65536 <=> P2 <= 697
    assert sldf.workspace_size(sldf.default_params(p2=697)) > 0
    with pytest.raises(sldf.SldfError):
        sldf.workspace_size(sldf.default_params(p2=698))


def test_fp16_compare_bound_is_tight():
    # the recurrence compares its terms as fp16 bit patterns: C'max + 2 P2'
    # < 0x7c00 = 31744; with one path it binds before the sum bound:
    # 1213 + 20 P2 < 31744 <=> P2 <= 1526
    assert sldf.workspace_size(sldf.default_params(num_paths=1, p2=1526)) > 0
    with pytest.raises(sldf.SldfError) as ei:
        sldf.workspace_size(sldf.default_params(num_paths=1, p2=1527))
    assert ei.value.status == sldf.EOVERFLOW


def test_status_strings():
    for s in range(-7, 1):
        assert sldf.status_string(s)
    assert sldf.status_string(-99) == "unknown status"


def test_full_census_parameters():
    # 5 x 5 full census: 24 bits, valid; the bound uses the larger bit count
    assert sldf.workspace_size(sldf.default_params(census_kind=1, census_w=5, census_h=5)) > 0
    assert sldf.default_params().census_kind == 0


def test_surrogate_blob_size():
    """weights (bf16) padded to 256 bytes, then the float biases"""
    L = sldf.lib()
    nw, nb = L.sldf_surrogate_num_weights(), L.sldf_surrogate_num_biases()
    assert L.sldf_surrogate_blob_bytes() == (nw * 2 + 255) // 256 * 256 + nb * 4


def test_taps_struct_matches_header():
    """sldf_taps: twelve device pointers then the int32 direction of the
    single-path tap, in the header's order."""
    src = open(HEADER).read()
    body = src[:src.index("} sldf_taps;")].rsplit("typedef struct {", 1)[1]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(\w+);", body)
    assert fields == [f for f, _ in sldf.Taps._fields_]
    assert sldf.Taps.path_dir.offset == 12 * ctypes.sizeof(ctypes.c_void_p)
