"""CPU oracle for the stereo-LiDAR SGM method: test infrastructure only.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module.  The product path (the HIP library and its
binding) never does.  It shares no code with the GPU library, and the GPU
library shares none with it.

The arithmetic lives in ``sldf_oracle.c`` (plain single-threaded C, int32),
which cites for each function the passage of the paper it follows:
Sec. III (Eq. 2 path recurrence, Eq. 3 winner-takes-all, parabola subpixel),
Sec. IV-A (Eq. 4 joint cost with DDC), Sec. IV-B (Eq. 5 semidensification)
and Sec. IV-C (Eq. 6 consistency check).  This module only marshals numpy
arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sldf_oracle.c")
_LIB = os.path.join(_HERE, "libsldf_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no vectorisation pragmas)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


u8, u32, i16, i32, f32 = (ctypes.c_uint8, ctypes.c_uint32, ctypes.c_int16,
                          ctypes.c_int32, ctypes.c_float)


@dataclass
class OracleParams:
    """Method parameters.  Defaults are Tab. II (paper units) with the
    paper-scale frame shape; alpha = a / b."""
    W: int = 1242
    H: int = 375
    D: int = 128
    cw: int = 9
    ch: int = 7
    num_paths: int = 8
    p1: int = 10
    p2: int = 120
    q1: int = 5
    q2: int = 160
    a: int = 7
    b: int = 10
    blend_mode: int = 0
    semidense: int = 1
    ts: int = 2
    rs: int = 6
    tc: int = 2
    rc: int = 20
    check_mode: int = 3
    subpixel: int = 1
    prior_cost: int = 0
    huber_k: int = 1
    census_kind: int = 0


class _CParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int) for k in (
        "W", "H", "D", "cw", "ch", "num_paths", "p1", "p2", "q1", "q2", "a", "b",
        "blend_mode", "semidense", "ts", "rs", "tc", "rc", "check_mode",
        "subpixel", "prior_cost", "huber_k", "census_kind")]


def _chk(rc):
    if rc != 0:
        raise RuntimeError(f"oracle returned status {rc}")


def census_bits(cw: int, ch: int, kind: int = 0) -> int:
    return (cw * ch - 1) // 2 if kind == 0 else cw * ch - 1


def quantize_lidar(lidar_f32: np.ndarray, D: int) -> np.ndarray:
    a = np.ascontiguousarray(lidar_f32, dtype=np.float32)
    H, W = a.shape
    out = np.empty((H, W), np.int16)
    _chk(_load().orc_quantize_lidar(_p(a, f32), W, H, D, _p(out, i16)))
    return out


def census(img: np.ndarray, cw: int, ch: int, kind: int = 0) -> np.ndarray:
    """kind 0: centre-symmetric census, 1: full census (sldf_oracle.c)."""
    a = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = a.shape
    out = np.empty((H, W), np.uint32)
    _chk(_load().orc_census_kind(_p(a, u8), W, H, W, cw, ch, kind, _p(out, u32)))
    return out


def semidense(cL, cR, lidar, n, ts, rs) -> np.ndarray:
    cL = np.ascontiguousarray(cL, np.uint32)
    cR = np.ascontiguousarray(cR, np.uint32)
    li = np.ascontiguousarray(lidar, np.int16)
    H, W = li.shape
    out = np.empty((H, W), np.int16)
    _chk(_load().orc_semidense(_p(cL, u32), _p(cR, u32), _p(li, i16), W, H, n, ts,
                               rs, _p(out, i16)))
    return out


def prior_penalty(adiff, q1, q2, prior_cost=0, huber_k=1) -> int:
    """Penalty q of a disparity |d - prior| = adiff away from the prior."""
    return int(_load().orc_prior_penalty(int(adiff), int(q1), int(q2), int(prior_cost),
                                         int(huber_k)))


def joint_cost(cL, cR, prior, D, n, view, a, b, q1, q2, blend_mode=0, prior_cost=0,
               huber_k=1):
    """C'(p,d) as int32 [H, W, D]; prior None means no prior anywhere."""
    cL = np.ascontiguousarray(cL, np.uint32)
    cR = np.ascontiguousarray(cR, np.uint32)
    H, W = cL.shape
    out = np.empty((H, W, D), np.int32)
    pr = None
    if prior is not None:
        pr = np.ascontiguousarray(prior, np.int16)
    _chk(_load().orc_joint_cost(_p(cL, u32), _p(cR, u32),
                                _p(pr, i16) if pr is not None else None, W, H, D, n,
                                view, a, b, q1, q2, blend_mode, prior_cost, huber_k,
                                _p(out, i32)))
    return out


def path(cost, dx, dy, P1, P2):
    """L_r for one direction r = (dx, dy) over a cost volume [H, W, D]."""
    c = np.ascontiguousarray(cost, np.int32)
    H, W, D = c.shape
    out = np.empty_like(c)
    _chk(_load().orc_path(_p(c, i32), W, H, D, dx, dy, P1, P2, _p(out, i32)))
    return out


def direction(i: int):
    dx, dy = ctypes.c_int(), ctypes.c_int()
    _chk(_load().orc_direction(i, ctypes.byref(dx), ctypes.byref(dy)))
    return dx.value, dy.value


def aggregate(cost, num_paths, P1, P2):
    c = np.ascontiguousarray(cost, np.int32)
    H, W, D = c.shape
    out = np.empty_like(c)
    _chk(_load().orc_aggregate(_p(c, i32), W, H, D, num_paths, P1, P2,
                               _p(out, i32)))
    return out


def wta(S, subpixel=1):
    s = np.ascontiguousarray(S, np.int32)
    H, W, D = s.shape
    dstar = np.empty((H, W), np.int32)
    dsub = np.empty((H, W), np.float32)
    _chk(_load().orc_wta(_p(s, i32), W, H, D, subpixel, _p(dstar, i32),
                         _p(dsub, f32)))
    return dstar, dsub


def check(dstar, dright, lidar, dsub, tc, rc, mode):
    ds = np.ascontiguousarray(dstar, np.int32)
    H, W = ds.shape
    dr = None if dright is None else np.ascontiguousarray(dright, np.int32)
    li = np.ascontiguousarray(lidar, np.int16)
    sub = None if dsub is None else np.ascontiguousarray(dsub, np.float32)
    disp = np.empty((H, W), np.float32)
    valid = np.empty((H, W), np.uint8)
    _chk(_load().orc_check(_p(ds, i32), _p(dr, i32) if dr is not None else None,
                           _p(li, i16), _p(sub, f32) if sub is not None else None,
                           W, H, tc, rc, mode, _p(disp, f32), _p(valid, u8)))
    return disp, valid


def lidar_residual(dstar, lidar, D, rc):
    """rho = min |d* - v| over valid sparse values in the (2 rc + 1)^2 window;
    65535 where there is none (uint16 [H, W])."""
    ds = np.ascontiguousarray(dstar, np.int32)
    li = np.ascontiguousarray(lidar, np.int16)
    H, W = ds.shape
    out = np.empty((H, W), np.uint16)
    _chk(_load().orc_lidar_residual(_p(ds, i32), _p(li, i16), W, H, D, rc,
                                    _p(out, ctypes.c_uint16)))
    return out


def surrogate_features(S, dstar, rho, num_paths, P2s):
    """float32 [H, W, 6] surrogate inputs (see sldf_oracle.c)."""
    s = np.ascontiguousarray(S, np.int32)
    H, W, D = s.shape
    ds = np.ascontiguousarray(dstar, np.int32)
    r = np.ascontiguousarray(rho, np.uint16)
    out = np.empty((H, W, 6), np.float32)
    _chk(_load().orc_surrogate_features(_p(s, i32), _p(ds, i32), _p(r, ctypes.c_uint16),
                                        W, H, D, num_paths, P2s, _p(out, f32)))
    return out


def bf16_round(x):
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_to_f32(b):
    return (np.ascontiguousarray(b, np.uint16).astype(np.uint32) << 16).view(np.float32)


def run(params: OracleParams, left, right, lidar_q, taps: bool = False):
    """Whole pipeline for one frame.  lidar_q is the int16 sparse map (-1 =
    invalid).  Returns (disp, valid) or, with taps, a dict of every
    intermediate."""
    P = params
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    li = np.ascontiguousarray(lidar_q, np.int16)
    H, W = left.shape
    assert (H, W) == (P.H, P.W) and right.shape == left.shape and li.shape == left.shape
    cp = _CParams(**asdict(P))
    disp = np.empty((H, W), np.float32)
    valid = np.empty((H, W), np.uint8)
    if not taps:
        _chk(_load().orc_run(ctypes.byref(cp), _p(left, u8), _p(right, u8), W,
                             _p(li, i16), _p(disp, f32), _p(valid, u8), None, None,
                             None, None, None, None, None))
        return disp, valid
    t = dict(census_l=np.empty((H, W), np.uint32), census_r=np.empty((H, W), np.uint32),
             prior=np.empty((H, W), np.int16), S=np.empty((H, W, P.D), np.int32),
             dstar=np.empty((H, W), np.int32), dright=np.empty((H, W), np.int32),
             dsub=np.empty((H, W), np.float32))
    _chk(_load().orc_run(ctypes.byref(cp), _p(left, u8), _p(right, u8), W,
                         _p(li, i16), _p(disp, f32), _p(valid, u8),
                         _p(t["census_l"], u32), _p(t["census_r"], u32),
                         _p(t["prior"], i16), _p(t["S"], i32), _p(t["dstar"], i32),
                         _p(t["dright"], i32), _p(t["dsub"], f32)))
    t["disp"] = disp
    t["valid"] = valid
    return t
