"""Thin ctypes binding of libsldf.so (include/sldf.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory (tensors) and the HIP stream
(``torch.cuda.current_stream().cuda_stream``).  If the library is missing,
every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsldf.so")

OK, EINVAL, ESHAPE, EALIGN, EOVERFLOW, ENOMEM, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7

_PARAM_FIELDS = ("struct_size", "width", "height", "max_disp", "census_w", "census_h",
                 "num_paths", "p1", "p2", "q1", "q2", "alpha_num", "alpha_den",
                 "blend_mode", "semidense", "ts", "rs", "tc", "rc", "check_mode",
                 "check_impl", "subpixel", "batch")


_PARAM_FLOATS = ("fallback_tau", "uncertain_margin")
_PARAM_TAIL = ("prior_cost", "huber_k", "schedule", "census_kind")   # int32 after the floats


class Params(ctypes.Structure):
    _fields_ = ([(k, ctypes.c_int32) for k in _PARAM_FIELDS] +
                [(k, ctypes.c_float) for k in _PARAM_FLOATS] +
                [(k, ctypes.c_int32) for k in _PARAM_TAIL])

    def as_dict(self):
        return {k: getattr(self, k) for k in _PARAM_FIELDS + _PARAM_FLOATS + _PARAM_TAIL}


class Taps(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in
                ("census_l", "census_r", "prior", "cost_sum", "dstar", "dright", "dsub",
                 "rho", "features", "sweep_errors", "cost", "path_cost")] + [
                ("path_dir", ctypes.c_int32)]


class SldfError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None
_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t


def lib():
    """Load libsldf.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsldf.so not built ({LIB_PATH}); run "
                               "paper_2504_05148_amd.build.build() first")
        L = ctypes.CDLL(LIB_PATH)
        L.sldf_status_string.restype = ctypes.c_char_p
        L.sldf_status_string.argtypes = [ctypes.c_int]
        L.sldf_abi_version.restype = _i32
        L.sldf_params_default.argtypes = [ctypes.POINTER(Params)]
        L.sldf_params_default.restype = None
        L.sldf_workspace_size.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(_sz)]
        L.sldf_create.argtypes = [ctypes.POINTER(Params), _vp, _sz, ctypes.POINTER(_vp)]
        L.sldf_destroy.argtypes = [_vp]
        L.sldf_set_taps.argtypes = [_vp, ctypes.POINTER(Taps)]
        L.sldf_run.argtypes = [_vp, _vp, _vp, _i32, _vp, _i32, _vp, _vp, _i32, _vp]
        L.sldf_run_batch.argtypes = [_vp, _i32, _vp, _vp, _i32, _i64, _vp, _i32, _i64,
                                     _vp, _vp, _i32, _i64, _vp]
        L.sldf_lidar_quantize.argtypes = [_vp, _i32, _i32, _i32, _i32, _vp, _i32, _vp]
        L.sldf_run_noalloc.argtypes = [ctypes.POINTER(Params), _vp, _vp, _i32, _vp, _i32, _vp,
                                       _vp, _i32, _vp]
        L.sldf_timing_enable.argtypes = [_vp, _i32]
        L.sldf_timing_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
        L.sldf_fallback_read.argtypes = [_vp, ctypes.POINTER(_i32), _i32, ctypes.POINTER(_i32)]
        L.sldf_fallback_read.restype = ctypes.c_int
        L.sldf_surrogate_num_weights.restype = _i32
        L.sldf_surrogate_num_biases.restype = _i32
        L.sldf_surrogate_set_weights.argtypes = [_vp, _vp, _vp]
        L.sldf_surrogate_load.argtypes = [_vp, _vp, _sz]
        L.sldf_surrogate_blob_bytes.restype = _sz
        L.sldf_surrogate_forward.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                                             _vp, _vp]
        L.sldf_surrogate_train_workspace_size.argtypes = [_i32, _i32, _i32,
                                                          ctypes.POINTER(_sz)]
        L.sldf_surrogate_sync_weights.argtypes = [_vp, _vp, _vp, _vp]
        _f = ctypes.c_float
        L.sldf_surrogate_train_step.argtypes = [_vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp,
                                                _vp, _vp, _vp, _vp, _f, _f, _f, _f, _i32,
                                                _i32, _vp, _sz, _vp, _vp, _vp]
        for f in ("sldf_workspace_size", "sldf_create", "sldf_destroy", "sldf_set_taps",
                  "sldf_run", "sldf_run_batch", "sldf_lidar_quantize", "sldf_run_noalloc",
                  "sldf_timing_enable", "sldf_timing_read", "sldf_surrogate_set_weights",
                  "sldf_surrogate_forward", "sldf_surrogate_train_workspace_size",
                  "sldf_surrogate_sync_weights", "sldf_surrogate_load",
                  "sldf_surrogate_train_step"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().sldf_status_string(status).decode()


def _check(status: int, what: str):
    if status != OK:
        raise SldfError(status, what)


def default_params(**overrides) -> Params:
    p = Params()
    lib().sldf_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if k in _PARAM_FIELDS or k in _PARAM_TAIL:
            setattr(p, k, int(v))
        elif k in _PARAM_FLOATS:
            setattr(p, k, float(v))
        else:
            raise KeyError(k)
    return p


def workspace_size(p: Params) -> int:
    n = _sz()
    _check(lib().sldf_workspace_size(ctypes.byref(p), ctypes.byref(n)), "sldf_workspace_size")
    return int(n.value)


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(t: torch.Tensor) -> int:
    return int(t.data_ptr())


def device_image(img, device="cuda") -> torch.Tensor:
    """uint8 [H, W] -> device tensor [H, W] whose rows sit on a 16-byte
    pitch (a view into an [H, pitch] buffer)."""
    t = torch.as_tensor(img, dtype=torch.uint8)
    H, W = t.shape
    pitch = (W + 15) // 16 * 16
    buf = torch.zeros((H, pitch), dtype=torch.uint8, device=device)
    buf[:, :W].copy_(t.to(device))
    return buf[:, :W]


def device_images(imgs, device="cuda") -> torch.Tensor:
    """Stack of uint8 [F, H, W] on a 16-byte row pitch (a view)."""
    t = torch.as_tensor(imgs, dtype=torch.uint8)
    F, H, W = t.shape
    pitch = (W + 15) // 16 * 16
    buf = torch.zeros((F, H, pitch), dtype=torch.uint8, device=device)
    buf[:, :, :W].copy_(t.to(device))
    return buf[:, :, :W]


def quantize_lidar(lidar: torch.Tensor, max_disp: int, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """float32 [H, W] (NaN = no return) -> int16 D-bar on the device."""
    assert lidar.dtype == torch.float32 and lidar.is_cuda and lidar.dim() == 2
    assert lidar.stride(1) == 1
    H, W = lidar.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.int16, device=lidar.device)
    assert out.stride(1) == 1
    _check(lib().sldf_lidar_quantize(_ptr(lidar), W, H, lidar.stride(0), max_disp, _ptr(out),
                                     out.stride(0), _stream_handle(stream)),
           "sldf_lidar_quantize")
    return out


class Context:
    """One context per rig / shape: parameters plus a caller-owned device
    workspace of exactly ``workspace_size(params)`` bytes."""

    def __init__(self, params: Params, device=None):
        self.params = params
        self.device = torch.device(device if device is not None else "cuda")
        self.ws_bytes = workspace_size(params)
        # 256-byte aligned workspace (the caching allocator aligns to 512)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-_ptr(self.workspace)) % 256
        self._ws = self.workspace[off:off + self.ws_bytes]
        h = _vp()
        with torch.cuda.device(self.device):
            _check(lib().sldf_create(ctypes.byref(params), _ptr(self._ws), self.ws_bytes,
                                     ctypes.byref(h)), "sldf_create")
        self._h = h
        self._taps_keep = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sldf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_taps(self, **tensors):
        """Debug taps (frame 0): census_l, census_r, prior, cost_sum, dstar,
        dright, dsub, rho, features, sweep_errors, cost, path_cost -> device
        tensors of the documented dtypes; path_dir (int) picks the direction
        of path_cost."""
        t = Taps()
        for k, v in tensors.items():
            if k == "path_dir":
                t.path_dir = int(v)
            else:
                setattr(t, k, _ptr(v) if v is not None else None)
        self._taps_keep = dict(tensors)
        _check(lib().sldf_set_taps(self._h, ctypes.byref(t)), "sldf_set_taps")

    STAGES = ("census", "semidense", "sgm", "check", "fallback")

    def timing_enable(self, max_runs: int):
        _check(lib().sldf_timing_enable(self._h, int(max_runs)), "sldf_timing_enable")

    def set_surrogate(self, weights: torch.Tensor | None, biases: torch.Tensor | None):
        """Attach learned-check parameters (device tensors: int16/uint16
        bf16 bit patterns and float32); they are referenced, not copied."""
        self._sur_keep = (weights, biases)
        _check(lib().sldf_surrogate_set_weights(
            self._h, _ptr(weights) if weights is not None else None,
            _ptr(biases) if biases is not None else None), "sldf_surrogate_set_weights")

    def load_surrogate(self, blob: torch.Tensor):
        """Attach learned-check parameters from one device blob
        (surrogate_blob(weights, biases)); referenced, not copied."""
        self._sur_keep = (blob,)
        _check(lib().sldf_surrogate_load(self._h, _ptr(blob), blob.numel() * blob.element_size()),
               "sldf_surrogate_load")

    def fallback_read(self, n: int):
        """(per-frame uncertain-pixel counts of the last learned run, limit);
        synchronises with the device."""
        counts = (_i32 * n)()
        lim = _i32()
        _check(lib().sldf_fallback_read(self._h, counts, n, ctypes.byref(lim)),
               "sldf_fallback_read")
        return list(counts), int(lim.value)

    def timing_read(self):
        """{stage: (total_ms, launches)} since the last read (waits on events)."""
        ms = (ctypes.c_double * 5)()
        n = (ctypes.c_int64 * 5)()
        _check(lib().sldf_timing_read(self._h, ms, n), "sldf_timing_read")
        return {k: (ms[i], n[i]) for i, k in enumerate(self.STAGES)}

    def new_outputs(self, n_frames: int | None = None):
        W, H = self.params.width, self.params.height
        shape = (H, W) if n_frames is None else (n_frames, H, W)
        disp = torch.empty(shape, dtype=torch.float32, device=self.device)
        valid = torch.empty(shape, dtype=torch.uint8, device=self.device)
        return disp, valid

    def run(self, left, right, lidar, disp=None, valid=None, stream=None):
        """One frame: left/right uint8 [H, W] (16-byte row pitch), lidar int16
        [H, W]; returns (disp float32, valid uint8), enqueued on stream."""
        if disp is None or valid is None:
            disp, valid = self.new_outputs()
        for t in (left, right, lidar, disp, valid):
            assert t.is_cuda and t.stride(-1) == 1
        assert left.stride(0) == right.stride(0)
        assert disp.stride(0) == valid.stride(0)
        _check(lib().sldf_run(self._h, _ptr(left), _ptr(right), left.stride(0), _ptr(lidar),
                              lidar.stride(0), _ptr(disp), _ptr(valid), disp.stride(0),
                              _stream_handle(stream)), "sldf_run")
        return disp, valid

    def run_batch(self, left, right, lidar, disp=None, valid=None, stream=None):
        """n frames: left/right uint8 [F, H, W], lidar int16 [F, H, W]."""
        F = left.shape[0]
        if disp is None or valid is None:
            disp, valid = self.new_outputs(F)
        assert left.stride() == right.stride() and disp.stride() == valid.stride()
        _check(lib().sldf_run_batch(self._h, F, _ptr(left), _ptr(right), left.stride(1),
                                    left.stride(0), _ptr(lidar), lidar.stride(1),
                                    lidar.stride(0), _ptr(disp), _ptr(valid), disp.stride(1),
                                    disp.stride(0), _stream_handle(stream)),
               "sldf_run_batch")
        return disp, valid


def run_noalloc(params: Params, left, right, lidar, disp, valid, stream=None):
    """sldf_run_noalloc: one frame without a context or workspace (the
    library's static per-GPU scratch); outputs are caller-provided device
    tensors (disp float32 [H, W], valid uint8 [H, W])."""
    for t in (left, right, lidar, disp, valid):
        assert t.is_cuda and t.stride(-1) == 1
    assert left.stride(0) == right.stride(0) and disp.stride(0) == valid.stride(0)
    _check(lib().sldf_run_noalloc(ctypes.byref(params), _ptr(left), _ptr(right), left.stride(0),
                                  _ptr(lidar), lidar.stride(0), _ptr(disp), _ptr(valid),
                                  disp.stride(0), _stream_handle(stream)), "sldf_run_noalloc")
    return disp, valid


# ---------------------------------------------------------------- surrogate --
def surrogate_blob(weights: torch.Tensor, biases: torch.Tensor) -> torch.Tensor:
    """One device blob for sldf_surrogate_load: the bf16 weight bits, zero
    padding to 256 bytes, the float32 biases (byte copies, no arithmetic)."""
    n = int(lib().sldf_surrogate_blob_bytes())
    blob = torch.zeros(n, dtype=torch.uint8, device=weights.device)
    wb = weights.contiguous().view(torch.uint8).reshape(-1)
    bb = biases.contiguous().view(torch.uint8).reshape(-1)
    off = n - bb.numel()
    blob[:wb.numel()] = wb
    blob[off:] = bb
    return blob


def surrogate_sizes():
    return int(lib().sldf_surrogate_num_weights()), int(lib().sldf_surrogate_num_biases())


def surrogate_forward(x0: torch.Tensor, weights: torch.Tensor, biases: torch.Tensor,
                      stream=None):
    """x0 bf16-bits [F, H, W, 8] (int16) -> (logits [F, H, W] f32, (a1, a2, a3))."""
    F, H, W, C = x0.shape
    assert C == 8 and x0.is_contiguous()
    acts = [torch.empty((F, H, W, 32), dtype=torch.int16, device=x0.device) for _ in range(3)]
    z = torch.empty((F, H, W), dtype=torch.float32, device=x0.device)
    _check(lib().sldf_surrogate_forward(_ptr(x0), W, H, F, _ptr(weights), _ptr(biases),
                                        _ptr(acts[0]), _ptr(acts[1]), _ptr(acts[2]), _ptr(z),
                                        _stream_handle(stream)), "sldf_surrogate_forward")
    return z, acts


class SurrogateTrainer:
    """Adam training of the learned check through sldf_surrogate_train_step
    (fp32 master parameters, bf16 working weights)."""

    def __init__(self, W, H, F, master: torch.Tensor, device="cuda", lr=1e-3, betas=(0.9, 0.999),
                 eps=1e-8):
        nw, nb = surrogate_sizes()
        assert master.numel() == nw + nb and master.dtype == torch.float32
        self.W, self.H, self.F = W, H, F
        self.master = master.to(device).contiguous()
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.nw, self.nb = nw, nb
        self.weights = torch.empty(nw, dtype=torch.int16, device=device)
        self.biases = torch.empty(nb, dtype=torch.float32, device=device)
        self.sync_working()
        n = _sz()
        _check(lib().sldf_surrogate_train_workspace_size(W, H, F, ctypes.byref(n)),
               "sldf_surrogate_train_workspace_size")
        self.ws = torch.empty(int(n.value) + 256, dtype=torch.uint8, device=device)
        off = (-_ptr(self.ws)) % 256
        self._ws = self.ws[off:off + int(n.value)]
        self.ws_bytes = int(n.value)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.step_count = 0
        self.stats = torch.zeros(4, dtype=torch.float32, device=device)

    def sync_working(self, stream=None):
        """Working parameters (bf16 weights, fp32 biases) from the master copy,
        by the library (sldf_surrogate_sync_weights)."""
        _check(lib().sldf_surrogate_sync_weights(_ptr(self.master), _ptr(self.weights),
                                                 _ptr(self.biases), _stream_handle(stream)),
               "sldf_surrogate_sync_weights")

    def step(self, x0, labels, rho, tc, update=True, grads_out=None, stream=None):
        F = x0.shape[0]
        assert F <= self.F
        if update:
            self.step_count += 1
        _check(lib().sldf_surrogate_train_step(
            _ptr(x0), _ptr(labels), _ptr(rho), int(tc), self.W, self.H, F, _ptr(self.master),
            _ptr(self.m), _ptr(self.v), _ptr(self.weights), _ptr(self.biases), self.lr,
            self.betas[0], self.betas[1], self.eps, max(self.step_count, 1), int(update),
            _ptr(self._ws), self.ws_bytes, _ptr(grads_out) if grads_out is not None else None,
            _ptr(self.stats), _stream_handle(stream)), "sldf_surrogate_train_step")
        return self.stats
