"""Python binding of libkaze (ctypes; argument marshalling only).

Every function here has the name and arguments of the C entry point it
wraps (``include/kaze.h``).  Device buffers are passed as torch tensors (or
raw integer device addresses); streams default to torch's current stream.
All computation happens in the HIP library: if the library is missing the
import fails, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libkaze.so")

KAZE_OK = 0
KAZE_ERR_INVALID_ARG = -1
KAZE_ERR_WORKSPACE = -2
KAZE_ERR_HIP = -3
KAZE_ERR_UNSUPPORTED = -4
KAZE_G1 = 1
KAZE_G2 = 2

# Every symbol include/kaze.h declares.
EXPORTS = (
    "kaze_default_params", "kaze_num_levels", "kaze_schedule",
    "kaze_workspace_bytes", "kaze_build_scale_space", "kaze_conductivity",
    "kaze_aos_step", "kaze_detector_response", "kaze_find_extrema",
    "kaze_last_error", "kaze_profile_begin", "kaze_profile_end",
    "kaze_kernel_names", "kaze_copy_f32",
)


class KazeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class kaze_params(ctypes.Structure):
    _fields_ = [
        ("octaves", ctypes.c_int),
        ("sublevels", ctypes.c_int),
        ("sigma0", ctypes.c_double),
        ("sigma_cond", ctypes.c_double),
        ("diffusivity", ctypes.c_int),
        ("k_bins", ctypes.c_int),
        ("k_percentile", ctypes.c_double),
        ("k_override", ctypes.c_double),
        ("det_threshold", ctypes.c_double),
    ]


class kaze_keypoint(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int), ("y", ctypes.c_int), ("level", ctypes.c_int),
                ("response", ctypes.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libkaze.so is not built (%s); run `python -m paper_1706_06750_amd.build`"
            % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(kaze_params)
    vp, sz, i32, f64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    sig = {
        "kaze_default_params": (i32, [P]),
        "kaze_num_levels": (i32, [P]),
        "kaze_schedule": (i32, [P, vp, vp, vp, vp, vp]),
        "kaze_workspace_bytes": (sz, [i32, i32, P]),
        "kaze_build_scale_space": (i32, [vp, i32, i32, i32, P, vp, vp, vp, sz, vp]),
        "kaze_conductivity": (i32, [vp, i32, i32, P, f64, vp, vp]),
        "kaze_aos_step": (i32, [vp, vp, i32, i32, f64, vp, vp, sz, vp]),
        "kaze_detector_response": (i32, [vp, i32, i32, P, vp, vp]),
        "kaze_find_extrema": (i32, [vp, i32, i32, P, vp, i32, vp, vp]),
        "kaze_last_error": (ctypes.c_char_p, []),
        "kaze_profile_begin": (i32, [ctypes.c_char_p]),
        "kaze_profile_end": (i32, [ctypes.POINTER(i32), ctypes.POINTER(f64)]),
        "kaze_kernel_names": (ctypes.c_char_p, []),
        "kaze_copy_f32": (i32, [vp, vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(st):
    if st != KAZE_OK:
        raise KazeError(st, lib.kaze_last_error().decode())


def _ptr(x):
    """Device address of a tensor, an int, or None (NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def kaze_default_params(**overrides) -> kaze_params:
    p = kaze_params()
    _check(lib.kaze_default_params(ctypes.byref(p)))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def kaze_num_levels(p: kaze_params) -> int:
    n = lib.kaze_num_levels(ctypes.byref(p))
    if n < 0:
        _check(n)
    return n


def kaze_schedule(p: kaze_params):
    """Per-level dict with sigma, t, tau, sigma_norm and deriv_step."""
    n = kaze_num_levels(p)
    arr = [(ctypes.c_double * n)() for _ in range(4)]
    steps = (ctypes.c_int * n)()
    _check(lib.kaze_schedule(ctypes.byref(p), *[ctypes.cast(a, ctypes.c_void_p) for a in arr],
                             ctypes.cast(steps, ctypes.c_void_p)))
    return [dict(sigma=arr[0][i], t=arr[1][i], tau=arr[2][i], sigma_norm=arr[3][i],
                 deriv_step=steps[i]) for i in range(n)]


def kaze_workspace_bytes(W: int, H: int, p: kaze_params) -> int:
    return int(lib.kaze_workspace_bytes(W, H, ctypes.byref(p)))


def kaze_build_scale_space(img, W, H, ld_img, p, levels, k_out, ws, ws_bytes, stream=None):
    _check(lib.kaze_build_scale_space(_ptr(img), W, H, ld_img, ctypes.byref(p), _ptr(levels),
                                      _ptr(k_out), _ptr(ws), ws_bytes, _stream(stream)))


def kaze_conductivity(L, W, H, p, k, g, stream=None):
    _check(lib.kaze_conductivity(_ptr(L), W, H, ctypes.byref(p), float(k), _ptr(g),
                                 _stream(stream)))


def kaze_aos_step(L, g, W, H, tau, L_next, ws, ws_bytes, stream=None):
    _check(lib.kaze_aos_step(_ptr(L), _ptr(g), W, H, float(tau), _ptr(L_next), _ptr(ws),
                             ws_bytes, _stream(stream)))


def kaze_detector_response(levels, W, H, p, det, stream=None):
    _check(lib.kaze_detector_response(_ptr(levels), W, H, ctypes.byref(p), _ptr(det),
                                      _stream(stream)))


def kaze_find_extrema(det, W, H, p, kps, capacity, count, stream=None):
    _check(lib.kaze_find_extrema(_ptr(det), W, H, ctypes.byref(p), _ptr(kps), capacity,
                                 _ptr(count), _stream(stream)))


def kaze_copy_f32(src, dst, n, stream=None):
    _check(lib.kaze_copy_f32(_ptr(src), _ptr(dst), n, _stream(stream)))


def kaze_profile_begin(kernel_name: str):
    _check(lib.kaze_profile_begin(kernel_name.encode()))


def kaze_profile_end():
    n = ctypes.c_int(0)
    ms = ctypes.c_double(0.0)
    _check(lib.kaze_profile_end(ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def kaze_kernel_names():
    return lib.kaze_kernel_names().decode().split(",")


# ---------------------------------------------------------------------------
# Convenience wrapper: torch tensors in, torch tensors out.
# ---------------------------------------------------------------------------
class Kaze:
    """Device buffers (torch allocations) plus the three C calls for one
    image size.  ``run(img)`` enqueues scale space, detector response and
    extrema on the current stream and returns device tensors."""

    def __init__(self, W: int, H: int, params: kaze_params | None = None,
                 capacity: int = 1 << 16, device="cuda"):
        import torch
        self.W, self.H = int(W), int(H)
        self.p = params if params is not None else kaze_default_params()
        self.N = kaze_num_levels(self.p)
        self.capacity = int(capacity)
        self.ws_bytes = kaze_workspace_bytes(self.W, self.H, self.p)
        if self.ws_bytes == 0:
            _check(KAZE_ERR_INVALID_ARG)
        dev = torch.device(device)
        self.levels = torch.empty((self.N, self.H, self.W), dtype=torch.float32, device=dev)
        self.det = torch.empty_like(self.levels)
        self.k = torch.empty(1, dtype=torch.float32, device=dev)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.kps = torch.empty((max(self.capacity, 1), 4), dtype=torch.int32, device=dev)
        self.count = torch.empty(1, dtype=torch.int32, device=dev)

    def scale_space(self, img, stream=None):
        kaze_build_scale_space(img, self.W, self.H, img.stride(0), self.p, self.levels,
                               self.k, self.ws, self.ws_bytes, stream)

    def detector(self, stream=None):
        kaze_detector_response(self.levels, self.W, self.H, self.p, self.det, stream)

    def extrema(self, stream=None):
        kaze_find_extrema(self.det, self.W, self.H, self.p, self.kps, self.capacity,
                          self.count, stream)

    def run(self, img, stream=None):
        self.scale_space(img, stream)
        self.detector(stream)
        self.extrema(stream)

    def keypoints(self):
        """Host (n, 4) float64 array (level, y, x, response) sorted by
        (level, y, x); synchronises."""
        import numpy as np
        n = int(self.count.item())
        n = min(n, self.capacity)
        raw = self.kps[:n].cpu()
        xyl = raw[:, :3].numpy().astype(np.int64)
        resp = raw[:, 3].contiguous().view(dtype=__import__("torch").float32).numpy()
        out = np.stack([xyl[:, 2], xyl[:, 1], xyl[:, 0], resp.astype(np.float64)], axis=1) \
            if n else np.zeros((0, 4))
        if n:
            order = np.lexsort((out[:, 2], out[:, 1], out[:, 0]))
            out = out[order]
        return out
