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
KAZE_AOS = 0
KAZE_FED = 1
KAZE_WINDOW_3X3 = 0
KAZE_WINDOW_SIGMA = 1

# Every symbol include/kaze.h declares.
EXPORTS = (
    "kaze_default_params", "kaze_num_levels", "kaze_schedule",
    "kaze_workspace_bytes", "kaze_build_scale_space", "kaze_build_scale_space_noalloc",
    "kaze_conductivity",
    "kaze_aos_step", "kaze_detector_response", "kaze_find_extrema",
    "kaze_last_error", "kaze_profile_begin", "kaze_profile_end",
    "kaze_kernel_names", "kaze_copy_f32", "kaze_batch_workspace_bytes",
    "kaze_batch_create", "kaze_batch_run", "kaze_batch_destroy", "kaze_batch_autotune",
    "kaze_batch_properties", "kaze_fed_schedule", "kaze_fed_cycle", "kaze_refine_keypoints",
    "kaze_derivatives", "kaze_describe_keypoints", "kaze_aos_shape_info",
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
        ("scheme", ctypes.c_int),
        ("extrema_window", ctypes.c_int),
        ("substeps", ctypes.c_int),
    ]


class kaze_keypoint(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int), ("y", ctypes.c_int), ("level", ctypes.c_int),
                ("response", ctypes.c_float)]


class kaze_keypoint_refined(ctypes.Structure):
    _fields_ = [("x", ctypes.c_float), ("y", ctypes.c_float), ("level", ctypes.c_int),
                ("response", ctypes.c_float), ("edge_ratio", ctypes.c_float),
                ("kept", ctypes.c_int)]


class kaze_image_desc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("W", ctypes.c_int), ("H", ctypes.c_int),
                ("ld_img", ctypes.c_int), ("levels", ctypes.c_void_p), ("det", ctypes.c_void_p),
                ("k", ctypes.c_void_p), ("kps", ctypes.c_void_p), ("capacity", ctypes.c_int),
                ("count", ctypes.c_void_p)]


class kaze_batch_config(ctypes.Structure):
    _fields_ = [("aos_shape", ctypes.c_int)]




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
        "kaze_build_scale_space_noalloc": (i32, [vp, i32, i32, i32, P, vp, vp, vp]),
        "kaze_conductivity": (i32, [vp, i32, i32, P, f64, vp, vp]),
        "kaze_aos_step": (i32, [vp, vp, i32, i32, f64, vp, vp, sz, vp]),
        "kaze_fed_schedule": (i32, [f64, vp, i32]),
        "kaze_fed_cycle": (i32, [vp, vp, i32, i32, f64, vp, vp, sz, vp]),
        "kaze_detector_response": (i32, [vp, i32, i32, P, vp, vp]),
        "kaze_find_extrema": (i32, [vp, i32, i32, P, vp, i32, vp, vp]),
        "kaze_refine_keypoints": (i32, [vp, i32, i32, P, vp, vp, i32, f64, vp, vp]),
        "kaze_derivatives": (i32, [vp, i32, i32, P, vp, vp, vp]),
        "kaze_describe_keypoints": (i32, [vp, vp, i32, i32, P, vp, vp, i32, vp, vp, vp]),
        "kaze_last_error": (ctypes.c_char_p, []),
        "kaze_profile_begin": (i32, [ctypes.c_char_p]),
        "kaze_profile_end": (i32, [ctypes.POINTER(i32), ctypes.POINTER(f64)]),
        "kaze_kernel_names": (ctypes.c_char_p, []),
        "kaze_copy_f32": (i32, [vp, vp, sz, vp]),
        "kaze_batch_workspace_bytes": (sz, [vp, i32, P, vp]),
        "kaze_batch_create": (i32, [vp, i32, P, vp, vp, sz, ctypes.POINTER(vp)]),
        "kaze_batch_run": (i32, [vp, i32, vp]),
        "kaze_batch_properties": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "kaze_batch_destroy": (i32, [vp]),
        "kaze_batch_autotune": (i32, [vp, i32, P, vp, sz, i32, vp, vp, vp]),
        "kaze_aos_shape_info": (i32, [i32] + [ctypes.POINTER(i32)] * 6),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _shape_table():
    out = []
    for sh in range(64):
        v = [ctypes.c_int() for _ in range(6)]
        if lib.kaze_aos_shape_info(sh, *[ctypes.byref(x) for x in v]) != KAZE_OK:
            break
        out.append(dict(zip(("tile_w", "tile_h", "row_chunk", "col_chunk", "iface_m",
                             "chunk_lanes"), (x.value for x in v))))
    return tuple(out)


# Launch shapes of the AOS steps (kaze_batch_config.aos_shape): tile width
# and height, chunk lengths of rows and columns, interface chunks per lane,
# sweep lanes per chunk.
AOS_SHAPES = _shape_table()


def shape_label(shape: int) -> str:
    """e.g. '60x32 c30/32 m4'."""
    a = AOS_SHAPES[shape]
    return "%dx%d c%d/%d m%d" % (a["tile_w"], a["tile_h"], a["row_chunk"], a["col_chunk"],
                                 a["iface_m"])


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


# Bytes of the device-resident scratch of kaze_build_scale_space_noalloc.
KAZE_NOALLOC_SCRATCH_BYTES = 64 << 20


def kaze_build_scale_space_noalloc(img, W, H, ld_img, p, levels, k_out, stream=None):
    _check(lib.kaze_build_scale_space_noalloc(_ptr(img), W, H, ld_img, ctypes.byref(p),
                                              _ptr(levels), _ptr(k_out), _stream(stream)))


def kaze_conductivity(L, W, H, p, k, g, stream=None):
    _check(lib.kaze_conductivity(_ptr(L), W, H, ctypes.byref(p), float(k), _ptr(g),
                                 _stream(stream)))


def kaze_aos_step(L, g, W, H, tau, L_next, ws, ws_bytes, stream=None):
    _check(lib.kaze_aos_step(_ptr(L), _ptr(g), W, H, float(tau), _ptr(L_next), _ptr(ws),
                             ws_bytes, _stream(stream)))


def kaze_fed_schedule(T):
    """Step sizes of one FED cycle of total time T in application order
    (list of floats)."""
    n = lib.kaze_fed_schedule(float(T), None, 0)
    if n < 0:
        _check(n)
    buf = (ctypes.c_double * n)()
    lib.kaze_fed_schedule(float(T), ctypes.cast(buf, ctypes.c_void_p), n)
    return [buf[i] for i in range(n)]


def kaze_fed_cycle(L, g, W, H, T, L_next, ws, ws_bytes, stream=None):
    _check(lib.kaze_fed_cycle(_ptr(L), _ptr(g), W, H, float(T), _ptr(L_next), _ptr(ws), ws_bytes,
                              _stream(stream)))


def kaze_detector_response(levels, W, H, p, det, stream=None):
    _check(lib.kaze_detector_response(_ptr(levels), W, H, ctypes.byref(p), _ptr(det),
                                      _stream(stream)))


def kaze_find_extrema(det, W, H, p, kps, capacity, count, stream=None):
    _check(lib.kaze_find_extrema(_ptr(det), W, H, ctypes.byref(p), _ptr(kps), capacity,
                                 _ptr(count), _stream(stream)))


def kaze_refine_keypoints(det, W, H, p, kps, count, capacity, edge_ratio, out, stream=None):
    _check(lib.kaze_refine_keypoints(_ptr(det), W, H, ctypes.byref(p), _ptr(kps), _ptr(count),
                                     capacity, float(edge_ratio), _ptr(out), _stream(stream)))


def kaze_derivatives(levels, W, H, p, lx, ly, stream=None):
    _check(lib.kaze_derivatives(_ptr(levels), W, H, ctypes.byref(p), _ptr(lx), _ptr(ly),
                                _stream(stream)))


def kaze_describe_keypoints(lx, ly, W, H, p, kps, count, capacity, angles, descriptors,
                            stream=None):
    _check(lib.kaze_describe_keypoints(_ptr(lx), _ptr(ly), W, H, ctypes.byref(p), _ptr(kps),
                                       _ptr(count), capacity, _ptr(angles), _ptr(descriptors),
                                       _stream(stream)))


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


def _descs(images):
    arr = (kaze_image_desc * len(images))(*images)
    return arr


def _cfg(shape):
    return None if shape is None else ctypes.byref(kaze_batch_config(int(shape)))


def kaze_batch_workspace_bytes(images, p, shape=None) -> int:
    return int(lib.kaze_batch_workspace_bytes(_descs(images), len(images), ctypes.byref(p),
                                              _cfg(shape)))


def kaze_batch_create(images, p, shape, ws, ws_bytes):
    h = ctypes.c_void_p()
    _check(lib.kaze_batch_create(_descs(images), len(images), ctypes.byref(p), _cfg(shape),
                                 _ptr(ws), ws_bytes, ctypes.byref(h)))
    return h


def kaze_batch_properties(handle):
    """(aos_shape, det_levels_in_segment) of a created batch."""
    a, d = ctypes.c_int(), ctypes.c_int()
    _check(lib.kaze_batch_properties(handle, ctypes.byref(a), ctypes.byref(d)))
    return a.value, d.value


def kaze_batch_run(handle, eager=False, stream=None):
    _check(lib.kaze_batch_run(handle, 1 if eager else 0, _stream(stream)))


def kaze_batch_destroy(handle):
    _check(lib.kaze_batch_destroy(handle))


def kaze_batch_autotune(images, p, ws, ws_bytes, reps=3, stream=None):
    """Returns (best shape index, ms per run of each shape in AOS_SHAPES)."""
    best = kaze_batch_config(-1)
    ms = (ctypes.c_double * len(AOS_SHAPES))()
    _check(lib.kaze_batch_autotune(_descs(images), len(images), ctypes.byref(p), _ptr(ws),
                                   ws_bytes, reps, _stream(stream), ctypes.byref(best),
                                   ctypes.cast(ms, ctypes.c_void_p)))
    return best.aos_shape, [ms[i] for i in range(len(AOS_SHAPES))]


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

    def refine(self, edge_ratio=10.0, stream=None):
        """Sub-pixel refinement and edge test of the extrema of the last
        run (kaze_refine_keypoints); fills ``self.refined``, an
        (capacity, 6) int32 tensor of kaze_keypoint_refined records in the
        order of ``self.kps``."""
        import torch
        if getattr(self, "refined", None) is None:
            self.refined = torch.empty((max(self.capacity, 1), 6), dtype=torch.int32,
                                       device=self.kps.device)
        kaze_refine_keypoints(self.det, self.W, self.H, self.p, self.kps, self.count,
                              self.capacity, edge_ratio, self.refined, stream)

    def describe(self, stream=None):
        """Derivatives of the last run's levels and the orientation and
        descriptor of every refined keypoint (kaze_derivatives,
        kaze_describe_keypoints; call refine() first): fills ``self.lx``,
        ``self.ly``, ``self.angles`` (capacity,) and ``self.descriptors``
        (capacity, 64), in the order of ``self.kps``."""
        import torch
        if getattr(self, "lx", None) is None:
            self.lx = torch.empty_like(self.levels)
            self.ly = torch.empty_like(self.levels)
            cap = max(self.capacity, 1)
            self.angles = torch.empty(cap, dtype=torch.float32, device=self.levels.device)
            self.descriptors = torch.empty((cap, 64), dtype=torch.float32,
                                           device=self.levels.device)
        kaze_derivatives(self.levels, self.W, self.H, self.p, self.lx, self.ly, stream)
        kaze_describe_keypoints(self.lx, self.ly, self.W, self.H, self.p, self.refined, self.count,
                                self.capacity, self.angles, self.descriptors, stream)

    def refined_keypoints(self):
        """Host (n, 6) float64 array (level, y, x, response, edge_ratio,
        kept) of the last refine(), sorted like keypoints(); synchronises."""
        import numpy as np
        import torch
        n = min(int(self.count.item()), self.capacity)
        raw = self.refined[:n].cpu()
        f = raw.view(torch.float32).numpy().astype(np.float64)
        i = raw.numpy()
        ints = self.kps[:n].cpu().numpy()
        out = np.stack([i[:, 2], f[:, 1], f[:, 0], f[:, 3], f[:, 4], i[:, 5]], axis=1) \
            if n else np.zeros((0, 6))
        if n:
            order = np.lexsort((ints[:, 0], ints[:, 1], ints[:, 2]))
            out = out[order]
        return out

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


class KazeBatch:
    """Many images of different sizes through one captured graph per run.

    ``sizes`` is a list of (W, H).  Per-image device buffers are allocated
    here (torch); ``inputs[j]`` is image j's input tensor [H][W] to fill
    before ``run()``.  ``shape`` selects the launch shape of the line
    solves (an index of AOS_SHAPES);
    ``shape="auto"`` runs the library's autotuner, caching the choice in the
    JSON file ``tune_cache`` when given (keyed by GPU architecture and the
    list of sizes).  With ``ld_pad`` > 0 each input is a view of W columns
    of a [H][W + ld_pad] allocation (row pitch W + ld_pad)."""

    def __init__(self, sizes, params=None, capacity=1 << 14, shape="auto", tune_cache=None,
                 device="cuda", with_detector=True, ld_pad=0):
        import torch
        self.p = params if params is not None else kaze_default_params()
        self.N = kaze_num_levels(self.p)
        self.sizes = [(int(w), int(h)) for w, h in sizes]
        dev = torch.device(device)
        self.inputs, self.levels, self.det, self.k, self.kps, self.count = [], [], [], [], [], []
        # every image's keypoint count in one tensor (one readback per run)
        self.counts = torch.zeros(len(self.sizes), dtype=torch.int32, device=dev)
        descs = []
        for j, (W, H) in enumerate(self.sizes):
            x = torch.zeros((H, W + int(ld_pad)), dtype=torch.float32, device=dev)[:, :W]
            lv = torch.empty((self.N, H, W), dtype=torch.float32, device=dev)
            dt = torch.empty_like(lv) if with_detector else None
            k = torch.empty(1, dtype=torch.float32, device=dev)
            kp = torch.empty((max(capacity, 1), 4), dtype=torch.int32, device=dev)
            ct = self.counts[j:j + 1]
            self.inputs.append(x)
            self.levels.append(lv)
            self.det.append(dt)
            self.k.append(k)
            self.kps.append(kp)
            self.count.append(ct)
            descs.append(kaze_image_desc(x.data_ptr(), W, H, x.stride(0), lv.data_ptr(),
                                         dt.data_ptr() if dt is not None else None, k.data_ptr(),
                                         kp.data_ptr() if with_detector else None,
                                         capacity if with_detector else 0,
                                         ct.data_ptr() if with_detector else None))
        self.descs = descs
        self.capacity = capacity
        self.ws_bytes = kaze_batch_workspace_bytes(descs, self.p)
        if self.ws_bytes == 0:
            raise KazeError(KAZE_ERR_INVALID_ARG, "batch sizes or parameters are invalid")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.tune_ms = None
        if shape == "auto":
            shape = self._tuned_shape(tune_cache)
        self.shape = int(shape)
        self.handle = kaze_batch_create(descs, self.p, self.shape, self.ws, self.ws_bytes)
        self.det_levels_in_segment = kaze_batch_properties(self.handle)[1]

    def _key(self):
        import hashlib
        import torch
        arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
        sig = hashlib.sha1(repr(sorted(self.sizes)).encode()).hexdigest()[:16]
        return "%s|n=%d|%s|shapes=%d" % (arch, len(self.sizes), sig, len(AOS_SHAPES))

    def _tuned_shape(self, cache_path):
        import json
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
        key = self._key()
        if key in cache:
            self.tune_ms = cache[key].get("ms")
            return cache[key]["shape"]
        best, ms = kaze_batch_autotune(self.descs, self.p, self.ws, self.ws_bytes)
        self.tune_ms = ms
        if cache_path:
            cache[key] = {"shape": best, "ms": ms, "label": shape_label(best),
                          "labels": [shape_label(i) for i in range(len(AOS_SHAPES))]}
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=1)
            os.replace(tmp, cache_path)
        return best

    def run(self, eager=False, stream=None):
        kaze_batch_run(self.handle, eager, stream)

    def keypoints(self, j):
        """Image j's keypoints as in Kaze.keypoints(); synchronises."""
        import numpy as np
        import torch
        n = min(int(self.count[j].item()), self.capacity)
        if n == 0:
            return np.zeros((0, 4))
        raw = self.kps[j][:n].cpu()
        xyl = raw[:, :3].numpy().astype(np.int64)
        resp = raw[:, 3].contiguous().view(dtype=torch.float32).numpy()
        out = np.stack([xyl[:, 2], xyl[:, 1], xyl[:, 0], resp.astype(np.float64)], axis=1)
        return out[np.lexsort((out[:, 2], out[:, 1], out[:, 0]))]

    def close(self):
        if getattr(self, "handle", None):
            kaze_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
