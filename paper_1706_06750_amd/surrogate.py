"""Python binding of the learned AOS-step surrogate (``include/kaze_surrogate.h``).

ctypes argument marshalling only: the forward pass, the backward pass and
Adam run in libkaze's HIP kernels.  Device buffers are torch tensors.
"""
from __future__ import annotations

import ctypes

from .kaze import (KAZE_OK, KazeError, _ptr, _stream, kaze_default_params, kaze_image_desc,
                   kaze_num_levels, kaze_params, lib)

# Every symbol include/kaze_surrogate.h declares.
EXPORTS = (
    "kaze_sg_param_count", "kaze_sg_packed_bytes", "kaze_sg_pack",
    "kaze_sg_workspace_bytes", "kaze_sg_plan_create", "kaze_sg_plan_destroy",
    "kaze_sg_forward", "kaze_sg_gradients", "kaze_sg_adam",
    "kaze_sg_default_config", "kaze_sg_scale_space_workspace_bytes",
    "kaze_sg_scale_space_create", "kaze_sg_scale_space_run", "kaze_sg_scale_space_destroy",
    "kaze_sg_batch_workspace_bytes", "kaze_sg_batch_create",
)


class kaze_sg_config(ctypes.Structure):
    _fields_ = [("bound", ctypes.c_double), ("probes", ctypes.c_int),
                ("probe_size", ctypes.c_int), ("aos_shape", ctypes.c_int)]


_vp, _sz, _i32, _f64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
for _name, (_res, _args) in {
    "kaze_sg_param_count": (_i32, []),
    "kaze_sg_packed_bytes": (_sz, []),
    "kaze_sg_pack": (_i32, [_vp, _vp, _vp]),
    "kaze_sg_workspace_bytes": (_sz, [_i32, _i32, _i32, _i32]),
    "kaze_sg_plan_create": (_i32, [_i32, _i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "kaze_sg_plan_destroy": (None, [_vp]),
    "kaze_sg_forward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "kaze_sg_gradients": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "kaze_sg_adam": (_i32, [_vp, _vp, _vp, _vp, _i32, _i32, _f64, _f64, _f64, _f64, _vp]),
    "kaze_sg_default_config": (_i32, [ctypes.POINTER(kaze_sg_config)]),
    "kaze_sg_scale_space_workspace_bytes": (_sz, [_i32, _i32, ctypes.POINTER(kaze_params),
                                                  ctypes.POINTER(kaze_sg_config)]),
    "kaze_sg_scale_space_create": (_i32, [ctypes.POINTER(kaze_image_desc),
                                          ctypes.POINTER(kaze_params),
                                          ctypes.POINTER(kaze_sg_config), _vp, _vp, _vp, _vp,
                                          _sz, ctypes.POINTER(_vp)]),
    "kaze_sg_scale_space_run": (_i32, [_vp, _i32, _vp]),
    "kaze_sg_scale_space_destroy": (_i32, [_vp]),
    "kaze_sg_batch_workspace_bytes": (_sz, [_vp, _i32, ctypes.POINTER(kaze_params),
                                            ctypes.POINTER(kaze_sg_config)]),
    "kaze_sg_batch_create": (_i32, [_vp, _i32, ctypes.POINTER(kaze_params),
                                    ctypes.POINTER(kaze_sg_config), _vp, _vp, _vp, _vp, _sz,
                                    ctypes.POINTER(_vp)]),
}.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def _check(st):
    if st != KAZE_OK:
        raise KazeError(st, lib.kaze_last_error().decode())


def kaze_sg_param_count() -> int:
    return int(lib.kaze_sg_param_count())


def kaze_sg_packed_bytes() -> int:
    return int(lib.kaze_sg_packed_bytes())


def kaze_sg_pack(params, packed, stream=None):
    _check(lib.kaze_sg_pack(_ptr(params), _ptr(packed), _stream(stream)))


def kaze_sg_workspace_bytes(n: int, W: int, H: int, training: int) -> int:
    return int(lib.kaze_sg_workspace_bytes(n, W, H, training))


def kaze_sg_plan_create(n, W, H, training, ws, ws_bytes, stream=None):
    h = _vp()
    _check(lib.kaze_sg_plan_create(n, W, H, training, _ptr(ws), ws_bytes, _stream(stream),
                                   ctypes.byref(h)))
    return h.value


def kaze_sg_plan_destroy(plan):
    lib.kaze_sg_plan_destroy(plan)


def kaze_sg_forward(plan, packed, L, g, tau, out, add_input=1, stream=None):
    _check(lib.kaze_sg_forward(plan, _ptr(packed), _ptr(L), _ptr(g), _ptr(tau), _ptr(out),
                               int(add_input), _stream(stream)))


def kaze_sg_gradients(plan, packed, L, g, tau, L_next, weight, grad, loss, stream=None):
    _check(lib.kaze_sg_gradients(plan, _ptr(packed), _ptr(L), _ptr(g), _ptr(tau), _ptr(L_next),
                                 _ptr(weight), _ptr(grad), _ptr(loss), _stream(stream)))


def kaze_sg_adam(params, grad, m, v, count, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
    _check(lib.kaze_sg_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(count), int(step),
                            float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


PARAM_COUNT = kaze_sg_param_count()


def _device_bytes(nbytes: int):
    import torch
    # the caching allocator hands out 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


class Weights:
    """FP32 master parameters, Adam moments and the packed operand buffer."""

    def __init__(self, params):
        import torch
        p = torch.as_tensor(params, dtype=torch.float32)
        if p.numel() != PARAM_COUNT:
            raise ValueError("expected %d parameters" % PARAM_COUNT)
        self.params = p.reshape(-1).to("cuda").contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.packed = _device_bytes(kaze_sg_packed_bytes())
        self.step = 0
        self.pack()

    def pack(self, stream=None):
        kaze_sg_pack(self.params, self.packed, stream)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        kaze_sg_adam(self.params, self.grad, self.m, self.v, PARAM_COUNT, self.step, lr, beta1,
                     beta2, eps, stream)
        self.pack(stream)


class Plan:
    """A surrogate plan over n samples of W x H with its own workspace."""

    def __init__(self, n: int, W: int, H: int, training: bool = False):
        import torch
        self.n, self.W, self.H, self.training = n, W, H, bool(training)
        nbytes = kaze_sg_workspace_bytes(n, W, H, int(training))
        if nbytes == 0:
            raise ValueError("unsupported surrogate plan %dx%dx%d" % (n, W, H))
        self.ws = _device_bytes(nbytes)
        self.handle = kaze_sg_plan_create(n, W, H, int(training), self.ws, nbytes)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def forward(self, w: Weights, L, g, tau, out=None, add_input=True, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(L)
        kaze_sg_forward(self.handle, w.packed, L, g, tau, out, add_input, stream)
        return out

    def gradients(self, w: Weights, L, g, tau, L_next, weight=None, stream=None):
        kaze_sg_gradients(self.handle, w.packed, L, g, tau, L_next, weight, w.grad, self.loss,
                          stream)
        return self.loss

    def close(self):
        if self.handle:
            kaze_sg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kaze_sg_default_config(**overrides) -> kaze_sg_config:
    c = kaze_sg_config()
    _check(lib.kaze_sg_default_config(ctypes.byref(c)))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def kaze_sg_scale_space_workspace_bytes(W, H, p, c) -> int:
    return int(lib.kaze_sg_scale_space_workspace_bytes(W, H, ctypes.byref(p), ctypes.byref(c)))


def kaze_sg_scale_space_create(desc, p, c, packed, probe_xy, err, ws, ws_bytes):
    h = _vp()
    pxy = None
    if probe_xy is not None:
        import numpy as np
        arr = np.ascontiguousarray(probe_xy, dtype=np.int32)
        pxy = arr.ctypes.data_as(_vp)
    _check(lib.kaze_sg_scale_space_create(ctypes.byref(desc), ctypes.byref(p), ctypes.byref(c),
                                          _ptr(packed), pxy, _ptr(err), _ptr(ws), ws_bytes,
                                          ctypes.byref(h)))
    return h.value


def kaze_sg_scale_space_run(handle, eager=False, stream=None):
    _check(lib.kaze_sg_scale_space_run(handle, int(bool(eager)), _stream(stream)))


def kaze_sg_scale_space_destroy(handle):
    _check(lib.kaze_sg_scale_space_destroy(handle))


def kaze_sg_batch_workspace_bytes(descs, p, c) -> int:
    arr = (kaze_image_desc * len(descs))(*descs)
    return int(lib.kaze_sg_batch_workspace_bytes(arr, len(descs), ctypes.byref(p),
                                                 ctypes.byref(c)))


def kaze_sg_batch_create(descs, p, c, packed, probe_xy, err, ws, ws_bytes):
    """probe_xy: (n, N, probes, 2) int32 corners, or None with no probes."""
    arr = (kaze_image_desc * len(descs))(*descs)
    h = _vp()
    pxy = None
    if probe_xy is not None:
        import numpy as np
        pa = np.ascontiguousarray(probe_xy, dtype=np.int32)
        pxy = pa.ctypes.data_as(_vp)
    _check(lib.kaze_sg_batch_create(arr, len(descs), ctypes.byref(p), ctypes.byref(c),
                                    _ptr(packed), pxy, _ptr(err), _ptr(ws), ws_bytes,
                                    ctypes.byref(h)))
    return h.value


def probe_windows(W, H, N, probes, size, seed):
    """Seeded uniform top-left corners of the probe windows, [N][probes][2]
    (level 0 unused)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    xy = np.zeros((N, max(probes, 1), 2), dtype=np.int32)
    if probes > 0:
        xy[:, :, 0] = rng.integers(0, max(1, W - size + 1), size=(N, probes))
        xy[:, :, 1] = rng.integers(0, max(1, H - size + 1), size=(N, probes))
    return xy[:, :probes]


class SurrogateScaleSpace:
    """Scale space of one W x H image with the surrogate and its per-level
    fallback (device buffers as torch tensors, graphs captured at creation).
    ``run()`` recomputes ``levels``, ``k``, ``err`` and, with the detector,
    ``det``, ``kps`` and ``count`` from ``img``."""

    def __init__(self, W, H, weights: Weights, config=None, params=None, probe_seed=0,
                 with_detector=True, capacity=1 << 16):
        import torch
        self.W, self.H = int(W), int(H)
        self.p = params if params is not None else kaze_default_params()
        self.c = config if config is not None else kaze_sg_default_config()
        self.N = kaze_num_levels(self.p)
        self.weights = weights
        dev = "cuda"
        self.img = torch.zeros((self.H, self.W), dtype=torch.float32, device=dev)
        self.levels = torch.empty((self.N, self.H, self.W), dtype=torch.float32, device=dev)
        self.k = torch.empty(1, dtype=torch.float32, device=dev)
        self.err = torch.zeros(self.N, dtype=torch.float32, device=dev)
        self.capacity = int(capacity) if with_detector else 0
        self.det = torch.empty_like(self.levels) if with_detector else None
        self.kps = torch.empty((max(self.capacity, 1), 4), dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev) if with_detector else None
        self.probe_xy = probe_windows(self.W, self.H, self.N, self.c.probes, self.c.probe_size,
                                      probe_seed)
        d = kaze_image_desc()
        d.img, d.W, d.H, d.ld_img = self.img.data_ptr(), self.W, self.H, self.W
        d.levels, d.k = self.levels.data_ptr(), self.k.data_ptr()
        d.det = self.det.data_ptr() if with_detector else None
        d.kps = self.kps.data_ptr() if with_detector else None
        d.capacity = self.capacity
        d.count = self.count.data_ptr() if with_detector else None
        self.desc = d
        nbytes = kaze_sg_scale_space_workspace_bytes(self.W, self.H, self.p, self.c)
        if nbytes == 0:
            raise ValueError("unsupported surrogate scale space %dx%d" % (self.W, self.H))
        self.ws = _device_bytes(nbytes)
        torch.cuda.synchronize()
        self.handle = kaze_sg_scale_space_create(d, self.p, self.c, weights.packed,
                                                 self.probe_xy if self.c.probes > 0 else None,
                                                 self.err, self.ws, nbytes)

    def run(self, eager=False, stream=None):
        kaze_sg_scale_space_run(self.handle, eager, stream)

    def accepted(self):
        """Host list: level i used the surrogate (synchronises)."""
        e = self.err.cpu().tolist()
        return [False] + [v <= self.c.bound for v in e[1:]]

    def keypoints(self):
        """Host (n, 4) float64 array (level, y, x, response) sorted by
        (level, y, x); synchronises."""
        import numpy as np
        n = min(int(self.count.item()), self.capacity)
        if n == 0:
            return np.zeros((0, 4))
        k = self.kps[:n].cpu().numpy()
        resp = k[:, 3].copy().view(np.float32).astype(np.float64)
        out = np.stack([k[:, 2], k[:, 1], k[:, 0], resp], axis=1).astype(np.float64)
        order = np.lexsort((out[:, 2], out[:, 1], out[:, 0]))
        return out[order]

    def close(self):
        if self.handle:
            kaze_sg_scale_space_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SurrogateBatch:
    """Surrogate scale space of many images of different sizes in one plan
    (kaze_sg_batch_create; run with kaze_batch_run).  ``inputs[j]`` is image
    j's input [H][W] to fill before ``run()``; ``err`` is the (n, N) table of
    probe errors each run writes (image j used the surrogate for level i iff
    err[j, i] <= bound).  Probe windows of image j are drawn with seed
    ``probe_seed + j``."""

    def __init__(self, sizes, weights: Weights, config=None, params=None, probe_seed=0,
                 with_detector=True, capacity=1 << 14):
        import numpy as np
        import torch
        from .kaze import kaze_batch_properties
        self.p = params if params is not None else kaze_default_params()
        self.c = config if config is not None else kaze_sg_default_config()
        self.N = kaze_num_levels(self.p)
        self.sizes = [(int(w), int(h)) for w, h in sizes]
        self.weights = weights
        self.capacity = int(capacity) if with_detector else 0
        dev = "cuda"
        self.inputs, self.levels, self.det, self.k, self.kps, self.count = [], [], [], [], [], []
        descs = []
        for W, H in self.sizes:
            x = torch.zeros((H, W), dtype=torch.float32, device=dev)
            lv = torch.empty((self.N, H, W), dtype=torch.float32, device=dev)
            dt = torch.empty_like(lv) if with_detector else None
            k = torch.empty(1, dtype=torch.float32, device=dev)
            kp = torch.empty((max(self.capacity, 1), 4), dtype=torch.int32, device=dev)
            ct = torch.zeros(1, dtype=torch.int32, device=dev) if with_detector else None
            self.inputs.append(x)
            self.levels.append(lv)
            self.det.append(dt)
            self.k.append(k)
            self.kps.append(kp)
            self.count.append(ct)
            d = kaze_image_desc()
            d.img, d.W, d.H, d.ld_img = x.data_ptr(), W, H, W
            d.levels, d.k = lv.data_ptr(), k.data_ptr()
            d.det = dt.data_ptr() if with_detector else None
            d.kps = kp.data_ptr() if with_detector else None
            d.capacity = self.capacity
            d.count = ct.data_ptr() if with_detector else None
            descs.append(d)
        self.descs = descs
        n = len(self.sizes)
        self.err = torch.zeros((n, self.N), dtype=torch.float32, device=dev)
        P = self.c.probes
        if P > 0:
            self.probe_xy = np.stack([probe_windows(W, H, self.N, P, self.c.probe_size,
                                                    probe_seed + j)
                                      for j, (W, H) in enumerate(self.sizes)])
        else:
            self.probe_xy = None
        nbytes = kaze_sg_batch_workspace_bytes(descs, self.p, self.c)
        if nbytes == 0:
            raise KazeError(-1, "surrogate batch sizes, parameters or config are invalid")
        self.ws_bytes = nbytes
        self.ws = _device_bytes(nbytes)
        torch.cuda.synchronize()
        self.handle = kaze_sg_batch_create(descs, self.p, self.c, weights.packed, self.probe_xy,
                                           self.err, self.ws, nbytes)
        self.shape = kaze_batch_properties(self.handle)[0]

    def run(self, eager=False, stream=None):
        from .kaze import kaze_batch_run
        kaze_batch_run(self.handle, eager, stream)

    def accepted(self):
        """Host (n, N) bool array: image j used the surrogate for level i
        (synchronises)."""
        import numpy as np
        acc = self.err.cpu().numpy() <= self.c.bound
        acc[:, 0] = False
        return np.asarray(acc)

    def keypoints(self, j):
        """Image j's keypoints (level, y, x, response) sorted by (level, y,
        x); synchronises."""
        import numpy as np
        n = min(int(self.count[j].item()), self.capacity)
        if n == 0:
            return np.zeros((0, 4))
        k = self.kps[j][:n].cpu().numpy()
        resp = k[:, 3].copy().view(np.float32).astype(np.float64)
        out = np.stack([k[:, 2], k[:, 1], k[:, 0], resp], axis=1).astype(np.float64)
        return out[np.lexsort((out[:, 2], out[:, 1], out[:, 0]))]

    def close(self):
        from .kaze import kaze_batch_destroy
        if getattr(self, "handle", None):
            kaze_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
