"""Parity helpers shared by the GPU tests (comparison rules only; no method
arithmetic)."""
import numpy as np

# Per-level bound on max |L_gpu - L_oracle| for images in [0, 1].
LEVEL_TOL = 1e-4
# Keypoints present on one side only are excused when the oracle response is
# this close to the threshold or to one of its 26 neighbours.
EXCUSE = 1e-5


def note(msg):
    print(msg, flush=True)


def neighbours26(det, lev, y, x):
    out = []
    for dl in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dl, dy, dx) != (0, 0, 0):
                    out.append(det[lev + dl, y + dy, x + dx])
    return np.array(out)


def window_neighbours(det, lev, y, x, h):
    """The 8 neighbours in level lev and the responses of levels lev-1 and
    lev+1 within h pixels (clipped to the image)."""
    N, H, W = det.shape
    own = det[lev, y - 1:y + 2, x - 1:x + 2].ravel()
    own = np.delete(own, 4)
    y0, y1, x0, x1 = max(0, y - h), min(H, y + h + 1), max(0, x - h), min(W, x + h + 1)
    return np.concatenate([own, det[lev - 1, y0:y1, x0:x1].ravel(),
                           det[lev + 1, y0:y1, x0:x1].ravel()])


def excused(det_orc, p, threshold, radii=None):
    lev, y, x = (int(v) for v in p)
    v = det_orc[lev, y, x]
    if abs(v - threshold) < EXCUSE:
        return True
    nb = neighbours26(det_orc, lev, y, x) if radii is None else \
        window_neighbours(det_orc, lev, y, x, int(radii[lev]))
    return bool(np.min(np.abs(v - nb)) < EXCUSE)


def compare_keypoints(kp_gpu, kp_orc, det_orc, threshold, radii=None):
    """Sets on (level, y, x) must agree up to excused points (radii: the
    cross-level window half-sides of the exact test, None for 3x3x3).
    Returns (n_common, unexcused_gpu_only, unexcused_oracle_only)."""
    g = {tuple(int(v) for v in r[:3]) for r in kp_gpu}
    o = {tuple(int(v) for v in r[:3]) for r in kp_orc}
    bad_g = [p for p in g - o if not excused(det_orc, p, threshold, radii)]
    bad_o = [p for p in o - g if not excused(det_orc, p, threshold, radii)]
    return len(g & o), bad_g, bad_o


def recall(kp_s, kp_orc, det_orc, threshold):
    """Keypoint recall |KP_s & KP_orc| / |KP_orc| on exact (level, y, x),
    with oracle points that the excuse rule covers and KP_s misses left out
    of the denominator.  Returns (recall, n_common, denominator)."""
    s = {tuple(int(v) for v in r[:3]) for r in kp_s}
    o = {tuple(int(v) for v in r[:3]) for r in kp_orc}
    common = len(s & o)
    excused_missing = sum(1 for p in o - s if excused(det_orc, p, threshold))
    den = len(o) - excused_missing
    return (common / den if den else 1.0), common, den
