"""Keypoint refinement and edge test (Sec. II-B, Eqs. 9-12) on the GPU
against the FP64 oracle, through the C ABI (kaze_refine_keypoints).

Stage test: the oracle's detector responses (rounded to FP32) and a set of
positions (the oracle's extrema plus random interior points, which reach
saddles, minima, flat spots and offsets beyond one pixel) go to the kernel
and to O.refine_keypoints.  Both then fit the same nine FP32 numbers, so
the differences are the kernel's rounding: with u = 2^-24 and m the largest
|response| of the window, every fitted coefficient is off by at most
c u m (c = 32 covers the sums of nine terms and the 1/6 scalings), so the
offset moves by at most c u m (1 + |du| + |dv|) / |lambda_min(H)| and the
refined value by c u m (1 + |du| + |dv|)^2; a kept flag may differ only
where the oracle's decision lies within those perturbations of a bound.

End to end: the whole GPU path and refinement against the oracle's path
and refinement.  The nine inputs of a fit then differ by the detector
difference of the two paths, which the parity tests bound; here its value
on the window (at most 2x per coefficient) joins c u m above, so that the
positions are compared at the precision the inputs allow.
"""
import numpy as np
import pytest

import oracle as O
from synthetic import kaze_image
from kaze_parity import LEVEL_TOL, compare_keypoints, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = 2.0 ** -24
C = 32.0
EDGE_R = O.EDGE_RATIO


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def kp_records(kps):
    """(n, 4) rows (level, y, x, response) -> device int32 (n, 4) records
    x, y, level, response bits."""
    n = len(kps)
    rec = np.zeros((max(n, 1), 4), dtype=np.int32)
    if n:
        rec[:n, 0:3] = np.stack([kps[:, 2], kps[:, 1], kps[:, 0]], axis=1).astype(np.int32)
        rec[:n, 3] = np.asarray(kps[:, 3], dtype=np.float32).view(np.int32)
    return torch.from_numpy(rec).cuda()


def run_refine(K, det32, kps, p, capacity=None, count=None, out=None):
    N, H, W = det32.shape
    cap = len(kps) if capacity is None else capacity
    d_det = dev(det32)
    d_kps = kp_records(kps)
    d_cnt = torch.tensor([len(kps) if count is None else count], dtype=torch.int32, device="cuda")
    if out is None:
        out = torch.full((max(cap, 1), 6), -7, dtype=torch.int32, device="cuda")
    K.kaze_refine_keypoints(d_det, W, H, p, d_kps, d_cnt, cap, EDGE_R, out)
    torch.cuda.synchronize()
    return out


def unpack(out, n):
    raw = out[:n].cpu()
    f = raw.view(torch.float32).numpy().astype(np.float64)
    i = raw.numpy()
    # (level, y, x, response, ratio, kept) like the oracle
    return np.stack([i[:, 2], f[:, 1], f[:, 0], f[:, 3], f[:, 4], i[:, 5]], axis=1)


def hessian_terms(det, lev, y, x):
    a, b, c, d, e, f = O.quadratic_fit_3x3(det[lev, y - 1:y + 2, x - 1:x + 2])
    hxx, hyy, hxy = 2 * d, 2 * e, f
    lam = np.linalg.eigvalsh(np.array([[hxx, hxy], [hxy, hyy]]))
    return hxx, hyy, hxy, float(np.min(np.abs(lam)))


def decision_margin_excused(hxx, hyy, hxy, dh):
    """True when the oracle's kept decision lies within the perturbation dh
    of the Hessian entries of the bound on Det(H), Tr(H) or the ratio."""
    dt = hxx * hyy - hxy * hxy
    tr = hxx + hyy
    ddt = (abs(hxx) + abs(hyy) + 2 * abs(hxy)) * dh + 2 * dh * dh
    dtr = 2 * dh
    if abs(dt) <= ddt or abs(tr) <= dtr:
        return True
    thr = (EDGE_R + 1) ** 2 / EDGE_R
    if dt > 0:
        ratio = tr * tr / dt
        rel = (2 * dtr / abs(tr) + ddt / abs(dt)) * 2
        if abs(ratio - thr) <= thr * rel:
            return True
    return False


def check_rows(got, ref, det, kps, coef_err, label):
    """coef_err(lev, y, x) -> bound on the error of every fitted coefficient."""
    n = len(ref)
    assert got.shape == ref.shape
    assert np.array_equal(got[:, 0], ref[:, 0])
    n_pos = n_flag = n_exc = 0
    worst = 0.0
    for j in range(n):
        lev, y, x = int(kps[j, 0]), int(kps[j, 1]), int(kps[j, 2])
        hxx, hyy, hxy, lam = hessian_terms(det, lev, y, x)
        e = coef_err(lev, y, x)
        du, dv = ref[j, 2] - x, ref[j, 1] - y
        finite = np.isfinite(du) and np.isfinite(dv)
        dh = 2 * e
        if finite and lam > 8 * dh:
            span = 1 + abs(du) + abs(dv)
            tol = 2 * e * span / (lam - 4 * dh) * 2 + 2.0 ** -22 * (abs(x) + abs(y) + 2)
            err = max(abs(got[j, 1] - ref[j, 1]), abs(got[j, 2] - ref[j, 2]))
            worst = max(worst, err / tol)
            assert err <= tol, (label, j, (lev, y, x), got[j], ref[j], tol)
            if abs(du) <= 1 and abs(dv) <= 1:
                vtol = 4 * e * span * span + 4 * U * abs(ref[j, 3])
                assert abs(got[j, 3] - ref[j, 3]) <= vtol, (label, j, got[j], ref[j], vtol)
            n_pos += 1
        if got[j, 5] != ref[j, 5]:
            off_tol = 2 * e * (1 + abs(du) + abs(dv)) / max(lam - 4 * dh, 1e-300) * 2
            near_unit = finite and (abs(abs(du) - 1) <= off_tol or abs(abs(dv) - 1) <= off_tol)
            ok = near_unit or decision_margin_excused(hxx, hyy, hxy, dh)
            assert ok, (label, j, (lev, y, x), got[j], ref[j])
            n_exc += 1
        else:
            n_flag += 1
    note(f"  {label}: {n} entries, positions checked {n_pos} (worst err/tol {worst:.2e}), "
         f"flags equal {n_flag}, excused {n_exc}, kept {int(ref[:, 5].sum())}")
    return n_pos, n_exc


def oracle_case(W, H, seed):
    img = kaze_image(W, H, seed)
    lev, k = O.build_scale_space(img.astype(np.float64))
    det = O.detector_response(lev)
    return det


@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (131, 97, 3)])
def test_refine_stage_matches_oracle(gpu_lib, W, H, seed):
    K = gpu_lib
    p = K.kaze_default_params()
    det = oracle_case(W, H, seed)
    det32 = det.astype(np.float32)
    det64 = det32.astype(np.float64)
    kp = O.find_extrema(det64, p.det_threshold)
    rng = np.random.default_rng(seed)
    N = det.shape[0]
    m = 3000
    extra = np.stack([rng.integers(0, N, m), rng.integers(1, H - 1, m),
                      rng.integers(1, W - 1, m), np.zeros(m)], axis=1).astype(np.float64)
    kps = np.concatenate([kp, extra])
    note(f"[refine] {W}x{H} seed {seed}: {len(kp)} extrema + {m} random positions")
    out = run_refine(K, det32, kps, p)
    got = unpack(out, len(kps))
    ref = O.refine_keypoints(det64, kps, EDGE_R)

    def coef_err(lev, y, x):
        return C * U * float(np.max(np.abs(det64[lev, y - 1:y + 2, x - 1:x + 2])))

    n_pos, n_exc = check_rows(got, ref, det64, kps, coef_err, "stage")
    assert n_pos >= len(kps) // 2 and n_exc <= max(2, len(kps) // 100)
    # every branch is reached: kept extrema, saddles (Det <= 0) and maxima
    # removed by the edge test
    thr = (EDGE_R + 1) ** 2 / EDGE_R
    assert ref[:len(kp), 5].sum() > 0
    assert np.isinf(ref[:, 4]).any()
    assert (np.isfinite(ref[:, 4]) & (ref[:, 4] >= thr) & (ref[:, 5] == 0)).any()


def test_refine_edge_cases(gpu_lib):
    """Windows that do not fit (border pixels, bad level) give kept 0 and
    NaN; count above capacity writes capacity entries; count 0 writes none;
    a flat window (Det 0) is not kept and has NaN response."""
    K = gpu_lib
    p = K.kaze_default_params()
    N = K.kaze_num_levels(p)
    W, H = 40, 30
    rng = np.random.default_rng(9)
    det32 = rng.normal(0, 1e-3, size=(N, H, W)).astype(np.float32)
    det32[2, 10:13, 10:13] = 0.5   # flat window
    kps = np.array([[1, 0, 5, 0], [1, 5, 0, 0], [1, H - 1, 5, 0], [1, 5, W - 1, 0],
                    [N, 5, 5, 0], [-1, 5, 5, 0], [2, 11, 11, 0], [3, 7, 9, 0]], dtype=np.float64)
    out = run_refine(K, det32, kps, p)
    got = unpack(out, len(kps))
    for j in range(6):
        assert got[j, 5] == 0 and np.isnan(got[j, 3]) and np.isnan(got[j, 4])
        assert got[j, 1] == kps[j, 1] and got[j, 2] == kps[j, 2]
    assert got[6, 5] == 0 and np.isnan(got[6, 3]) and np.isinf(got[6, 4])
    ref = O.refine_keypoints(det32.astype(np.float64), kps[6:], EDGE_R)
    assert got[6, 5] == ref[0, 5] and got[7, 5] == ref[1, 5]
    # count above capacity: capacity entries, the rest untouched
    out = run_refine(K, det32, kps[6:], p, capacity=1, count=2,
                     out=torch.full((2, 6), -7, dtype=torch.int32, device="cuda"))
    assert (out[1] == -7).all().item() and out[0, 5].item() in (0, 1)
    # count 0: nothing written
    out = run_refine(K, det32, kps[6:], p, capacity=2, count=0)
    assert (out == -7).all().item()
    # bad arguments are rejected on the host
    with pytest.raises(K.KazeError):
        run_refine(K, det32, kps, p, capacity=-1)
    with pytest.raises(K.KazeError):
        K.kaze_refine_keypoints(dev(det32), W, H, p, kp_records(kps),
                                torch.zeros(1, dtype=torch.int32, device="cuda"), 1, 1.0,
                                torch.empty((1, 6), dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (200, 130, 2)])
def test_refine_end_to_end(gpu_lib, W, H, seed):
    K = gpu_lib
    img = kaze_image(W, H, seed)
    kz = K.Kaze(W, H)
    kz.run(dev(img))
    kz.refine(EDGE_R)
    torch.cuda.synchronize()
    got_all = kz.refined_keypoints()
    kp_g = kz.keypoints()
    det_o = oracle_case(W, H, seed)
    thr = kz.p.det_threshold
    kp_o = O.find_extrema(det_o, thr)
    _, bad_g, bad_o = compare_keypoints(kp_g, kp_o, det_o, thr)
    assert not bad_g and not bad_o
    common = sorted({tuple(int(v) for v in r[:3]) for r in kp_g}
                    & {tuple(int(v) for v in r[:3]) for r in kp_o})
    idx_g = {tuple(int(v) for v in r[:3]): i for i, r in enumerate(kp_g)}
    kps = np.array([[l, y, x, 0.0] for l, y, x in common], dtype=np.float64)
    ref = O.refine_keypoints(det_o, kps, EDGE_R)
    got = np.array([got_all[idx_g[c]] for c in common])
    det_g = kz.det.cpu().numpy().astype(np.float64)
    sched = K.kaze_schedule(kz.p)

    def coef_err(lev, y, x):
        win = (lev, slice(y - 1, y + 2), slice(x - 1, x + 2))
        dd = float(np.max(np.abs(det_g[win] - det_o[win])))
        # the detector bound of the parity tests holds for dd
        sn2, s = sched[lev]["sigma_norm"] ** 2, sched[lev]["deriv_step"]
        assert dd <= sn2 * (3.0 * LEVEL_TOL / s ** 4 + 1e-7)
        return 2 * dd + C * U * float(np.max(np.abs(det_o[win])))

    note(f"[refine e2e] {W}x{H} seed {seed}: {len(common)} common extrema")
    n_pos, _ = check_rows(got, ref, det_o, kps, coef_err, "end-to-end")
    assert n_pos >= len(common) // 2
