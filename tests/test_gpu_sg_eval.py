"""What the trained surrogate gains, measured against the FP64 oracle.

1. One step at a time: from the oracle's level L_{i-1} and conductivity, the
   trained network's L_i against the oracle's AOS step, next to an untrained
   network of the same architecture and to taking no step at all.
2. The whole surrogate scale space at 1920x1200 with its per-level probe
   check and fallback: error of every level against the oracle's plain scale
   space, the levels that kept the surrogate, and keypoint recall.
"""
import os

import numpy as np
import pytest

import oracle as O
from synthetic import kaze_image, surrogate_params
from kaze_parity import LEVEL_TOL, compare_keypoints, note, recall

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1706_06750_amd", "weights", "surrogate_512.npz")


@pytest.fixture(scope="module")
def trained(gpu_lib):
    from paper_1706_06750_amd import surrogate as S
    from paper_1706_06750_amd import train_surrogate as T
    if not os.path.exists(WEIGHTS):
        pytest.fail("trained surrogate weights missing: %s" % WEIGHTS)
    params, meta = T.load(WEIGHTS)
    return S, params, meta


def step_errors(S, params, lev, gs, sched):
    """Per level i: RMS and max |L_i(net) - L_i(oracle)| with the oracle's
    L_{i-1} and g as inputs (one GPU batch over the 15 steps)."""
    n = len(lev) - 1
    H, W = lev.shape[1:]
    L = torch.from_numpy(lev[:-1].astype(np.float32)).cuda()
    g = torch.from_numpy(gs[1:].astype(np.float32)).cuda()
    tau = torch.tensor([sched[i]["t"] - sched[i - 1]["t"] for i in range(1, n + 1)],
                       dtype=torch.float32, device="cuda")
    w = S.Weights(params)
    plan = S.Plan(n, W, H)
    out = plan.forward(w, L, g, tau).cpu().numpy().astype(np.float64)
    d = out - lev[1:]
    return np.sqrt((d ** 2).mean(axis=(1, 2))), np.abs(d).max(axis=(1, 2))


def test_trained_network_gains_over_untrained_and_no_step(trained):
    S, params, meta = trained
    W = H = 256
    img = kaze_image(W, H, 420000).astype(np.float64)   # not a training image
    lev, k, gs = O.build_scale_space(img, return_g=True)
    sched = O.level_schedule()
    rms_t, max_t = step_errors(S, params, lev, gs, sched)
    rms_u, max_u = step_errors(S, surrogate_params(1), lev, gs, sched)
    d0 = lev[1:] - lev[:-1]
    rms_0, max_0 = np.sqrt((d0 ** 2).mean(axis=(1, 2))), np.abs(d0).max(axis=(1, 2))
    note("[sg eval] per-step RMS error vs FP64 oracle, levels 1..15")
    note("  trained   %s" % " ".join("%.1e" % v for v in rms_t))
    note("  untrained %s" % " ".join("%.1e" % v for v in rms_u))
    note("  no step   %s" % " ".join("%.1e" % v for v in rms_0))
    note("  max: trained %s" % " ".join("%.1e" % v for v in max_t))
    note("  max: no step %s" % " ".join("%.1e" % v for v in max_0))
    # the trained network is better than an untrained one at every level and
    # than no step at all in RMS over the whole scale space
    assert np.all(rms_t < rms_u)
    assert np.sum(rms_t ** 2) < np.sum(rms_0 ** 2)


def test_surrogate_scale_space_1920x1200(trained, gpu_lib):
    """Default check (bound and probe windows of kaze_sg_default_config):
    levels before the first accepted one meet the plain parity bar; every
    level's error against the oracle, the accepted levels and the keypoint
    recall are reported."""
    S, params, meta = trained
    W, H, seed = 1920, 1200, 410000
    w = S.Weights(params)
    ss = S.SurrogateScaleSpace(W, H, w, probe_seed=seed)
    img = kaze_image(W, H, seed)
    ss.img.copy_(torch.from_numpy(img))
    ss.run()
    torch.cuda.synchronize()
    acc = ss.accepted()
    lev_g = ss.levels.cpu().numpy()
    kp_g = ss.keypoints()
    err_probe = ss.err.cpu().numpy()
    lev_o, k_o = O.build_scale_space(img.astype(np.float64))
    det_o = O.detector_response(lev_o)
    kp_o = O.find_extrema(det_o, 0.001)
    errs = [float(np.abs(lev_g[i] - lev_o[i]).max()) for i in range(len(lev_o))]
    common, bad_g, bad_o = compare_keypoints(kp_g, kp_o, det_o, 0.001)
    rc, _, den = recall(kp_g, kp_o, det_o, 0.001)
    note("[sg eval] 1920x1200 seed %d bound %.1e probes %d" % (seed, ss.c.bound, ss.c.probes))
    note("  accepted  %s" % " ".join(str(int(a)) for a in acc))
    note("  probe err %s" % " ".join("%.1e" % e for e in err_probe))
    note("  max|L - L_oracle| %s" % " ".join("%.1e" % e for e in errs))
    note("  keypoints %d / oracle %d, recall %.4f (%d of %d)" % (len(kp_g), len(kp_o), rc,
                                                                  common, den))
    first = next((i for i, a in enumerate(acc) if a), len(acc))
    for i in range(first):
        assert errs[i] <= LEVEL_TOL, i
    if first == len(acc):   # every level fell back: the plain path exactly
        assert not bad_g and not bad_o
    else:                   # the surrogate bar: 1e-3 on every level, 98% recall
        assert max(errs) <= 1e-3, errs
        assert rc >= 0.98, rc
    ss.close()
