"""The library's FED schedule (host code behind kaze_fed_schedule) against
the oracle's: the cycle length, the step sizes of Eq. 5 scaled to the cycle
time and the application order, for the level steps of the default scale
space and for other cycle times.  Runs without a GPU."""
import numpy as np
import pytest

import oracle as O


@pytest.fixture(scope="module")
def K():
    from paper_1706_06750_amd import kaze
    return kaze


def level_taus():
    s = O.level_schedule()
    return [s[i]["t"] - s[i - 1]["t"] for i in range(1, len(s))]


@pytest.mark.parametrize("T", level_taus() + [0.01, 0.1, 0.5, 1.0, 100.0, 300.0])
def test_schedule_matches_oracle(K, T):
    got = np.array(K.kaze_fed_schedule(T))
    tau = O.fed_step_sizes(T)
    want = tau[O.fed_order(tau)]
    assert len(got) == len(want)
    # same order (step sizes are distinct within a cycle), same values
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    assert np.isclose(got.sum(), T, rtol=1e-12)


def test_schedule_rejects_bad_times(K):
    for T in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(K.KazeError):
            K.kaze_fed_schedule(T)
