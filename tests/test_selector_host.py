"""Host logic of the selector (no GPU): the threshold calibrated on the
step's critical path against a brute force over every threshold, and a case
where summing per-block costs picks the wrong rule."""
import numpy as np

from paper_2308_06484_amd import selector as S


def _cp_brute(X, Y, step, tau):
    cost = np.where(X[:, 3] > tau, np.exp2(Y[:, 1]), np.exp2(Y[:, 0])).astype(np.float64)
    return sum(cost[step == t].max() for t in np.unique(step))


def test_critical_path_threshold_is_optimal_among_thresholds():
    rng = np.random.default_rng(0)
    for trial in range(20):
        m = int(rng.integers(5, 60))
        X = np.zeros((m, 16), np.float32)
        X[:, 3] = rng.integers(0, 30, size=m)
        Y = rng.uniform(1, 12, size=(m, 2)).astype(np.float32)
        step = np.sort(rng.integers(0, 6, size=m))
        tau = S.calibrate_threshold_cp(X, Y, step, candidates=4096)
        got = _cp_brute(X, Y, step, tau)
        best = min(_cp_brute(X, Y, step, t) for t in list(np.unique(X[:, 3])) + [-1.0, 1e9])
        assert np.isclose(got, best), trial


def test_summed_costs_pick_a_rule_that_slows_the_step():
    # one step, two blocks with the same feature: rebuilding both saves
    # summed cost (141 < 150) but makes the slowest block slower (140 > 100)
    X = np.zeros((2, 16), np.float32)
    X[:, 3] = 10.0
    Y = np.log2(np.array([[100.0, 1.0], [50.0, 140.0]])).astype(np.float32)
    step = np.array([0, 0])
    assert S.calibrate_threshold(X, Y) < 10.0          # rebuild both
    assert S.calibrate_threshold_cp(X, Y, step) >= 10.0  # repair both
    assert np.isclose(S.step_time(np.array([100.0, 50.0]), step), 100.0)


def test_rebuilds_after_the_kernel_add_to_the_step():
    # two blocks whose rebuilds run after the step's kernel: their costs add
    # to the slowest block that stays in the kernel
    step = np.array([0, 0, 0])
    cost = np.array([100.0, 30.0, 50.0])
    after = np.array([False, True, True])
    assert np.isclose(S.step_time(cost, step, after), 100.0 + 50.0)
    assert np.isclose(S.step_time(cost, step), 100.0)


def test_ties_keep_the_largest_threshold():
    # no rebuild pays: every threshold at or above the largest feature
    # value is optimal, and the largest candidate (rebuild nothing, also on
    # unseen larger values) is kept rather than the largest observed value
    X = np.zeros((3, 16), np.float32)
    X[:, 3] = [1.0, 5.0, 17.25]
    Y = np.log2(np.array([[10.0, 900.0], [20.0, 800.0], [30.0, 700.0]])).astype(np.float32)
    step = np.array([0, 0, 1])
    tau = S.calibrate_threshold_cp(X, Y, step, np.ones(3, bool))
    assert tau > 17.25
    # no rebuild paid on the samples: the rule never rebuilds
    assert tau == S.NEVER and not (np.float32(1e30) > np.float32(tau))


def test_dlimit_feature_calibrates_on_its_own_column():
    X = np.zeros((4, 16), np.float32)
    X[:, 3] = [1.0, 1.0, 1.0, 1.0]
    X[:, 15] = [0.5, 0.7, 3.0, 4.0]
    # the two blocks that move farthest relative to d are cheaper rebuilt
    Y = np.log2(np.array([[10.0, 50.0], [10.0, 50.0], [400.0, 20.0], [400.0, 20.0]])).astype(np.float32)
    step = np.array([0, 1, 2, 3])
    tau = S.calibrate_threshold_cp(X, Y, step, feature=15)
    assert 0.7 <= tau < 3.0
