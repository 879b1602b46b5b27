"""T1/T2 oracle, pinned to the pad-cone closed form and to exhaustive plan-tree search."""
import numpy as np
import pytest

from oracle import dp
from oracle import enumerate as en


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 3, 3), (2, 3, 4), (4, 4, 2), (4, 3, 3)])
def test_t2_equals_exhaustive_tree_optimum(shape):
    rng = np.random.default_rng(sum(shape))
    for trial in range(8):
        T0 = rng.uniform(0.5, 20.0, size=shape)
        if trial % 2:       # landscape-like: time grows with volume plus noise
            g = np.meshgrid(*[np.arange(1, n + 1) for n in shape], indexing="ij")
            T0 = 1.0 + 0.2 * g[0] * g[1] * g[2] + rng.uniform(0, 3, size=shape)
        T1, T2, act, arg = dp.tables(T0)
        assert np.allclose(T2, en.best_over_trees(T0), rtol=0, atol=1e-12)


def test_t1_is_the_pad_cone_minimum():
    rng = np.random.default_rng(3)
    for _ in range(10):
        T0 = rng.uniform(1, 9, size=(5, 4, 6))
        T1, target = dp.t1_pad(T0)
        assert np.array_equal(T1, en.pad_cone_min(T0))
        # the recorded target realises the value and dominates the cell
        for s in np.ndindex(T0.shape):
            t = np.unravel_index(target[s], T0.shape)
            assert T0[t] == T1[s] and all(t[a] >= s[a] for a in range(3))


def test_invariants_monotone_and_subadditive():
    rng = np.random.default_rng(4)
    T0 = rng.uniform(1, 9, size=(6, 6, 6))
    T1, T2, act, arg = dp.tables(T0)
    assert np.all(T2 <= T1) and np.all(T1 <= T0)
    for X in (T1, T2):
        for ax in range(3):
            assert np.all(np.diff(X, axis=ax) >= 0)          # larger problems never cheaper
    for m in range(6):
        for i in range(1, m + 1):
            if m + 1 - i >= 1:
                assert T2[m, 2, 3] <= T2[i - 1, 2, 3] + T2[m - i, 2, 3] + 1e-12


def test_strictly_increasing_affine_time_never_pads_or_splits():
    g = np.meshgrid(*[np.arange(1, 6)] * 3, indexing="ij")
    T0 = 0.7 * g[0] * g[1] * g[2] + 3.0      # overhead 3 > 0: splitting costs an extra 3
    T1, T2, act, arg = dp.tables(T0)
    assert np.array_equal(T1, T0) and np.array_equal(T2, T0)
    assert np.all(act == dp.AS_IS)


def test_pure_volume_time_prefers_nothing_but_ties_keep_as_is():
    g = np.meshgrid(*[np.arange(1, 5)] * 3, indexing="ij")
    T0 = (g[0] * g[1] * g[2]).astype(np.float64)   # splits cost exactly the same: tie
    T1, T2, act, arg = dp.tables(T0)
    assert np.array_equal(T2, T0) and np.all(act == dp.AS_IS)


def test_plan_leaves_tile_the_problem_and_sum_to_t2():
    rng = np.random.default_rng(5)
    T0 = rng.uniform(1, 9, size=(5, 5, 5))
    T1, T2, act, arg = dp.tables(T0)
    for cell in np.ndindex(T0.shape):
        leaves = dp.plan_leaves(T0.shape, act, arg, cell)
        cover = np.zeros((cell[0] + 1, cell[1] + 1, cell[2] + 1), dtype=int)
        cost = 0.0
        for (m0, n0, k0, m, n, k, run) in leaves:
            cover[m0:m0 + m, n0:n0 + n, k0:k0 + k] += 1
            assert all(run[a] >= (m, n, k)[a] - 1 for a in range(3))
            cost += T0[run]
        assert np.all(cover == 1)
        assert abs(cost - T2[cell]) < 1e-9


def test_planted_mistake_missing_k_split_is_caught():
    # a DP that forgets the K term disagrees with the exhaustive optimum on some grid
    def broken(T1, target):
        T2 = T1.copy()
        n = T1.shape
        for m in range(n[0]):
            for nn in range(n[1]):
                for k in range(n[2]):
                    for i in range(1, m + 1):
                        T2[m, nn, k] = min(T2[m, nn, k], T2[m - i, nn, k] + T2[i - 1, nn, k])
                    for j in range(1, nn + 1):
                        T2[m, nn, k] = min(T2[m, nn, k], T2[m, nn - j, k] + T2[m, j - 1, k])
        return T2
    rng = np.random.default_rng(6)
    caught = False
    for _ in range(20):
        T0 = rng.uniform(0.5, 20.0, size=(3, 3, 3))
        T1, tgt = dp.t1_pad(T0)
        if not np.allclose(broken(T1, tgt), en.best_over_trees(T0)):
            caught = True
            break
    assert caught


def test_planted_mistake_wrong_pad_direction_is_caught():
    rng = np.random.default_rng(7)
    T0 = rng.uniform(1, 9, size=(4, 4, 4))
    wrong = T0.copy()        # "padding" toward smaller sizes
    for s in np.ndindex(T0.shape):
        wrong[s] = T0[:s[0] + 1, :s[1] + 1, :s[2] + 1].min()
    assert not np.array_equal(wrong, en.pad_cone_min(T0))
    assert np.array_equal(dp.t1_pad(T0)[0], en.pad_cone_min(T0))
