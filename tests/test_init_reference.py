"""Host checks of the initial-centroid re-implementations themselves (no
GPU): published SplitMix64 outputs, permutation properties of the two
shuffles, and k-means++ weighting on cases with a known answer."""
import json
import os

import numpy as np

from tests import init_reference as ir

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_matches_published_outputs():
    g = json.load(open(os.path.join(GOLD, "splitmix64_seed0.json")))
    outs = [int(v, 16) for v in g["first_outputs_hex"]]
    assert ir.splitmix64_stream(0, len(outs)) == outs


def test_shuffles_give_distinct_rows_and_full_permutations():
    for n, k, seed in [(10, 10, 1), (1000, 37, 5), (7, 3, 123)]:
        for f in (ir.forgy_rows, ir.shuffle_first_k_rows):
            r = f(n, k, seed)
            assert len(set(r)) == k and all(0 <= x < n for x in r)
    # k = n: the front-to-back shuffle is a permutation of 0..n-1
    assert sorted(ir.shuffle_first_k_rows(50, 50, 9)) == list(range(50))
    assert sorted(ir.forgy_rows(50, 50, 9)) == list(range(50))


def test_kmeanspp_never_picks_a_zero_weight_point():
    # two tight groups far apart: after the first pick, the second must come
    # from the other group (points of the first group weigh floor(0) = 0)
    X = np.zeros((200, 2))
    X[100:] = 1e6
    for seed in range(20):
        r = ir.kmeanspp_rows(X, 2, seed)
        assert (r[0] < 100) != (r[1] < 100)


def test_kmeanspp_degenerate_data_draws_uniformly():
    X = np.zeros((64, 3))                    # every weight is zero after one pick
    rows = ir.kmeanspp_rows(X, 5, 7)
    rs = ir.splitmix64_stream(7, 5)
    assert rows == [(r * 64) >> 64 for r in rs]


def test_kmeanspp_weights_follow_squared_distance():
    # points at distances 1, 2, 3 from the first centre (the origin, forced by
    # picking with n=4 and a seed whose first draw selects row 0): weights are
    # exactly proportional to 1 : 4 : 9
    X = np.array([[0.0], [1.0], [2.0], [3.0]])
    seed = next(s for s in range(1000) if (ir.splitmix64_stream(s, 1)[0] * 4) >> 64 == 0)
    rs = ir.splitmix64_stream(seed, 2)
    rows = ir.kmeanspp_rows(X, 2, seed)
    assert rows[0] == 0
    # B = 61, M = 9 < 2^4: w = D * 2^57 exactly; W = 14 * 2^57
    W = 14 << 57
    q = (rs[1] * W) >> 64
    expect = 1 if q < (1 << 57) else (2 if q < (5 << 57) else 3)
    assert rows[1] == expect
