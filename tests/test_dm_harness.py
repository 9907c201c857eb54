"""The benchmarking definitions of Sec. V-A (Dolan-More performance ratios
and profile, shifted geometric mean) on hand-computed cases, and the LASSO
family generator of Sec. V-C against its stated sizes and conditioning."""
import math

import numpy as np

import bench
from paper_1903_06477_amd import generators as G

INF = math.inf


def test_performance_ratios_and_profile():
    T = [[1.0, 2.0, INF], [3.0, 3.0, 6.0], [INF, INF, INF]]
    R = bench.performance_ratios(T)
    np.testing.assert_array_equal(R, [[1.0, 2.0, INF], [1.0, 1.0, 2.0], [INF, INF, INF]])
    rho = bench.performance_profile(R, [1.0, 2.0, 1e9])
    np.testing.assert_allclose(rho, [[2 / 3, 1 / 3, 0.0], [2 / 3, 2 / 3, 1 / 3], [2 / 3, 2 / 3, 1 / 3]])


def test_shifted_geometric_mean():
    # a failure counts as 100 x the largest finite time (3 -> 300)
    got = bench.shifted_geometric_mean([1.0, 3.0, INF], 10.0)
    assert abs(got - ((11.0 * 13.0 * 310.0) ** (1.0 / 3.0) - 10.0)) <= 1e-12
    # times below 1 with no shift: every log term is ln 1
    assert bench.shifted_geometric_mean([0.2, 0.5], 0.0) == 1.0
    # a single problem: sgm reduces to the time itself (for sigma + t >= 1)
    assert abs(bench.shifted_geometric_mean([7.5], 10.0) - 7.5) <= 1e-12


def test_lasso_family_sizes_and_conditioning():
    for n, kap in [(631, 215.0), (1000, 1e5)]:
        p = G.lasso_dm_instance(n, kap, 0.1, seed=3)
        Ad = p.meta["Ad"].toarray()
        md = math.ceil(n / 5)
        assert Ad.shape == (md, n)
        s = np.linalg.svd(Ad, compute_uv=False)
        assert abs(s[0] - 1.0) <= 1e-12 and abs(s[0] / s[-1] / kap - 1.0) <= 1e-8
        assert p.A.shape == (2 * n + md + 2, 2 * n + 1) and p.cone.q == [md + 2] and p.cone.l == 2 * n
    fam = G.lasso_dm_family(1)
    assert len(fam) == 48
    assert sorted({f.meta["n_data"] for f in fam}) == [631, 1000, 1585, 2512]
    assert sorted({f.meta["mu"] for f in fam}) == [0.01, 0.1, 1.0]
