"""Structure of the seeded operator generators used by the SpMV cases
(input only: they hold none of the method's arithmetic)."""
import numpy as np

from paper_1903_06477_amd import generators as G


def test_spmv_ragged_rows_are_sorted_distinct_and_span_the_range():
    p = G.spmv_ragged(5000, 64, 12, seed=3)
    A = p.A
    lens = np.diff(A.indptr)
    assert lens.min() == 0 and lens.max() == 12            # empty rows and full rows both occur
    assert abs(lens.mean() - 6.0) < 0.3
    for i in range(A.shape[0]):
        c = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert np.all(np.diff(c) > 0) and (c.size == 0 or (c[0] >= 0 and c[-1] < 64))
    q = G.spmv_ragged(5000, 64, 12, seed=3)
    assert np.array_equal(q.A.indices, A.indices) and np.array_equal(q.A.data, A.data)


def test_spmv_scaled_rows_have_the_stated_length():
    p = G.spmv_scaled(m=300, n=50, per_row=7, seed=1)
    assert np.all(np.diff(p.A.indptr) == 7)
    for i in range(300):
        c = p.A.indices[7 * i:7 * i + 7]
        assert np.all(np.diff(c) > 0) and c[-1] < 50
