"""Pins of the oracle's step-rule comparison variant and best-iterate selection (section 4.B):
special cases that reduce to the literal rule, resumption, and the kept image equals a plain run of
the recorded length."""
import numpy as np

import oracle
from paper_1903_10088_amd import phantom as ph

G = ph.Geometry(n=37, pixel_mm=10.0, n_views=33, n_channels=51, start_angle_rad=0.3)


def slice_():
    return ph.make_slice(G, 5, 5e3, supersample=1)


def test_same_subset_comparison_is_literal_with_one_subset():
    sl = slice_()
    a, ta = oracle.os_iterate(G, 1, 1e-3, sl.counts, sl.i0, None, 9)
    b, tb = oracle.os_iterate(G, 1, 1e-3, sl.counts, sl.i0, None, 9, params=dict(lambda_compare=1))
    assert np.array_equal(a, b) and np.array_equal(ta, tb)


def test_same_subset_comparison_keeps_the_first_epoch():
    sl = slice_()
    M = 5
    _, ta = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, 12)
    _, tb = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, 12, params=dict(lambda_compare=1))
    assert np.array_equal(ta[:M], tb[:M])
    assert not np.array_equal(ta[:, 1], tb[:, 1])  # later decisions do differ on this data
    # each later decision follows the same subset's f one epoch earlier
    for n in range(M, 12):
        step = tb[n, 1] - tb[n - 1, 1]
        expect = 1e-4 if tb[n, 0] < tb[n - M, 0] else -2e-4
        assert abs(step - expect) < 1e-15 or tb[n, 1] == 1e-4


def test_same_subset_comparison_resumes():
    sl = slice_()
    M, p = 5, dict(lambda_compare=1)
    a, ta = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, 17, params=p)
    st, h = oracle.State(), np.zeros(M)
    b, t1 = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, 8, state=st, params=p, f_hist=h)
    b, t2 = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, b, 9, state=st, params=p, f_hist=h)
    # (the image crosses the call boundary in 1/mm: x / 10 * 10 is not always x in FP64)
    t = np.concatenate([t1, t2])
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(t[:, 0], ta[:, 0], rtol=1e-12)
    assert np.array_equal(t[:, 1], ta[:, 1])


def test_best_iterate_is_a_plain_run_of_its_length():
    sl = slice_()
    M, n = 5, 40
    best = np.zeros((G.n, G.n))
    st = oracle.State()
    final, tr = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, n, state=st, params=dict(keep_best=1),
                                  best=best)
    assert st.best_n % M == 0 and M <= st.best_n <= n
    sums = tr[:, 0].reshape(-1, M).sum(axis=1)
    assert st.best_f == sums.min() and st.best_n == M * (int(np.argmin(sums)) + 1)
    plain, _ = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, st.best_n)
    assert np.array_equal(best, plain)
    # one epoch: the kept image is the final one
    b1 = np.zeros((G.n, G.n))
    f1, _ = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, M, params=dict(keep_best=1), best=b1)
    assert np.array_equal(b1, f1)


def test_best_iterate_survives_a_split_run():
    sl = slice_()
    M, p = 5, dict(keep_best=1)
    b_all, st_all = np.zeros((G.n, G.n)), oracle.State()
    oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, 33, state=st_all, params=p, best=b_all)
    b, st = np.zeros((G.n, G.n)), oracle.State()
    img, _ = oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, None, 13, state=st, params=p, best=b)
    oracle.os_iterate(G, M, 1e-3, sl.counts, sl.i0, img, 20, state=st, params=p, best=b)
    np.testing.assert_allclose(b, b_all, rtol=1e-12, atol=1e-18)
    assert st.best_n == st_all.best_n and abs(st.best_f - st_all.best_f) <= 1e-12 * st_all.best_f
