"""Pins of the oracle of Algorithm 4.4 (fast randomized LU, Section 4.5) and
of its parts: the SRFT of Section 3.3 (here with the real Hartley transform,
a reading) and the interpolative decomposition of Section 3.4.

  * the draws: signs are +1 / -1 and balanced, the selection is l distinct
    indices with every index equally likely (chi-square over many seeds);
  * the transform is orthogonal and symmetric and equals Re(FFT) - Im(FFT)
    (NumPy's FFT), so R = D F S has orthonormal columns and A R equals the
    FFT of the rows of A D, subsampled;
  * the ID: Y = X Y(J, :), X(J, :) = I, small entries, and the inequality
    from the proof of the ID lemma, ||A - X A(J, :)|| <= (1 + ||X||) ||A -
    Q Q^T A|| with Q an orthonormal basis of range(Y);
  * the pipeline: exact rank-k reconstruction, Eckart-Young lower bound,
    structure of the factors, B = L_y^+ P X A(J, :) against NumPy least
    squares;
  * planted mistakes (no D, the ID from the first l rows, P left out of
    Step 6) fail these pins.
"""
import numpy as np
import pytest
import scipy.stats

from oracle import fast, philox, rlu
import workloads


def test_signs_are_balanced_plus_minus_one():
    d = philox.srft_signs(100000, 11)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(d.mean()) < 4.0 / np.sqrt(d.size)
    # neighbouring signs uncorrelated
    assert abs(np.mean(d[1:] * d[:-1])) < 4.0 / np.sqrt(d.size)
    # a different seed gives different signs
    assert np.mean(d == philox.srft_signs(100000, 12)) < 0.52


def test_selection_is_distinct_and_uniform():
    n, l = 50, 10
    counts = np.zeros(n)
    first = np.zeros(n)
    for seed in range(2000):
        s = philox.srft_selection(n, l, seed)
        assert len(set(s.tolist())) == l and s.min() >= 0 and s.max() < n
        counts[s] += 1
        first[s[0]] += 1
    # every index equally likely, also in the first position
    assert scipy.stats.chisquare(counts).pvalue > 1e-4
    assert scipy.stats.chisquare(first).pvalue > 1e-4
    # the full draw is a permutation
    assert sorted(philox.srft_selection(37, 37, 3).tolist()) == list(range(37))


@pytest.mark.parametrize("n", [1, 2, 7, 64, 100])
def test_hartley_transform_is_orthogonal_and_is_re_minus_im_of_the_fft(n):
    F = fast.hartley_matrix(n)
    np.testing.assert_allclose(F @ F.T, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(F, F.T, atol=0)
    E = np.fft.fft(np.eye(n), axis=0) / np.sqrt(n)
    np.testing.assert_allclose(F, E.real - E.imag, atol=1e-12)


def test_srft_sketch_equals_the_subsampled_fft_of_the_rows():
    m, n, l = 40, 96, 12
    A = workloads.gaussian((m, n), 21)
    d = philox.srft_signs(n, 22)
    s = philox.srft_selection(n, l, 22)
    R = fast.srft_matrix(n, d, s)
    np.testing.assert_allclose(R.T @ R, np.eye(l), atol=1e-13)
    Fr = np.fft.fft(A * d[None, :], axis=1) / np.sqrt(n)
    np.testing.assert_allclose(A @ R, (Fr.real - Fr.imag)[:, s], atol=1e-12)


def _problem(m=300, n=260, rate=6.0, seed=30):
    return workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), seed)


@pytest.mark.parametrize("k,l", [(8, 16), (15, 45), (30, 40)])
def test_interpolative_decomposition(k, l):
    A = _problem()
    o = fast.fast_randomized_lu_seeded(A, k, l, 31)
    Y, X, J = o["Y"], o["X"], o["J"]
    assert len(set(J.tolist())) == l
    np.testing.assert_allclose(X[J, :], np.eye(l), atol=1e-12)
    np.testing.assert_allclose(X @ Y[J, :], Y, atol=1e-12 * np.abs(Y).max())
    # the LU-based ID keeps its entries small (Section 3.4 bounds a
    # QR-based ID's by 2)
    assert np.abs(X).max() <= 4.0
    Q, _ = np.linalg.qr(Y)
    err_id = np.linalg.norm(A - X @ A[J, :], 2)
    err_range = np.linalg.norm(A - Q @ (Q.T @ A), 2)
    assert err_id <= (1.0 + np.linalg.norm(X, 2)) * err_range * (1 + 1e-10)


def test_exact_rank_reconstruction():
    A = workloads.low_rank_plus_noise(200, 150, 9, 0.0, 32)
    for k, l in ((9, 9), (9, 20)):
        o = fast.fast_randomized_lu_seeded(A, k, l, 33)
        assert rlu.relative_residual(A, o) < 1e-11


def test_error_is_above_eckart_young_and_close_to_the_range_finder():
    A = _problem(rate=5.0, seed=34)
    s = np.linalg.svd(A, compute_uv=False)
    for k, l in ((10, 30), (20, 60)):
        o = fast.fast_randomized_lu_seeded(A, k, l, 35)
        e = rlu.residual(A, o)
        assert e >= s[k] * (1 - 1e-10)
        assert e <= 50 * s[k]


def test_step_6_is_the_least_squares_solution():
    A = _problem(seed=36)
    k, l = 12, 24
    o = fast.fast_randomized_lu_seeded(A, k, l, 37)
    XA = o["X"] @ A[o["J"], :]
    B_ls = np.linalg.lstsq(o["Ly"], XA[o["p"], :], rcond=None)[0]
    np.testing.assert_allclose(o["B"], B_ls, atol=1e-10 * np.abs(B_ls).max())


def test_structure_of_the_factors():
    A = _problem(m=120, n=170, seed=38)
    o = fast.fast_randomized_lu_seeded(A, 10, 18, 39)
    L, U = o["L"], o["U"]
    assert np.all(np.diag(L[:10]) == 1.0) and np.all(np.triu(L[:10], 1) == 0.0)
    assert np.all(np.tril(U, -1) == 0.0)
    np.testing.assert_array_equal(np.sort(o["p"]), np.arange(120))
    np.testing.assert_array_equal(np.sort(o["q"]), np.arange(170))


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_planted_no_sign_flips(monkeypatch):
    good = fast.srft_matrix
    monkeypatch.setattr(fast, "srft_matrix", lambda n, d, s: good(n, np.ones_like(d), s))
    assert _fails(test_srft_sketch_equals_the_subsampled_fft_of_the_rows)


def test_planted_id_from_the_first_rows(monkeypatch):
    good = fast.row_id_from_lu
    monkeypatch.setattr(fast, "row_id_from_lu", lambda Y, p: good(Y, np.arange(Y.shape[0])))
    assert _fails(test_interpolative_decomposition, 15, 45)


def test_planted_step_6_without_p(monkeypatch):
    good = fast.fast_randomized_lu

    def without_p(A, k, l, d, s, step3="partial"):
        o = good(A, k, l, d, s, step3)
        o["B"] = rlu.pinv_apply(o["Ly"], o["X"] @ A[o["J"], :])   # X A(J, :) without P
        return o

    monkeypatch.setattr(fast, "fast_randomized_lu", without_p)
    assert _fails(test_step_6_is_the_least_squares_solution)
