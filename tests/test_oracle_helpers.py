"""Pins of the oracle's measuring helpers: the spectral-norm estimators that
judge the reduced-precision and full-size cases, the pivot gate that decides
which pivots the FP64 parity rule compares, the condition number, and the
plain power sketch of Section 5.2.

Each helper is pinned against something other than itself: an exact SVD, a
closed form of a matrix built from its singular value decomposition, or
diagnostics constructed to sit on either side of a threshold.  The planted
mistakes at the end (a swapped inverse permutation, too few iterations, an
off-by-one in the gate, a power round with A in place of A^T) must each fail
one of these pins.
"""
import numpy as np
import pytest

from oracle import rlu
import workloads

# ---------------------------------------------------------------------------
# Spectral norm estimates (Section 5.1's relative error uses ||.||_2)
# ---------------------------------------------------------------------------


def _svd_matrix(m, n, sigma, seed):
    """U diag(sigma) V^T with Haar U, V: its singular values are sigma."""
    g = workloads.rng(seed)
    U = workloads.haar(m, g, len(sigma))
    V = workloads.haar(n, g, len(sigma))
    return U, V, (U * sigma) @ V.T


def _norm_cases():
    # (m, n, sigma): a clear top gap, a clustered top (exp(-i/100), slower
    # than the 8192^2 workload's exp(-i/50)) and the paper's slowly
    # decaying spectrum
    return [
        (300, 200, np.r_[3.0, np.linspace(1.0, 0.01, 199)]),
        (250, 400, workloads.exp_decay(250, 100.0)),
        (500, 500, workloads.slow_decay(500) / workloads.slow_decay(1)[0]),
    ]


@pytest.mark.parametrize("case", range(3))
def test_norm_estimate_matches_exact_svd(case):
    m, n, sigma = _norm_cases()[case]
    _, _, A = _svd_matrix(m, n, sigma, 900 + case)
    est = rlu._power_norm(A)
    assert abs(est - sigma[0]) <= 1e-6 * sigma[0], (est, sigma[0])


@pytest.mark.parametrize("shape,k,l,rate", [((400, 300), 20, 25, 30.0),
                                            ((260, 420), 15, 15, 50.0),
                                            ((350, 350), 40, 48, 8.0)])
def test_residual_estimate_matches_exact_svd(shape, k, l, rate):
    m, n = shape
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), 910 + m)
    G = workloads.gaussian((n, l), 911 + n)
    out = rlu.randomized_lu(A, k, l, G)
    E = out["L"] @ out["U"] - A[np.ix_(out["p"], out["q"])]
    exact = np.linalg.svd(E, compute_uv=False)[0]
    est = rlu.residual(A, out, exact=False)
    assert abs(est - exact) <= 1e-6 * exact, (est, exact)
    # and the relative form divides by the same estimate of ||A||_2
    rel = rlu.relative_residual(A, out, exact=False)
    assert abs(rel - exact / np.linalg.norm(A, 2)) <= 1e-6 * rel


def test_norm_estimate_is_a_lower_bound():
    # twelve equal leading singular values (more than the block holds) and
    # a random start: any orthonormal block gives ||E X|| <= ||E||
    sigma = np.r_[np.ones(12), np.linspace(0.999, 0.5, 88)]
    for seed in range(4):
        _, _, A = _svd_matrix(150, 120, sigma, 920 + seed)
        est = rlu.spectral_norm_estimate(lambda X: A @ X, lambda Y: A.T @ Y, 120,
                                         iters=3, seed=seed)
        assert est <= 1.0 * (1 + 1e-12)
        assert est >= 0.5


def test_norm_estimate_of_zero_and_rank_one():
    Z = np.zeros((30, 20))
    assert rlu._power_norm(Z) == 0.0
    u = workloads.gaussian(30, 930)
    v = workloads.gaussian(20, 931)
    R1 = np.outer(u, v)
    assert rlu._power_norm(R1) == pytest.approx(np.linalg.norm(u) * np.linalg.norm(v), rel=1e-13)


def test_residual_operator_products_equal_the_explicit_difference():
    # the operator never forms L U - P A Q; check its products against the
    # formed difference with the index-vector conventions (P A)(i,:) =
    # A(p[i],:) and (A Q)(:,j) = A(:,q[j]), on a case with nontrivial p, q
    A = workloads.spectral_matrix(90, 70, workloads.exp_decay(70, 5.0), 940)
    out = rlu.randomized_lu(A, 6, 9, workloads.gaussian((70, 9), 941))
    assert not np.array_equal(out["p"], np.arange(90))
    assert not np.array_equal(out["q"], np.arange(70))
    E = out["L"] @ out["U"] - A[out["p"]][:, out["q"]]
    mv, rmv, n = rlu.residual_operator(A, out)
    X = workloads.gaussian((70, 3), 942)
    Y = workloads.gaussian((90, 3), 943)
    np.testing.assert_allclose(mv(X), E @ X, rtol=0, atol=1e-13)
    np.testing.assert_allclose(rmv(Y), E.T @ Y, rtol=0, atol=1e-13)
    assert n == 70


# ---------------------------------------------------------------------------
# Pivot gate: which leading pivots two correct implementations must share
# ---------------------------------------------------------------------------

U64 = 2.0 ** -53


def _diag(gaps, mags, max_abs=1.0):
    return {"gap": np.asarray(gaps, float), "piv_abs": np.asarray(mags, float),
            "max_abs": float(max_abs)}


def test_pivot_gate_gap_threshold_is_inclusive():
    g = 1e-8
    assert rlu.pivot_gate(_diag([0.5, g, 0.3], [1, 1, 1])) == 3
    assert rlu.pivot_gate(_diag([0.5, g * (1 - 1e-6), 0.3], [1, 1, 1])) == 1
    assert rlu.pivot_gate(_diag([g * (1 - 1e-6), 0.5, 0.5], [1, 1, 1])) == 0


def test_pivot_gate_magnitude_threshold_scales_with_max_abs():
    M = 7.5
    thr = 1e3 * U64 * M
    assert rlu.pivot_gate(_diag([1, 1, 1, 1], [2, 1, thr, 1], M)) == 4
    assert rlu.pivot_gate(_diag([1, 1, 1, 1], [2, 1, thr * (1 - 1e-9), 1], M)) == 2
    # the threshold is relative: the same magnitudes pass with a smaller max
    assert rlu.pivot_gate(_diag([1, 1, 1, 1], [2, 1, thr * (1 - 1e-9), 1], M / 2)) == 4


def test_pivot_gate_stops_at_the_first_failure():
    # a later step that passes again does not extend the prefix
    d = _diag([1, 1, 0.0, 1, 1], [1, 1, 1, 1, 1])
    assert rlu.pivot_gate(d) == 2
    d = _diag([1, 1, 1, 1, 1], [1, 0.0, 1, 1, 1])
    assert rlu.pivot_gate(d) == 1


def test_pivot_gate_custom_unit_roundoff():
    # the reduced-precision rules pass their own u and gap
    u32 = 2.0 ** -24
    d = _diag([1e-3, 1e-3, 5e-4], [1, 1e3 * u32, 1])
    assert rlu.pivot_gate(d, u=u32, gap_min=1e-3) == 2
    assert rlu.pivot_gate(d, u=u32 * 1.01, gap_min=1e-3) == 1


def test_pivot_gate_on_an_exact_tie_and_on_full_rank():
    # column 0 of Y holds two entries of equal magnitude: step 0 is not
    # decided, so no pivot may be compared
    Y = np.array([[2.0, 1.0], [-2.0, 3.0], [1.0, 0.5], [0.5, 1.0]])
    _, _, _, _, d = rlu.lu_partial_pivot(Y)
    assert d["gap"][0] == 0.0
    assert rlu.pivot_gate(d) == 0
    # a generic Gaussian matrix: every step decided, and the oracle's
    # pivots equal LAPACK getrf's over (at least) the gated prefix
    import scipy.linalg
    X = workloads.gaussian((60, 12), 950)
    _, ipiv, _, _, d = rlu.lu_partial_pivot(X)
    gate = rlu.pivot_gate(d)
    assert gate == 12
    _, ipiv_lapack = scipy.linalg.lu_factor(X)
    np.testing.assert_array_equal(ipiv[:gate], ipiv_lapack[:gate])


def test_pivot_gate_zero_pivot_and_rank_deficiency():
    # an exactly rank-2 block: step 2 meets a (rounded) zero column, whose
    # magnitude is far below 1e3 u max|Y|, so the gate stops at 2
    X = workloads.gaussian((40, 2), 951)
    Y = X @ workloads.gaussian((2, 5), 952)
    _, _, _, _, d = rlu.lu_partial_pivot(Y)
    assert rlu.pivot_gate(d) == 2


# ---------------------------------------------------------------------------
# Condition number (the Gram route of Step 5 loses kappa(L_y)^2 u)
# ---------------------------------------------------------------------------


def test_kappa_closed_forms():
    assert rlu.kappa(np.diag([4.0, 2.0, 0.5])) == pytest.approx(8.0, rel=1e-15)
    Q = workloads.haar(30, workloads.rng(960))
    assert rlu.kappa(Q) == pytest.approx(1.0, rel=1e-13)
    _, _, A = _svd_matrix(50, 20, np.geomspace(1.0, 1e-6, 20), 961)
    assert rlu.kappa(A) == pytest.approx(1e6, rel=1e-8)
    assert rlu.kappa(np.array([[1.0, 2.0], [2.0, 4.0]])) > 1e15


def test_kappa_of_unit_lower_factor_bounds_the_gram_route():
    # with kappa(L_y)^2 u well under 1e-10, the normal equations of the
    # Gram route (the GPU's form of Step 5) agree with the oracle's QR
    # least squares to the FP64 parity tolerance
    A = workloads.spectral_matrix(400, 300, workloads.exp_decay(300, 20.0), 962)
    out = rlu.randomized_lu(A, 30, 36, workloads.gaussian((300, 36), 963))
    Ly = out["Ly"]
    kap = rlu.kappa(Ly)
    assert kap ** 2 * U64 < 1e-10
    S = Ly.T @ Ly
    B_gram = np.linalg.solve(S, Ly.T @ A[out["p"]])
    assert np.abs(B_gram - out["B"]).max() <= 1e-10 * np.abs(out["B"]).max()


# ---------------------------------------------------------------------------
# Section 5.2: the plain power sketch (A A^*)^q A G for small q
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("shape", [(120, 90), (80, 150), (100, 100)])
def test_plain_power_sketch_closed_form(q, shape):
    # with A = U S V^T, (A A^T)^q A G = U S^(2q+1) V^T G
    m, n = shape
    r = min(m, n)
    sigma = np.geomspace(2.0, 0.2, r)
    U, V, A = _svd_matrix(m, n, sigma, 970 + q)
    G = workloads.gaussian((n, 11), 971)
    want = (U * sigma ** (2 * q + 1)) @ (V.T @ G)
    got = rlu.power_sketch_plain(A, G, q)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # the default Step 2 forms the plain product for these q
    np.testing.assert_array_equal(rlu.power_sketch(A, G, q), got)


def test_power_sketch_switches_to_normalized_above_small_q():
    A = workloads.spectral_matrix(70, 60, workloads.exp_decay(60, 6.0), 972)
    G = workloads.gaussian((60, 8), 973)
    q = rlu.PLAIN_POWER_MAX_Q + 1
    np.testing.assert_array_equal(rlu.power_sketch(A, G, q),
                                  rlu.power_sketch_normalized(A, G, q))


@pytest.mark.parametrize("q", [1, 2])
@pytest.mark.parametrize("shape,k,l,rate", [((600, 500), 30, 36, 20.0),
                                            ((300, 700), 20, 24, 15.0)])
def test_normalized_scheme_matches_the_plain_definition(q, shape, k, l, rate):
    # the normalized reading gives the pivots and factors of the plain
    # product at sizes where the plain product is well conditioned
    m, n = shape
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), 974 + q)
    G = workloads.gaussian((n, l), 975)
    a = rlu.randomized_lu(A, k, l, G, q=q, scheme="plain")
    b = rlu.randomized_lu(A, k, l, G, q=q, scheme="normalized")
    gy = rlu.pivot_gate(a["diag_y"])
    assert gy >= k
    np.testing.assert_array_equal(a["ipiv"][:gy], b["ipiv"][:gy])
    np.testing.assert_array_equal(a["q"], b["q"])
    Lp = np.empty_like(a["L"]); Lp[a["p"]] = a["L"]
    Ln = np.empty_like(b["L"]); Ln[b["p"]] = b["L"]
    assert np.abs(Lp - Ln).max() <= 1e-10 * np.abs(Lp).max()
    assert np.abs(a["U"] - b["U"]).max() <= 1e-10 * np.abs(a["U"]).max()


# ---------------------------------------------------------------------------
# Planted mistakes in the helpers
# ---------------------------------------------------------------------------


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_planted_swapped_inverse_permutations(monkeypatch):
    good = rlu.residual_operator

    def swapped(A, out):
        o = dict(out)
        p, q = out["p"], out["q"]
        qinv = np.empty_like(q); qinv[q] = np.arange(q.size)
        pinv = np.empty_like(p); pinv[p] = np.arange(p.size)
        o["p"], o["q"] = pinv, qinv      # p^{-1} and q^{-1} in place of p and q
        return good(A, o)

    monkeypatch.setattr(rlu, "residual_operator", swapped)
    assert _fails(test_residual_estimate_matches_exact_svd, (400, 300), 20, 25, 30.0)


def test_planted_too_few_iterations(monkeypatch):
    good = rlu.spectral_norm_estimate

    def short(mv, rmv, n, iters=60, block=8, seed=0):
        return good(mv, rmv, n, iters=2, block=block, seed=seed)

    monkeypatch.setattr(rlu, "spectral_norm_estimate", short)
    assert _fails(test_norm_estimate_matches_exact_svd, 1)


def test_planted_single_vector_power_iteration(monkeypatch):
    # a single-vector power iteration: 60 steps do not resolve the
    # exp(-i/100) cluster to 1e-6
    good = rlu.spectral_norm_estimate

    def single(mv, rmv, n, iters=60, block=8, seed=0):
        return good(mv, rmv, n, iters=iters, block=1, seed=seed)

    monkeypatch.setattr(rlu, "spectral_norm_estimate", single)
    assert _fails(test_norm_estimate_matches_exact_svd, 1)


@pytest.mark.parametrize("variant", ["one_past", "strict_gap", "strict_mag", "no_max_scale"])
def test_planted_gate_mistakes(variant, monkeypatch):
    def gate(diag, u=U64, gap_min=1e-8, mag_factor=1e3):
        thr = mag_factor * u * (1.0 if variant == "no_max_scale" else diag["max_abs"])
        n = 0
        for g, a in zip(diag["gap"], diag["piv_abs"]):
            bad_gap = g <= gap_min if variant == "strict_gap" else g < gap_min
            bad_mag = a <= thr if variant == "strict_mag" else a < thr
            if bad_gap or bad_mag:
                return n + 1 if variant == "one_past" else n
            n += 1
        return n

    monkeypatch.setattr(rlu, "pivot_gate", gate)
    assert (_fails(test_pivot_gate_gap_threshold_is_inclusive)
            or _fails(test_pivot_gate_magnitude_threshold_scales_with_max_abs)
            or _fails(test_pivot_gate_stops_at_the_first_failure))


@pytest.mark.parametrize("variant", ["a_not_at", "one_round_short", "extra_round"])
def test_planted_plain_power_mistakes(variant, monkeypatch):
    def plain(A, G, q):
        Y = A @ G
        rounds = {"one_round_short": q - 1, "extra_round": q + 1}.get(variant, q)
        for _ in range(max(rounds, 0)):
            Y = A @ (A @ Y) if variant == "a_not_at" else A @ (A.T @ Y)
        return Y

    monkeypatch.setattr(rlu, "power_sketch_plain", plain)
    assert _fails(test_plain_power_sketch_closed_form, 1, (100, 100))


def test_planted_normalized_without_unpermute(monkeypatch):
    def no_unpermute(X):
        LU, _, _, _, _ = rlu.lu_partial_pivot(X)
        return rlu.unit_lower(LU, X.shape[1])

    monkeypatch.setattr(rlu, "lu_normalize", no_unpermute)
    assert _fails(test_normalized_scheme_matches_the_plain_definition, 1, (600, 500), 30, 36, 20.0)
