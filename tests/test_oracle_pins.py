"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (never against the oracle itself).

Each test names what it pins.  A plausible slip in the oracle (a dropped
term, a wrong sign or index, a transposed operand, a wrong pivot rule) makes
at least one of them fail; ``test_planted_mistakes_are_caught`` checks that
claim for a set of deliberately broken copies of the oracle's steps.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats
import sympy

from oracle import bounds, philox, rlu
import workloads

# ---------------------------------------------------------------------------
# Table 4.1 (Section 4): success probability of Theorem 4.1
# ---------------------------------------------------------------------------


def _read_table(path):
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a, b, c, d = line.split()
            rows.append((int(a), float(b), float(c), float(d)))
    return rows


def test_table_4_1_reproduces(golden_dir):
    rows = _read_table(os.path.join(golden_dir, "table_4_1.txt"))
    assert len(rows) == 9
    for lk, beta, gamma, printed in rows:
        got = bounds.one_minus_xi(lk, beta, gamma, n=1000)
        # the table prints two significant digits, sometimes rounded
        # (5.17e-16 -> 5.2e-16) and sometimes truncated (5.25e-8 -> 5.2e-8):
        # allow one unit of the last printed digit
        e = math.floor(math.log10(printed))
        assert abs(got - printed) <= 0.1001 * 10.0 ** e, (lk, beta, gamma, got, printed)


def test_xi_second_term_negligible_in_n():
    # the paper omits n from Table 4.1 because the gamma term decays fast
    a = bounds.one_minus_xi(5, 5, 5, n=200)
    b = bounds.one_minus_xi(5, 5, 5, n=20000)
    assert a == pytest.approx(b, rel=1e-12)


def test_theorem_bound_constant_grows_as_stated():
    # C(n,k,l) = 2 sqrt(2 n l b^2 g^2 + 1) + 2 sqrt(2 n l) b g (k(n-k)+1)
    c = bounds.rand_lu_bound(n=100, k=10, l=15, beta=1.0, gamma=2.0)
    exp = 2 * math.sqrt(2 * 100 * 15 * 4 + 1) + 2 * math.sqrt(3000) * 2 * (10 * 90 + 1)
    assert c == pytest.approx(exp, rel=1e-15)


# ---------------------------------------------------------------------------
# Step 1: Philox4x32-10 + Box-Muller
# ---------------------------------------------------------------------------


def test_philox_known_answers(golden_dir):
    with open(os.path.join(golden_dir, "philox_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        vals = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*vals[:6])
        assert [int(x) for x in out] == vals[6:]


def test_box_muller_closed_forms():
    # u1 = 2^-53 (all-zero words), u2 = 0  ->  z0 = sqrt(2*53*ln 2), z1 = 0
    z0, z1 = philox.box_muller(0, 0, 0, 0)
    assert float(z0) == pytest.approx(math.sqrt(2 * 53 * math.log(2.0)), rel=1e-15)
    assert float(z1) == 0.0
    # u1 = 1 (all-one low words) -> r = 0
    z0, z1 = philox.box_muller(0xFFFFFFFF, 0xFFFFFFFF, 0x12345678, 0x9ABCDEF0)
    assert float(z0) == 0.0 and float(z1) == 0.0
    # u2 = 1/4 -> theta = pi/2: z0 ~ 0, z1 = r
    z0, z1 = philox.box_muller(0, 0x80000000, 0, 0x40000000)  # u1 = 1/2
    r = math.sqrt(-2.0 * math.log(0.5))
    assert abs(float(z0)) < 1e-15 and float(z1) == pytest.approx(r, rel=1e-15)


def test_gaussian_matrix_distribution():
    G = philox.gaussian_matrix(1000, 97, seed=7202)
    assert G.shape == (1000, 97)
    x = G.ravel()
    assert abs(x.mean()) < 5.0 / math.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5.0 * math.sqrt(2.0 / x.size)
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-3
    # columns are uncorrelated
    C = np.corrcoef(G[:, :8].T)
    assert np.max(np.abs(C - np.eye(8))) < 0.15


def test_gaussian_matrix_column_major_counter():
    # element (i, j) uses pair index (i + j n) // 2
    n, l, seed = 7, 3, 99
    G = philox.gaussian_matrix(n, l, seed)
    e = 2 + 1 * n          # (i=2, j=1): e = 9 -> pair 4, odd -> z1
    x = philox.philox4x32_10(4, 0, 0, 0, seed, 0)
    z0, z1 = philox.box_muller(*x)
    assert G[2, 1] == float(z1)
    assert e % 2 == 1


def test_gaussian_seeds_differ():
    a = philox.gaussian_matrix(64, 4, 1)
    b = philox.gaussian_matrix(64, 4, 2)
    assert not np.allclose(a, b)


# ---------------------------------------------------------------------------
# Step 3: partial-pivot LU of Y
# ---------------------------------------------------------------------------


def test_lu_partial_pivot_equals_lapack_getrf():
    Y = workloads.gaussian((300, 40), 5)
    LU, ipiv, p, info, _ = rlu.lu_partial_pivot(Y)
    lu_ref, piv_ref = scipy.linalg.lu_factor(Y)
    assert info == 0
    np.testing.assert_array_equal(ipiv, piv_ref)
    np.testing.assert_allclose(LU, lu_ref, rtol=0, atol=1e-13 * np.abs(lu_ref).max())
    # P Y = L U
    L = np.tril(LU, -1)[:, :40] + np.eye(300, 40)
    U = np.triu(LU[:40])
    np.testing.assert_allclose(L @ U, Y[p], atol=1e-13 * np.abs(Y).max())


def _exact_schur_pivots(Yint):
    """Closed-form partial pivoting: the pivot of step j maximizes the
    magnitude of the Schur complement column  Y[i,j] - Y[i,:j] Y[R,:j]^{-1} Y[R,j]
    over the rows not yet chosen (R = rows chosen so far), in exact rationals.
    Returns the chosen original rows and the exact packed L, U values."""
    m, w = Yint.shape
    Ys = sympy.Matrix(Yint.tolist())
    chosen = []
    U = {}
    Lmult = {}
    for j in range(w):
        R = chosen[:]
        if j:
            Y11inv = Ys.extract(R, list(range(j))).inv()
        best, best_i, vals = None, None, {}
        for i in range(m):
            if i in R:
                continue
            s = Ys[i, j]
            if j:
                s -= (Ys.extract([i], list(range(j))) * Y11inv * Ys.extract(R, [j]))[0, 0]
            vals[i] = s
            if best is None or abs(s) > best:
                best, best_i = abs(s), i
        # the test inputs are chosen so that the maximum is unique
        assert sum(1 for v in vals.values() if abs(v) == best) == 1
        chosen.append(best_i)
        piv = vals[best_i]
        for i, s in vals.items():
            if i != best_i:
                Lmult[(i, j)] = s / piv
        for c in range(j, w):
            s = Ys[best_i, c]
            if j:
                s -= (Ys.extract([best_i], list(range(j))) * Y11inv * Ys.extract(R, [c]))[0, 0]
            U[(j, c)] = s
    return chosen, U, Lmult


def _tie_free_int_matrix(shape, seed):
    g = np.random.default_rng(seed)
    while True:
        Y = g.integers(-9, 10, size=shape)
        try:
            _exact_schur_pivots(Y)
            return Y
        except (AssertionError, ValueError, ZeroDivisionError):
            continue


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_lu_partial_pivot_schur_brute_force(seed):
    Y = _tie_free_int_matrix((7, 4), seed)
    chosen, U, Lmult = _exact_schur_pivots(Y)
    LU, ipiv, p, info, _ = rlu.lu_partial_pivot(Y.astype(float))
    assert info == 0
    assert list(p[:4]) == chosen
    for (j, c), v in U.items():
        assert LU[j, c] == pytest.approx(float(v), rel=1e-13, abs=1e-13)
    pos = {int(o): i for i, o in enumerate(p)}
    for (i, j), v in Lmult.items():
        if pos[i] > j:
            assert LU[pos[i], j] == pytest.approx(float(v), rel=1e-13, abs=1e-13)


# ---------------------------------------------------------------------------
# Step 5: least-squares application of the pseudo-inverse
# ---------------------------------------------------------------------------


def test_pinv_apply_equals_lstsq_and_normal_equations():
    Y = workloads.gaussian((200, 12), 11)
    LU, _, p, _, _ = rlu.lu_partial_pivot(Y)
    Ly = rlu.unit_lower(LU, 8)
    A = workloads.gaussian((200, 50), 12)
    B = rlu.pinv_apply(Ly, A[p])
    ref = np.linalg.lstsq(Ly, A[p], rcond=None)[0]
    np.testing.assert_allclose(B, ref, atol=1e-12 * np.abs(ref).max())
    # the paper's Remark: (Ly^T Ly)^{-1} Ly^T PA
    gram = np.linalg.solve(Ly.T @ Ly, Ly.T @ A[p])
    np.testing.assert_allclose(B, gram, atol=1e-10 * np.abs(ref).max())
    # the residual of a least-squares solution is orthogonal to range(Ly)
    res = A[p] - Ly @ B
    assert np.abs(Ly.T @ res).max() < 1e-10 * np.abs(A).max() * 200


# ---------------------------------------------------------------------------
# Step 6: column-pivoted LU of B
# ---------------------------------------------------------------------------


def test_lu_col_pivot_equals_getrf_of_transpose():
    B = workloads.gaussian((25, 300), 21)
    Lb, Ub, qpiv, q, info, _ = rlu.lu_col_pivot(B)
    lu_t, piv_t = scipy.linalg.lu_factor(B.T)
    assert info == 0
    np.testing.assert_array_equal(qpiv, piv_t)
    # getrf(B^T) = L' U'  ->  L_b = U'^T D^{-1}, U_b = D L'^T
    Lp = np.tril(lu_t, -1)[:, :25] + np.eye(300, 25)
    Up = np.triu(lu_t[:25])
    D = np.diag(Up)
    np.testing.assert_allclose(Lb, Up.T / D, atol=1e-12)
    np.testing.assert_allclose(Ub, D[:, None] * Lp.T, atol=1e-12 * np.abs(B).max())
    np.testing.assert_allclose(Lb @ Ub, B[:, q], atol=1e-12 * np.abs(B).max())


@pytest.mark.parametrize("seed", [4, 5])
def test_lu_col_pivot_schur_brute_force(seed):
    Bt = _tie_free_int_matrix((7, 4), seed)    # B = Bt^T is 4 x 7
    chosen, U, Lmult = _exact_schur_pivots(Bt)
    Lb, Ub, qpiv, q, info, _ = rlu.lu_col_pivot(Bt.T.astype(float))
    assert list(q[:4]) == chosen
    # U_b(j, c) for the pivot columns = Schur entries of B's rows:
    # the Schur complement of B^T at (row chosen_j, col c) is U'(j,c) and
    # U_b = D L'^T, L_b = U'^T D^{-1}
    for (j, c), v in U.items():
        if c > j:
            assert Lb[c, j] == pytest.approx(float(v / U[(j, j)]), rel=1e-13, abs=1e-13)
        else:
            assert Ub[j, j] == pytest.approx(float(v), rel=1e-13)


# ---------------------------------------------------------------------------
# The whole of Algorithm 4.1
# ---------------------------------------------------------------------------


def _run(A, k, l, seed=3):
    G = workloads.gaussian((A.shape[1], l), seed)
    return rlu.randomized_lu(A, k, l, G), G


def test_exact_rank_k_reconstruction():
    A = workloads.low_rank_plus_noise(300, 200, 10, 0.0, 31)
    out, _ = _run(A, 10, 15)
    rel = rlu.relative_residual(A, out)
    assert rel < 1e-13


@pytest.mark.parametrize("shape,k,l", [((120, 90), 7, 12), ((60, 140), 9, 9), ((80, 80), 5, 20)])
def test_structure_of_factors(shape, k, l):
    m, n = shape
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), 4.0), 41)
    out, _ = _run(A, k, l)
    L, U, p, q = out["L"], out["U"], out["p"], out["q"]
    assert L.shape == (m, k) and U.shape == (k, n)
    np.testing.assert_array_equal(np.sort(p), np.arange(m))
    np.testing.assert_array_equal(np.sort(q), np.arange(n))
    # L unit lower trapezoidal, U upper trapezoidal
    np.testing.assert_array_equal(np.diag(L[:k]), np.ones(k))
    assert np.all(np.triu(L[:k], 1) == 0)
    assert np.all(np.tril(U, -1) == 0)
    # partial-pivot multipliers are bounded by one
    assert np.abs(out["Ly"]).max() <= 1.0
    # column pivoting of B: each pivot dominates the rest of its U_b row
    for j in range(k):
        assert abs(U[j, j]) >= np.abs(U[j, j:]).max() * (1 - 1e-15)


@pytest.mark.parametrize("seed", [51, 52, 53])
def test_error_between_eckart_young_and_theorem_4_1(seed):
    m, n, k, l = 150, 120, 10, 15
    sig = workloads.exp_decay(min(m, n), 5.0)
    A = workloads.spectral_matrix(m, n, sig, seed)
    out, _ = _run(A, k, l, seed)
    err = rlu.residual(A, out)
    s = np.linalg.svd(A, compute_uv=False)
    assert err >= s[k] * (1 - 1e-10)                     # best rank-k error
    C = bounds.rand_lu_bound(n, k, l, beta=5.0, gamma=5.0)
    assert err <= C * s[k]                               # Theorem 4.1


def test_projection_identity_of_the_proof():
    # proof of Theorem 4.1: ||LU - PAQ|| = ||L_y L_y^+ PAQ - PAQ||, and with
    # partial pivoting range(L_y(:,1:k)) = P range(A G(:,1:k)), so
    # P^T L U Q^T equals the orthogonal projection of A onto range(A G_k).
    m, n, k, l = 160, 130, 12, 18
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), 6.0), 61)
    out, G = _run(A, k, l, 62)
    p, q = out["p"], out["q"]
    recon = np.empty((m, n))
    recon[np.ix_(p, q)] = out["L"] @ out["U"]
    Qk, _ = np.linalg.qr(A @ G[:, :k])
    proj = Qk @ (Qk.T @ A)
    np.testing.assert_allclose(recon, proj, atol=1e-11 * np.abs(A).max())
    err = rlu.residual(A, out)
    assert err == pytest.approx(np.linalg.norm(A - proj, 2), rel=1e-8)


def test_oversampling_invariance_under_partial_pivoting():
    m, n, k, l = 140, 110, 9, 16
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), 5.0), 71)
    G = workloads.gaussian((n, l), 72)
    full = rlu.randomized_lu(A, k, l, G)
    cut = rlu.randomized_lu(A, k, k, G[:, :k].copy())
    np.testing.assert_array_equal(full["ipiv"][:k], cut["ipiv"][:k])
    np.testing.assert_array_equal(full["q"], cut["q"])
    # unpermuted L and U agree
    Lf = np.empty_like(full["L"]); Lf[full["p"]] = full["L"]
    Lc = np.empty_like(cut["L"]); Lc[cut["p"]] = cut["L"]
    np.testing.assert_allclose(Lf, Lc, atol=1e-12)
    np.testing.assert_allclose(full["U"], cut["U"], atol=1e-12 * np.abs(full["U"]).max())


def test_full_rank_reconstruction():
    m, n = 70, 50
    A = workloads.gaussian((m, n), 81)
    out, _ = _run(A, n, n, 82)
    np.testing.assert_allclose(out["L"] @ out["U"], rlu.permuted(A, out["p"], out["q"]),
                               atol=1e-12 * np.abs(A).max())


def test_identity_sketch_reduces_to_getrf():
    m, n = 90, 40
    A = workloads.gaussian((m, n), 91)
    out = rlu.randomized_lu(A, n, n, np.eye(n))
    lu_ref, piv_ref = scipy.linalg.lu_factor(A)
    np.testing.assert_array_equal(out["ipiv"], piv_ref)
    np.testing.assert_allclose(out["LUy"], lu_ref, atol=1e-13 * np.abs(lu_ref).max())


def test_zero_matrix_and_rank_deficiency_set_info():
    A = np.zeros((30, 20))
    out, _ = _run(A, 4, 6)
    assert out["info"] == (1, 1)
    assert np.all(out["U"] == 0)
    assert np.all(np.diag(out["L"][:4]) == 1)
    # rank one input, k = 2: second pivot of Y is exactly zero
    A = np.zeros((30, 20)); A[3, 5] = 2.0
    out, _ = _run(A, 2, 3)
    assert out["info"][0] == 2
    assert rlu.residual(A, out) == 0.0


def test_small_config_magnitude():
    A, k, l = workloads.config_small(101)
    G = philox.gaussian_matrix(512, l, 7203)
    out = rlu.randomized_lu(A, k, l, G)
    rel = rlu.relative_residual(A, out)
    s = np.linalg.svd(A, compute_uv=False)
    assert s[k] / s[0] * 0.99 <= rel < 1e-6
    assert out["info"] == (0, 0)


# ---------------------------------------------------------------------------
# Section 5.2: power iterations, Y = (A A^*)^q A G with LU normalization
# ---------------------------------------------------------------------------


def _plain_power_sketch(A, G, q):
    """(A A^T)^q A G by plain products, with no normalization."""
    Y = A @ G
    for _ in range(q):
        Y = A @ (A.T @ Y)
    return Y


def test_lu_normalize_equals_lapack_p_times_l():
    # scipy.linalg.lu (LAPACK getrf) gives X = P L U; the normalized block
    # is P L = X U^{-1}, in X's row order
    for seed, shape in ((63, (50, 7)), (64, (31, 31)), (65, (200, 12))):
        X = workloads.gaussian(shape, seed)
        P, Lsc, Usc = scipy.linalg.lu(X)
        N = rlu.lu_normalize(X)
        np.testing.assert_allclose(N, P @ Lsc, rtol=0, atol=1e-13)
        np.testing.assert_allclose(N @ Usc, X, rtol=0, atol=1e-12 * np.abs(X).max())
        assert np.abs(N).max() <= 1.0


@pytest.mark.parametrize("q", [1, 2])
@pytest.mark.parametrize("shape", [(70, 70), (90, 60), (60, 90)])
def test_power_sketch_gives_the_factors_of_the_plain_product(q, shape):
    # each normalization multiplies the block on the right by an upper
    # triangular matrix, so Steps 3-8 on the normalized sketch and on the
    # plain (A A^T)^q A G agree: same pivots, same factors up to rounding
    m, n = shape
    k, l = 6, 9
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), 12.0), 61)
    G = workloads.gaussian((n, l), 62)
    got = rlu.randomized_lu(A, k, l, G, q=q, scheme="normalized")
    ref = rlu.randomized_lu_from_sketch(A, k, _plain_power_sketch(A, G, q))
    np.testing.assert_array_equal(got["ipiv"], ref["ipiv"])
    np.testing.assert_array_equal(got["p"], ref["p"])
    np.testing.assert_array_equal(got["q"], ref["q"])
    np.testing.assert_allclose(got["L"], ref["L"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(got["U"], ref["U"], rtol=0, atol=1e-9 * np.abs(ref["U"]).max())
    # and the sketch spans the same columns as the plain product
    Yp = _plain_power_sketch(A, G, q)
    Qp, _ = np.linalg.qr(Yp)
    np.testing.assert_allclose(Qp @ (Qp.T @ got["Y"]), got["Y"], rtol=0,
                               atol=1e-9 * np.abs(got["Y"]).max())


def test_power_iterations_with_q_zero_are_step_2():
    A = workloads.spectral_matrix(80, 70, workloads.exp_decay(70, 6.0), 66)
    G = workloads.gaussian((70, 10), 67)
    np.testing.assert_array_equal(rlu.power_sketch(A, G, 0), A @ G)
    a, b = rlu.randomized_lu(A, 8, 10, G), rlu.randomized_lu(A, 8, 10, G, q=0)
    np.testing.assert_array_equal(a["L"], b["L"])
    np.testing.assert_array_equal(a["U"], b["U"])


@pytest.mark.parametrize("q", [1, 2, 3])
def test_power_iterations_exact_rank_reconstruction(q):
    A = workloads.low_rank_plus_noise(150, 120, 9, 0.0, 68)
    G = workloads.gaussian((120, 12), 69)
    out = rlu.randomized_lu(A, 9, 12, G, q=q)
    assert rlu.relative_residual(A, out) < 1e-12


def test_power_iterations_lower_the_error_on_slow_decay():
    # Section 5.2: on sigma_j = 100 / (9 + j)^2 the error falls with q and
    # never drops below sigma_{k+1} (Eckart-Young)
    m, n, k, l = 240, 200, 15, 20
    sig = workloads.slow_decay(n)
    sig = sig / sig[0]
    A = workloads.spectral_matrix(m, n, sig, 70)
    errs = []
    for q in (0, 1, 2, 3):
        G = workloads.gaussian((n, l), 71)
        errs.append(rlu.relative_residual(A, rlu.randomized_lu(A, k, l, G, q=q)))
    assert errs[1] < 0.8 * errs[0]
    assert errs[2] < errs[1]
    assert errs[3] < errs[2]          # q = 3 takes the normalized scheme
    assert min(errs) >= sig[k] * (1 - 1e-9)


# ---------------------------------------------------------------------------
# Algorithm 4.3: rank-deficient least squares on the factors
# ---------------------------------------------------------------------------


def _rank_k_problem(m, n, k, seed):
    A = workloads.low_rank_plus_noise(m, n, k, 0.0, seed)
    G = workloads.gaussian((n, k + 4), seed + 1)
    return A, rlu.randomized_lu(A, k, k + 4, G)


def test_lstsq_consistent_system_is_solved_with_k_nonzeros():
    # rank(A) = k and b in range(A): the minimum of ||A x - b|| is 0, and x
    # has at most k nonzero entries (the remark after Algorithm 4.3)
    A, out = _rank_k_problem(150, 110, 8, 81)
    x0 = workloads.gaussian((110, 2), 83)
    b = A @ x0
    x = rlu.lstsq_rank_deficient(out, b)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    assert np.all(np.count_nonzero(x, axis=0) <= 8)
    xv = rlu.lstsq_rank_deficient(out, b[:, 0])
    assert xv.shape == (110,)
    np.testing.assert_allclose(xv, x[:, 0], rtol=0, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("shape,k", [((150, 110), 8), ((90, 140), 12), ((200, 200), 30)])
def test_lstsq_residual_is_the_least_squares_minimum(shape, k):
    # for a general b the residual equals the one of LAPACK's minimum-norm
    # solution (numpy.linalg.lstsq): both minimize ||A x - b|| over all x
    m, n = shape
    A, out = _rank_k_problem(m, n, k, 85 + k)
    b = workloads.gaussian((m, 3), 86 + k)
    x = rlu.lstsq_rank_deficient(out, b)
    xr = np.linalg.lstsq(A, b, rcond=None)[0]
    r = np.linalg.norm(A @ x - b, axis=0)
    rr = np.linalg.norm(A @ xr - b, axis=0)
    np.testing.assert_allclose(r, rr, rtol=1e-10)


def test_lstsq_full_rank_square_is_the_inverse():
    # k = l = m = n: A x = b has the unique solution A^{-1} b
    n = 60
    A = workloads.spectral_matrix(n, n, workloads.exp_decay(n, 40.0), 87)
    out = rlu.randomized_lu(A, n, n, workloads.gaussian((n, n), 88))
    b = workloads.gaussian((n, 2), 89)
    np.testing.assert_allclose(rlu.lstsq_rank_deficient(out, b), np.linalg.solve(A, b),
                               rtol=0, atol=1e-9 * np.abs(np.linalg.solve(A, b)).max())


def test_upper_solve_is_back_substitution():
    U = np.triu(workloads.gaussian((9, 9), 90)) + 4 * np.eye(9)
    y = workloads.gaussian((9, 2), 91)
    np.testing.assert_allclose(rlu.upper_solve(U, y), scipy.linalg.solve_triangular(U, y),
                               rtol=1e-13, atol=1e-13)
    # a zero pivot of Step 6 leaves a zero row of U: its unknown is free, set to 0
    Z = np.array([[2.0, 1.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 4.0]])
    np.testing.assert_allclose(rlu.upper_solve(Z, np.array([3.0, 0.0, 8.0]))[:, 0],
                               [0.5, 0.0, 2.0])


# ---------------------------------------------------------------------------
# Planted mistakes: each broken copy of a step must fail a pin above
# ---------------------------------------------------------------------------


def _broken_variants():
    def wrong_sign_update(Y):
        LU = np.array(Y, float); m, w = LU.shape
        p = np.arange(m); ipiv = np.zeros(w, int)
        for j in range(w):
            r = j + int(np.argmax(np.abs(LU[j:, j]))); ipiv[j] = r
            LU[[j, r]] = LU[[r, j]]; p[[j, r]] = p[[r, j]]
            LU[j + 1:, j] /= LU[j, j]
            LU[j + 1:, j + 1:] += np.outer(LU[j + 1:, j], LU[j, j + 1:])
        return LU, ipiv, p, 0, None

    def max_not_abs(Y):
        LU = np.array(Y, float); m, w = LU.shape
        p = np.arange(m); ipiv = np.zeros(w, int)
        for j in range(w):
            r = j + int(np.argmax(LU[j:, j])); ipiv[j] = r
            LU[[j, r]] = LU[[r, j]]; p[[j, r]] = p[[r, j]]
            LU[j + 1:, j] /= LU[j, j]
            LU[j + 1:, j + 1:] -= np.outer(LU[j + 1:, j], LU[j, j + 1:])
        return LU, ipiv, p, 0, None

    def transposed_projection(Ly, PA):
        Q, R = np.linalg.qr(Ly)
        return scipy.linalg.solve_triangular(R, Q.T @ PA, lower=False, trans=1)

    def normalize_keeps_pivot_order(X):
        LU, _, _, _, _ = rlu.lu_partial_pivot(X)
        return rlu.unit_lower(LU, X.shape[1])

    def power_without_transpose(A, G, q):
        Y = rlu.sketch(A, G)
        for _ in range(q):
            Y = A @ rlu.lu_normalize(A @ rlu.lu_normalize(Y))
        return Y

    def power_one_round_short(A, G, q):
        Y = rlu.sketch(A, G)
        for _ in range(q - 1):
            Y = A @ rlu.lu_normalize(A.T @ rlu.lu_normalize(Y))
        return Y

    def lstsq_without_p(out, b):
        bb = np.asarray(b, float).reshape(b.shape[0], -1)
        k = out["L"].shape[1]
        z1 = rlu.upper_solve(out["U"][:, :k], rlu.pinv_apply(out["L"], bb))
        x = np.zeros((out["U"].shape[1], bb.shape[1])); x[out["q"][:k]] = z1
        return x

    def lstsq_without_q(out, b):
        bb = np.asarray(b, float).reshape(b.shape[0], -1)
        k = out["L"].shape[1]
        z1 = rlu.upper_solve(out["U"][:, :k], rlu.pinv_apply(out["L"], bb[out["p"]]))
        x = np.zeros((out["U"].shape[1], bb.shape[1])); x[:k] = z1
        return x

    return {"lstsq_without_p": ("lstsq", lstsq_without_p),
            "lstsq_without_q": ("lstsq", lstsq_without_q),
            "normalize_keeps_pivot_order": ("normalize", normalize_keeps_pivot_order),
            "power_without_transpose": ("power", power_without_transpose),
            "power_one_round_short": ("power", power_one_round_short),
            "wrong_sign_update": ("lu", wrong_sign_update),
            "max_not_abs": ("lu", max_not_abs),
            "transposed_projection": ("pinv", transposed_projection)}


@pytest.mark.parametrize("name", ["wrong_sign_update", "max_not_abs", "transposed_projection",
                                  "lstsq_without_p", "lstsq_without_q",
                                  "normalize_keeps_pivot_order", "power_without_transpose",
                                  "power_one_round_short"])
def test_planted_mistakes_are_caught(name, monkeypatch):
    kind, fn = _broken_variants()[name]
    if kind == "lu":
        monkeypatch.setattr(rlu, "lu_partial_pivot",
                            lambda Y: fn(Y)[:4] + ({"piv_abs": np.ones(Y.shape[1]),
                                                     "gap": np.ones(Y.shape[1]),
                                                     "max_abs": 1.0},))
    elif kind == "pinv":
        monkeypatch.setattr(rlu, "pinv_apply", fn)
    elif kind == "lstsq":
        monkeypatch.setattr(rlu, "lstsq_rank_deficient", fn)
        failed = False
        for t in (test_lstsq_consistent_system_is_solved_with_k_nonzeros,
                  lambda: test_lstsq_residual_is_the_least_squares_minimum((150, 110), 8)):
            try:
                t()
            except AssertionError:
                failed = True
        assert failed, name
        return
    else:
        monkeypatch.setattr(rlu, "lu_normalize" if kind == "normalize" else "power_sketch_normalized",
                            fn)
    if kind in ("normalize", "power"):
        failed = False
        for q in (1, 2):
            try:
                test_power_sketch_gives_the_factors_of_the_plain_product(q, (70, 70))
            except AssertionError:
                failed = True
        assert failed, name
        return
    failed = False
    for t in (test_lu_partial_pivot_equals_lapack_getrf,
              test_projection_identity_of_the_proof,
              test_pinv_apply_equals_lstsq_and_normal_equations):
        try:
            t()
        except AssertionError:
            failed = True
    assert failed, name
