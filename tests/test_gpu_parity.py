"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Rules (FP64 path):
  * the sketch Y matches to 1e-13 relative (one GEMM, FP64 both sides);
  * pivot sequences match on every step whose choice is numerically decided
    (oracle.rlu.pivot_gate: relative gap >= 1e-8, magnitude >= 1e3 u max|.|);
  * with the first k pivots of Step 3 decided, B and the unpermuted factors
    P^T L and U Q^T match to 1e-10 relative (the tolerance the FP64 path is
    held to), and when every pivot is decided, L, U, p and q match directly;
  * structure is exact: unit diagonal and zeros above it in L, zeros below
    the diagonal of U, p and q permutations, info words equal.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import (ensure_built, power_references, rel_maxdiff, to_dev_colmajor, to_host,
                           unpermute_cols,
                           unpermute_rows)
from oracle import philox, rlu as orl
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def rlu():
    ensure_built()
    import paper_1310_7202_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return m


def run_and_compare(rlu, A, k, l, G, label="", power=0):
    print(f"[parity] {label} m={A.shape[0]} n={A.shape[1]} k={k} l={l} power={power}",
          flush=True)
    out = rlu.factor(to_dev_colmajor(A), k, l, G=to_dev_colmajor(G), diagnostics=True,
                     power_iters=power)
    torch.cuda.synchronize()
    if power == 0:
        o = orl.randomized_lu(A, k, l, G)
    else:
        # the element-by-element rule against the normalized reading of
        # Section 5.2, and the definition (A A^T)^q A G within the distance
        # of the two readings (the plain product's own rounding)
        o, o_plain, d = power_references(orl, A, k, l, G, power)
    info = to_host(out.info)
    assert info[2] == 0, "pivot exchange failed"
    assert (int(info[0]), int(info[1])) == o["info"]
    m, n = A.shape
    L, U, p, q = to_host(out.L), to_host(out.U), to_host(out.p), to_host(out.q)
    # exact structure
    np.testing.assert_array_equal(np.sort(p), np.arange(m))
    np.testing.assert_array_equal(np.sort(q), np.arange(n))
    assert np.all(np.diag(L[:k]) == 1.0)
    assert np.all(np.triu(L[:k], 1) == 0.0)
    assert np.all(np.tril(U, -1) == 0.0)
    # Step 2
    if power == 0:
        assert rel_maxdiff(to_host(out.Y), o["Y"]) < 1e-13
    else:
        # power scheme: the normalizations may round differently past the
        # numerical rank, so compare what Steps 3-8 use, the span of the
        # leading k columns of the sketch
        Yg = to_host(out.Y)[:, :k]
        Qo, _ = np.linalg.qr(o["Y"][:, :k])
        assert np.abs(Yg - Qo @ (Qo.T @ Yg)).max() < 1e-10 * np.abs(Yg).max()
    # Step 3 pivots on the decided prefix
    gy = orl.pivot_gate(o["diag_y"])
    np.testing.assert_array_equal(to_host(out.ipiv)[:gy], o["ipiv"][:gy])
    if gy < k:
        pytest.skip(f"Step 3 pivot {gy} is not numerically decided; factors not comparable")
    # Step 5
    assert rel_maxdiff(to_host(out.B), o["B"]) < TOL
    # Step 6 pivots on the decided prefix
    gb = orl.pivot_gate(o["diag_b"])
    np.testing.assert_array_equal(to_host(out.qpiv)[:gb], o["qpiv"][:gb])
    if gb == k:
        np.testing.assert_array_equal(q, o["q"])
        assert rel_maxdiff(unpermute_rows(L, p), unpermute_rows(o["L"], o["p"])) < TOL
        assert rel_maxdiff(U, o["U"]) < TOL
    if gy == l and gb == k:
        np.testing.assert_array_equal(p, o["p"])
        assert rel_maxdiff(L, o["L"]) < TOL
    if power and gb == k:
        e = rel_maxdiff(unpermute_rows(L, p), unpermute_rows(o_plain["L"], o_plain["p"]))
        print(f"  vs plain (A A^T)^q A G: {e:.2e} (readings differ by {d:.2e})", flush=True)
        assert e < TOL + 2 * d
    return out, o


def test_small_config(rlu):
    A, k, l = workloads.config_small(101)
    G = workloads.gaussian((A.shape[1], l), 7203)
    run_and_compare(rlu, A, k, l, G, "512^2 rank-10")


@pytest.mark.parametrize("m,n,k,l,rate", [
    (3000, 2500, 50, 60, 20.0),     # several workgroups per panel, ragged tails
    (700, 1300, 33, 41, 8.0),       # m < n, ragged GEMM tiles
    (1300, 700, 40, 40, 8.0),       # k = l
    (200, 64, 64, 64, 30.0),        # l = min(m, n): full-rank reconstruction
    (97, 131, 5, 9, 3.0),           # sizes below one tile
])
def test_spectral_shapes(rlu, m, n, k, l, rate):
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), 1000 + m)
    G = workloads.gaussian((n, l), 2000 + n)
    out, o = run_and_compare(rlu, A, k, l, G, f"spectral rate={rate}")
    if k == l == min(m, n):
        L, U, p, q = to_host(out.L), to_host(out.U), to_host(out.p), to_host(out.q)
        np.testing.assert_allclose(L @ U, A[np.ix_(p, q)], atol=1e-11 * np.abs(A).max())


def test_one_by_one(rlu):
    A = np.array([[3.0]])
    G = np.array([[0.5]])
    out, o = run_and_compare(rlu, A, 1, 1, G, "1x1")
    assert to_host(out.U)[0, 0] == pytest.approx(3.0, rel=1e-15)


def test_single_column_rank_one(rlu):
    A = np.zeros((40, 30))
    A[:, 4] = np.linspace(-1.0, 2.0, 40)
    G = workloads.gaussian((30, 3), 5)
    out, o = run_and_compare(rlu, A, 1, 3, G, "rank one")


@pytest.mark.parametrize("power", [0, 1, 2])
def test_zero_matrix_sets_info(rlu, power):
    # with power iterations every normalization meets only zero pivots too
    A = np.zeros((64, 48))
    G = workloads.gaussian((48, 6), 3)
    print(f"[parity] zero matrix power={power}", flush=True)
    out = rlu.factor(to_dev_colmajor(A), 4, 6, G=to_dev_colmajor(G), diagnostics=True,
                     power_iters=power)
    torch.cuda.synchronize()
    o = orl.randomized_lu(A, 4, 6, G, q=power)
    assert o["info"] == (1, 1)
    info = to_host(out.info)
    assert tuple(info) == (1, 1, 0)
    assert rlu.check_info(info) == 2  # RLU_WARN_ZERO_PIVOT
    L, U = to_host(out.L), to_host(out.U)
    assert np.all(U == 0.0)
    assert np.all(np.diag(L[:4]) == 1.0)
    np.testing.assert_array_equal(L, o["L"])
    np.testing.assert_array_equal(to_host(out.p), o["p"])
    np.testing.assert_array_equal(to_host(out.q), o["q"])


def test_rank_deficient_second_pivot_zero(rlu):
    A = np.zeros((30, 20))
    A[3, 5] = 2.0
    G = workloads.gaussian((20, 3), 4)
    out = rlu.factor(to_dev_colmajor(A), 2, 3, G=to_dev_colmajor(G), diagnostics=True)
    torch.cuda.synchronize()
    o = orl.randomized_lu(A, 2, 3, G)
    info = to_host(out.info)
    assert (int(info[0]), int(info[1])) == o["info"] == (2, 2)
    L, U, p, q = to_host(out.L), to_host(out.U), to_host(out.p), to_host(out.q)
    np.testing.assert_allclose(L @ U, A[np.ix_(p, q)], atol=1e-14)


def test_device_gaussian_matches_host_generator(rlu):
    n, l, seed = 300, 7, 0x1234_5678_9ABC
    A = np.eye(n)
    out = rlu.factor(to_dev_colmajor(A), 3, l, seed=seed, diagnostics=True)
    torch.cuda.synchronize()
    Yd = to_host(out.Y)            # A = I: Y is G itself (exact products)
    Gh = philox.gaussian_matrix(n, l, seed)
    diff = np.abs(Yd - Gh)
    # libm differences only: a few ulp of each entry
    assert np.all(diff <= 8 * np.spacing(np.abs(Gh)) + 1e-300)
    assert diff.max() < 1e-14


def test_generated_sketch_end_to_end(rlu):
    A = workloads.spectral_matrix(900, 800, workloads.exp_decay(800, 10.0), 77)
    k, l, seed = 30, 36, 99
    out = rlu.factor(to_dev_colmajor(A), k, l, seed=seed, diagnostics=True)
    torch.cuda.synchronize()
    G = philox.gaussian_matrix(800, l, seed)
    o = orl.randomized_lu(A, k, l, G)
    L, U, p, q = to_host(out.L), to_host(out.U), to_host(out.p), to_host(out.q)
    assert rel_maxdiff(unpermute_rows(L, p), unpermute_rows(o["L"], o["p"])) < TOL
    assert rel_maxdiff(unpermute_cols(U, q), unpermute_cols(o["U"], o["q"])) < TOL


def test_repeat_calls_are_bitwise_identical_and_resize(rlu):
    A = workloads.spectral_matrix(1500, 1200, workloads.exp_decay(1200, 15.0), 5)
    G = workloads.gaussian((1200, 40), 6)
    dA, dG = to_dev_colmajor(A), to_dev_colmajor(G)
    a = rlu.factor(dA, 32, 40, G=dG)
    small = rlu.factor(to_dev_colmajor(A[:300, :200]), 8, 10, G=to_dev_colmajor(G[:200, :10]))
    b = rlu.factor(dA, 32, 40, G=dG)
    torch.cuda.synchronize()
    for x, y in ((a.L, b.L), (a.U, b.U), (a.p, b.p), (a.q, b.q)):
        assert torch.equal(x, y)
    o = orl.randomized_lu(A[:300, :200], 8, 10, G[:200, :10])
    assert rel_maxdiff(unpermute_rows(to_host(small.L), to_host(small.p)),
                       unpermute_rows(o["L"], o["p"])) < TOL


def test_leading_dimensions(rlu):
    m, n, k, l = 300, 250, 12, 16
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), 5.0), 8)
    G = workloads.gaussian((n, l), 9)
    big = torch.zeros((n, m + 37), dtype=torch.float64, device="cuda")
    big[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    dA = big.t()[:m]       # m x n view with lda = m + 37
    assert dA.stride() == (1, m + 37)
    out = rlu.factor(dA, k, l, G=to_dev_colmajor(G))
    torch.cuda.synchronize()
    o = orl.randomized_lu(A, k, l, G)
    assert rel_maxdiff(unpermute_rows(to_host(out.L), to_host(out.p)),
                       unpermute_rows(o["L"], o["p"])) < TOL


@pytest.mark.parametrize("m,n,k,l", [
    (1500, 1200, 65, 70),      # one full block and a 1-wide block
    (3000, 2600, 200, 210),    # the 8192^2 configuration's rank
    (4000, 3000, 300, 310),    # five blocks, ragged last one
])
def test_large_rank_blocked_gram_inverse(rlu, m, n, k, l):
    """k > 64: the Gram inverse of Step 5 runs as blocked Gauss-Jordan."""
    A = workloads.low_rank_plus_noise(m, n, k, 1e-6, 610 + k)
    G = workloads.gaussian((n, l), 620 + k)
    run_and_compare(rlu, A, k, l, G, f"k={k}")


@pytest.mark.parametrize("m,n,k,l", [
    (2000, 4500, 230, 240),    # Y = A G: K = 4500, short side l = 240 in 128 x 224 tiles
    (4500, 1500, 250, 260),    # Lv^T A: K = 4500, short side k = 250 in 128 x 224 tiles
])
def test_wide_short_side_products(rlu, m, n, k, l):
    """Long products whose short side spans two 128 x 224 tiles (ragged
    second tile), with split-K."""
    A = workloads.low_rank_plus_noise(m, n, k, 1e-6, 660 + k)
    G = workloads.gaussian((n, l), 670 + k)
    run_and_compare(rlu, A, k, l, G, f"wide {m}x{n}")


@pytest.mark.parametrize("m,n,k,l", [
    (16384, 2000, 290, 300),   # Y (16384 x 300) factored in column blocks
    (2000, 16384, 290, 300),   # B^T (16384 x 290) factored in column blocks
])
def test_blocked_panels(rlu, m, n, k, l):
    """Panels too tall and wide for one resident launch: column blocks, each
    continuing from the row positions of the ones before, with a triangular
    solve and a GEMM update in between."""
    A = workloads.low_rank_plus_noise(m, n, k, 1e-6, 640 + m)
    G = workloads.gaussian((n, l), 650 + n)
    run_and_compare(rlu, A, k, l, G, f"blocked {m}x{n}")


@pytest.mark.parametrize("m,seed", [(6000, 77), (20000, 78), (1500, 79), (500, 80)])
def test_exact_pivot_ties_go_to_lowest_position(rlu, m, seed):
    """Pivot searches with many equal magnitudes, in exact arithmetic.

    Entries are +-1 and G = [I; 0], so Y is the first l columns of A.  While
    every pivot is a power of two, multipliers and updates are exact on both
    sides, so each pivot choice up to and including the first other pivot is
    made on identical values; every tie (the first step is an m-way one, and
    ties span workgroups) must go to the lowest current position, as the
    oracle's search does."""
    n, k, l = 40, 12, 16
    rng = np.random.default_rng(seed)
    A = rng.choice([-1.0, 1.0], size=(m, n))
    G = np.zeros((n, l))
    G[:l, :l] = np.eye(l)
    print(f"[parity] exact ties m={m} seed={seed}", flush=True)
    out = rlu.factor(to_dev_colmajor(A), k, l, G=to_dev_colmajor(G), diagnostics=True)
    torch.cuda.synchronize()
    _, ipiv, _, _, diag = orl.lu_partial_pivot(A[:, :l])
    exact = 0
    for a in diag["piv_abs"]:
        if a == 0.0 or np.frexp(a)[0] != 0.5:
            break
        exact += 1
    assert exact >= 4, "the input no longer exercises exact ties"
    upto = min(exact + 1, l)
    assert to_host(out.info)[2] == 0
    np.testing.assert_array_equal(to_host(out.Y), A[:, :l])
    np.testing.assert_array_equal(to_host(out.ipiv)[:upto], ipiv[:upto])


@pytest.mark.parametrize("m,n,k,l,rate,q", [
    (512, 512, 10, 15, 0.0, 1),         # the 512^2 rank-10 configuration
    (512, 512, 10, 15, 0.0, 2),
    (3000, 2500, 50, 60, 20.0, 1),      # several workgroups per panel, ragged tails
    (3000, 2500, 50, 60, 20.0, 3),
    (1500, 2600, 33, 41, 12.0, 1),      # m < n: the n x l normalization is the taller
    (97, 131, 5, 9, 3.0, 2),            # sizes below one tile
    (200, 64, 64, 64, 30.0, 1),         # l = min(m, n)
])
def test_power_iterations(rlu, m, n, k, l, rate, q):
    """Section 5.2: Y = (A A^T)^q A G with the LU normalization, against the
    oracle's power scheme."""
    if rate == 0.0:
        A, k, l = workloads.config_small(101)
    else:
        A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), 1100 + m)
    G = workloads.gaussian((A.shape[1], l), 2100 + n + q)
    run_and_compare(rlu, A, k, l, G, f"power rate={rate}", power=q)


def test_power_iterations_blocked_normalization(rlu):
    """The n x l normalization (16384 x 300) factored in column blocks."""
    m, n, k, l = 2000, 16384, 290, 300
    A = workloads.low_rank_plus_noise(m, n, k, 1e-6, 660)
    G = workloads.gaussian((n, l), 661)
    run_and_compare(rlu, A, k, l, G, "power blocked", power=1)



def _register_panel_cases():
    rng = np.random.default_rng(4100)
    ties = rng.choice([-1.0, 1.0], size=(60, 50))
    few = np.zeros((300, 200))
    few[rng.choice(300, 5, replace=False)] = rng.standard_normal((5, 200))
    return [
        ("512^2 rank-10", *workloads.config_small(101)),
        ("97x131", workloads.spectral_matrix(97, 131, workloads.exp_decay(97, 3.0), 4101), 5, 9),
        ("400x300 l=28", workloads.spectral_matrix(400, 300, workloads.exp_decay(300, 9.0),
                                                   4102), 20, 28),
        ("480x350 l=32", workloads.spectral_matrix(480, 350, workloads.exp_decay(350, 12.0),
                                                   4103), 24, 32),
        ("1000x700 l=30", workloads.spectral_matrix(1000, 700, workloads.exp_decay(700, 9.0),
                                                    4104), 20, 30),
        ("1800x900 l=14", workloads.spectral_matrix(1800, 900, workloads.exp_decay(900, 5.0),
                                                    4105), 8, 14),
        ("+-1 ties", np.vstack([ties, ties, ties]), 12, 16),
        ("5 nonzero rows", few, 6, 12),
    ]


@pytest.mark.parametrize("case", range(8))
def test_register_panel_bitwise_equal_to_lds_panel(rlu, monkeypatch, case):
    """Panels of one workgroup with at most 32 columns (up to 1024 or 2048
    rows for 32 or 16 columns) run in registers; with
    RLU_PANEL_REGS=0 the same panels go to the LDS-resident kernels (one
    workgroup up to 512 rows, several beyond).  Both take the same
    multipliers, updates, ranking and ties, so every output agrees bit for
    bit: on spectral inputs, on exact +-1 ties between identical rows, and
    on a sketch whose later pivots are exactly zero."""
    label, A, k, l = _register_panel_cases()[case]
    m, n = A.shape
    G = workloads.gaussian((n, l), 4200 + case)
    Ad, Gd = to_dev_colmajor(A), to_dev_colmajor(G)
    print(f"[parity] register panel vs LDS panel: {label} m={m} n={n} k={k} l={l}", flush=True)
    outs = []
    for regs in ("1", "0"):
        monkeypatch.setenv("RLU_PANEL_REGS", regs)
        out = rlu.factor(Ad, k, l, G=Gd, diagnostics=True)
        torch.cuda.synchronize()
        outs.append({x: to_host(getattr(out, x)) for x in ("L", "U", "p", "q", "ipiv", "Y", "info")})
    monkeypatch.delenv("RLU_PANEL_REGS")
    a, b = outs
    assert a["info"][2] == 0
    for x in a:
        np.testing.assert_array_equal(a[x], b[x], err_msg=x)
    if label == "5 nonzero rows":
        assert tuple(a["info"][:2]) == (6, 6)   # zero pivots from step 6 on
