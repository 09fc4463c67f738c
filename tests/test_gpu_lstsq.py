"""Rank-deficient least squares on the factors (Section 4.4, Algorithm 4.3)
through the C ABI, against the FP64 oracle.

  * Same seeded factors on both sides (stand-ins for the outputs of
    Algorithm 4.1): x within 1e-10 relative in FP64 (the GPU applies L^+
    through the Gram matrix, the oracle through QR; with a tall L of
    bounded entries both are far inside that), FP32 storage within 1e-6
    (the output is rounded to FP32);
  * structure: x has at most k nonzeros, at the positions q[0:k];
  * a zero row of U (a zero pivot of Step 6) leaves its unknown at zero;
  * end to end: factors from rlu_factor, a consistent right-hand side on a
    rank-k matrix is solved to 1e-10, and the solution matches the one the
    oracle computes from its own factors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import ensure_built, rel_maxdiff, to_dev_colmajor, to_host
from oracle import rlu as orl
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rlu():
    ensure_built()
    import paper_1310_7202_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return m


def _dev_factors(rlu, L, U, p, q, dtype):
    return rlu.Factors(to_dev_colmajor(L, dtype=dtype), to_dev_colmajor(U, dtype=dtype),
                       torch.as_tensor(p, dtype=torch.int64, device="cuda"),
                       torch.as_tensor(q, dtype=torch.int64, device="cuda"), None)


@pytest.mark.parametrize("m,n,k,r", [
    (2000, 1500, 40, 1),
    (2000, 1500, 40, 7),
    (700, 1300, 33, 3),       # m < n
    (300, 200, 200, 2),       # k = n: no z_2
    (97, 131, 5, 1),          # below one tile
    (3000, 2500, 300, 2),     # k > 256: several rows of U_1 per thread
    (4000, 3000, 700, 1),     # k > 512, blocked Gram inverse
])
def test_lstsq_same_factors_fp64(rlu, m, n, k, r):
    print(f"[lstsq] fp64 m={m} n={n} k={k} r={r}", flush=True)
    L, U, p, q = workloads.synthetic_factors(m, n, k, 900 + k)
    b = workloads.gaussian((m, r), 901 + k)
    f = _dev_factors(rlu, L, U, p, q, torch.float64)
    x = to_host(rlu.lstsq(f, to_dev_colmajor(b)))
    torch.cuda.synchronize()
    xo = orl.lstsq_rank_deficient({"L": L, "U": U, "p": p, "q": q}, b)
    assert rel_maxdiff(x, xo) < 1e-10
    zero = np.ones(n, bool)
    zero[q[:k]] = False
    assert np.all(x[zero] == 0.0)


def test_lstsq_vector_rhs_and_fp32(rlu):
    m, n, k = 1800, 1200, 24
    L, U, p, q = workloads.synthetic_factors(m, n, k, 910)
    b = workloads.gaussian((m,), 911)
    print(f"[lstsq] vector and fp32 m={m} n={n} k={k}", flush=True)
    f64 = _dev_factors(rlu, L, U, p, q, torch.float64)
    x = to_host(rlu.lstsq(f64, torch.as_tensor(b, device="cuda")))
    assert x.shape == (n,)
    xo = orl.lstsq_rank_deficient({"L": L, "U": U, "p": p, "q": q}, b)
    assert rel_maxdiff(x, xo) < 1e-10
    L32, U32, b32 = L.astype(np.float32), U.astype(np.float32), b.astype(np.float32)
    f32 = _dev_factors(rlu, L32, U32, p, q, torch.float32)
    x32 = to_host(rlu.lstsq(f32, torch.as_tensor(b32, device="cuda")))
    assert x32.dtype == np.float32
    xo32 = orl.lstsq_rank_deficient({"L": L32.astype(np.float64), "U": U32.astype(np.float64),
                                     "p": p, "q": q}, b32.astype(np.float64))
    assert rel_maxdiff(x32.astype(np.float64), xo32) < 1e-6


def test_lstsq_zero_row_of_u_gives_zero_unknown(rlu):
    m, n, k = 600, 500, 20
    L, U, p, q = workloads.synthetic_factors(m, n, k, 920)
    U[7, :] = 0.0
    b = workloads.gaussian((m, 2), 921)
    print("[lstsq] zero row of U", flush=True)
    x = to_host(rlu.lstsq(_dev_factors(rlu, L, U, p, q, torch.float64), to_dev_colmajor(b)))
    xo = orl.lstsq_rank_deficient({"L": L, "U": U, "p": p, "q": q}, b)
    assert np.all(x[q[7]] == 0.0)
    assert rel_maxdiff(x, xo) < 1e-10


@pytest.mark.parametrize("m,n,k", [(2500, 1800, 30), (900, 1400, 17)])
def test_lstsq_end_to_end_consistent_rank_k(rlu, m, n, k):
    A = workloads.low_rank_plus_noise(m, n, k, 0.0, 930 + k)
    G = workloads.gaussian((n, k + 5), 931 + k)
    x0 = workloads.gaussian((n, 3), 932 + k)
    b = A @ x0
    print(f"[lstsq] end to end m={m} n={n} k={k}", flush=True)
    f = rlu.factor(to_dev_colmajor(A), k, k + 5, G=to_dev_colmajor(G))
    x = to_host(rlu.lstsq(f, to_dev_colmajor(b)))
    torch.cuda.synchronize()
    assert np.all(to_host(f.info) == 0)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)
    assert np.all(np.count_nonzero(x, axis=0) <= k)
    o = orl.randomized_lu(A, k, k + 5, G)
    xo = orl.lstsq_rank_deficient(o, b)
    if np.array_equal(to_host(f.q)[:k], o["q"][:k]):
        assert rel_maxdiff(x, xo) < 1e-8
