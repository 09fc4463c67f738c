"""Parity at the full sizes the benchmark times, in the same launch
configuration (one rlu_factor call on the whole matrix).

  * 8192 x 8192, sigma_i = exp(-i/50), k = 200, l = 210, FP64: element by
    element against the FP64 oracle under the rules of test_gpu_parity, with
    and without one power iteration (Section 5.2);
  * the same matrix in FP32 storage: the reduced-precision residual rule;
  * 16384 x 16384, sigma_i = i^-2, k = 500, l = 520, BF16 products with FP32
    accumulation: the residual rule against the oracle on the same FP32 A;
  * the least-squares solve (Algorithm 4.3) on the 8192^2 factors.
The matrices are generated on the device (a host QR of the Haar factors
would take minutes); G comes from the host generator and is passed in.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import ensure_built, to_dev_colmajor, to_host
from tests.test_gpu_parity import run_and_compare
from oracle import philox, rlu as orl
import workloads

pytestmark = pytest.mark.gpu

BAR = 1e-3


@pytest.fixture(scope="module")
def rlu():
    ensure_built()
    import paper_1310_7202_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return m


@pytest.fixture(scope="module")
def exp8192():
    A_dev, k, l = workloads.config_exp_spectrum(8192, 102, device="cuda")
    A = to_host(A_dev)
    del A_dev
    torch.cuda.empty_cache()
    return A, k, l, philox.gaussian_matrix(8192, l, 7202)


@pytest.mark.parametrize("q", [0, 1])
def test_exp_spectrum_8192_fp64(rlu, exp8192, q):
    A, k, l, G = exp8192
    out, o = run_and_compare(rlu, A, k, l, G, "8192^2 exp(-i/50)", power=q)
    if q == 1:
        e1 = orl.relative_residual(A, o, exact=False)
        e0 = orl.relative_residual(A, orl.randomized_lu(A, k, l, G), exact=False)
        print(f"  oracle residual q=1 {e1:.3e} q=0 {e0:.3e}", flush=True)
        assert e1 < e0


def test_exp_spectrum_8192_rrlu(rlu, exp8192):
    """The rank-revealing Step 3 (Algorithm 4.1 as listed) at the full size,
    element by element under the rule of test_gpu_rrlu."""
    from tests.test_gpu_rrlu import compare_rrlu
    A, k, l, G = exp8192
    compare_rrlu(rlu, A, k, l, G, "8192^2 exp(-i/50)")


def test_exp_spectrum_8192_fast(rlu, exp8192):
    """Algorithm 4.4 (fast randomized LU) at the full size, element by
    element under the rule of test_gpu_fast."""
    from tests.test_gpu_fast import compare_fast
    A, k, l, _ = exp8192
    compare_fast(rlu, A, k, l, 7208, "8192^2 exp(-i/50)")


def test_exp_spectrum_8192_lstsq(rlu, exp8192):
    """Algorithm 4.3 on the full-size factors, as the least-squares form of
    the benchmark runs it (b = A x0): the GPU solve on the GPU factors
    against the oracle's solve on its own factors of the same A and G."""
    A, k, l, G = exp8192
    print("[full] 8192^2 least squares, 4 right-hand sides", flush=True)
    Ad = to_dev_colmajor(A)
    f = rlu.factor(Ad, k, l, G=to_dev_colmajor(G))
    x0 = np.random.default_rng(7206).standard_normal((A.shape[1], 4))
    b = A @ x0
    x = to_host(rlu.lstsq(f, to_dev_colmajor(b)))
    torch.cuda.synchronize()
    o = orl.randomized_lu(A, k, l, G)
    assert np.array_equal(to_host(f.q)[:k], o["q"][:k])
    xo = orl.lstsq_rank_deficient(o, b)
    assert np.abs(x - xo).max() <= 1e-9 * np.abs(xo).max()
    zero = np.ones(A.shape[1], bool)
    zero[o["q"][:k]] = False
    assert np.all(x[zero] == 0.0)


def _residual_rule(rlu, A32, k, l, G32, precision, label):
    m, n = A32.shape
    print(f"[full] {label} m={m} n={n} k={k} l={l} prec={precision}", flush=True)
    out = rlu.factor(to_dev_colmajor(A32, dtype=torch.float32), k, l,
                     G=to_dev_colmajor(G32, dtype=torch.float32), precision=precision)
    torch.cuda.synchronize()
    info = to_host(out.info)
    assert info[2] == 0
    L = to_host(out.L).astype(np.float64)
    U = to_host(out.U).astype(np.float64)
    p, q = to_host(out.p), to_host(out.q)
    del out
    np.testing.assert_array_equal(np.sort(p), np.arange(m))
    np.testing.assert_array_equal(np.sort(q), np.arange(n))
    assert np.all(np.diag(L[:k]) == 1.0) and np.all(np.triu(L[:k], 1) == 0.0)
    assert np.all(np.tril(U, -1) == 0.0)
    A = A32.astype(np.float64)
    o = orl.randomized_lu(A, k, l, G32.astype(np.float64))
    r_gpu = orl.relative_residual(A, {"L": L, "U": U, "p": p, "q": q}, exact=False)
    r_ora = orl.relative_residual(A, o, exact=False)
    print(f"  residual gpu {r_gpu:.3e} oracle {r_ora:.3e}", flush=True)
    assert r_gpu <= r_ora + BAR
    return r_gpu, r_ora


def test_exp_spectrum_8192_fp32(rlu, exp8192):
    A, k, l, G = exp8192
    _residual_rule(rlu, A.astype(np.float32), k, l, G.astype(np.float32), rlu.PREC_FP32,
                   "8192^2 FP32")


@pytest.mark.parametrize("fp16", [False, True])
def test_inverse_square_spectrum_16384_mixed(rlu, fp16):
    n, k, l = 16384, 500, 520
    A_dev = workloads.spectral_matrix_torch(n, n, workloads.inv_square(n), 103,
                                            device="cuda", dtype=torch.float32)
    A32 = to_host(A_dev)
    del A_dev
    torch.cuda.empty_cache()
    G32 = philox.gaussian_matrix(n, l, 7203).astype(np.float32)
    prec = rlu.PREC_MIXED_FP16 if fp16 else rlu.PREC_MIXED_BF16
    _residual_rule(rlu, A32, k, l, G32, prec, f"16384^2 i^-2 {'FP16' if fp16 else 'BF16'}")
