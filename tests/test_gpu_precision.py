"""Reduced-precision forms of the HIP path against the FP64 CPU oracle.

Rule (reduced precision): the relative residual ||L U - P A Q||_2 / ||A||_2 of
the GPU factors may exceed the oracle's by at most 1e-3, both computed the
same way on the same FP32-stored A (upcast to FP64) with the same G; the
structure of the factors is exact; and the pivots agree on every step whose
choice is decided by a wide margin (relative gap >= 1e-3 and magnitude >= 1e3
FP32 unit roundoffs of max|Y|, far above FP32 rounding of the sketch; for
the BF16 / FP16 products a gap >= 1/4 and a magnitude >= 16 unit roundoffs
of the 16-bit format).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import ensure_built, to_dev_colmajor, to_host
from oracle import rlu as orl
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


def rel_residual(A, L, U, p, q):
    return np.linalg.norm(L @ U - A[np.ix_(p, q)], 2) / np.linalg.norm(A, 2)


def check(rlu, A64, k, l, seed, precision, label, q=0):
    A32 = A64.astype(np.float32)
    A = A32.astype(np.float64)            # the matrix both sides factor
    m, n = A.shape
    G32 = workloads.gaussian((n, l), seed).astype(np.float32)
    print(f"[precision] {label} m={m} n={n} k={k} l={l} prec={precision} q={q}", flush=True)
    out = rlu.factor(to_dev_colmajor(A32, dtype=torch.float32), k, l,
                     G=to_dev_colmajor(G32, dtype=torch.float32), precision=precision,
                     diagnostics=True, power_iters=q)
    torch.cuda.synchronize()
    assert out.L.dtype == torch.float32 and out.U.dtype == torch.float32
    info = to_host(out.info)
    assert info[2] == 0
    o = orl.randomized_lu(A, k, l, G32.astype(np.float64), q=q)
    L = to_host(out.L).astype(np.float64)
    U = to_host(out.U).astype(np.float64)
    p, q = to_host(out.p), to_host(out.q)
    np.testing.assert_array_equal(np.sort(p), np.arange(m))
    np.testing.assert_array_equal(np.sort(q), np.arange(n))
    assert np.all(np.diag(L[:k]) == 1.0) and np.all(np.triu(L[:k], 1) == 0.0)
    assert np.all(np.tril(U, -1) == 0.0)
    r_gpu = rel_residual(A, L, U, p, q)
    r_ora = rel_residual(A, o["L"], o["U"], o["p"], o["q"])
    print(f"  residual gpu {r_gpu:.3e} oracle {r_ora:.3e}", flush=True)
    assert r_gpu <= r_ora + BAR
    # decided by a margin the rounding of the sketch cannot flip: for FP32,
    # relative gap >= 1e-3 and magnitude >= 1e3 FP32 unit roundoffs of
    # max|Y|; the 16-bit products round their operands to u = 2^-8 (BF16)
    # or 2^-11 (FP16), so there the gap must be >= 1/4 and the pivot
    # >= 16 u max|Y|
    if precision == rlu.PREC_FP32:
        gy = orl.pivot_gate(o["diag_y"], u=2.0 ** -24, gap_min=1e-3, mag_factor=1e3)
    else:
        u16 = 2.0 ** -8 if precision == rlu.PREC_MIXED_BF16 else 2.0 ** -11
        gy = orl.pivot_gate(o["diag_y"], u=u16, gap_min=0.25, mag_factor=16)
    np.testing.assert_array_equal(to_host(out.ipiv)[:gy], o["ipiv"][:gy])
    return r_gpu, r_ora


@pytest.mark.parametrize("m,n,k,l,rate", [
    (3000, 2500, 50, 60, 20.0),
    (700, 1300, 33, 41, 8.0),
    (97, 131, 5, 9, 3.0),
])
def test_fp32_spectral(rlu, m, n, k, l, rate):
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), 300 + m)
    check(rlu, A, k, l, 400 + n, rlu.PREC_FP32, "fp32 spectral")


def test_fp32_low_rank(rlu):
    A, k, l = workloads.config_small(101)
    r_gpu, r_ora = check(rlu, A, k, l, 7203, rlu.PREC_FP32, "fp32 512^2 rank-10")
    # the FP32 storage of A itself limits the attainable residual
    assert r_gpu < 1e-5


def test_fp32_default_precision_for_float_input(rlu):
    A = workloads.spectral_matrix(400, 300, workloads.exp_decay(300, 6.0), 9).astype(np.float32)
    out = rlu.factor(to_dev_colmajor(A, dtype=torch.float32), 10, 14, seed=3)
    torch.cuda.synchronize()
    assert tuple(to_host(out.info)) == (0, 0, 0)
    assert out.L.dtype == torch.float32


def _round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), kept in FP32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def check_mixed(rlu, A64, k, l, seed, fp16, label):
    """As check(), with G already representable in the 16-bit type so that
    both sides use the same sketch matrix."""
    A32 = A64.astype(np.float32)
    A = A32.astype(np.float64)
    m, n = A.shape
    G = workloads.gaussian((n, l), seed).astype(np.float32)
    G = G.astype(np.float16).astype(np.float32) if fp16 else _round_bf16(G)
    prec = rlu.PREC_MIXED_FP16 if fp16 else rlu.PREC_MIXED_BF16
    print(f"[precision] {label} m={m} n={n} k={k} l={l} fp16={fp16}", flush=True)
    out = rlu.factor(to_dev_colmajor(A32, dtype=torch.float32), k, l,
                     G=to_dev_colmajor(G, dtype=torch.float32), precision=prec, diagnostics=True)
    torch.cuda.synchronize()
    assert out.Y.dtype == torch.float64  # diagnostics of the mixed form are FP64
    info = to_host(out.info)
    assert info[2] == 0
    o = orl.randomized_lu(A, k, l, G.astype(np.float64))
    L = to_host(out.L).astype(np.float64)
    U = to_host(out.U).astype(np.float64)
    p, q = to_host(out.p), to_host(out.q)
    np.testing.assert_array_equal(np.sort(p), np.arange(m))
    np.testing.assert_array_equal(np.sort(q), np.arange(n))
    assert np.all(np.diag(L[:k]) == 1.0) and np.all(np.triu(L[:k], 1) == 0.0)
    assert np.all(np.tril(U, -1) == 0.0)
    r_gpu = rel_residual(A, L, U, p, q)
    r_ora = rel_residual(A, o["L"], o["U"], o["p"], o["q"])
    print(f"  residual gpu {r_gpu:.3e} oracle {r_ora:.3e}", flush=True)
    assert r_gpu <= r_ora + BAR
    # the sketch itself: A rounded to 16 bits times an exact G, FP32 sums
    u = 2.0 ** -11 if fp16 else 2.0 ** -8
    Yd = to_host(out.Y)
    assert np.abs(Yd - o["Y"]).max() <= 4 * u * (np.abs(A) @ np.abs(G.astype(np.float64))).max()
    return r_gpu, r_ora


@pytest.mark.parametrize("fp16", [False, True])
@pytest.mark.parametrize("m,n,k,l,rate", [
    (3000, 2500, 50, 60, 20.0),
    (700, 1300, 33, 41, 8.0),
])
def test_mixed_spectral(rlu, m, n, k, l, rate, fp16):
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), 500 + m)
    check_mixed(rlu, A, k, l, 600 + n, fp16, "mixed spectral")


@pytest.mark.parametrize("fp16", [False, True])
def test_mixed_slow_decay_inverse_square(rlu, fp16):
    # sigma_i = i^-2 (the spectrum of the mixed-precision workload), smaller size
    m = n = 2048
    A = workloads.spectral_matrix(m, n, workloads.inv_square(m), 77)
    check_mixed(rlu, A, 120, 130, 78, fp16, "mixed i^-2")


@pytest.mark.parametrize("precision", [1, 2, 3])
@pytest.mark.parametrize("q", [1, 2])
def test_power_iterations_reduced_precision(rlu, precision, q):
    """Section 5.2 in the FP32 and mixed forms: the residual rule against the
    oracle with the same q, on the paper's slowly decaying spectrum, where
    the power scheme lowers the error."""
    m, n, k, l = 2600, 1900, 40, 48
    sig = workloads.slow_decay(n)
    A64 = workloads.spectral_matrix(m, n, sig / sig[0], 1700 + q)
    r_gpu, r_ora = check(rlu, A64, k, l, 1710 + q, precision, "power", q=q)
    r0_gpu, _ = check(rlu, A64, k, l, 1710 + q, precision, "power q=0")
    assert r_gpu < r0_gpu


@pytest.mark.parametrize("fp16", [False, True])
@pytest.mark.parametrize("e", [24, -24])
def test_mixed_power_of_two_scale_equivariance(rlu, fp16, e):
    """A times 2^e gives the same pivots and L, and U times 2^e, bit for bit.
    Every step of Algorithm 4.1 commutes with a power-of-two scale of A as
    long as nothing leaves the range of its format; FP16 has a range of only
    about 2^-24 .. 2^16, so for it this holds only because the products scale
    A by a power of two chosen from max|A| before rounding it (entries near
    2^24 would round to infinity, entries near 2^-30 to zero)."""
    m, n, k, l = 1500, 1100, 30, 38
    A32 = workloads.spectral_matrix(m, n, workloads.exp_decay(n, 10.0), 820).astype(np.float32)
    G = workloads.gaussian((n, l), 821).astype(np.float32)
    G = G.astype(np.float16).astype(np.float32) if fp16 else _round_bf16(G)
    prec = rlu.PREC_MIXED_FP16 if fp16 else rlu.PREC_MIXED_BF16
    Gd = to_dev_colmajor(G, dtype=torch.float32)
    print(f"[precision] scale 2^{e} fp16={fp16} m={m} n={n} k={k} l={l}", flush=True)
    outs = []
    for scale in (1.0, 2.0 ** e):
        As = (A32 * np.float32(scale)).astype(np.float32)
        assert np.array_equal(As / np.float32(scale), A32)   # the scaling is exact
        out = rlu.factor(to_dev_colmajor(As, dtype=torch.float32), k, l, G=Gd, precision=prec,
                         diagnostics=True)
        torch.cuda.synchronize()
        assert tuple(to_host(out.info)) == (0, 0, 0)
        outs.append({x: to_host(getattr(out, x)) for x in ("L", "U", "p", "q", "ipiv", "Y")})
    a, b = outs
    for x in ("p", "q", "ipiv"):
        np.testing.assert_array_equal(a[x], b[x])
    np.testing.assert_array_equal(a["L"], b["L"])
    for x in ("U", "Y"):
        np.testing.assert_array_equal(a[x].astype(np.float64) * 2.0 ** e, b[x].astype(np.float64))


@pytest.mark.parametrize("scale", [1e7, 1e-6])
def test_fp16_far_from_unit_scale(rlu, scale):
    """FP16 products on entries far above and far below unit scale (max|A|
    about 1.2e5 after a 1e7 scale, past FP16's largest finite value, and
    about 1.2e-8 after a 1e-6 scale, under its smallest subnormal): the
    residual rule against the oracle and the sketch within 4 u of |A||G|,
    as at unit scale."""
    A = workloads.spectral_matrix(1600, 1200, workloads.exp_decay(1200, 12.0), 830) * scale
    check_mixed(rlu, A, 40, 48, 831, True, f"fp16 scale {scale:g}")


@pytest.mark.parametrize("fp16", [False, True])
@pytest.mark.parametrize("m,n,k,l", [
    (2048, 1536, 280, 300),   # sketch 384 padded columns, projection 384 rows (eight waves)
    (2048, 1200, 430, 450),   # 512 columns, 512 rows (eight waves)
    (3000, 1100, 560, 700),   # 768 columns (eight waves), 576 rows (four waves)
])
def test_mixed_wide_streaming_tiles(rlu, m, n, k, l, fp16):
    """The streaming products at the wider compiled widths (K >= 1024 on
    both passes), by the same rule as every mixed case."""
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), l / 4.0), 900 + l)
    check_mixed(rlu, A, k, l, 910 + l, fp16, "mixed wide tiles")
