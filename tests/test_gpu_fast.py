"""Parity of Algorithm 4.4, fast randomized LU (RLU_FLAG_FAST, Section 4.5),
with the oracle (oracle/fast.py), through the C ABI.

Both sides draw the SRFT from the same seed by the same definition (the
integer draws are equal bit for bit; the Hartley entries differ by the
rounding of two sine/cosine implementations), so:
  * the sketch Y = A R matches to 1e-12 relative;
  * the pivots of Step 3 match on the decided prefix (oracle.rlu.pivot_gate)
    and, with all l decided, the ID's rows J = p[0:l] match exactly;
  * B = L_y^+ P X A(J, :) and the unpermuted factors P^T L, U Q^T match to
    1e-10 relative (the FP64 rule), with Step 6's pivots decided;
  * the structure is exact.
FP32 storage: the residual rule.  The flag is refused where it is not
supported.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import (ensure_built, rel_maxdiff, to_dev_colmajor, to_host, unpermute_cols,
                           unpermute_rows)
from oracle import fast as ofast, rlu as orl
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


def compare_fast(rlu, A, k, l, seed, label="", rrlu=False):
    print(f"[fast] {label} m={A.shape[0]} n={A.shape[1]} k={k} l={l} rrlu={rrlu}", flush=True)
    out = rlu.factor(to_dev_colmajor(A), k, l, seed=seed, diagnostics=True, fast=True, rrlu=rrlu)
    torch.cuda.synchronize()
    o = ofast.fast_randomized_lu_seeded(A, k, l, seed, step3="rrlu" if rrlu else "partial")
    info = to_host(out.info)
    assert info[2] == 0
    assert (int(info[0]), int(info[1])) == o["info"]
    m, n = A.shape
    L, U, p, q = to_host(out.L), to_host(out.U), to_host(out.p), to_host(out.q)
    np.testing.assert_array_equal(np.sort(p), np.arange(m))
    np.testing.assert_array_equal(np.sort(q), np.arange(n))
    assert np.all(np.diag(L[:k]) == 1.0) and np.all(np.triu(L[:k], 1) == 0.0)
    assert np.all(np.tril(U, -1) == 0.0)
    assert rel_maxdiff(to_host(out.Y), o["Y"]) < 1e-12
    if rrlu:
        gq = orl.pivot_gate(orl.column_pivoted_qr(o["Y"])[2], u=2.0 ** -26, gap_min=1e-4)
        if gq < l:
            pytest.skip(f"column order decided on {gq} of {l}")
        np.testing.assert_array_equal(to_host(out.qy), o["qy"])
    gy = orl.pivot_gate(o["diag_y"])
    np.testing.assert_array_equal(to_host(out.ipiv)[:gy], o["ipiv"][:gy])
    if gy < l:
        # the ID takes all l pivot rows: undecided pivots change J
        pytest.skip(f"Step 3 pivot {gy} of {l} is not numerically decided")
    np.testing.assert_array_equal(p[:l], o["J"])
    assert rel_maxdiff(to_host(out.B), o["B"]) < TOL
    gb = orl.pivot_gate(o["diag_b"])
    np.testing.assert_array_equal(to_host(out.qpiv)[:gb], o["qpiv"][:gb])
    if gb == k:
        np.testing.assert_array_equal(q, o["q"])
        np.testing.assert_array_equal(p, o["p"])
        assert rel_maxdiff(L, o["L"]) < TOL
        assert rel_maxdiff(U, o["U"]) < TOL
    return out, o


@pytest.mark.parametrize("m,n,k,l,rate", [
    (3000, 2500, 50, 80, 20.0),     # several workgroups per panel, l above k
    (700, 1300, 33, 41, 8.0),       # m < n
    (1300, 700, 40, 40, 8.0),       # k = l (T is empty)
    (97, 131, 5, 9, 3.0),           # below one tile
    (2048, 1536, 64, 200, 30.0),    # l = 200: the ID solve over a wide sketch
])
def test_fast_spectral_shapes(rlu, m, n, k, l, rate):
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), 6000 + m)
    compare_fast(rlu, A, k, l, 6100 + n, f"spectral rate={rate}")


def test_fast_small_config(rlu):
    A, k, l = workloads.config_small(101)
    compare_fast(rlu, A, k, l, 7207, "512^2 rank-10")


def test_fast_with_the_rank_revealing_step(rlu):
    A = workloads.spectral_matrix(1500, 1200, workloads.exp_decay(1200, 15.0), 6200)
    compare_fast(rlu, A, 30, 60, 6201, "rrlu", rrlu=True)


def test_fast_exact_rank(rlu):
    A = workloads.low_rank_plus_noise(900, 700, 12, 0.0, 6300)
    out = rlu.factor(to_dev_colmajor(A), 12, 20, seed=6301, fast=True)
    torch.cuda.synchronize()
    g = {"L": to_host(out.L), "U": to_host(out.U), "p": to_host(out.p), "q": to_host(out.q)}
    assert orl.relative_residual(A, g) < 1e-11


def test_fast_fp32_residual_rule(rlu):
    A = workloads.spectral_matrix(3000, 2500, workloads.exp_decay(2500, 20.0), 6400)
    A32 = A.astype(np.float32)
    out = rlu.factor(to_dev_colmajor(A32), 50, 80, seed=6401, fast=True)
    torch.cuda.synchronize()
    assert to_host(out.info).tolist() == [0, 0, 0]
    A64 = A32.astype(np.float64)
    o = ofast.fast_randomized_lu_seeded(A64, 50, 80, 6401)
    g = {"L": to_host(out.L).astype(np.float64), "U": to_host(out.U).astype(np.float64),
         "p": to_host(out.p), "q": to_host(out.q)}
    r_gpu, r_ora = orl.relative_residual(A64, g), orl.relative_residual(A64, o)
    print(f"  fp32 fast: residual gpu {r_gpu:.3e} oracle {r_ora:.3e}", flush=True)
    assert r_gpu <= r_ora + 1e-3


def test_fast_is_refused_where_unsupported(rlu):
    A = workloads.gaussian((300, 200), 6500)
    Ad = to_dev_colmajor(A)
    G = to_dev_colmajor(workloads.gaussian((200, 8), 6501))
    with pytest.raises(rlu.RluError):
        rlu.factor(Ad, 5, 8, G=G, fast=True)                   # caller's G
    with pytest.raises(rlu.RluError):
        rlu.factor(Ad, 5, 8, fast=True, power_iters=1)         # no power scheme
    with pytest.raises(rlu.RluError):
        rlu.factor(Ad.float(), 5, 8, fast=True, precision=rlu.PREC_MIXED_BF16)
    pb, io, out = rlu._prepare(Ad, 5, 8, None, 0, None, False, None)
    pb.flags |= rlu.FLAG_FAST
    h = rlu.Handle(0)
    try:
        st = rlu.lib().rlu_factor_batched(h.ptr, 1, ctypes.byref(pb), ctypes.byref(io),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == -8
    finally:
        h.close()
