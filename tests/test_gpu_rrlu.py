"""Parity of the rank-revealing Step 3 (RLU_FLAG_RRLU: Algorithm 4.1 as
listed, P Y Q_y = L_y U_y with Q_y the column order of a column-pivoted QR)
with the oracle, through the C ABI.

FP64 rule: the GPU takes the column order from a pivoted Cholesky of the
Gram matrix Y^T Y (the column-pivoted QR's order in exact arithmetic), whose
squared norms carry an absolute error of about u ||Y||^2, so the order is
compared on the prefix the oracle's column-pivoted QR decides with a
relative norm gap >= 1e-4 and a norm >= 1e3 sqrt(u) max column norm.  Where
near ties leave part of the first k undecided (the 8192^2 sketch's columns
have nearly equal norms), the GPU's order must be a valid column-pivoted
order (each choice the largest remaining norm up to the Gram route's
rounding) and the rest is compared with the oracle following that order.
Then Step 3's pivots on the decided prefix and the unpermuted factors P^T L,
U Q^T within 1e-10 as in the plain rule.  FP32 and BF16: the residual rule.
The flag is refused where it is not supported.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import (ensure_built, rel_maxdiff, to_dev_colmajor, to_host, unpermute_cols,
                           unpermute_rows)
from oracle import rlu as orl
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-10
QY_GATE = dict(u=2.0 ** -26, gap_min=1e-4, mag_factor=1e3)


@pytest.fixture(scope="module")
def rlu():
    ensure_built()
    import paper_1310_7202_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return m


def compare_rrlu(rlu, A, k, l, G, label=""):
    print(f"[rrlu] {label} m={A.shape[0]} n={A.shape[1]} k={k} l={l}", flush=True)
    out = rlu.factor(to_dev_colmajor(A), k, l, G=to_dev_colmajor(G), diagnostics=True, rrlu=True)
    torch.cuda.synchronize()
    o = orl.randomized_lu(A, k, l, G, step3="rrlu")
    info = to_host(out.info)
    assert info[2] == 0
    m, n = A.shape
    L, U, p, q = to_host(out.L), to_host(out.U), to_host(out.p), to_host(out.q)
    np.testing.assert_array_equal(np.sort(p), np.arange(m))
    np.testing.assert_array_equal(np.sort(q), np.arange(n))
    qy = to_host(out.qy)
    np.testing.assert_array_equal(np.sort(qy), np.arange(l))
    assert np.all(np.diag(L[:k]) == 1.0) and np.all(np.triu(L[:k], 1) == 0.0)
    assert np.all(np.tril(U, -1) == 0.0)
    assert rel_maxdiff(to_host(out.Y), o["Y"]) < 1e-13
    gq = orl.pivot_gate(o["diag_qy"], **QY_GATE)
    np.testing.assert_array_equal(qy[:gq], o["qy"][:gq])
    print(f"  column order decided on {gq} of {l}", flush=True)
    if gq < k:
        # near ties in the column norms: several orders are correct.  The
        # GPU's must be a valid column-pivoted QR order over its first k
        # entries (each chosen remaining norm the largest, up to the Gram
        # route's rounding: squared norms carry an error of about l^2 u
        # max|y_c|^2, relative 10 l^2 u (max|y_c| / norm)^2 on a norm), and
        # the rest is compared with the oracle following that order
        o = orl.randomized_lu(A, k, l, G, step3="rrlu", order=qy)
        dq = o["diag_qy"]
        tol = 10 * l * l * 2.0 ** -53 * (dq["max_abs"] / dq["piv_abs"][:k]) ** 2 + 1e-12
        worst = float(np.max((1.0 - dq["ratio"][:k]) / tol))
        print(f"  GPU order valid over its first {k}: worst ratio deficit {worst:.3f} of "
              f"the rounding bound", flush=True)
        assert np.all(dq["ratio"][:k] >= 1.0 - tol)
    gy = orl.pivot_gate(o["diag_y"])
    upto = min(gy, k)
    np.testing.assert_array_equal(to_host(out.ipiv)[:upto], o["ipiv"][:upto])
    if gy < k:
        pytest.skip(f"Step 3 pivot {gy} is not numerically decided")
    assert rel_maxdiff(to_host(out.B), o["B"]) < TOL
    gb = orl.pivot_gate(o["diag_b"])
    np.testing.assert_array_equal(to_host(out.qpiv)[:gb], o["qpiv"][:gb])
    if gb == k:
        np.testing.assert_array_equal(q, o["q"])
        assert rel_maxdiff(unpermute_rows(L, p), unpermute_rows(o["L"], o["p"])) < TOL
        assert rel_maxdiff(unpermute_cols(U, q), unpermute_cols(o["U"], o["q"])) < TOL
    return out, o


@pytest.mark.parametrize("m,n,k,l,rate", [
    (3000, 2500, 50, 80, 20.0),     # several workgroups per panel, l well above k
    (700, 1300, 33, 41, 8.0),       # m < n
    (1300, 700, 40, 40, 8.0),       # k = l: only the order of the columns changes
    (97, 131, 5, 9, 3.0),           # below one tile
    (2000, 1800, 100, 300, 40.0),   # l = 300: the Gram-route order over a wide sketch
])
def test_rrlu_spectral_shapes(rlu, m, n, k, l, rate):
    A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), rate), 5000 + m)
    G = workloads.gaussian((n, l), 5100 + n)
    compare_rrlu(rlu, A, k, l, G, f"spectral rate={rate}")


def test_rrlu_small_config(rlu):
    A, k, l = workloads.config_small(101)
    G = workloads.gaussian((A.shape[1], l), 7203)
    compare_rrlu(rlu, A, k, l, G, "512^2 rank-10")


def test_rrlu_lowers_the_error_with_oversampling(rlu):
    # the extra sketch columns reach the result: mean error over draws
    # below partial pivoting's, as the oracle's pin states
    k = 20
    ratios = []
    for seed in range(5200, 5206):
        A = workloads.spectral_matrix(400, 300, workloads.exp_decay(300, 6.0), seed)
        Ad = to_dev_colmajor(A)
        G = to_dev_colmajor(workloads.gaussian((300, 3 * k), seed + 1))
        part = rlu.factor(Ad, k, 3 * k, G=G)
        rr = rlu.factor(Ad, k, 3 * k, G=G, rrlu=True)
        torch.cuda.synchronize()
        e = [orl.relative_residual(A, {"L": to_host(f.L), "U": to_host(f.U), "p": to_host(f.p),
                                       "q": to_host(f.q)}) for f in (part, rr)]
        ratios.append(e[1] / e[0])
    print(f"  rrlu / partial error ratios {np.round(ratios, 3)}", flush=True)
    assert np.mean(ratios) < 0.75


@pytest.mark.parametrize("precision", [1, 2])
def test_rrlu_reduced_precision_residual_rule(rlu, precision):
    A = workloads.spectral_matrix(3000, 2500, workloads.exp_decay(2500, 20.0), 5300)
    A32 = A.astype(np.float32)
    G32 = workloads.gaussian((2500, 70), 5301).astype(np.float32)
    out = rlu.factor(to_dev_colmajor(A32), 50, 70, G=to_dev_colmajor(G32), precision=precision,
                     rrlu=True)
    torch.cuda.synchronize()
    assert to_host(out.info).tolist() == [0, 0, 0]
    A64 = A32.astype(np.float64)
    o = orl.randomized_lu(A64, 50, 70, G32.astype(np.float64), step3="rrlu")
    g = {"L": to_host(out.L).astype(np.float64), "U": to_host(out.U).astype(np.float64),
         "p": to_host(out.p), "q": to_host(out.q)}
    r_gpu, r_ora = orl.relative_residual(A64, g), orl.relative_residual(A64, o)
    print(f"  precision {precision}: residual gpu {r_gpu:.3e} oracle {r_ora:.3e}", flush=True)
    assert r_gpu <= r_ora + 1e-3


def test_rrlu_is_refused_where_unsupported(rlu):
    A = to_dev_colmajor(workloads.gaussian((300, 200), 5400))
    pb, io, out = rlu._prepare(A, 5, 8, None, 0, None, False, None)
    pb.flags |= rlu.FLAG_RRLU
    h = rlu.Handle(0)
    try:
        st = rlu.lib().rlu_factor_batched(h.ptr, 1, ctypes.byref(pb), ctypes.byref(io),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == -8   # RLU_ERR_UNSUPPORTED
    finally:
        h.close()
    srv = rlu.Server(0)
    try:
        t = ctypes.c_uint64()
        st = rlu.lib().rlu_serve_submit(srv._s, ctypes.byref(pb), ctypes.c_void_p(A.data_ptr()),
                                        300, ctypes.byref(t))
        assert st == -8
    finally:
        srv.close()
