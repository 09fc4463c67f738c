"""C ABI checks that need no GPU: the library loads, exports every function
include/rlu.h declares, and validates arguments before touching a device."""
import ctypes
import os
import re

import pytest

from tests.helpers import ROOT, ensure_built


@pytest.fixture(scope="module")
def rlu():
    ensure_built()
    import paper_1310_7202_amd as m
    return m


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "rlu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rlu_[a-z_]+)\s*\(", src)))


def test_header_declares_what_the_binding_lists(rlu):
    assert _declared_functions() == sorted(rlu.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(rlu):
    lib = ctypes.CDLL(rlu.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(rlu):
    for st in rlu.STATUS:
        s = rlu.status_string(st)
        assert isinstance(s, str) and s and s != "unknown status"
    assert rlu.lib().rlu_version().decode().startswith("rlu-mi355x")


def test_check_info_mapping(rlu):
    assert rlu.check_info([0, 0, 0]) == 0
    assert rlu.check_info([3, 0, 0]) == 2
    assert rlu.check_info([0, 1, 0]) == 2
    assert rlu.check_info([0, 0, 1]) == -3
    # info[2] bit 1: the requested non-finite check found a NaN / infinity
    assert rlu.check_info([0, 0, 2]) == -6
    assert rlu.check_info([4, 0, 2]) == -6
    # an exchange failure dominates (the outputs are undefined)
    assert rlu.check_info([0, 0, 3]) == -3
    # bits this version does not define read as a device failure
    assert rlu.check_info([0, 0, 4]) == -3


def test_check_finite_flag_is_accepted(rlu):
    # the flag is implemented, not reserved: valid on every precision
    for dtype, prec in ((0, 0), (1, 1), (1, 2), (1, 3)):
        assert _ws(rlu, 100, 100, 5, 8, dtype=dtype, prec=prec, flags=rlu.FLAG_CHECK_FINITE)[0] == 0
        assert _ws(rlu, 100, 100, 5, 8, dtype=dtype, prec=prec,
                   flags=rlu.FLAG_CHECK_FINITE | rlu.FLAG_DIAGNOSTICS)[0] == 0


def test_rrlu_flag_workspace_and_limits(rlu):
    st, plain = _ws(rlu, 3000, 2500, 50, 80)
    st2, rr = _ws(rlu, 3000, 2500, 50, 80, flags=rlu.FLAG_RRLU)
    assert st == 0 and st2 == 0
    # the Gram matrix, R and the column order (l x l, l x l, l) and Y Q_y (m x l)
    # (each absent area already holds one 256-byte aligned slot)
    assert rr - plain >= 8 * (2 * 80 * 80 + 3000 * 80) - 4 * 256
    assert _ws(rlu, 4000, 4000, 10, 1024, flags=rlu.FLAG_RRLU)[0] == 0
    assert _ws(rlu, 4000, 4000, 10, 1025, flags=rlu.FLAG_RRLU)[0] == -8
    assert _ws(rlu, 4000, 4000, 10, 1025)[0] == 0
    # the batched form (and so the server) does not take the flag
    pb = rlu.Problem(300, 200, 5, 8, 0, 0, 0, None, 0, rlu.FLAG_RRLU, 0)
    out = ctypes.c_size_t()
    assert rlu.lib().rlu_serve_footprint(ctypes.byref(pb), ctypes.byref(out)) == -8


def test_fast_flag_validation(rlu):
    F = rlu.FLAG_FAST
    st, plain = _ws(rlu, 3000, 2500, 50, 80)
    st2, fast = _ws(rlu, 3000, 2500, 50, 80, flags=F)
    assert st == 0 and st2 == 0
    # the ID's A(J, :) (l x n) and the k x l Gram, T and W matrices
    assert fast - plain >= 8 * (80 * 2500 + 3 * 50 * 30)
    assert _ws(rlu, 3000, 2500, 50, 80, dtype=1, prec=1, flags=F)[0] == 0
    assert _ws(rlu, 3000, 2500, 50, 80, flags=F | rlu.FLAG_RRLU)[0] == 0
    assert _ws(rlu, 3000, 2500, 50, 80, G=1, ldg=2500, flags=F)[0] == -1        # caller's G
    assert _ws(rlu, 3000, 2500, 50, 80, flags=F, power_iters=1)[0] == -1        # power scheme
    assert _ws(rlu, 3000, 2500, 50, 80, dtype=1, prec=2, flags=F)[0] == -8      # BF16 products
    assert _ws(rlu, 4000, 4000, 10, 1025, flags=F)[0] == -8
    pb = rlu.Problem(300, 200, 5, 8, 0, 0, 0, None, 0, F, 0)
    out = ctypes.c_size_t()
    assert rlu.lib().rlu_serve_footprint(ctypes.byref(pb), ctypes.byref(out)) == -8


def test_exchange_limit_argument_checks(rlu):
    lib = rlu.lib()
    assert lib.rlu_set_exchange_limit(None, 0, 0) == -1
    h = ctypes.c_void_p(1)   # never dereferenced: the argument check comes first
    assert lib.rlu_set_exchange_limit(h, 0, 2) == -1
    assert lib.rlu_set_exchange_limit(h, 0, -1) == -1


def _ws(rlu, m, n, k, l, dtype=0, prec=0, G=None, ldg=0, flags=0, power_iters=0):
    pb = rlu.Problem(m, n, k, l, dtype, prec, 0, G, ldg, flags, power_iters)
    out = ctypes.c_size_t()
    st = rlu.lib().rlu_workspace_size(ctypes.byref(pb), ctypes.byref(out))
    return st, out.value


@pytest.mark.parametrize("m,n,k,l", [
    (0, 10, 1, 1), (10, 0, 1, 1), (10, 10, 0, 1), (10, 10, 3, 2),
    (10, 5, 3, 6), (5, 10, 3, 6), (10, 10, -1, 2),
])
def test_invalid_shapes_rejected(rlu, m, n, k, l):
    st, _ = _ws(rlu, m, n, k, l)
    assert st == -1


def test_invalid_dtype_precision_rejected(rlu):
    assert _ws(rlu, 100, 100, 5, 8, dtype=0, prec=1)[0] == -1   # FP32 arithmetic on FP64 storage
    assert _ws(rlu, 100, 100, 5, 8, dtype=7, prec=0)[0] == -1
    assert _ws(rlu, 100, 100, 5, 8, dtype=0, prec=9)[0] == -1
    assert _ws(rlu, 100, 100, 5, 8, G=1, ldg=50)[0] == -1       # ldg < n
    assert _ws(rlu, 100, 100, 5, 8, flags=1 << 7)[0] == -1


def test_workspace_size_grows_with_problem(rlu):
    st1, a = _ws(rlu, 512, 512, 10, 15)
    st2, b = _ws(rlu, 8192, 8192, 200, 210)
    assert st1 == 0 and st2 == 0 and 0 < a < b
    # G passed by the caller: no G workspace
    st3, c = _ws(rlu, 8192, 8192, 200, 210, G=1, ldg=8192)
    assert st3 == 0 and c < b
    # the dominant terms: Y (m l), C and B (2 k n) in FP64
    assert b >= 8 * (8192 * 210 + 2 * 200 * 8192)


def test_power_iterations_range_and_workspace(rlu):
    """Section 5.2: q in 0..RLU_MAX_POWER_ITERS; q > 0 adds the n x l blocks
    of the power scheme (Z^T and Z in FP64, the normalized block in the
    storage type) even when the caller passes G."""
    assert rlu.MAX_POWER_ITERS == 16
    assert _ws(rlu, 100, 100, 5, 8, power_iters=-1)[0] == -1
    assert _ws(rlu, 100, 100, 5, 8, power_iters=17)[0] == -1
    st0, a = _ws(rlu, 4096, 3000, 40, 48)
    st1, b = _ws(rlu, 4096, 3000, 40, 48, power_iters=1)
    st2, c = _ws(rlu, 4096, 3000, 40, 48, power_iters=16)
    assert st0 == st1 == st2 == 0
    assert b - a >= 2 * 8 * 3000 * 48 - 4096 and c == b  # slots are 256-byte aligned
    st3, d = _ws(rlu, 4096, 3000, 40, 48, G=1, ldg=3000, power_iters=1)
    assert st3 == 0 and d == b
    # the server runs a request with power iterations alone, so its
    # footprint is the single-problem workspace
    pb = rlu.Problem(512, 512, 10, 15, 0, 0, 0, None, 0, 0, 1)
    out = ctypes.c_size_t()
    assert rlu.lib().rlu_serve_footprint(ctypes.byref(pb), ctypes.byref(out)) == 0
    assert out.value > _ws(rlu, 512, 512, 10, 15, power_iters=1)[1]
    pb.power_iters = 17
    assert rlu.lib().rlu_serve_footprint(ctypes.byref(pb), ctypes.byref(out)) == -1
    pb.power_iters = 1
    io = rlu.Buffers()
    io.A = io.L = io.U = io.p = io.q = io.info = 1
    io.lda = io.ldl = 512
    io.ldu = 10
    # one q per batched call
    pbs = (rlu.Problem * 2)(rlu.Problem(512, 512, 10, 15, 0, 0, 0, None, 0, 0, 1),
                            rlu.Problem(512, 512, 10, 15, 0, 0, 0, None, 0, 0, 2))
    ios = (rlu.Buffers * 2)(io, io)
    assert rlu.lib().rlu_factor_batched(ctypes.c_void_p(1), 2, pbs, ios, None) == -1


def test_factor_rejects_null_handle_and_buffers(rlu):
    lib = rlu.lib()
    pb = rlu.Problem(100, 100, 5, 8, 0, 0, 0, None, 0, 0)
    io = rlu.Buffers()
    assert lib.rlu_factor(None, ctypes.byref(pb), ctypes.byref(io), None) == -1
    # a fake non-null handle is never dereferenced before validation fails
    assert lib.rlu_factor(ctypes.c_void_p(1), ctypes.byref(pb), None, None) == -1
    assert lib.rlu_factor(ctypes.c_void_p(1), ctypes.byref(pb), ctypes.byref(io), None) == -1


def test_create_rejects_bad_device(rlu):
    h = ctypes.c_void_p()
    assert rlu.lib().rlu_create(ctypes.byref(h), -1) < 0
    assert rlu.lib().rlu_create(None, 0) == -1


def test_serve_footprint_counts_workspace_and_outputs(rlu):
    small = rlu.serve_footprint(512, 512, 10, 15)
    big = rlu.serve_footprint(4096, 3000, 64, 72)
    assert 0 < small < big
    # at least the outputs (L, U, p, q) and the sketch Y, B, C it must hold
    m, n, k, l = 4096, 3000, 64, 72
    assert big >= 8 * (m * k + k * n) + 8 * (m + n) + 8 * (m * l + 2 * k * n)
    # FP32 storage charges less than FP64 for the same shape
    assert rlu.serve_footprint(m, n, k, l, rlu.F32, rlu.PREC_FP32) < big


def test_serve_footprint_rejects_bad_problems(rlu):
    lib = rlu.lib()
    out = ctypes.c_size_t()
    bad = rlu.Problem(10, 10, 3, 2, 0, 0, 0, None, 0, 0)
    assert lib.rlu_serve_footprint(ctypes.byref(bad), ctypes.byref(out)) == -1
    diag = rlu.Problem(100, 100, 5, 8, 0, 0, 0, None, 0, rlu.FLAG_DIAGNOSTICS)
    assert lib.rlu_serve_footprint(ctypes.byref(diag), ctypes.byref(out)) == -1
    assert lib.rlu_serve_footprint(None, ctypes.byref(out)) == -1


def test_serve_entry_points_reject_null_server(rlu):
    lib = rlu.lib()
    pb = rlu.Problem(100, 100, 5, 8, 0, 0, 0, None, 0, 0)
    t = ctypes.c_uint64()
    assert lib.rlu_serve_submit(None, ctypes.byref(pb), ctypes.c_void_p(1), 100,
                                ctypes.byref(t)) == -1
    assert lib.rlu_serve_poll(None, 1, None) == -1
    assert lib.rlu_serve_release(None, 1) == -1
    assert lib.rlu_serve_copy(None, 1, None, None) == -1
    assert lib.rlu_serve_stats(None, None, None, None) == -1
    assert lib.rlu_serve_destroy(None) == -1
    assert lib.rlu_serve_create(None, None) == -1


def test_batched_rejects_bad_arguments_before_any_device_work(rlu):
    lib = rlu.lib()
    assert lib.rlu_factor_batched(ctypes.c_void_p(1), 0, None, None, None) == 0
    assert lib.rlu_factor_batched(None, 1, None, None, None) == -1
    assert lib.rlu_factor_batched(ctypes.c_void_p(1), 2, None, None, None) == -1
    pbs = (rlu.Problem * 2)(rlu.Problem(100, 100, 5, 8, 0, 0, 0, None, 0, 0),
                            rlu.Problem(100, 100, 5, 8, 1, 1, 0, None, 0, 0))
    ios = (rlu.Buffers * 2)()
    for i in range(2):
        ios[i].A = ios[i].L = ios[i].U = ios[i].p = ios[i].q = ios[i].info = 1
        ios[i].lda = ios[i].ldl = 100
        ios[i].ldu = 5
    # mixed dtypes in one call
    assert lib.rlu_factor_batched(ctypes.c_void_p(1), 2, pbs, ios, None) == -1


def test_timing_rejects_null_handle_and_unknown_modes(rlu):
    """rlu_set_timing: 0 off, 1 every phase, 2 the sketch product only;
    a null handle or any other mode is an argument error (no device work)."""
    lib = rlu.lib()
    for mode in (0, 1, 2):
        assert lib.rlu_set_timing(None, mode) == -1
    assert lib.rlu_set_timing(None, 3) == -1


def _ls(rlu, m=100, n=80, k=5, nrhs=1, dtype=0, ldl=None, ldu=None, ldb=None, ldx=None):
    d = rlu.LstsqDesc(m, n, k, dtype, 1, ldl if ldl is not None else m,
                      1, ldu if ldu is not None else k, 1, 1, nrhs,
                      1, ldb if ldb is not None else m, 1, ldx if ldx is not None else n)
    out = ctypes.c_size_t()
    return rlu.lib().rlu_lstsq_workspace_size(ctypes.byref(d), ctypes.byref(out)), out.value, d


def test_lstsq_argument_checks(rlu):
    """Algorithm 4.3 entry point: shapes, leading dimensions and the k limit
    are checked on the host before any device work."""
    assert _ls(rlu)[0] == 0
    assert _ls(rlu, k=0)[0] == -1
    assert _ls(rlu, k=81)[0] == -1            # k > min(m, n)
    assert _ls(rlu, nrhs=-1)[0] == -1
    assert _ls(rlu, dtype=5)[0] == -1
    assert _ls(rlu, ldl=99)[0] == -1
    assert _ls(rlu, ldu=4)[0] == -1
    assert _ls(rlu, ldb=99)[0] == -1
    assert _ls(rlu, ldx=79)[0] == -1
    assert _ls(rlu, m=3000, n=2000, k=1025)[0] == -8
    st1, a, _ = _ls(rlu, m=3000, n=2000, k=40, nrhs=1)
    st2, b, _ = _ls(rlu, m=3000, n=2000, k=40, nrhs=64)
    st3, c, _ = _ls(rlu, m=3000, n=2000, k=40, nrhs=64, dtype=1)
    assert st1 == st2 == st3 == 0 and a < b < c   # FP32 b is widened to FP64
    assert b >= 8 * (3000 * 40 + 2 * 40 * 64)
    _, _, d = _ls(rlu)
    assert rlu.lib().rlu_lstsq(None, ctypes.byref(d), None) == -1
    assert rlu.lib().rlu_lstsq(ctypes.c_void_p(1), None, None) == -1
    d.ldx = 3
    assert rlu.lib().rlu_lstsq(ctypes.c_void_p(1), ctypes.byref(d), None) == -1
