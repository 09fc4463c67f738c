"""Failure reporting of the HIP path, through the C ABI.

  * RLU_FLAG_CHECK_FINITE: a NaN or an infinity in A (or in a caller's G)
    sets info[2] bit 1 and maps to RLU_ERR_NONFINITE, in the single,
    batched and served forms and in every precision; on finite input the
    flag changes nothing (bitwise-equal factors).
  * The pivot exchange's failure path, forced from the host: the failure
    word starts set (as if a partner workgroup had given up), every kernel
    exits normally, info[2] bit 0 is set and maps to RLU_ERR_DEVICE, and the
    next call on the same handle is correct again.  A per-wait limit of zero
    ticks ends every wait at its second unsuccessful poll: the call still
    completes and reports consistently.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import ensure_built, rel_maxdiff, to_dev_colmajor, to_host
from oracle import rlu as orl
import workloads

pytestmark = pytest.mark.gpu

NONFINITE, DEVICE = -6, -3


@pytest.fixture(scope="module")
def rlu():
    ensure_built()
    import paper_1310_7202_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return m


def _matrix(m=600, n=500, seed=3100):
    return workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), 10.0), seed)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_nonfinite_input_is_reported(rlu, bad, precision):
    print(f"[failure] non-finite {bad} precision={precision}", flush=True)
    A = _matrix()
    A[123, 77] = bad
    dt = torch.float64 if precision == 0 else torch.float32
    out = rlu.factor(to_dev_colmajor(A, dt), 20, 26, seed=5, precision=precision,
                     check_finite=True)
    torch.cuda.synchronize()
    info = to_host(out.info).tolist()
    assert info[2] == 2, info
    assert rlu.check_info(info) == NONFINITE


def test_nonfinite_in_callers_g_is_reported(rlu):
    A = _matrix()
    G = workloads.gaussian((A.shape[1], 26), 3101)
    G[40, 3] = np.nan
    out = rlu.factor(to_dev_colmajor(A), 20, 26, G=to_dev_colmajor(G), check_finite=True)
    torch.cuda.synchronize()
    assert rlu.check_info(out.info) == NONFINITE


def test_check_is_opt_in_and_changes_nothing_on_finite_input(rlu):
    A = _matrix()
    Ad = to_dev_colmajor(A)
    plain = rlu.factor(Ad, 20, 26, seed=7)
    checked = rlu.factor(Ad, 20, 26, seed=7, check_finite=True)
    torch.cuda.synchronize()
    assert to_host(checked.info).tolist() == [0, 0, 0]
    for a, b in ((plain.L, checked.L), (plain.U, checked.U), (plain.p, checked.p),
                 (plain.q, checked.q)):
        assert torch.equal(a, b)
    # without the flag a NaN is not looked for (the run still completes)
    A[5, 5] = np.nan
    out = rlu.factor(to_dev_colmajor(A), 20, 26, seed=7)
    torch.cuda.synchronize()
    assert to_host(out.info)[2] == 0


def test_nonfinite_in_one_problem_of_a_batch(rlu):
    print("[failure] batched non-finite", flush=True)
    mats = [_matrix(400, 300, 3110 + i) for i in range(3)]
    clean = [to_dev_colmajor(M) for M in mats]
    ref = rlu.factor_batched([(Ad, 12, 16, 9) for Ad in clean], check_finite=True)
    torch.cuda.synchronize()
    assert all(to_host(f.info).tolist() == [0, 0, 0] for f in ref)
    bad = mats[1].copy()
    bad[10, 20] = np.inf
    devs = [clean[0], to_dev_colmajor(bad), clean[2]]
    outs = rlu.factor_batched([(Ad, 12, 16, 9) for Ad in devs], check_finite=True)
    torch.cuda.synchronize()
    infos = [to_host(f.info).tolist() for f in outs]
    assert infos[1][2] == 2 and rlu.check_info(infos[1]) == NONFINITE
    for i in (0, 2):
        assert infos[i] == [0, 0, 0]
        assert torch.equal(outs[i].L, ref[i].L) and torch.equal(outs[i].U, ref[i].U)


def test_nonfinite_served_request(rlu):
    print("[failure] served non-finite", flush=True)
    srv = rlu.Server(0)
    try:
        A = _matrix(500, 400, 3120).astype(np.float32)
        A[7, 9] = np.nan
        t_bad = srv.submit(to_dev_colmajor(A), 10, 16, seed=1, check_finite=True)
        B = _matrix(500, 400, 3121).astype(np.float32)
        t_ok = srv.submit(to_dev_colmajor(B), 10, 16, seed=1, check_finite=True)
        assert srv.wait(t_bad) == NONFINITE
        assert srv.wait(t_ok) == 0
        srv.release(t_bad)
        srv.release(t_ok)
    finally:
        srv.close()


def test_exchange_failure_forced_from_the_host(rlu):
    # a panel of several workgroups (3000 rows): the exchange is in use
    print("[failure] preset exchange failure", flush=True)
    A = workloads.spectral_matrix(3000, 2500, workloads.exp_decay(2500, 20.0), 3130)
    G = workloads.gaussian((2500, 60), 3131)
    Ad, Gd = to_dev_colmajor(A), to_dev_colmajor(G)
    h = rlu.Handle(0)
    try:
        h.set_exchange_limit(preset_failure=True)
        out = rlu.factor(Ad, 50, 60, G=Gd, handle=h)
        torch.cuda.synchronize()
        info = to_host(out.info).tolist()
        assert info[2] & 1, info
        assert rlu.check_info(info) == DEVICE
        # the next call on the same handle starts clean and is correct
        h.set_exchange_limit()
        out = rlu.factor(Ad, 50, 60, G=Gd, handle=h)
        torch.cuda.synchronize()
        assert to_host(out.info).tolist() == [0, 0, 0]
        o = orl.randomized_lu(A, 50, 60, G)
        L, p = to_host(out.L), to_host(out.p)
        Lu = np.empty_like(L); Lu[p] = L
        Lo = np.empty_like(o["L"]); Lo[o["p"]] = o["L"]
        assert rel_maxdiff(Lu, Lo) < 1e-10
    finally:
        h.close()


def test_zero_tick_wait_limit_completes_and_reports(rlu):
    print("[failure] zero-tick wait limit", flush=True)
    A = workloads.spectral_matrix(3000, 2500, workloads.exp_decay(2500, 20.0), 3132)
    Ad = to_dev_colmajor(A)
    h = rlu.Handle(0)
    try:
        ref = rlu.factor(Ad, 50, 60, seed=3, handle=h)
        torch.cuda.synchronize()
        h.set_exchange_limit(timeout_ticks=0)
        out = rlu.factor(Ad, 50, 60, seed=3, handle=h)
        torch.cuda.synchronize()
        info = to_host(out.info).tolist()
        st = rlu.check_info(info)
        print(f"  info {info} status {st}", flush=True)
        assert info[2] in (0, 1)
        if info[2] == 0:
            assert torch.equal(out.L, ref.L) and torch.equal(out.U, ref.U)
        else:
            assert st == DEVICE
    finally:
        h.close()
