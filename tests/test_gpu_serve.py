"""Serving form (rlu_serve_*): continuous batching with HBM-footprint
admission, checked against the FP64 oracle, for alone == in-mix, and for the
admission rules (budget, queue bound, oversize rejection).

Rules: FP64 requests follow the FP64 parity rule of the batched tests; a
request's factors are bitwise identical whether it ran alone or in a mix
(each problem's arithmetic depends only on that problem); the server never
admits beyond its budget.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import ensure_built, rel_maxdiff, to_dev_colmajor, to_host, unpermute_rows
from oracle import rlu as orl
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


SHAPES = [(300, 500, 8, 16), (1200, 700, 40, 48), (2048, 1500, 64, 72), (97, 131, 5, 9),
          (640, 640, 20, 28), (4096, 300, 12, 20)]


def _inputs(seed0):
    out = []
    for i, (m, n, k, l) in enumerate(SHAPES):
        A = workloads.low_rank_plus_noise(m, n, k, 1e-6, seed0 + i)
        G = workloads.gaussian((n, l), seed0 + 50 + i)
        out.append((A, k, l, G))
    return out


def _check(A, k, l, G, f, power=0):
    # the power scheme's element-by-element rule uses the normalized reading
    # of Section 5.2 (low rank + noise: the plain product's rounding would
    # dominate at these k)
    o = orl.randomized_lu(A, k, l, G, q=power, scheme="normalized" if power else "auto")
    L, U, p, q, info = (to_host(f.L), to_host(f.U), to_host(f.p), to_host(f.q),
                        to_host(f.info))
    assert info[2] == 0 and (int(info[0]), int(info[1])) == o["info"]
    gy, gb = orl.pivot_gate(o["diag_y"]), orl.pivot_gate(o["diag_b"])
    assert gy >= k and gb == k
    np.testing.assert_array_equal(q, o["q"])
    assert rel_maxdiff(unpermute_rows(L, p), unpermute_rows(o["L"], o["p"])) < TOL
    assert rel_maxdiff(U, o["U"]) < TOL


def test_served_results_match_oracle(rlu):
    srv = rlu.Server(0)
    probs = _inputs(1200)
    print(f"[serve] {len(probs)} FP64 requests", flush=True)
    devs = [(to_dev_colmajor(A), to_dev_colmajor(G)) for A, k, l, G in probs]
    tickets = [srv.submit(Ad, k, l, G=Gd) for (Ad, Gd), (A, k, l, G) in zip(devs, probs)]
    for t in tickets:
        assert srv.wait(t) == 0
    for t, (A, k, l, G) in zip(tickets, probs):
        st, r = srv.poll(t)
        assert st == 0
        assert 0 <= r.t_submit_us <= r.t_start_us <= r.t_done_us
        _check(A, k, l, G, srv.result(t))
        assert srv.release(t) == 0
    assert srv.poll(tickets[0])[0] == -7  # released: unknown ticket
    used, queued, inflight = srv.stats()
    assert used == 0 and queued == 0 and inflight == 0
    srv.close()


def test_alone_equals_in_mix(rlu):
    srv = rlu.Server(0)
    probs = _inputs(1300)
    devs = [(to_dev_colmajor(A), to_dev_colmajor(G)) for A, k, l, G in probs]
    print("[serve] alone vs in-mix", flush=True)
    alone = []
    for (Ad, Gd), (A, k, l, G) in zip(devs, probs):
        t = srv.submit(Ad, k, l, G=Gd)
        assert srv.wait(t) == 0
        f = srv.result(t)
        alone.append(tuple(to_host(x).copy() for x in (f.L, f.U, f.p, f.q)))
        srv.release(t)
    # the same requests, each twice, interleaved with FP64 requests of other
    # shapes, submitted at once
    extra = _inputs(1400)
    exdev = [(to_dev_colmajor(A), to_dev_colmajor(G)) for A, k, l, G in extra]
    tickets = []
    for i in range(2):
        for j, ((Ad, Gd), (A, k, l, G)) in enumerate(zip(devs, probs)):
            tickets.append((j, srv.submit(Ad, k, l, G=Gd)))
            (Ed, EGd), (EA, ek, el, EG) = exdev[j], extra[j]
            tickets.append((-1, srv.submit(Ed, ek, el, G=EGd)))
    for j, t in tickets:
        assert srv.wait(t) == 0
        if j >= 0:
            f = srv.result(t)
            got = tuple(to_host(x) for x in (f.L, f.U, f.p, f.q))
            for a, b in zip(got, alone[j]):
                np.testing.assert_array_equal(a, b)
        srv.release(t)
    srv.close()


def _out_bytes(m, n, k):
    """Outputs the server keeps per FP64 request (L, U, p, q), up to alignment."""
    return 8 * (m * k + k * n + m + n)


def test_admission_respects_budget_and_fifo(rlu):
    m, n, k, l = 2048, 1500, 32, 40
    fp = rlu.serve_footprint(m, n, k, l)
    out = _out_bytes(m, n, k)
    assert 1.5 * out < fp
    # one request at a time fits; a finished request's outputs stay charged
    budget = int(fp + 1.5 * out)
    srv = rlu.Server(0, budget_bytes=budget)
    A = to_dev_colmajor(workloads.low_rank_plus_noise(m, n, k, 1e-6, 77))
    print(f"[serve] budget {budget} bytes, footprint {fp}", flush=True)
    ts = [srv.submit(A, k, l, seed=i) for i in range(3)]
    assert srv.wait(ts[0]) == 0 and srv.wait(ts[1]) == 0
    r0, r1 = srv.poll(ts[0])[1], srv.poll(ts[1])[1]
    assert r1.t_start_us >= r0.t_done_us       # admitted only after the first finished
    time.sleep(0.05)
    assert srv.poll(ts[2])[0] == 1             # two outputs held: no room
    used, queued, inflight = srv.stats()
    assert used <= budget and queued == 1 and inflight == 0
    assert srv.release(ts[2]) == 1             # pending: cannot be released
    srv.release(ts[0])
    assert srv.wait(ts[2]) == 0                # admitted as memory freed up
    for t in ts[1:]:
        srv.release(t)
    # a request larger than the whole budget is rejected at submit
    big = to_dev_colmajor(workloads.low_rank_plus_noise(4096, 4096, 8, 1e-6, 78))
    with pytest.raises(rlu.RluError) as e:
        srv.submit(big, 64, 72)
    assert e.value.status == -4
    srv.close()


def test_queue_bound(rlu):
    m, n, k, l = 1024, 1024, 16, 24
    fp = rlu.serve_footprint(m, n, k, l)
    out = _out_bytes(m, n, k)
    srv = rlu.Server(0, budget_bytes=int(fp + 0.5 * out), max_queue=2)
    A = to_dev_colmajor(workloads.low_rank_plus_noise(m, n, k, 1e-6, 79))
    t0 = srv.submit(A, k, l, seed=1)
    assert srv.wait(t0) == 0           # its outputs hold the budget until released
    t1 = srv.submit(A, k, l, seed=2)
    t2 = srv.submit(A, k, l, seed=3)
    time.sleep(0.05)
    with pytest.raises(rlu.RluError) as e:
        srv.submit(A, k, l, seed=4)
    assert e.value.status == -5
    srv.release(t0)
    assert srv.wait(t1) == 0
    srv.release(t1)
    assert srv.wait(t2) == 0
    srv.release(t2)
    srv.close()


def test_serve_mixed_precision_stream(rlu):
    """A short stream of BF16 requests with sigma_i = exp(-i / k) (the
    serving workload's spectra, smaller sizes): residual rule against the
    oracle on every request."""
    srv = rlu.Server(0)
    g = np.random.default_rng(5)
    reqs = []
    print("[serve] bf16 stream", flush=True)
    for i in range(8):
        m = int(np.exp(g.uniform(np.log(300), np.log(1500))))
        n = int(np.exp(g.uniform(np.log(300), np.log(1200))))
        k = int(g.integers(8, 40))
        l = min(k + 10, m, n)
        A32 = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), k), 900 + i)
        A32 = A32.astype(np.float32)
        Ad = to_dev_colmajor(A32, dtype=torch.float32)
        reqs.append((A32, k, l, srv.submit(Ad, k, l, seed=31 + i,
                                          precision=rlu.PREC_MIXED_BF16), Ad, 31 + i))
        time.sleep(0.002)              # arrivals while earlier requests run
    from oracle import philox
    for A32, k, l, t, _, seed in reqs:
        assert srv.wait(t) == 0
        f = srv.result(t)
        A = A32.astype(np.float64)
        m, n = A.shape
        G = philox.gaussian_matrix(n, l, seed).astype(np.float32).astype(np.float64)
        o = orl.randomized_lu(A, k, l, G)
        g_ = {"L": to_host(f.L).astype(np.float64), "U": to_host(f.U).astype(np.float64),
              "p": to_host(f.p), "q": to_host(f.q)}
        r_gpu = orl.relative_residual(A, g_)
        r_ora = orl.relative_residual(A, o)
        print(f"  {A.shape} k={k} residual gpu {r_gpu:.3e} oracle {r_ora:.3e}", flush=True)
        assert r_gpu <= r_ora + 1e-3
        srv.release(t)
    srv.close()


def test_oversize_request_runs_alone_in_the_mix(rlu):
    """A request whose panel does not fit the batched kernels (30000 rows,
    l = 210: at most 91 rows of that width fit one workgroup's LDS, so the
    panel would need 330 workgroups, more than a gang may have) runs through
    the single-problem path, interleaved with batched requests; its factors
    equal a direct rlu_factor call."""
    srv = rlu.Server(0)
    m, n, k, l = 30000, 1500, 200, 210
    A = workloads.low_rank_plus_noise_torch(m, n, k, 1e-6, 31, dtype=torch.float64)
    ref = rlu.factor(A, k, l, seed=9)
    small = _inputs(1600)
    devs = [(to_dev_colmajor(X), to_dev_colmajor(G)) for X, kk, ll, G in small]
    print("[serve] oversize request in a mix", flush=True)
    ts = [srv.submit(Xd, kk, ll, G=Gd) for (Xd, Gd), (X, kk, ll, G) in zip(devs[:3], small[:3])]
    tb = srv.submit(A, k, l, seed=9)
    ts += [srv.submit(Xd, kk, ll, G=Gd) for (Xd, Gd), (X, kk, ll, G) in zip(devs[3:], small[3:])]
    assert srv.wait(tb) == 0
    f = srv.result(tb)
    torch.cuda.synchronize()
    for a, b in zip((f.L, f.U, f.p, f.q), (ref.L, ref.U, ref.p, ref.q)):
        np.testing.assert_array_equal(to_host(a), to_host(b))
    for t, (X, kk, ll, G) in zip(ts, small):
        assert srv.wait(t) == 0
        _check(X, kk, ll, G, srv.result(t))
        srv.release(t)
    srv.release(tb)
    srv.close()


def test_power_iteration_requests_run_alone_in_the_mix(rlu):
    """Requests with power iterations (Section 5.2) run through the
    single-problem path between batched requests: each equals a direct
    rlu_factor call bitwise and the oracle's power scheme under the FP64
    rule."""
    srv = rlu.Server(0)
    small = _inputs(1700)
    devs = [(to_dev_colmajor(X), to_dev_colmajor(G)) for X, kk, ll, G in small]
    pw = []
    for i, (m, n, k, l, q) in enumerate([(1500, 1100, 30, 38, 1), (900, 1300, 20, 26, 2)]):
        A = workloads.spectral_matrix(m, n, workloads.exp_decay(min(m, n), 15.0), 1750 + i)
        G = workloads.gaussian((n, l), 1760 + i)
        pw.append((A, k, l, G, q, to_dev_colmajor(A), to_dev_colmajor(G)))
    print("[serve] power-iteration requests in a mix", flush=True)
    ts = [srv.submit(Xd, kk, ll, G=Gd) for (Xd, Gd), (X, kk, ll, G) in zip(devs[:3], small[:3])]
    tp = [srv.submit(Ad, k, l, G=Gd, power_iters=q) for A, k, l, G, q, Ad, Gd in pw]
    ts += [srv.submit(Xd, kk, ll, G=Gd) for (Xd, Gd), (X, kk, ll, G) in zip(devs[3:], small[3:])]
    for t, (A, k, l, G, q, Ad, Gd) in zip(tp, pw):
        assert srv.wait(t) == 0
        f = srv.result(t)
        ref = rlu.factor(Ad, k, l, G=Gd, power_iters=q)
        torch.cuda.synchronize()
        for a, b in zip((f.L, f.U, f.p, f.q), (ref.L, ref.U, ref.p, ref.q)):
            np.testing.assert_array_equal(to_host(a), to_host(b))
        _check(A, k, l, G, f, power=q)
        srv.release(t)
    for t, (X, kk, ll, G) in zip(ts, small):
        assert srv.wait(t) == 0
        _check(X, kk, ll, G, srv.result(t))
        srv.release(t)
    srv.close()
