"""rlu_factor_noalloc (the entry point that allocates nothing, its workspace
in the library's fixed device scratch) against rlu_factor, through the C
ABI: two calls in a row on one handle, the second with a smaller input, each
bitwise equal to rlu_factor's output and within the FP64 parity tolerance
of the oracle; a problem whose workspace exceeds the scratch is refused
before any device work."""
import ctypes

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


def _call(rlu, h, A, k, l, G, noalloc):
    pb, io, out = rlu._prepare(A, k, l, None, 0, G, False, None)
    fn = rlu.lib().rlu_factor_noalloc if noalloc else rlu.lib().rlu_factor
    s = torch.cuda.current_stream()
    st = fn(h.ptr, ctypes.byref(pb), ctypes.byref(io), ctypes.c_void_p(s.cuda_stream))
    return st, out


def _unpermuted(L, U, p, q):
    Lu = np.empty_like(L); Lu[p] = L
    Uu = np.empty_like(U); Uu[:, q] = U
    return Lu, Uu


def test_noalloc_equals_rlu_factor_on_two_calls(rlu):
    h = rlu.Handle(0)
    try:
        big = workloads.spectral_matrix(3000, 2500, workloads.exp_decay(2500, 20.0), 4100)
        small, k1, l1 = workloads.config_small(101)
        cases = [(big, 50, 60, workloads.gaussian((2500, 60), 4101)),
                 (small, k1, l1, workloads.gaussian((512, l1), 4102))]
        for A, k, l, G in cases:
            print(f"[noalloc] {A.shape} k={k} l={l}", flush=True)
            Ad, Gd = to_dev_colmajor(A), to_dev_colmajor(G)
            st_ref, ref = _call(rlu, h, Ad, k, l, Gd, noalloc=False)
            st, got = _call(rlu, h, Ad, k, l, Gd, noalloc=True)
            torch.cuda.synchronize()
            assert st_ref == 0 and st == 0, (st_ref, st)
            assert to_host(got.info).tolist() == to_host(ref.info).tolist() == [0, 0, 0]
            for a, b in ((got.L, ref.L), (got.U, ref.U), (got.p, ref.p), (got.q, ref.q)):
                assert torch.equal(a, b)
            o = orl.randomized_lu(A, k, l, G)
            Lg, Ug = _unpermuted(to_host(got.L), to_host(got.U), to_host(got.p), to_host(got.q))
            Lo, Uo = _unpermuted(o["L"], o["U"], o["p"], o["q"])
            assert rel_maxdiff(Lg, Lo) < 1e-10 and rel_maxdiff(Ug, Uo) < 1e-10
    finally:
        h.close()


def test_noalloc_refuses_a_workspace_beyond_the_scratch(rlu):
    m = n = 16384
    k, l = 500, 520
    assert rlu.workspace_size(m, n, k, l) > (64 << 20)
    # real buffers of the full shape, so nothing could be out of bounds
    A = torch.empty((n, m), dtype=torch.float64, device="cuda").t()
    h = rlu.Handle(0)
    try:
        st, _ = _call(rlu, h, A, k, l, None, noalloc=True)
        torch.cuda.synchronize()
        assert st == -4   # RLU_ERR_TOO_LARGE
    finally:
        h.close()
    del A
    torch.cuda.empty_cache()
