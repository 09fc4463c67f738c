"""MI355X-native randomized LU decomposition (Shabat et al., arXiv 1310.7202,
Section 4, Algorithm 4.1).

Thin Python binding over the C ABI of ``librlu.so`` (declared in
``include/rlu.h``): argument marshalling only.  Every step of the
factorization runs in the library's HIP kernels; torch provides device
memory and streams.  If the library has not been built, every call raises
(there is no other compute path).
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass

__all__ = ["RluError", "Handle", "factor", "factor_batched", "lstsq", "Batch", "Server",
           "serve_footprint", "lib", "status_string", "LIB_PATH",
           "F64", "F32", "PREC_FP64", "PREC_FP32", "PREC_MIXED_BF16", "PREC_MIXED_FP16",
           "FLAG_CHECK_FINITE", "FLAG_DIAGNOSTICS", "FLAG_RRLU", "FLAG_FAST", "EXPORTED_SYMBOLS",
           "close_default_handles"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librlu.so")

F64, F32 = 0, 1
PREC_FP64, PREC_FP32, PREC_MIXED_BF16, PREC_MIXED_FP16 = 0, 1, 2, 3
FLAG_CHECK_FINITE, FLAG_DIAGNOSTICS, FLAG_RRLU, FLAG_FAST = 1, 2, 4, 8

STATUS = {
    0: "RLU_OK", 1: "RLU_PENDING", 2: "RLU_WARN_ZERO_PIVOT", -1: "RLU_ERR_INVALID_ARG",
    -2: "RLU_ERR_OUT_OF_MEMORY", -3: "RLU_ERR_DEVICE", -4: "RLU_ERR_TOO_LARGE",
    -5: "RLU_ERR_QUEUE_FULL", -6: "RLU_ERR_NONFINITE", -7: "RLU_ERR_UNKNOWN_TICKET",
    -8: "RLU_ERR_UNSUPPORTED",
}

# every function include/rlu.h declares
EXPORTED_SYMBOLS = ["rlu_create", "rlu_destroy", "rlu_workspace_size", "rlu_factor",
                    "rlu_factor_batched", "rlu_set_tile", "rlu_tile_name", "rlu_serve_create", "rlu_serve_submit",
                    "rlu_serve_poll", "rlu_serve_copy", "rlu_serve_release",
                    "rlu_serve_footprint", "rlu_serve_stats", "rlu_serve_destroy",
                    "rlu_set_timing", "rlu_phase_times", "rlu_check_info",
                    "rlu_status_string", "rlu_version", "rlu_lstsq",
                    "rlu_lstsq_workspace_size", "rlu_set_exchange_limit", "rlu_factor_noalloc"]


class RluError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status_string(status)})")


class Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("l", ctypes.c_int64), ("dtype", ctypes.c_int), ("precision", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("G", ctypes.c_void_p), ("ldg", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("power_iters", ctypes.c_int32)]


MAX_POWER_ITERS = 16


class LstsqDesc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("dtype", ctypes.c_int),
                ("L", ctypes.c_void_p), ("ldl", ctypes.c_int64),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
                ("p", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("nrhs", ctypes.c_int64),
                ("b", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("ldx", ctypes.c_int64)]


class Buffers(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("L", ctypes.c_void_p), ("ldl", ctypes.c_int64),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
                ("p", ctypes.c_void_p), ("q", ctypes.c_void_p), ("info", ctypes.c_void_p),
                ("Y", ctypes.c_void_p), ("ldy", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("ipiv", ctypes.c_void_p), ("qpiv", ctypes.c_void_p), ("qy", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t),
                ("max_inflight", ctypes.c_int32), ("max_queue", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("L", ctypes.c_void_p), ("ldl", ctypes.c_int64),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
                ("p", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("info", ctypes.c_int32 * 3),
                ("t_submit_us", ctypes.c_double), ("t_start_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load librlu.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1310_7202_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.rlu_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
        L.rlu_destroy.argtypes = [ctypes.c_void_p]
        L.rlu_workspace_size.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)]
        L.rlu_factor.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem),
                                 ctypes.POINTER(Buffers), ctypes.c_void_p]
        L.rlu_factor_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem),
                                         ctypes.POINTER(Buffers), ctypes.c_void_p]
        L.rlu_factor_batched.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Problem),
                                         ctypes.POINTER(Buffers), ctypes.c_void_p]
        L.rlu_check_info.argtypes = [ctypes.POINTER(ctypes.c_int32)]
        L.rlu_set_tile.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
        L.rlu_tile_name.argtypes = [ctypes.c_int32]
        L.rlu_tile_name.restype = ctypes.c_char_p
        L.rlu_serve_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]
        L.rlu_serve_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
        L.rlu_serve_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Result)]
        L.rlu_serve_copy.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Buffers),
                                     ctypes.c_void_p]
        L.rlu_serve_release.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.rlu_serve_footprint.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)]
        L.rlu_serve_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]
        L.rlu_serve_destroy.argtypes = [ctypes.c_void_p]
        L.rlu_status_string.argtypes = [ctypes.c_int]
        L.rlu_status_string.restype = ctypes.c_char_p
        L.rlu_version.restype = ctypes.c_char_p
        L.rlu_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.rlu_set_exchange_limit.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        L.rlu_lstsq.argtypes = [ctypes.c_void_p, ctypes.POINTER(LstsqDesc), ctypes.c_void_p]
        L.rlu_lstsq_workspace_size.argtypes = [ctypes.POINTER(LstsqDesc),
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.rlu_phase_times.argtypes = [ctypes.c_void_p, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_char_p), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
        for name in ("rlu_create", "rlu_destroy", "rlu_workspace_size", "rlu_factor",
                     "rlu_factor_batched", "rlu_set_tile", "rlu_check_info", "rlu_set_timing",
                     "rlu_phase_times", "rlu_serve_create", "rlu_serve_submit",
                     "rlu_serve_poll", "rlu_serve_copy", "rlu_serve_release",
                     "rlu_serve_footprint", "rlu_serve_stats", "rlu_serve_destroy",
                     "rlu_lstsq", "rlu_lstsq_workspace_size", "rlu_set_exchange_limit",
                     "rlu_factor_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(st: int) -> str:
    try:
        return lib().rlu_status_string(st).decode()
    except RuntimeError:
        return STATUS.get(st, "unknown")


def _check(st: int, where: str):
    if st < 0:
        raise RluError(st, where)
    return st


class Handle:
    """A library handle bound to one device (caches device workspace)."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().rlu_create(ctypes.byref(self._h), device), "rlu_create")
        self.device = device

    def close(self):
        if self._h:
            lib().rlu_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ptr(self):
        return self._h

    def set_tile(self, product: int, cfg: int):
        """Tile shape of a grouped product of the batched form (-1: tuned table)."""
        _check(lib().rlu_set_tile(self._h, product, cfg), "rlu_set_tile")

    def set_exchange_limit(self, timeout_ticks: int = -1, preset_failure: bool = False):
        """Test hook of the failure path of the pivot exchange (see
        rlu_set_exchange_limit): per-wait limit in 100 MHz ticks (< 0: the
        default) and whether calls start with the failure word set."""
        _check(lib().rlu_set_exchange_limit(self._h, int(timeout_ticks), int(bool(preset_failure))),
               "rlu_set_exchange_limit")

    def set_timing(self, enable=True):
        """True / 1: every phase; 2: the sketch product only; 3: the sketch
        product and every pivoted-LU kernel launch; False / 0: off."""
        mode = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        _check(lib().rlu_set_timing(self._h, mode), "rlu_set_timing")

    def phase_times(self, back: int = 0) -> dict:
        """{phase name: ms} of the call `back` calls before the latest; in
        timing mode 3 also "panel_lu_kernel": [ms of each launch]."""
        cap = 32
        ms = (ctypes.c_float * cap)()
        names = (ctypes.c_char_p * cap)()
        cnt = ctypes.c_int()
        _check(lib().rlu_phase_times(self._h, back, ms, names, cap, ctypes.byref(cnt)),
               "rlu_phase_times")
        out, kern = {}, []
        for i in range(min(cnt.value, cap)):
            name = names[i].decode()
            if name == "panel_lu_kernel":
                kern.append(float(ms[i]))
            else:
                out[name] = float(ms[i])
        if kern:
            out["panel_lu_kernel"] = kern
        return out


# Default handles, one per (device, stream): a handle's workspace is reused by
# every call and nothing orders calls on different streams.
_handles: dict = {}


def default_handle(device: int = 0, stream=None) -> Handle:
    key = (device, int(stream.cuda_stream) if stream is not None else 0)
    h = _handles.get(key)
    if h is None:
        h = _handles[key] = Handle(device)
    return h


def close_default_handles():
    """Destroy the default handles (registered to run at interpreter exit,
    before the HIP runtime and any profiler attached to it shut down)."""
    while _handles:
        _, h = _handles.popitem()
        h.close()


atexit.register(close_default_handles)


def workspace_size(m, n, k, l, dtype=F64, precision=PREC_FP64, with_g=False,
                   power_iters=0) -> int:
    pb = Problem(m, n, k, l, dtype, precision, 0, None, 0, 0, power_iters)
    if with_g:
        pb.G = 1
        pb.ldg = n
    out = ctypes.c_size_t()
    _check(lib().rlu_workspace_size(ctypes.byref(pb), ctypes.byref(out)), "rlu_workspace_size")
    return out.value


@dataclass
class Factors:
    L: "object"
    U: "object"
    p: "object"
    q: "object"
    info: "object"
    Y: "object" = None
    B: "object" = None
    ipiv: "object" = None
    qpiv: "object" = None
    qy: "object" = None


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _prepare(A, k, l, precision, seed, G, diagnostics, out, power_iters=0):
    """ctypes problem and buffer structs for one factorization (allocating
    the outputs that `out` does not provide)."""
    import torch

    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor")
    m, n = A.shape
    if A.stride(0) != 1:
        raise ValueError("A must be column-major (stride(0) == 1)")
    lda = max(A.stride(1), m) if n > 1 else m
    if A.dtype == torch.float64:
        dtype = F64
        prec = PREC_FP64 if precision is None else precision
    elif A.dtype == torch.float32:
        dtype = F32
        prec = PREC_FP32 if precision is None else precision
    else:
        raise ValueError("A must be float64 or float32")
    dev = A.device
    if out is None:
        L = torch.empty((k, m), dtype=A.dtype, device=dev).t()
        U = torch.empty((n, k), dtype=A.dtype, device=dev).t()
        p = torch.empty(m, dtype=torch.int64, device=dev)
        q = torch.empty(n, dtype=torch.int64, device=dev)
        info = torch.empty(3, dtype=torch.int32, device=dev)
        out = Factors(L, U, p, q, info)
        if diagnostics:
            ytype = torch.float32 if prec == PREC_FP32 else torch.float64
            out.Y = torch.empty((l, m), dtype=ytype, device=dev).t()
            out.B = torch.empty((n, k), dtype=ytype, device=dev).t()
            out.ipiv = torch.empty(l, dtype=torch.int32, device=dev)
            out.qpiv = torch.empty(k, dtype=torch.int32, device=dev)
            out.qy = torch.empty(l, dtype=torch.int32, device=dev)
    pb = Problem(m, n, k, l, dtype, prec, seed, None, 0, FLAG_DIAGNOSTICS if diagnostics else 0,
                 power_iters)
    if G is not None:
        if G.shape != (n, l) or G.stride(0) != 1 or G.dtype != A.dtype:
            raise ValueError("G must be an n x l column-major tensor of A's dtype")
        pb.G = G.data_ptr()
        pb.ldg = max(G.stride(1), n) if l > 1 else n
    io = Buffers(A.data_ptr(), lda,
                 out.L.data_ptr(), max(out.L.stride(1), m) if k > 1 else m,
                 out.U.data_ptr(), max(out.U.stride(1), k) if n > 1 else k,
                 out.p.data_ptr(), out.q.data_ptr(), out.info.data_ptr(),
                 out.Y.data_ptr() if out.Y is not None else None,
                 (max(out.Y.stride(1), m) if l > 1 else m) if out.Y is not None else 0,
                 out.B.data_ptr() if out.B is not None else None,
                 (max(out.B.stride(1), k) if n > 1 else k) if out.B is not None else 0,
                 out.ipiv.data_ptr() if out.ipiv is not None else None,
                 out.qpiv.data_ptr() if out.qpiv is not None else None,
                 out.qy.data_ptr() if out.qy is not None else None)
    return pb, io, out


def factor(A, k: int, l: int, *, precision: int | None = None, seed: int = 0, G=None,
           diagnostics: bool = False, handle: Handle | None = None, stream=None,
           out: Factors | None = None, power_iters: int = 0,
           check_finite: bool = False, rrlu: bool = False, fast: bool = False) -> Factors:
    """Randomized LU of the device matrix A (torch tensor, m x n, float64 or
    float32, column-major: pass ``X.t()`` of a contiguous n x m tensor, or any
    tensor with stride (1, lda)).  Returns device tensors L (m x k), U (k x n),
    p, q (int64) and info (int32[3]); the work is enqueued on ``stream`` (the
    current torch stream by default) and not synchronized.  ``power_iters``
    is q of the power scheme, Y = (A A^T)^q A G (Section 5.2).
    ``check_finite`` asks for the scan for NaN / infinity (info[2] bit 1);
    ``rrlu`` for the rank-revealing Step 3 as Algorithm 4.1 lists it (the
    sketch columns in column-pivoted QR order before partial pivoting);
    ``fast`` for Algorithm 4.4 (SRFT sketch drawn from ``seed`` and the
    interpolative decomposition; G must be None)."""
    import torch

    pb, io, out = _prepare(A, k, l, precision, seed, G, diagnostics, out, power_iters)
    if check_finite:
        pb.flags |= FLAG_CHECK_FINITE
    if rrlu:
        pb.flags |= FLAG_RRLU
    if fast:
        pb.flags |= FLAG_FAST
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    h = handle or default_handle(A.device.index or 0, s)
    st = lib().rlu_factor(h.ptr, ctypes.byref(pb), ctypes.byref(io),
                          ctypes.c_void_p(s.cuda_stream))
    _check(st, "rlu_factor")
    return out


def _ld(t, rows):
    return max(t.stride(1), rows) if t.dim() == 2 and t.shape[1] > 1 else rows


def lstsq(f: Factors, b, *, handle: Handle | None = None, stream=None, x=None):
    """Rank-deficient least squares on the factors of ``factor`` (Section
    4.4, Algorithm 4.3): x = Q (U_1^{-1} L^+ P b; 0) minimizes ||A x - b||.
    ``b`` is an m-vector or an m x r column-major device tensor of the
    factors' dtype; returns x (n, or n x r) on the same stream, not
    synchronized."""
    import torch

    L, U = f.L, f.U
    m, k = L.shape
    n = U.shape[1]
    if not b.is_cuda or b.dtype != L.dtype or b.shape[0] != m:
        raise ValueError("b must be a device tensor of L's dtype with m rows")
    vec = b.dim() == 1
    B = b.view(m, 1) if vec else b
    if B.stride(0) != 1:
        raise ValueError("b must be column-major (stride(0) == 1)")
    r = B.shape[1]
    if x is None:
        x = torch.empty((r, n), dtype=L.dtype, device=L.device).t()
    X = x.view(n, 1) if x.dim() == 1 else x
    if X.stride(0) != 1 or X.shape != (n, r):
        raise ValueError("x must be an n x r column-major tensor")
    d = LstsqDesc(m, n, k, F64 if L.dtype == torch.float64 else F32,
                  L.data_ptr(), _ld(L, m), U.data_ptr(), _ld(U, k),
                  f.p.data_ptr(), f.q.data_ptr(), r,
                  B.data_ptr(), _ld(B, m), X.data_ptr(), _ld(X, n))
    s = stream if stream is not None else torch.cuda.current_stream(L.device)
    h = handle or default_handle(L.device.index or 0, s)
    _check(lib().rlu_lstsq(h.ptr, ctypes.byref(d), ctypes.c_void_p(s.cuda_stream)), "rlu_lstsq")
    return x[:, 0] if vec and x.dim() == 2 else x


class Batch:
    """A prepared batch for rlu_factor_batched: the problem and buffer
    arrays stay alive (and unchanged) so that repeated calls replay the
    library's recorded launch graph."""

    def __init__(self, problems, *, precision: int | None = None, outs=None,
                 power_iters: int = 0, check_finite: bool = False):
        """problems: sequence of (A, k, l) or (A, k, l, seed) or
        (A, k, l, seed, G) with A a column-major device tensor; power_iters
        (Section 5.2) and check_finite apply to every problem."""
        items = [tuple(p) + (0, None)[len(p) - 3:] if len(p) < 5 else tuple(p) for p in problems]
        self.count = len(items)
        self.pbs = (Problem * max(1, self.count))()
        self.ios = (Buffers * max(1, self.count))()
        self.outs = []
        self.inputs = []
        for i, (A, k, l, seed, G) in enumerate(items):
            o = outs[i] if outs is not None else None
            pb, io, o = _prepare(A, k, l, precision, seed, G, False, o, power_iters)
            if check_finite:
                pb.flags |= FLAG_CHECK_FINITE
            self.pbs[i] = pb
            self.ios[i] = io
            self.outs.append(o)
            self.inputs.append((A, G))
        self.device = items[0][0].device if items else None

    def run(self, handle: Handle | None = None, stream=None):
        import torch

        if self.count == 0:
            return self.outs
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = handle or default_handle(self.device.index or 0, s)
        st = lib().rlu_factor_batched(h.ptr, self.count, self.pbs, self.ios,
                                      ctypes.c_void_p(s.cuda_stream))
        _check(st, "rlu_factor_batched")
        return self.outs


def factor_batched(problems, *, precision: int | None = None, handle: Handle | None = None,
                   stream=None, outs=None, power_iters: int = 0,
                   check_finite: bool = False) -> list:
    """Algorithm 4.1 for every (A, k, l[, seed[, G]]) in `problems`, as one
    batched call (with q = power_iters power iterations, Section 5.2, for
    all of them).  Returns a list of Factors (device tensors, not
    synchronized)."""
    return Batch(problems, precision=precision, outs=outs, power_iters=power_iters,
                 check_finite=check_finite).run(handle, stream)


def tile_names() -> dict:
    """{cfg: "BMxBNxBK"} of the tiles the grouped products can use."""
    out = {}
    for c in range(64):
        n = lib().rlu_tile_name(c)
        if n:
            out[c] = n.decode()
    return out


def serve_footprint(m, n, k, l, dtype=F64, precision=PREC_FP64) -> int:
    """HBM bytes the server charges for a request of this shape."""
    pb = Problem(m, n, k, l, dtype, precision, 0, None, 0, 0)
    out = ctypes.c_size_t()
    _check(lib().rlu_serve_footprint(ctypes.byref(pb), ctypes.byref(out)), "rlu_serve_footprint")
    return out.value


class Server:
    """Continuous-batching request loop of the library (rlu_serve_*).  Keeps a
    reference to each request's A (and G) until the ticket is released."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, max_inflight: int = 0,
                 max_queue: int = 0):
        cfg = ServerConfig(device, budget_bytes, max_inflight, max_queue)
        self._s = ctypes.c_void_p()
        _check(lib().rlu_serve_create(ctypes.byref(cfg), ctypes.byref(self._s)),
               "rlu_serve_create")
        self.device = device
        self._keep = {}

    def submit(self, A, k: int, l: int, *, seed: int = 0, precision: int | None = None,
               G=None, power_iters: int = 0, check_finite: bool = False) -> int:
        """Queue A (column-major device tensor); returns the ticket.  Raises
        RluError on rejection (e.g. RLU_ERR_TOO_LARGE, RLU_ERR_QUEUE_FULL).
        A request with power iterations (Section 5.2) runs alone."""
        import torch

        if A.dim() != 2 or not A.is_cuda or A.stride(0) != 1:
            raise ValueError("A must be a column-major 2-D device tensor")
        m, n = A.shape
        lda = max(A.stride(1), m) if n > 1 else m
        if A.dtype == torch.float64:
            dtype, prec = F64, (PREC_FP64 if precision is None else precision)
        elif A.dtype == torch.float32:
            dtype, prec = F32, (PREC_FP32 if precision is None else precision)
        else:
            raise ValueError("A must be float64 or float32")
        pb = Problem(m, n, k, l, dtype, prec, seed, None, 0,
                     FLAG_CHECK_FINITE if check_finite else 0, power_iters)
        if G is not None:
            pb.G = G.data_ptr()
            pb.ldg = max(G.stride(1), n) if l > 1 else n
        t = ctypes.c_uint64()
        _check(lib().rlu_serve_submit(self._s, ctypes.byref(pb), ctypes.c_void_p(A.data_ptr()),
                                      lda, ctypes.byref(t)), "rlu_serve_submit")
        self._keep[t.value] = (A, G, m, n, k, A.dtype)
        return t.value

    def poll(self, ticket: int):
        r = Result()
        st = lib().rlu_serve_poll(self._s, ticket, ctypes.byref(r))
        return st, r

    def wait(self, ticket: int, timeout: float = 120.0) -> int:
        import time
        t0 = time.perf_counter()
        while True:
            st, _ = self.poll(ticket)
            if st != 1:  # RLU_PENDING
                return st
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} still pending after {timeout} s")
            time.sleep(50e-6)

    def result(self, ticket: int, stream=None) -> Factors:
        """Copy a finished request's factors into new device tensors."""
        import torch

        A, G, m, n, k, dt = self._keep[ticket]
        dev = A.device
        L = torch.empty((k, m), dtype=dt, device=dev).t()
        U = torch.empty((n, k), dtype=dt, device=dev).t()
        p = torch.empty(m, dtype=torch.int64, device=dev)
        q = torch.empty(n, dtype=torch.int64, device=dev)
        info = torch.empty(3, dtype=torch.int32, device=dev)
        io = Buffers(None, 0, L.data_ptr(), m, U.data_ptr(), k, p.data_ptr(), q.data_ptr(),
                     info.data_ptr(), None, 0, None, 0, None, None)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        _check(lib().rlu_serve_copy(self._s, ticket, ctypes.byref(io),
                                    ctypes.c_void_p(s.cuda_stream)), "rlu_serve_copy")
        s.synchronize()
        return Factors(L, U, p, q, info)

    def release(self, ticket: int) -> int:
        st = lib().rlu_serve_release(self._s, ticket)
        if st == 0:
            self._keep.pop(ticket, None)
        return st

    def stats(self):
        used = ctypes.c_size_t()
        qd = ctypes.c_int32()
        fl = ctypes.c_int32()
        _check(lib().rlu_serve_stats(self._s, ctypes.byref(used), ctypes.byref(qd),
                                     ctypes.byref(fl)), "rlu_serve_stats")
        return used.value, qd.value, fl.value

    def close(self):
        if self._s:
            lib().rlu_serve_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_info(info) -> int:
    """Status for the three info words (host ints or a tensor)."""
    vals = [int(x) for x in (info.tolist() if hasattr(info, "tolist") else info)]
    arr = (ctypes.c_int32 * 3)(*vals)
    return lib().rlu_check_info(arr)
