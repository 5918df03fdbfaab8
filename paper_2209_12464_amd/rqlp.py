"""ctypes binding of librqlp.so (include/rqlp.h), same names as the C ABI.

Argument marshalling only: torch tensors supply device pointers and the
current HIP stream; every step runs in the library's HIP kernels.  Loading
fails loudly when the library is missing -- there is no fallback path.
"""

import atexit
import ctypes
import os
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librqlp.so")

RQLP_OK = 0
RQLP_FP64, RQLP_FP32, RQLP_BF16_REFINED = 0, 1, 2
KT_GEMM_NN, KT_GEMM_TN, KT_SPMM, KT_GRAM, KT_CHOL, KT_APPLY = range(6)
KERNEL_CLASSES = {"gemm_nn": KT_GEMM_NN, "gemm_tn": KT_GEMM_TN, "spmm": KT_SPMM,
                  "gram": KT_GRAM, "chol": KT_CHOL, "apply": KT_APPLY}


class RqlpError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib().rqlp_status_string(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("completed_cols", ctypes.c_int32),
                ("breakdown_pass", ctypes.c_int32), ("nonfinite", ctypes.c_int32)]


class Problem(ctypes.Structure):
    """rqlp_problem: one decomposition of a batch."""
    _fields_ = [("A", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("k", ctypes.c_int), ("p", ctypes.c_int), ("q", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("Q", ctypes.c_void_p), ("L", ctypes.c_void_p), ("V", ctypes.c_void_p)]


_LIB = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_INT = ctypes.c_int
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2209_12464_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        sig = {
            "rqlp_create": (_INT, [ctypes.POINTER(_P), _INT]),
            "rqlp_destroy": (_INT, [_P]),
            "rqlp_workspace_size": (_SZ, [_I64, _I64, _INT, _INT, _INT, _INT]),
            "rqlp_workspace_size_csr": (_SZ, [_I64, _I64, _I64, _INT, _INT, _INT, _INT]),
            "rqlp_decompose": (_INT, [_P, _P, _I64, _I64, _I64, _INT, _INT, _INT, _INT, _U64,
                                      _P, _P, _P, _P, _SZ, _P]),
            "rqlp_decompose_noalloc": (_INT, [_P, _P, _I64, _I64, _I64, _INT, _INT, _INT, _INT, _U64,
                                              _P, _P, _P, _P]),
            "rqlp_decompose_csr": (_INT, [_P, _P, _P, _P, _I64, _I64, _I64, _INT, _INT, _INT, _INT,
                                          _U64, _P, _P, _P, _P, _SZ, _P]),
            "rqlp_get_info": (_INT, [_P, ctypes.POINTER(Info)]),
            "rqlp_status_string": (ctypes.c_char_p, [_INT]),
            "rqlp_gaussian": (_INT, [_P, _U64, ctypes.c_uint32, _I64, _I64, _INT, _P, _I64, _P]),
            "rqlp_gemm_workspace_size": (_SZ, [_INT, _I64, _I64, _INT, _INT]),
            "rqlp_gemm": (_INT, [_P, _INT, _P, _I64, _I64, _I64, _P, _I64, _INT, _P, _I64, _INT,
                                 _P, _SZ, _P]),
            "rqlp_orth_workspace_size": (_SZ, [_I64, _INT, _INT]),
            "rqlp_orth": (_INT, [_P, _P, _I64, _INT, _I64, _P, _I64, _P, _INT, _U64, _P, _SZ, _P]),
            "rqlp_spmm": (_INT, [_P, _P, _P, _P, _I64, _I64, _I64, _P, _I64, _INT, _P, _I64, _INT, _P]),
            "rqlp_csr_transpose_workspace_size": (_SZ, [_I64, _I64, _I64]),
            "rqlp_csr_transpose": (_INT, [_P, _P, _P, _P, _I64, _I64, _I64, _INT, _P, _P, _P, _P,
                                          _SZ, _P]),
            "rqlp_workspace_size_batched": (_SZ, [_INT, ctypes.POINTER(Problem), _INT]),
            "rqlp_decompose_batched": (_INT, [_P, _INT, ctypes.POINTER(Problem), _INT, _P, _SZ, _P]),
            "rqlp_set_graphs": (_INT, [_P, _INT]),
            "rqlp_set_batch_grouping": (_INT, [_P, _INT]),
            "rqlp_autotune": (_INT, [_P, _P, _I64, _I64, _I64, _INT, _INT, _P, ctypes.POINTER(_INT),
                                     ctypes.POINTER(_INT)]),
            "rqlp_autotune_clear": (_INT, [_P]),
            "rqlp_autotune_count": (_INT, [_P, ctypes.POINTER(_INT)]),
            "rqlp_autotune_save": (_INT, [_P, ctypes.c_char_p]),
            "rqlp_autotune_load": (_INT, [_P, ctypes.c_char_p]),
            "rqlp_svd_workspace_size": (_SZ, [_INT]),
            "rqlp_svd_small": (_INT, [_P, _P, _INT, _I64, _P, _I64, _P, _P, _I64, _INT, _P, _SZ, _P]),
            "rqlp_workspace_size_svd": (_SZ, [_I64, _I64, _INT, _INT, _INT, _INT]),
            "rqlp_decompose_svd": (_INT, [_P, _P, _I64, _I64, _I64, _INT, _INT, _INT, _INT, _U64,
                                          _P, _P, _P, _P, _SZ, _P]),
            "rqlp_workspace_size_paper": (_SZ, [_I64, _I64, _INT, _INT, _INT, _INT]),
            "rqlp_decompose_paper": (_INT, [_P, _P, _I64, _I64, _I64, _INT, _INT, _INT, _INT, _U64,
                                            _P, _P, _P, _P, _SZ, _P]),
            "rqlp_server_create": (_INT, [ctypes.POINTER(_P), _P, _SZ, _INT, _INT]),
            "rqlp_server_destroy": (_INT, [_P]),
            "rqlp_server_request_bytes": (_SZ, [ctypes.POINTER(Problem), _INT]),
            "rqlp_server_set_tick": (_INT, [_P, _INT]),
            "rqlp_server_submit": (_INT, [_P, ctypes.POINTER(Problem), _P, ctypes.POINTER(_I64)]),
            "rqlp_server_poll": (_INT, [_P, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_int32), _INT,
                                        ctypes.POINTER(_INT), ctypes.POINTER(_INT), ctypes.POINTER(_INT)]),
            "rqlp_set_timing": (_INT, [_P, _INT]),
            "rqlp_set_timing_mask": (_INT, [_P, ctypes.c_uint32]),
            "rqlp_get_timing": (_INT, [_P, _INT, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(_I64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def exported_symbols():
    """Names of the C ABI functions this binding expects."""
    return ["rqlp_create", "rqlp_destroy", "rqlp_workspace_size", "rqlp_workspace_size_csr",
            "rqlp_decompose", "rqlp_decompose_noalloc", "rqlp_decompose_csr", "rqlp_get_info", "rqlp_status_string",
            "rqlp_gaussian", "rqlp_gemm_workspace_size", "rqlp_gemm", "rqlp_orth_workspace_size",
            "rqlp_orth", "rqlp_spmm", "rqlp_csr_transpose_workspace_size", "rqlp_csr_transpose",
            "rqlp_set_timing", "rqlp_set_timing_mask", "rqlp_get_timing",
            "rqlp_workspace_size_batched", "rqlp_decompose_batched", "rqlp_set_graphs",
            "rqlp_set_batch_grouping", "rqlp_svd_workspace_size", "rqlp_svd_small",
            "rqlp_autotune", "rqlp_autotune_clear", "rqlp_autotune_count", "rqlp_autotune_save",
            "rqlp_autotune_load",
            "rqlp_workspace_size_svd", "rqlp_decompose_svd",
            "rqlp_server_create", "rqlp_server_destroy", "rqlp_server_request_bytes", "rqlp_server_set_tick",
            "rqlp_server_submit",
            "rqlp_server_poll", "rqlp_workspace_size_paper", "rqlp_decompose_paper"]


def _check(status, where):
    if status != RQLP_OK:
        raise RqlpError(status, where)


def _prec(dtype, bf16=False):
    if bf16:
        if dtype != torch.float32:
            raise TypeError("bfloat16 products take a float32 A")
        return RQLP_BF16_REFINED
    if dtype == torch.float64:
        return RQLP_FP64
    if dtype == torch.float32:
        return RQLP_FP32
    raise TypeError(f"unsupported dtype {dtype}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# Every live Context and Server, so that they can be destroyed at
# interpreter exit while the HIP runtime is still up (not from __del__
# during module teardown, when the runtime may already be gone).
_LIVE = weakref.WeakSet()


@atexit.register
def close_all():
    """Destroy every live server, then every live context."""
    for obj in [o for o in list(_LIVE) if isinstance(o, Server)]:
        obj.close()
    for obj in list(_LIVE):
        obj.close()
    _DEFAULT.clear()


class Context:
    """Owns an rqlp_ctx on one device (and its info record)."""

    def __init__(self, device=0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        _check(_lib().rqlp_create(ctypes.byref(h), self.device.index or 0), "rqlp_create")
        self._h = h
        _LIVE.add(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            _lib().rqlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self):
        out = Info()
        _check(_lib().rqlp_get_info(self._h, ctypes.byref(out)), "rqlp_get_info")
        return dict(status=out.status, completed_cols=out.completed_cols,
                    breakdown_pass=out.breakdown_pass, nonfinite=out.nonfinite)

    def set_graphs(self, enabled):
        """Capture a batch submitted twice in a row into a HIP graph and replay it."""
        _check(_lib().rqlp_set_graphs(self._h, 1 if enabled else 0), "rqlp_set_graphs")

    def autotune(self, A, d):
        """Tune the split-K plans of the products of a decomposition of A
        with d columns; returns (nsplit of A X, nsplit of A^T X)."""
        if A.dim() != 2 or A.stride(1) != 1:
            raise ValueError("A must be a 2-D row-major tensor")
        nn, tn = _INT(0), _INT(0)
        _check(_lib().rqlp_autotune(self._h, _ptr(A), A.shape[0], A.shape[1], A.stride(0), d, _prec(A.dtype),
                                    _stream(A.device), ctypes.byref(nn), ctypes.byref(tn)), "rqlp_autotune")
        return nn.value, tn.value

    def autotune_count(self):
        n = _INT(0)
        _check(_lib().rqlp_autotune_count(self._h, ctypes.byref(n)), "rqlp_autotune_count")
        return n.value

    def autotune_clear(self):
        _check(_lib().rqlp_autotune_clear(self._h), "rqlp_autotune_clear")

    def autotune_save(self, path):
        _check(_lib().rqlp_autotune_save(self._h, str(path).encode()), "rqlp_autotune_save")

    def autotune_load(self, path):
        _check(_lib().rqlp_autotune_load(self._h, str(path).encode()), "rqlp_autotune_load")

    def set_batch_grouping(self, enabled):
        """Grouped launches for batches (on by default; off: one lane stream per problem)."""
        _check(_lib().rqlp_set_batch_grouping(self._h, 1 if enabled else 0), "rqlp_set_batch_grouping")

    def set_timing(self, enabled, classes=None):
        """Event timing of every kernel class, or only of `classes` (names
        from KERNEL_CLASSES)."""
        if classes is None:
            _check(_lib().rqlp_set_timing(self._h, 1 if enabled else 0), "rqlp_set_timing")
            return
        mask = 0
        if enabled:
            for name in classes:
                mask |= 1 << KERNEL_CLASSES[name]
        _check(_lib().rqlp_set_timing_mask(self._h, mask), "rqlp_set_timing_mask")

    def timing(self, cls):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(_lib().rqlp_get_timing(self._h, KERNEL_CLASSES.get(cls, cls), ctypes.byref(ms),
                                      ctypes.byref(n)), "rqlp_get_timing")
        return ms.value, n.value


_DEFAULT = {}


def default_context(device=0):
    if device not in _DEFAULT:
        _DEFAULT[device] = Context(device)
    return _DEFAULT[device]


def workspace_size(m, n, k, p, q, dtype, bf16=False):
    return int(_lib().rqlp_workspace_size(m, n, k, p, q, _prec(dtype, bf16)))


def workspace_size_csr(m, n, nnz, k, p, q, dtype):
    return int(_lib().rqlp_workspace_size_csr(m, n, nnz, k, p, q, _prec(dtype)))


def alloc_workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def decompose(A, k, p, q=0, seed=0, ctx=None, workspace=None, out=None, bf16=False):
    """RU-QLP of a dense device matrix A (m x n, float32 or float64, row
    stride >= n).  Returns (Q, L, V) on A's device; enqueued on the current
    stream (not synchronized).  bf16=True (float32 A) takes the products
    with A in bfloat16 with float32 accumulation (RQLP_BF16_REFINED)."""
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor")
    ctx = ctx or default_context(A.device.index or 0)
    m, n = A.shape
    d = k + p
    prec = _prec(A.dtype, bf16)
    if out is None:
        Q = torch.empty((m, d), dtype=A.dtype, device=A.device)
        L = torch.empty((d, d), dtype=A.dtype, device=A.device)
        V = torch.empty((n, d), dtype=A.dtype, device=A.device)
    else:
        Q, L, V = out
    if workspace is None:
        ws_bytes = workspace_size(m, n, k, p, q, A.dtype, bf16)
        workspace = alloc_workspace(ws_bytes, A.device) if ws_bytes else None
    ws_ptr = _ptr(workspace)
    ws_bytes = workspace.numel() if workspace is not None else 0
    _check(_lib().rqlp_decompose(ctx.handle, _ptr(A), m, n, A.stride(0), k, p, q, prec, seed,
                                 _ptr(Q), _ptr(L), _ptr(V), ws_ptr, ws_bytes, _stream(A.device)),
           "rqlp_decompose")
    return Q, L, V


NOALLOC_SCRATCH_BYTES = 256 << 20  # RQLP_NOALLOC_SCRATCH_BYTES


def decompose_noalloc(A, k, p, q=0, seed=0, ctx=None, out=None, bf16=False):
    """rqlp_decompose_noalloc: decompose() with the library's fixed scratch
    array as workspace (no device allocation by the library; pass `out` to
    avoid torch's allocations too)."""
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor")
    ctx = ctx or default_context(A.device.index or 0)
    m, n = A.shape
    d = k + p
    if out is None:
        out = (torch.empty((m, d), dtype=A.dtype, device=A.device), torch.empty((d, d), dtype=A.dtype, device=A.device),
               torch.empty((n, d), dtype=A.dtype, device=A.device))
    Q, L, V = out
    _check(_lib().rqlp_decompose_noalloc(ctx.handle, _ptr(A), m, n, A.stride(0), k, p, q, _prec(A.dtype, bf16), seed,
                                         _ptr(Q), _ptr(L), _ptr(V), _stream(A.device)), "rqlp_decompose_noalloc")
    return Q, L, V


def decompose_paper(A, k, p, q=0, seed=0, ctx=None, workspace=None, out=None):
    """RU-QLP in the paper's row-sketch orientation (Algorithm 1 as printed):
    returns (Q, L, P) with A ~ Q L P^T; float32 or float64 dense A."""
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor")
    ctx = ctx or default_context(A.device.index or 0)
    m, n = A.shape
    d = k + p
    prec = _prec(A.dtype)
    if out is None:
        Q = torch.empty((m, d), dtype=A.dtype, device=A.device)
        L = torch.empty((d, d), dtype=A.dtype, device=A.device)
        P = torch.empty((n, d), dtype=A.dtype, device=A.device)
    else:
        Q, L, P = out
    if workspace is None:
        ws_bytes = int(_lib().rqlp_workspace_size_paper(m, n, k, p, q, prec))
        workspace = alloc_workspace(ws_bytes, A.device) if ws_bytes else None
    ws_bytes = workspace.numel() if workspace is not None else 0
    _check(_lib().rqlp_decompose_paper(ctx.handle, _ptr(A), m, n, A.stride(0), k, p, q, prec, seed, _ptr(Q),
                                       _ptr(L), _ptr(P), _ptr(workspace), ws_bytes, _stream(A.device)),
           "rqlp_decompose_paper")
    return Q, L, P


def svd_small(M, ctx=None, workspace=None, out=None):
    """SVD of a small square device matrix (float32 or float64, d <= 544):
    returns (U, S, V) with M = U diag(S) V^T (rqlp_svd_small's conventions)."""
    if M.dim() != 2 or M.shape[0] != M.shape[1] or M.stride(1) != 1:
        raise ValueError("M must be a square row-major matrix")
    ctx = ctx or default_context(M.device.index or 0)
    d = M.shape[0]
    if out is None:
        U = torch.empty((d, d), dtype=M.dtype, device=M.device)
        S = torch.empty((d,), dtype=M.dtype, device=M.device)
        V = torch.empty((d, d), dtype=M.dtype, device=M.device)
    else:
        U, S, V = out
    if workspace is None:
        ws_bytes = int(_lib().rqlp_svd_workspace_size(d))
        workspace = alloc_workspace(ws_bytes, M.device) if ws_bytes else None
    ws_bytes = workspace.numel() if workspace is not None else 0
    _check(_lib().rqlp_svd_small(ctx.handle, _ptr(M), d, M.stride(0), _ptr(U), U.stride(0), _ptr(S), _ptr(V),
                                 V.stride(0), _prec(M.dtype), _ptr(workspace), ws_bytes, _stream(M.device)),
           "rqlp_svd_small")
    return U, S, V


def workspace_size_svd(m, n, k, p, q, dtype, bf16=False):
    return int(_lib().rqlp_workspace_size_svd(m, n, k, p, q, _prec(dtype, bf16)))


def decompose_svd(A, k, p, q=0, seed=0, ctx=None, workspace=None, out=None, bf16=False):
    """RU-QLP in its SVD-like form (Remark 1): returns (U, S, W) with
    A ~ U diag(S) W^T."""
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor")
    ctx = ctx or default_context(A.device.index or 0)
    m, n = A.shape
    d = k + p
    prec = _prec(A.dtype, bf16)
    if out is None:
        U = torch.empty((m, d), dtype=A.dtype, device=A.device)
        S = torch.empty((d,), dtype=A.dtype, device=A.device)
        W = torch.empty((n, d), dtype=A.dtype, device=A.device)
    else:
        U, S, W = out
    if workspace is None:
        ws_bytes = int(_lib().rqlp_workspace_size_svd(m, n, k, p, q, prec))
        workspace = alloc_workspace(ws_bytes, A.device) if ws_bytes else None
    ws_bytes = workspace.numel() if workspace is not None else 0
    _check(_lib().rqlp_decompose_svd(ctx.handle, _ptr(A), m, n, A.stride(0), k, p, q, prec, seed, _ptr(U), _ptr(S),
                                     _ptr(W), _ptr(workspace), ws_bytes, _stream(A.device)), "rqlp_decompose_svd")
    return U, S, W


def _problems(As, params, outs):
    arr = (Problem * len(As))()
    for i, (A, (k, p, q, seed), (Q, L, V)) in enumerate(zip(As, params, outs)):
        if A.dim() != 2 or A.stride(1) != 1:
            raise ValueError("every A must be a 2-D row-major tensor")
        arr[i] = Problem(_ptr(A), A.shape[0], A.shape[1], A.stride(0), k, p, q, seed, _ptr(Q), _ptr(L), _ptr(V))
    return arr


def workspace_size_batched(shapes, dtype, bf16=False):
    """Workspace bytes for problems given as (m, n, k, p, q) tuples."""
    arr = (Problem * len(shapes))()
    for i, (m, n, k, p, q) in enumerate(shapes):
        arr[i] = Problem(1, m, n, n, k, p, q, 0, 1, 1, 1)
    return int(_lib().rqlp_workspace_size_batched(len(shapes), arr, _prec(dtype, bf16)))


def decompose_batched(As, params, ctx=None, workspace=None, outs=None, bf16=False):
    """Batched RU-QLP: As is a list of dense device matrices (one dtype),
    params a list of (k, p, q, seed).  Returns a list of (Q, L, V), each
    bitwise what decompose() gives for that problem; enqueued on the
    current stream."""
    if not As:
        return []
    dev = As[0].device
    ctx = ctx or default_context(dev.index or 0)
    dtype = As[0].dtype
    if outs is None:
        outs = []
        for A, (k, p, q, seed) in zip(As, params):
            m, n = A.shape
            d = k + p
            outs.append((torch.empty((m, d), dtype=dtype, device=dev), torch.empty((d, d), dtype=dtype, device=dev),
                         torch.empty((n, d), dtype=dtype, device=dev)))
    arr = _problems(As, params, outs)
    if workspace is None:
        ws_bytes = int(_lib().rqlp_workspace_size_batched(len(As), arr, _prec(dtype, bf16)))
        workspace = alloc_workspace(ws_bytes, dev) if ws_bytes else None
    ws_bytes = workspace.numel() if workspace is not None else 0
    _check(_lib().rqlp_decompose_batched(ctx.handle, len(As), arr, _prec(dtype, bf16), _ptr(workspace), ws_bytes,
                                         _stream(dev)), "rqlp_decompose_batched")
    return outs


def server_request_bytes(m, n, k, p, q, dtype=torch.float32, bf16=False):
    """Workspace bytes a request takes from a server's HBM budget."""
    pr = Problem(1, m, n, n, k, p, q, 0, 1, 1, 1)
    return int(_lib().rqlp_server_request_bytes(ctypes.byref(pr), _prec(dtype, bf16)))


class Server:
    """Continuous-batching request server (rqlp_server_*): an HBM budget for
    the requests' workspaces, `slots` concurrent requests.  submit() queues a
    request (device tensors stay owned and kept alive by the caller until
    poll() reports its ticket); poll() returns finished tickets and admits
    queued requests."""

    def __init__(self, budget_bytes, slots=8, dtype=torch.float32, bf16=False, ctx=None, device=0, max_tick=None):
        self.ctx = ctx or default_context(device)
        self._prec = _prec(dtype, bf16)
        h = ctypes.c_void_p()
        _check(_lib().rqlp_server_create(ctypes.byref(h), self.ctx.handle, int(budget_bytes), int(slots),
                                         self._prec), "rqlp_server_create")
        self._h = h
        if max_tick is not None:
            _check(_lib().rqlp_server_set_tick(self._h, int(max_tick)), "rqlp_server_set_tick")
        self._done = (ctypes.c_int64 * 2048)()
        self._status = (ctypes.c_int32 * 2048)()
        self.failed = {}  # ticket -> status of requests whose launch failed
        _LIVE.add(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            _lib().rqlp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, A, k, p, q, seed, out):
        """Queue a request; its launches wait for the work enqueued so far on
        the current stream of A's device."""
        Q, L, V = out
        pr = Problem(_ptr(A), A.shape[0], A.shape[1], A.stride(0), k, p, q, seed, _ptr(Q), _ptr(L), _ptr(V))
        t = ctypes.c_int64()
        _check(_lib().rqlp_server_submit(self._h, ctypes.byref(pr), _stream(A.device), ctypes.byref(t)),
               "rqlp_server_submit")
        return t.value

    def poll(self):
        """(finished tickets, in flight, queued).  Tickets whose launch failed
        are reported too and recorded in self.failed (ticket -> status)."""
        nd, inf, qd = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib().rqlp_server_poll(self._h, self._done, self._status, len(self._done), ctypes.byref(nd),
                                       ctypes.byref(inf), ctypes.byref(qd)), "rqlp_server_poll")
        out = []
        for i in range(nd.value):
            out.append(self._done[i])
            if self._status[i] != RQLP_OK:
                self.failed[self._done[i]] = self._status[i]
        return out, inf.value, qd.value


def decompose_csr(rowptr, colidx, vals, m, n, k, p, q=0, seed=0, ctx=None, workspace=None, out=None):
    """RU-QLP of a CSR device matrix (int32 rowptr/colidx, float vals)."""
    dev = vals.device
    ctx = ctx or default_context(dev.index or 0)
    d = k + p
    nnz = colidx.numel()
    prec = _prec(vals.dtype)
    if out is None:
        Q = torch.empty((m, d), dtype=vals.dtype, device=dev)
        L = torch.empty((d, d), dtype=vals.dtype, device=dev)
        V = torch.empty((n, d), dtype=vals.dtype, device=dev)
    else:
        Q, L, V = out
    if workspace is None:
        ws_bytes = workspace_size_csr(m, n, nnz, k, p, q, vals.dtype)
        workspace = alloc_workspace(ws_bytes, dev) if ws_bytes else None
    ws_bytes = workspace.numel() if workspace is not None else 0
    _check(_lib().rqlp_decompose_csr(ctx.handle, _ptr(rowptr), _ptr(colidx), _ptr(vals), m, n, nnz, k, p,
                                     q, prec, seed, _ptr(Q), _ptr(L), _ptr(V), _ptr(workspace), ws_bytes,
                                     _stream(dev)), "rqlp_decompose_csr")
    return Q, L, V


def gaussian(rows, cols, seed, dtype=torch.float64, stream_id=0, ld=None, device="cuda", ctx=None):
    ld = ld or cols
    dev = torch.device(device)
    ctx = ctx or default_context(dev.index or 0)
    out = torch.empty((rows, ld), dtype=dtype, device=dev)
    _check(_lib().rqlp_gaussian(ctx.handle, seed, stream_id, rows, cols, _prec(dtype), _ptr(out), ld,
                                _stream(dev)), "rqlp_gaussian")
    return out


def gemm(A, X, trans=False, ctx=None, bf16=False):
    """Y = A X (trans=False) or A^T X (trans=True) on the matrix cores;
    bf16=True (float32 A, X) rounds both to bfloat16 and accumulates in
    float32."""
    ctx = ctx or default_context(A.device.index or 0)
    m, n = A.shape
    d = X.shape[1]
    rows_out = n if trans else m
    prec = _prec(A.dtype, bf16)
    Y = torch.empty((rows_out, d), dtype=A.dtype, device=A.device)
    ws = alloc_workspace(_lib().rqlp_gemm_workspace_size(int(trans), m, n, d, prec), A.device)
    _check(_lib().rqlp_gemm(ctx.handle, int(trans), _ptr(A), m, n, A.stride(0), _ptr(X), X.stride(0), d,
                            _ptr(Y), Y.stride(0), prec, _ptr(ws), ws.numel(), _stream(A.device)),
           "rqlp_gemm")
    return Y


def orth(Y, seed=0, want_r=False, ctx=None):
    """Unpivoted QR Y = Q R (diag(R) >= 0) by CholeskyQR2; returns Q or (Q, R)."""
    ctx = ctx or default_context(Y.device.index or 0)
    rows, d = Y.shape
    Q = torch.empty((rows, d), dtype=Y.dtype, device=Y.device)
    R = torch.empty((d, d), dtype=Y.dtype, device=Y.device) if want_r else None
    ws = alloc_workspace(_lib().rqlp_orth_workspace_size(rows, d, _prec(Y.dtype)), Y.device)
    _check(_lib().rqlp_orth(ctx.handle, _ptr(Y), rows, d, Y.stride(0), _ptr(Q), Q.stride(0), _ptr(R),
                            _prec(Y.dtype), seed, _ptr(ws), ws.numel(), _stream(Y.device)), "rqlp_orth")
    return (Q, R) if want_r else Q


def spmm(rowptr, colidx, vals, rows, cols, X, ctx=None):
    ctx = ctx or default_context(X.device.index or 0)
    d = X.shape[1]
    Y = torch.empty((rows, d), dtype=X.dtype, device=X.device)
    _check(_lib().rqlp_spmm(ctx.handle, _ptr(rowptr), _ptr(colidx), _ptr(vals), rows, cols, colidx.numel(),
                            _ptr(X), X.stride(0), d, _ptr(Y), Y.stride(0), _prec(X.dtype),
                            _stream(X.device)), "rqlp_spmm")
    return Y


def csr_transpose(rowptr, colidx, vals, m, n, ctx=None):
    dev = vals.device
    ctx = ctx or default_context(dev.index or 0)
    nnz = colidx.numel()
    rt = torch.empty(n + 1, dtype=torch.int32, device=dev)
    ct = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    vt = torch.empty(max(nnz, 1), dtype=vals.dtype, device=dev)
    ws = alloc_workspace(_lib().rqlp_csr_transpose_workspace_size(m, n, nnz), dev)
    _check(_lib().rqlp_csr_transpose(ctx.handle, _ptr(rowptr), _ptr(colidx), _ptr(vals), m, n, nnz,
                                     _prec(vals.dtype), _ptr(rt), _ptr(ct), _ptr(vt), _ptr(ws), ws.numel(),
                                     _stream(dev)), "rqlp_csr_transpose")
    return rt, ct[:nnz], vt[:nnz]
