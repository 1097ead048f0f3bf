"""Python binding of libmbdp.so: the C-ABI of include/mbdp.h, by the same names.

Argument marshalling only: every step runs in the HIP library.  Tensors are
torch tensors on the current HIP device; their data pointers are passed
through, and the current torch stream is used unless one is given.  A
missing library raises ``MbdpLibraryMissing``; a failing call raises
``MbdpError`` with the library's status and message (a not-converged solve
returns its statistics with ``converged`` False instead).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbdp.so")

MBDP_OK = 0
MBDP_ERR_INVALID_ARG = 1
MBDP_ERR_UNSUPPORTED = 2
MBDP_ERR_WORKSPACE = 3
MBDP_ERR_HIP = 4
MBDP_ERR_NOT_CONVERGED = 5
MBDP_ERR_VALIDATION = 6
MBDP_ERR_DEVICE = 7

# storage types of transition probabilities (mbdp_dtype)
MBDP_F32 = 0
MBDP_BF16 = 1
MBDP_FP8_E4M3 = 2
DTYPES = {"bf16": MBDP_BF16, "fp8": MBDP_FP8_E4M3}

STATUS_NAMES = {
    0: "MBDP_OK", 1: "MBDP_ERR_INVALID_ARG", 2: "MBDP_ERR_UNSUPPORTED",
    3: "MBDP_ERR_WORKSPACE", 4: "MBDP_ERR_HIP", 5: "MBDP_ERR_NOT_CONVERGED",
    6: "MBDP_ERR_VALIDATION", 7: "MBDP_ERR_DEVICE",
}

# Every symbol include/mbdp.h declares.
EXPORTS = [
    "mdp_create_dense", "mdp_create_csr", "mdp_create_dense_q", "mdp_create_csr_q",
    "mdp_quantize_rows", "mdp_policy_transpose", "mdp_value_gradients", "mdp_destroy",
    "mdp_set_tuning", "mdp_batch_workspace_bytes", "mdp_batch_upload", "mdp_batch_launch",
    "mdp_batch_read_stats", "mdp_multi_workspace_bytes", "mdp_multi_solve",
    "mdp_column_blocks_prepare", "mdp_column_blocks_attach",
    "mdp_workspace_bytes", "mdp_engine", "mdp_validate", "mbdp_permutation", "mb_sweep",
    "mbdp_sync_status", "vi_solve", "vi_solve_noalloc", "mpi_solve", "mdp_refine",
    "mbdp_last_error",
]


class MbdpLibraryMissing(RuntimeError):
    pass


class MbdpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("outer_iters", ctypes.c_int64),
                ("policy_changes_last", ctypes.c_int64), ("recentrings", ctypes.c_int64),
                ("final_dv_inf", ctypes.c_double), ("final_err_ref", ctypes.c_double),
                ("converged", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class RefineStats(ctypes.Structure):
    _fields_ = [("residual_in", ctypes.c_double), ("residual_out", ctypes.c_double),
                ("bound_out", ctypes.c_double), ("final_dv_inf", ctypes.c_double),
                ("final_err_ref", ctypes.c_double), ("sweeps", ctypes.c_int64),
                ("outer_iters", ctypes.c_int64), ("converged", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Validation(ctypes.Structure):
    _fields_ = [("bad_probability", ctypes.c_int64), ("bad_row_sum", ctypes.c_int64),
                ("empty_rows", ctypes.c_int64), ("bad_column", ctypes.c_int64),
                ("bad_row_ptr", ctypes.c_int64), ("bad_cost", ctypes.c_int64),
                ("no_admissible_action", ctypes.c_int64), ("max_row_sum_dev", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchItem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("ld", ctypes.c_int64), ("P", ctypes.c_void_p), ("row_scale", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("gamma", ctypes.c_double), ("b", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("V", ctypes.c_void_p), ("policy", ctypes.c_void_p),
                ("lanes", ctypes.c_int32), ("team", ctypes.c_int32)]


class BatchStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("final_dv_inf", ctypes.c_double),
                ("converged", ctypes.c_int32), ("team", ctypes.c_int32),
                ("start_us", ctypes.c_double), ("end_us", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("threads_per_block", ctypes.c_int32),
                ("recentre_every", ctypes.c_int32), ("recentre_force", ctypes.c_int32),
                ("band_window", ctypes.c_int32)]


class MultiStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("final_dv_inf", ctypes.c_double),
                ("recentrings", ctypes.c_int64), ("converged", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_I32 = ctypes.c_int32
_D = ctypes.c_double
_SIGS = {
    "mdp_create_dense": (_I32, [_I64, _I32, _P, _P, _D, ctypes.POINTER(_P)]),
    "mdp_create_csr": (_I32, [_I64, _I32, _P, _P, _P, _I64, _P, _D, _P, ctypes.POINTER(_P)]),
    "mdp_destroy": (_I32, [_P]),
    "mdp_create_dense_q": (_I32, [_I64, _I32, _P, _I32, _P, _P, _D, ctypes.POINTER(_P)]),
    "mdp_create_csr_q": (_I32, [_I64, _I32, _P, _P, _P, _I32, _P, _I64, _P, _D, _P,
                                ctypes.POINTER(_P)]),
    "mdp_quantize_rows": (_I32, [_P, _I64, _I64, _I32, _P, _P, _P]),
    "mdp_policy_transpose": (_I32, [_P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mdp_batch_workspace_bytes": (ctypes.c_size_t, [_I32]),
    "mdp_batch_upload": (_I32, [ctypes.POINTER(BatchItem), _I32, _P, ctypes.c_size_t, _P]),
    "mdp_batch_launch": (_I32, [_I32, _D, _I64, _P, ctypes.c_size_t, _P]),
    "mdp_batch_read_stats": (_I32, [_P, _I32, ctypes.POINTER(BatchStats), _P]),
    "mdp_multi_workspace_bytes": (ctypes.c_size_t, [_P, _I32, _I64]),
    "mdp_multi_solve": (_I32, [_P, _I32, _P, _P, _P, _I64, _U64, _U64, _D, _I64, _P,
                               ctypes.c_size_t, _P, ctypes.POINTER(MultiStats)]),
    "mdp_value_gradients": (_I32, [_P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mdp_set_tuning": (_I32, [_P, ctypes.POINTER(Tuning)]),
    "mdp_column_blocks_prepare": (_I32, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "mdp_column_blocks_attach": (_I32, [_P, _P, ctypes.c_size_t, _P]),
    "mdp_workspace_bytes": (ctypes.c_size_t, [_P, _I64]),
    "mdp_engine": (_I32, [_P, _I64, ctypes.POINTER(ctypes.c_char_p)]),
    "mdp_validate": (_I32, [_P, _D, _P, ctypes.c_size_t, _P, ctypes.POINTER(Validation)]),
    "mbdp_permutation": (_I32, [_I64, _U64, _U64, _P, _P]),
    "mb_sweep": (_I32, [_P, _P, _P, _I64, _U64, _U64, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mbdp_sync_status": (_I32, [_P, ctypes.c_size_t, _P]),
    "vi_solve": (_I32, [_P, _P, _P, _P, _I64, _U64, _U64, _D, _D, _P, _I64, _P,
                        ctypes.c_size_t, _P, ctypes.POINTER(Stats)]),
    "mpi_solve": (_I32, [_P, _P, _P, _P, _I32, _I32, _I64, _U64, _U64, _D, _D, _P, _I64, _P,
                         ctypes.c_size_t, _P, ctypes.POINTER(Stats)]),
    "vi_solve_noalloc": (_I32, [_P, _P, _P, _P, _I64, _U64, _U64, _D, _D, _P, _I64, _P,
                                ctypes.POINTER(Stats)]),
    "mdp_refine": (_I32, [_P, _P, _P, _I32, _I64, _U64, _U64, _D, _P, _I64, _P,
                          ctypes.c_size_t, _P, ctypes.POINTER(RefineStats)]),
    "mbdp_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libmbdp.so (loaded once)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MbdpLibraryMissing(
                "libmbdp.so is not built (%s); run __graft_entry__.build() or "
                "python -m paper_2110_02901_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().mbdp_last_error().decode()


def _check(status):
    if status != MBDP_OK:
        raise MbdpError(status, last_error())
    return status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _require(t, dtype, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))


class Handle:
    """An mbdp_mdp_t plus references that keep its borrowed tensors alive."""

    def __init__(self, ptr, n, m, keep):
        self.ptr = ptr
        self.n = n
        self.m = m
        self._keep = keep

    def close(self):
        if self.ptr:
            lib().mdp_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mdp_create_dense(P, c, gamma):
    import torch
    n, m = c.shape
    _require(P, torch.float32, n * m * n, "P")
    _require(c, torch.float32, n * m, "c")
    h = ctypes.c_void_p()
    _check(lib().mdp_create_dense(n, m, _ptr(P), _ptr(c), float(gamma), ctypes.byref(h)))
    return Handle(h, n, m, (P, c))


def mdp_create_csr(row_ptr, col, val, c, gamma, stream=None):
    import torch
    n, m = c.shape
    _require(row_ptr, torch.int64, n * m + 1, "row_ptr")
    _require(col, torch.int32, None, "col")
    _require(val, torch.float32, col.numel(), "val")
    _require(c, torch.float32, n * m, "c")
    h = ctypes.c_void_p()
    _check(lib().mdp_create_csr(n, m, _ptr(row_ptr), _ptr(col), _ptr(val), col.numel(),
                                _ptr(c), float(gamma), _stream(stream), ctypes.byref(h)))
    return Handle(h, n, m, (row_ptr, col, val, c))


def _code_dtype(dtype):
    import torch
    return torch.int16 if dtype == "bf16" else torch.uint8


def mdp_quantize_rows(src, dtype, stream=None):
    """src: FP32 [rows, row_len] on the GPU.  Returns (codes, row_scale):
    int16 (BF16 bit patterns) or uint8 (FP8 E4M3) codes of the same shape and
    FP32 scales [rows], written by the library's quantiser."""
    import torch
    rows, row_len = src.shape
    _require(src, torch.float32, None, "src")
    codes = torch.empty((rows, row_len), dtype=_code_dtype(dtype), device=src.device)
    scale = torch.empty(rows, dtype=torch.float32, device=src.device)
    _check(lib().mdp_quantize_rows(_ptr(src), rows, row_len, DTYPES[dtype], _ptr(codes),
                                   _ptr(scale), _stream(stream)))
    return codes, scale


def mdp_create_dense_q(Pq, dtype, row_scale, c, gamma):
    """Dense MDP from BF16 / FP8 codes [n*m*n] and row scales [n*m]."""
    import torch
    n, m = c.shape
    _require(Pq, _code_dtype(dtype), None, "P")
    if Pq.numel() != n * m * n:
        raise ValueError("P must have %d elements, got %d" % (n * m * n, Pq.numel()))
    _require(row_scale, torch.float32, n * m, "row_scale")
    _require(c, torch.float32, n * m, "c")
    h = ctypes.c_void_p()
    _check(lib().mdp_create_dense_q(n, m, _ptr(Pq), DTYPES[dtype], _ptr(row_scale), _ptr(c),
                                    float(gamma), ctypes.byref(h)))
    return Handle(h, n, m, (Pq, row_scale, c))


def mdp_create_csr_q(row_ptr, col, valq, dtype, row_scale, c, gamma, stream=None):
    """Sparse MDP with BF16 / FP8 values (constant row length k <= 64)."""
    import torch
    n, m = c.shape
    _require(row_ptr, torch.int64, n * m + 1, "row_ptr")
    _require(col, torch.int32, None, "col")
    _require(valq, _code_dtype(dtype), None, "val")
    if valq.numel() != col.numel():
        raise ValueError("val must have %d elements, got %d" % (col.numel(), valq.numel()))
    _require(row_scale, torch.float32, n * m, "row_scale")
    _require(c, torch.float32, n * m, "c")
    h = ctypes.c_void_p()
    _check(lib().mdp_create_csr_q(n, m, _ptr(row_ptr), _ptr(col), _ptr(valq), DTYPES[dtype],
                                  _ptr(row_scale), col.numel(), _ptr(c), float(gamma),
                                  _stream(stream), ctypes.byref(h)))
    return Handle(h, n, m, (row_ptr, col, valq, row_scale, c))


def mdp_policy_transpose(h, policy, k, ws, stream=None):
    """P_mu^T of an ELL handle as device CSR arrays (row_ptr, col, val)."""
    import torch
    n = h.n
    _require(policy, torch.int32, n, "policy")
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=policy.device)
    col = torch.empty(n * k, dtype=torch.int32, device=policy.device)
    val = torch.empty(n * k, dtype=torch.float32, device=policy.device)
    _check(lib().mdp_policy_transpose(h.ptr, _ptr(policy), _ptr(row_ptr), _ptr(col), _ptr(val),
                                      _ptr(ws), ws.numel(), _stream(stream)))
    return row_ptr, col, val


def mdp_value_gradients(h, policy, lam, V, ws, grad_c=True, grad_val=True, k=None, stream=None):
    """(dL/dc FP64 [n*m] or None, dL/dval FP64 [n*m*k] or None)."""
    import torch
    n, m = h.n, h.m
    _require(policy, torch.int32, n, "policy")
    _require(lam, torch.float64, n, "lambda")
    _require(V, torch.float64, n, "V")
    gc = torch.empty(n * m, dtype=torch.float64, device=V.device) if grad_c else None
    gv = torch.empty(n * m * k, dtype=torch.float64, device=V.device) if grad_val else None
    _check(lib().mdp_value_gradients(h.ptr, _ptr(policy), _ptr(lam), _ptr(V),
                                     _ptr(gc) if gc is not None else None,
                                     _ptr(gv) if gv is not None else None,
                                     _ptr(ws), ws.numel(), _stream(stream)))
    return gc, gv


_BATCH_DTYPES = {"f32": MBDP_F32, "bf16": MBDP_BF16, "fp8": MBDP_FP8_E4M3}


def batch_workspace(count):
    """A torch uint8 workspace for a batch of `count` MDPs (256-byte aligned)."""
    import torch
    nbytes = int(lib().mdp_batch_workspace_bytes(int(count)))
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def multi_workspace(h, r, b):
    """A torch uint8 workspace for mdp_multi_solve (256-byte aligned)."""
    import torch
    nbytes = int(lib().mdp_multi_workspace_bytes(h.ptr, int(r), int(b)))
    if nbytes == 0:
        raise MbdpError(MBDP_ERR_INVALID_ARG, "no multi-vector workspace for this handle, r and b")
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def mdp_multi_solve(h, C, V, b, seed, ws, tol_dv=1e-8, max_sweeps=100000, first_sweep=0,
                    policy=None, stream=None):
    """MB-VI on r vectors at once: C FP32 [n, m, r], V FP64 [n, r] (V0 in, result
    out), policy int32 [n, r] or None.  Returns the statistics as a dict."""
    import torch
    r = int(C.shape[2])
    _require(C, torch.float32, h.n * h.m * r, "C")
    _require(V, torch.float64, h.n * r, "V")
    if policy is not None:
        _require(policy, torch.int32, h.n * r, "policy")
    st = MultiStats()
    status = lib().mdp_multi_solve(h.ptr, r, _ptr(C), _ptr(V), _ptr(policy), int(b),
                                   int(seed), int(first_sweep), float(tol_dv), int(max_sweeps),
                                   _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(st))
    if status not in (MBDP_OK, MBDP_ERR_NOT_CONVERGED):
        _check(status)
    return st.as_dict()


def mdp_batch_upload(items, ws, stream=None):
    """items: list of dicts with n, m, dtype ('f32' / 'bf16' / 'fp8'), ld, P,
    row_scale (or None), c, gamma, b, seed, V (FP64, V0 in / result out),
    policy (int32 or None), lanes (0 = default), team (workgroups; 0 = by work).  The tensors must stay
    alive while launches use them."""
    arr = (BatchItem * len(items))()
    for i, it in enumerate(items):
        arr[i] = BatchItem(int(it["n"]), int(it["m"]), _BATCH_DTYPES[it.get("dtype", "f32")],
                           int(it["ld"]), it["P"].data_ptr(),
                           it["row_scale"].data_ptr() if it.get("row_scale") is not None else None,
                           it["c"].data_ptr(), float(it["gamma"]), int(it["b"]),
                           int(it.get("seed", 0)), it["V"].data_ptr(),
                           it["policy"].data_ptr() if it.get("policy") is not None else None,
                           int(it.get("lanes", 0)), int(it.get("team", 0)))
    _check(lib().mdp_batch_upload(arr, len(items), _ptr(ws), ws.numel(), _stream(stream)))


def mdp_batch_launch(count, tol_dv, max_sweeps, ws, stream=None):
    _check(lib().mdp_batch_launch(int(count), float(tol_dv), int(max_sweeps), _ptr(ws),
                                  ws.numel(), _stream(stream)))


def mdp_batch_read_stats(ws, count, stream=None):
    out = (BatchStats * count)()
    _check(lib().mdp_batch_read_stats(_ptr(ws), int(count), out, _stream(stream)))
    return [{"sweeps": o.sweeps, "final_dv_inf": o.final_dv_inf, "converged": o.converged,
             "team": o.team, "start_us": o.start_us, "end_us": o.end_us} for o in out]


def mdp_destroy(h):
    h.close()


def mdp_column_blocks(h, stream=None):
    """Builds and attaches the column-sorted blocks (b = n kernel) of an
    ELL FP32 handle; returns the device buffer, which the handle keeps."""
    import torch
    nbytes = ctypes.c_size_t(0)
    _check(lib().mdp_column_blocks_prepare(h.ptr, _stream(stream), ctypes.byref(nbytes)))
    buf = torch.empty((nbytes.value + 255) // 256 * 256 // 4, dtype=torch.int32,
                      device=torch.device("cuda", torch.cuda.current_device()))
    _check(lib().mdp_column_blocks_attach(h.ptr, _ptr(buf), buf.numel() * 4, _stream(stream)))
    h._keep = list(h._keep) + [buf]
    return buf


def mdp_set_tuning(h, blocks_per_cu=0, threads_per_block=0, recentre_every=0, recentre_force=0,
                   band_window=0):
    t = Tuning(blocks_per_cu, threads_per_block, recentre_every, int(bool(recentre_force)),
               band_window)
    _check(lib().mdp_set_tuning(h.ptr, ctypes.byref(t)))


def mdp_engine(h, b):
    """Kernel family the solvers run for this handle and batch size."""
    name = ctypes.c_char_p()
    _check(lib().mdp_engine(h.ptr, int(b), ctypes.byref(name)))
    return name.value.decode()


def mdp_workspace_bytes(h, b):
    return int(lib().mdp_workspace_bytes(h.ptr, int(b)))


def workspace(h, b):
    """A torch uint8 workspace tensor of the required size (256-byte aligned)."""
    import torch
    nbytes = mdp_workspace_bytes(h, b)
    if nbytes == 0:
        raise MbdpError(MBDP_ERR_INVALID_ARG, "bad handle or batch size %r" % (b,))
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def mdp_validate(h, row_sum_tol, ws, stream=None):
    rep = Validation()
    st = lib().mdp_validate(h.ptr, float(row_sum_tol), _ptr(ws), ws.numel(), _stream(stream),
                            ctypes.byref(rep))
    if st not in (MBDP_OK, MBDP_ERR_VALIDATION):
        _check(st)
    return st == MBDP_OK, rep.as_dict()


def mbdp_permutation(n, seed, sweep_index, out, stream=None):
    import torch
    _require(out, torch.int32, n, "out")
    _check(lib().mbdp_permutation(int(n), int(seed), int(sweep_index), _ptr(out), _stream(stream)))
    return out


def mb_sweep(h, V, b, seed, sweep_index, ws, policy=None, perm=None, argmin_out=None,
             dv_out=None, stream=None):
    import torch
    _require(V, torch.float32, h.n, "V")
    if policy is not None:
        _require(policy, torch.int32, h.n, "policy")
    if perm is not None:
        _require(perm, torch.int32, h.n, "perm")
    if argmin_out is not None:
        _require(argmin_out, torch.int32, h.n, "argmin_out")
    if dv_out is not None:
        _require(dv_out, torch.float32, 1, "dv_out")
    _check(lib().mb_sweep(h.ptr, _ptr(V), _ptr(policy), int(b), int(seed), int(sweep_index),
                          _ptr(perm), _ptr(argmin_out), _ptr(dv_out), _ptr(ws), ws.numel(),
                          _stream(stream)))


def mbdp_sync_status(ws, stream=None):
    _check(lib().mbdp_sync_status(_ptr(ws), ws.numel(), _stream(stream)))


def vi_solve(h, V, b, seed, ws, first_sweep=0, tol_dv=-1.0, eps=0.0, V_ref=None,
             max_sweeps=100000, policy_out=None, V64_out=None, stream=None):
    """Returns the statistics dict (``converged`` False when the limit was hit)."""
    import torch
    _require(V, torch.float32, h.n, "V")
    if V_ref is not None:
        _require(V_ref, torch.float64, h.n, "V_ref")
    if policy_out is not None:
        _require(policy_out, torch.int32, h.n, "policy_out")
    if V64_out is not None:
        _require(V64_out, torch.float64, h.n, "V64_out")
    st = Stats()
    status = lib().vi_solve(h.ptr, _ptr(V), _ptr(V64_out), _ptr(policy_out), int(b), int(seed),
                            int(first_sweep), float(tol_dv), float(eps), _ptr(V_ref),
                            int(max_sweeps), _ptr(ws), ws.numel(), _stream(stream),
                            ctypes.byref(st))
    if status != MBDP_ERR_NOT_CONVERGED:
        _check(status)
    return st.as_dict()


def vi_solve_noalloc(h, V, b, seed, first_sweep=0, tol_dv=-1.0, eps=0.0, V_ref=None,
                     max_sweeps=100000, policy_out=None, V64_out=None, stream=None):
    """vi_solve without a workspace (the library's own scratch memory)."""
    import torch
    _require(V, torch.float32, h.n, "V")
    if V_ref is not None:
        _require(V_ref, torch.float64, h.n, "V_ref")
    if policy_out is not None:
        _require(policy_out, torch.int32, h.n, "policy_out")
    if V64_out is not None:
        _require(V64_out, torch.float64, h.n, "V64_out")
    st = Stats()
    status = lib().vi_solve_noalloc(h.ptr, _ptr(V), _ptr(V64_out), _ptr(policy_out), int(b),
                                    int(seed), int(first_sweep), float(tol_dv), float(eps),
                                    _ptr(V_ref), int(max_sweeps), _stream(stream),
                                    ctypes.byref(st))
    if status != MBDP_ERR_NOT_CONVERGED:
        _check(status)
    return st.as_dict()


def mpi_solve(h, V, policy, K, b, seed, ws, policy_is_init=True, first_sweep=0, tol_dv=-1.0,
              eps=0.0, V_ref=None, max_outer=10000, V64_out=None, stream=None):
    import torch
    _require(V, torch.float32, h.n, "V")
    _require(policy, torch.int32, h.n, "policy")
    if V_ref is not None:
        _require(V_ref, torch.float64, h.n, "V_ref")
    if V64_out is not None:
        _require(V64_out, torch.float64, h.n, "V64_out")
    st = Stats()
    status = lib().mpi_solve(h.ptr, _ptr(V), _ptr(V64_out), _ptr(policy), int(bool(policy_is_init)),
                             int(K), int(b), int(seed), int(first_sweep), float(tol_dv),
                             float(eps), _ptr(V_ref), int(max_outer), _ptr(ws), ws.numel(),
                             _stream(stream), ctypes.byref(st))
    if status != MBDP_ERR_NOT_CONVERGED:
        _check(status)
    return st.as_dict()


def mdp_refine(h, V, b, seed, ws, K=0, eps=1e-6, V_ref=None, first_sweep=0, max_iters=100000,
               policy_out=None, stream=None):
    """Certified FP64 correction of V (FP64, in place) on an FP32 handle.

    Returns the statistics dict (``converged`` False when the limit was hit).
    """
    import torch
    _require(V, torch.float64, h.n, "V")
    if V_ref is not None:
        _require(V_ref, torch.float64, h.n, "V_ref")
    if policy_out is not None:
        _require(policy_out, torch.int32, h.n, "policy_out")
    st = RefineStats()
    status = lib().mdp_refine(h.ptr, _ptr(V), _ptr(policy_out), int(K), int(b), int(seed),
                              int(first_sweep), float(eps), _ptr(V_ref), int(max_iters),
                              _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(st))
    if status != MBDP_ERR_NOT_CONVERGED:
        _check(status)
    return st.as_dict()
