"""Python binding of libpluq.so, the MI355X rank-profile PLUQ library.

Argument marshalling only: every step of the decomposition runs in the HIP
library.  PyTorch provides device memory and the current stream.  The
functions carry the names of the C ABI in include/pluq.h; ``pluq`` is a
convenience wrapper that allocates P, Q and the workspace.

There is no fallback: if libpluq.so is missing or a call fails, an exception
is raised.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpluq.so")

PLUQ_OK = 0
PLUQ_ERR_ARG = 1
PLUQ_ERR_UNSUPPORTED = 4
PLUQ_ERR_WORKSPACE = 7
STATUS = {0: "ok", 1: "invalid argument", 2: "modulus outside [2, 2^26)", 3: "entry outside [0, p)",
          4: "form cannot be exact for this modulus", 5: "host allocation failed",
          6: "device (HIP) error", 7: "workspace too small"}
DTYPES = {"int64": 0, "float64": 1, "int32": 2}
FORMS = {"fp64": 0, "int8": 1, "fp32": 2}

_lib = None
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)


class PluqError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class pluq_opts(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("validate_entries", ctypes.c_int32),
                ("cutoff_override", ctypes.c_int32),
                ("batch_panel", ctypes.c_int32), ("batch_groups", ctypes.c_int32),
                ("no_speculation", ctypes.c_int32), ("branches", ctypes.c_int32),
                ("in_place", ctypes.c_int32)]


class pluq_tune(ctypes.Structure):
    _fields_ = [("mm_tiles128", ctypes.c_int32), ("mm_tiles64", ctypes.c_int32), ("cutoff", ctypes.c_int32),
                ("fork_min_dim", ctypes.c_int32), ("i8_min_work", ctypes.c_int64), ("batch_panel", ctypes.c_int32),
                ("batch_groups", ctypes.c_int32), ("strassen_min", ctypes.c_int32)]


TUNE_FIELDS = [f for f, _ in pluq_tune._fields_]
TUNE_FORM_BATCHED = 3
TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


class pluq_kernel_stat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


KERNEL_CLASSES = ["modmm", "trsm_leaf", "perm", "basecase", "scan", "limb", "modmm_i8", "trsm_diag",
                  "basecase_rpm", "lincomb"]


def load():
    """Load libpluq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1301_4438_amd/build.py")
    # torch first: the library must bind to the HIP runtime torch has loaded
    # (loaded before torch, it would bring in a second runtime, and the one
    # it calls then sees no device)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.pluq_status_string.restype = ctypes.c_char_p
    L.pluq_status_string.argtypes = [ctypes.c_int]
    L.pluq_version.restype = ctypes.c_char_p
    L.pluq_last_error.restype = ctypes.c_char_p
    L.pluq_last_error.argtypes = []
    L.pluq_workspace_size.restype = ctypes.c_size_t
    L.pluq_workspace_size.argtypes = [_i64, _i64, ctypes.c_int, _u64, ctypes.POINTER(pluq_opts)]
    L.pluq_modp.restype = ctypes.c_int
    L.pluq_modp.argtypes = [_i64, _i64, _vp, _i64, ctypes.c_int, _u64, _vp, _vp, _i64p,
                            ctypes.POINTER(pluq_opts), _vp, ctypes.c_size_t, _vp]
    L.pluq_rank_profiles.restype = ctypes.c_int
    L.pluq_rank_profiles.argtypes = [_i64, _i64, _i64, _i64p, _i64p, _i64p, _i64p]
    L.pluq_leading_rank_profiles.restype = ctypes.c_int
    L.pluq_leading_rank_profiles.argtypes = [_i64, _i64, _i64, _i64p, _i64p, _i64, _i64, _i64p, _i64p, _i64p]
    L.pluq_batched_workspace_size.restype = ctypes.c_size_t
    L.pluq_batched_workspace_size.argtypes = [_i64, _i64p, _i64p, ctypes.c_int, _u64, ctypes.POINTER(pluq_opts)]
    L.pluq_modp_batched.restype = ctypes.c_int
    L.pluq_modp_batched.argtypes = [_i64, _i64p, _i64p, ctypes.POINTER(_vp), _i64p, ctypes.c_int, _u64,
                                    ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, ctypes.POINTER(pluq_opts),
                                    _vp, ctypes.c_size_t, _vp]
    L.pluq_batched_prepare.restype = ctypes.c_int
    L.pluq_batched_prepare.argtypes = [_i64, _i64p, _i64p, ctypes.POINTER(_vp), _i64p, ctypes.c_int, _u64,
                                       ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, ctypes.POINTER(pluq_opts),
                                       _vp, ctypes.c_size_t]
    L.pluq_batched_run.restype = ctypes.c_int
    L.pluq_batched_run.argtypes = [_i64, ctypes.c_int, _u64, ctypes.POINTER(pluq_opts), _vp, ctypes.c_size_t, _vp]
    L.pluq_modmm_workspace_size.restype = ctypes.c_size_t
    L.pluq_modmm_workspace_size.argtypes = [_i64, _i64, _i64, ctypes.c_int32]
    L.pluq_modmm_winograd_workspace_size.restype = ctypes.c_size_t
    L.pluq_modmm_winograd_workspace_size.argtypes = [_i64, _i64, _i64, ctypes.c_int]
    L.pluq_modmm_winograd.restype = ctypes.c_int
    L.pluq_modmm_winograd.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, _u64,
                                      ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
    L.pluq_modmm.restype = ctypes.c_int
    L.pluq_modmm.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, _u64,
                             ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
    L.pluq_post_workspace_size.restype = ctypes.c_size_t
    L.pluq_post_workspace_size.argtypes = [_i64, _i64]
    L.pluq_leu.restype = ctypes.c_int
    L.pluq_leu.argtypes = [_i64, _i64, _i64, _vp, _i64, ctypes.c_int, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp,
                           ctypes.c_size_t, _vp]
    L.pluq_echelon.restype = ctypes.c_int
    L.pluq_echelon.argtypes = [ctypes.c_int32, _i64, _i64, _i64, _vp, _i64, ctypes.c_int, _vp, _vp, _vp, _i64, _vp,
                               _i64, _vp, _vp, ctypes.c_size_t, _vp]
    L.pluq_leading_ranks.restype = ctypes.c_int
    L.pluq_leading_ranks.argtypes = [_i64, _i64, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.pluq_leading_rank_profiles_device.restype = ctypes.c_int
    L.pluq_leading_rank_profiles_device.argtypes = [_i64, _i64, _i64, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp,
                                                    ctypes.c_size_t, _vp]
    L.pluq_tune_set.restype = ctypes.c_int
    L.pluq_tune_set.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    L.pluq_tune_clear.restype = None
    L.pluq_tune_clear.argtypes = []
    L.pluq_tune_get.restype = ctypes.c_int
    L.pluq_tune_get.argtypes = [ctypes.c_int32, _u64, ctypes.c_int32, _i64, _i64, ctypes.c_void_p, ctypes.c_void_p]
    L.pluq_modmm_noalloc.restype = ctypes.c_int
    L.pluq_modmm_noalloc.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, _u64,
                                     ctypes.c_int32, _vp]
    L.pluq_trsm_workspace_size.restype = ctypes.c_size_t
    L.pluq_trsm_workspace_size.argtypes = [_i64, ctypes.c_int]
    L.pluq_trsm.restype = ctypes.c_int
    L.pluq_trsm.argtypes = [ctypes.c_int32, _i64, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, _u64,
                            ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
    L.pluq_profile_enable.restype = None
    L.pluq_profile_enable.argtypes = [ctypes.c_int32]
    L.pluq_profile_read.restype = None
    L.pluq_profile_read.argtypes = [ctypes.POINTER(pluq_kernel_stat)]
    L.pluq_last_stats.restype = None
    L.pluq_last_stats.argtypes = [_i64p, _i64p, _i64p, _i64p]
    _lib = L
    if os.environ.get("PLUQ_NO_TUNE_CACHE") != "1":
        load_tune_cache()
    return L


# --------------------------------------------------------------- helpers --

def _dtype_code(t) -> int:
    import torch
    m = {torch.int64: 0, torch.float64: 1, torch.int32: 2}
    if t.dtype not in m:
        raise TypeError(f"unsupported element type {t.dtype} (int64, float64 or int32)")
    return m[t.dtype]


def _ld(t) -> int:
    """Row stride of a row-major 2-D tensor; a single row's is immaterial
    (torch may report any stride for a dimension of size one)."""
    return t.stride(0) if t.shape[0] > 1 else max(1, t.shape[1])


def _torch():
    import torch
    return torch


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _opts(form="fp64", validate=False, cutoff=0, batch_panel=0, batch_groups=0, speculate=True, branches=0,
          in_place=False):
    o = pluq_opts()
    o.no_speculation = 0 if speculate else 1
    o.branches = int(branches)
    o.in_place = int(bool(in_place))
    o.form = FORMS[form] if isinstance(form, str) else int(form)
    o.validate_entries = int(bool(validate))
    o.cutoff_override = int(cutoff)
    o.batch_panel = int(batch_panel)
    o.batch_groups = int(batch_groups)
    return o


def _check(st, where):
    if st != PLUQ_OK:
        detail = _lib.pluq_last_error().decode() if _lib is not None else ""
        raise PluqError(st, f"{where} [{detail}]" if detail else where)


# Workspace buffers kept between calls, per host thread and device: calls
# from different threads may run concurrently (each on its own stream), so
# they must not share scratch memory.
_ws_local = threading.local()


def _workspace(device, nbytes):
    import torch
    cache = getattr(_ws_local, "cache", None)
    if cache is None:
        cache = _ws_local.cache = {}
    key = str(device)
    buf = cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        cache[key] = buf
    return buf


# ------------------------------------------------------------ C ABI names --

def tune_set(form, pclass, dtype, bucket, **params):
    """Register tuned parameters for a key (form code or 3 for the batched
    form, p class, element type code, shape bucket; -1 matches anything)."""
    t = pluq_tune()
    for k, v in params.items():
        setattr(t, k, int(v))
    _check(load().pluq_tune_set(int(form), int(pclass), int(dtype), int(bucket), ctypes.byref(t)), "pluq_tune_set")


def tune_clear():
    load().pluq_tune_clear()


def tune_get(form, p, dtype, m, n):
    """(parameters a call with these arguments uses, whether a table entry matched)."""
    t = pluq_tune()
    hit = ctypes.c_int32(0)
    _check(load().pluq_tune_get(int(form), int(p), int(dtype), int(m), int(n), ctypes.byref(t), ctypes.byref(hit)),
           "pluq_tune_get")
    return {f: getattr(t, f) for f in TUNE_FIELDS}, bool(hit.value)


def load_tune_cache(path=None):
    """Register the entries of the tuner's cache (gfx950 entries only).
    Returns the number of entries registered."""
    import json
    path = path or TUNE_CACHE
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        cache = json.load(f)
    if cache.get("arch") != "gfx950":
        return 0
    for e in cache.get("entries", []):
        tune_set(e["form"], e["pclass"], e["dtype"], e["bucket"], **e["params"])
    return len(cache.get("entries", []))


def pluq_status_string(status: int) -> str:
    return load().pluq_status_string(int(status)).decode()


def pluq_version() -> str:
    return load().pluq_version().decode()


def pluq_workspace_size(m, n, dtype_code, p, opts=None) -> int:
    return int(load().pluq_workspace_size(m, n, dtype_code, p, ctypes.byref(opts) if opts else None))


def pluq_modp(A, p: int, P, Q, opts=None, work=None):
    """In-place decomposition of the 2-D device tensor A (row-major, any
    leading dimension).  P, Q: device int64 tensors of length m, n.
    Returns r."""
    L = load()
    m, n = A.shape
    lda = A.stride(0) if m > 1 else max(1, n)
    if A.dim() != 2 or (m > 0 and n > 1 and A.stride(1) != 1):
        raise ValueError("A must be a row-major 2-D tensor with unit column stride")
    if m == 0 or n == 0:
        lda = max(1, n)
    dt = _dtype_code(A)
    need = L.pluq_workspace_size(m, n, dt, p, ctypes.byref(opts) if opts else None)
    if work is None:
        work = _workspace(A.device, need)
    r = ctypes.c_int64(0)
    st = L.pluq_modp(m, n, ctypes.c_void_p(A.data_ptr()), max(lda, 1), dt, p,
                     ctypes.c_void_p(P.data_ptr() if m else 0), ctypes.c_void_p(Q.data_ptr() if n else 0),
                     ctypes.byref(r), ctypes.byref(opts) if opts else None,
                     ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(A))
    _check(st, "pluq_modp")
    return int(r.value)


def pluq_rank_profiles(P, Q, r):
    """Host arrays (numpy/torch CPU int64) -> (row_rp, col_rp) numpy arrays."""
    import numpy as np
    P = np.ascontiguousarray(np.asarray(P, dtype=np.int64))
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.int64))
    rr = np.zeros(max(r, 1), np.int64)
    cc = np.zeros(max(r, 1), np.int64)
    st = load().pluq_rank_profiles(len(P), len(Q), r, P.ctypes.data_as(_i64p), Q.ctypes.data_as(_i64p),
                                   rr.ctypes.data_as(_i64p), cc.ctypes.data_as(_i64p))
    _check(st, "pluq_rank_profiles")
    return rr[:r], cc[:r]


def pluq_leading_rank_profiles(P, Q, r, k, t):
    import numpy as np
    P = np.ascontiguousarray(np.asarray(P, dtype=np.int64))
    Q = np.ascontiguousarray(np.asarray(Q, dtype=np.int64))
    rows = np.zeros(max(r, 1), np.int64)
    cols = np.zeros(max(r, 1), np.int64)
    cnt = ctypes.c_int64(0)
    st = load().pluq_leading_rank_profiles(len(P), len(Q), r, P.ctypes.data_as(_i64p), Q.ctypes.data_as(_i64p),
                                           k, t, rows.ctypes.data_as(_i64p), cols.ctypes.data_as(_i64p),
                                           ctypes.byref(cnt))
    _check(st, "pluq_leading_rank_profiles")
    return rows[:cnt.value], cols[:cnt.value]


class BatchedCall:
    """Arguments of one batched decomposition, marshalled once: the device
    tensors (in place), P and Q per matrix, the rank vector and the
    workspace.  `prepare()` writes the descriptor table (synchronous),
    `run()` enqueues the single kernel (capturable into a HIP graph)."""

    def __init__(self, mats, p: int, Ps, Qs, d_r, opts=None, work=None):
        import numpy as np
        self.L = load()
        self.mats, self.Ps, self.Qs, self.d_r = list(mats), list(Ps), list(Qs), d_r
        self.p = int(p)
        self.opts = opts
        b = len(self.mats)
        self.batch = b
        if len(self.Ps) != b or len(self.Qs) != b or d_r.numel() != b or d_r.dtype != _torch().int64:
            raise ValueError("need one P, one Q and one int64 rank slot per matrix")
        dts = {_dtype_code(a) for a in self.mats}
        if len(dts) > 1:
            raise TypeError("all matrices of a batch must share one element type")
        self.dt = dts.pop() if dts else 1
        for a in self.mats:
            if a.dim() != 2 or (a.shape[0] > 0 and a.shape[1] > 1 and a.stride(1) != 1):
                raise ValueError("matrices must be row-major 2-D tensors with unit column stride")
        self.m = np.array([a.shape[0] for a in self.mats], np.int64)
        self.n = np.array([a.shape[1] for a in self.mats], np.int64)
        # a single row's leading dimension is immaterial (torch may report any
        # stride for a dimension of size one)
        self.lda = np.array([a.stride(0) if a.shape[0] > 1 else max(1, a.shape[1]) for a in self.mats], np.int64)
        self.pa = (_vp * max(b, 1))(*[a.data_ptr() for a in self.mats])
        self.pp = (_vp * max(b, 1))(*[t.data_ptr() for t in self.Ps])
        self.pq = (_vp * max(b, 1))(*[t.data_ptr() for t in self.Qs])
        o = ctypes.byref(opts) if opts else None
        need = int(self.L.pluq_batched_workspace_size(b, self.m.ctypes.data_as(_i64p), self.n.ctypes.data_as(_i64p),
                                                      self.dt, self.p, o))
        if b and need == 0:
            raise PluqError(PLUQ_ERR_UNSUPPORTED, "pluq_batched_workspace_size")
        dev = self.mats[0].device if b else "cuda"
        self.work = work if work is not None else _torch().empty(max(need, 256), dtype=_torch().uint8, device=dev)

    def prepare(self):
        o = ctypes.byref(self.opts) if self.opts else None
        st = self.L.pluq_batched_prepare(self.batch, self.m.ctypes.data_as(_i64p), self.n.ctypes.data_as(_i64p),
                                         self.pa, self.lda.ctypes.data_as(_i64p), self.dt, self.p, self.pp, self.pq,
                                         ctypes.c_void_p(self.d_r.data_ptr()), o,
                                         ctypes.c_void_p(self.work.data_ptr()), self.work.numel())
        _check(st, "pluq_batched_prepare")
        return self

    def run(self, stream=None):
        o = ctypes.byref(self.opts) if self.opts else None
        s = stream if stream is not None else (_stream(self.mats[0]) if self.batch else None)
        st = self.L.pluq_batched_run(self.batch, self.dt, self.p, o, ctypes.c_void_p(self.work.data_ptr()),
                                     self.work.numel(), s)
        _check(st, "pluq_batched_run")


def pluq_modp_batched(mats, p: int, Ps, Qs, d_r, opts=None):
    """In-place decomposition of every 2-D device tensor in `mats` (one
    element type, m, n <= 512) in one persistent launch; ranks into the
    device int64 tensor d_r.  Asynchronous."""
    call = BatchedCall(mats, p, Ps, Qs, d_r, opts)
    o = ctypes.byref(opts) if opts else None
    st = call.L.pluq_modp_batched(call.batch, call.m.ctypes.data_as(_i64p), call.n.ctypes.data_as(_i64p), call.pa,
                                  call.lda.ctypes.data_as(_i64p), call.dt, call.p, call.pp, call.pq,
                                  ctypes.c_void_p(d_r.data_ptr()), o, ctypes.c_void_p(call.work.data_ptr()),
                                  call.work.numel(), _stream(mats[0]) if call.batch else None)
    _check(st, "pluq_modp_batched")
    return call


def pluq_modmm(C, A, B, p: int, form="fp64", work=None):
    """C <- C - A B mod p on device tensors (in place, asynchronous)."""
    L = load()
    m, n = C.shape
    k = A.shape[1]
    if tuple(A.shape) != (m, k) or tuple(B.shape) != (k, n):
        raise ValueError(f"shape mismatch: C {tuple(C.shape)}, A {tuple(A.shape)}, B {tuple(B.shape)}")
    if A.dtype != C.dtype or B.dtype != C.dtype:
        raise TypeError("A, B and C must share one element type")
    for t in (A, B, C):
        if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
            raise ValueError("operands must be row-major 2-D tensors with unit column stride")
    dt = _dtype_code(C)
    fcode = FORMS[form] if isinstance(form, str) else int(form)
    need = int(L.pluq_modmm_workspace_size(m, n, k, fcode))
    if work is None and need:
        work = _workspace(C.device, need)
    st = L.pluq_modmm(m, n, k, ctypes.c_void_p(C.data_ptr()), _ld(C), ctypes.c_void_p(A.data_ptr()),
                      _ld(A), ctypes.c_void_p(B.data_ptr()), _ld(B), dt, p, fcode,
                      ctypes.c_void_p(work.data_ptr() if work is not None else 0),
                      work.numel() if work is not None else 0, _stream(C))
    _check(st, "pluq_modmm")


def pluq_modmm_winograd(C, A, B, p: int, form="fp64", work=None):
    """C <- C - A B mod p by one level of Winograd's scheme (FP64 or FP32
    form; m, n, k >= 2), in place and asynchronous."""
    L = load()
    m, n = C.shape
    k = A.shape[1]
    if tuple(A.shape) != (m, k) or tuple(B.shape) != (k, n):
        raise ValueError(f"shape mismatch: C {tuple(C.shape)}, A {tuple(A.shape)}, B {tuple(B.shape)}")
    if A.dtype != C.dtype or B.dtype != C.dtype:
        raise TypeError("A, B and C must share one element type")
    for t in (A, B, C):
        if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
            raise ValueError("operands must be row-major 2-D tensors with unit column stride")
    dt = _dtype_code(C)
    fcode = FORMS[form] if isinstance(form, str) else int(form)
    need = int(L.pluq_modmm_winograd_workspace_size(m, n, k, dt))
    if work is None:
        work = _workspace(C.device, max(need, 256))
    st = L.pluq_modmm_winograd(m, n, k, ctypes.c_void_p(C.data_ptr()), _ld(C), ctypes.c_void_p(A.data_ptr()),
                               _ld(A), ctypes.c_void_p(B.data_ptr()), _ld(B), dt, p, fcode,
                               ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(C))
    _check(st, "pluq_modmm_winograd")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)


def _post_ws(m, n, device):
    return _workspace(device, int(load().pluq_post_workspace_size(m, n)))


def pluq_leu(X, P, Q, r: int):
    """LEU decomposition (Section 3) of a finished decomposition (X packed,
    P, Q device int64): returns (Lbar m x m, Ubar n x n, Erow) with Erow[i]
    the column of row i's rank-profile entry or -1.  Asynchronous."""
    import torch
    L = load()
    m, n = X.shape
    Lb = torch.empty((m, m), dtype=X.dtype, device=X.device)
    Ub = torch.empty((n, n), dtype=X.dtype, device=X.device)
    Er = torch.empty(m, dtype=torch.int64, device=X.device)
    ws = _post_ws(m, n, X.device)
    st = L.pluq_leu(m, n, int(r), _ptr(X), _ld(X) if m else max(n, 1), _dtype_code(X), _ptr(P), _ptr(Q), _ptr(Lb),
                    max(m, 1), _ptr(Ub), max(n, 1), _ptr(Er), _ptr(ws), ws.numel(), _stream(X))
    _check(st, "pluq_leu")
    return Lb, Ub, Er


def pluq_echelon(X, P, Q, r: int, kind="column"):
    """kind "column": (C m x r, R r x n, row rank profile), A = C R;
    kind "row": (E r x n, L_E m x r, column rank profile), A = L_E E."""
    import torch
    L = load()
    m, n = X.shape
    k = 0 if kind == "column" else 1
    F = torch.empty((m, r) if k == 0 else (r, n), dtype=X.dtype, device=X.device)
    G = torch.empty((r, n) if k == 0 else (m, r), dtype=X.dtype, device=X.device)
    prof = torch.empty(r, dtype=torch.int64, device=X.device)
    ws = _post_ws(m, n, X.device)
    st = L.pluq_echelon(k, m, n, int(r), _ptr(X), _ld(X) if m else max(n, 1), _dtype_code(X), _ptr(P), _ptr(Q),
                        _ptr(F), max(F.shape[1], 1), _ptr(G), max(G.shape[1], 1), _ptr(prof), _ptr(ws),
                        ws.numel(), _stream(X))
    _check(st, "pluq_echelon")
    return F, G, prof


def pluq_leading_ranks(P, Q, r: int, ks, ts):
    """Ranks of the leading ks[q] x ts[q] blocks (device int64 tensors)."""
    import torch
    L = load()
    m, n = P.numel(), Q.numel()
    out = torch.empty(ks.numel(), dtype=torch.int64, device=ks.device)
    ws = _post_ws(m, n, ks.device)
    st = L.pluq_leading_ranks(m, n, int(r), _ptr(P), _ptr(Q), ks.numel(), _ptr(ks), _ptr(ts), _ptr(out), _ptr(ws),
                              ws.numel(), _stream(ks))
    _check(st, "pluq_leading_ranks")
    return out


def pluq_leading_rank_profiles_device(P, Q, r: int, k: int, t: int):
    """(rows, cols) of the leading k x t block, sorted, as device tensors."""
    import torch
    L = load()
    m, n = P.numel(), Q.numel()
    rows = torch.empty(max(r, 1), dtype=torch.int64, device=P.device)
    cols = torch.empty(max(r, 1), dtype=torch.int64, device=P.device)
    cnt = torch.zeros(2, dtype=torch.int64, device=P.device)
    ws = _post_ws(m, n, P.device)
    st = L.pluq_leading_rank_profiles_device(m, n, int(r), _ptr(P), _ptr(Q), int(k), int(t), _ptr(rows),
                                             _ptr(cols), _ptr(cnt), _ptr(ws), ws.numel(), _stream(P))
    _check(st, "pluq_leading_rank_profiles_device")
    c = cnt.cpu().tolist()
    return rows[:c[0]], cols[:c[1]]


def pluq_modmm_noalloc(C, A, B, p: int, form="fp64"):
    """pluq_modmm through the entry point that allocates nothing (the INT8
    form's digit planes in the library's static device scratch)."""
    L = load()
    m, n = C.shape
    k = A.shape[1]
    if tuple(A.shape) != (m, k) or tuple(B.shape) != (k, n):
        raise ValueError(f"shape mismatch: C {tuple(C.shape)}, A {tuple(A.shape)}, B {tuple(B.shape)}")
    if A.dtype != C.dtype or B.dtype != C.dtype:
        raise TypeError("A, B and C must share one element type")
    for t in (A, B, C):
        if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
            raise ValueError("operands must be row-major 2-D tensors with unit column stride")
    fcode = FORMS[form] if isinstance(form, str) else int(form)
    st = L.pluq_modmm_noalloc(m, n, k, ctypes.c_void_p(C.data_ptr()), _ld(C), ctypes.c_void_p(A.data_ptr()),
                              _ld(A), ctypes.c_void_p(B.data_ptr()), _ld(B), _dtype_code(C), p, fcode, _stream(C))
    _check(st, "pluq_modmm_noalloc")


def pluq_trsm(side: int, T, B, p: int, form="fp64"):
    """side 0: B <- L^{-1} B (L unit lower, r x r); side 1: B <- B U^{-1}."""
    L = load()
    r = T.shape[0]
    other = B.shape[1] if side == 0 else B.shape[0]
    if tuple(T.shape) != (r, r) or (B.shape[0] if side == 0 else B.shape[1]) != r:
        raise ValueError(f"shape mismatch: T {tuple(T.shape)}, B {tuple(B.shape)}, side {side}")
    if T.dtype != B.dtype:
        raise TypeError("T and B must share one element type")
    dt = _dtype_code(B)
    fcode = FORMS[form] if isinstance(form, str) else int(form)
    work = _workspace(B.device, int(L.pluq_trsm_workspace_size(r, dt)))
    st = L.pluq_trsm(side, r, other, ctypes.c_void_p(T.data_ptr()), _ld(T), ctypes.c_void_p(B.data_ptr()),
                     _ld(B), dt, p, fcode, ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(B))
    _check(st, "pluq_trsm")


def pluq_profile_enable(mask=-1):
    """mask: bit c times kernel class c (KERNEL_CLASSES order); -1 all, 0 off."""
    load().pluq_profile_enable(int(mask))


def pluq_profile_read():
    arr = (pluq_kernel_stat * len(KERNEL_CLASSES))()
    load().pluq_profile_read(arr)
    return {name: {"launches": arr[i].launches, "ms": arr[i].ms, "flops": arr[i].flops, "bytes": arr[i].bytes}
            for i, name in enumerate(KERNEL_CLASSES)}


def pluq_last_stats():
    a, b, c, d = (ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64())
    load().pluq_last_stats(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d))
    return {"nodes": a.value, "basecases": b.value, "launches": c.value, "syncs": d.value}


# ------------------------------------------------------------ convenience --

def pluq(A, p: int, form="fp64", validate=False, cutoff=0):
    """Decompose the device tensor A in place.  Returns (P, Q, r) with P, Q
    device int64 tensors."""
    import torch
    m, n = A.shape
    P = torch.empty(m, dtype=torch.int64, device=A.device)
    Q = torch.empty(n, dtype=torch.int64, device=A.device)
    r = pluq_modp(A, p, P, Q, _opts(form, validate, cutoff))
    return P, Q, r
