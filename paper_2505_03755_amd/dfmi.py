"""Python binding of libdfmi (ctypes over the C ABI in include/dfmi.h).

Argument marshalling only: torch tensors provide device memory and the current
stream; every contraction runs in the library's HIP kernels.  There is no
fallback path: if libdfmi.so is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfmi.so")

DF_OK = 0
DF_ERR_ARG = -1
DF_ERR_SHAPE = -2
DF_ERR_WORKSPACE = -3
DF_ERR_HIP = -4
DF_ERR_UNSUPPORTED = -5
STATUS_NAMES = {0: "DF_OK", -1: "DF_ERR_ARG", -2: "DF_ERR_SHAPE", -3: "DF_ERR_WORKSPACE",
                -4: "DF_ERR_HIP", -5: "DF_ERR_UNSUPPORTED"}

DF_OP_HALF_TRANSFORM = 1
DF_OP_JK = 2
DF_OP_ACTIVE_ERI = 3
DF_OP_PAPA = 4
DF_OP_STEP = 5
DF_OP_STEP_BACKWARD = 6
DF_OP_SPLIT_MATMUL = 7
DF_OP_STEP_SPLIT = 8
DF_OP_STEP_BACKWARD_SPLIT = 9
DF_OP_PPAA = 10
DF_OP_BUILD_CHOLESKY = 11
DF_OP_EMBED_CHOLESKY = 12

DF_PAPA_FULL = 0x1
DF_ACCUMULATE = 0x2
DF_PREC_SPLIT = 0x4
DF_CALLER_X = 0x10
DF_BWD_GJ = 0x20
DF_BWD_GK = 0x40
DF_BWD_GERI = 0x80
DF_SPLIT_K_FP64 = 0x100
DF_WEIGHTED = 0x200

KERNEL_KINDS = ["half_transform", "jvec", "coulomb", "k_syrk", "k_reduce", "mo_transform", "papa", "eri",
                "other", "adjoint", "split", "build"]

EXPORTED = ["df_create", "df_destroy", "df_last_error", "df_set_stream", "df_set_workspace",
            "df_set_timing", "df_timing_read", "df_workspace_size", "df_half_transform", "df_jk",
            "df_active_eri", "df_papa", "df_step", "df_step_backward", "df_split_matmul",
            "df_split_cholesky", "df_step_split", "df_batched_workspace_size", "df_batched_step",
            "df_set_autotune", "df_batched_tuning", "df_batched_set_tuning", "df_split_cholesky_t",
            "df_step_backward_split", "df_batched_split_workspace_size", "df_batched_step_split",
            "df_ppaa", "df_build_cholesky", "df_embed_cholesky", "df_workspace_query", "df_set_scratch_limit",
            "df_backward_chunk", "df_set_split_slices", "df_register_split", "df_jk_noalloc",
            "df_autotune_save", "df_autotune_load"]


class DFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [("naux", ctypes.c_int64), ("nao", ctypes.c_int64), ("ndm", ctypes.c_int64),
                ("nocc", ctypes.c_int64), ("nac", ctypes.c_int64), ("np", ctypes.c_int64),
                ("nq", ctypes.c_int64), ("ncol", ctypes.c_int64), ("n2", ctypes.c_int64),
                ("flags", ctypes.c_int), ("nslice", ctypes.c_int),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64)]


_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdfmi.so and declare its signatures (raises if it is not built)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built (run python -m paper_2505_03755_amd.build)")
        # torch brings its own HIP runtime (same soname as ROCm's).  Loading it first makes
        # libdfmi bind to that one runtime instead of pulling a second copy into the process.
        import torch  # noqa: F401
        L = ctypes.CDLL(path)
        vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.df_create.argtypes = [ctypes.POINTER(vp), i32, vp]
        L.df_destroy.argtypes = [vp]
        L.df_last_error.argtypes = [vp]
        L.df_last_error.restype = ctypes.c_char_p
        L.df_set_stream.argtypes = [vp, vp]
        L.df_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
        L.df_workspace_size.argtypes = [i32, ctypes.POINTER(Dims), ctypes.POINTER(ctypes.c_size_t)]
        L.df_workspace_query.argtypes = [vp, i32, ctypes.POINTER(Dims), ctypes.POINTER(ctypes.c_size_t)]
        L.df_set_scratch_limit.argtypes = [vp, ctypes.c_size_t]
        L.df_backward_chunk.argtypes = [vp, ctypes.POINTER(Dims), ctypes.POINTER(ctypes.c_int64)]
        L.df_set_split_slices.argtypes = [vp, i32]
        L.df_register_split.argtypes = [vp, dp, i64, i64, vp, vp, i32]
        L.df_set_timing.argtypes = [vp, i32]
        L.df_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32]
        L.df_half_transform.argtypes = [vp, dp, i64, i64, dp, i64, dp, dp, i64, dp, i32]
        L.df_jk.argtypes = [vp, dp, i64, i64, i64, dp, i64, dp, dp, dp, dp, i32]
        L.df_jk_noalloc.argtypes = [vp, dp, i64, i64, i64, dp, i64, dp, dp, dp, dp, i32]
        L.df_active_eri.argtypes = [vp, dp, i64, i64, dp, i64, dp, dp, i32]
        L.df_papa.argtypes = [vp, dp, i64, i64, dp, i64, dp, i64, dp, i64, dp, i32]
        L.df_ppaa.argtypes = [vp, dp, i64, i64, dp, i64, dp, i64, dp, i64, dp, i32]
        L.df_build_cholesky.argtypes = [vp, dp, dp, i64, i64, dp, dp, vp, i32]
        L.df_embed_cholesky.argtypes = [vp, dp, i64, i64, dp, i64, dp, i32]
        L.df_step.argtypes = [vp, dp, i64, i64, dp, i64, dp, dp, i64, dp, i64, dp, dp, dp, dp, dp, dp, dp, i32]
        L.df_step_backward.argtypes = [vp, dp, i64, i64, dp, i64, dp, i64, dp, dp, dp, dp, dp, dp, dp, i32]
        L.df_batched_workspace_size.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.df_batched_step.argtypes = [vp, vp, i32, i32]
        L.df_set_autotune.argtypes = [vp, i32]
        pi = ctypes.POINTER(ctypes.c_int)
        L.df_batched_tuning.argtypes = [vp, vp, i32, pi, pi, pi, pi]
        L.df_batched_set_tuning.argtypes = [vp, vp, i32, i32, i32, i32]
        L.df_autotune_save.argtypes = [vp, ctypes.c_char_p]
        L.df_autotune_load.argtypes = [vp, ctypes.c_char_p]
        L.df_batched_split_workspace_size.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.df_batched_step_split.argtypes = [vp, vp, vp, vp, i32, i32, i32]
        L.df_split_matmul.argtypes = [vp, dp, i64, i64, dp, i64, i64, i64, i32, dp, i64, i32]
        L.df_split_cholesky.argtypes = [vp, dp, i64, i64, i32, vp, vp, i32]
        L.df_step_split.argtypes = [vp, dp, vp, vp, i32, i64, i64, dp, i64, dp, i64, dp, i64,
                                    dp, dp, dp, dp, dp, dp, dp, i32]
        L.df_split_cholesky_t.argtypes = [vp, dp, i64, i64, i32, vp, vp, i32]
        L.df_step_backward_split.argtypes = [vp, dp, vp, vp, i32, i64, i64, dp, i64, dp, i64, dp, dp, dp, dp, dp,
                                             dp, dp, i32]
        for name in EXPORTED:
            if name != "df_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
        return L


def workspace_size(op: int, **dims) -> int:
    L = load_library()
    d = Dims(**{k: int(v) for k, v in dims.items()})
    out = ctypes.c_size_t(0)
    st = L.df_workspace_size(op, ctypes.byref(d), ctypes.byref(out))
    if st != DF_OK:
        raise DFError(st, "df_workspace_size")
    return out.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """One library context on one device; owns a growable workspace tensor."""

    def __init__(self, device=None):
        import torch
        L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("dfmi needs a GPU (torch.cuda is not available)")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        h = ctypes.c_void_p()
        st = L.df_create(ctypes.byref(h), self.device.index, None)
        if st != DF_OK:
            raise DFError(st, L.df_last_error(None).decode())
        self._h = h
        self._ws = None
        self._lib = L
        self.nslice = 7
        self._splits = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.df_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def check(self, st: int):
        if st != DF_OK:
            raise DFError(st, self._lib.df_last_error(self._h).decode())

    def bind_stream(self):
        """Make the library launch on torch's current stream of this device."""
        import torch
        stream = torch.cuda.current_stream(self.device)
        self.check(self._lib.df_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def workspace_query(self, op: int, **dims) -> int:
        """Workspace bytes of `op` for calls on this context (df_workspace_query: the context's
        scratch limit and split slice count apply)."""
        d = Dims(**{k: int(v) for k, v in dims.items()})
        out = ctypes.c_size_t(0)
        self.check(self._lib.df_workspace_query(self._h, op, ctypes.byref(d), ctypes.byref(out)))
        return out.value

    def set_scratch_limit(self, nbytes: int):
        """Bound df_step_backward's workspace (0: none); the adjoint then runs in P chunks."""
        self.check(self._lib.df_set_scratch_limit(self._h, int(nbytes)))

    def backward_chunk(self, **dims) -> int:
        """Auxiliary rows per chunk df_step_backward uses for these sizes (df_backward_chunk)."""
        d = Dims(**{k: int(v) for k, v in dims.items()})
        out = ctypes.c_int64(0)
        self.check(self._lib.df_backward_chunk(self._h, ctypes.byref(d), ctypes.byref(out)))
        return out.value

    def set_split_slices(self, nslice: int):
        """Slice count of the DF_PREC_SPLIT calls on this context."""
        self.check(self._lib.df_set_split_slices(self._h, int(nslice)))
        self.nslice = int(nslice)

    def register_split(self, B, nao: int, Bs, Be):
        """Register split_cholesky's planes of B for DF_PREC_SPLIT calls (nslice from Bs); Bs =
        None removes the registration of B for the context's slice count."""
        naux = _naux_of(B, nao)
        if Bs is None:
            self.check(self._lib.df_register_split(self._h, _ptr(B), naux, nao, None, None, self.nslice))
            self._splits.pop((B.data_ptr(), self.nslice), None)
            return
        nslice = Bs.shape[0]
        self.check(self._lib.df_register_split(self._h, _ptr(B), naux, nao, _ptr(Bs), _ptr(Be), nslice))
        self._splits[(B.data_ptr(), nslice)] = (Bs, Be)   # kept alive while registered

    def prepare(self, op: int, **dims):
        """Bind the current torch stream and a workspace big enough for `op`."""
        import torch
        self.bind_stream()
        need = self.workspace_query(op, **dims)
        if need and (self._ws is None or self._ws.numel() < need):
            self._ws = None
            self._ws = _aligned_empty((need,), torch.uint8, self.device)
        if self._ws is not None:
            self.check(self._lib.df_set_workspace(self._h, ctypes.c_void_p(self._ws.data_ptr()),
                                                  self._ws.numel()))

    def set_autotune(self, on: bool):
        """Tune df_batched_step's tiles on the first call of each new problem-group shape."""
        self.check(self._lib.df_set_autotune(self._h, 1 if on else 0))

    def autotune_save(self, path: str):
        """Write the context's tuning table to a file (df_autotune_save)."""
        self.check(self._lib.df_autotune_save(self._h, os.fsencode(path)))

    def autotune_load(self, path: str):
        """Merge a tuning file into the context's table (df_autotune_load)."""
        self.check(self._lib.df_autotune_load(self._h, os.fsencode(path)))

    def set_timing(self, on: bool):
        self.check(self._lib.df_set_timing(self._h, 1 if on else 0))

    def timing_read(self) -> dict:
        """{kernel kind: (milliseconds, launches)} since the last read (waits for the GPU)."""
        n = len(KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        self.check(self._lib.df_timing_read(self._h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}

    def release_workspace(self):
        self._ws = None
        self.check(self._lib.df_set_workspace(self._h, None, 0))


_contexts: dict = {}


def context(device=None) -> Context:
    import torch
    idx = torch.cuda.current_device() if device is None else (torch.device(device).index or 0)
    c = _contexts.get(idx)
    if c is None:
        c = Context(idx)
        _contexts[idx] = c
    return c


def _check_tensor(name, t, device, ndim=None):
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != device or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor on {device}")
    if ndim is not None and t.dim() not in ndim:
        raise ValueError(f"{name} has {t.dim()} dims, expected {ndim}")


def _npair(nao):
    return nao * (nao + 1) // 2


def _aligned_empty(shape, dtype, device, align: int = 4096):
    """An uninitialised tensor whose data starts on an `align`-byte boundary: a view into an
    allocation `align` bytes larger (torch's caching allocator promises 512 bytes only).  The int8
    planes of the split-precision calls are read in 1 KB blocks, fastest when none crosses a page."""
    import math
    import torch
    n = math.prod(shape)
    nbytes = n * torch.empty((), dtype=dtype).element_size()
    raw = torch.empty(nbytes + align, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % align
    return raw[off:off + nbytes].view(dtype).view(shape)


def _naux_of(B, nao):
    if B.dim() != 2 or B.shape[1] != _npair(nao):
        raise ValueError("B must be [naux, nao*(nao+1)/2]")
    return B.shape[0]


def _flags(accumulate: bool, split: bool) -> int:
    return (DF_ACCUMULATE if accumulate else 0) | (DF_PREC_SPLIT if split else 0)


def _out(name, t, shape, dev, accumulate):
    """The caller's output tensor (required with accumulate) or a new one."""
    import torch
    if t is None:
        if accumulate:
            raise ValueError(f"accumulate needs the output {name}")
        return torch.empty(shape, dtype=torch.float64, device=dev)
    _check_tensor(name, t, dev)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}")
    return t


def half_transform(B, nao: int, C, C2=None, out=None, accumulate=False, split=False, ctx: Context | None = None):
    """X[P] = b^P C (Eq. ao2mo_1); with C2 also Y[P] = C2^T X[P] (Eq. ao2mo_2).

    out: X, or (X, Y) with C2, to write into; accumulate adds to them (DF_ACCUMULATE).  split runs
    the products in split precision against the planes registered for B (DF_PREC_SPLIT)."""
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("C", C), ("C2", C2)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    ncol = C.shape[1]
    Xo, Yo = (out if C2 is not None else (out, None)) if out is not None else (None, None)
    X = _out("X", Xo, (naux, nao, ncol), ctx.device, accumulate)
    Y = None
    n2 = 0
    if C2 is not None:
        n2 = C2.shape[1]
        Y = _out("Y", Yo, (naux, n2, ncol), ctx.device, accumulate)
    fl = _flags(accumulate, split)
    ctx.prepare(DF_OP_HALF_TRANSFORM, naux=naux, nao=nao, ncol=ncol, n2=n2, flags=fl)
    ctx.check(ctx._lib.df_half_transform(ctx.handle, _ptr(B), naux, nao, _ptr(C), ncol, _ptr(X),
                                         _ptr(C2), n2, _ptr(Y), fl))
    return (X, Y) if C2 is not None else X


def jk(B, nao: int, Cocc, w=None, want_j=True, want_k=True, want_v=True, out=None, accumulate=False, split=False,
       ctx: Context | None = None):
    """JK call for D_k = C_k diag(w_k) C_k^T; Cocc is [nao, nocc] or [ndm, nao, nocc].

    out: dict with any of "J", "K" [ndm, nao, nao] and "v" [ndm, naux] to write into (accumulate
    adds to them); split: DF_PREC_SPLIT against the planes registered for B."""
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cocc", Cocc), ("w", w)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    single = Cocc.dim() == 2
    C3 = Cocc.unsqueeze(0) if single else Cocc
    ndm, nocc = C3.shape[0], C3.shape[2]
    if C3.shape[1] != nao:
        raise ValueError("Cocc rows must equal nao")
    if w is not None and w.numel() != ndm * nocc:
        raise ValueError("w must have ndm*nocc entries")
    o = out or {}
    dev = ctx.device
    J = _out("J", o.get("J"), (ndm, nao, nao), dev, accumulate) if want_j else None
    K = _out("K", o.get("K"), (ndm, nao, nao), dev, accumulate) if want_k else None
    v = _out("v", o.get("v"), (ndm, naux), dev, accumulate) if want_v else None
    fl = _flags(accumulate, split)
    ctx.prepare(DF_OP_JK, naux=naux, nao=nao, ndm=ndm, nocc=nocc,
                flags=fl | (DF_WEIGHTED if w is not None else 0))
    ctx.check(ctx._lib.df_jk(ctx.handle, _ptr(B), naux, nao, ndm, _ptr(C3), nocc, _ptr(w),
                             _ptr(J), _ptr(K), _ptr(v), fl))
    if single and out is None:
        J = J[0] if J is not None else None
        K = K[0] if K is not None else None
        v = v[0] if v is not None else None
    return J, K, v


def jk_noalloc(B, nao: int, Cocc, w=None, out=None, accumulate=False, ctx: Context | None = None):
    """df_jk_noalloc: the FP64 JK call on the library's static scratch (no workspace, no allocation in
    the library).  Cocc is [ndm, nao, nocc]; out: dict with any of "J", "K" [ndm, nao, nao] and
    "v" [ndm, naux], each written (or added to with accumulate); missing entries are not computed."""
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cocc", Cocc), ("w", w)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    if Cocc.dim() != 3 or Cocc.shape[1] != nao:
        raise ValueError("Cocc must be [ndm, nao, nocc]")
    ndm, nocc = Cocc.shape[0], Cocc.shape[2]
    o = out or {}
    J = _out("J", o["J"], (ndm, nao, nao), ctx.device, accumulate) if "J" in o else None
    K = _out("K", o["K"], (ndm, nao, nao), ctx.device, accumulate) if "K" in o else None
    v = _out("v", o["v"], (ndm, naux), ctx.device, accumulate) if "v" in o else None
    ctx.bind_stream()
    ctx.check(ctx._lib.df_jk_noalloc(ctx.handle, _ptr(B), naux, nao, ndm, _ptr(Cocc), nocc, _ptr(w),
                                     _ptr(J), _ptr(K), _ptr(v), DF_ACCUMULATE if accumulate else 0))
    return J, K, v


def active_eri(B, nao: int, Cact, return_buv=False, out=None, accumulate=False, split=False,
               ctx: Context | None = None):
    """(uv|wx) = sum_P b^P_uv b^P_wx with b^P_uv = (Cact^T b^P Cact)_uv.

    out: eri, or (eri, buv) with return_buv, to write into (accumulate adds to them); split:
    DF_PREC_SPLIT against the planes registered for B."""
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cact", Cact)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    nac = Cact.shape[1]
    eo, bo = (out if return_buv else (out, None)) if out is not None else (None, None)
    eri = _out("eri", eo, (nac,) * 4, ctx.device, accumulate)
    buv = _out("buv", bo, (naux, nac, nac), ctx.device, accumulate) if return_buv else None
    fl = _flags(accumulate, split)
    ctx.prepare(DF_OP_ACTIVE_ERI, naux=naux, nao=nao, nac=nac, flags=fl)
    ctx.check(ctx._lib.df_active_eri(ctx.handle, _ptr(B), naux, nao, _ptr(Cact), nac, _ptr(eri), _ptr(buv), fl))
    return (eri, buv) if return_buv else eri


def papa(B, nao: int, Cp, Cact, Cq=None, out=None, accumulate=False, split=False, ctx: Context | None = None):
    """(pu|vw) by default; with Cq the (pu|qv) block of Eq. (papa).  out / accumulate / split as in
    active_eri."""
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cp", Cp), ("Cact", Cact), ("Cq", Cq)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    np_, nac = Cp.shape[1], Cact.shape[1]
    flags, nq = 0, 0
    if Cq is not None:
        flags, nq = DF_PAPA_FULL, Cq.shape[1]
        shape = (np_, nac, nq, nac)
    else:
        shape = (np_, nac, nac, nac)
    res = _out("out", out, shape, ctx.device, accumulate)
    flags |= _flags(accumulate, split)
    ctx.prepare(DF_OP_PAPA, naux=naux, nao=nao, nac=nac, np=np_, nq=nq, flags=flags)
    ctx.check(ctx._lib.df_papa(ctx.handle, _ptr(B), naux, nao, _ptr(Cp), np_, _ptr(Cact), nac, _ptr(Cq), nq,
                               _ptr(res), flags))
    return res


def ppaa(B, nao: int, Cp, Cact, Cq=None, ctx: Context | None = None):
    """(pq|uv) of Eq. (ppaa) as [nac(nac+1)/2][np][nq], the (uv) index packed (u >= v); Cq
    defaults to Cp."""
    import torch
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cp", Cp), ("Cact", Cact), ("Cq", Cq)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    np_, nac = Cp.shape[1], Cact.shape[1]
    nq = Cq.shape[1] if Cq is not None else 0
    out = torch.empty((nac * (nac + 1) // 2, np_, nq if Cq is not None else np_), dtype=torch.float64,
                      device=ctx.device)
    ctx.prepare(DF_OP_PPAA, naux=naux, nao=nao, nac=nac, np=np_, nq=nq)
    ctx.check(ctx._lib.df_ppaa(ctx.handle, _ptr(B), naux, nao, _ptr(Cp), np_, _ptr(Cq), nq, _ptr(Cact), nac,
                               _ptr(out), 0))
    return out


def build_cholesky(metric, eri3, nao: int, in_place: bool = False, check: bool = True,
                   ctx: Context | None = None):
    """df_build_cholesky: (L, B, info) with (P|Q) = L L^T and B = L^-1 (Q|mu nu), Eq. (cholesky).
    in_place factors `metric` and overwrites `eri3` (returned as L and B).  info is a device int32
    (0, or P + 1 of the first pivot that is not positive); with check it is read (waiting for the
    stream) and a metric that is not positive definite raises."""
    import torch
    ctx = ctx or context(metric.device)
    _check_tensor("metric", metric, ctx.device, (2,))
    _check_tensor("eri3", eri3, ctx.device, (2,))
    naux = metric.shape[0]
    if tuple(metric.shape) != (naux, naux) or tuple(eri3.shape) != (naux, _npair(nao)):
        raise ValueError("metric must be [naux, naux] and eri3 [naux, nao(nao+1)/2]")
    Lt = metric if in_place else torch.empty_like(metric)
    Bt = eri3 if in_place else torch.empty_like(eri3)
    info = torch.empty(1, dtype=torch.int32, device=ctx.device)
    ctx.prepare(DF_OP_BUILD_CHOLESKY, naux=naux, nao=nao)
    ctx.check(ctx._lib.df_build_cholesky(ctx.handle, _ptr(metric), _ptr(eri3), naux, nao, _ptr(Lt), _ptr(Bt),
                                         ctypes.c_void_p(info.data_ptr()), 0))
    if check:
        bad = int(info.item())
        if bad:
            raise ValueError(f"the metric is not positive definite (pivot of auxiliary index {bad - 1})")
    return Lt, Bt, info


def embed_cholesky(B, nao: int, M, ctx: Context | None = None):
    """df_embed_cholesky: packed b^P in the basis of the columns of M [nao, nemb]."""
    import torch
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("M", M)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    nemb = M.shape[1]
    Be = torch.empty((naux, _npair(nemb)), dtype=torch.float64, device=ctx.device)
    ctx.prepare(DF_OP_EMBED_CHOLESKY, naux=naux, nao=nao, ncol=nemb)
    ctx.check(ctx._lib.df_embed_cholesky(ctx.handle, _ptr(B), naux, nao, _ptr(M), nemb, _ptr(Be), 0))
    return Be


def step(B, nao: int, Cocc, Cact, Cp, w=None, outputs=None, keep_x=False, ctx: Context | None = None):
    """J, K, v, (uv|wx) and (pu|vw) from one shared half transform (df_step).

    With keep_x the half-transformed factors are returned too, as "Xocc" [naux, nao, nocc]
    and "Xact" [nao, naux, nac] (what df_step_backward reuses)."""
    import torch
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cocc", Cocc), ("w", w), ("Cact", Cact), ("Cp", Cp)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    nocc, nac, np_ = Cocc.shape[1], Cact.shape[1], Cp.shape[1]
    dev = ctx.device
    if outputs is None:
        outputs = {
            "J": torch.empty((nao, nao), dtype=torch.float64, device=dev),
            "K": torch.empty((nao, nao), dtype=torch.float64, device=dev),
            "v": torch.empty((naux,), dtype=torch.float64, device=dev),
            "eri": torch.empty((nac,) * 4, dtype=torch.float64, device=dev),
            "papa": torch.empty((np_, nac, nac, nac), dtype=torch.float64, device=dev),
        }
    if keep_x:
        outputs.setdefault("Xocc", torch.empty((naux, nao, nocc), dtype=torch.float64, device=dev))
        outputs.setdefault("Xact", torch.empty((nao, naux, nac), dtype=torch.float64, device=dev))
    o = outputs
    for k in ("J", "K", "v", "eri", "papa", "Xocc", "Xact"):
        _check_tensor(k, o.get(k), dev)
    caller_x = o.get("Xocc") is not None
    ctx.prepare(DF_OP_STEP, naux=naux, nao=nao, ndm=1, nocc=nocc, nac=nac, np=np_,
                flags=DF_CALLER_X if caller_x else 0)
    ctx.check(ctx._lib.df_step(ctx.handle, _ptr(B), naux, nao, _ptr(Cocc), nocc, _ptr(w), _ptr(Cact), nac,
                               _ptr(Cp), np_, _ptr(o.get("J")), _ptr(o.get("K")), _ptr(o.get("v")),
                               _ptr(o.get("eri")), _ptr(o.get("papa")), _ptr(o.get("Xocc")), _ptr(o.get("Xact")), 0))
    return outputs


def step_backward(B, nao: int, Cocc, Cact, gJ=None, gK=None, geri=None, Xocc=None, Xact=None,
                  ctx: Context | None = None):
    """Vector-Jacobian product of (J, K, eri) w.r.t. (Cocc, Cact) (df_step_backward)."""
    import torch
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cocc", Cocc), ("Cact", Cact), ("gJ", gJ), ("gK", gK), ("geri", geri),
                 ("Xocc", Xocc), ("Xact", Xact)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    nocc, nac = Cocc.shape[1], Cact.shape[1]
    dCocc = torch.empty_like(Cocc)
    dCact = torch.empty_like(Cact)
    flags = ((DF_BWD_GJ if gJ is not None else 0) | (DF_BWD_GK if gK is not None else 0)
             | (DF_BWD_GERI if geri is not None else 0) | (DF_CALLER_X if Xocc is not None else 0))
    ctx.prepare(DF_OP_STEP_BACKWARD, naux=naux, nao=nao, ndm=1, nocc=nocc, nac=nac, flags=flags)
    ctx.check(ctx._lib.df_step_backward(ctx.handle, _ptr(B), naux, nao, _ptr(Cocc), nocc, _ptr(Cact), nac,
                                        _ptr(gJ), _ptr(gK), _ptr(geri), _ptr(Xocc), _ptr(Xact),
                                        _ptr(dCocc), _ptr(dCact), 0))
    return dCocc, dCact


class Problem(ctypes.Structure):
    _fields_ = [("B", ctypes.c_void_p), ("naux", ctypes.c_int64), ("nao", ctypes.c_int64),
                ("ndm", ctypes.c_int64), ("Cocc", ctypes.c_void_p), ("nocc", ctypes.c_int64),
                ("Cact", ctypes.c_void_p), ("nac", ctypes.c_int64), ("Cp", ctypes.c_void_p),
                ("np", ctypes.c_int64), ("J", ctypes.c_void_p), ("K", ctypes.c_void_p),
                ("eri", ctypes.c_void_p), ("papa", ctypes.c_void_p), ("ppaa", ctypes.c_void_p)]


def batched_step(problems, ppaa: bool = False, ctx: Context | None = None):
    """df_batched_step over a list of dicts {B, nao, Cocc [ndm, nao, nocc], Cact, Cp}; returns one
    dict of outputs per problem: J, K [ndm, nao, nao], eri [nac]^4, papa (pu|qv) [np, nac, np, nac],
    and with ppaa also (pq|uv) [nac(nac+1)/2, np, np]."""
    import torch
    if not problems:
        return []
    dev = problems[0]["B"].device
    ctx = ctx or context(dev)
    arr = (Problem * len(problems))()
    outs = []
    for i, pr in enumerate(problems):
        B, nao, Co, Ca, Cp = pr["B"], pr["nao"], pr["Cocc"], pr["Cact"], pr["Cp"]
        for n, t in (("B", B), ("Cocc", Co), ("Cact", Ca), ("Cp", Cp)):
            _check_tensor(n, t, ctx.device)
        naux = _naux_of(B, nao)
        ndm, nocc = Co.shape[0], Co.shape[2]
        nac, np_ = Ca.shape[1], Cp.shape[1]
        o = {"J": torch.empty((ndm, nao, nao), dtype=torch.float64, device=dev),
             "K": torch.empty((ndm, nao, nao), dtype=torch.float64, device=dev),
             "eri": torch.empty((nac,) * 4, dtype=torch.float64, device=dev),
             "papa": torch.empty((np_, nac, np_, nac), dtype=torch.float64, device=dev)}
        if ppaa:
            o["ppaa"] = torch.empty((nac * (nac + 1) // 2, np_, np_), dtype=torch.float64, device=dev)
        outs.append(o)
        arr[i] = Problem(_ptr(B), naux, nao, ndm, _ptr(Co), nocc, _ptr(Ca), nac, _ptr(Cp), np_,
                         _ptr(o["J"]), _ptr(o["K"]), _ptr(o["eri"]), _ptr(o["papa"]), _ptr(o.get("ppaa")))
    L = ctx._lib
    need = ctypes.c_size_t(0)
    ctx.check(L.df_batched_workspace_size(arr, len(problems), ctypes.byref(need)))
    ctx.bind_stream()
    if need.value and (ctx._ws is None or ctx._ws.numel() < need.value):
        ctx._ws = None
        ctx._ws = _aligned_empty((need.value,), torch.uint8, ctx.device)
    if ctx._ws is not None:
        ctx.check(L.df_set_workspace(ctx._h, ctypes.c_void_p(ctx._ws.data_ptr()), ctx._ws.numel()))
    ctx.check(L.df_batched_step(ctx.handle, arr, len(problems), 0))
    return outs


def batched_step_split(problems, nslice: int = 7, k_fp64: bool = False, ppaa: bool = False,
                       ctx: Context | None = None):
    """df_batched_step_split: as batched_step, in split precision; each problem dict also carries
    "Bs", "Be" from split_cholesky(B, nao, nslice).  k_fp64 computes K in FP64 from the
    split-precision X_occ (DF_SPLIT_K_FP64); (pq|uv) (with ppaa) is FP64."""
    import torch
    if not problems:
        return []
    dev = problems[0]["B"].device
    ctx = ctx or context(dev)
    arr = (Problem * len(problems))()
    bs = (ctypes.c_void_p * len(problems))()
    be = (ctypes.c_void_p * len(problems))()
    outs = []
    for i, pr in enumerate(problems):
        B, nao, Co, Ca, Cp = pr["B"], pr["nao"], pr["Cocc"], pr["Cact"], pr["Cp"]
        for n, t in (("B", B), ("Cocc", Co), ("Cact", Ca), ("Cp", Cp)):
            _check_tensor(n, t, ctx.device)
        naux = _naux_of(B, nao)
        Bs, Be = pr["Bs"], pr["Be"]
        if (Bs.dtype != torch.int8 or Be.dtype != torch.int32
                or tuple(Bs.shape) != split_plane_shape(naux * nao, nao, nslice) or tuple(Be.shape) != (naux * nao,)
                or not Bs.is_contiguous() or not Be.is_contiguous()):
            raise ValueError(f"problem {i}: Bs, Be must come from split_cholesky(B, nao, {nslice})")
        ndm, nocc = Co.shape[0], Co.shape[2]
        nac, np_ = Ca.shape[1], Cp.shape[1]
        o = {"J": torch.empty((ndm, nao, nao), dtype=torch.float64, device=dev),
             "K": torch.empty((ndm, nao, nao), dtype=torch.float64, device=dev),
             "eri": torch.empty((nac,) * 4, dtype=torch.float64, device=dev),
             "papa": torch.empty((np_, nac, np_, nac), dtype=torch.float64, device=dev)}
        if ppaa:
            o["ppaa"] = torch.empty((nac * (nac + 1) // 2, np_, np_), dtype=torch.float64, device=dev)
        outs.append(o)
        arr[i] = Problem(_ptr(B), naux, nao, ndm, _ptr(Co), nocc, _ptr(Ca), nac, _ptr(Cp), np_,
                         _ptr(o["J"]), _ptr(o["K"]), _ptr(o["eri"]), _ptr(o["papa"]), _ptr(o.get("ppaa")))
        bs[i], be[i] = Bs.data_ptr(), Be.data_ptr()
    L = ctx._lib
    need = ctypes.c_size_t(0)
    flags = DF_SPLIT_K_FP64 if k_fp64 else 0
    ctx.check(L.df_batched_split_workspace_size(arr, len(problems), nslice, flags, ctypes.byref(need)))
    ctx.bind_stream()
    if need.value and (ctx._ws is None or ctx._ws.numel() < need.value):
        ctx._ws = None
        ctx._ws = _aligned_empty((need.value,), torch.uint8, ctx.device)
    if ctx._ws is not None:
        ctx.check(L.df_set_workspace(ctx._h, ctypes.c_void_p(ctx._ws.data_ptr()), ctx._ws.numel()))
    ctx.check(L.df_batched_step_split(ctx.handle, arr, bs, be, len(problems), nslice, flags))
    return outs


def _shape_array(problems):
    """df_problem array carrying the sizes of `problems` and placeholder (never dereferenced)
    output pointers: what the tuning calls read is the sizes and which outputs are requested."""
    arr = (Problem * len(problems))()
    one = 1
    for i, pr in enumerate(problems):
        nao = pr["nao"]
        naux = _naux_of(pr["B"], nao)
        Co, Ca, Cp = pr["Cocc"], pr["Cact"], pr["Cp"]
        arr[i] = Problem(one, naux, nao, Co.shape[0], one, Co.shape[2], one, Ca.shape[1], one, Cp.shape[1],
                         one, one, one, one)
    return arr


def batched_tuning(problems, ctx: Context | None = None) -> dict:
    """Configuration df_batched_step uses for this group's shape (df_batched_tuning)."""
    ctx = ctx or context(problems[0]["B"].device)
    arr = _shape_array(problems)
    v = [ctypes.c_int(0) for _ in range(4)]
    ctx.check(ctx._lib.df_batched_tuning(ctx.handle, arr, len(problems), *[ctypes.byref(x) for x in v]))
    return {"half_tile_n": v[0].value, "k_tile": v[1].value, "k_rounds": v[2].value, "tuned": bool(v[3].value)}


def batched_set_tuning(problems, half_tile_n: int, k_tile: int, k_rounds: int, ctx: Context | None = None):
    """Store a configuration for this group's shape (df_batched_set_tuning)."""
    ctx = ctx or context(problems[0]["B"].device)
    arr = _shape_array(problems)
    ctx.check(ctx._lib.df_batched_set_tuning(ctx.handle, arr, len(problems), half_tile_n, k_tile, k_rounds))


def dev_of(ctx):
    return ctx.device


def kpad64(n: int) -> int:
    return (n + 63) // 64 * 64


def rpad32(n: int) -> int:
    return (n + 31) // 32 * 32


def split_plane_shape(rows: int, K: int, nslice: int):
    """Shape of the int8 planes of `rows` rows of length K: [nslice][row group][k block][1024],
    1 KB blocks of 32 rows x 32 k whose 16-byte slot rr + 32 c holds k = 32 b + 16 c + [0, 16) of
    row 32 g + rr (zeros past `rows` and past K)."""
    return (nslice, rpad32(rows) // 32, kpad64(K) // 32, 1024)


def split_matmul(A, B, nslice: int = 7, ctx: Context | None = None):
    """C = A B^T by the int8 slice method (df_split_matmul); A [M, K], B [N, K] FP64 on the GPU."""
    import torch
    ctx = ctx or context(A.device)
    for n, t in (("A", A), ("B", B)):
        _check_tensor(n, t, ctx.device)
    M, K = A.shape
    N = B.shape[0]
    if B.shape[1] != K:
        raise ValueError("A and B need the same number of columns")
    C = torch.empty((M, N), dtype=torch.float64, device=ctx.device)
    ctx.prepare(DF_OP_SPLIT_MATMUL, m=M, n=N, k=K, nslice=nslice)
    ctx.check(ctx._lib.df_split_matmul(ctx.handle, _ptr(A), K, M, _ptr(B), K, N, K, nslice, _ptr(C), N, 0))
    return C


def split_cholesky(B, nao: int, nslice: int = 7, ctx: Context | None = None):
    """int8 planes (split_plane_shape(naux*nao, nao, nslice)) and exponents [naux*nao] of the
    unpacked b^P rows."""
    import torch
    ctx = ctx or context(B.device)
    _check_tensor("B", B, ctx.device)
    naux = _naux_of(B, nao)
    Bs = _aligned_empty(split_plane_shape(naux * nao, nao, nslice), torch.int8, ctx.device)
    Be = torch.empty((naux * nao,), dtype=torch.int32, device=ctx.device)
    ctx.bind_stream()
    ctx.check(ctx._lib.df_split_cholesky(ctx.handle, _ptr(B), naux, nao, nslice, _ptr(Bs), _ptr(Be), 0))
    return Bs, Be


def step_split(B, Bs, Be, nao: int, Cocc, Cact, Cp, outputs=None, keep_x=False, ctx: Context | None = None):
    """df_step in split precision (df_step_split); nslice is taken from Bs.  With keep_x the
    half-transformed factors are returned too, as "Xocc" [naux, nao, nocc] and "Xact"
    [nao, naux, nac] (what df_step_backward_split takes)."""
    import torch
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cocc", Cocc), ("Cact", Cact), ("Cp", Cp)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    nslice = Bs.shape[0]
    if (Bs.dtype != torch.int8 or Be.dtype != torch.int32 or tuple(Bs.shape) != split_plane_shape(naux * nao, nao, nslice)
            or tuple(Be.shape) != (naux * nao,) or Bs.device != dev_of(ctx) or Be.device != dev_of(ctx)
            or not Bs.is_contiguous() or not Be.is_contiguous()):
        raise ValueError("Bs, Be must come from split_cholesky(B, nao) on the same device")
    nocc, nac, np_ = Cocc.shape[1], Cact.shape[1], Cp.shape[1]
    dev = ctx.device
    if outputs is None:
        outputs = {
            "J": torch.empty((nao, nao), dtype=torch.float64, device=dev),
            "K": torch.empty((nao, nao), dtype=torch.float64, device=dev),
            "v": torch.empty((naux,), dtype=torch.float64, device=dev),
            "eri": torch.empty((nac,) * 4, dtype=torch.float64, device=dev),
            "papa": torch.empty((np_, nac, nac, nac), dtype=torch.float64, device=dev),
        }
    if keep_x:
        outputs.setdefault("Xocc", torch.empty((naux, nao, nocc), dtype=torch.float64, device=dev))
        outputs.setdefault("Xact", torch.empty((nao, naux, nac), dtype=torch.float64, device=dev))
    o = outputs
    for k in ("J", "K", "v", "eri", "papa", "Xocc", "Xact"):
        _check_tensor(k, o.get(k), dev)
    caller_x = o.get("Xocc") is not None
    ctx.prepare(DF_OP_STEP_SPLIT, naux=naux, nao=nao, ndm=1, nocc=nocc, nac=nac, np=np_, nslice=nslice,
                flags=DF_CALLER_X if caller_x else 0)
    ctx.check(ctx._lib.df_step_split(ctx.handle, _ptr(B), _ptr(Bs), _ptr(Be), nslice, naux, nao, _ptr(Cocc), nocc,
                                     _ptr(Cact), nac, _ptr(Cp), np_, _ptr(o.get("J")), _ptr(o.get("K")),
                                     _ptr(o.get("v")), _ptr(o.get("eri")), _ptr(o.get("papa")),
                                     _ptr(o.get("Xocc")), _ptr(o.get("Xact")), 0))
    return outputs


def split_cholesky_t(B, nao: int, nslice: int = 7, ctx: Context | None = None):
    """int8 planes (split_plane_shape(nao, naux*nao, nslice)) and exponents [nao] of the rows mu of
    the DF tensor over k = P*nao + nu (df_split_cholesky_t)."""
    import torch
    ctx = ctx or context(B.device)
    _check_tensor("B", B, ctx.device)
    naux = _naux_of(B, nao)
    Bt = _aligned_empty(split_plane_shape(nao, naux * nao, nslice), torch.int8, ctx.device)
    Bte = torch.empty((nao,), dtype=torch.int32, device=ctx.device)
    ctx.bind_stream()
    ctx.check(ctx._lib.df_split_cholesky_t(ctx.handle, _ptr(B), naux, nao, nslice, _ptr(Bt), _ptr(Bte), 0))
    return Bt, Bte


def step_backward_split(B, Bt, Bte, nao: int, Cocc, Cact, gJ=None, gK=None, geri=None, Xocc=None, Xact=None,
                        ctx: Context | None = None):
    """step_backward with the exchange part as slice products (df_step_backward_split); nslice is
    taken from Bt.  Xocc and Xact come from step_split(..., keep_x=True) or step(..., keep_x=True)."""
    import torch
    ctx = ctx or context(B.device)
    for n, t in (("B", B), ("Cocc", Cocc), ("Cact", Cact), ("gJ", gJ), ("gK", gK), ("geri", geri),
                 ("Xocc", Xocc), ("Xact", Xact)):
        _check_tensor(n, t, ctx.device)
    naux = _naux_of(B, nao)
    nslice = Bt.shape[0]
    if (Bt.dtype != torch.int8 or Bte.dtype != torch.int32 or tuple(Bt.shape) != split_plane_shape(nao, naux * nao, nslice)
            or tuple(Bte.shape) != (nao,) or not Bt.is_contiguous() or not Bte.is_contiguous()):
        raise ValueError("Bt, Bte must come from split_cholesky_t(B, nao)")
    nocc, nac = Cocc.shape[1], Cact.shape[1]
    dCocc = torch.empty_like(Cocc)
    dCact = torch.empty_like(Cact)
    flags = ((DF_BWD_GJ if gJ is not None else 0) | (DF_BWD_GK if gK is not None else 0)
             | (DF_BWD_GERI if geri is not None else 0))
    ctx.prepare(DF_OP_STEP_BACKWARD_SPLIT, naux=naux, nao=nao, ndm=1, nocc=nocc, nac=nac, nslice=nslice, flags=flags)
    ctx.check(ctx._lib.df_step_backward_split(ctx.handle, _ptr(B), _ptr(Bt), _ptr(Bte), nslice, naux, nao,
                                              _ptr(Cocc), nocc, _ptr(Cact), nac, _ptr(gJ), _ptr(gK), _ptr(geri),
                                              _ptr(Xocc), _ptr(Xact), _ptr(dCocc), _ptr(dCact), 0))
    return dCocc, dCact


def _autograd_function():
    import torch

    class DFStep(torch.autograd.Function):
        """(J, K, eri) = DFStep.apply(B, nao, Cocc, Cact, keep_x): differentiable in Cocc and Cact.

        The forward keeps the half-transformed factors for the backward when keep_x is set
        (13.8 GB + 1.8 GB at paper scale); otherwise the backward recomputes them."""

        @staticmethod
        def forward(fctx, B, nao, Cocc, Cact, keep_x=True):
            Cocc = Cocc.contiguous()
            Cact = Cact.contiguous()
            Cp = Cact[:, :0]   # no (pu|vw) needed here
            out = step(B, nao, Cocc, Cact, Cp.contiguous(), keep_x=keep_x)
            fctx.nao = nao
            fctx.save_for_backward(B, Cocc, Cact)
            fctx.xs = (out.get("Xocc"), out.get("Xact"))
            return out["J"], out["K"], out["eri"]

        @staticmethod
        def backward(fctx, gJ, gK, geri):
            B, Cocc, Cact = fctx.saved_tensors
            c = lambda g: None if g is None else g.contiguous()
            Xo, Xa = fctx.xs
            dCocc, dCact = step_backward(B, fctx.nao, Cocc, Cact, c(gJ), c(gK), c(geri), Xo, Xa)
            fctx.xs = None
            return None, None, dCocc, dCact, None

    return DFStep


_DFStep = None
_RotationExp = None


def _rotation_exp_function():
    import torch

    class RotationExp(torch.autograd.Function):
        """U = exp(R), differentiable.  The backward is the adjoint of the Frechet derivative,
        L_exp(R^T, G) = the upper-right block of exp([[R^T, G], [0, R^T]]).  The cotangent G is
        scaled to a unit largest entry first (the derivative is linear in it), so that the block
        matrix's norm, and with it the number of squarings, is R's own; torch's own backward of
        matrix_exp takes G as it comes, and a G of norm 1e4 costs it several digits."""

        @staticmethod
        def forward(fctx, R):
            fctx.save_for_backward(R)
            return torch.linalg.matrix_exp(R)

        @staticmethod
        def backward(fctx, G):
            (R,) = fctx.saved_tensors
            n = R.shape[-1]
            s = G.abs().max()
            if s == 0:
                return torch.zeros_like(R)
            M = R.new_zeros((2 * n, 2 * n))
            M[:n, :n] = R.T
            M[n:, n:] = R.T
            M[:n, n:] = G / s
            return torch.linalg.matrix_exp(M)[:n, n:] * s

    return RotationExp


def rotation_exp(R):
    """exp(R) for a square R, with an accurate adjoint for autograd (see RotationExp)."""
    global _RotationExp
    if _RotationExp is None:
        _RotationExp = _rotation_exp_function()
    return _RotationExp.apply(R)


def dfstep_apply(B, nao: int, Cocc, Cact, keep_x=True):
    """(J, K, eri) with autograd support through the library's hand-written adjoint."""
    global _DFStep
    if _DFStep is None:
        _DFStep = _autograd_function()
    return _DFStep.apply(B, nao, Cocc, Cact, keep_x)


def energy(B, nao: int, C0, kappa, nocc: int, nac: int, h, Gamma, keep_x=True):
    """E(kappa) = tr(D h) + 1/2 tr(D J) - 1/4 tr(D K) + 1/2 sum (uv|wx) Gamma, C = C0 exp(kappa - kappa^T).

    Differentiable in kappa: the matrix exponential (rotation_exp) supplies dC/dkappa, the
    library's adjoint supplies the contraction part."""
    C = C0 @ rotation_exp(kappa - kappa.T)
    Cocc = C[:, :nocc]
    Cact = C[:, nocc:nocc + nac]
    J, K, eri = dfstep_apply(B, nao, Cocc, Cact, keep_x)
    D = Cocc @ Cocc.T
    return (D * h).sum() + 0.5 * (D * J).sum() - 0.25 * (D * K).sum() + 0.5 * (eri * Gamma).sum()
