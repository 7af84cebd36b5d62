"""m-double matrix product by error-free summation on the MI355X.

Thin Python binding of ``libmdgemm.so`` (C ABI in ``include/mdgemm.h``):
argument marshalling only; every step of the product runs in the library's
HIP kernels.  Torch supplies device memory and the current stream.

An m-double matrix is a float64 tensor of shape (m, rows, cols) on the HIP
device, one plane per word (word 0 the leading one).

    C = gemm(A, B, form="int8")          # (m, M, K) x (m, K, N) -> (m, M, N)
    C = gemm(A, B, form="int8bal")       # balanced 8-bit INT8 digits
    C = MDGemm.apply(A, B, "fp64")       # differentiable; C.backward(W)

The backward pass of ``MDGemm`` takes dC as m-double planes and returns the
m-double gradients dA = dC B^T and dB = A^T dC through the same error-free
product (the adjoint of a matrix product).  Torch sees the planes as
independent floats, so call ``C.backward(gradient=W)`` with W in m-double
planes rather than a plane-wise torch loss.

Exact integers before the rounding, and a product cut along its depth:

    E, F = exponents(A, B)                           # the full matrices' grids
    X1, sc, _ = gemm_fixed(A[:, :, :k], B[:, :k], E, F, S=27, beta=8, form="int8bal",
                           nlimb=fixed_limbs(8, 27, K))
    X2, _, _ = gemm_fixed(A[:, :, k:], B[:, k:], E, F, S=27, beta=8, form="int8bal",
                          nlimb=fixed_limbs(8, 27, K))
    C = fixed_round(fixed_add(X1, X2), sc, m)       # = gemm_ex(A, B, ..., force_S=27)

Other entry points: ``gemm_ex`` and ``dot_ex`` (options, events, validation),
``dot`` (batched inner products), ``gemm_ordinary`` (the classical m-double
baseline), ``choose_params``.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdgemm.so")

FORM_FP64 = 0
FORM_INT8 = 1
FORM_INT8_BAL = 2
_FORMS = {"fp64": FORM_FP64, "int8": FORM_INT8, "int8bal": FORM_INT8_BAL}
_RULES = {"rho": 0, "span": 1}

ERRORS = {
    0: "MD_OK", 1: "MD_EINVAL_M", 2: "MD_EINVAL_DIM", 3: "MD_ENULL", 4: "MD_EALIAS",
    5: "MD_ENOMEM", 6: "MD_EHIP", 7: "MD_EINVAL_OPT", 8: "MD_ERANGE", 9: "MD_EINPUT",
}


class MDInfo(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int), ("beta", ctypes.c_int), ("kc", ctypes.c_int),
                ("band", ctypes.c_int), ("span_A", ctypes.c_int), ("span_B", ctypes.c_int),
                ("G", ctypes.c_int), ("G_span", ctypes.c_int), ("G_rho", ctypes.c_int),
                ("target_bits", ctypes.c_int), ("log2_bound", ctypes.c_double),
                ("input_flags", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MDDebug(ctypes.Structure):
    _fields_ = [("E", ctypes.c_void_p), ("F", ctypes.c_void_p), ("digits_A", ctypes.c_void_p),
                ("digits_B", ctypes.c_void_p), ("D", ctypes.c_void_p)]


class MDCert(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_int32), ("S_min", ctypes.c_int32), ("S", ctypes.c_int32),
                ("G", ctypes.c_int32), ("G_span", ctypes.c_int32), ("G_rho", ctypes.c_int32),
                ("log2_bound", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


CERT_SMALL = 1   # the hinted S is below the rule's: 2^-T not certified
CERT_RANGE = 2   # a product may leave the double range: no bound


class MDOpts(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("s_rule", ctypes.c_int), ("target_bits", ctypes.c_int),
                ("force_S", ctypes.c_int), ("force_beta", ctypes.c_int),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("dbg", ctypes.POINTER(MDDebug)), ("info", ctypes.POINTER(MDInfo)),
                ("ev_gemm_begin", ctypes.c_void_p), ("ev_gemm_end", ctypes.c_void_p),
                ("validate", ctypes.c_int), ("exp_flags", ctypes.c_void_p),
                ("s_hint", ctypes.c_int), ("cert", ctypes.c_void_p)]


class MDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2606_20863_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    L.md_gemm.argtypes = [i32, i64, i64, i64, p, p, p, p]
    L.md_gemm.restype = i32
    L.md_gemm_ex.argtypes = [i32, i32, i32, i64, i64, i64, p, i64, i64, p, i64, i64, p, i64, i64,
                             ctypes.POINTER(MDOpts), p]
    L.md_gemm_ex.restype = i32
    L.md_gemm_ex_noalloc.argtypes = L.md_gemm_ex.argtypes
    L.md_gemm_ex_noalloc.restype = i32
    L.md_dot_ex.argtypes = [i32, i64, i64, p, i64, i64, p, i64, i64, p, i64, ctypes.POINTER(MDOpts), p]
    L.md_dot_ex.restype = i32
    L.md_dot.argtypes = [i32, i64, i64, p, p, p, p]
    L.md_dot.restype = i32
    L.md_gemm_ordinary.argtypes = [i32, i64, i64, i64, p, p, p, p]
    L.md_gemm_ordinary.restype = i32
    L.md_dot_ordinary.argtypes = [i32, i64, i64, p, p, p, p]
    L.md_dot_ordinary.restype = i32
    L.md_choose_params.argtypes = [i32, i64, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.md_choose_params.restype = i32
    L.md_gemm_workspace_size.argtypes = [i32, i64, i64, i64, i32]
    L.md_gemm_workspace_size.restype = ctypes.c_size_t
    L.md_workspace_size.argtypes = [i32, i64, i64, i64, i32]
    L.md_workspace_size.restype = ctypes.c_size_t
    L.md_dot_workspace_size.argtypes = [i32, i64, i64, i32]
    L.md_dot_workspace_size.restype = ctypes.c_size_t
    L.md_fixed_limbs.argtypes = [i32, i32, i64]
    L.md_fixed_limbs.restype = i32
    L.md_exponents.argtypes = [i64, i64, i64, p, i64, p, i64, p, p, p]
    L.md_exponents.restype = i32
    L.md_gemm_fixed.argtypes = [i32, i64, i64, i64, p, i64, i64, p, i64, i64, p, p, p, i32, p,
                                ctypes.POINTER(MDOpts), p]
    L.md_gemm_fixed.restype = i32
    L.md_fixed_add.argtypes = [i64, i32, p, p, p, p]
    L.md_fixed_add.restype = i32
    L.md_fixed_round.argtypes = [i32, i64, i32, p, p, p, i64, p]
    L.md_fixed_round.restype = i32
    L.md_strerror.argtypes = [i32]
    L.md_strerror.restype = ctypes.c_char_p
    L.md_last_hip_error.restype = i32
    L.md_version.restype = i32
    _lib = L
    return L


def _check(rc: int, info: "MDInfo | None" = None):
    if rc != 0:
        L = lib()
        msg = L.md_strerror(rc).decode()
        if rc == 6:
            msg += f" (hipError {L.md_last_hip_error()})"
        err = MDError(rc, msg)
        if info is not None and rc == 9:
            err.input_flags = info.input_flags
            err.args = (f"{msg} (flags {info.input_flags})",)
        raise err


def choose_params(form: str, K: int, T: int, G: int):
    """(beta, S, kc, band) the library's slice rule picks (host only)."""
    b, s, k, bd = (ctypes.c_int() for _ in range(4))
    _check(lib().md_choose_params(_FORMS[form], K, T, G, ctypes.byref(b), ctypes.byref(s),
                                  ctypes.byref(k), ctypes.byref(bd)))
    return b.value, s.value, k.value, bd.value


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _check_planes(X: torch.Tensor, name: str):
    if X.dtype != torch.float64 or X.dim() != 3 or not X.is_cuda:
        raise ValueError(f"{name} must be a float64 (m, rows, cols) tensor on the HIP device")


def _device_buffer(t: torch.Tensor, name: str, device, nbytes: int = 1):
    """Pointer and size of a caller's device buffer: contiguous, on the
    operands' device, at least nbytes long (checked before any call, so no
    host pointer reaches a kernel)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous tensor on {device}")
    size = t.numel() * t.element_size()
    if size < nbytes:
        raise ValueError(f"{name} holds {size} bytes, {nbytes} needed")
    return ctypes.c_void_p(t.data_ptr()), size


def new_cert(device=None) -> torch.Tensor:
    """A device buffer for one md_cert record (see ``read_cert``)."""
    return torch.zeros(ctypes.sizeof(MDCert), dtype=torch.uint8, device=device or "cuda")


def read_cert(cert: torch.Tensor) -> dict:
    """The md_cert record a hinted call wrote (synchronises with the copy)."""
    raw = bytes(cert[:ctypes.sizeof(MDCert)].cpu().numpy().tobytes())
    return MDCert.from_buffer_copy(raw).as_dict()


# S of the last call per shape and options (keys below), for sizing the
# scratch of the next one before the slice rule has run
_S_SEEN: dict = {}


def _auto_workspace(key, size_of_S, S, device, stream):
    """Scratch for a call from torch's caching allocator: with it the library
    allocates nothing and a call only queues kernels (its own pool's
    stream-ordered allocation and release put work on the GPU's queue in
    every call, 10-70 us of it measured per call).  Sized for S, else for
    the S this shape and these options took last time; None when neither is
    known (the library's pool serves that call)."""
    if S <= 0:
        S = _S_SEEN.get(key, 0)
    if S <= 0:
        return None
    ws = torch.empty(int(size_of_S(S)), dtype=torch.uint8, device=device)
    if stream is not None:
        ws.record_stream(stream)
    return ws


def _run_with_scratch(call, opts: "MDOpts", ws, key, info: "MDInfo"):
    """call() with ws as the workspace; a call whose slice rule chose a larger
    S than ws holds stops with MD_ENOMEM before it writes any output, and
    runs again on the library's pool.  Records the S taken under key."""
    if ws is not None:
        opts.workspace, opts.workspace_bytes = ctypes.c_void_p(ws.data_ptr()), ws.numel()
    rc = call()
    if rc == 5 and ws is not None:
        opts.workspace, opts.workspace_bytes = None, 0
        rc = call()
    _check(rc, info)
    if key is not None:
        if len(_S_SEEN) >= 4096 and key not in _S_SEEN:
            _S_SEEN.clear()   # bounded: a process that meets many shapes starts over
        _S_SEEN[key] = info.S
    return rc


def _slice_opts(opts: "MDOpts", device, force_S, force_beta, s_hint, cert, workspace):
    opts.force_S = force_S
    opts.force_beta = force_beta
    opts.s_hint = s_hint
    if s_hint:
        if cert is None:
            raise ValueError("s_hint needs a cert buffer (new_cert())")
        opts.cert, _ = _device_buffer(cert, "cert", device, ctypes.sizeof(MDCert))
    if workspace is not None:
        opts.workspace, opts.workspace_bytes = _device_buffer(workspace, "workspace", device)


def gemm_ex(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None, *, transA=False,
            transB=False, form="fp64", rule="rho", target_bits=0, force_S=0, force_beta=0,
            debug=None, workspace: torch.Tensor | None = None, events=None, stream=None,
            validate=False, s_hint=0, cert: torch.Tensor | None = None, noalloc=False, pool=False):
    """C = op(A) op(B) in m-double arithmetic.

    A is (m, M, K) (or (m, K, M) with transA), B is (m, K, N) (or (m, N, K)
    with transB); both contiguous per plane.  Returns (C, info dict).
    ``debug`` may be a dict of preallocated device tensors with keys E, F,
    digits_A, digits_B, D (see ``md_debug``).  ``events`` may be a pair of
    raw hipEvent_t handles recorded around the slice contraction.
    ``validate``: check the input preconditions first (MDError MD_EINPUT,
    C untouched, when an entry breaks them).  ``s_hint`` (with ``cert``, a
    ``new_cert()`` buffer): run on that S without waiting for the rule; the
    device writes the data's certificate into ``cert`` (``read_cert``).
    ``workspace``: a contiguous device buffer of at least
    ``md_gemm_workspace_size`` bytes (the call then allocates nothing).
    ``noalloc``: call md_gemm_ex_noalloc (the library's own fixed scratch
    array, no workspace; C must then be given to allocate nothing at all).
    Without a workspace the scratch comes from torch's caching allocator
    (``_auto_workspace``); ``pool=True`` leaves it to the library's pool.
    """
    _check_planes(A, "A")
    _check_planes(B, "B")
    A = A.contiguous()
    B = B.contiguous()
    m = A.shape[0]
    if B.shape[0] != m:
        raise ValueError("A and B have different word counts")
    M, K = (A.shape[2], A.shape[1]) if transA else (A.shape[1], A.shape[2])
    Kb, N = (B.shape[2], B.shape[1]) if transB else (B.shape[1], B.shape[2])
    if Kb != K:
        raise ValueError(f"inner sizes differ: {K} vs {Kb}")
    if C is None:
        C = torch.empty((m, M, N), dtype=torch.float64, device=A.device)
    elif C.shape != (m, M, N) or not C.is_contiguous() or C.dtype != torch.float64:
        raise ValueError("C must be a contiguous float64 (m, M, N) tensor")
    info = MDInfo()
    opts = MDOpts()
    opts.form = _FORMS[form]
    opts.s_rule = _RULES[rule]
    opts.target_bits = target_bits
    opts.validate = 1 if validate else 0
    opts.info = ctypes.pointer(info)
    _slice_opts(opts, A.device, force_S, force_beta, s_hint, cert, workspace)
    if events is not None:
        opts.ev_gemm_begin = ctypes.c_void_p(events[0])
        opts.ev_gemm_end = ctypes.c_void_p(events[1])
    dbg = None
    if debug:
        dbg = MDDebug()
        need = {"E": (M, torch.int32), "F": (N, torch.int32),
                "digits_A": (force_S * M * K, torch.int32), "digits_B": (force_S * N * K, torch.int32),
                "D": (force_S * M * N, torch.int64)}
        for key in ("E", "F", "digits_A", "digits_B", "D"):
            t = debug.get(key)
            if t is None:
                continue
            if key not in ("E", "F") and force_S <= 0:
                raise ValueError(f"debug {key} is sized by S: pass force_S")
            n, dt = need[key]
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
                raise ValueError(f"debug {key} must be a contiguous {dt} device tensor of >= {n} elements")
            setattr(dbg, key, t.data_ptr())
        opts.dbg = ctypes.pointer(dbg)
    lda = A.shape[2]
    ldb = B.shape[2]
    if noalloc and workspace is not None:
        raise ValueError("md_gemm_ex_noalloc takes no workspace")
    fn = lib().md_gemm_ex_noalloc if noalloc else lib().md_gemm_ex
    sh = _stream_handle(stream)

    def call():
        return fn(m, int(transA), int(transB), M, N, K, _ptr(A), lda, A.shape[1] * A.shape[2],
                  _ptr(B), ldb, B.shape[1] * B.shape[2], _ptr(C), N, M * N, ctypes.byref(opts), sh)

    if workspace is None and not noalloc and not debug and not pool:
        key = ("gemm", form, rule, target_bits, force_beta, m, M, N, K, bool(transA), bool(transB))
        ws = _auto_workspace(key, lambda S: lib().md_gemm_workspace_size(_FORMS[form], M, N, K, S),
                             force_S or s_hint, A.device, stream)
        _run_with_scratch(call, opts, ws, key, info)
    else:
        _check(call(), info)
    return C, info.as_dict()


def gemm(A: torch.Tensor, B: torch.Tensor, form: str = "fp64", stream=None) -> torch.Tensor:
    """C = A B for m-double planes A (m, M, K) and B (m, K, N)."""
    if form == "fp64" and stream is None:
        _check_planes(A, "A")
        _check_planes(B, "B")
        A = A.contiguous()
        B = B.contiguous()
        m, M, K = A.shape
        N = B.shape[2]
        if B.shape[:2] != (m, K):
            raise ValueError("shape mismatch")
        C = torch.empty((m, M, N), dtype=torch.float64, device=A.device)
        _check(lib().md_gemm(m, M, N, K, _ptr(A), _ptr(B), _ptr(C), _stream_handle(None)))
        return C
    return gemm_ex(A, B, form=form, stream=stream)[0]


def dot_ex(X: torch.Tensor, Y: torch.Tensor, out: torch.Tensor | None = None, *, form="fp64",
           rule="rho", target_bits=0, force_S=0, force_beta=0, events=None, stream=None,
           validate=False, workspace: torch.Tensor | None = None, s_hint=0,
           cert: torch.Tensor | None = None, pool=False):
    """Batched m-double inner products out_b = sum_k X[:, b, k] Y[:, b, k].

    X and Y are (m, batch, n) float64 planes on the HIP device (m = 1, 2, 4,
    8 or 16); out is (m, batch).  Returns (out, info dict); ``events`` and
    ``validate`` as in ``gemm_ex`` (events recorded around the contraction
    and the fold).  ``workspace``: a device byte buffer of at least
    ``md_dot_workspace_size`` bytes (the library then allocates nothing);
    ``s_hint``, ``cert`` and ``pool`` as in ``gemm_ex``.
    """
    _check_planes(X, "X")
    _check_planes(Y, "Y")
    X = X.contiguous()
    Y = Y.contiguous()
    if X.shape != Y.shape:
        raise ValueError(f"X and Y differ in shape: {tuple(X.shape)} vs {tuple(Y.shape)}")
    m, batch, n = X.shape
    if out is None:
        out = torch.empty((m, batch), dtype=torch.float64, device=X.device)
    elif out.shape != (m, batch) or not out.is_contiguous() or out.dtype != torch.float64:
        raise ValueError("out must be a contiguous float64 (m, batch) tensor")
    info = MDInfo()
    opts = MDOpts()
    opts.form = _FORMS[form]
    opts.s_rule = _RULES[rule]
    opts.target_bits = target_bits
    opts.validate = 1 if validate else 0
    opts.info = ctypes.pointer(info)
    _slice_opts(opts, X.device, force_S, force_beta, s_hint, cert, workspace)
    if events is not None:
        opts.ev_gemm_begin = ctypes.c_void_p(events[0])
        opts.ev_gemm_end = ctypes.c_void_p(events[1])
    sh = _stream_handle(stream)

    def call():
        return lib().md_dot_ex(m, batch, n, _ptr(X), n, batch * n, _ptr(Y), n, batch * n, _ptr(out), batch,
                               ctypes.byref(opts), sh)

    if workspace is None and not pool:
        key = ("dot", form, rule, target_bits, force_beta, m, batch, n)
        ws = _auto_workspace(key, lambda S: lib().md_dot_workspace_size(_FORMS[form], batch, n, S),
                             force_S or s_hint, X.device, stream)
        _run_with_scratch(call, opts, ws, key, info)
    else:
        _check(call(), info)
    return out, info.as_dict()


def dot(X: torch.Tensor, Y: torch.Tensor, form: str = "fp64", stream=None) -> torch.Tensor:
    """out_b = sum_k X[:, b, k] Y[:, b, k] for m-double planes (m, batch, n)."""
    return dot_ex(X, Y, form=form, stream=stream)[0]


def gemm_ordinary(A: torch.Tensor, B: torch.Tensor, stream=None) -> torch.Tensor:
    """C = A B in ordinary m-double arithmetic (m = 1, 2, 4, 8), every
    operation renormalised: the comparison baseline, not error-free."""
    _check_planes(A, "A")
    _check_planes(B, "B")
    A = A.contiguous()
    B = B.contiguous()
    m, M, K = A.shape
    N = B.shape[2]
    if B.shape[:2] != (m, K):
        raise ValueError("shape mismatch")
    C = torch.empty((m, M, N), dtype=torch.float64, device=A.device)
    _check(lib().md_gemm_ordinary(m, M, N, K, _ptr(A), _ptr(B), _ptr(C), _stream_handle(stream)))
    return C


def dot_ordinary(X: torch.Tensor, Y: torch.Tensor, stream=None) -> torch.Tensor:
    """Batched inner products in ordinary m-double arithmetic (m = 1, 2, 4,
    8, 16) of (m, batch, n) planes, 64 partial sums per pair met pairwise:
    the comparison baseline of ``dot``, not error-free."""
    _check_planes(X, "X")
    _check_planes(Y, "Y")
    X = X.contiguous()
    Y = Y.contiguous()
    if X.shape != Y.shape:
        raise ValueError("X and Y differ in shape")
    m, batch, n = X.shape
    out = torch.empty((m, batch), dtype=torch.float64, device=X.device)
    _check(lib().md_dot_ordinary(m, batch, n, _ptr(X), _ptr(Y), _ptr(out), _stream_handle(stream)))
    return out


def fixed_limbs(beta: int, S: int, K: int) -> int:
    """32-bit limbs that hold the exact integer of any product of depth up
    to K with these slices (host only)."""
    n = lib().md_fixed_limbs(beta, S, K)
    if n < 0:
        raise ValueError(f"no limb count for beta={beta}, S={S}, K={K}")
    return n


def _strided_planes(X: torch.Tensor, name: str):
    """(pointer, leading dimension, plane stride) of float64 planes whose
    rows are contiguous (a column block of larger planes is allowed).  The
    view's own strides are passed, so the library reads exactly the view's
    elements; only a dimension of size 1 (whose stride is never used) gets
    the dense value.  Rows or planes that overlap (a broadcast view) are
    refused."""
    _check_planes(X, name)
    ld, ps = _plane_layout(tuple(X.shape), tuple(X.stride()), name)
    return _ptr(X), ld, ps


def _plane_layout(shape, strides, name="X"):
    """(leading dimension, plane stride) for planes of the given shape and
    element strides; ValueError for non-contiguous rows or overlapping rows
    or planes."""
    m, R, Cc = shape
    if strides[2] != 1 and Cc > 1:
        raise ValueError(f"{name} must have contiguous rows")
    ld = strides[1] if R > 1 else Cc
    ps = strides[0] if m > 1 else R * ld
    if (R > 1 and ld < Cc) or (m > 1 and ps < (R - 1) * ld + Cc):
        raise ValueError(f"{name}: rows or planes overlap")
    return ld, ps


def exponents(A: torch.Tensor, B: torch.Tensor, stream=None):
    """Shared exponents (int32 device tensors) of the rows of A (m, M, K)
    and the columns of B (m, K, N): the largest exponent of the nonzero
    leading words, 0 where there is none."""
    pa, lda, _ = _strided_planes(A, "A")
    pb, ldb, _ = _strided_planes(B, "B")
    M, K = A.shape[1], A.shape[2]
    N = B.shape[2]
    if B.shape[1] != K:
        raise ValueError(f"inner sizes differ: {K} vs {B.shape[1]}")
    E = torch.empty(M, dtype=torch.int32, device=A.device)
    F = torch.empty(N, dtype=torch.int32, device=A.device)
    _check(lib().md_exponents(M, N, K, pa, lda, pb, ldb, _ptr(E), _ptr(F), _stream_handle(stream)))
    return E, F


def gemm_fixed(A: torch.Tensor, B: torch.Tensor, E: torch.Tensor | None = None,
               F: torch.Tensor | None = None, *, S: int, beta: int, form="fp64", nlimb=None,
               flags: torch.Tensor | None = None, stream=None):
    """Exact integer X (nlimb, M, N) int32 limb planes and scale (M, N) of
    the product A B before its rounding, C~ = X 2^scale.

    A (m, M, K) and B (m, K, N) may be depth blocks of larger planes (views
    with contiguous rows); E, F: the shared exponents to split on (those of
    the full matrices for a depth-split product), None for the data's own.
    nlimb defaults to the limbs of a depth-K product.  ``flags``: an int32
    device tensor into which bit 8 is ORed when a given exponent is not
    taken, without synchronising (else the call waits and raises).  Returns
    (X, scale, info dict)."""
    pa, lda, psa = _strided_planes(A, "A")
    pb, ldb, psb = _strided_planes(B, "B")
    m, M, K = A.shape
    N = B.shape[2]
    if B.shape[:2] != (m, K):
        raise ValueError("shape mismatch")
    if nlimb is None:
        nlimb = fixed_limbs(beta, S, K)
    X = torch.empty((nlimb, M, N), dtype=torch.int32, device=A.device)
    scale = torch.empty((M, N), dtype=torch.int32, device=A.device)
    for T, name, n in ((E, "E", M), (F, "F", N)):
        if T is not None and (T.dtype != torch.int32 or T.shape != (n,) or not T.is_cuda
                              or not T.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous int32 device vector of {n} entries")
    info = MDInfo()
    opts = MDOpts()
    opts.form = _FORMS[form]
    opts.force_S = S
    opts.force_beta = beta
    opts.info = ctypes.pointer(info)
    if flags is not None:
        if flags.dtype != torch.int32 or not flags.is_cuda or flags.numel() < 1:
            raise ValueError("flags must be an int32 device tensor")
        opts.exp_flags = ctypes.c_void_p(flags.data_ptr())
    rc = lib().md_gemm_fixed(m, M, N, K, pa, lda, psa, pb, ldb, psb,
                             None if E is None else _ptr(E), None if F is None else _ptr(F),
                             _ptr(X), nlimb, _ptr(scale), ctypes.byref(opts), _stream_handle(stream))
    _check(rc, info)
    return X, scale, info.as_dict()


def fixed_add(X: torch.Tensor, Y: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """out = X + Y for int32 limb planes (nlimb, ...) at the same scale."""
    if X.dtype != torch.int32 or Y.dtype != torch.int32 or X.shape != Y.shape or X.dim() < 1:
        raise ValueError("X and Y must be int32 limb planes of one shape")
    X = X.contiguous()
    Y = Y.contiguous()
    if out is None:
        out = torch.empty_like(X)
    elif out.shape != X.shape or out.dtype != torch.int32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor of X's shape")
    nlimb = X.shape[0]
    count = X.numel() // max(nlimb, 1)
    _check(lib().md_fixed_add(count, nlimb, _ptr(X), _ptr(Y), _ptr(out), _stream_handle(stream)))
    return out


def fixed_round(X: torch.Tensor, scale: torch.Tensor, m: int, stream=None) -> torch.Tensor:
    """X 2^scale rounded greedily to nearest into m words: (m, *scale.shape)."""
    if X.dtype != torch.int32 or scale.dtype != torch.int32 or X.shape[1:] != scale.shape:
        raise ValueError("X must be int32 limb planes (nlimb, *scale.shape), scale int32")
    X = X.contiguous()
    scale = scale.contiguous()
    count = scale.numel()
    C = torch.empty((m,) + tuple(scale.shape), dtype=torch.float64, device=X.device)
    _check(lib().md_fixed_round(m, count, X.shape[0], _ptr(X), _ptr(scale), _ptr(C), count,
                                _stream_handle(stream)))
    return C


class MDGemm(torch.autograd.Function):
    """C = A B with the hand-written m-double adjoint.

    forward(A, B, form) -> C; backward(dC) -> (dC B^T, A^T dC, None), each an
    m-double product through the same error-free summation.
    """

    @staticmethod
    def forward(ctx, A, B, form="fp64"):
        ctx.save_for_backward(A, B)
        ctx.form = form
        return gemm_ex(A, B, form=form)[0]

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        dC = dC.contiguous()
        dA = dB = None
        if ctx.needs_input_grad[0]:
            dA = gemm_ex(dC, B, transB=True, form=ctx.form)[0]
        if ctx.needs_input_grad[1]:
            dB = gemm_ex(A, dC, transA=True, form=ctx.form)[0]
        return dA, dB, None


__all__ = ["gemm", "gemm_ex", "gemm_ordinary", "dot_ordinary", "dot", "dot_ex", "MDGemm", "choose_params", "lib",
           "MDError", "MDInfo", "MDCert", "new_cert", "read_cert"]
