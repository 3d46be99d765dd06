"""Python binding of libtsmm (include/tsmm.h): argument marshalling only.

Every step of the multiply runs in the library's HIP kernels; this module
checks tensor devices, types, shapes and contiguity, passes raw device
pointers and torch's current HIP stream, and turns status codes into
exceptions.  PyTorch provides device memory and streams.  There is no
fallback: if ``libtsmm.so`` has not been built, every call raises.

The names follow the C ABI: :func:`pack`, :func:`plan`, :func:`execute`,
:func:`plan_batched`, ... (AutoTSMM, Algorithm 1: PACKB, the runtime
execution plan, COMPUTE).
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsmm.so")

SUCCESS, INVALID_VALUE, SHAPE_MISMATCH, NOT_SUPPORTED, TABLE, OUT_OF_MEMORY, NO_DEVICE, HIP = range(8)
F64, F32, BF16 = 0, 1, 2
OP_N, OP_T, COLMAJOR = 0, 1, 2
MODE_NATIVE, MODE_BF16X3, MODE_BF16X6 = 0, 1, 2
(KERNEL_AUTO, KERNEL_SIMPLE, KERNEL_STREAM, KERNEL_SPLITK, KERNEL_SPLITBF16, KERNEL_VALU64, KERNEL_WIDE,
 KERNEL_BATCHED, KERNEL_SLAB, KERNEL_COLMAJOR) = range(10)

_MODES = {"native": MODE_NATIVE, "bf16x3": MODE_BF16X3, "bf16x6": MODE_BF16X6}
_LAYOUTS = {"N": OP_N, "T": OP_T, "C": COLMAJOR}
_DT_OF_TORCH = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
_TORCH_OF_DT = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}
_OUT_OF_DT = {F64: torch.float64, F32: torch.float32, BF16: torch.float32}


class TsmmError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, _lib().tsmm_status_string(status).decode(), detail))


class _Tile(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in
                ("kernel", "rows_per_wave", "waves_per_wg", "wg_per_cu", "splitk", "nsplit", "chunk_rows")]


def _set_tile(h, **fields):
    t = _Tile(**fields)
    _check(_lib().tsmm_plan_set_tile(h, ctypes.byref(t)), "tsmm_plan_set_tile")


def _get_tile(h) -> dict:
    t = _Tile()
    _check(_lib().tsmm_plan_get_tile(h, ctypes.byref(t)), "tsmm_plan_get_tile")
    return {f: getattr(t, f) for f, _ in _Tile._fields_}


def _describe(h) -> str:
    buf = ctypes.create_string_buffer(512)
    _check(_lib().tsmm_plan_describe(h, buf, 512), "tsmm_plan_describe")
    return buf.value.decode()


class _Caps(ctypes.Structure):
    _fields_ = [("compute_units", ctypes.c_int32), ("lds_bytes_per_cu", ctypes.c_int32),
                ("gcn_arch", ctypes.c_int32)]


_LIB = None

# (name, restype, argtypes) of every exported entry point of include/tsmm.h
_VP, _I64, _DBL, _I32, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_size_t
_PVP = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = [
    ("tsmm_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("tsmm_last_error", ctypes.c_char_p, []),
    ("tsmm_version", _I32, []),
    ("tsmm_table_key", ctypes.c_int, [_I32, ctypes.c_char_p, _SZ]),
    ("tsmm_pack", ctypes.c_int, [_VP, _I64, _I64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _PVP]),
    ("tsmm_packed_bytes", ctypes.c_int, [_VP, ctypes.POINTER(_SZ)]),
    ("tsmm_unpack", ctypes.c_int, [_VP, _VP, _VP]),
    ("tsmm_packed_split_planes", ctypes.c_int, [_VP, _VP, _VP, _VP]),
    ("tsmm_packed_destroy", None, [_VP]),
    ("tsmm_plan", ctypes.c_int, [_I64, _I64, _I64, ctypes.c_int, ctypes.c_int, _PVP]),
    ("tsmm_plan_with_caps", ctypes.c_int, [_I64, _I64, _I64, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(_Caps), _PVP]),
    ("tsmm_plan_set_mode", ctypes.c_int, [_VP, ctypes.c_int]),
    ("tsmm_plan_set_tile", ctypes.c_int, [_VP, ctypes.POINTER(_Tile)]),
    ("tsmm_plan_tune", ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    ("tsmm_tune_cache_clear", None, []),
    ("tsmm_plan_get_tile", ctypes.c_int, [_VP, ctypes.POINTER(_Tile)]),
    ("tsmm_plan_set_stream", ctypes.c_int, [_VP, _VP]),
    ("tsmm_plan_workspace_bytes", ctypes.c_int, [_VP, ctypes.POINTER(_SZ)]),
    ("tsmm_plan_set_workspace", ctypes.c_int, [_VP, _VP, _SZ]),
    ("tsmm_plan_describe", ctypes.c_int, [_VP, ctypes.c_char_p, _SZ]),
    ("tsmm_plan_destroy", None, [_VP]),
    ("tsmm_execute", ctypes.c_int, [_VP, _VP, _VP, _VP, _DBL, _DBL]),
    ("tsmm_execute_ld", ctypes.c_int, [_VP, _VP, _I64, _VP, _VP, _I64, _DBL, _DBL]),
    ("tsmm_execute_noalloc", ctypes.c_int, [_VP, _VP, _VP, _VP, _DBL, _DBL]),
    ("tsmm_pack_a", ctypes.c_int, [_VP, _I64, _I64, _I64, ctypes.c_int, ctypes.c_int, _DBL, _VP, _PVP]),
    ("tsmm_execute_packed_a", ctypes.c_int, [_VP, _VP, _VP, _VP, _DBL]),
    ("tsmm_plan_batched", ctypes.c_int, [_I64, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                         ctypes.POINTER(_I64), ctypes.c_int, _PVP]),
    ("tsmm_batched_bind", ctypes.c_int, [_VP, _PVP, _PVP, _PVP, ctypes.POINTER(_DBL), ctypes.POINTER(_DBL)]),
    ("tsmm_execute_batched", ctypes.c_int, [_VP, _PVP, _PVP, _PVP, ctypes.POINTER(_DBL),
                                            ctypes.POINTER(_DBL)]),
    ("tsmm_graph_create_batched", ctypes.c_int, [_VP, _PVP]),
    ("tsmm_graph_launch", ctypes.c_int, [_VP, _VP]),
    ("tsmm_graph_destroy", None, [_VP]),
]


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtsmm.so is not built (%s): run `python -m paper_2208_08088_amd.build`"
                               % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def _check(status, where):
    if status != SUCCESS:
        raise TsmmError(status, where, _lib().tsmm_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _need_cuda(t, name, dtype=None, shape=None, colmajor=False):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor" % name)
    if colmajor:
        # a column-major matrix is the transpose of a contiguous tensor
        if t.dim() != 2 or not t.t().is_contiguous():
            raise ValueError("%s must be column-major (the transpose of a contiguous tensor)" % name)
    elif not t.is_contiguous():
        raise ValueError("%s must be contiguous (row-major)" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def version():
    return _lib().tsmm_version()


def table_key(gcn_arch: int = 0) -> str:
    """The key lines a tile table needs to be used by this library on this
    runtime (tsmm_table_key); gcn_arch 0 means the current device's."""
    buf = ctypes.create_string_buffer(256)
    _check(_lib().tsmm_table_key(int(gcn_arch), buf, 256), "tsmm_table_key")
    return buf.value.decode()


# ---------------------------------------------------------------- packed

class Packed:
    """A packed small operand (tsmm_pack); reusable by any number of executes."""

    def __init__(self, handle, k, n, dtype, layout, mode, keep):
        self._h = handle
        self.k, self.n, self.dtype, self.layout, self.mode = k, n, dtype, layout, mode
        self._keep = keep  # op T handles refer to the caller's B

    @property
    def handle(self):
        return self._h

    def nbytes(self):
        b = ctypes.c_size_t(0)
        _check(_lib().tsmm_packed_bytes(self._h, ctypes.byref(b)), "tsmm_packed_bytes")
        return b.value

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            _LIB.tsmm_packed_destroy(h)


def pack(B: torch.Tensor, layout: str = "N", mode: str = "native") -> Packed:
    """Pack B (k x n on the device; row-major, or column-major for layout
    "C") once for reuse."""
    if B.dtype not in _DT_OF_TORCH:
        raise TypeError("B must be float64, float32 or bfloat16")
    _need_cuda(B, "B", colmajor=layout == "C")
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    k, n = B.shape
    dt = _DT_OF_TORCH[B.dtype]
    h = ctypes.c_void_p(0)
    _check(_lib().tsmm_pack(_ptr(B), k, n, _LAYOUTS[layout], dt, _MODES[mode], _stream(), ctypes.byref(h)),
           "tsmm_pack")
    return Packed(h.value, k, n, dt, _LAYOUTS[layout], _MODES[mode], B if layout == "T" else None)


class PackedA:
    """A packed big operand (tsmm_pack_a): alpha*A, pre-split into bfloat16
    terms in the split-bf16 modes; reusable by any number of
    execute_packed_a calls."""

    def __init__(self, handle, m, k, dtype, mode, alpha):
        self._h = handle
        self.m, self.k, self.dtype, self.mode, self.alpha = m, k, dtype, mode, alpha

    @property
    def handle(self):
        return self._h

    def nbytes(self):
        b = ctypes.c_size_t(0)
        _check(_lib().tsmm_packed_bytes(self._h, ctypes.byref(b)), "tsmm_packed_bytes")
        return b.value

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            _LIB.tsmm_packed_destroy(h)


def pack_a(A: torch.Tensor, mode: str = "native", alpha: float = 1.0) -> PackedA:
    """Pack A (m x k on the device, rows with adjacent elements; a row
    stride is taken as the leading dimension) once, with alpha folded in."""
    if A.dtype not in _DT_OF_TORCH:
        raise TypeError("A must be float64, float32 or bfloat16")
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    m, k = A.shape
    lda = _leading_dim(A, "A", A.dtype, (m, k), False)
    dt = _DT_OF_TORCH[A.dtype]
    h = ctypes.c_void_p(0)
    _check(_lib().tsmm_pack_a(_ptr(A), m, k, lda, dt, _MODES[mode], float(alpha), _stream(), ctypes.byref(h)),
           "tsmm_pack_a")
    return PackedA(h.value, m, k, dt, _MODES[mode], float(alpha))


def unpack(p: Packed) -> torch.Tensor:
    out_dt = torch.float32 if p.mode != MODE_NATIVE else _TORCH_OF_DT[p.dtype]
    if p.layout == COLMAJOR:  # the stored copy is column-major
        out = torch.empty((p.n, p.k), dtype=out_dt, device="cuda").t()
    else:
        out = torch.empty((p.k, p.n), dtype=out_dt, device="cuda")
    _check(_lib().tsmm_unpack(p.handle, _ptr(out), _stream()), "tsmm_unpack")
    return out


def split_planes(p: Packed):
    """(planes, exps): uint16 bit patterns [terms, k, n] (as int16 storage)
    and int32 column exponents [n] of a split-mode handle."""
    terms = {MODE_BF16X3: 2, MODE_BF16X6: 3}.get(p.mode, 0)
    planes = torch.empty((terms, p.k, p.n), dtype=torch.int16, device="cuda")
    exps = torch.empty((p.n,), dtype=torch.int32, device="cuda")
    _check(_lib().tsmm_packed_split_planes(p.handle, _ptr(planes), _ptr(exps), _stream()),
           "tsmm_packed_split_planes")
    return planes, exps


# ------------------------------------------------------------------ plan

class Plan:
    """An execution plan (tsmm_plan) for one shape."""

    def __init__(self, handle, m, n, k, layout, dtype):
        self._h = handle
        self.m, self.n, self.k, self.layout, self.dtype = m, n, k, layout, dtype
        self.mode = MODE_NATIVE
        self._ws = None
        self._ws_bytes = None  # the plan's workspace need, while its tile stands
        self._stream_set = None  # the stream last given to tsmm_plan_set_stream

    @property
    def handle(self):
        return self._h

    def set_mode(self, mode: str):
        _check(_lib().tsmm_plan_set_mode(self._h, _MODES[mode]), "tsmm_plan_set_mode")
        self.mode = _MODES[mode]
        self._drop_workspace()
        return self

    def set_tile(self, kernel=0, rows_per_wave=0, waves_per_wg=0, wg_per_cu=0, splitk=0, nsplit=0, chunk_rows=0):
        _set_tile(self._h, kernel=kernel, rows_per_wave=rows_per_wave, waves_per_wg=waves_per_wg,
                  wg_per_cu=wg_per_cu, splitk=splitk, nsplit=nsplit, chunk_rows=chunk_rows)
        self._drop_workspace()
        return self

    def get_tile(self) -> dict:
        return _get_tile(self._h)

    def tune(self, A: torch.Tensor, packed: "Packed", C: torch.Tensor, reps: int = 3) -> float:
        """Runtime evaluator (tsmm_plan_tune): time the candidate tiles on
        these operands, keep the fastest (also for later plans of the same
        shape class in this process).  C is overwritten.  Returns the
        winner's median milliseconds."""
        in_dt = _TORCH_OF_DT[self.dtype]
        a_shape = (self.k, self.m) if self.layout == OP_T else (self.m, self.k)
        cm = self.layout == COLMAJOR
        _need_cuda(A, "A", in_dt, a_shape, colmajor=cm)
        _need_cuda(C, "C", _OUT_OF_DT[self.dtype], (self.m, self.n), colmajor=cm)
        lib = _lib()
        self._set_stream()
        # the candidates run on plan-owned scratch, never on this binding's
        # tensor, which is released first
        self._drop_workspace()
        ms = ctypes.c_double(0.0)
        _check(lib.tsmm_plan_tune(self._h, _ptr(A), packed.handle, _ptr(C), int(reps), ctypes.byref(ms)),
               "tsmm_plan_tune")
        return ms.value

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t(0)
        _check(_lib().tsmm_plan_workspace_bytes(self._h, ctypes.byref(b)), "tsmm_plan_workspace_bytes")
        return b.value

    def describe(self) -> str:
        return _describe(self._h)

    def info(self) -> dict:
        out = {}
        for kv in self.describe().split():
            key, _, val = kv.partition("=")
            out[key] = val
        return out

    def _drop_workspace(self):
        """Detach this binding's workspace tensor from the C plan, then let
        it go: the plan must never keep a pointer into memory that torch's
        allocator may hand to another tensor."""
        if self._ws is not None:
            _check(_lib().tsmm_plan_set_workspace(self._h, None, 0), "tsmm_plan_set_workspace")
            self._ws = None
        self._ws_bytes = None  # the tile (or mode) changes with every caller of this

    def _ensure_workspace(self):
        if self._ws_bytes is None:
            self._ws_bytes = self.workspace_bytes()
        nb = self._ws_bytes
        if nb and (self._ws is None or self._ws.numel() < nb):
            self._ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
            _check(_lib().tsmm_plan_set_workspace(self._h, _ptr(self._ws), nb), "tsmm_plan_set_workspace")

    def _set_stream(self):
        """Queue this plan's launches on torch's current stream (the C call
        only when the stream changed)."""
        st = torch.cuda.current_stream().cuda_stream
        if st != self._stream_set:
            _check(_lib().tsmm_plan_set_stream(self._h, ctypes.c_void_p(st)), "tsmm_plan_set_stream")
            self._stream_set = st

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            _LIB.tsmm_plan_destroy(h)


def tune_cache_clear():
    """Forget the tiles the runtime evaluator chose in this process."""
    _lib().tsmm_tune_cache_clear()


def plan(m: int, n: int, k: int, layout: str = "N", dtype=torch.float64) -> Plan:
    """Execution plan for C(m x n) = alpha*op(A)*B + beta*C with B k x n."""
    h = ctypes.c_void_p(0)
    dt = _DT_OF_TORCH[dtype]
    _check(_lib().tsmm_plan(m, n, k, _LAYOUTS[layout], dt, ctypes.byref(h)), "tsmm_plan")
    return Plan(h.value, m, n, k, _LAYOUTS[layout], dt)


def plan_with_caps(m, n, k, layout="N", dtype=torch.float64, compute_units=256, lds_bytes_per_cu=163840,
                   gcn_arch=950) -> Plan:
    """Plan against explicit device properties (no GPU needed; not executable)."""
    h = ctypes.c_void_p(0)
    caps = _Caps(compute_units, lds_bytes_per_cu, gcn_arch)
    dt = _DT_OF_TORCH[dtype]
    _check(_lib().tsmm_plan_with_caps(m, n, k, _LAYOUTS[layout], dt, ctypes.byref(caps), ctypes.byref(h)),
           "tsmm_plan_with_caps")
    return Plan(h.value, m, n, k, _LAYOUTS[layout], dt)


def _leading_dim(t, name, dtype, shape, colmajor):
    """The stride between rows (row-major) or columns (column-major) of a
    2-D device tensor whose elements within a row (column) are adjacent."""
    if (not colmajor and isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.shape == shape
            and t.is_contiguous()):
        return max(1, shape[1])  # a dense row-major matrix: the common case, checked in one pass
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    rows, cols = shape
    inner, outer = (0, 1) if colmajor else (1, 0)
    lines, width = (cols, rows) if colmajor else (rows, cols)
    if t.numel() == 0:  # nothing is read or written
        return max(1, width)
    if width > 1 and t.stride(inner) != 1:
        raise ValueError("%s: elements within a %s must be adjacent" % (name, "column" if colmajor else "row"))
    if lines <= 1:
        return max(1, width)
    ld = t.stride(outer)
    if ld < width:
        raise ValueError("%s: stride %d below the %s length %d" % (name, ld, "column" if colmajor else "row", width))
    return ld


def execute(p: Plan, A: torch.Tensor, packed: Packed, C: torch.Tensor, alpha: float = 1.0,
            beta: float = 0.0) -> torch.Tensor:
    """C = alpha*op(A)*B + beta*C in place on torch's current stream.  A and
    C may be strided views (rows, or columns for layout "C", with adjacent
    elements): their strides go to tsmm_execute_ld as leading dimensions."""
    in_dt = _TORCH_OF_DT[p.dtype]
    a_shape = (p.k, p.m) if p.layout == OP_T else (p.m, p.k)
    cm = p.layout == COLMAJOR
    lda = _leading_dim(A, "A", in_dt, a_shape, cm)
    ldc = _leading_dim(C, "C", _OUT_OF_DT[p.dtype], (p.m, p.n), cm)
    if packed.layout == OP_T and packed._keep is not None:
        _need_cuda(packed._keep, "B")
    p._ensure_workspace()
    p._set_stream()
    _check(_lib().tsmm_execute_ld(p.handle, _ptr(A), lda, packed.handle, _ptr(C), ldc, float(alpha), float(beta)),
           "tsmm_execute_ld")
    return C


def execute_noalloc(p: Plan, A: torch.Tensor, packed: Packed, C: torch.Tensor, alpha: float = 1.0,
                    beta: float = 0.0) -> torch.Tensor:
    """C = alpha*op(A)*B + beta*C in place on torch's current stream without
    any device allocation (tsmm_execute_noalloc): split-k partial sums go to
    the library's static scratch, never to a workspace.  A and C contiguous
    (column-major for layout "C")."""
    in_dt = _TORCH_OF_DT[p.dtype]
    a_shape = (p.k, p.m) if p.layout == OP_T else (p.m, p.k)
    cm = p.layout == COLMAJOR
    _need_cuda(A, "A", in_dt, a_shape, colmajor=cm)
    _need_cuda(C, "C", _OUT_OF_DT[p.dtype], (p.m, p.n), colmajor=cm)
    if packed.layout == OP_T and packed._keep is not None:
        _need_cuda(packed._keep, "B")
    p._set_stream()
    _check(_lib().tsmm_execute_noalloc(p.handle, _ptr(A), packed.handle, _ptr(C), float(alpha), float(beta)),
           "tsmm_execute_noalloc")
    return C


def execute_packed_a(p: Plan, packed_a: PackedA, packed: Packed, C: torch.Tensor, beta: float = 0.0) -> torch.Tensor:
    """C = A_packed*B + beta*C (alpha folded into A_packed) in place on
    torch's current stream; C row-major m x n, contiguous."""
    _need_cuda(C, "C", _OUT_OF_DT[p.dtype], (p.m, p.n))
    p._ensure_workspace()
    p._set_stream()
    _check(_lib().tsmm_execute_packed_a(p.handle, packed_a.handle, packed.handle, _ptr(C), float(beta)),
           "tsmm_execute_packed_a")
    return C


# --------------------------------------------------------------- batched

class BatchedPlan:
    """Many independent op N multiplies in one persistent launch."""

    def __init__(self, handle, ms, ns, ks, dtype):
        self._h = handle
        self.ms, self.ns, self.ks, self.dtype = list(ms), list(ns), list(ks), dtype
        self._bound = None

    @property
    def handle(self):
        return self._h

    def set_chunk_rows(self, chunk_rows: int = 0, wg_per_cu: int = 0):
        """Rows per work item of the persistent launch (0: the tile table's
        or the default) and resident workgroups per compute unit (1, 2 or 4
        as the LDS allows; 0: the table's with the table's chunk size, else
        the plan's current count); the plan must be idle and have no live
        graph."""
        _set_tile(self._h, kernel=KERNEL_BATCHED, chunk_rows=chunk_rows, wg_per_cu=wg_per_cu)
        return self

    def get_tile(self) -> dict:
        return _get_tile(self._h)

    def describe(self) -> str:
        return _describe(self._h)

    def _arrays(self, As, packeds, Cs, alphas, betas):
        cnt = len(self.ms)
        if not (len(As) == len(packeds) == len(Cs) == cnt):
            raise ValueError("need %d A, packed and C operands" % cnt)
        in_dt, out_dt = _TORCH_OF_DT[self.dtype], _OUT_OF_DT[self.dtype]
        for b in range(cnt):
            _need_cuda(As[b], "A[%d]" % b, in_dt, (self.ms[b], self.ks[b]))
            _need_cuda(Cs[b], "C[%d]" % b, out_dt, (self.ms[b], self.ns[b]))
        VA = ctypes.c_void_p * cnt
        a = VA(*[t.data_ptr() for t in As])
        pk = VA(*[p.handle for p in packeds])
        c = VA(*[t.data_ptr() for t in Cs])
        DA = ctypes.c_double * cnt
        al = DA(*([1.0] * cnt if alphas is None else [float(x) for x in alphas]))
        be = DA(*([0.0] * cnt if betas is None else [float(x) for x in betas]))
        return a, pk, c, al, be

    def bind(self, As, packeds, Cs, alphas=None, betas=None):
        a, pk, c, al, be = self._arrays(As, packeds, Cs, alphas, betas)
        lib = _lib()
        _check(lib.tsmm_plan_set_stream(self._h, _stream()), "tsmm_plan_set_stream")
        _check(lib.tsmm_batched_bind(self._h, a, pk, c, al, be), "tsmm_batched_bind")
        self._bound = (list(As), list(packeds), list(Cs))  # keep operands alive
        return self

    def execute(self, As=None, packeds=None, Cs=None, alphas=None, betas=None):
        lib = _lib()
        _check(lib.tsmm_plan_set_stream(self._h, _stream()), "tsmm_plan_set_stream")
        if As is not None:
            self.bind(As, packeds, Cs, alphas, betas)
        _check(lib.tsmm_execute_batched(self._h, None, None, None, None, None), "tsmm_execute_batched")

    def graph(self) -> "Graph":
        g = ctypes.c_void_p(0)
        _check(_lib().tsmm_graph_create_batched(self._h, ctypes.byref(g)), "tsmm_graph_create_batched")
        return Graph(g.value, self)

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            _LIB.tsmm_plan_destroy(h)


def plan_batched(ms, ns, ks, dtype=torch.float32) -> BatchedPlan:
    cnt = len(ms)
    IA = ctypes.c_int64 * cnt
    h = ctypes.c_void_p(0)
    _check(_lib().tsmm_plan_batched(cnt, IA(*[int(x) for x in ms]), IA(*[int(x) for x in ns]),
                                    IA(*[int(x) for x in ks]), _DT_OF_TORCH[dtype], ctypes.byref(h)),
           "tsmm_plan_batched")
    return BatchedPlan(h.value, ms, ns, ks, _DT_OF_TORCH[dtype])


class Graph:
    """A captured, instantiated batched launch (tsmm_graph_create_batched)."""

    def __init__(self, handle, owner):
        self._h = handle
        self._owner = owner  # keeps the plan and its bound operands alive

    def launch(self):
        _check(_lib().tsmm_graph_launch(self._h, _stream()), "tsmm_graph_launch")

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            _LIB.tsmm_graph_destroy(h)
