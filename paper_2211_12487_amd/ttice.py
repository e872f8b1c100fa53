"""Thin ctypes binding of libttice.so (include/ttice.h).

Argument marshalling only: device buffers are torch CUDA tensors whose
data_ptr() is handed to the C ABI; every step of TT-ICE runs in the
library's HIP kernels.  There is no CPU fallback: if the library is missing
the import of :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import List, Optional, Sequence

import torch  # loads the HIP runtime the library binds to (same soname)

__all__ = ["lib", "TTICE", "Server", "TTICEError", "UpdateInfo", "library_path", "EXPORTS"]

TTICE_MAX_D = 16
_HERE = os.path.dirname(os.path.abspath(__file__))

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
ALGO = {"plain": 0, "star": 1}
SKIP = {"mean": 0, "batch": 1, "none": 2}
OPT_PREC, OPT_ALGO, OPT_SKIP_RULE, OPT_TAU, OPT_STREAM, OPT_PROFILE, OPT_SVD = 1, 2, 3, 4, 5, 6, 7
SVD = {"auto": 1, "dense": 0}
KERNEL_PROJ_L1 = 0
F32, F64 = 0, 1

EXPORTS = [
    "ttice_create",
    "ttice_set_option",
    "ttice_update",
    "ttice_reconstruct",
    "ttice_project",
    "ttice_project_noalloc",
    "ttice_reserve",
    "ttice_ranks",
    "ttice_get_core",
    "ttice_get_kernel_stats",
    "ttice_save",
    "ttice_load",
    "ttice_shape",
    "ttice_destroy",
    "ttice_strerror",
    "ttice_server_create",
    "ttice_server_add_stream",
    "ttice_server_submit",
    "ttice_server_poll",
    "ttice_server_wait",
    "ttice_server_stream_state",
    "ttice_server_remove_stream",
    "ttice_server_stats",
    "ttice_server_destroy",
]


class ServerCounters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in ("reserved_bytes", "budget_bytes", "pending", "waiting_streams",
                                                    "groups", "grouped_increments")]


class UpdateInfo(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("skipped", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("used", ctypes.c_int64),
        ("n_total", ctypes.c_int64),
        ("norm_y2", ctypes.c_double),
        ("eps_core", ctypes.c_double),
        ("eps_upd", ctypes.c_double),
        ("ranks", ctypes.c_int64 * (TTICE_MAX_D + 2)),
        ("r_new", ctypes.c_int64 * TTICE_MAX_D),
        ("rho2", ctypes.c_double * TTICE_MAX_D),
        ("tail2", ctypes.c_double * TTICE_MAX_D),
        ("margin", ctypes.c_double * TTICE_MAX_D),
        ("achieved2", ctypes.c_double),
        ("solver", ctypes.c_int32 * TTICE_MAX_D),
    ]

    def as_dict(self) -> dict:
        d = self.d
        return dict(
            n=self.n, used=self.used, n_total=self.n_total, skipped=bool(self.skipped),
            normY2=self.norm_y2, eps_core=self.eps_core, eps_upd=self.eps_upd,
            ranks=list(self.ranks[: d + 2]), rR=list(self.r_new[:d]), rho2=list(self.rho2[:d]),
            tail2=list(self.tail2[:d]), margin=list(self.margin[:d]),
            achieved2=(self.achieved2 if self.achieved2 >= 0 else None),
            solver=list(self.solver[:d]),
        )


class KernelStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


def _output_ready(out: torch.Tensor) -> None:
    """The library writes `out` on the state's own stream (for a served state,
    a worker's non-blocking stream), unordered with torch's current stream:
    work torch has queued on that memory (an allocation's previous user)
    must be done first.  The library call returns after its write."""
    torch.cuda.current_stream(out.device).synchronize()


class TTICEError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_strerror(code)} ({code})")
        self.code = code


_LIB = None


def library_path() -> str:
    return os.environ.get("TTICE_LIBRARY", os.path.join(_HERE, "libttice.so"))


def lib():
    """Load libttice.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(path)
    c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    L.ttice_create.argtypes = [c_i32, ctypes.POINTER(c_i64), c_dbl, ctypes.POINTER(c_vp)]
    L.ttice_set_option.argtypes = [c_vp, c_i32, c_vp]
    L.ttice_update.argtypes = [c_vp, c_vp, c_i64, c_i32, ctypes.POINTER(UpdateInfo)]
    L.ttice_reconstruct.argtypes = [c_vp, c_i64, c_i64, c_vp, c_i32]
    L.ttice_project.argtypes = [c_vp, c_vp, c_i64, c_i32, c_vp, c_vp, c_vp]
    L.ttice_project_noalloc.argtypes = [c_vp, c_vp, c_i64, c_i32, c_vp, c_vp, c_vp]
    L.ttice_reserve.argtypes = [c_vp, c_i64]
    L.ttice_ranks.argtypes = [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]
    L.ttice_get_core.argtypes = [c_vp, c_i32, c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]
    L.ttice_get_kernel_stats.argtypes = [c_vp, c_i32, ctypes.POINTER(KernelStats)]
    L.ttice_save.argtypes = [c_vp, c_vp, c_i64, ctypes.POINTER(c_i64)]
    L.ttice_load.argtypes = [c_vp, c_i64, ctypes.POINTER(c_vp)]
    L.ttice_shape.argtypes = [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64), ctypes.POINTER(c_dbl)]
    L.ttice_destroy.argtypes = [c_vp]
    L.ttice_destroy.restype = None
    L.ttice_strerror.argtypes = [ctypes.c_int]
    L.ttice_strerror.restype = ctypes.c_char_p
    L.ttice_server_create.argtypes = [c_i32, c_i64, ctypes.POINTER(c_vp)]
    L.ttice_server_add_stream.argtypes = [c_vp, c_i32, ctypes.POINTER(c_i64), c_dbl, c_i32, c_i32, c_i64, c_i64,
                                          ctypes.POINTER(c_i32)]
    L.ttice_server_submit.argtypes = [c_vp, c_i32, c_vp, c_i64, c_i32, c_vp, ctypes.POINTER(c_i64)]
    L.ttice_server_poll.argtypes = [c_vp, c_i64, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                                    ctypes.POINTER(UpdateInfo)]
    L.ttice_server_wait.argtypes = [c_vp, c_i64, ctypes.POINTER(c_i32), ctypes.POINTER(UpdateInfo)]
    L.ttice_server_stream_state.argtypes = [c_vp, c_i32, ctypes.POINTER(c_vp)]
    L.ttice_server_remove_stream.argtypes = [c_vp, c_i32]
    L.ttice_server_stats.argtypes = [c_vp, ctypes.POINTER(ServerCounters)]
    L.ttice_server_destroy.argtypes = [c_vp]
    L.ttice_server_destroy.restype = None
    for name in ("ttice_create", "ttice_set_option", "ttice_update", "ttice_reconstruct",
                 "ttice_project", "ttice_reserve", "ttice_ranks", "ttice_get_core", "ttice_get_kernel_stats",
                 "ttice_save", "ttice_load", "ttice_shape",
                 "ttice_server_create", "ttice_server_add_stream", "ttice_server_submit", "ttice_server_poll",
                 "ttice_server_wait", "ttice_server_stream_state", "ttice_server_remove_stream",
                 "ttice_server_stats"):
        getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


def _strerror(code: int) -> str:
    try:
        return lib().ttice_strerror(code).decode()
    except Exception:  # pragma: no cover
        return "unknown"


def _check(code: int, what: str) -> None:
    if code != 0:
        raise TTICEError(code, what)


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float32:
        return F32
    if t == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t}")


class TTICE:
    """One TT-ICE accumulation living on the current HIP device."""

    _owner = True

    @classmethod
    def _borrowed(cls, handle: ctypes.c_void_p, dims: Sequence[int], eps: float) -> "TTICE":
        """A view of a state owned elsewhere (a server stream): read-only use,
        never destroyed from here."""
        self = cls.__new__(cls)
        self.dims = tuple(int(n) for n in dims)
        self.d = len(self.dims)
        self.eps = float(eps)
        self._h = handle
        self.stream = None
        self._owner = False
        return self

    def __init__(self, dims: Sequence[int], eps: float, prec: str = "fp64", algo: str = "plain",
                 skip_rule: str = "mean", tau: float = 1.0, stream: Optional[torch.cuda.Stream] = None,
                 svd: str = "auto"):
        L = lib()
        self.dims = tuple(int(n) for n in dims)
        self.d = len(self.dims)
        self.eps = float(eps)
        arr = (ctypes.c_int64 * max(self.d, 1))(*self.dims)
        h = ctypes.c_void_p()
        _check(L.ttice_create(self.d, arr, self.eps, ctypes.byref(h)), "ttice_create")
        self._h = h
        self.stream = stream
        self.set_option(OPT_PREC, ctypes.c_int32(PREC[prec]))
        self.set_option(OPT_ALGO, ctypes.c_int32(ALGO[algo]))
        self.set_option(OPT_SKIP_RULE, ctypes.c_int32(SKIP[skip_rule]))
        self.set_option(OPT_TAU, ctypes.c_double(tau))
        self.set_option(OPT_SVD, ctypes.c_int32(SVD[svd]))
        if stream is not None:
            self.set_option(OPT_STREAM, ctypes.c_void_p(stream.cuda_stream))

    def set_option(self, key: int, value) -> None:
        _check(lib().ttice_set_option(self._h, key, ctypes.byref(value)), "ttice_set_option")

    def _batch(self, Y: torch.Tensor) -> torch.Tensor:
        if not Y.is_cuda:
            raise ValueError("batch must be a device tensor")
        if self.stream is None:
            # the library's work is ordered after the caller's on torch's current stream
            self.set_option(OPT_STREAM, ctypes.c_void_p(torch.cuda.current_stream(Y.device).cuda_stream))
        if tuple(Y.shape) == self.dims:
            Y = Y.unsqueeze(0)
        if tuple(Y.shape[1:]) != self.dims:
            raise ValueError(f"batch shape {tuple(Y.shape)} does not match dims {self.dims}")
        return Y.contiguous()

    def update(self, Y: torch.Tensor) -> dict:
        Y = self._batch(Y)
        info = UpdateInfo()
        _check(lib().ttice_update(self._h, ctypes.c_void_p(Y.data_ptr()), Y.shape[0],
                                  _dtype_code(Y.dtype), ctypes.byref(info)), "ttice_update")
        return info.as_dict()

    def project(self, Y: torch.Tensor):
        """(coef [n, r_d], err2 [n], y2 [n]) under the current cores (no update)."""
        Y = self._batch(Y)
        n = Y.shape[0]
        rd = self.ranks()[self.d]
        coef = torch.empty((n, max(rd, 1)), dtype=torch.float64, device=Y.device)
        err2 = torch.empty(n, dtype=torch.float64, device=Y.device)
        y2 = torch.empty(n, dtype=torch.float64, device=Y.device)
        _check(lib().ttice_project(self._h, ctypes.c_void_p(Y.data_ptr()), n, _dtype_code(Y.dtype),
                                   ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(err2.data_ptr()),
                                   ctypes.c_void_p(y2.data_ptr())), "ttice_project")
        return coef[:, :rd], err2, y2

    def project_noalloc(self, Y: torch.Tensor, coef: torch.Tensor, err2: Optional[torch.Tensor] = None,
                        y2: Optional[torch.Tensor] = None) -> None:
        """ttice_project_noalloc into caller buffers: coef [n, max(r_d, 1)] FP64,
        err2 / y2 [n] FP64 or None (the library allocates nothing)."""
        if not Y.is_cuda or not Y.is_contiguous() or tuple(Y.shape[1:]) != self.dims:
            raise ValueError("batch must be a contiguous device tensor of shape (n, *dims)")
        n = Y.shape[0]
        rd = max(self.ranks()[self.d], 1)
        if coef.dtype != torch.float64 or not coef.is_contiguous() or coef.numel() < n * rd:
            raise ValueError("coef must be a contiguous FP64 buffer of n * max(r_d, 1) values")
        for t in (err2, y2):
            if t is not None and (t.dtype != torch.float64 or t.numel() < n):
                raise ValueError("err2 / y2 must be FP64 buffers of n values")
        ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)
        _check(lib().ttice_project_noalloc(self._h, ctypes.c_void_p(Y.data_ptr()), n, _dtype_code(Y.dtype),
                                           ptr(coef), ptr(err2), ptr(y2)), "ttice_project_noalloc")

    def reconstruct(self, first: int = 0, count: Optional[int] = None,
                    dtype: torch.dtype = torch.float64, device=None) -> torch.Tensor:
        if count is None:
            count = self.n_total - first
        out = torch.empty((count,) + self.dims, dtype=dtype,
                          device=device if device is not None else torch.device("cuda"))
        _output_ready(out)
        _check(lib().ttice_reconstruct(self._h, first, count, ctypes.c_void_p(out.data_ptr()),
                                       _dtype_code(dtype)), "ttice_reconstruct")
        return out

    def ranks(self) -> List[int]:
        r = (ctypes.c_int64 * (self.d + 2))()
        n = ctypes.c_int64()
        _check(lib().ttice_ranks(self._h, r, ctypes.byref(n)), "ttice_ranks")
        return list(r)

    @property
    def n_total(self) -> int:
        r = (ctypes.c_int64 * (self.d + 2))()
        n = ctypes.c_int64()
        _check(lib().ttice_ranks(self._h, r, ctypes.byref(n)), "ttice_ranks")
        return int(n.value)

    def core(self, i: int) -> torch.Tensor:
        """Core i (0..d-1: U_{i+1}, (r_i n_{i+1}) x r_{i+1}); i == d: last core transposed."""
        rows, cols = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ttice_get_core(self._h, i, None, ctypes.byref(rows), ctypes.byref(cols)), "ttice_get_core")
        out = torch.empty((rows.value, cols.value), dtype=torch.float64, device="cuda")
        if out.numel():
            _output_ready(out)
            _check(lib().ttice_get_core(self._h, i, ctypes.c_void_p(out.data_ptr()), None, None), "ttice_get_core")
        return out

    def save(self) -> bytes:
        """Checkpoint image of the state (ttice_save)."""
        n = ctypes.c_int64()
        _check(lib().ttice_save(self._h, None, 0, ctypes.byref(n)), "ttice_save")
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().ttice_save(self._h, buf, n.value, ctypes.byref(n)), "ttice_save")
        return buf.raw

    @classmethod
    def load(cls, image: bytes, stream: Optional[torch.cuda.Stream] = None) -> "TTICE":
        """A new state on the current device from a checkpoint image (ttice_load)."""
        L = lib()
        h = ctypes.c_void_p()
        _check(L.ttice_load(image, len(image), ctypes.byref(h)), "ttice_load")
        d = ctypes.c_int32()
        dims = (ctypes.c_int64 * TTICE_MAX_D)()
        eps = ctypes.c_double()
        _check(L.ttice_shape(h, ctypes.byref(d), dims, ctypes.byref(eps)), "ttice_shape")
        self = cls.__new__(cls)
        self.dims = tuple(int(dims[i]) for i in range(d.value))
        self.d = d.value
        self.eps = float(eps.value)
        self._h = h
        self.stream = stream
        if stream is not None:
            self.set_option(OPT_STREAM, ctypes.c_void_p(stream.cuda_stream))
        return self

    def reserve(self, max_batch: int) -> None:
        """Allocate the workspace of increments up to max_batch tensors now."""
        _check(lib().ttice_reserve(self._h, int(max_batch)), "ttice_reserve")

    def profile(self, on: bool = True) -> None:
        """Time the profiled kernels with HIP events (resets the counters)."""
        self.set_option(OPT_PROFILE, ctypes.c_int32(1 if on else 0))

    def kernel_stats(self, kernel: int = KERNEL_PROJ_L1) -> dict:
        ks = KernelStats()
        _check(lib().ttice_get_kernel_stats(self._h, kernel, ctypes.byref(ks)), "ttice_get_kernel_stats")
        return dict(launches=int(ks.launches), total_ms=float(ks.total_ms), bytes=float(ks.bytes))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            if self._owner:
                lib().ttice_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Many independent TT-ICE streams on one device (ttice_server_*): a
    native scheduler with `workers` threads, each on its own HIP stream."""

    def __init__(self, workers: int = 4, budget_bytes: int = 64 << 30):
        h = ctypes.c_void_p()
        _check(lib().ttice_server_create(int(workers), int(budget_bytes), ctypes.byref(h)), "ttice_server_create")
        self._h = h
        self._streams = {}
        self._inflight = {}  # ticket -> batch tensor kept alive until completion

    def add_stream(self, dims: Sequence[int], eps: float, prec: str = "fp64", algo: str = "plain",
                   max_batch: int = 64, max_tensors: int = 4096) -> int:
        """A new stream (admitted now, or once removed streams free budget)."""
        dims = tuple(int(n) for n in dims)
        arr = (ctypes.c_int64 * len(dims))(*dims)
        sid = ctypes.c_int32()
        _check(lib().ttice_server_add_stream(self._h, len(dims), arr, float(eps), PREC[prec], ALGO[algo],
                                             int(max_batch), int(max_tensors), ctypes.byref(sid)),
               "ttice_server_add_stream")
        self._streams[sid.value] = (dims, float(eps))
        return sid.value

    def submit(self, sid: int, Y: torch.Tensor) -> int:
        dims = self._streams[sid][0]
        if not Y.is_cuda:
            raise ValueError("batch must be a device tensor")
        if tuple(Y.shape) == dims:
            Y = Y.unsqueeze(0)
        if tuple(Y.shape[1:]) != dims:
            raise ValueError(f"batch shape {tuple(Y.shape)} does not match dims {dims}")
        Y = Y.contiguous()
        t = ctypes.c_int64()
        # the update reads Y after the work queued so far on torch's current stream
        producer = ctypes.c_void_p(torch.cuda.current_stream(Y.device).cuda_stream)
        _check(lib().ttice_server_submit(self._h, int(sid), ctypes.c_void_p(Y.data_ptr()), Y.shape[0],
                                         _dtype_code(Y.dtype), producer, ctypes.byref(t)), "ttice_server_submit")
        self._inflight[t.value] = Y
        return t.value

    def poll(self, ticket: int):
        """(done, status, info) without blocking; info is None until done."""
        done, status, info = ctypes.c_int32(), ctypes.c_int32(), UpdateInfo()
        _check(lib().ttice_server_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(status),
                                       ctypes.byref(info)), "ttice_server_poll")
        if not done.value:
            return False, None, None
        self._inflight.pop(ticket, None)
        return True, status.value, info.as_dict()

    def wait(self, ticket: int):
        """(status, info) once the ticket completes."""
        status, info = ctypes.c_int32(), UpdateInfo()
        _check(lib().ttice_server_wait(self._h, int(ticket), ctypes.byref(status), ctypes.byref(info)),
               "ttice_server_wait")
        self._inflight.pop(ticket, None)
        return status.value, info.as_dict()

    def stream(self, sid: int) -> TTICE:
        """The stream's state for read-only calls (its queue must have drained)."""
        h = ctypes.c_void_p()
        _check(lib().ttice_server_stream_state(self._h, int(sid), ctypes.byref(h)), "ttice_server_stream_state")
        dims, eps = self._streams[sid]
        return TTICE._borrowed(h, dims, eps)

    def remove_stream(self, sid: int) -> None:
        _check(lib().ttice_server_remove_stream(self._h, int(sid)), "ttice_server_remove_stream")
        self._streams.pop(sid, None)

    def stats(self) -> dict:
        c = ServerCounters()
        _check(lib().ttice_server_stats(self._h, ctypes.byref(c)), "ttice_server_stats")
        return {name: getattr(c, name) for name, _ in ServerCounters._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ttice_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._inflight.clear()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
