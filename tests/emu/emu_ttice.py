"""ctypes wrapper of the host-emulation build of libttice (tests only).

Same C ABI as the product library, but "device" pointers are host memory
(NumPy arrays).  Import only in a process started with the AddressSanitizer
runtime preloaded (see tests/test_emu.py)."""
import ctypes
import os

import numpy as np

TTICE_MAX_D = 16


class ServerCounters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in ("reserved_bytes", "budget_bytes", "pending", "waiting_streams",
                                                    "groups", "grouped_increments")]


class UpdateInfo(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("skipped", ctypes.c_int32), ("n", ctypes.c_int64),
        ("used", ctypes.c_int64), ("n_total", ctypes.c_int64), ("norm_y2", ctypes.c_double),
        ("eps_core", ctypes.c_double), ("eps_upd", ctypes.c_double),
        ("ranks", ctypes.c_int64 * (TTICE_MAX_D + 2)), ("r_new", ctypes.c_int64 * TTICE_MAX_D),
        ("rho2", ctypes.c_double * TTICE_MAX_D), ("tail2", ctypes.c_double * TTICE_MAX_D),
        ("margin", ctypes.c_double * TTICE_MAX_D), ("achieved2", ctypes.c_double),
        ("solver", ctypes.c_int32 * TTICE_MAX_D),
    ]

    def as_dict(self):
        d = self.d
        return dict(n=self.n, used=self.used, n_total=self.n_total, skipped=bool(self.skipped),
                    normY2=self.norm_y2, eps_core=self.eps_core, eps_upd=self.eps_upd,
                    ranks=list(self.ranks[: d + 2]), rR=list(self.r_new[:d]), rho2=list(self.rho2[:d]),
                    tail2=list(self.tail2[:d]), margin=list(self.margin[:d]),
                    achieved2=(self.achieved2 if self.achieved2 >= 0 else None),
                    solver=list(self.solver[:d]))


class EmuError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"status {code}")
        self.code = code


def load(path):
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.ttice_create.argtypes = [i32, ctypes.POINTER(i64), dbl, ctypes.POINTER(vp)]
    L.ttice_set_option.argtypes = [vp, i32, vp]
    L.ttice_update.argtypes = [vp, vp, i64, i32, ctypes.POINTER(UpdateInfo)]
    L.ttice_reconstruct.argtypes = [vp, i64, i64, vp, i32]
    L.ttice_project.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    L.ttice_ranks.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.ttice_get_core.argtypes = [vp, i32, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.ttice_save.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
    L.ttice_load.argtypes = [vp, i64, ctypes.POINTER(vp)]
    L.ttice_shape.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    L.ttice_destroy.argtypes = [vp]
    L.ttice_destroy.restype = None
    L.hipemu_fail_alloc_after.argtypes = [ctypes.c_longlong]
    L.hipemu_fail_alloc_after.restype = None
    L.ttice_server_create.argtypes = [i32, i64, ctypes.POINTER(vp)]
    L.ttice_server_add_stream.argtypes = [vp, i32, ctypes.POINTER(i64), dbl, i32, i32, i64, i64, ctypes.POINTER(i32)]
    L.ttice_server_submit.argtypes = [vp, i32, vp, i64, i32, vp, ctypes.POINTER(i64)]
    L.ttice_server_poll.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(UpdateInfo)]
    L.ttice_server_wait.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(UpdateInfo)]
    L.ttice_server_stream_state.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.ttice_server_remove_stream.argtypes = [vp, i32]
    L.ttice_server_stats.argtypes = [vp, ctypes.POINTER(ServerCounters)]
    L.ttice_server_destroy.argtypes = [vp]
    L.ttice_server_destroy.restype = None
    return L


class EmuTTICE:
    @classmethod
    def borrowed(cls, L, handle, dims):
        """Read-only view of a state owned by a server stream."""
        self = cls.__new__(cls)
        self.L, self.dims, self.d, self.h, self.owner = L, tuple(dims), len(dims), handle, False
        return self

    owner = True

    def __init__(self, L, dims, eps, algo=0, prec=0, tau=None, skip_rule=None, svd=None):
        self.L = L
        self.dims = tuple(dims)
        self.d = len(dims)
        h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * self.d)(*dims)
        rc = L.ttice_create(self.d, arr, eps, ctypes.byref(h))
        if rc:
            raise EmuError(rc)
        self.h = h
        self._opt(2, ctypes.c_int32(algo))
        self._opt(1, ctypes.c_int32(prec))
        if tau is not None:
            self._opt(4, ctypes.c_double(tau))
        if skip_rule is not None:
            self._opt(3, ctypes.c_int32(skip_rule))
        if svd is not None:
            self._opt(7, ctypes.c_int32(svd))

    def save(self):
        n = ctypes.c_int64()
        rc = self.L.ttice_save(self.h, None, 0, ctypes.byref(n))
        if rc:
            raise EmuError(rc)
        buf = ctypes.create_string_buffer(n.value)
        rc = self.L.ttice_save(self.h, buf, n.value, ctypes.byref(n))
        if rc:
            raise EmuError(rc)
        return buf.raw

    @classmethod
    def load(cls, L, image):
        h = ctypes.c_void_p()
        rc = L.ttice_load(image, len(image), ctypes.byref(h))
        if rc:
            raise EmuError(rc)
        d = ctypes.c_int32()
        dims = (ctypes.c_int64 * TTICE_MAX_D)()
        eps = ctypes.c_double()
        L.ttice_shape(h, ctypes.byref(d), dims, ctypes.byref(eps))
        self = cls.__new__(cls)
        self.L, self.h = L, h
        self.dims = tuple(dims[i] for i in range(d.value))
        self.d = d.value
        self.eps = eps.value
        return self

    def _opt(self, k, v):
        rc = self.L.ttice_set_option(self.h, k, ctypes.byref(v))
        if rc:
            raise EmuError(rc)

    def update(self, Y):
        Y = np.ascontiguousarray(Y)
        code = 1 if Y.dtype == np.float64 else 0
        info = UpdateInfo()
        rc = self.L.ttice_update(self.h, Y.ctypes.data_as(ctypes.c_void_p), Y.shape[0], code, ctypes.byref(info))
        if rc:
            raise EmuError(rc)
        return info.as_dict()

    def ranks(self):
        r = (ctypes.c_int64 * (self.d + 2))()
        n = ctypes.c_int64()
        self.L.ttice_ranks(self.h, r, ctypes.byref(n))
        return list(r), n.value

    def reconstruct(self, first=0, count=None):
        _, nt = self.ranks()
        if count is None:
            count = nt - first
        out = np.zeros((count,) + self.dims)
        rc = self.L.ttice_reconstruct(self.h, first, count, out.ctypes.data_as(ctypes.c_void_p), 1)
        if rc:
            raise EmuError(rc)
        return out

    def project(self, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        r, _ = self.ranks()
        n = Y.shape[0]
        coef = np.zeros((n, max(r[self.d], 1)))
        err2 = np.zeros(n)
        y2 = np.zeros(n)
        rc = self.L.ttice_project(self.h, Y.ctypes.data_as(ctypes.c_void_p), n, 1,
                                  coef.ctypes.data_as(ctypes.c_void_p), err2.ctypes.data_as(ctypes.c_void_p),
                                  y2.ctypes.data_as(ctypes.c_void_p))
        if rc:
            raise EmuError(rc)
        return coef[:, : r[self.d]], err2, y2

    def core(self, i):
        rows, cols = ctypes.c_int64(), ctypes.c_int64()
        self.L.ttice_get_core(self.h, i, None, ctypes.byref(rows), ctypes.byref(cols))
        out = np.zeros((rows.value, cols.value))
        if out.size:
            self.L.ttice_get_core(self.h, i, out.ctypes.data_as(ctypes.c_void_p), None, None)
        return out

    def close(self):
        if self.h:
            if self.owner:
                self.L.ttice_destroy(self.h)
            self.h = None
