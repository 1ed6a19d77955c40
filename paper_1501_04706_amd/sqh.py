"""ctypes binding of libsqh.so (argument marshalling only).

The functions ``sqh_create`` ... ``sqh_strerror`` mirror the C ABI in
``include/sqh.h`` one to one; device buffers are passed as torch CUDA (HIP)
tensors and the stream as a torch stream. Every step of the hull runs in the
library's HIP kernels; nothing here computes geometry, and there is no CPU
fallback: ``load()`` raises if the library has not been built.

``hull`` / ``hull_batched`` are conveniences that allocate the workspace and
outputs with torch and call the C functions.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SQH_LIB may name another build of the same library (A/B measurements)
LIB_PATH = os.environ.get("SQH_LIB") or os.path.join(HERE, "libsqh.so")

SQH_OK = 0
SQH_EINVAL = -1
SQH_ENOMEM = -2
SQH_ECAPACITY = -3
SQH_EDEVICE = -4
SQH_EBUSY = -5
SQH_ENOTFOUND = -6
SQH_FP32_FILTER = 0
SQH_FP64_ONLY = 1

_lib = None


class SqhError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = f"sqh error {code}"
        if _lib is not None:
            msg += f": {_lib.sqh_strerror(code).decode()}"
        if what:
            msg = f"{what}: {msg}"
        super().__init__(msg)


SQH_MAX_TIMED_PASSES = 64


class SqhStats(ctypes.Structure):
    _fields_ = [
        ("passes", ctypes.c_int64),
        ("points", ctypes.c_int64),
        ("first_survivors", ctypes.c_int64),
        ("survivors_total", ctypes.c_int64),
        ("orient_evals", ctypes.c_int64),
        ("orient_exact", ctypes.c_int64),
        ("cmp_exact", ctypes.c_int64),
        ("hull_size", ctypes.c_int64),
        ("max_segments", ctypes.c_int64),
        ("ms_total", ctypes.c_double),
        ("ms_seed", ctypes.c_double),
        ("ms_split", ctypes.c_double),
        ("ms_first", ctypes.c_double),
        ("ms_pass", ctypes.c_double),
        ("ms_table", ctypes.c_double),
        ("ms_emit", ctypes.c_double),
        ("pass_points", ctypes.c_int64 * SQH_MAX_TIMED_PASSES),
        ("pass_segments", ctypes.c_int64 * SQH_MAX_TIMED_PASSES),
        ("pass_ms", ctypes.c_double * SQH_MAX_TIMED_PASSES),
    ]

    def as_dict(self) -> dict:
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            if k.startswith("pass_"):
                v = list(v)[: min(self.passes, SQH_MAX_TIMED_PASSES)]
            d[k] = v
        return d


def load() -> ctypes.CDLL:
    """Load libsqh.so (built in-tree by ``paper_1501_04706_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1501_04706_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    lib.sqh_create.argtypes = [ctypes.POINTER(vp), c_int]
    lib.sqh_create.restype = c_int
    lib.sqh_destroy.argtypes = [vp]
    lib.sqh_destroy.restype = None
    lib.sqh_set_precision.argtypes = [vp, c_int]
    lib.sqh_set_precision.restype = c_int
    lib.sqh_workspace_bytes.argtypes = [i64, i64]
    lib.sqh_workspace_bytes.restype = ctypes.c_size_t
    lib.sqh_hull.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(i64), vp, ctypes.c_size_t, vp]
    lib.sqh_hull.restype = c_int
    lib.sqh_hull_batched.argtypes = [vp, vp, vp, i64, i64, vp, vp, i64, ctypes.POINTER(i64), vp,
                                     ctypes.c_size_t, vp]
    lib.sqh_hull_batched.restype = c_int
    lib.sqh_get_stats.argtypes = [vp, ctypes.POINTER(SqhStats)]
    lib.sqh_get_stats.restype = c_int
    lib.sqh_get_trace.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), c_int]
    lib.sqh_get_trace.restype = c_int
    lib.sqh_strerror.argtypes = [c_int]
    lib.sqh_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


# ---- one-to-one wrappers of the C ABI ----

def sqh_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    rc = load().sqh_create(ctypes.byref(h), device)
    if rc != SQH_OK:
        raise SqhError(rc, "sqh_create")
    return h.value


def sqh_destroy(ctx: int) -> None:
    load().sqh_destroy(ctx)


def sqh_set_precision(ctx: int, mode: int) -> int:
    return load().sqh_set_precision(ctx, mode)


def sqh_workspace_bytes(n_total: int, n_sets: int = 1) -> int:
    return int(load().sqh_workspace_bytes(n_total, n_sets))


def sqh_hull(ctx: int, xy, n: int, out, out_cap: int, ws, ws_bytes: int, stream=None):
    """Returns (return code, h)."""
    h = ctypes.c_int64(0)
    rc = load().sqh_hull(ctx, _ptr(xy), n, _ptr(out), out_cap, ctypes.byref(h), _ptr(ws), ws_bytes,
                         _stream_handle(stream))
    return rc, h.value


def sqh_hull_batched(ctx: int, xy, set_off, n_sets: int, n_total: int, out, out_off, out_cap: int, ws,
                     ws_bytes: int, stream=None):
    """Returns (return code, total h)."""
    h = ctypes.c_int64(0)
    rc = load().sqh_hull_batched(ctx, _ptr(xy), _ptr(set_off), n_sets, n_total, _ptr(out), _ptr(out_off),
                                 out_cap, ctypes.byref(h), _ptr(ws), ws_bytes, _stream_handle(stream))
    return rc, h.value


def sqh_get_stats(ctx: int) -> dict:
    st = SqhStats()
    rc = load().sqh_get_stats(ctx, ctypes.byref(st))
    if rc != SQH_OK:
        raise SqhError(rc, "sqh_get_stats")
    return st.as_dict()


def sqh_get_trace(ctx: int, max_entries: int = 8 * 512) -> list:
    buf = (ctypes.c_uint64 * max_entries)()
    n = load().sqh_get_trace(ctx, buf, max_entries)
    if n < 0:
        raise SqhError(n, "sqh_get_trace")
    return list(buf[:n])


def sqh_strerror(code: int) -> str:
    return load().sqh_strerror(code).decode()


# ---- conveniences ----

class Hull:
    """A context plus a reusable torch-allocated workspace."""

    def __init__(self, device: int = 0, precision: int = SQH_FP32_FILTER):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = sqh_create(device)
        rc = sqh_set_precision(self.ctx, precision)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_set_precision")
        self.ws = None

    def close(self):
        if self.ctx:
            sqh_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, mode: int):
        rc = sqh_set_precision(self.ctx, mode)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_set_precision")

    def workspace(self, n_total: int, n_sets: int = 1):
        need = sqh_workspace_bytes(n_total, n_sets)
        if need == 0:
            raise SqhError(SQH_EINVAL, "sqh_workspace_bytes")
        if self.ws is None or self.ws.numel() < need:
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self.ws

    def hull(self, xy, out=None, stream=None):
        """xy: (n, 2) float32 device tensor -> int32 device tensor of hull indices."""
        torch = self.torch
        xy = xy.contiguous()
        n = xy.shape[0]
        ws = self.workspace(n, 1)
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        rc, h = sqh_hull(self.ctx, xy, n, out, out.numel(), ws, ws.numel(), stream)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_hull")
        return out[:h]

    def hull_batched(self, xy, set_off, out=None, stream=None):
        """xy: (N, 2) float32; set_off: int64 (nsets+1) device tensor.
        Returns (out int32 (H,), out_off int64 (nsets+1,)) device tensors."""
        torch = self.torch
        xy = xy.contiguous()
        n_total = xy.shape[0]
        nsets = set_off.numel() - 1
        ws = self.workspace(n_total, nsets)
        if out is None:
            out = torch.empty(max(n_total, 1), dtype=torch.int32, device=self.device)
        out_off = torch.empty(nsets + 1, dtype=torch.int64, device=self.device)
        rc, h = sqh_hull_batched(self.ctx, xy, set_off, nsets, n_total, out, out_off, out.numel(), ws,
                                 ws.numel(), stream)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_hull_batched")
        return out[:h], out_off

    def stats(self) -> dict:
        return sqh_get_stats(self.ctx)
