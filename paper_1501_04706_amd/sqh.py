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
SQH_PREFILTER_NONE = 0
SQH_PREFILTER_QUAD = 1
SQH_PREFILTER_OCTAGON = 2
SQH_VARIANT_PARTITION = 0
SQH_VARIANT_SORTED = 1
SQH_FP32_FILTER = 0
SQH_FP64_ONLY = 1
SQH_FP32_SEMISTATIC = 2

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
        ("ms_kernel", ctypes.c_double),
        ("ms_seed", ctypes.c_double),
        ("ms_split", ctypes.c_double),
        ("ms_first", ctypes.c_double),
        ("ms_pass", ctypes.c_double),
        ("ms_emit", ctypes.c_double),
        ("ms_prefilter", ctypes.c_double),
        ("prefilter_points", ctypes.c_int64),
        ("pass_points", ctypes.c_int64 * SQH_MAX_TIMED_PASSES),
        ("pass_segments", ctypes.c_int64 * SQH_MAX_TIMED_PASSES),
        ("pass_ms", ctypes.c_double * SQH_MAX_TIMED_PASSES),
        ("ms_sort", ctypes.c_double),
        ("sorted_points", ctypes.c_int64),
        ("sort_violations", ctypes.c_int64),
        ("stream_path", ctypes.c_int64),
        ("line_filter", ctypes.c_int64),
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
    lib.sqh_set_prefilter.argtypes = [vp, c_int]
    lib.sqh_set_prefilter.restype = c_int
    lib.sqh_set_variant.argtypes = [vp, c_int]
    lib.sqh_set_variant.restype = c_int
    lib.sqh_set_streaming.argtypes = [vp, c_int]
    lib.sqh_set_streaming.restype = c_int
    lib.sqh_workspace_bytes_soa.argtypes = [i64]
    lib.sqh_workspace_bytes_soa.restype = ctypes.c_size_t
    lib.sqh_hull_soa.argtypes = [vp, vp, vp, i64, vp, i64, ctypes.POINTER(i64), vp, ctypes.c_size_t, vp]
    lib.sqh_hull_soa.restype = c_int
    lib.sqh_diag_orient.argtypes = [vp, i64, c_int, vp, vp, vp, vp]
    lib.sqh_diag_orient.restype = c_int
    lib.sqh_diag_compare.argtypes = [vp, vp, i64, c_int, vp, vp]
    lib.sqh_diag_compare.restype = c_int
    lib.sqh_diag_scan.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.sqh_diag_scan.restype = c_int
    lib.sqh_set_launch_timing.argtypes = [vp, c_int, ctypes.c_char_p]
    lib.sqh_set_launch_timing.restype = c_int
    lib.sqh_get_launch_times.argtypes = [vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                         c_int]
    lib.sqh_get_launch_times.restype = c_int
    lib.sqh_workspace_bytes.argtypes = [i64, i64]
    lib.sqh_workspace_bytes.restype = ctypes.c_size_t
    lib.sqh_hull.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(i64), vp, ctypes.c_size_t, vp]
    lib.sqh_hull.restype = c_int
    lib.sqh_hull_noalloc.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(i64), vp]
    lib.sqh_hull_noalloc.restype = c_int
    lib.sqh_hull_batched.argtypes = [vp, vp, vp, i64, i64, vp, vp, i64, ctypes.POINTER(i64), vp,
                                     ctypes.c_size_t, vp]
    lib.sqh_hull_batched.restype = c_int
    lib.sqh_get_stats.argtypes = [vp, ctypes.POINTER(SqhStats)]
    lib.sqh_get_stats.restype = c_int
    lib.sqh_get_trace.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), c_int]
    lib.sqh_get_trace.restype = c_int
    lib.sqh_strerror.argtypes = [c_int]
    lib.sqh_strerror.restype = ctypes.c_char_p
    lib.sqh_autotune.argtypes = [vp, vp, vp, i64, i64, vp, vp, i64, vp, ctypes.c_size_t, vp, c_int]
    lib.sqh_autotune.restype = c_int
    lib.sqh_get_tuning.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.sqh_get_tuning.restype = c_int
    lib.sqh_set_tuning.argtypes = [vp, ctypes.c_char_p]
    lib.sqh_set_tuning.restype = c_int
    lib.sqh_graph_create.argtypes = [vp, vp, vp, i64, i64, vp, vp, i64, vp, ctypes.c_size_t,
                                     ctypes.POINTER(vp)]
    lib.sqh_graph_create.restype = c_int
    lib.sqh_graph_launch.argtypes = [vp, vp]
    lib.sqh_graph_launch.restype = c_int
    lib.sqh_graph_result.argtypes = [vp, ctypes.POINTER(i64), vp]
    lib.sqh_graph_result.restype = c_int
    lib.sqh_graph_destroy.argtypes = [vp]
    lib.sqh_graph_destroy.restype = None
    lib.sqh_engine_bytes.argtypes = [i64, i64, i64]
    lib.sqh_engine_bytes.restype = ctypes.c_size_t
    lib.sqh_engine_create.argtypes = [vp, vp, ctypes.c_size_t, i64, i64, i64, ctypes.POINTER(vp)]
    lib.sqh_engine_create.restype = c_int
    lib.sqh_engine_destroy.argtypes = [vp]
    lib.sqh_engine_destroy.restype = None
    lib.sqh_engine_admit.argtypes = [vp, vp, i64, ctypes.c_uint64, c_int, vp]
    lib.sqh_engine_admit.restype = c_int
    lib.sqh_engine_step.argtypes = [vp, c_int, vp]
    lib.sqh_engine_step.restype = c_int
    lib.sqh_engine_launch.argtypes = [vp, c_int, vp]
    lib.sqh_engine_launch.restype = c_int
    lib.sqh_engine_finish.argtypes = [vp]
    lib.sqh_engine_finish.restype = c_int
    lib.sqh_engine_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), vp, i64, ctypes.POINTER(i64)]
    lib.sqh_engine_poll.restype = c_int
    lib.sqh_engine_status.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64)]
    lib.sqh_engine_status.restype = c_int
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


def sqh_set_prefilter(ctx: int, mode: int) -> int:
    return load().sqh_set_prefilter(ctx, mode)


def sqh_set_variant(ctx: int, variant: int) -> int:
    return load().sqh_set_variant(ctx, variant)


def sqh_set_streaming(ctx: int, on: int) -> int:
    return load().sqh_set_streaming(ctx, on)


def sqh_workspace_bytes_soa(n: int) -> int:
    return load().sqh_workspace_bytes_soa(n)


def sqh_hull_soa(ctx: int, x, y, n: int, out, out_cap: int, ws, ws_bytes: int, stream=None):
    h = ctypes.c_int64(0)
    rc = load().sqh_hull_soa(ctx, _ptr(x), _ptr(y), n, _ptr(out), out_cap, ctypes.byref(h), _ptr(ws), ws_bytes,
                             _stream_handle(stream))
    return rc, h.value


def sqh_diag_orient(tri, n: int, fp64_only: int, sign, vals, flags, stream=None) -> int:
    return load().sqh_diag_orient(_ptr(tri), n, fp64_only, _ptr(sign), _ptr(vals), _ptr(flags),
                                  _stream_handle(stream))


def sqh_diag_compare(cases, ids, n: int, fp64_only: int, out, stream=None) -> int:
    return load().sqh_diag_compare(_ptr(cases), _ptr(ids), n, fp64_only, _ptr(out), _stream_handle(stream))


def sqh_diag_scan(x, n: int, ex_a, ex_b, tot, stream=None) -> int:
    return load().sqh_diag_scan(_ptr(x), n, _ptr(ex_a), _ptr(ex_b), _ptr(tot), _stream_handle(stream))


def sqh_set_launch_timing(ctx: int, on: int, only: str | None = None) -> int:
    return load().sqh_set_launch_timing(ctx, on, only.encode() if only else None)


def sqh_get_launch_times(ctx: int, cap: int = 32) -> list:
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    n = load().sqh_get_launch_times(ctx, names, ms, cap)
    if n < 0:
        raise SqhError(n, "sqh_get_launch_times")
    return [(names[i].decode(), ms[i]) for i in range(n)]


def sqh_workspace_bytes(n_total: int, n_sets: int = 1) -> int:
    return int(load().sqh_workspace_bytes(n_total, n_sets))


def sqh_hull(ctx: int, xy, n: int, out, out_cap: int, ws, ws_bytes: int, stream=None):
    """Returns (return code, h)."""
    h = ctypes.c_int64(0)
    rc = load().sqh_hull(ctx, _ptr(xy), n, _ptr(out), out_cap, ctypes.byref(h), _ptr(ws), ws_bytes,
                         _stream_handle(stream))
    return rc, h.value


def sqh_hull_noalloc(ctx: int, xy, n: int, out, out_cap: int, stream=None):
    """Returns (return code, h)."""
    h = ctypes.c_int64(0)
    rc = load().sqh_hull_noalloc(ctx, _ptr(xy), n, _ptr(out), out_cap, ctypes.byref(h), _stream_handle(stream))
    return rc, h.value


SQH_NOALLOC_MAX_POINTS = 262144


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


def sqh_autotune(ctx: int, xy, set_off, n_sets: int, n_total: int, out, out_off, out_cap: int, ws,
                 ws_bytes: int, stream=None, reps: int = 3) -> int:
    return load().sqh_autotune(ctx, _ptr(xy), _ptr(set_off), n_sets, n_total, _ptr(out), _ptr(out_off),
                               out_cap, _ptr(ws), ws_bytes, _stream_handle(stream), reps)


def sqh_get_tuning(ctx: int) -> str:
    lib = load()
    need = lib.sqh_get_tuning(ctx, None, 0)
    if need < 0:
        raise SqhError(need, "sqh_get_tuning")
    buf = ctypes.create_string_buffer(need)
    lib.sqh_get_tuning(ctx, buf, need)
    return buf.value.decode()


def sqh_set_tuning(ctx: int, text: str) -> int:
    return load().sqh_set_tuning(ctx, text.encode())


def sqh_graph_create(ctx: int, xy, set_off, n_sets: int, n_total: int, out, out_off, out_cap: int, ws,
                     ws_bytes: int):
    """Returns (return code, graph handle)."""
    g = ctypes.c_void_p()
    rc = load().sqh_graph_create(ctx, _ptr(xy), _ptr(set_off), n_sets, n_total, _ptr(out), _ptr(out_off),
                                 out_cap, _ptr(ws), ws_bytes, ctypes.byref(g))
    return rc, g.value


def sqh_graph_launch(graph: int, stream=None) -> int:
    return load().sqh_graph_launch(graph, _stream_handle(stream))


def sqh_graph_result(graph: int, stream=None):
    """Returns (return code, total h)."""
    h = ctypes.c_int64(0)
    rc = load().sqh_graph_result(graph, ctypes.byref(h), _stream_handle(stream))
    return rc, h.value


def sqh_graph_destroy(graph: int) -> None:
    load().sqh_graph_destroy(graph)


def sqh_engine_bytes(slots: int, max_requests: int, stage_points: int) -> int:
    return int(load().sqh_engine_bytes(slots, max_requests, stage_points))


def sqh_engine_create(ctx: int, arena, arena_bytes: int, slots: int, max_requests: int, stage_points: int):
    """Returns (return code, engine handle)."""
    e = ctypes.c_void_p()
    rc = load().sqh_engine_create(ctx, _ptr(arena), arena_bytes, slots, max_requests, stage_points,
                                  ctypes.byref(e))
    return rc, e.value


def sqh_engine_destroy(engine: int) -> None:
    load().sqh_engine_destroy(engine)


def sqh_engine_admit(engine: int, xy, n: int, tag: int, stream=None) -> int:
    """xy: a (n, 2) float32 numpy array (host) or torch tensor (device or host)."""
    import numpy as np
    if isinstance(xy, np.ndarray):
        xy = np.ascontiguousarray(xy, dtype=np.float32)
        return load().sqh_engine_admit(engine, xy.ctypes.data if n > 0 else None, n, tag, 0,
                                       _stream_handle(stream))
    on_dev = 1 if xy.is_cuda else 0
    return load().sqh_engine_admit(engine, _ptr(xy) if n > 0 else None, n, tag, on_dev, _stream_handle(stream))


def sqh_engine_step(engine: int, max_passes: int, stream=None) -> int:
    return load().sqh_engine_step(engine, max_passes, _stream_handle(stream))


def sqh_engine_launch(engine: int, max_passes: int, stream=None) -> int:
    return load().sqh_engine_launch(engine, max_passes, _stream_handle(stream))


def sqh_engine_finish(engine: int) -> int:
    return load().sqh_engine_finish(engine)


def sqh_engine_poll(engine: int, h_out, cap: int):
    """h_out: host int32 numpy array of cap entries. Returns (rc, tag, h)."""
    tag = ctypes.c_uint64(0)
    h = ctypes.c_int64(0)
    rc = load().sqh_engine_poll(engine, ctypes.byref(tag), h_out.ctypes.data if cap > 0 else None, cap,
                                ctypes.byref(h))
    return rc, tag.value, h.value


def sqh_engine_status(engine: int):
    """Returns (rc, resident, staged, finished, free_slots)."""
    v = [ctypes.c_int64(0) for _ in range(4)]
    rc = load().sqh_engine_status(engine, *[ctypes.byref(x) for x in v])
    return (rc,) + tuple(x.value for x in v)


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

    def set_prefilter(self, mode: int):
        rc = sqh_set_prefilter(self.ctx, mode)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_set_prefilter")

    def set_launch_timing(self, on: bool, only: str | None = None):
        rc = sqh_set_launch_timing(self.ctx, 1 if on else 0, only)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_set_launch_timing")

    def launch_times(self) -> list:
        """[(kernel name, ms)] of the last call, launch timing on."""
        return sqh_get_launch_times(self.ctx)

    def set_streaming(self, on: bool):
        rc = sqh_set_streaming(self.ctx, 1 if on else 0)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_set_streaming")

    def set_variant(self, variant: int):
        rc = sqh_set_variant(self.ctx, variant)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_set_variant")

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

    def hull_soa(self, x, y, out=None, stream=None):
        """x, y: (n,) float32 device tensors -> int32 device tensor of hull indices."""
        torch = self.torch
        x = x.contiguous()
        y = y.contiguous()
        n = x.shape[0]
        need = sqh_workspace_bytes_soa(n)
        if need == 0:
            raise SqhError(SQH_EINVAL, "sqh_workspace_bytes_soa")
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        rc, h = sqh_hull_soa(self.ctx, x, y, n, out, out.numel(), self.ws, self.ws.numel(), stream)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_hull_soa")
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

    def autotune(self, xy, set_off=None, reps: int = 3, stream=None):
        """Time the candidate launch shapes on this problem and keep the best."""
        torch = self.torch
        xy = xy.contiguous()
        n_total = xy.shape[0]
        nsets = 1 if set_off is None else set_off.numel() - 1
        ws = self.workspace(n_total, nsets)
        out = torch.empty(max(n_total, 1), dtype=torch.int32, device=self.device)
        out_off = None if set_off is None else torch.empty(nsets + 1, dtype=torch.int64, device=self.device)
        rc = sqh_autotune(self.ctx, xy, set_off, nsets, n_total, out, out_off, out.numel(), ws, ws.numel(),
                          stream, reps)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_autotune")
        return sqh_get_tuning(self.ctx)

    def tuning(self) -> str:
        return sqh_get_tuning(self.ctx)

    def set_tuning(self, text: str):
        rc = sqh_set_tuning(self.ctx, text)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_set_tuning")

    def engine(self, slots: int, max_requests: int = 4096, stage_points: int | None = None) -> "Engine":
        return Engine(self, slots, max_requests, stage_points)

    def graph(self, xy, set_off=None):
        """A replayable HIP graph of one (batched) hull on fixed buffers."""
        return HullGraph(self, xy, set_off)


class Engine:
    """Continuous-batching serving engine over a torch-allocated arena."""

    def __init__(self, H: "Hull", slots: int, max_requests: int = 4096, stage_points: int | None = None):
        import numpy as np
        torch = H.torch
        self.H = H
        slots = (slots + 63) // 64 * 64
        stage_points = stage_points or slots
        need = sqh_engine_bytes(slots, max_requests, stage_points)
        if need == 0:
            raise SqhError(SQH_EINVAL, "sqh_engine_bytes")
        self.arena = torch.empty(need, dtype=torch.uint8, device=H.device)
        rc, self.e = sqh_engine_create(H.ctx, self.arena, need, slots, max_requests, stage_points)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_engine_create")
        self.slots = slots
        self.buf = np.empty(1 << 16, dtype=np.int32)

    def admit(self, xy, tag: int, stream=None) -> bool:
        """True if admitted, False if the engine has no room right now."""
        n = int(xy.shape[0])
        rc = sqh_engine_admit(self.e, xy, n, tag, stream)
        if rc == SQH_EBUSY:
            return False
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_engine_admit")
        return True

    def step(self, max_passes: int = 4, stream=None) -> int:
        rc = sqh_engine_step(self.e, max_passes, stream)
        if rc < 0:
            raise SqhError(rc, "sqh_engine_step")
        return rc

    def launch(self, max_passes: int = 4, stream=None) -> bool:
        """Enqueue a step; False if there is nothing to do."""
        rc = sqh_engine_launch(self.e, max_passes, stream)
        if rc == SQH_ENOTFOUND:
            return False
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_engine_launch")
        return True

    def finish(self) -> int:
        rc = sqh_engine_finish(self.e)
        if rc < 0:
            raise SqhError(rc, "sqh_engine_finish")
        return rc

    def poll(self):
        """Next finished request as (tag, hull int32 array or None if its input
        was invalid), or None if nothing is finished."""
        import numpy as np
        while True:
            rc, tag, h = sqh_engine_poll(self.e, self.buf, self.buf.size)
            if rc == SQH_ENOTFOUND:
                return None
            if rc == SQH_ECAPACITY:
                self.buf = np.empty(max(h, 2 * self.buf.size), dtype=np.int32)
                continue
            if rc == SQH_EINVAL:
                return tag, None
            if rc != SQH_OK:
                raise SqhError(rc, "sqh_engine_poll")
            return tag, self.buf[:h].copy()

    def status(self) -> dict:
        rc, res, stg, fin, free = sqh_engine_status(self.e)
        return {"ok": rc == SQH_OK, "resident": res, "staged": stg, "finished": fin, "free_slots": free}

    def close(self):
        if self.e:
            sqh_engine_destroy(self.e)
            self.e = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HullGraph:
    """Owns the buffers of one captured batched hull; launch() replays it."""

    def __init__(self, H: "Hull", xy, set_off=None):
        torch = H.torch
        self.H = H
        self.xy = xy.contiguous()
        self.n_total = self.xy.shape[0]
        self.set_off = set_off
        self.nsets = 1 if set_off is None else set_off.numel() - 1
        need = sqh_workspace_bytes(self.n_total, self.nsets)
        if need == 0:
            raise SqhError(SQH_EINVAL, "sqh_workspace_bytes")
        self.ws = torch.empty(need, dtype=torch.uint8, device=H.device)  # own workspace
        self.out = torch.empty(max(self.n_total, 1), dtype=torch.int32, device=H.device)
        self.out_off = torch.empty(self.nsets + 1, dtype=torch.int64, device=H.device)
        rc, self.g = sqh_graph_create(H.ctx, self.xy, set_off, self.nsets, self.n_total, self.out,
                                      self.out_off if set_off is not None else None, self.out.numel(),
                                      self.ws, self.ws.numel())
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_graph_create")

    def launch(self, stream=None):
        rc = sqh_graph_launch(self.g, stream)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_graph_launch")

    def result(self, stream=None):
        """Synchronise; returns (out[:h], out_off or None)."""
        rc, h = sqh_graph_result(self.g, stream)
        if rc != SQH_OK:
            raise SqhError(rc, "sqh_graph_result")
        return self.out[:h], (self.out_off if self.set_off is not None else None)

    def close(self):
        if self.g:
            sqh_graph_destroy(self.g)
            self.g = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
