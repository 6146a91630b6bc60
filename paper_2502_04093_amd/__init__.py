"""Python binding of the IPComp MI355X library (``libipcomp.so``).

Thin ctypes wrappers with the names of the C ABI in ``include/ipcomp.h``;
every step of compression, retrieval and refinement runs in the library's HIP
kernels.  PyTorch supplies device memory (the field and output tensors) and
the HIP stream calls are ordered on.  There is no CPU fallback: if the library
is not built, importing the binding's entry points raises.
"""

from __future__ import annotations

import ctypes
import os
import weakref
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libipcomp.so")

IPC_F32, IPC_F64 = 0, 1
IPC_LINEAR, IPC_CUBIC = 0, 1
IPC_TARGET_EB, IPC_TARGET_BITRATE = 0, 1
IPC_TARGET_LEVEL_GROUPS = 0x100
IPC_FLAG_CLAMPED_TO_EB, IPC_FLAG_BUDGET_BELOW_MIN, IPC_FLAG_NOOP = 1, 2, 4
IPC_MAX_PASSES = 100
STATUS = {0: "IPC_OK", -1: "IPC_EINVAL", -2: "IPC_ENOMEM", -3: "IPC_ECORRUPT", -4: "IPC_EHIP",
          -5: "IPC_ESTATE", -6: "IPC_EUNSUPPORTED"}

c_void_p, c_int, c_uint8, c_uint32, c_uint64, c_double, c_float = (
    ctypes.c_void_p, ctypes.c_int, ctypes.c_uint8, ctypes.c_uint32, ctypes.c_uint64,
    ctypes.c_double, ctypes.c_float)


class ipc_target(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("value", c_double)]


class ipc_options(ctypes.Structure):
    _fields_ = [("interp", ctypes.c_int32), ("nonprog_levels", ctypes.c_int32),
                ("chunk_log2", c_uint8 * 3), ("errq_mode", c_uint8), ("lossless", c_uint8),
                ("reserved", c_uint8 * 3), ("debug_flags", c_uint32)]


IPC_ERRQ_EXACT, IPC_ERRQ_BOUND = 0, 1
IPC_LOSSLESS_ZWE, IPC_LOSSLESS_CODED = 0, 1
IPC_DEBUG_PER_PASS, IPC_DEBUG_VERIFY = 1, 2


def _options(interp: str, nonprog_levels: int, chunk_log2=None, errq_mode: str = "exact",
             lossless: str = "zwe", debug_flags: int = 0) -> ipc_options:
    if errq_mode not in ("exact", "bound") or lossless not in ("zwe", "coded"):
        raise ValueError("errq_mode is 'exact' or 'bound', lossless is 'zwe' or 'coded'")
    opts = ipc_options()
    opts.interp = IPC_CUBIC if interp == "cubic" else IPC_LINEAR
    opts.nonprog_levels = nonprog_levels
    if chunk_log2 is not None:
        for j, c in enumerate(chunk_log2):
            opts.chunk_log2[j] = c
    opts.errq_mode = IPC_ERRQ_BOUND if errq_mode == "bound" else IPC_ERRQ_EXACT
    opts.lossless = IPC_LOSSLESS_CODED if lossless == "coded" else IPC_LOSSLESS_ZWE
    opts.debug_flags = int(debug_flags)
    return opts


class ipc_info(ctypes.Structure):
    _fields_ = [("bound", c_double), ("bytes_loaded", c_uint64), ("bytes_total", c_uint64),
                ("bytes_read", c_uint64), ("n_passes", c_uint32), ("flags", c_uint32),
                ("plan", c_uint8 * IPC_MAX_PASSES), ("t_plan_ms", c_float),
                ("t_device_ms", c_float)]

    def plan_list(self):
        return [int(self.plan[i]) for i in range(self.n_passes)]


class ipc_pass_info(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_targets", c_uint64),
                ("n_chunks", c_uint64), ("plane_bytes", c_uint64 * 32), ("errq", c_uint32 * 33),
                ("progressive", c_uint32),
                ("launch_pass", c_uint32)]


class ipc_stream_desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("dims", ctypes.c_uint64 * 3), ("interp", ctypes.c_int32),
                ("nonprog_levels", ctypes.c_int32), ("abs_eb", ctypes.c_double),
                ("n_passes", ctypes.c_uint32), ("coding", ctypes.c_int32)]


class ipc_request(ctypes.Structure):
    _fields_ = [("stream", c_void_p), ("state", c_void_p), ("target", ipc_target),
                ("refine", ctypes.c_int32), ("status", ctypes.c_int32), ("info", ipc_info)]


P = ctypes.POINTER
SIGNATURES = {
    "ipc_ctx_create": (c_int, [c_int, c_void_p, P(c_void_p)]),
    "ipc_ctx_destroy": (None, [c_void_p]),
    "ipc_ctx_set_stream": (c_int, [c_void_p, c_void_p]),
    "ipc_compress": (c_int, [c_void_p, c_void_p, P(c_uint64), c_int, c_int, c_double,
                             P(ipc_options), P(c_void_p)]),
    "ipc_stream_size": (c_int, [c_void_p, P(c_uint64)]),
    "ipc_stream_describe": (c_int, [c_void_p, P(ipc_stream_desc)]),
    "ipc_stream_to_host": (c_int, [c_void_p, c_void_p, c_void_p, c_uint64]),
    "ipc_stream_from_host": (c_int, [c_void_p, c_void_p, c_uint64, c_int, P(c_void_p)]),
    "ipc_stream_free": (None, [c_void_p]),
    "ipc_stream_entropy_code": (c_int, [c_void_p, c_void_p]),
    "ipc_refine_additive": (c_int, [c_void_p, c_void_p, ipc_target, P(ipc_info)]),
    "ipc_stream_coding": (c_int, [c_void_p, P(c_int)]),
    "ipc_stream_passes": (c_int, [c_void_p, P(c_uint32)]),
    "ipc_stream_pass_info": (c_int, [c_void_p, c_uint32, P(ipc_pass_info)]),
    "ipc_retrieve": (c_int, [c_void_p, c_void_p, ipc_target, P(c_void_p), P(ipc_info)]),
    "ipc_retrieve_plan": (c_int, [c_void_p, c_void_p, P(c_uint8), c_uint32, P(c_void_p),
                                  P(ipc_info)]),
    "ipc_retrieve_noalloc": (c_int, [c_void_p, c_void_p, ipc_target, c_void_p, c_uint64,
                                     P(ipc_info)]),
    "ipc_state_field": (c_void_p, [c_void_p]),
    "ipc_state_copy_field": (c_int, [c_void_p, c_void_p, c_void_p, c_uint64]),
    "ipc_refine": (c_int, [c_void_p, c_void_p, ipc_target, P(ipc_info)]),
    "ipc_state_free": (None, [c_void_p]),
    "ipc_plan_host": (c_int, [c_void_p, c_uint64, ipc_target, P(c_uint8), P(c_uint8), c_uint32,
                              P(c_double), P(c_uint32), P(c_uint64)]),
    "ipc_compress_batch": (c_int, [c_void_p, c_uint32, P(c_void_p), P(c_uint64), c_int, c_int,
                                   P(c_double), P(ipc_options), P(c_void_p)]),
    "ipc_retrieve_batch": (c_int, [c_void_p, c_uint32, P(c_void_p), P(ipc_target), P(c_void_p),
                                   P(ipc_info)]),
    "ipc_autotune": (c_int, [c_void_p, c_void_p, P(c_uint64), c_int, c_int, c_double,
                             P(ipc_options), P(ctypes.c_int32), P(ctypes.c_int32), c_uint32]),
    "ipc_autotune_clear": (c_int, [c_void_p]),
    "ipc_autotune_set": (c_int, [c_void_p, P(c_uint64), c_int, c_int, c_int, P(ctypes.c_int32),
                                 P(ctypes.c_int32), c_uint32]),
    "ipc_serve_batch": (c_int, [c_void_p, c_uint32, P(ipc_request)]),
    "ipc_stream_field_bytes": (c_int, [c_void_p, P(c_uint64)]),
    "ipc_state_field_bytes": (c_int, [c_void_p, P(c_uint64)]),
    "ipc_server_create": (c_int, [c_void_p, c_uint64, c_uint32, P(c_void_p)]),
    "ipc_server_submit": (c_int, [c_void_p, c_void_p, c_void_p, ipc_target, P(c_uint64)]),
    "ipc_server_wait": (c_int, [c_void_p, c_uint64, ctypes.c_int64, P(c_void_p), P(ipc_info),
                                P(c_double)]),
    "ipc_server_release": (c_int, [c_void_p, c_void_p]),
    "ipc_server_lock": (c_int, [c_void_p]),
    "ipc_server_unlock": (c_int, [c_void_p]),
    "ipc_server_stats": (c_int, [c_void_p, P(c_uint64), P(c_uint64), P(c_uint64), P(c_uint64)]),
    "ipc_server_destroy": (None, [c_void_p]),
    "ipc_ctx_set_profiling": (c_int, [c_void_p, c_int, c_int]),
    "ipc_ctx_pass_times": (c_int, [c_void_p, P(c_float), c_uint32, P(c_uint32)]),
    "ipc_ctx_set_batch_graphs": (c_int, [c_void_p, c_int]),
    "ipc_autotune_batch": (c_int, [c_void_p, c_void_p, P(c_uint64), c_int, c_int, c_double, c_void_p,
                                   c_uint32, P(ctypes.c_int32)]),
    "ipc_ctx_graph_stats": (c_int, [c_void_p, P(c_uint64), P(c_uint64)]),
    "ipc_status_string": (ctypes.c_char_p, [c_int]),
    "ipc_last_error": (ctypes.c_char_p, [c_void_p]),
}

_lib = None


class IpcError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libipcomp.so not built ({LIB_PATH}); run "
                              "`python -m paper_2502_04093_amd.build` first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int, ctx=None):
    if st != 0:
        msg = lib().ipc_last_error(ctx).decode() if ctx else ""
        raise IpcError(st, msg)


def _target(eb: Optional[float], bitrate: Optional[float], level_groups: bool = False) -> ipc_target:
    """Error-bound or bitrate target; level_groups plans with one discarded-
    plane count per level (IPC_TARGET_LEVEL_GROUPS)."""
    if (eb is None) == (bitrate is None):
        raise ValueError("give exactly one of eb= and bitrate=")
    flag = IPC_TARGET_LEVEL_GROUPS if level_groups else 0
    if eb is not None:
        return ipc_target(IPC_TARGET_EB | flag, float(eb))
    return ipc_target(IPC_TARGET_BITRATE | flag, float(bitrate))


# PyBytes_FromStringAndSize(NULL, n): an uninitialized bytes object of n bytes
_new_bytes = ctypes.pythonapi.PyBytes_FromStringAndSize
_new_bytes.restype = ctypes.py_object
_new_bytes.argtypes = [c_void_p, ctypes.c_ssize_t]


def plan_host(stream_bytes: bytes, eb=None, bitrate=None, limit: Optional[Sequence[int]] = None,
              level_groups: bool = False):
    """Host-only planner: (plan, bound, flags, loaded_bytes) for a serialized stream."""
    L = lib()
    data = stream_bytes if isinstance(stream_bytes, bytes) else bytes(stream_bytes)
    buf = ctypes.cast(ctypes.c_char_p(data), c_void_p)  # read in place during the call
    out = (c_uint8 * IPC_MAX_PASSES)()
    lim = (c_uint8 * IPC_MAX_PASSES)(*limit) if limit is not None else None
    bound, flags, loaded = c_double(), c_uint32(), c_uint64()
    st = L.ipc_plan_host(buf, len(data), _target(eb, bitrate, level_groups), lim, out,
                         IPC_MAX_PASSES,
                         ctypes.byref(bound), ctypes.byref(flags), ctypes.byref(loaded))
    _check(st)
    return list(out), bound.value, flags.value, loaded.value


class Context:
    """ipc_ctx on a device.

    With no stream given, calls are ordered after torch's current stream: a
    non-default torch stream is handed to the library as is; for torch's
    default stream (the null stream, handle 0) the library issues work on a
    blocking stream of its own, which HIP orders after the work queued on the
    null stream (ipc_ctx_create with a NULL stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        handle = c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        p = c_void_p()
        _check(L.ipc_ctx_create(int(device), handle, ctypes.byref(p)))
        self._p = p
        self.device = device
        self._states = weakref.WeakSet()
        self._streams = weakref.WeakSet()

    def close(self):
        """Free every live state and stream of this context, then the context."""
        if getattr(self, "_p", None):
            for st in list(self._states):
                st.free()
            for s in list(self._streams):
                s.free()
            lib().ipc_ctx_destroy(self._p)
            self._p = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._p

    def set_profiling(self, on: bool = True, only_pass: int = -1):
        _check(lib().ipc_ctx_set_profiling(self._p, int(bool(on)), int(only_pass)), self._p)

    def set_batch_graphs(self, on=True):
        """Batches as queue launches replayed from captured HIP graphs: True
        (always), False (direct launches) or "auto" (the batch autotuner's
        choice, else by field size); see ipc_ctx_set_batch_graphs."""
        mode = 2 if on == "auto" else int(bool(on))
        _check(lib().ipc_ctx_set_batch_graphs(self._p, mode), self._p)

    def graph_stats(self):
        """(graphs captured, graph replays) so far."""
        c, r = c_uint64(), c_uint64()
        _check(lib().ipc_ctx_graph_stats(self._p, ctypes.byref(c), ctypes.byref(r)), self._p)
        return int(c.value), int(r.value)

    def pass_times(self):
        """Per-pass kernel milliseconds of the last call (profiling on)."""
        n = c_uint32()
        _check(lib().ipc_ctx_pass_times(self._p, None, 0, ctypes.byref(n)), self._p)
        arr = (c_float * max(1, n.value))()
        _check(lib().ipc_ctx_pass_times(self._p, arr, n.value, ctypes.byref(n)), self._p)
        return [float(arr[i]) for i in range(n.value)]

    def compress(self, field, eb: float, interp: str = "cubic", nonprog_levels: int = 0,
                 chunk_log2: Optional[Sequence[int]] = None, errq_mode: str = "exact",
                 lossless: str = "zwe", debug_flags: int = 0) -> "Stream":
        """ipc_compress; errq_mode 'exact' or 'bound' (IPC_ERRQ_*), lossless
        'zwe' or 'coded' (IPC_LOSSLESS_*), debug_flags IPC_DEBUG_*."""
        import torch
        if not (field.is_cuda and field.is_contiguous()):
            raise ValueError("field must be a contiguous device tensor")
        if field.dtype not in (torch.float32, torch.float64):
            raise TypeError("field must be float32 or float64")
        dims = (c_uint64 * field.dim())(*field.shape)
        opts = _options(interp, nonprog_levels, chunk_log2, errq_mode, lossless, debug_flags)
        out = c_void_p()
        dt = IPC_F32 if field.dtype == torch.float32 else IPC_F64
        _check(lib().ipc_compress(self._p, c_void_p(field.data_ptr()), dims, field.dim(), dt,
                                  float(eb), ctypes.byref(opts), ctypes.byref(out)), self._p)
        return Stream(self, out, tuple(field.shape), field.dtype)

    def autotune(self, field, eb: float, interp: str = "cubic"):
        """Tune the fused launches for this field's shape, dtype and
        interpolation; returns the chosen column lengths per level
        (compression, retrieval; index = level)."""
        import torch
        if not (field.is_cuda and field.is_contiguous()):
            raise ValueError("field must be a contiguous device tensor")
        dims = (c_uint64 * field.dim())(*field.shape)
        opts = ipc_options()
        opts.interp = IPC_CUBIC if interp == "cubic" else IPC_LINEAR
        zc = (ctypes.c_int32 * 32)()
        zr = (ctypes.c_int32 * 32)()
        dt = IPC_F32 if field.dtype == torch.float32 else IPC_F64
        _check(lib().ipc_autotune(self._p, c_void_p(field.data_ptr()), dims, field.dim(), dt,
                                  float(eb), ctypes.byref(opts), zc, zr, 32), self._p)
        return list(zc), list(zr)

    def autotune_batch(self, field, eb: float, copies: int = 2, interp: str = "cubic"):
        """Choose the batch schedule for this field's shape, dtype and
        interpolation (ipc_autotune_batch); returns {"compress": (graphs,
        workgroups per CU), "retrieve": (...)}."""
        import torch
        if not (field.is_cuda and field.is_contiguous()):
            raise ValueError("field must be a contiguous device tensor")
        dims = (c_uint64 * field.dim())(*field.shape)
        opts = ipc_options()
        opts.interp = IPC_CUBIC if interp == "cubic" else IPC_LINEAR
        ch = (ctypes.c_int32 * 4)()
        dt = IPC_F32 if field.dtype == torch.float32 else IPC_F64
        _check(lib().ipc_autotune_batch(self._p, c_void_p(field.data_ptr()), dims, field.dim(), dt,
                                        float(eb), ctypes.byref(opts), int(copies), ch), self._p)
        return {"compress": (bool(ch[0]), int(ch[1])), "retrieve": (bool(ch[2]), int(ch[3]))}

    def autotune_set(self, shape, dtype, zseg_c, zseg_r, interp: str = "cubic"):
        """Install column lengths (lists indexed by level, 0 = default) for a
        shape and torch dtype."""
        import torch
        n = max(len(zseg_c), len(zseg_r))
        zc = (ctypes.c_int32 * n)(*(list(zseg_c) + [0] * (n - len(zseg_c))))
        zr = (ctypes.c_int32 * n)(*(list(zseg_r) + [0] * (n - len(zseg_r))))
        dims = (c_uint64 * len(shape))(*shape)
        _check(lib().ipc_autotune_set(self._p, dims, len(shape),
                                      IPC_F32 if dtype == torch.float32 else IPC_F64,
                                      IPC_CUBIC if interp == "cubic" else IPC_LINEAR, zc, zr, n),
               self._p)

    def autotune_clear(self):
        _check(lib().ipc_autotune_clear(self._p), self._p)

    def compress_batch(self, fields, ebs, interp: str = "cubic", nonprog_levels: int = 0,
                       errq_mode: str = "exact", lossless: str = "zwe", debug_flags: int = 0,
                       chunk_log2: Optional[Sequence[int]] = None):
        """Compress several device tensors of one dtype and rank in one call
        (3-D and 2-D fields with the default chunks share one launch per
        level, other fields one launch per pass); returns a list of Streams."""
        import torch
        n = len(fields)
        if n == 0 or len(ebs) != n:
            raise ValueError("give one error bound per field")
        nd = fields[0].dim()
        dt = fields[0].dtype
        for f in fields:
            if not (f.is_cuda and f.is_contiguous()):
                raise ValueError("fields must be contiguous device tensors")
            if f.dim() != nd or f.dtype != dt:
                raise ValueError("fields of one batch share dtype and rank")
        if dt not in (torch.float32, torch.float64):
            raise TypeError("fields must be float32 or float64")
        ptrs = (c_void_p * n)(*[f.data_ptr() for f in fields])
        dims = (c_uint64 * (n * nd))(*[d for f in fields for d in f.shape])
        eba = (c_double * n)(*[float(e) for e in ebs])
        opts = _options(interp, nonprog_levels, chunk_log2, errq_mode, lossless, debug_flags)
        out = (c_void_p * n)()
        _check(lib().ipc_compress_batch(self._p, n, ptrs, dims, nd,
                                        IPC_F32 if dt == torch.float32 else IPC_F64, eba,
                                        ctypes.byref(opts), out), self._p)
        return [Stream(self, c_void_p(out[i]), tuple(fields[i].shape), dt) for i in range(n)]

    def retrieve_batch(self, streams, eb=None, bitrate=None):
        """Retrieve several streams of this context in one call (eb= or
        bitrate=: one value, or one per stream); returns a list of States."""
        n = len(streams)
        vals = eb if eb is not None else bitrate
        if not isinstance(vals, (list, tuple)):
            vals = [vals] * n
        tg = (ipc_target * n)(*[_target(v if eb is not None else None,
                                        v if bitrate is not None else None) for v in vals])
        ptrs = (c_void_p * n)(*[s._p.value if isinstance(s._p, c_void_p) else s._p for s in streams])
        out = (c_void_p * n)()
        infos = (ipc_info * n)()
        _check(lib().ipc_retrieve_batch(self._p, n, ptrs, tg, out, infos), self._p)
        return [State(streams[i], c_void_p(out[i]), infos[i]) for i in range(n)]

    def serve_batch(self, requests):
        """One mixed batch: requests are (Stream, None, target) retrievals or
        (None, State, target) refinements, target a dict like {"eb": 1e-3} or
        {"bitrate": 2.0}; returns per request (State, info, status)."""
        n = len(requests)
        arr = (ipc_request * n)()
        for k, (stream, state, tg) in enumerate(requests):
            arr[k].stream = stream._p if stream is not None else None
            arr[k].state = state._p if state is not None else None
            arr[k].refine = 1 if state is not None else 0
            arr[k].target = _target(tg.get("eb"), tg.get("bitrate"))
        _check(lib().ipc_serve_batch(self._p, n, arr), self._p)
        out = []
        for k, (stream, state, tg) in enumerate(requests):
            r = arr[k]
            if state is not None:
                if r.status == 0:
                    state.info = r.info
                out.append((state, r.info, r.status))
            else:
                st = State(stream, c_void_p(r.state), r.info) if r.status == 0 and r.state else None
                out.append((st, r.info, r.status))
        return out

    def stream_from_bytes(self, data: bytes, device_resident: bool = True) -> "Stream":
        """ipc_stream_from_host; device_resident=False keeps the bitplanes in
        pinned host memory that retrievals read in place."""
        out = c_void_p()
        if not isinstance(data, bytes):
            data = bytes(data)
        # the library only reads the bytes during the call: their own buffer,
        # not a copy
        src = ctypes.cast(ctypes.c_char_p(data), c_void_p)
        _check(lib().ipc_stream_from_host(self._p, src, len(data), int(bool(device_resident)),
                                          ctypes.byref(out)), self._p)
        return Stream.from_handle(self, out)


class Stream:
    """ipc_stream: a device-resident compressed field."""

    def __init__(self, ctx: Context, p, shape, dtype):
        self.ctx, self._p, self.shape, self.dtype = ctx, p, shape, dtype
        ctx._streams.add(self)

    @classmethod
    def from_handle(cls, ctx: Context, p) -> "Stream":
        """A Stream for a library handle, its shape and dtype from
        ipc_stream_describe."""
        import torch
        d = ipc_stream_desc()
        _check(lib().ipc_stream_describe(p, ctypes.byref(d)))
        shape = tuple(int(d.dims[j]) for j in range(d.ndim))
        return cls(ctx, p, shape, torch.float32 if d.dtype == IPC_F32 else torch.float64)

    def describe(self) -> dict:
        """ipc_stream_describe as a dict."""
        d = ipc_stream_desc()
        _check(lib().ipc_stream_describe(self._p, ctypes.byref(d)))
        return {"shape": tuple(int(d.dims[j]) for j in range(d.ndim)),
                "dtype": "f32" if d.dtype == IPC_F32 else "f64",
                "interp": "cubic" if d.interp == IPC_CUBIC else "linear",
                "nonprog_levels": int(d.nonprog_levels), "abs_eb": float(d.abs_eb),
                "n_passes": int(d.n_passes), "coding": int(d.coding)}

    def free(self):
        if getattr(self, "_p", None):
            for st in list(self.ctx._states):
                if st.stream is self:
                    st.free()
            lib().ipc_stream_free(self._p)
            self._p = None

    def __del__(self):  # pragma: no cover
        try:
            self.free()
        except Exception:
            pass

    @property
    def nbytes(self) -> int:
        n = c_uint64()
        _check(lib().ipc_stream_size(self._p, ctypes.byref(n)))
        return n.value

    @property
    def n_passes(self) -> int:
        n = c_uint32()
        _check(lib().ipc_stream_passes(self._p, ctypes.byref(n)))
        return n.value

    def pass_info(self, i: int) -> dict:
        pi = ipc_pass_info()
        _check(lib().ipc_stream_pass_info(self._p, i, ctypes.byref(pi)))
        return {"level": pi.level, "dim": pi.dim, "n_targets": pi.n_targets,
                "n_chunks": pi.n_chunks, "plane_bytes": list(pi.plane_bytes),
                "errq": list(pi.errq), "progressive": bool(pi.progressive),
                "launch_pass": int(pi.launch_pass)}

    def entropy_code(self) -> "Stream":
        """ipc_stream_entropy_code: entropy-code the stored blocks on the
        device; serialization and the planner then use the coded form."""
        _check(lib().ipc_stream_entropy_code(self.ctx.handle, self._p), self.ctx.handle)
        return self

    @property
    def coding(self) -> int:
        c = c_int()
        _check(lib().ipc_stream_coding(self._p, ctypes.byref(c)))
        return c.value

    def to_bytes(self) -> bytes:
        n = self.nbytes
        # a new bytes object, not yet shared, filled in place by the library
        # (no zero fill and no second copy)
        out = _new_bytes(None, n)
        _check(lib().ipc_stream_to_host(self.ctx.handle, self._p,
                                        ctypes.cast(ctypes.c_char_p(out), c_void_p), n),
               self.ctx.handle)
        return out

    def retrieve(self, eb=None, bitrate=None, level_groups: bool = False) -> "State":
        out = c_void_p()
        info = ipc_info()
        _check(lib().ipc_retrieve(self.ctx.handle, self._p, _target(eb, bitrate, level_groups),
                                  ctypes.byref(out), ctypes.byref(info)), self.ctx.handle)
        return State(self, out, info)

    def retrieve_noalloc(self, out, eb=None, bitrate=None) -> ipc_info:
        """ipc_retrieve_noalloc: the reconstruction written into `out` (a
        contiguous device tensor of the stream's shape and dtype), with no
        device allocation; returns the call's ipc_info."""
        if not out.is_contiguous() or out.dtype != self.dtype or tuple(out.shape) != tuple(self.shape):
            raise ValueError("out must be a contiguous tensor of the stream's shape and dtype")
        info = ipc_info()
        _check(lib().ipc_retrieve_noalloc(self.ctx.handle, self._p, _target(eb, bitrate),
                                          c_void_p(out.data_ptr()), out.numel() * out.element_size(),
                                          ctypes.byref(info)), self.ctx.handle)
        return info

    def retrieve_plan(self, plan: Sequence[int]) -> "State":
        out = c_void_p()
        info = ipc_info()
        arr = (c_uint8 * len(plan))(*plan)
        _check(lib().ipc_retrieve_plan(self.ctx.handle, self._p, arr, len(plan),
                                       ctypes.byref(out), ctypes.byref(info)), self.ctx.handle)
        return State(self, out, info)


class State:
    """ipc_state: a resident reconstruction plus the planes it was built from."""

    def __init__(self, stream: Stream, p, info: ipc_info):
        self.stream, self._p, self.info = stream, p, info
        stream.ctx._states.add(self)

    def free(self):
        if getattr(self, "_p", None):
            lib().ipc_state_free(self._p)
            self._p = None

    def __del__(self):  # pragma: no cover
        try:
            self.free()
        except Exception:
            pass

    @property
    def plan(self):
        return self.info.plan_list()

    @property
    def bound(self) -> float:
        return self.info.bound

    def field_ptr(self) -> int:
        return lib().ipc_state_field(self._p)

    def view(self):
        """The reconstruction as a torch tensor that aliases the state's own
        device memory (no copy, through __cuda_array_interface__).  It is
        valid until the next refine of this state or its free, and refine
        updates it in place; the tensor keeps this State object alive."""
        import torch

        state = self

        class _Field:
            @property
            def __cuda_array_interface__(self):
                return {"shape": tuple(state.stream.shape),
                        "typestr": "<f4" if state.stream.dtype == torch.float32 else "<f8",
                        "data": (int(state.field_ptr()), False), "version": 3, "strides": None}

        holder = _Field()
        t = torch.as_tensor(holder, device=f"cuda:{self.stream.ctx.device}")
        t._ipc_state = self  # the state outlives the view
        return t

    def tensor(self):
        """A copy of the reconstruction as a torch tensor on the device."""
        import torch
        t = torch.empty(self.stream.shape, dtype=self.stream.dtype,
                        device=f"cuda:{self.stream.ctx.device}")
        self.copy_into(t)
        return t

    def copy_into(self, t):
        _check(lib().ipc_state_copy_field(self.stream.ctx.handle, self._p, c_void_p(t.data_ptr()),
                                          t.numel() * t.element_size()), self.stream.ctx.handle)

    def refine(self, eb=None, bitrate=None, level_groups: bool = False) -> ipc_info:
        info = ipc_info()
        _check(lib().ipc_refine(self.stream.ctx.handle, self._p, _target(eb, bitrate, level_groups),
                                ctypes.byref(info)), self.stream.ctx.handle)
        if not info.flags & IPC_FLAG_NOOP:
            self.info = info
        return info

    def refine_additive(self, eb=None, bitrate=None, level_groups: bool = False) -> ipc_info:
        """ipc_refine_additive: the paper's additive form of Alg. 2."""
        info = ipc_info()
        _check(lib().ipc_refine_additive(self.stream.ctx.handle, self._p,
                                         _target(eb, bitrate, level_groups), ctypes.byref(info)),
               self.stream.ctx.handle)
        if not info.flags & IPC_FLAG_NOOP:
            self.info = info
        return info


__all__ = ["lib", "plan_host", "Context", "Stream", "State", "IpcError", "ipc_info",
           "ipc_target", "ipc_options", "LIB_PATH"]


class Server:
    """ipc_server: resident streams, requests admitted by a device-memory
    budget and served in continuous batches by a native worker thread.

    While a server exists, use its context only through it (``locked()``
    around any other call on the context)."""

    def __init__(self, ctx: Context, budget_bytes: int, max_batch: int = 64, batch_graphs: bool = True):
        # batched retrievals replayed from captured HIP graphs (the faster
        # configuration for serving mixes; see Context.set_batch_graphs)
        ctx.set_batch_graphs(batch_graphs)
        p = c_void_p()
        _check(lib().ipc_server_create(ctx.handle, int(budget_bytes), int(max_batch), ctypes.byref(p)),
               ctx.handle)
        self._p = p
        self.ctx = ctx

    def submit(self, stream: "Stream" = None, state: "State" = None, eb=None, bitrate=None) -> int:
        """Queue a retrieval of `stream` or a refinement of `state`; returns a ticket."""
        t = c_uint64()
        st = lib().ipc_server_submit(self._p, stream._p if stream is not None else None,
                                     state._p if state is not None else None,
                                     _target(eb, bitrate), ctypes.byref(t))
        if st != 0:
            raise IpcError(st, "submit refused")
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1, stream: "Stream" = None, state: "State" = None):
        """(State, info, latency_ms) of a served request (the refined State
        itself for refinements; a new ServedState for retrievals)."""
        out = c_void_p()
        info = ipc_info()
        lat = c_double()
        st = lib().ipc_server_wait(self._p, int(ticket), int(timeout_ms), ctypes.byref(out),
                                   ctypes.byref(info), ctypes.byref(lat))
        if st != 0:
            raise IpcError(st, "request failed" if st != -5 else "not finished")
        if state is not None:
            state.info = info
            return state, info, lat.value
        return ServedState(self, stream, out, info), info, lat.value

    def release(self, state: "State"):
        if getattr(state, "_p", None):
            _check(lib().ipc_server_release(self._p, state._p))
            state._p = None

    def locked(self):
        srv = self

        class _Lock:
            def __enter__(self):
                _check(lib().ipc_server_lock(srv._p))

            def __exit__(self, *a):
                _check(lib().ipc_server_unlock(srv._p))
        return _Lock()

    def stats(self) -> dict:
        v = [c_uint64() for _ in range(4)]
        _check(lib().ipc_server_stats(self._p, *[ctypes.byref(x) for x in v]))
        return {"used": v[0].value, "peak": v[1].value, "batches": v[2].value, "served": v[3].value}

    def close(self):
        if getattr(self, "_p", None):
            lib().ipc_server_destroy(self._p)
            self._p = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class ServedState(State):
    """A State made by a Server: freed through it, copied under its lock."""

    def __init__(self, server: Server, stream: "Stream", p, info: ipc_info):
        self.server = server
        self.stream, self._p, self.info = stream, p, info

    def free(self):
        if getattr(self, "_p", None):
            self.server.release(self)

    def copy_into(self, t):
        with self.server.locked():
            State.copy_into(self, t)

    def refine(self, eb=None, bitrate=None):
        tk = self.server.submit(state=self, eb=eb, bitrate=bitrate)
        _, info, _ = self.server.wait(tk, state=self)
        return info
