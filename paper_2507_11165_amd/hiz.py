"""Python binding of the hiz C ABI (include/hiz.h).

Argument marshalling only: torch supplies device memory and streams, every step
of compression and decompression runs in the library's HIP kernels. Loading
fails loudly when libhiz.so is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhiz.so")

OK, ERR_ARG, ERR_NONFINITE, ERR_BUFSZ, ERR_CORRUPT, ERR_NOMEM, ERR_HIP = range(7)
ABS, REL = 0, 1
LINEAR, CUBIC, NATURAL = 0, 1, 2
MD, SEQ = 0, 1
PIPE_HUFFMAN, PIPE_TP, PIPE_CR = 0, 1, 2
_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_NONFINITE", 3: "ERR_BUFSZ", 4: "ERR_CORRUPT",
           5: "ERR_NOMEM", 6: "ERR_HIP"}

# exported symbols (kept in step with include/hiz.h)
SYMBOLS = ["hiz_create", "hiz_destroy", "hiz_last_error", "hiz_compress_bound",
           "hiz_workspace_bound", "hiz_compress", "hiz_decompress", "hiz_inspect",
           "hiz_compress_batch", "hiz_decompress_batch", "hiz_compress_batch_submit",
           "hiz_decompress_batch_submit", "hiz_batch_ready", "hiz_batch_finish", "hiz_set_graphs",
           "hiz_graph_stats", "hiz_server_create", "hiz_server_submit", "hiz_server_poll",
           "hiz_server_drain", "hiz_server_get_stats", "hiz_server_clock", "hiz_server_destroy",
           "hiz_set_profiling", "hiz_get_profile", "hiz_reset_profile", "hiz_compress_noalloc"]
OP_COMPRESS, OP_DECOMPRESS = 0, 1


class Params(C.Structure):
    _fields_ = [("tune", C.c_int), ("level_cfg", (C.c_uint8 * 3) * 4), ("chunk", C.c_uint32),
                ("tile_z", C.c_uint32), ("pipeline", C.c_uint32), ("reorder", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("dims", C.c_uint64 * 3), ("mode", C.c_int), ("eb", C.c_double),
                ("eps", C.c_float), ("vmin", C.c_float), ("vmax", C.c_float),
                ("constant", C.c_int), ("level_cfg", (C.c_uint8 * 3) * 4), ("chunk", C.c_uint32),
                ("n_outliers", C.c_uint64), ("n_chunks", C.c_uint64),
                ("payload_words", C.c_uint64), ("total_bytes", C.c_uint64),
                ("pipeline", C.c_int), ("reorder", C.c_int), ("lc_bytes", C.c_uint64)]


class Request(C.Structure):
    _fields_ = [("id", C.c_uint64), ("op", C.c_int), ("d_in", C.c_void_p), ("in_size", C.c_uint64),
                ("dims", C.c_uint64 * 3), ("mode", C.c_int), ("eb", C.c_double),
                ("d_out", C.c_void_p), ("out_cap", C.c_uint64)]


class Completion(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int), ("size", C.c_uint64),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("batch_size", C.c_int), ("slot", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("batches", C.c_uint64),
                ("max_running", C.c_int), ("slots", C.c_int), ("slot_capacity", C.c_uint64)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_uint64), ("total_ms", C.c_double)]


class HizError(RuntimeError):
    def __init__(self, status, msg, needed=None):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.needed = needed


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded libhiz.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                    "(hipcc, gfx950); there is no CPU fallback")
            L = C.CDLL(LIB_PATH)
            u64p = C.POINTER(C.c_uint64)
            L.hiz_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(C.c_void_p)]
            L.hiz_destroy.argtypes = [C.c_void_p]
            L.hiz_destroy.restype = None
            L.hiz_last_error.argtypes = [C.c_void_p]
            L.hiz_last_error.restype = C.c_char_p
            L.hiz_compress_bound.argtypes = [u64p]
            L.hiz_compress_bound.restype = C.c_uint64
            L.hiz_compress.argtypes = [C.c_void_p, C.c_void_p, u64p, C.c_int, C.c_double,
                                       C.POINTER(Params), C.c_void_p, C.c_uint64, u64p,
                                       C.c_void_p]
            L.hiz_compress_noalloc.argtypes = L.hiz_compress.argtypes
            L.hiz_decompress.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                         C.c_uint64, u64p, C.c_void_p]
            L.hiz_inspect.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Info)]
            vpp = C.POINTER(C.c_void_p)
            ip = C.POINTER(C.c_int)
            dp = C.POINTER(C.c_double)
            L.hiz_compress_batch.argtypes = [C.c_void_p, C.c_int, vpp, u64p, ip, dp,
                                             C.POINTER(Params), vpp, u64p, u64p, ip, C.c_void_p]
            L.hiz_decompress_batch.argtypes = [C.c_void_p, C.c_int, vpp, u64p, vpp, u64p, u64p,
                                               ip, C.c_void_p]
            L.hiz_compress_batch_submit.argtypes = [C.c_void_p, C.c_int, vpp, u64p, ip, dp,
                                                    C.POINTER(Params), vpp, u64p, C.c_void_p]
            L.hiz_decompress_batch_submit.argtypes = [C.c_void_p, C.c_int, vpp, u64p, vpp, u64p,
                                                      C.c_void_p]
            L.hiz_batch_ready.argtypes = [C.c_void_p]
            L.hiz_batch_finish.argtypes = [C.c_void_p, u64p, u64p, ip]
            L.hiz_set_graphs.argtypes = [C.c_void_p, C.c_int]
            L.hiz_graph_stats.argtypes = [C.c_void_p, u64p, u64p]
            L.hiz_graph_stats.restype = None
            L.hiz_workspace_bound.argtypes = [u64p]
            L.hiz_workspace_bound.restype = C.c_uint64
            L.hiz_server_create.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_int,
                                            C.POINTER(Params), C.POINTER(C.c_void_p)]
            L.hiz_server_submit.argtypes = [C.c_void_p, C.POINTER(Request)]
            L.hiz_server_poll.argtypes = [C.c_void_p, C.POINTER(Completion), C.c_int]
            L.hiz_server_drain.argtypes = [C.c_void_p, C.c_double]
            L.hiz_server_get_stats.argtypes = [C.c_void_p, C.POINTER(ServerStats)]
            L.hiz_server_get_stats.restype = None
            L.hiz_server_clock.argtypes = []
            L.hiz_server_clock.restype = C.c_double
            L.hiz_server_destroy.argtypes = [C.c_void_p]
            L.hiz_server_destroy.restype = None
            L.hiz_set_profiling.argtypes = [C.c_void_p, C.c_int]
            L.hiz_set_profiling.restype = None
            L.hiz_get_profile.argtypes = [C.c_void_p, C.POINTER(KernelStat), C.c_int]
            L.hiz_reset_profile.argtypes = [C.c_void_p]
            L.hiz_reset_profile.restype = None
            _lib = L
    return _lib


def _dims(shape):
    return (C.c_uint64 * 3)(*[int(s) for s in shape])


def compress_bound(shape) -> int:
    return int(lib().hiz_compress_bound(_dims(shape)))


def workspace_bound(shape) -> int:
    return int(lib().hiz_workspace_bound(_dims(shape)))


def make_params(tune=True, level_cfg=None, chunk=0, tile_z=0, pipeline=PIPE_HUFFMAN,
                reorder=-1) -> Params:
    p = Params()
    p.pipeline = int(pipeline)
    p.reorder = int(reorder)
    p.tune = 1 if tune else 0
    cfg = level_cfg or ((CUBIC, MD, 0),) * 4
    for l in range(4):
        for k in range(3):
            p.level_cfg[l][k] = int(cfg[l][k])
    p.chunk = int(chunk)
    p.tile_z = int(tile_z)
    return p


def _mode(mode):
    if isinstance(mode, str):
        return {"abs": ABS, "rel": REL}[mode.lower()]
    return int(mode)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def inspect(stream_bytes) -> dict:
    """Header fields of a stream (host bytes, numpy array or tensor)."""
    import numpy as np
    try:
        import torch
        if isinstance(stream_bytes, torch.Tensor):
            stream_bytes = stream_bytes[:512].cpu().numpy()
    except ImportError:  # pragma: no cover
        pass
    b = np.ascontiguousarray(np.frombuffer(bytes(stream_bytes), dtype=np.uint8))
    info = Info()
    rc = lib().hiz_inspect(b.ctypes.data, b.size, C.byref(info))
    if rc:
        raise HizError(rc, "inspect")
    return {
        "dims": tuple(int(v) for v in info.dims), "mode": info.mode, "eb": info.eb,
        "eps": info.eps, "vmin": info.vmin, "vmax": info.vmax, "constant": bool(info.constant),
        "level_cfg": tuple(tuple(int(info.level_cfg[l][k]) for k in range(3)) for l in range(4)),
        "chunk": info.chunk, "n_outliers": info.n_outliers, "n_chunks": info.n_chunks,
        "payload_words": info.payload_words, "total_bytes": info.total_bytes,
        "pipeline": info.pipeline, "reorder": bool(info.reorder), "lc_bytes": info.lc_bytes,
    }


class Context:
    """A hiz context on one device: owns device workspaces (not thread-safe)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        h = C.c_void_p()
        rc = lib().hiz_create(int(device), int(workspace_bytes), C.byref(h))
        if rc:
            raise HizError(rc, f"hiz_create on device {device}")
        self._h = h
        self.device = int(device)

    def close(self):
        if self._h:
            lib().hiz_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc, what, needed=None):
        msg = lib().hiz_last_error(self._h).decode(errors="replace")
        return HizError(rc, f"{what}: {msg}", needed)

    # -- raw pointer calls (C-ABI shaped) --
    def compress_ptr(self, field_ptr, shape, mode, eb, out_ptr, out_cap, params=None,
                     stream_handle=None) -> int:
        size = C.c_uint64()
        p = C.byref(params) if params is not None else None
        rc = lib().hiz_compress(self._h, C.c_void_p(field_ptr), _dims(shape), _mode(mode),
                                float(eb), p, C.c_void_p(out_ptr), int(out_cap), C.byref(size),
                                stream_handle)
        if rc:
            raise self._err(rc, "compress", int(size.value))
        return int(size.value)

    def compress_noalloc_ptr(self, field_ptr, shape, mode, eb, out_ptr, out_cap, params=None,
                             stream_handle=None) -> int:
        """hiz_compress_noalloc: the same stream as compress_ptr, with the
        library's fixed scratch array as workspace (nothing allocated)."""
        size = C.c_uint64()
        p = C.byref(params) if params is not None else None
        rc = lib().hiz_compress_noalloc(self._h, C.c_void_p(field_ptr), _dims(shape), _mode(mode),
                                        float(eb), p, C.c_void_p(out_ptr), int(out_cap),
                                        C.byref(size), stream_handle)
        if rc:
            raise self._err(rc, "compress_noalloc", int(size.value))
        return int(size.value)

    def decompress_ptr(self, in_ptr, in_size, out_ptr, out_cap, stream_handle=None):
        dims = (C.c_uint64 * 3)()
        rc = lib().hiz_decompress(self._h, C.c_void_p(in_ptr), int(in_size), C.c_void_p(out_ptr),
                                  int(out_cap), dims, stream_handle)
        if rc:
            raise self._err(rc, "decompress")
        return tuple(int(v) for v in dims)

    # -- torch-facing calls --
    def compress(self, field, mode="rel", eb=1e-3, params=None, out=None, stream=None):
        """Compress a contiguous 3-D float32 CUDA tensor; returns a uint8 tensor view."""
        import torch
        if field.dtype != torch.float32 or field.dim() not in (1, 2, 3) or not field.is_cuda:
            raise ValueError("compress needs a 1-, 2- or 3-D float32 tensor on a HIP device")
        # a 2-D field (H, W) is the 3-D field (1, H, W); a 1-D one (1, 1, W)
        field = field.contiguous()
        while field.dim() < 3:
            field = field.unsqueeze(0)
        n = field.numel()
        if out is None:
            cap = min(compress_bound(field.shape), 5 * n + (1 << 16))
            out = torch.empty(cap, dtype=torch.uint8, device=field.device)
        sh = _stream_handle(stream)
        try:
            size = self.compress_ptr(field.data_ptr(), field.shape, mode, eb, out.data_ptr(),
                                     out.numel(), params, sh)
        except HizError as e:
            if e.status != ERR_BUFSZ or not e.needed:
                raise
            out = torch.empty(e.needed, dtype=torch.uint8, device=field.device)
            size = self.compress_ptr(field.data_ptr(), field.shape, mode, eb, out.data_ptr(),
                                     out.numel(), params, sh)
        return out[:size]

    def decompress(self, stream_t, out=None, stream=None, squeeze=False):
        """Decompress a uint8 CUDA tensor holding one stream; returns float32 (dx, dy, dz),
        or with squeeze=True without the leading size-1 axes of a 2-D or 1-D field."""
        import torch
        if stream_t.dtype != torch.uint8 or not stream_t.is_cuda:
            raise ValueError("decompress needs a uint8 tensor on a HIP device")
        stream_t = stream_t.contiguous()
        info = inspect(stream_t[:512].cpu().numpy().tobytes())
        shape = info["dims"]
        n = shape[0] * shape[1] * shape[2]
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=stream_t.device)
        self.decompress_ptr(stream_t.data_ptr(), stream_t.numel(), out.data_ptr(), out.numel(),
                            _stream_handle(stream))
        y = out.view(shape) if out.numel() == n else out
        if squeeze and out.numel() == n:
            while y.dim() > 1 and y.shape[0] == 1:
                y = y[0]
        return y

    # -- batches (C-ABI shaped: lists of device pointers) --
    def compress_batch_ptr(self, field_ptrs, shapes, modes, ebs, out_ptrs, out_caps,
                           params=None, stream_handle=None, submit_only=False):
        """Compress n fields in one launch per stage. Returns (sizes, statuses), or
        None when submit_only (then call batch_finish)."""
        n = len(field_ptrs)
        fp = (C.c_void_p * max(n, 1))(*field_ptrs)
        dims = (C.c_uint64 * max(3 * n, 1))(*[int(v) for sh in shapes for v in sh])
        md = (C.c_int * max(n, 1))(*[_mode(m) for m in modes])
        eb = (C.c_double * max(n, 1))(*[float(e) for e in ebs])
        op = (C.c_void_p * max(n, 1))(*out_ptrs)
        cp = (C.c_uint64 * max(n, 1))(*[int(c) for c in out_caps])
        p = C.byref(params) if params is not None else None
        if submit_only:
            rc = lib().hiz_compress_batch_submit(self._h, n, fp, dims, md, eb, p, op, cp,
                                                 stream_handle)
            if rc:
                raise self._err(rc, "compress_batch_submit")
            return None
        sizes = (C.c_uint64 * max(n, 1))()
        st = (C.c_int * max(n, 1))()
        rc = lib().hiz_compress_batch(self._h, n, fp, dims, md, eb, p, op, cp, sizes, st,
                                      stream_handle)
        if rc and not any(st[i] for i in range(n)):
            raise self._err(rc, "compress_batch")
        return [int(sizes[i]) for i in range(n)], [int(st[i]) for i in range(n)]

    def decompress_batch_ptr(self, in_ptrs, in_sizes, out_ptrs, out_caps, stream_handle=None,
                             submit_only=False):
        """Decompress n streams in one launch per stage. Returns (dims, statuses), or
        None when submit_only (then call batch_finish)."""
        n = len(in_ptrs)
        ip_ = (C.c_void_p * max(n, 1))(*in_ptrs)
        isz = (C.c_uint64 * max(n, 1))(*[int(v) for v in in_sizes])
        op = (C.c_void_p * max(n, 1))(*out_ptrs)
        cp = (C.c_uint64 * max(n, 1))(*[int(c) for c in out_caps])
        if submit_only:
            rc = lib().hiz_decompress_batch_submit(self._h, n, ip_, isz, op, cp, stream_handle)
            if rc:
                raise self._err(rc, "decompress_batch_submit")
            return None
        dims = (C.c_uint64 * max(3 * n, 1))()
        st = (C.c_int * max(n, 1))()
        rc = lib().hiz_decompress_batch(self._h, n, ip_, isz, op, cp, dims, st, stream_handle)
        if rc and not any(st[i] for i in range(n)):
            raise self._err(rc, "decompress_batch")
        return ([tuple(int(dims[3 * i + k]) for k in range(3)) for i in range(n)],
                [int(st[i]) for i in range(n)])

    def batch_ready(self) -> bool:
        return bool(lib().hiz_batch_ready(self._h))

    def batch_finish(self, n):
        """Wait for the pending batch of n fields: (sizes, dims, statuses)."""
        sizes = (C.c_uint64 * max(n, 1))()
        dims = (C.c_uint64 * max(3 * n, 1))()
        st = (C.c_int * max(n, 1))()
        rc = lib().hiz_batch_finish(self._h, sizes, dims, st)
        if rc and not any(st[i] for i in range(n)):
            raise self._err(rc, "batch_finish")
        return ([int(sizes[i]) for i in range(n)],
                [tuple(int(dims[3 * i + k]) for k in range(3)) for i in range(n)],
                [int(st[i]) for i in range(n)])

    def set_graphs(self, on: bool):
        rc = lib().hiz_set_graphs(self._h, 1 if on else 0)
        if rc:
            raise self._err(rc, "set_graphs")

    def graph_stats(self):
        b, r = C.c_uint64(), C.c_uint64()
        lib().hiz_graph_stats(self._h, C.byref(b), C.byref(r))
        return int(b.value), int(r.value)

    # -- torch-facing batches --
    def compress_batch(self, fields, modes="rel", ebs=1e-3, params=None, stream=None):
        """Compress a list of 3-D float32 CUDA tensors in one batch; returns a list of
        uint8 tensor views (raises on the first failing field)."""
        import torch
        n = len(fields)
        if isinstance(modes, (str, int)):
            modes = [modes] * n
        if isinstance(ebs, (float, int)):
            ebs = [ebs] * n
        fields = [f.contiguous() for f in fields]
        for f in fields:
            if f.dtype != torch.float32 or f.dim() != 3 or not f.is_cuda:
                raise ValueError("compress_batch needs 3-D float32 tensors on a HIP device")
        outs = [torch.empty(min(compress_bound(f.shape), 5 * f.numel() + (1 << 16)),
                            dtype=torch.uint8, device=f.device) for f in fields]
        sh = _stream_handle(stream)
        sizes, st = self.compress_batch_ptr([f.data_ptr() for f in fields],
                                            [f.shape for f in fields], modes, ebs,
                                            [o.data_ptr() for o in outs],
                                            [o.numel() for o in outs], params, sh)
        for i, s_ in enumerate(st):
            if s_ == ERR_BUFSZ:
                outs[i] = torch.empty(sizes[i], dtype=torch.uint8, device=fields[i].device)
                sizes[i] = self.compress_ptr(fields[i].data_ptr(), fields[i].shape, modes[i],
                                             ebs[i], outs[i].data_ptr(), outs[i].numel(),
                                             params, sh)
            elif s_:
                raise HizError(s_, f"compress_batch field {i}: "
                               + lib().hiz_last_error(self._h).decode(errors="replace"))
        return [o[:sz] for o, sz in zip(outs, sizes)]

    def decompress_batch(self, streams, stream=None):
        """Decompress a list of uint8 CUDA tensors in one batch; returns float32 tensors."""
        import torch
        streams = [s_.contiguous() for s_ in streams]
        shapes = [inspect(s_[:512].cpu().numpy().tobytes())["dims"] for s_ in streams]
        outs = [torch.empty(sh_, dtype=torch.float32, device=s_.device)
                for sh_, s_ in zip(shapes, streams)]
        dims, st = self.decompress_batch_ptr([s_.data_ptr() for s_ in streams],
                                             [s_.numel() for s_ in streams],
                                             [o.data_ptr() for o in outs],
                                             [o.numel() for o in outs], _stream_handle(stream))
        for i, s_ in enumerate(st):
            if s_:
                raise HizError(s_, f"decompress_batch field {i}: "
                               + lib().hiz_last_error(self._h).decode(errors="replace"))
        return outs

    # -- profiling --
    def set_profiling(self, on: bool):
        lib().hiz_set_profiling(self._h, 1 if on else 0)

    def reset_profile(self):
        lib().hiz_reset_profile(self._h)

    def profile(self) -> dict:
        arr = (KernelStat * 64)()
        n = lib().hiz_get_profile(self._h, arr, 64)
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms))
                for i in range(min(n, 64))}


class Server:
    """Continuous-batching request loop on one device (hiz_server_* of the C ABI).

    Requests carry raw device pointers; the caller keeps their buffers alive until
    the request's completion has been polled."""

    def __init__(self, device=0, slots=4, mem_budget=0, max_batch=32, params=None):
        h = C.c_void_p()
        p = C.byref(params) if params is not None else None
        rc = lib().hiz_server_create(int(device), int(slots), int(mem_budget), int(max_batch), p,
                                     C.byref(h))
        if rc:
            raise HizError(rc, "hiz_server_create")
        self._h = h

    def submit_compress(self, rid, field_ptr, shape, mode, eb, out_ptr, out_cap):
        r = Request(id=int(rid), op=OP_COMPRESS, d_in=field_ptr, in_size=0, mode=_mode(mode),
                    eb=float(eb), d_out=out_ptr, out_cap=int(out_cap))
        for k in range(3):
            r.dims[k] = int(shape[k])
        rc = lib().hiz_server_submit(self._h, C.byref(r))
        if rc:
            raise HizError(rc, "hiz_server_submit")

    def submit_decompress(self, rid, stream_ptr, stream_size, out_ptr, out_elems):
        r = Request(id=int(rid), op=OP_DECOMPRESS, d_in=stream_ptr, in_size=int(stream_size),
                    mode=0, eb=0.0, d_out=out_ptr, out_cap=int(out_elems))
        rc = lib().hiz_server_submit(self._h, C.byref(r))
        if rc:
            raise HizError(rc, "hiz_server_submit")

    def poll(self, max_n=256):
        arr = (Completion * max_n)()
        n = lib().hiz_server_poll(self._h, arr, max_n)
        return [{"id": arr[i].id, "status": arr[i].status, "size": arr[i].size,
                 "t_submit": arr[i].t_submit, "t_start": arr[i].t_start,
                 "t_done": arr[i].t_done, "batch_size": arr[i].batch_size,
                 "slot": arr[i].slot} for i in range(n)]

    def drain(self, timeout_s=0.0):
        rc = lib().hiz_server_drain(self._h, float(timeout_s))
        if rc:
            raise HizError(rc, "hiz_server_drain (timeout)")

    def stats(self):
        st = ServerStats()
        lib().hiz_server_get_stats(self._h, C.byref(st))
        return {"submitted": st.submitted, "completed": st.completed, "batches": st.batches,
                "max_running": st.max_running, "slots": st.slots,
                "slot_capacity": st.slot_capacity}

    @staticmethod
    def clock():
        return float(lib().hiz_server_clock())

    def close(self):
        if self._h:
            lib().hiz_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ctx = {}


def default_context(device=None) -> Context:
    import torch
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _ctx:
        _ctx[d] = Context(d)
    return _ctx[d]


def compress(field, mode="rel", eb=1e-3, params=None, out=None, stream=None):
    """Z = Cmp(X) on the tensor's device."""
    return default_context(field.device.index).compress(field, mode, eb, params, out, stream)


def decompress(stream_t, out=None, stream=None, squeeze=False):
    """X' = Dec(Z) on the tensor's device."""
    return default_context(stream_t.device.index).decompress(stream_t, out, stream, squeeze)
