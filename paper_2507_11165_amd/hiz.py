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
LINEAR, CUBIC = 0, 1
MD, SEQ = 0, 1
_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_NONFINITE", 3: "ERR_BUFSZ", 4: "ERR_CORRUPT",
           5: "ERR_NOMEM", 6: "ERR_HIP"}

# exported symbols (kept in step with include/hiz.h)
SYMBOLS = ["hiz_create", "hiz_destroy", "hiz_last_error", "hiz_compress_bound", "hiz_compress",
           "hiz_decompress", "hiz_inspect", "hiz_set_profiling", "hiz_get_profile",
           "hiz_reset_profile"]


class Params(C.Structure):
    _fields_ = [("tune", C.c_int), ("level_cfg", (C.c_uint8 * 3) * 4), ("chunk", C.c_uint32),
                ("tile_z", C.c_uint32)]


class Info(C.Structure):
    _fields_ = [("dims", C.c_uint64 * 3), ("mode", C.c_int), ("eb", C.c_double),
                ("eps", C.c_float), ("vmin", C.c_float), ("vmax", C.c_float),
                ("constant", C.c_int), ("level_cfg", (C.c_uint8 * 3) * 4), ("chunk", C.c_uint32),
                ("n_outliers", C.c_uint64), ("n_chunks", C.c_uint64),
                ("payload_words", C.c_uint64), ("total_bytes", C.c_uint64)]


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
            L.hiz_decompress.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                         C.c_uint64, u64p, C.c_void_p]
            L.hiz_inspect.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Info)]
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


def make_params(tune=True, level_cfg=None, chunk=0, tile_z=0) -> Params:
    p = Params()
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
        if field.dtype != torch.float32 or field.dim() != 3 or not field.is_cuda:
            raise ValueError("compress needs a 3-D float32 tensor on a HIP device")
        field = field.contiguous()
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

    def decompress(self, stream_t, out=None, stream=None):
        """Decompress a uint8 CUDA tensor holding one stream; returns float32 (dx, dy, dz)."""
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
        return out.view(shape) if out.numel() == n else out

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


def decompress(stream_t, out=None, stream=None):
    """X' = Dec(Z) on the tensor's device."""
    return default_context(stream_t.device.index).decompress(stream_t, out, stream)
