"""ctypes wrapper of the CPU oracle (test infrastructure only).

Every function mirrors one routine of ``hiz_oracle.c``; see that file for the
paper passages each follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "hiz_oracle.c")

OK, ERR_ARG, ERR_NONFINITE, ERR_BUFSZ, ERR_CORRUPT, ERR_NOMEM = 0, 1, 2, 3, 4, 5
ABS, REL = 0, 1
LIN, CUB, NAT = 0, 1, 2
CANDS = 21  # tuner candidates: {LIN, CUB, NAT} x {MD, SEQ x 6 orders}
MD, SEQ = 0, 1
PIPE_HF, PIPE_TP, PIPE_CR = 0, 1, 2
FLAG_REORDER = 4
LC_TCMS, LC_BIT, LC_RRE, LC_RZE = 0, 1, 2, 3
LC_CHUNK = 16384
LC_STAGE_OUT = 16384 + 16384 // 4 + 64  # output capacity orc_lc_stage assumes
PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "hiz_oracle.h"))):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-Wall",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("tune", C.c_int), ("cfg", (C.c_uint8 * 3) * 4), ("chunk", C.c_uint32),
                ("pipeline", C.c_int), ("reorder", C.c_int)]


class Debug(C.Structure):
    _fields_ = [("codes", C.c_void_p), ("recon", C.c_void_p), ("hist", C.c_uint64 * 256),
                ("cfg", (C.c_uint8 * 3) * 4), ("tune_err", (C.c_uint64 * CANDS) * 4),
                ("eps", C.c_float), ("n_out", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        u64p = C.POINTER(C.c_uint64)
        L.orc_eps.restype = C.c_float
        L.orc_eps.argtypes = [C.c_int, C.c_double, C.c_float, C.c_float]
        L.orc_stencil.restype = C.c_float
        L.orc_stencil.argtypes = [C.c_int] + [C.c_float] * 4 + [C.c_int] * 3 + [C.POINTER(C.c_int)]
        L.orc_predict.restype = C.c_float
        L.orc_predict.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int,
                                  C.c_int, C.c_int, C.c_int]
        L.orc_tune.argtypes = [C.c_void_p, u64p, C.c_float, C.c_void_p, C.c_void_p]
        L.orc_codebook.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_canonical.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_huff_encode.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p, C.c_void_p,
                                      C.c_void_p, u64p, C.c_void_p]
        L.orc_huff_decode.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_uint32,
                                      C.c_void_p, C.c_void_p]
        L.orc_compress.argtypes = [C.c_void_p, u64p, C.c_int, C.c_double, C.POINTER(Params),
                                   C.POINTER(C.c_void_p), u64p, C.POINTER(Debug)]
        L.orc_decompress.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, u64p,
                                     C.c_void_p]
        L.orc_stream_dims.argtypes = [C.c_void_p, C.c_uint64, u64p]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_level.argtypes = [C.c_uint64] * 3
        L.orc_reorder_index.argtypes = [u64p, C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_reorder_index.restype = C.c_uint64
        L.orc_reorder.argtypes = [C.c_void_p, u64p, C.c_void_p]
        L.orc_reorder.restype = None
        L.orc_unreorder.argtypes = [C.c_void_p, u64p, C.c_void_p]
        L.orc_unreorder.restype = None
        L.orc_lc_chunks.argtypes = [C.c_uint64]
        L.orc_lc_chunks.restype = C.c_uint64
        L.orc_lc_encode.argtypes = [C.c_int, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, u64p]
        L.orc_lc_decode.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                    C.c_uint64]
        L.orc_lc_stage.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"{what}: oracle status {rc}")
        self.rc = rc


def _dims(shape):
    return (C.c_uint64 * 3)(*[int(s) for s in shape])


def eps(mode, eb, vmin, vmax) -> np.float32:
    return np.float32(lib().orc_eps(mode, eb, float(vmin), float(vmax)))


def stencil(spline, a, b, c, d, pa, pc, pd):
    r = C.c_int()
    v = lib().orc_stencil(spline, a, b, c, d, int(pa), int(pc), int(pd), C.byref(r))
    return np.float32(v), r.value


def predict(buf: np.ndarray, t, s, spline, scheme, perm=0) -> np.float32:
    """Prediction of local target t of a block array buf (extents = buf.shape)."""
    b = np.ascontiguousarray(buf, dtype=np.float32)
    n = (C.c_int * 3)(*b.shape)
    tt = (C.c_int * 3)(*[int(v) for v in t])
    return np.float32(lib().orc_predict(b.ctypes.data, n, tt, s, spline, scheme, perm))


def cfg_array(cfg):
    arr = ((C.c_uint8 * 3) * 4)()
    for l in range(4):
        for k in range(3):
            arr[l][k] = int(cfg[l][k])
    return arr


def cfg_tuple(arr):
    return tuple(tuple(int(arr[l][k]) for k in range(3)) for l in range(4))


DEFAULT_CFG = ((CUB, MD, 0),) * 4


def tune(x: np.ndarray, eps_value):
    x = np.ascontiguousarray(x, dtype=np.float32)
    cfg = ((C.c_uint8 * 3) * 4)()
    err = np.zeros((4, CANDS), dtype=np.uint64)
    rc = lib().orc_tune(x.ctypes.data, _dims(x.shape), float(eps_value), C.byref(cfg),
                        err.ctypes.data)
    if rc:
        raise OracleError(rc, "tune")
    return cfg_tuple(cfg), err


def codebook(hist):
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    assert h.shape == (256,)
    ln = np.zeros(256, dtype=np.uint8)
    cd = np.zeros(256, dtype=np.uint32)
    lib().orc_codebook(h.ctypes.data, ln.ctypes.data, cd.ctypes.data)
    return ln, cd


def canonical(lengths):
    ln = np.zeros(256, dtype=np.uint8)
    ln[:len(lengths)] = lengths
    cd = np.zeros(256, dtype=np.uint32)
    rc = lib().orc_canonical(ln.ctypes.data, cd.ctypes.data)
    if rc:
        raise OracleError(rc, "canonical")
    return cd[:len(lengths)].copy()


def huff_encode(codes: np.ndarray, chunk, ln, cd):
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    n = codes.size
    nch = (n + chunk - 1) // chunk
    words = np.zeros(n + nch + 1, dtype=np.uint32)
    counts = np.zeros(max(nch, 1), dtype=np.uint32)
    nw = C.c_uint64()
    rc = lib().orc_huff_encode(codes.ctypes.data, n, chunk, np.ascontiguousarray(ln).ctypes.data,
                               np.ascontiguousarray(cd).ctypes.data, words.ctypes.data,
                               C.byref(nw), counts.ctypes.data)
    if rc:
        raise OracleError(rc, "huff_encode")
    return words[:nw.value].copy(), counts[:nch].copy()


def huff_decode(words, counts, n, chunk, ln):
    words = np.ascontiguousarray(words, dtype=np.uint32)
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    out = np.zeros(n, dtype=np.uint8)
    rc = lib().orc_huff_decode(words.ctypes.data, words.size, counts.ctypes.data, n, chunk,
                               np.ascontiguousarray(ln, dtype=np.uint8).ctypes.data,
                               out.ctypes.data)
    if rc:
        raise OracleError(rc, "huff_decode")
    return out


class Result:
    """Compressed stream plus the oracle's debug view of the run."""

    def __init__(self, stream, codes, recon, hist, cfg, eps_value, n_out, tune_err):
        self.stream = stream
        self.codes = codes
        self.recon = recon
        self.hist = hist
        self.cfg = cfg
        self.eps = eps_value
        self.n_out = n_out
        self.tune_err = tune_err


def compress(x: np.ndarray, mode, eb, tune=True, cfg=DEFAULT_CFG, chunk=1024,
             debug=True, pipeline=PIPE_HF, reorder=False) -> Result:
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.ndim != 3:
        raise ValueError("oracle.compress needs a 3-D array")
    p = Params(int(bool(tune)), cfg_array(cfg), int(chunk), int(pipeline), int(bool(reorder)))
    out = C.c_void_p()
    size = C.c_uint64()
    dbg = Debug()
    codes = recon = None
    if debug:
        codes = np.zeros(x.shape, dtype=np.uint8)
        recon = np.zeros(x.shape, dtype=np.float32)
        dbg.codes = codes.ctypes.data
        dbg.recon = recon.ctypes.data
    rc = lib().orc_compress(x.ctypes.data, _dims(x.shape), int(mode), float(eb), C.byref(p),
                            C.byref(out), C.byref(size), C.byref(dbg))
    if rc:
        raise OracleError(rc, "compress")
    try:
        stream = np.ctypeslib.as_array(C.cast(out, C.POINTER(C.c_uint8)),
                                       shape=(size.value,)).copy()
    finally:
        lib().orc_free(out)
    hist = np.frombuffer(bytes(dbg.hist), dtype=np.uint64).copy()
    terr = np.frombuffer(bytes(dbg.tune_err), dtype=np.uint64).reshape(4, CANDS).copy()
    return Result(stream, codes, recon, hist, cfg_tuple(dbg.cfg), np.float32(dbg.eps),
                  int(dbg.n_out), terr)


def stream_dims(stream: np.ndarray):
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    d = (C.c_uint64 * 3)()
    rc = lib().orc_stream_dims(s.ctypes.data, s.size, d)
    if rc:
        raise OracleError(rc, "stream_dims")
    return tuple(int(v) for v in d)


def decompress(stream: np.ndarray, with_codes=False):
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    dims = stream_dims(s)
    out = np.zeros(dims, dtype=np.float32)
    codes = np.zeros(dims, dtype=np.uint8) if with_codes else None
    d = (C.c_uint64 * 3)()
    rc = lib().orc_decompress(s.ctypes.data, s.size, out.ctypes.data, out.size, d,
                              codes.ctypes.data if with_codes else None)
    if rc:
        raise OracleError(rc, "decompress")
    return (out, codes) if with_codes else out


def decompress_status(stream: np.ndarray) -> int:
    """Status code of decompressing a (possibly corrupt) stream."""
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    d = (C.c_uint64 * 3)()
    rc = lib().orc_stream_dims(s.ctypes.data, s.size, d)
    if rc:
        return rc
    n = int(d[0]) * int(d[1]) * int(d[2])
    out = np.zeros(n, dtype=np.float32)
    return lib().orc_decompress(s.ctypes.data, s.size, out.ctypes.data, n, d, None)


def level(x, y, z) -> int:
    return lib().orc_level(int(x), int(y), int(z))


def reorder_index(shape, x, y, z) -> int:
    return int(lib().orc_reorder_index(_dims(shape), int(x), int(y), int(z)))


def reorder(codes: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    out = np.zeros(c.size, dtype=np.uint8)
    lib().orc_reorder(c.ctypes.data, _dims(c.shape), out.ctypes.data)
    return out


def unreorder(seq: np.ndarray, shape) -> np.ndarray:
    s_ = np.ascontiguousarray(seq, dtype=np.uint8)
    out = np.zeros(shape, dtype=np.uint8)
    lib().orc_unreorder(s_.ctypes.data, _dims(shape), out.ctypes.data)
    return out


def lc_encode(pipeline, data: np.ndarray):
    """Chunked bitwise-redundancy stages: (sizes u32[n_chunks], stored bytes)."""
    d = np.ascontiguousarray(data, dtype=np.uint8)
    n = d.size
    nc = int(lib().orc_lc_chunks(n))
    sizes = np.zeros(max(nc, 1), dtype=np.uint32)
    out = np.zeros(max(n, 1), dtype=np.uint8)
    nb = C.c_uint64()
    rc = lib().orc_lc_encode(int(pipeline), d.ctypes.data, n, sizes.ctypes.data, out.ctypes.data,
                             C.byref(nb))
    if rc:
        raise OracleError(rc, "lc_encode")
    return sizes[:nc].copy(), out[:nb.value].copy()


def lc_decode(pipeline, sizes, stored, n) -> np.ndarray:
    sz = np.ascontiguousarray(sizes, dtype=np.uint32)
    st = np.ascontiguousarray(stored, dtype=np.uint8)
    out = np.zeros(max(int(n), 1), dtype=np.uint8)
    rc = lib().orc_lc_decode(int(pipeline), sz.ctypes.data, st.ctypes.data, st.size,
                             out.ctypes.data, int(n))
    if rc:
        raise OracleError(rc, "lc_decode")
    return out[:int(n)].copy()


def lc_stage(op, k, data, inverse=False) -> np.ndarray:
    """One bitwise-redundancy stage on one buffer (at most 20 KB)."""
    d = np.ascontiguousarray(data, dtype=np.uint8)
    out = np.zeros(LC_STAGE_OUT, dtype=np.uint8)  # the C routine may write this much
    n = lib().orc_lc_stage(int(op), int(k), int(bool(inverse)), d.ctypes.data, d.size,
                           out.ctypes.data)
    if n < 0:
        raise OracleError(n, "lc_stage")
    return out[:n].copy()


def psnr(x: np.ndarray, y: np.ndarray) -> float:
    """PSNR over the value range (Sec. 6.1.4)."""
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    rng = x.max() - x.min()
    mse = np.mean((x - y) ** 2)
    if mse == 0:
        return float("inf")
    return float(20 * np.log10(rng) - 10 * np.log10(mse))
