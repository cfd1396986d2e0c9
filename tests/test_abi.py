"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/hiz.h declares, and parses stream headers written by
the oracle."""
import os
import re

import numpy as np
import pytest

import fieldgen as G
import oracle as O
from paper_2507_11165_amd import hiz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hiz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hiz_[a-z_]+)\s*\(", src)))


def test_header_declares_what_binding_lists():
    assert set(declared_symbols()) == set(hiz.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = hiz.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_compress_bound():
    assert hiz.compress_bound((0, 4, 4)) == 0
    n = 64 ** 3
    b = hiz.compress_bound((64, 64, 64))
    assert b >= 12 * n + 4 * n


@pytest.mark.parametrize("shape,mode,eb", [((33, 20, 47), O.REL, 1e-3), ((16, 16, 16), O.ABS, 0.01),
                                           ((70, 3, 5), O.REL, 1e-5)])
def test_inspect_reads_oracle_streams(shape, mode, eb):
    x = G.grf(shape, 3.0, 4)
    r = O.compress(x, mode, eb, chunk=512)
    info = hiz.inspect(r.stream.tobytes())
    assert info["dims"] == shape
    assert info["mode"] == mode and info["eb"] == eb
    assert np.float32(info["eps"]) == r.eps
    assert info["n_outliers"] == r.n_out
    assert info["total_bytes"] == r.stream.size
    assert info["chunk"] == 512
    assert info["level_cfg"] == r.cfg
    assert np.float32(info["vmin"]) == x.min() and np.float32(info["vmax"]) == x.max()


def test_inspect_rejects_corrupt_headers():
    x = G.grf((20, 20, 20), 3.0, 4)
    s = O.compress(x, O.REL, 1e-3, chunk=256).stream
    for mutate in (lambda t: t.__setitem__(0, t[0] ^ 1), lambda t: t.__setitem__(68, 3),
                   lambda t: t.__setitem__(8, 0)):
        t = s.copy()
        mutate(t)
        with pytest.raises(hiz.HizError) as e:
            hiz.inspect(t.tobytes())
        assert e.value.status == hiz.ERR_CORRUPT
    with pytest.raises(hiz.HizError):
        hiz.inspect(s[:64].tobytes())


def test_inspect_constant_stream():
    x = np.full((5, 6, 7), -1.25, np.float32)
    r = O.compress(x, O.REL, 1e-3)
    info = hiz.inspect(r.stream.tobytes())
    assert info["constant"] and info["total_bytes"] == 132


@pytest.mark.parametrize("pipeline,reorder", [(O.PIPE_TP, False), (O.PIPE_TP, True),
                                              (O.PIPE_CR, True), (O.PIPE_CR, False),
                                              (O.PIPE_HF, True)])
def test_inspect_pipeline_streams(pipeline, reorder):
    # the library's header parser accepts the oracle's streams of every
    # lossless pipeline and reports their sections
    x = G.grf((40, 33, 50), 3.0, 21)
    r = O.compress(x, O.REL, 1e-3, chunk=512, pipeline=pipeline, reorder=reorder)
    info = hiz.inspect(r.stream.tobytes())
    assert info["pipeline"] == pipeline and info["reorder"] == reorder
    assert info["total_bytes"] == r.stream.size
    if pipeline == O.PIPE_HF:
        assert info["lc_bytes"] == 0
    else:
        assert 0 < info["lc_bytes"] < r.stream.size
    bad = r.stream.copy()
    bad[54] = 7
    with pytest.raises(hiz.HizError):
        hiz.inspect(bad.tobytes())
