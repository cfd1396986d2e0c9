"""Planted mistakes in the oracle's tuner must fail the tuner pins.

Each case copies the oracle's C source, changes one step of the sampled-block
tuner (Sec. 5.1.3) in the way a plausible misreading or typo would, builds the
copy in a temporary folder and runs the pins of test_oracle_tuner_pins against
it. The mistakes stay on the CPU, in throw-away copies; the oracle itself is
never modified.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as OO
from test_oracle_tuner_pins import check_tuner

MUTATIONS = {
    # evenly spaced samples at the stratum starts instead of their midpoints
    "sample_index": ("uint64_t idx = ((2 * j + 1) * n_full) / (2 * n_s);",
                     "uint64_t idx = (j * n_full) / n_s;"),
    # 2 % of the volume instead of 0.2 %
    "sample_count": ("cdiv(2 * N, 1000ull * vol)", "cdiv(20 * N, 1000ull * vol)"),
    # rounding the sample count down instead of up
    "sample_count_floor": ("uint64_t n_s = cdiv(2 * N, 1000ull * vol);",
                           "uint64_t n_s = (2 * N) / (1000ull * vol);"),
    # ties to the higher candidate index
    "tie_rule": ("if (err[l][cand] < err[l][best])", "if (err[l][cand] <= err[l][best])"),
    # error units truncated instead of rounded to nearest
    "unit_rounding": ("(uint64_t)(w + 0.5)", "(uint64_t)(w)"),
    # target values perturbed before the error is taken
    "target_scaled": ("float e = fabsf(xv - p);", "float e = fabsf(xv * 1.0001f - p);"),
    # block index decomposed with the axes swapped
    "block_order": ("uint64_t c = idx % f[2], b = (idx / f[2]) % f[1], a = idx / (f[1] * f[2]);",
                    "uint64_t a = idx % f[2], b = (idx / f[2]) % f[1], c = idx / (f[1] * f[2]);"),
    # candidates mapped to the wrong spline
    "candidate_spline": ("int spline = cand / 7, r = cand % 7;",
                         "int spline = 1 - cand / 7, r = cand % 7;"),
}


def _build(tmp_path, name, old, new):
    src = open(OO.SRC).read()
    assert src.count(old) == 1, f"mutation {name}: pattern not found exactly once"
    d = tmp_path / name
    d.mkdir()
    (d / "hiz_oracle.c").write_text(src.replace(old, new))
    (d / "hiz_oracle.h").write_text(open(os.path.join(OO.HERE, "hiz_oracle.h")).read())
    lib = d / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(lib), str(d / "hiz_oracle.c"), "-lm"])
    L = C.CDLL(str(lib))
    L.orc_tune.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.c_float, C.c_void_p, C.c_void_p]
    return L


def _tune_with(L):
    def tune(x, eps):
        x = np.ascontiguousarray(x, dtype=np.float32)
        cfg = ((C.c_uint8 * 3) * 4)()
        err = np.zeros((4, OO.CANDS), dtype=np.uint64)
        dims = (C.c_uint64 * 3)(*x.shape)
        rc = L.orc_tune(x.ctypes.data, dims, float(eps), C.byref(cfg), err.ctypes.data)
        assert rc == 0
        return OO.cfg_tuple(cfg), err
    return tune


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_tuner_mutation_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    L = _build(tmp_path, name, old, new)
    assert check_tuner(_tune_with(L)), f"mutation {name} passed every tuner pin"


def test_unmutated_copy_passes(tmp_path):
    L = _build(tmp_path, "none", "float e = fabsf(xv - p);", "float e = fabsf(xv - p);")
    assert check_tuner(_tune_with(L)) == []
