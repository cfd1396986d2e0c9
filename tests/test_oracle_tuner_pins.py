"""Pins of the oracle's sampled-block tuner (Sec. 5.1.3) by construction.

The tuner samples full 17^3 blocks uniformly with 0.2 % of the volume, tests
each level with every candidate predicting from the original values, sums the
errors per level and keeps the candidate with the smallest sum (ties to the
lower candidate index). The fields below make every one of those steps
visible in the result:

* Only the blocks the sampling rule selects hold a smooth field,
  f = C + K * X^2 (X the global first coordinate); every other point is
  noise. Sampling the wrong blocks, or a different number of them, brings
  noise into the sums.
* On f the cubic stencil and both one-sided quadratics are exact, so every
  cubic candidate scores exactly 0 at strides 4, 2 and 1 (where the cubic
  family is available in a full block), and the exact tie among the seven
  cubic candidates must go to cubic + multi-dimensional (index 7).
* The linear stencil along x misses f by exactly K*s^2, and along y or z it
  is exact. Each candidate's sum is then a count of targets times a fixed
  per-target error, derived by hand below. With eps = 2^18 one error unit is
  2*eps/65536 = 8, so a stride-1 miss of K = 12 is 1.5 units, which rounding
  to nearest takes to 2 (truncation would give 1).

Candidate index = spline*7 + (0 for MD, else 1 + order), order as in the
stream header: 0 (x,y,z) 1 (x,z,y) 2 (y,x,z) 3 (y,z,x) 4 (z,x,y) 5 (z,y,x).
"""
import numpy as np
import pytest

import oracle as O

K = 12           # quadratic coefficient: K*s^2/3 and K*s^2/2 stay integers
C0 = 1 << 17     # offset: every value stays below 2^19, so every stencil is exact in FP32
EPS = np.float32(2.0 ** 18)
UNIT = 2.0 * float(EPS) / 65536.0  # = 8


def _units(err):
    # error units, rounded to nearest, as the reading of "aggregated errors" states
    return int(np.floor(err / UNIT + 0.5))


# Counts of stride-s targets of one full block (local coordinates 0..16):
# O = odd multiples of s, E = even multiples, A = all multiples, per axis.
def _oea(s):
    odd = 8 // s
    even = 16 // (2 * s) + 1
    return odd, even, odd + even


def expected_lin_sums(n_blocks):
    """Hand-derived sums of the seven linear candidates per level (strides 8, 4, 2, 1)."""
    out = np.zeros((4, 7), dtype=np.int64)
    for l, s in enumerate((8, 4, 2, 1)):
        o, e, a = _oea(s)
        miss = K * s * s        # linear miss along x; y and z are exact
        # MD: x in S, |S| predictions averaged: the error is miss/|S| (exact here)
        md = (o * e * e * _units(miss) + o * (2 * o * e) * _units(miss / 2)
              + o * o * o * _units(miss / 3))
        seq_x_first = o * e * e * _units(miss)   # x last of S only when S = {x}
        seq_x_middle = o * a * e * _units(miss)  # x last when the later axis is even
        seq_x_last = o * a * a * _units(miss)    # every target with x in S
        out[l] = [md, seq_x_first, seq_x_first, seq_x_middle, seq_x_last, seq_x_middle,
                  seq_x_last]
    return out * n_blocks


def tuner_field(shape, blocks, seed):
    """Noise everywhere except the 17^3 regions of `blocks`, which hold C0 + K*X^2."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 1 << 18, size=shape).astype(np.float32)
    X = np.arange(shape[0], dtype=np.float64)[:, None, None]
    smooth = (C0 + K * X * X) * np.ones((1, shape[1], shape[2]))
    for (a, b, c) in blocks:
        sl = (slice(16 * a, 16 * a + 17), slice(16 * b, 16 * b + 17), slice(16 * c, 16 * c + 17))
        x[sl] = smooth[sl].astype(np.float32)
    return x


def check_tuner(tune):
    """Failures of the tuner pins for a tune(x, eps) -> (cfg, err) function."""
    fails = []
    # 161x145x129: 10 x 9 x 8 = 720 full blocks; N = 3,011,505 points, so
    # 0.2 % of N is 1.23 blocks of 4913 points -> 2 samples. Evenly spaced
    # at the midpoints of 720/2-wide strata: blocks floor(180) = 180 and
    # floor(540) = 540, i.e. (2,4,4) and (7,4,4) in block row-major order
    # (180 = 2*72 + 4*8 + 4, 540 = 7*72 + 4*8 + 4).
    shape = (161, 145, 129)
    x = tuner_field(shape, [(2, 4, 4), (7, 4, 4)], seed=5)
    cfg, err = tune(x, EPS)
    err = np.asarray(err, dtype=np.int64)
    want = expected_lin_sums(2)
    for l in range(4):
        if not np.array_equal(err[l, :7], want[l]):
            fails.append(f"level {l}: linear sums {err[l, :7].tolist()} != {want[l].tolist()}")
    # cubic and natural-spline candidates: linear at stride 8 (no third sample
    # in a full block); the cubic is exact at strides 4, 2, 1
    for lo in (7, 14):
        if not np.array_equal(err[0, lo:lo + 7], want[0]):
            fails.append(f"stride 8 sums {err[0, lo:lo + 7].tolist()} != {want[0].tolist()}")
    for l in (1, 2, 3):
        if np.any(err[l, 7:14] != 0):
            fails.append(f"level {l}: cubic sums {err[l, 7:14].tolist()} not all 0")
    # natural spline, SEQ(y,z,x) (index 18): along x it misses a quadratic by
    # 0.2*K*s^2 where all four samples exist, i.e. only at x = 6, 10 of stride
    # 2 (9.6 = 1.2 units -> 1); elsewhere the one-sided quadratics are exact.
    # 2 x-values x 9 x 9 targets x 2 blocks = 324 units at stride 2.
    # at stride 1 the interior miss is 2.4 = 0.3 units, which rounds to 0
    if err[1, 18] != 0 or err[2, 18] != 324 or err[3, 18] != 0:
        fails.append(f"natural-spline SEQ(y,z,x) sums {err[:, 18].tolist()}")
    # stride 8: SEQ(x,y,z) and SEQ(x,z,y) tie (and so do their cubic twins):
    # the lowest index, 1, wins. Strides 4, 2, 1: the seven zeros tie: index 7.
    want_cfg = ((O.LIN, O.SEQ, 0), (O.CUB, O.MD, 0), (O.CUB, O.MD, 0), (O.CUB, O.MD, 0))
    if tuple(tuple(int(v) for v in c) for c in cfg) != want_cfg:
        fails.append(f"picks {cfg} != {want_cfg}")

    # One sample: 0.2 % of 81^3 = 531,441 points is 0.22 blocks -> 1 sample,
    # at floor(0.5 * 125) = 62 = (2,2,2) in a 5x5x5 grid of full blocks.
    shape = (81, 81, 81)
    x = tuner_field(shape, [(2, 2, 2)], seed=6)
    cfg, err = tune(x, EPS)
    err = np.asarray(err, dtype=np.int64)
    if not np.array_equal(err[:, :7], expected_lin_sums(1)):
        fails.append(f"81^3: linear sums {err[:, :7].tolist()}")
    if np.any(err[1:, 7:14] != 0):
        fails.append("81^3: cubic sums not 0")

    # A 2-D field (flat x axis): blocks of 17 x 17 points, 0.2 % of N is
    # 0.16 blocks of 289 -> 1 sample, at floor(0.5 * 90) = 45 of the 10 x 9
    # grid of full 2-D blocks = (0, 5, 0). The quadratic now runs along y:
    # SEQ orders with z after y predict {y, z} targets along z (exact), the
    # others along y.
    shape = (1, 161, 145)
    rng = np.random.default_rng(8)
    x = rng.integers(0, 1 << 18, size=shape).astype(np.float32)
    Y = np.arange(80, 97, dtype=np.float64)[:, None]
    x[0, 80:97, 0:17] = ((C0 + K * Y * Y) * np.ones((1, 17))).astype(np.float32)
    cfg, err = tune(x, EPS)
    err = np.asarray(err, dtype=np.int64)
    for l, s_ in enumerate((8, 4, 2, 1)):
        o, e, a = _oea(s_)
        miss = K * s_ * s_
        oe, oa = o * e * _units(miss), o * a * _units(miss)
        md = o * e * _units(miss) + o * o * _units(miss / 2)
        want2 = [md, oe, oa, oe, oe, oa, oa]
        if err[l, :7].tolist() != want2:
            fails.append(f"2-D level {l}: linear sums {err[l, :7].tolist()} != {want2}")
        if l > 0 and np.any(err[l, 7:14] != 0):
            fails.append(f"2-D level {l}: cubic sums not 0")
    if tuple(tuple(int(v) for v in c) for c in cfg) != want_cfg:
        fails.append(f"2-D picks {cfg}")

    # No full block (a side below 17): the default, cubic + MD everywhere.
    x = np.random.default_rng(7).standard_normal((40, 16, 40)).astype(np.float32)
    cfg, err = tune(x, np.float32(1e-3))
    if tuple(tuple(int(v) for v in c) for c in cfg) != ((O.CUB, O.MD, 0),) * 4 or np.any(
            np.asarray(err) != 0):
        fails.append(f"no full block: {cfg}")
    return fails


def test_tuner_sampling_scoring_and_ties():
    fails = check_tuner(O.tune)
    assert not fails, "\n".join(fails)


def test_expected_sums_are_not_degenerate():
    # the hand-derived sums separate the candidates they are meant to separate
    want = expected_lin_sums(2)
    assert want[0, 1] == want[0, 2] < want[0, 3] < want[0, 4] < want[0, 0] + 10 ** 6
    assert _units(K * 1.0) == 2 and int(K / UNIT) == 1  # rounding, not truncation, at stride 1
