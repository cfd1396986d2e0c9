"""Pins of the oracle's code reordering (Sec. 5.1.4, Eq. reorder) and of its
bitwise-redundancy lossless stages (Sec. 5.2.3).

Reordering: the equation as printed is checked directly on the stride-1 level
(where it is well defined), and the whole permutation against its plain
definition by brute force -- codes grouped by interpolation level, coarsest
(largest stride) first, row-major inside a level.

Stages: small inputs whose outputs are derived by hand from the stage
definitions, and round trips.
"""
import itertools

import numpy as np
import pytest

import fieldgen as G
import oracle as O

SHAPES = [(5, 6, 7), (17, 17, 17), (33, 20, 9), (40, 3, 18), (1, 1, 1), (16, 16, 16),
          (1, 40, 33), (2, 31, 2)]


def _level(x, y, z):
    # the largest l <= 4 with 2^l dividing x, y and z
    l = 0
    while l < 4 and x % (2 << l) == 0 and y % (2 << l) == 0 and z % (2 << l) == 0:
        l += 1
    return l


@pytest.mark.parametrize("shape", SHAPES)
def test_reorder_is_level_major_row_major(shape):
    # plain definition, by brute force: stable sort of the row-major points by
    # decreasing level
    pts = list(itertools.product(*(range(d) for d in shape)))
    lv = [_level(*p) for p in pts]
    order = sorted(range(len(pts)), key=lambda i: (-lv[i], i))
    want = np.empty(len(pts), dtype=np.int64)
    want[np.array(order)] = np.arange(len(pts))
    got = np.array([O.reorder_index(shape, *p) for p in pts])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("shape", SHAPES)
def test_reorder_matches_printed_equation_at_stride_one(shape):
    # Eq. reorder as printed, at level 0 (points with an odd coordinate):
    # prefix(0) + x dy dz + y dz + z - floor((x+1)/2) floor((dy+1)/2) floor((dz+1)/2)
    #   - [x even] floor((y+1)/2) floor((dz+1)/2) - [x, y even] floor((z+1)/2),
    # prefix(0) = f_x(0) f_y(0) f_z(0), f(0) = floor((d+1)/2)
    dx, dy, dz = shape
    f0 = ((dx + 1) // 2) * ((dy + 1) // 2) * ((dz + 1) // 2)
    for x, y, z in itertools.product(range(dx), range(dy), range(dz)):
        if x % 2 == 0 and y % 2 == 0 and z % 2 == 0:
            continue
        I = f0 + x * dy * dz + y * dz + z - ((x + 1) // 2) * ((dy + 1) // 2) * ((dz + 1) // 2)
        if x % 2 == 0:
            I -= ((y + 1) // 2) * ((dz + 1) // 2)
            if y % 2 == 0:
                I -= (z + 1) // 2
        assert O.reorder_index(shape, x, y, z) == I, (x, y, z)


def test_reorder_anchors_first_and_round_trip():
    shape = (40, 33, 50)
    codes = np.random.default_rng(1).integers(0, 256, size=shape).astype(np.uint8)
    seq = O.reorder(codes)
    # the anchors (every coordinate a multiple of 16) come first, in anchor-grid order
    anchors = codes[::16, ::16, ::16].ravel()
    assert np.array_equal(seq[:anchors.size], anchors)
    assert np.array_equal(O.unreorder(seq, shape), codes)
    # the stride-1 targets are the last 7/8 or so, in row-major order
    odd = np.ones(shape, bool)
    odd[::2, ::2, ::2] = False
    assert np.array_equal(seq[-int(odd.sum()):], codes[odd])


# ---------------------------------------------------------------------------
# Stages, by hand
# ---------------------------------------------------------------------------

def _b(*v):
    return np.array(v, dtype=np.uint8)


def test_tcms1_hand():
    # (w << 1) ^ (w >> 7), arithmetic shift, on signed bytes: the quantization
    # code 128 (-128 as a signed byte) maps to 0xFF, its neighbours to 0xFE, 0xFD
    got = O.lc_stage(O.LC_TCMS, 1, _b(0x80, 0x7F, 0x81, 0x00, 0x01, 0xFF))
    assert got.tolist() == [0xFF, 0xFE, 0xFD, 0x00, 0x02, 0x01]


def test_tcms8_hand():
    words = np.array([1, -1, -2, 0, -(2 ** 63)], dtype=np.int64)
    got = O.lc_stage(O.LC_TCMS, 8, words.view(np.uint8)).view(np.uint64)
    assert got.tolist() == [2, 1, 3, 0, 2 ** 64 - 1]
    # a 3-byte tail passes through
    tail = np.concatenate([words[:1].view(np.uint8), _b(7, 8, 9)])
    assert O.lc_stage(O.LC_TCMS, 8, tail)[8:].tolist() == [7, 8, 9]


def test_bit1_hand():
    # bit p of input byte 8j+i goes to bit i of byte j of plane p
    got = O.lc_stage(O.LC_BIT, 1, _b(0x01, 0, 0, 0, 0, 0, 0, 0x80, 0xFF, 0, 0, 0, 0, 0, 0, 0, 0x5A))
    # two groups of 8 bytes -> planes of 2 bytes each, then the 1 leftover byte
    want = np.zeros(17, np.uint8)
    want[0 * 2 + 0] = 0x01          # plane 0, group 0: byte 0 has bit 0
    want[7 * 2 + 0] = 0x80          # plane 7, group 0: byte 7 has bit 7
    for p in range(8):
        want[p * 2 + 1] = 0x01      # group 1: byte 8 = 0xFF has every bit
    want[16] = 0x5A
    assert got.tolist() == want.tolist()


def test_rre1_rze1_hand():
    # RRE1 [5,5,5,7,7,0]: kept where different from the byte before (0 before
    # the first): positions 0, 3, 5 -> bitmap 0b00101001
    assert O.lc_stage(O.LC_RRE, 1, _b(5, 5, 5, 7, 7, 0)).tolist() == [6, 0, 0x29, 5, 7, 0]
    # RZE1 [0,0,3,0,4,4]: nonzero at 2, 4, 5 -> bitmap 0b00110100
    assert O.lc_stage(O.LC_RZE, 1, _b(0, 0, 3, 0, 4, 4)).tolist() == [6, 0, 0x34, 3, 4, 4]


def test_rre4_words_and_tail_hand():
    w = np.array([9, 9, 0x01020304], dtype=np.uint32).view(np.uint8)
    data = np.concatenate([w, _b(0xAA, 0xBB)])  # 14 bytes: 3 words + 2 tail bytes
    got = O.lc_stage(O.LC_RRE, 4, data)
    # kept words 0 (9 != 0) and 2 -> bitmap 0b101
    assert got.tolist() == [14, 0, 0x05, 9, 0, 0, 0, 4, 3, 2, 1, 0xAA, 0xBB]


def test_bitmap_recursion_hand():
    # 128 bytes, all zero: 16 bitmap bytes of zeros -> recursion: no bitmap
    # byte differs from the one before -> 2 zero bytes of sub-bitmap
    assert O.lc_stage(O.LC_RZE, 1, np.zeros(128, np.uint8)).tolist() == [128, 0, 0, 0]
    # one nonzero byte at 100: bitmap byte 12 = 0x10; bytes 12 and 13 differ
    # from their predecessors -> sub-bitmap bits 12, 13 = bytes [0x00, 0x30],
    # then the kept bitmap bytes 0x10, 0x00, then the kept value
    d = np.zeros(128, np.uint8)
    d[100] = 77
    assert O.lc_stage(O.LC_RZE, 1, d).tolist() == [128, 0, 0x00, 0x30, 0x10, 0x00, 77]


def test_pipelines_hand():
    # TP on 16 bytes of code 128: TCMS1 -> 0xFF x16; BIT1 -> 0xFF x16; RRE1
    # keeps the first byte only: [16, 0, bitmap 0x01 0x00, 0xFF]
    sizes, data = O.lc_encode(O.PIPE_TP, np.full(16, 128, np.uint8))
    assert sizes.tolist() == [5] and data.tolist() == [16, 0, 0x01, 0x00, 0xFF]
    # CR on 16 zero bytes: RRE4 keeps nothing -> [16, 0, 0x00]; TCMS8 has no
    # whole word; RZE1 keeps the 16 -> [3, 0, 0x01, 16]
    sizes, data = O.lc_encode(O.PIPE_CR, np.zeros(16, np.uint8))
    assert sizes.tolist() == [4] and data.tolist() == [3, 0, 0x01, 16]
    # incompressible chunks are stored raw
    rnd = np.random.default_rng(3).integers(0, 256, size=40000).astype(np.uint8)
    sizes, data = O.lc_encode(O.PIPE_TP, rnd)
    assert sizes.tolist() == [16384, 16384, 40000 - 32768] and np.array_equal(data, rnd)


@pytest.mark.parametrize("op,k", [(O.LC_TCMS, 1), (O.LC_TCMS, 8), (O.LC_BIT, 1), (O.LC_RRE, 1),
                                  (O.LC_RRE, 4), (O.LC_RZE, 1), (O.LC_RZE, 8)])
@pytest.mark.parametrize("kind", ["random", "runs", "zeros", "short"])
def test_stage_round_trip(op, k, kind):
    rng = np.random.default_rng(op * 10 + k)
    n = {"random": 16384, "runs": 16381, "zeros": 4099, "short": 5}[kind]
    if kind == "random":
        d = rng.integers(0, 256, size=n)
    elif kind == "runs":
        d = np.repeat(rng.integers(0, 4, size=n // 37 + 1), 37)[:n]
    else:
        d = np.zeros(n)
    d = d.astype(np.uint8)
    enc = O.lc_stage(op, k, d)
    assert np.array_equal(O.lc_stage(op, k, enc, inverse=True), d)


@pytest.mark.parametrize("pipeline", [O.PIPE_TP, O.PIPE_CR])
def test_lc_round_trip_chunks(pipeline):
    rng = np.random.default_rng(9)
    for n in (0, 1, 16383, 16384, 16385, 50000):
        d = np.where(rng.random(n) < 0.9, 128, rng.integers(0, 256, size=n)).astype(np.uint8)
        sizes, data = O.lc_encode(pipeline, d)
        assert len(sizes) == -(-n // 16384)
        assert np.array_equal(O.lc_decode(pipeline, sizes, data, n), d)


@pytest.mark.parametrize("pipeline", [O.PIPE_HF, O.PIPE_TP, O.PIPE_CR])
@pytest.mark.parametrize("reorder", [False, True])
def test_stream_round_trip_and_bound(pipeline, reorder):
    for shape, eb in [((40, 33, 50), 1e-3), ((17, 33, 16), 1e-4), ((3, 70, 5), 1e-2)]:
        x = G.grf(shape, 3.0, 4)
        r = O.compress(x, O.REL, eb, pipeline=pipeline, reorder=reorder, chunk=256)
        y = O.decompress(r.stream)
        assert np.array_equal(y.view(np.uint32), r.recon.view(np.uint32))
        assert np.abs(y.astype(np.float64) - x.astype(np.float64)).max() <= float(r.eps)
        assert r.stream[54] == pipeline and bool(r.stream[7] & O.FLAG_REORDER) == reorder


def test_pipelines_share_codes_and_hf_is_unchanged():
    x = G.grf((40, 33, 50), 3.0, 5)
    base = O.compress(x, O.REL, 1e-3, chunk=512)
    hf = O.compress(x, O.REL, 1e-3, chunk=512, pipeline=O.PIPE_HF, reorder=False)
    assert np.array_equal(base.stream, hf.stream)
    for pipe in (O.PIPE_TP, O.PIPE_CR):
        r = O.compress(x, O.REL, 1e-3, chunk=512, pipeline=pipe, reorder=True)
        assert np.array_equal(r.codes, base.codes)
        _, codes = O.decompress(r.stream, with_codes=True)
        assert np.array_equal(codes, base.codes)


def test_corrupt_lossless_sections_are_rejected():
    x = G.grf((40, 33, 50), 3.0, 6)
    for pipe in (O.PIPE_TP, O.PIPE_CR):
        r = O.compress(x, O.REL, 1e-3, chunk=512, pipeline=pipe, reorder=True)
        s = r.stream.copy()
        s[54] = 3  # unknown pipeline
        assert O.decompress_status(s) == O.ERR_CORRUPT
        s = r.stream.copy()
        s[120] ^= 1  # chunk count of the last stages
        assert O.decompress_status(s) == O.ERR_CORRUPT
