"""Pins of the CPU oracle to what the paper and the mathematics fix.

None of these tests re-types the oracle's formulas: each checks a property that
a mistake in the oracle (a wrong weight, sign, index, axis, order or rounding)
would break -- polynomial exactness of the spline stencils, closed forms of the
block machinery, the error bound of Eq. "general", hand-derived golden codes,
optimality and canonical form of the Huffman code, and symmetry under axis
transposition.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import fieldgen as G
import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def f32(v):
    return np.float32(v)


# ---------------------------------------------------------------------------
# Spline stencils (Sec. 5.1.2): Lagrange exactness on integer polynomials
# ---------------------------------------------------------------------------

def _poly(coefs, t):
    return sum(c * t ** i for i, c in enumerate(coefs))


@pytest.mark.parametrize("seed", range(20))
@pytest.mark.parametrize("s", [1, 2, 4, 8])
def test_stencil_polynomial_exactness(seed, s):
    rng = np.random.default_rng(seed)
    t0 = int(rng.integers(-40, 40))
    # values at t0-3s, t0-s, t0+s, t0+3s of integer polynomials; all |v| < 2^19
    def samples(coefs):
        return [f32(_poly(coefs, t0 + k * s)) for k in (-3, -1, 1, 3)]
    cub = [int(v) for v in rng.integers(-3, 4, size=4)]
    a, b, c, d = samples(cub)
    v, r = O.stencil(O.CUB, a, b, c, d, 1, 1, 1)
    assert r == 4 and v == f32(_poly(cub, t0)), "cubic stencil must reproduce cubics"
    quad = [int(v) for v in rng.integers(-5, 6, size=3)]
    a, b, c, d = samples(quad)
    v, r = O.stencil(O.CUB, a, b, c, d, 0, 1, 1)  # right-sided quadratic
    assert r == 3 and v == f32(_poly(quad, t0))
    v, r = O.stencil(O.CUB, a, b, c, d, 1, 1, 0)  # left-sided quadratic
    assert r == 3 and v == f32(_poly(quad, t0))
    lin = [int(v) for v in rng.integers(-9, 10, size=2)]
    a, b, c, d = samples(lin)
    for spline in (O.LIN, O.CUB):
        v, r = O.stencil(spline, a, b, c, d, 0, 1, 0)
        assert r == 2 and v == f32(_poly(lin, t0))
        v, r = O.stencil(spline, a, b, c, d, 1, 0, 0)  # extrapolation from below
        assert r == 1 and v == f32(_poly(lin, t0))
    v, r = O.stencil(O.LIN, a, b, c, d, 1, 1, 1)  # LIN spline ignores the outer samples
    assert r == 2 and v == f32(_poly(lin, t0))
    const = f32(rng.integers(-100, 100))
    v, r = O.stencil(O.CUB, 0, const, 0, 0, 0, 0, 0)
    assert r == 0 and v == const


def test_stencil_orders_are_not_higher_than_claimed():
    # the cubic stencil must fail on a quartic, the quadratic ones on a cubic,
    # the linear one on a quadratic: catches a stencil that is "too exact"
    t = [-3, -1, 1, 3]
    q4 = [f32(v ** 4) for v in t]
    v, _ = O.stencil(O.CUB, *q4, 1, 1, 1)
    assert v != 0
    c3 = [f32(v ** 3 + 5) for v in t]
    v, _ = O.stencil(O.CUB, *c3, 0, 1, 1)
    assert v != 5
    v, _ = O.stencil(O.CUB, *c3, 1, 1, 0)
    assert v != 5
    sq = [f32(v ** 2) for v in t]
    v, _ = O.stencil(O.LIN, *sq, 0, 1, 0)
    assert v != 0


@pytest.mark.parametrize("s", [1, 2, 4, 8])
def test_stencil_error_closed_forms_on_cube(s):
    # Interpolating f(t) = t^3 at t0 from nodes t0 + k*s: the error f - p is
    # f'''/3! * prod(t0 - node) = prod over the node offsets of (-k*s).
    for t0 in (-17, 0, 5, 23):
        f = lambda t: f32(t ** 3)  # noqa: E731
        a, b, c, d = f(t0 - 3 * s), f(t0 - s), f(t0 + s), f(t0 + 3 * s)
        v, _ = O.stencil(O.CUB, a, b, c, d, 0, 1, 1)  # nodes -1, 1, 3
        assert v == f32(t0 ** 3 - (s * (-s) * (-3 * s)))
        v, _ = O.stencil(O.CUB, a, b, c, d, 1, 1, 0)  # nodes -3, -1, 1
        assert v == f32(t0 ** 3 - ((3 * s) * s * (-s)))
        v, _ = O.stencil(O.LIN, a, b, c, d, 0, 1, 0)  # nodes -1, 1 (f'' term too)
        assert v == f32(((t0 - s) ** 3 + (t0 + s) ** 3) / 2)


# ---------------------------------------------------------------------------
# Block machinery from original values (the tuner's predictions)
# ---------------------------------------------------------------------------

def _targets(n, s):
    for t in itertools.product(*(range(0, k, s) for k in n)):
        odd = [(v // s) & 1 for v in t]
        if any(odd):
            yield t, odd


def _presence(t, axis, s, n):
    tk = t[axis]
    return tk - 3 * s >= 0, tk + s <= n[axis] - 1, tk + 3 * s <= n[axis] - 1


@pytest.mark.parametrize("shape", [(17, 17, 17), (17, 9, 13), (5, 17, 11)])
def test_cubic_exact_inside_blocks(shape):
    # sum of per-axis integer cubics: the cubic stencil along any axis is exact,
    # so every target whose used stencils are all cubic is predicted exactly,
    # for MD (averages of equal exact values) and for every SEQ order.
    x, y, z = np.meshgrid(*(np.arange(k, dtype=np.float64) for k in shape), indexing="ij")
    f = (x ** 3 - 4 * x ** 2 + 2 * x) + (2 * y ** 3 - y) + (-(z ** 3) + 3 * z ** 2 + 7)
    buf = f.astype(np.float32)
    n = shape
    checked = 0
    for s in (8, 4, 2, 1):
        for t, odd in _targets(n, s):
            axes = [k for k in range(3) if odd[k]]
            full = [all(_presence(t, k, s, n)) for k in axes]
            if all(full):
                assert O.predict(buf, t, s, O.CUB, O.MD) == buf[t]
                checked += 1
            for perm in range(6):
                last = [k for k in O.PERMS[perm] if odd[k]][-1]
                if all(_presence(t, last, s, n)):
                    assert O.predict(buf, t, s, O.CUB, O.SEQ, perm) == buf[t]
    assert checked > 0


def test_md_average_closed_form():
    # f = x^2 y^2 (z-independent). At a 2-D target (x/s, y/s odd, z/s even) the
    # linear stencils give p_x = (x^2+s^2) y^2 and p_y = x^2 (y^2+s^2); the MD
    # prediction is their mean x^2y^2 + s^2 (x^2+y^2)/2. At a 3-D target the
    # z stencil is exact (p_z = x^2y^2) and all three are averaged.
    n = (17, 17, 17)
    x, y, z = np.meshgrid(*(np.arange(k, dtype=np.float64) for k in n), indexing="ij")
    buf = (x ** 2 * y ** 2).astype(np.float32)
    for s in (1, 2, 4):
        for t, odd in _targets(n, s):
            if not (odd[0] and odd[1]):
                continue
            X, Y, Z = t
            if not (X + s <= 16 and Y + s <= 16):
                continue
            if odd[2] and not Z + s <= 16:
                continue
            px = (X * X + s * s) * Y * Y
            py = X * X * (Y * Y + s * s)
            got = O.predict(buf, t, s, O.LIN, O.MD)
            if not odd[2]:
                assert got == f32((px + py) / 2)
            else:
                pz = X * X * Y * Y
                assert got == f32(((f32(px) + f32(py)) + f32(pz)) / f32(3))


def test_md_keeps_only_highest_order():
    # one axis has a cubic stencil, the other only a quadratic one: MD must use
    # the cubic prediction alone (Sec. 5.1.2 example).
    n = (17, 17, 17)
    t = (2, 6, 0)  # s = 2: x=2 (no t-3s -> quadratic), y=6 (cubic), z even
    x, y, z = np.meshgrid(*(np.arange(k, dtype=np.float64) for k in n), indexing="ij")
    buf = (x ** 3 + (y - 3) ** 3).astype(np.float32)
    # y-cubic exact along y; along x the quadratic stencil is off by 3s^3 = 24
    assert O.predict(buf, t, 2, O.CUB, O.MD) == buf[t]
    assert O.predict(buf, t, 2, O.CUB, O.SEQ, 1) == buf[t]          # order (x,z,y): y last
    assert O.predict(buf, t, 2, O.CUB, O.SEQ, 2) == f32(buf[t] - 24)  # order (y,x,z): x last


# ---------------------------------------------------------------------------
# Error bound (Sec. 3.1 Eq. "general", Sec. 6.1.4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("eb", [1e-1, 1e-2, 1e-3, 1e-4, 1e-6, 3.7e-5])
def test_eps_rounds_down(eb):
    rng = np.random.default_rng(7)
    for _ in range(50):
        lo, hi = sorted(rng.normal(size=2).astype(np.float32))
        e = O.eps(O.REL, eb, lo, hi)
        exact = eb * (float(hi) - float(lo))
        assert float(e) <= exact
        assert float(np.nextafter(e, np.float32(np.inf))) > exact


def _check_bound(x, y, eps):
    err = np.abs(x.astype(np.float64) - y.astype(np.float64))
    assert err.max() <= float(eps), (err.max(), float(eps))


CFGS = [O.DEFAULT_CFG, ((O.LIN, O.MD, 0),) * 4, ((O.CUB, O.SEQ, 0),) * 4,
        ((O.LIN, O.SEQ, 5),) * 4, ((O.CUB, O.SEQ, 3), (O.LIN, O.MD, 0), (O.CUB, O.SEQ, 1),
                                   (O.CUB, O.MD, 0))]


@pytest.mark.parametrize("seed", range(12))
def test_bound_random_shapes(seed):
    rng = np.random.default_rng(1000 + seed)
    shape = tuple(int(v) for v in rng.integers(1, 41, size=3))
    kind = ["grf", "noise", "grf", "const"][seed % 4]
    x = G.random_small(shape, seed, kind) * np.float32(rng.uniform(0.1, 50))
    eb = float(10 ** rng.uniform(-6, -1))
    mode = int(rng.integers(0, 2))
    cfg = CFGS[seed % len(CFGS)]
    chunk = int(2 ** rng.integers(8, 12))
    r = O.compress(x, mode, eb if mode == O.REL else eb * float(np.ptp(x) or 1), tune=bool(seed % 2),
                   cfg=cfg, chunk=chunk)
    y = O.decompress(r.stream)
    _check_bound(x, y, r.eps)
    # encoder and decoder agree bit for bit on every reconstructed value
    assert np.array_equal(r.recon.view(np.uint32), y.view(np.uint32))
    if r.stream[7] & 1:  # constant-field stream: header and one value
        assert r.stream.size == 132 and np.all(x == x.flat[0])
        return
    # the histogram counts all N codes; code 0 marks exactly the outliers
    assert int(r.hist.sum()) == x.size and int(r.hist[0]) == r.n_out
    assert int((r.codes == 0).sum()) == r.n_out


def test_bound_small_field_all_ebs():
    x = G.field_small()
    for eb in (1e-2, 1e-3, 1e-4, 1e-5):
        r = O.compress(x, O.REL, eb, chunk=512)
        y = O.decompress(r.stream)
        _check_bound(x, y, r.eps)
        assert float(r.eps) <= eb * (float(x.max()) - float(x.min()))


def test_smooth_field_has_no_outliers_and_centred_codes():
    # a sign or scale mistake in quantization makes a smooth field mostly outliers
    x = G.grf((40, 40, 40), 4.0, 5)
    r = O.compress(x, O.REL, 1e-2, tune=False)
    assert r.n_out == 0
    q = r.codes.astype(np.int64) - 128
    assert abs(q.mean()) < 0.05 and np.abs(q).max() < 40


# ---------------------------------------------------------------------------
# Closed form: multilinear fields are reproduced exactly
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cfg", CFGS)
def test_multilinear_closed_form(cfg):
    shape = (33, 49, 65)  # every side = 1 (mod 16): no truncated stencils
    x = G.multilinear(shape)
    chunk = 1024
    r = O.compress(x, O.ABS, 0.5, tune=False, cfg=cfg, chunk=chunk)
    assert np.all(r.codes == 128)
    assert r.n_out == 0
    assert np.array_equal(r.recon.view(np.uint32), x.view(np.uint32))
    ln, _ = O.codebook(r.hist)
    assert ln[128] == 1 and ln.sum() == 1
    n = x.size
    words = sum(-(-min(chunk, n - k) // 32) for k in range(0, n, chunk))
    total = int(np.frombuffer(r.stream[80:88].tobytes(), np.uint64)[0])
    assert total == words
    assert np.array_equal(O.decompress(r.stream), x)


# ---------------------------------------------------------------------------
# Hand-derived golden codes of a tiny block
# ---------------------------------------------------------------------------

def test_tiny_block_golden(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "tiny_block_2x2x2.json")))
    x = np.array(g["values_xyz"], dtype=np.float32)
    for case in g["cases"]:
        spline = {"lin": O.LIN, "cub": O.CUB}[case["spline"]]
        scheme = {"md": O.MD, "seq": O.SEQ}[case["scheme"]]
        cfg = ((spline, scheme, case["order"]),) * 4
        r = O.compress(x, O.ABS, g["eb"], tune=False, cfg=cfg, chunk=256)
        assert r.codes.tolist() == case["codes_xyz"], case
        assert r.recon.tolist() == case["recon_xyz"], case
        assert np.array_equal(O.decompress(r.stream), r.recon)


def test_quantizer_edges():
    # dims (1,1,3), ABS eb 0.5 (2 eps = 1): z=2 is predicted by copying z=0
    # (no upper neighbour), then z=1 by the linear midpoint.
    def code_at_2(v2):
        x = np.array([[[0.0, 0.0, v2]]], dtype=np.float32)
        return int(O.compress(x, O.ABS, 0.5, tune=False, chunk=256).codes[0, 0, 2])
    assert code_at_2(127.0) == 255
    assert code_at_2(-127.0) == 1
    assert code_at_2(128.0) == 0          # |q| = 128 -> outlier
    assert code_at_2(127.5) == 0          # rounds half to even -> 128 -> outlier
    assert code_at_2(126.5) == 254        # rounds half to even -> 126; |err| = eps accepted
    assert code_at_2(-127.5) == 0
    assert code_at_2(0.49) == 128


# ---------------------------------------------------------------------------
# Axis symmetry: transposing the field permutes the dimension order
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("axes", [(2, 1, 0), (1, 0, 2), (0, 2, 1), (1, 2, 0)])
@pytest.mark.parametrize("perm", [0, 3, 5])
def test_transpose_symmetry_seq(axes, perm):
    # SEQ(order) on x equals SEQ(order mapped through the transposition) on x.T,
    # code for code and value for value: pins axis strides, extents and ownership.
    x = G.grf((20, 37, 50), 3.0, 11)
    order = O.PERMS[perm]
    inv = {a: i for i, a in enumerate(axes)}  # old axis -> new axis
    new_order = tuple(inv[a] for a in order)
    new_perm = O.PERMS.index(new_order)
    r1 = O.compress(x, O.REL, 1e-3, tune=False, cfg=((O.CUB, O.SEQ, perm),) * 4, chunk=256)
    xt = np.ascontiguousarray(np.transpose(x, axes))
    r2 = O.compress(xt, O.REL, 1e-3, tune=False, cfg=((O.CUB, O.SEQ, new_perm),) * 4, chunk=256)
    assert np.array_equal(np.transpose(r1.codes, axes), r2.codes)
    assert np.array_equal(np.transpose(r1.recon, axes).view(np.uint32), r2.recon.view(np.uint32))


def test_transpose_symmetry_tuner_single_block():
    # one full 17^3 block is the whole sample: transposing x<->z maps SEQ order
    # (a,b,c) to its mirror and leaves MD error sums unchanged.
    x = G.grf((17, 17, 17), 3.0, 3)
    eps = O.eps(O.REL, 1e-3, x.min(), x.max())
    _, e1 = O.tune(x, eps)
    _, e2 = O.tune(np.ascontiguousarray(x.transpose(2, 1, 0)), eps)
    swap = {0: 2, 1: 1, 2: 0}
    for spline in (0, 1):
        for perm in range(6):
            mapped = O.PERMS.index(tuple(swap[a] for a in O.PERMS[perm]))
            assert np.array_equal(e1[:, spline * 7 + 1 + perm], e2[:, spline * 7 + 1 + mapped])
    # LIN-MD: 3-term averages are summed in x,y,z order, so allow the last bit
    # of those terms; 1- and 2-term averages are symmetric exactly
    assert np.allclose(e1[:, 0].astype(float), e2[:, 0].astype(float), rtol=1e-6)


def test_tuner_prefers_cubic_on_cubic_field():
    shape = (33, 33, 33)
    x, y, z = np.meshgrid(*(np.arange(k, dtype=np.float64) for k in shape), indexing="ij")
    f = ((z - 16) ** 3 / 300.0 + np.sin(x / 5.0) + (y / 9.0) ** 2).astype(np.float32)
    eps = O.eps(O.REL, 1e-4, f.min(), f.max())
    cfg, err = O.tune(f, eps)
    assert cfg[3][0] == O.CUB  # stride 1
    assert err[3, 7] < err[3, 0]


# ---------------------------------------------------------------------------
# Huffman codebook (Sec. 5.2.2-5.2.3)
# ---------------------------------------------------------------------------

def _brute_force_cost(freqs):
    # minimal sum f*l over all complete prefix codes (Kraft equality)
    n = len(freqs)
    best = None
    for ls in itertools.product(range(1, n), repeat=n):
        if sum(2.0 ** -l for l in ls) != 1.0:
            continue
        c = sum(f * l for f, l in zip(freqs, ls))
        best = c if best is None or c < best else best
    return best


@pytest.mark.parametrize("seed", range(25))
def test_codebook_optimal_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    syms = rng.choice(256, size=n, replace=False)
    freqs = [int(v) for v in rng.integers(1, 60, size=n)]
    if seed % 5 == 0:
        freqs = [5] * n  # all ties
    hist = np.zeros(256, np.uint64)
    hist[syms] = freqs
    ln, _ = O.codebook(hist)
    cost = sum(f * int(ln[s]) for s, f in zip(syms, freqs))
    assert cost == _brute_force_cost(freqs)
    assert ln[np.setdiff1d(np.arange(256), syms)].sum() == 0


def _check_prefix_code(ln, cd):
    used = [(int(ln[s]), int(cd[s]), s) for s in range(256) if ln[s]]
    if len(used) > 1:
        assert sum(2.0 ** -l for l, _, _ in used) == 1.0  # Kraft equality
    strs = [format(c, f"0{l}b") for l, c, _ in used]
    assert all(len(s) == l for s, (l, _, _) in zip(strs, used))
    for a, b in itertools.permutations(strs, 2):
        assert not b.startswith(a)  # prefix-free
    # canonical: ordered by (length, symbol) the codes increase as bit strings
    order = sorted(used, key=lambda u: (u[0], u[2]))
    for (l1, c1, _), (l2, c2, _) in zip(order, order[1:]):
        assert (c1 + 1) << (l2 - l1) == c2


@pytest.mark.parametrize("seed", range(10))
def test_codebook_prefix_canonical_shannon(seed):
    rng = np.random.default_rng(seed)
    hist = np.zeros(256, np.uint64)
    k = int(rng.integers(2, 257))
    syms = rng.choice(256, size=k, replace=False)
    hist[syms] = rng.geometric(0.05, size=k)
    ln, cd = O.codebook(hist)
    _check_prefix_code(ln, cd)
    p = hist[hist > 0].astype(np.float64) / hist.sum()
    H = -(p * np.log2(p)).sum()
    avg = (hist.astype(np.float64) * ln).sum() / hist.sum()
    assert H <= avg + 1e-12 < H + 1


def test_codebook_single_symbol_and_length_cap():
    hist = np.zeros(256, np.uint64)
    hist[128] = 1000
    ln, cd = O.codebook(hist)
    assert ln[128] == 1 and ln.sum() == 1 and cd[128] == 0
    # Fibonacci counts make the Huffman tree a chain of depth n-1 = 39 > 32
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    hist = np.zeros(256, np.uint64)
    hist[:40] = fib
    ln, cd = O.codebook(hist)
    assert ln.max() <= 32 and (ln[:40] > 0).all()
    _check_prefix_code(ln, cd)


def test_canonical_rfc1951_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "rfc1951_canonical.json")))
    cd = O.canonical(g["lengths"])
    got = [format(int(c), f"0{l}b") for c, l in zip(cd, g["lengths"])]
    assert got == g["codes_binary"]


@pytest.mark.parametrize("kind", ["random", "skewed", "single", "all256", "fib"])
@pytest.mark.parametrize("chunk", [256, 1024, 4096])
def test_lossless_roundtrip(kind, chunk):
    rng = np.random.default_rng(hash((kind, chunk)) % 2 ** 32)
    n = int(rng.integers(1, 20000))
    if kind == "random":
        codes = rng.integers(0, 256, size=n).astype(np.uint8)
    elif kind == "skewed":
        codes = np.clip(np.round(rng.normal(128, 4, size=n)), 0, 255).astype(np.uint8)
    elif kind == "single":
        codes = np.full(n, 77, np.uint8)
    elif kind == "all256":
        codes = np.concatenate([np.arange(256, dtype=np.uint8),
                                rng.integers(0, 256, size=n).astype(np.uint8)])
    else:
        fib = [1, 1]
        while len(fib) < 40:
            fib.append(fib[-1] + fib[-2])
        codes = np.concatenate([np.full(min(f, 3000), i, np.uint8) for i, f in enumerate(fib)])
        rng.shuffle(codes)
    hist = np.bincount(codes, minlength=256).astype(np.uint64)
    if kind == "fib":
        hist = np.zeros(256, np.uint64)
        hist[:40] = fib
    ln, cd = O.codebook(hist)
    words, counts = O.huff_encode(codes, chunk, ln, cd)
    assert len(counts) == -(-codes.size // chunk)
    bits = sum(int(ln[c]) for c in codes)
    assert words.size * 32 >= bits
    assert np.array_equal(O.huff_decode(words, counts, codes.size, chunk, ln), codes)


# ---------------------------------------------------------------------------
# Stream and error paths
# ---------------------------------------------------------------------------

def test_error_paths():
    x = G.grf((20, 20, 20), 3.0, 1)
    with pytest.raises(O.OracleError) as e:
        O.compress(x, O.REL, 0.0)
    assert e.value.rc == O.ERR_ARG
    with pytest.raises(O.OracleError) as e:
        O.compress(x, O.REL, 1e-3, chunk=300)
    assert e.value.rc == O.ERR_ARG
    bad = x.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.compress(bad, O.REL, 1e-3)
    assert e.value.rc == O.ERR_NONFINITE
    bad[3, 4, 5] = np.inf
    with pytest.raises(O.OracleError) as e:
        O.compress(bad, O.ABS, 1e-3)
    assert e.value.rc == O.ERR_NONFINITE


def test_corrupt_streams_are_rejected():
    x = G.grf((24, 30, 18), 3.0, 2)
    s = O.compress(x, O.REL, 1e-4, chunk=256).stream
    assert O.decompress_status(s) == O.OK
    assert O.decompress_status(s[:100]) == O.ERR_CORRUPT       # truncated header
    assert O.decompress_status(s[:-4]) == O.ERR_CORRUPT        # truncated payload
    t = s.copy(); t[0] ^= 1
    assert O.decompress_status(t) == O.ERR_CORRUPT             # magic
    t = s.copy(); t[384] ^= 1
    assert O.decompress_status(t) == O.ERR_CORRUPT             # chunk word count
    t = s.copy(); t[68] = 3
    assert O.decompress_status(t) == O.ERR_CORRUPT             # chunk size
    t = s.copy(); t[128 + 128] += 1
    assert O.decompress_status(t) == O.ERR_CORRUPT             # code lengths break Kraft


def test_constant_field_rel_and_abs():
    x = np.full((9, 20, 33), 2.5, np.float32)
    r = O.compress(x, O.REL, 1e-3)
    assert r.stream.size == 132
    assert np.array_equal(O.decompress(r.stream), x)
    r = O.compress(x, O.ABS, 1e-3, tune=False)
    assert np.all(r.codes == 128) and np.array_equal(O.decompress(r.stream), x)


def test_degenerate_shapes():
    for shape in [(1, 1, 1), (1, 1, 50), (1, 40, 1), (17, 1, 17), (16, 16, 16), (2, 3, 65)]:
        x = G.random_small(shape, 3, "noise")
        r = O.compress(x, O.REL, 1e-2, chunk=256)
        y = O.decompress(r.stream)
        _check_bound(x, y, r.eps)
        assert np.array_equal(r.recon.view(np.uint32), y.view(np.uint32))


def test_psnr_closed_form():
    # PSNR over the value range (Sec. 6.1.4): values on a 2^-7 grid spanning
    # 999/128, every one shifted by exactly 2^-6, so MSE = 2^-12 and
    # PSNR = 20 log10(999/128) + 120 log10(2) = 59.97 dB.
    x = ((np.arange(1000) - 300) / 128.0).astype(np.float32)
    y = x + np.float32(2.0 ** -6)
    assert O.psnr(x, y) == pytest.approx(20 * math.log10(999 / 128) + 120 * math.log10(2), abs=1e-9)
    assert O.psnr(x, x) == float("inf")


def test_huffman_tie_rule_golden(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "huffman_tiebreak.json")))
    hist = np.zeros(256, np.uint64)
    hist[g["symbols"]] = g["counts"]
    ln, _ = O.codebook(hist)
    assert [int(ln[s]) for s in g["symbols"]] == g["lengths"]


# ---------------------------------------------------------------------------
# Natural cubic spline candidate (Sec. 5.1.3, "multiple interpolation splines")
# ---------------------------------------------------------------------------

def test_natural_spline_matches_scipy():
    # the natural cubic spline through the samples at -3s, -s, s, 3s (zero
    # second derivative at the outer two), evaluated at the midpoint, as
    # scipy's CubicSpline(bc_type="natural") computes it
    from scipy.interpolate import CubicSpline
    rng = np.random.default_rng(77)
    for _ in range(200):
        a, b, c, d = rng.uniform(-4, 4, 4).astype(np.float32)
        want = CubicSpline([-3.0, -1.0, 1.0, 3.0], np.array([a, b, c, d], np.float64),
                           bc_type="natural")(0.0)
        got, rank = O.stencil(O.NAT, a, b, c, d, True, True, True)
        assert rank == 4
        assert abs(float(got) - float(want)) <= 4 * np.spacing(np.float32(abs(want) + 8))


def test_natural_spline_exact_cases():
    # weights (-3, 23, 23, -3) / 40: a line is reproduced, a parabola is not
    for (a, b, c, d) in [(-3.0, -1.0, 1.0, 3.0), (10.0, 14.0, 18.0, 22.0)]:
        got, _ = O.stencil(O.NAT, a, b, c, d, True, True, True)
        assert got == np.float32((b + c) / 2)
    got, _ = O.stencil(O.NAT, 9.0, 1.0, 1.0, 9.0, True, True, True)  # x^2 at -3, -1, 1, 3
    assert got == np.float32(-0.2)
    # without all four samples it falls back exactly like the cubic
    for pa, pc, pd in [(False, True, True), (True, True, False), (False, True, False),
                       (True, False, False), (False, False, False)]:
        n = O.stencil(O.NAT, 2.0, 3.0, 7.0, 5.0, pa, pc, pd)
        cb = O.stencil(O.CUB, 2.0, 3.0, 7.0, 5.0, pa, pc, pd)
        assert n == cb
