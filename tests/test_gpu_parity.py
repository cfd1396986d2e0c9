"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

For every case the compressed stream must be byte-identical to the oracle's
and the decompressed field bit-identical to the oracle's decompression; the
error bound is checked in FP64 on every element.
"""
import sys

import numpy as np
import pytest

import fieldgen as G
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_11165_amd import hiz
    return hiz.Context(0)


def _gpu_roundtrip(ctx, x, mode, eb, tune, cfg, chunk, tile_z=0):
    from paper_2507_11165_amd import hiz
    dev = torch.device("cuda:0")
    p = hiz.make_params(tune=tune, level_cfg=cfg, chunk=chunk, tile_z=tile_z)
    z = ctx.compress(torch.from_numpy(np.ascontiguousarray(x)).to(dev), mode, eb, p)
    y = ctx.decompress(z)
    torch.cuda.synchronize()
    return z.cpu().numpy(), y.cpu().numpy()


def check_case(ctx, x, mode=O.REL, eb=1e-3, tune=True, cfg=O.DEFAULT_CFG, chunk=1024, tile_z=0):
    _say(f"case shape={x.shape} mode={mode} eb={eb} tune={tune} cfg={cfg} chunk={chunk} tz={tile_z}")
    zs, y = _gpu_roundtrip(ctx, x, mode, eb, tune, cfg, chunk, tile_z)
    ref = O.compress(x, mode, eb, tune=tune, cfg=cfg, chunk=chunk, debug=False)
    if zs.size != ref.stream.size or not np.array_equal(zs, ref.stream):
        n = min(zs.size, ref.stream.size)
        diff = np.nonzero(zs[:n] != ref.stream[:n])[0]
        raise AssertionError(f"stream differs: sizes gpu {zs.size} oracle {ref.stream.size}; "
                             f"first differing byte {diff[:8]}")
    yr = O.decompress(ref.stream)
    assert np.array_equal(y.view(np.uint32), yr.view(np.uint32)), "reconstruction differs"
    err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max()
    eps = float(ref.eps) if not (ref.stream[7] & 1) else 0.0
    assert err <= eps, (err, eps)
    return zs, y


def test_small_field_default(ctx):
    check_case(ctx, G.field_small(), O.REL, 1e-3, tune=True, chunk=256)


@pytest.mark.parametrize("tile_z", [1, 2, 4])
def test_tile_shapes_do_not_change_output(ctx, tile_z):
    x = G.grf((50, 47, 99), 3.0, 21)
    check_case(ctx, x, O.REL, 1e-3, tune=True, chunk=512, tile_z=tile_z)


CFGS = [((O.CUB, O.MD, 0),) * 4, ((O.LIN, O.MD, 0),) * 4, ((O.CUB, O.SEQ, 0),) * 4,
        ((O.CUB, O.SEQ, 5),) * 4, ((O.LIN, O.SEQ, 3),) * 4,
        ((O.CUB, O.SEQ, 1), (O.LIN, O.MD, 0), (O.CUB, O.SEQ, 4), (O.CUB, O.MD, 0)),
        ((O.LIN, O.SEQ, 2), (O.CUB, O.SEQ, 5), (O.LIN, O.MD, 0), (O.CUB, O.SEQ, 3)),
        ((O.NAT, O.MD, 0),) * 4, ((O.NAT, O.SEQ, 4),) * 4,
        ((O.NAT, O.SEQ, 0), (O.CUB, O.MD, 0), (O.NAT, O.MD, 0), (O.LIN, O.SEQ, 1))]


@pytest.mark.parametrize("ci", range(len(CFGS)))
def test_every_scheme(ctx, ci):
    x = G.grf((37, 41, 66), 3.5, 30 + ci)
    check_case(ctx, x, O.REL, 1e-3, tune=False, cfg=CFGS[ci], chunk=1024, tile_z=1 + ci % 2)


# Dimensions that are multiples of 16 leave the last block along an axis
# without its +1 face: those tiles still run their coarse levels in the
# pre-pass (on a half grid cut short by the field), with every scheme.
@pytest.mark.parametrize("tile_z", [1, 2, 4])
@pytest.mark.parametrize("shape", [(64, 48, 96), (48, 64, 33), (32, 33, 128)])
def test_tiles_without_far_faces(ctx, shape, tile_z):
    x = G.grf(shape, 3.0, 31 + shape[2] + tile_z)
    check_case(ctx, x, O.REL, 1e-3, tune=True, chunk=512, tile_z=tile_z)


@pytest.mark.parametrize("ci", [0, 3, 4, 6])
def test_tiles_without_far_faces_every_scheme(ctx, ci):
    x = G.grf((48, 32, 64), 2.5, 41 + ci)
    check_case(ctx, x, O.REL, 1e-3, tune=False, cfg=CFGS[ci], chunk=256, tile_z=2)


@pytest.mark.parametrize("seed", range(16))
def test_random_shapes(ctx, seed):
    rng = np.random.default_rng(500 + seed)
    shape = tuple(int(v) for v in rng.integers(1, 81, size=3))
    kind = ["grf", "noise", "grf", "grf"][seed % 4]
    x = G.random_small(shape, seed, kind) * np.float32(rng.uniform(0.01, 100))
    mode = int(rng.integers(0, 2))
    eb = float(10 ** rng.uniform(-5, -1.5))
    if mode == O.ABS:
        eb *= float(np.ptp(x) or 1.0)
    chunk = int(2 ** rng.integers(8, 13))
    check_case(ctx, x, mode, eb, tune=bool(seed % 3), cfg=CFGS[seed % len(CFGS)], chunk=chunk,
               tile_z=[1, 2, 4][seed % 3])


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 70), (1, 40, 1), (17, 1, 17), (16, 16, 16),
                                   (2, 3, 65), (33, 33, 33), (18, 18, 18), (65, 2, 2)])
def test_degenerate_shapes(ctx, shape):
    x = G.random_small(shape, 3, "noise")
    check_case(ctx, x, O.REL, 1e-2, tune=True, chunk=256)


@pytest.mark.parametrize("eb", [1e-2, 1e-4, 1e-6])
def test_outlier_heavy(ctx, eb):
    x = G.grf((48, 64, 80), 2.0, 9)
    zs, _ = check_case(ctx, x, O.REL, eb, tune=True, chunk=1024)
    if eb == 1e-6:
        # nearly every point is an outlier: the stream outgrows the binding's
        # first capacity guess (5N + 64 KiB), so its BUFSZ retry at the size the
        # library reported is what produced the byte-exact stream above
        assert zs.size > 5 * x.size + (1 << 16)


@pytest.mark.parametrize("chunk", [256, 2048, 4096, 65536])
def test_chunk_lengths(ctx, chunk):
    x = G.grf((45, 60, 70), 3.0, 12)
    check_case(ctx, x, O.REL, 1e-4, tune=False, cfg=CFGS[0], chunk=chunk)


def test_constant_fields(ctx):
    x = np.full((20, 30, 40), 3.5, np.float32)
    zs, _ = check_case(ctx, x, O.REL, 1e-3, chunk=256)
    assert zs.size == 132
    check_case(ctx, x, O.ABS, 1e-3, tune=False, chunk=256)
    y = np.zeros((9, 9, 9), np.float32)
    y[0, 0, 0] = -0.0
    check_case(ctx, y, O.REL, 1e-3, chunk=256)


def test_multilinear_exact(ctx):
    x = G.multilinear((33, 49, 65))
    zs, y = check_case(ctx, x, O.ABS, 0.5, tune=False, cfg=CFGS[2], chunk=1024)
    assert np.array_equal(y, x)


def test_errors(ctx):
    from paper_2507_11165_amd import hiz
    dev = torch.device("cuda:0")
    x = torch.from_numpy(G.grf((24, 24, 24), 3.0, 1)).to(dev)
    with pytest.raises(hiz.HizError) as e:
        ctx.compress(x, "rel", 0.0)
    assert e.value.status == hiz.ERR_ARG
    bad = x.clone()
    bad[3, 4, 5] = float("nan")
    with pytest.raises(hiz.HizError) as e:
        ctx.compress(bad, "rel", 1e-3)
    assert e.value.status == hiz.ERR_NONFINITE
    bad[3, 4, 5] = float("inf")
    with pytest.raises(hiz.HizError) as e:
        ctx.compress(bad, "abs", 1e-3)
    assert e.value.status == hiz.ERR_NONFINITE
    # too small an output buffer: BUFSZ with the exact size needed
    full = ctx.compress(x, "rel", 1e-4)
    small = torch.empty(1000, dtype=torch.uint8, device=dev)
    with pytest.raises(hiz.HizError) as e:
        ctx.compress_ptr(x.data_ptr(), x.shape, "rel", 1e-4, small.data_ptr(), small.numel(),
                         None, None)
    assert e.value.status == hiz.ERR_BUFSZ and e.value.needed == full.numel()
    torch.cuda.synchronize()


def test_corrupt_streams(ctx):
    from paper_2507_11165_amd import hiz
    dev = torch.device("cuda:0")
    x = G.grf((24, 30, 18), 3.0, 2)
    s = O.compress(x, O.REL, 1e-4, chunk=256).stream
    out = torch.empty(x.size, dtype=torch.float32, device=dev)

    def status(b):
        t = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
        try:
            ctx.decompress_ptr(t.data_ptr(), t.numel(), out.data_ptr(), out.numel(), None)
            return hiz.OK
        except hiz.HizError as e:
            return e.status
    assert status(s) == hiz.OK
    assert status(s[:100]) == hiz.ERR_CORRUPT
    assert status(s[:-4]) == hiz.ERR_CORRUPT
    t = s.copy(); t[0] ^= 1
    assert status(t) == hiz.ERR_CORRUPT
    t = s.copy(); t[384] ^= 1
    assert status(t) == hiz.ERR_CORRUPT
    t = s.copy(); t[68] = 3
    assert status(t) == hiz.ERR_CORRUPT
    t = s.copy(); t[128 + 128] += 1
    assert status(t) == hiz.ERR_CORRUPT
    torch.cuda.synchronize()


def test_deterministic(ctx):
    x = G.grf((64, 64, 64), 11 / 3, 5)
    a, _ = _gpu_roundtrip(ctx, x, O.REL, 1e-3, True, O.DEFAULT_CFG, 1024)
    for _ in range(3):
        b, _ = _gpu_roundtrip(ctx, x, O.REL, 1e-3, True, O.DEFAULT_CFG, 1024)
        assert np.array_equal(a, b)


def test_decompress_oracle_streams(ctx):
    # the GPU decoder reads streams the oracle wrote (with any configuration)
    from paper_2507_11165_amd import hiz
    dev = torch.device("cuda:0")
    for seed, cfg in enumerate(CFGS[:4]):
        x = G.grf((30 + seed, 35, 40), 3.0, 70 + seed)
        r = O.compress(x, O.REL, 1e-4, tune=False, cfg=cfg, chunk=512)
        y = ctx.decompress(torch.from_numpy(r.stream).to(dev)).cpu().numpy()
        assert np.array_equal(y.view(np.uint32), O.decompress(r.stream).view(np.uint32))


@pytest.mark.slow
def test_anisotropic_front_full_size(ctx):
    x = G.field_front()
    for eb in (1e-3, 1e-4):
        check_case(ctx, x, O.REL, eb, tune=True, chunk=256)


@pytest.fixture(scope="module")
def turb512():
    return G.field_turb()


@pytest.mark.slow
@pytest.mark.parametrize("eb", [1e-3, 1e-2, 1e-4])
def test_turbulence_512_full_size(ctx, turb512, eb):
    # the benchmark's workload and launch configuration (default tile and chunk),
    # compared in full at the three bounds of the 512^3 configuration; at 1e-4
    # about a quarter of the points are outliers
    zs, _ = check_case(ctx, turb512, O.REL, eb, tune=True, chunk=1024, tile_z=0)
    from paper_2507_11165_amd import hiz
    info = hiz.inspect(zs[:512].tobytes())
    _say(f"512^3 eb={eb}: n_out/N = {info['n_outliers'] / turb512.size:.4f}, "
         f"ratio {turb512.nbytes / zs.size:.3f}")


@pytest.mark.parametrize("shape", [(1, 180, 360), (1, 1, 5000), (1, 97, 33), (40, 1, 70)])
def test_two_and_one_dimensional_fields(ctx, shape):
    # flat axes (size 1): 2-D and 1-D fields, tuned on 17 x 17 (or 17) blocks
    x = G.grf(shape, 3.0, 60 + shape[1])
    check_case(ctx, x, O.REL, 1e-3, tune=True, chunk=512)


@pytest.mark.slow
def test_two_dimensional_climate_size(ctx):
    # a 1800 x 3600 2-D field (the size of the paper's CESM climate fields)
    x = G.grf((1, 1800, 3600), 3.0, 61)
    zs, _ = check_case(ctx, x, O.REL, 1e-3, tune=True, chunk=1024)
    from paper_2507_11165_amd import hiz
    info = hiz.inspect(zs[:512].tobytes())
    _say(f"1800x3600: ratio {x.nbytes / zs.size:.3f}, level config {info['level_cfg']}")


def test_two_dimensional_tensor_through_binding(ctx):
    # a 2-D tensor goes in as it is and comes back 2-D
    x = G.grf((1, 130, 250), 3.0, 62)
    from paper_2507_11165_amd import hiz
    t = torch.from_numpy(x[0].copy()).to("cuda:0")
    z = ctx.compress(t, "rel", 1e-3, hiz.make_params(tune=True, chunk=512))
    ref = O.compress(x, O.REL, 1e-3, tune=True, chunk=512, debug=False)
    assert np.array_equal(z.cpu().numpy(), ref.stream)
    y = ctx.decompress(z, squeeze=True)
    assert tuple(y.shape) == (130, 250)
    assert np.array_equal(y.cpu().numpy().view(np.uint32), O.decompress(ref.stream)[0].view(np.uint32))
