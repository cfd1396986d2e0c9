"""GPU batches: many uneven fields per call, eager and HIP-graph replay.

Every stream a batch writes must be byte-identical to the oracle's stream of
that field alone (same parameters), every decompressed field bit-identical to
the oracle's decompression, and the bound must hold on every element. The
full-size batch of 64 fields (sides 32..384) is checked against single-field
calls of the same library and against the bound on every element, and against
the oracle on a sample of its smaller fields.
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
def hz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_11165_amd import hiz
    return hiz


@pytest.fixture()
def ctx(hz):
    c = hz.Context(0)
    yield c
    c.close()


DEV = "cuda:0"


def _mixed_fields():
    """Uneven shapes, ragged tails, degenerate axes, a constant and a noisy field."""
    out = []
    shapes = [(40, 33, 50), (17, 17, 17), (1, 70, 90), (65, 1, 3), (33, 48, 31), (5, 5, 5),
              (80, 64, 16), (2, 2, 2)]
    for i, sh in enumerate(shapes):
        out.append((G.random_small(sh, 700 + i), O.REL, [1e-2, 1e-3, 1e-4][i % 3]))
    out.append((G.random_small((30, 20, 40), 777, "const"), O.REL, 1e-3))
    out.append((G.random_small((24, 36, 20), 778, "noise"), O.ABS, 0.05))
    out.append((G.random_small((48, 40, 36), 779), O.ABS, 1e-3))
    return out


def _to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _compress_batch(ctx, hz, xs, modes, ebs, params, caps=None):
    fields = [_to_dev(x) for x in xs]
    caps = caps or [hz.compress_bound(x.shape) for x in xs]
    outs = [torch.empty(c, dtype=torch.uint8, device=DEV) for c in caps]
    sh = hz._stream_handle(None)
    sizes, st = ctx.compress_batch_ptr([f.data_ptr() for f in fields], [x.shape for x in xs],
                                       modes, ebs, [o.data_ptr() for o in outs], caps, params, sh)
    torch.cuda.synchronize()
    return fields, outs, sizes, st


def _decompress_batch(ctx, hz, outs, sizes, shapes):
    ys = [torch.empty(sh, dtype=torch.float32, device=DEV) for sh in shapes]
    dims, st = ctx.decompress_batch_ptr([o.data_ptr() for o in outs], sizes,
                                        [y.data_ptr() for y in ys], [y.numel() for y in ys],
                                        hz._stream_handle(None))
    torch.cuda.synchronize()
    return ys, dims, st


def _check_against_oracle(x, mode, eb, zs, y, chunk, tune=True):
    ref = O.compress(x, mode, eb, tune=tune, cfg=O.DEFAULT_CFG, chunk=chunk, debug=False)
    assert zs.size == ref.stream.size and np.array_equal(zs, ref.stream), \
        f"stream differs for shape {x.shape}"
    yr = O.decompress(ref.stream)
    assert np.array_equal(y.view(np.uint32), yr.view(np.uint32)), f"recon differs {x.shape}"
    if not (ref.stream[7] & 1):
        err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max()
        assert err <= float(ref.eps)


@pytest.mark.parametrize("graphs", [False, True])
def test_mixed_batch_matches_oracle(ctx, hz, graphs):
    cases = _mixed_fields()
    xs = [c[0] for c in cases]
    modes = [c[1] for c in cases]
    ebs = [c[2] for c in cases]
    chunk = 512
    p = hz.make_params(tune=True, chunk=chunk)
    ctx.set_graphs(graphs)
    _say(f"mixed batch of {len(xs)} fields, graphs={graphs}")
    _, outs, sizes, st = _compress_batch(ctx, hz, xs, modes, ebs, p)
    assert st == [0] * len(xs), st
    ys, dims, st2 = _decompress_batch(ctx, hz, outs, sizes, [x.shape for x in xs])
    assert st2 == [0] * len(xs), st2
    for i, x in enumerate(xs):
        assert dims[i] == x.shape
        zs = outs[i][:sizes[i]].cpu().numpy()
        _check_against_oracle(x, modes[i], ebs[i], zs, ys[i].cpu().numpy(), chunk)


def test_batch_equals_single_calls_default_params(ctx, hz):
    specs = G.batch_specs(n=12, seed=4242, lo=20, hi=96)
    xs = [G.grf(sh, beta, seed) for sh, beta, seed in specs]
    _say(f"12-field batch, default params: {[x.shape for x in xs]}")
    _, outs, sizes, st = _compress_batch(ctx, hz, xs, ["rel"] * 12, [1e-3] * 12, None)
    assert st == [0] * 12
    for i, x in enumerate(xs):
        single = ctx.compress(_to_dev(x), "rel", 1e-3).cpu().numpy()
        assert np.array_equal(outs[i][:sizes[i]].cpu().numpy(), single), i


def test_graph_replays_match_eager(ctx, hz):
    cases = _mixed_fields()[:6]
    xs = [c[0] for c in cases]
    modes = [c[1] for c in cases]
    ebs = [c[2] for c in cases]
    p = hz.make_params(tune=True, chunk=256)
    ctx.set_graphs(False)
    _, eager_outs, eager_sizes, st = _compress_batch(ctx, hz, xs, modes, ebs, p)
    assert st == [0] * len(xs)
    eager = [o[:s].cpu().numpy() for o, s in zip(eager_outs, eager_sizes)]
    eager_y, _, _ = _decompress_batch(ctx, hz, eager_outs, eager_sizes, [x.shape for x in xs])
    eager_y = [y.cpu().numpy() for y in eager_y]
    ctx.set_graphs(True)
    b0, r0 = ctx.graph_stats()
    for rep in range(4):
        _say(f"graph replay {rep}")
        # the program's own eager work and synchronizations between replays
        junk = torch.randn(1 << 20, device=DEV).sum()
        torch.cuda.synchronize()
        _, outs, sizes, st = _compress_batch(ctx, hz, xs, modes, ebs, p)
        assert st == [0] * len(xs)
        for i in range(len(xs)):
            assert np.array_equal(outs[i][:sizes[i]].cpu().numpy(), eager[i]), (rep, i)
        ys, _, st2 = _decompress_batch(ctx, hz, outs, sizes, [x.shape for x in xs])
        assert st2 == [0] * len(xs)
        for i in range(len(xs)):
            assert np.array_equal(ys[i].cpu().numpy().view(np.uint32),
                                  eager_y[i].view(np.uint32)), (rep, i)
        del junk
    b1, r1 = ctx.graph_stats()
    assert b1 - b0 == 2, (b0, b1)   # one compress and one decompress graph
    assert r1 - r0 == 8, (r0, r1)
    ctx.set_graphs(False)


def test_per_field_failures_do_not_stop_the_batch(ctx, hz):
    xs = [G.random_small((20, 20, 20), 801), G.random_small((20, 20, 20), 802),
          G.random_small((20, 20, 20), 803)]
    bad = xs[1].copy()
    bad[3, 4, 5] = np.nan
    xs_in = [xs[0], bad, xs[2]]
    caps = [hz.compress_bound(x.shape) for x in xs_in]
    caps[2] = 600   # far below the stream size
    p = hz.make_params(chunk=256)
    _say("batch with a NaN field and a short output")
    _, outs, sizes, st = _compress_batch(ctx, hz, xs_in, ["rel"] * 3, [1e-3] * 3, p, caps)
    assert st == [hz.OK, hz.ERR_NONFINITE, hz.ERR_BUFSZ], st
    assert sizes[2] > 600
    single = ctx.compress(_to_dev(xs[0]), "rel", 1e-3, p).cpu().numpy()
    assert np.array_equal(outs[0][:sizes[0]].cpu().numpy(), single)
    # the size reported for the short output is the one a retry needs
    out2 = torch.empty(sizes[2], dtype=torch.uint8, device=DEV)
    n2 = ctx.compress_ptr(_to_dev(xs[2]).data_ptr(), xs[2].shape, "rel", 1e-3, out2.data_ptr(),
                          sizes[2], p, hz._stream_handle(None))
    assert n2 == sizes[2]


def test_decompress_batch_with_corrupt_member(ctx, hz):
    xs = [G.random_small((30, 30, 30), 811), G.random_small((30, 30, 30), 812)]
    p = hz.make_params(chunk=256)
    _, outs, sizes, st = _compress_batch(ctx, hz, xs, ["rel"] * 2, [1e-3] * 2, p)
    assert st == [0, 0]
    outs[1][0] ^= 0xFF   # magic
    ys, _, st2 = _decompress_batch(ctx, hz, outs, sizes, [x.shape for x in xs])
    assert st2 == [hz.OK, hz.ERR_CORRUPT], st2
    ref = O.decompress(O.compress(xs[0], O.REL, 1e-3, tune=True, cfg=O.DEFAULT_CFG, chunk=256,
                                  debug=False).stream)
    assert np.array_equal(ys[0].cpu().numpy().view(np.uint32), ref.view(np.uint32))


def test_submit_finish_and_pending_guard(ctx, hz):
    xs = [G.random_small((33, 17, 40), 821), G.random_small((9, 50, 20), 822)]
    fields = [_to_dev(x) for x in xs]
    caps = [hz.compress_bound(x.shape) for x in xs]
    outs = [torch.empty(c, dtype=torch.uint8, device=DEV) for c in caps]
    p = hz.make_params(chunk=256)
    sh = hz._stream_handle(None)
    ctx.compress_batch_ptr([f.data_ptr() for f in fields], [x.shape for x in xs], ["rel"] * 2,
                           [1e-3] * 2, [o.data_ptr() for o in outs], caps, p, sh,
                           submit_only=True)
    with pytest.raises(hz.HizError) as e:
        ctx.compress(fields[0], "rel", 1e-3, p)
    assert e.value.status == hz.ERR_ARG
    with pytest.raises(hz.HizError):
        ctx.set_graphs(True)
    sizes, _, st = ctx.batch_finish(2)
    assert st == [0, 0]
    assert ctx.batch_ready()
    for i, x in enumerate(xs):
        single = ctx.compress(fields[i], "rel", 1e-3, p).cpu().numpy()
        assert np.array_equal(outs[i][:sizes[i]].cpu().numpy(), single)


def test_empty_batch(ctx, hz):
    sizes, st = ctx.compress_batch_ptr([], [], [], [], [], [], None, hz._stream_handle(None))
    assert sizes == [] and st == []
    dims, st = ctx.decompress_batch_ptr([], [], [], [], hz._stream_handle(None))
    assert dims == [] and st == []


@pytest.mark.slow
def test_full_batch_64_fields(ctx, hz):
    """64 fields, sides uniform in 32..384, spectra k^-2..k^-4, rel eb 1e-3."""
    specs = G.batch_specs()
    _say("generating the 64-field batch")
    xs = [G.grf(sh, beta, seed) for sh, beta, seed in specs]
    n = len(xs)
    for graphs in (False, True):
        ctx.set_graphs(graphs)
        _say(f"64-field batch, graphs={graphs}")
        _, outs, sizes, st = _compress_batch(ctx, hz, xs, ["rel"] * n, [1e-3] * n, None)
        assert st == [0] * n
        ys, dims, st2 = _decompress_batch(ctx, hz, outs, sizes, [x.shape for x in xs])
        assert st2 == [0] * n
        for i, x in enumerate(xs):
            info = hz.inspect(outs[i][:512].cpu().numpy().tobytes())
            y = ys[i].cpu().numpy()
            err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max()
            assert err <= info["eps"], (i, err, info["eps"])
            if not graphs:
                single = ctx.compress(_to_dev(x), "rel", 1e-3).cpu().numpy()
                assert np.array_equal(outs[i][:sizes[i]].cpu().numpy(), single), i
        del outs, ys
        torch.cuda.empty_cache()
    ctx.set_graphs(False)
    # oracle on the smallest fields of the batch
    order = sorted(range(n), key=lambda i: xs[i].size)[:4]
    p = hz.make_params(chunk=256)
    sub = [xs[i] for i in order]
    _, outs, sizes, st = _compress_batch(ctx, hz, sub, ["rel"] * 4, [1e-3] * 4, p)
    ys, _, _ = _decompress_batch(ctx, hz, outs, sizes, [x.shape for x in sub])
    for k, x in enumerate(sub):
        _check_against_oracle(x, O.REL, 1e-3, outs[k][:sizes[k]].cpu().numpy(),
                              ys[k].cpu().numpy(), 256)
