"""GPU serving loop: continuous batching gives each request the result it gets alone.

Requests of mixed sizes, bounds and kinds go through hiz_server (several slots,
batches overlapping on the device); every compressed stream must be
byte-identical to a single hiz_compress call on the same field, every
decompressed field bit-identical to a single hiz_decompress call, and a few
small ones are also checked against the CPU oracle.
"""
import sys
import time

import numpy as np
import pytest

import fieldgen as G
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_11165_amd import hiz
    return hiz


def _wait_all(srv, n, timeout=60.0):
    got = {}
    t_end = time.time() + timeout
    while len(got) < n:
        for c in srv.poll():
            got[c["id"]] = c
        if time.time() > t_end:
            raise AssertionError(f"only {len(got)} of {n} requests completed")
        time.sleep(0.001)
    return got


def test_served_results_equal_single_calls(hz):
    rng = np.random.default_rng(900)
    shapes = [tuple(int(v) for v in rng.integers(9, 72, size=3)) for _ in range(40)]
    ebs = [float(rng.choice([1e-2, 1e-3, 1e-4])) for _ in shapes]
    xs = [G.grf(sh, float(rng.uniform(2.0, 4.0)), 9000 + i) for i, sh in enumerate(shapes)]
    fields = [torch.from_numpy(x).to(DEV) for x in xs]
    caps = [hz.compress_bound(x.shape) for x in xs]
    outs = [torch.empty(c, dtype=torch.uint8, device=DEV) for c in caps]
    torch.cuda.synchronize()
    # an explicit chunk length, so that the oracle below takes the same one
    params = hz.make_params(tune=True, chunk=256)
    srv = hz.Server(0, slots=3, mem_budget=1 << 30, max_batch=8, params=params)
    _say(f"serving {len(xs)} compress requests")
    # bursts: some requests arrive while others run
    for i, x in enumerate(xs):
        srv.submit_compress(i, fields[i].data_ptr(), x.shape, "rel", ebs[i], outs[i].data_ptr(),
                            caps[i])
        if i % 10 == 9:
            time.sleep(0.002)
    got = _wait_all(srv, len(xs))
    st = srv.stats()
    _say(f"stats {st}")
    assert st["completed"] == len(xs)
    assert st["batches"] < len(xs), "waiting requests are batched"
    ctx = hz.Context(0)
    sizes = []
    for i, x in enumerate(xs):
        c = got[i]
        assert c["status"] == 0, (i, c)
        single = ctx.compress(fields[i], "rel", ebs[i], params).cpu().numpy()
        served = outs[i][:c["size"]].cpu().numpy()
        assert np.array_equal(served, single), f"request {i} {x.shape} differs from a single call"
        assert c["t_submit"] <= c["t_start"] <= c["t_done"]
        sizes.append(c["size"])
    # decompression through the server, mixed sizes again
    ys = [torch.empty(x.shape, dtype=torch.float32, device=DEV) for x in xs]
    torch.cuda.synchronize()
    _say("serving decompress requests")
    for i, x in enumerate(xs):
        srv.submit_decompress(1000 + i, outs[i].data_ptr(), sizes[i], ys[i].data_ptr(), x.size)
    got = _wait_all(srv, len(xs))
    for i, x in enumerate(xs):
        assert got[1000 + i]["status"] == 0
        alone = ctx.decompress(outs[i][:sizes[i]]).cpu().numpy()
        assert np.array_equal(ys[i].cpu().numpy().view(np.uint32), alone.view(np.uint32)), i
    # the smallest few against the oracle, at the same chunk length
    for i in sorted(range(len(xs)), key=lambda k: xs[k].size)[:3]:
        ref = O.compress(xs[i], O.REL, ebs[i], tune=True, cfg=O.DEFAULT_CFG, chunk=256,
                         debug=False)
        assert np.array_equal(outs[i][:sizes[i]].cpu().numpy(), ref.stream)
    srv.close()
    ctx.close()


def test_oversize_request_is_rejected_and_queue_continues(hz):
    x_big = G.grf((64, 64, 64), 3.0, 920)
    x_small = G.grf((20, 24, 28), 3.0, 921)
    fb = torch.from_numpy(x_big).to(DEV)
    fs = torch.from_numpy(x_small).to(DEV)
    ob = torch.empty(hz.compress_bound(x_big.shape), dtype=torch.uint8, device=DEV)
    os_ = torch.empty(hz.compress_bound(x_small.shape), dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    # a slot workspace too small for 64^3 but enough for the small field
    budget = hz.workspace_bound(x_small.shape) * 3
    srv = hz.Server(0, slots=1, mem_budget=budget, max_batch=4)
    srv.submit_compress(1, fb.data_ptr(), x_big.shape, "rel", 1e-3, ob.data_ptr(), ob.numel())
    srv.submit_compress(2, fs.data_ptr(), x_small.shape, "rel", 1e-3, os_.data_ptr(), os_.numel())
    got = _wait_all(srv, 2)
    assert got[1]["status"] == hz.ERR_NOMEM
    assert got[2]["status"] == 0
    srv.close()


def test_latency_percentiles_reported(hz):
    xs = [G.grf((32, 32, 32), 3.0, 930 + i) for i in range(24)]
    fields = [torch.from_numpy(x).to(DEV) for x in xs]
    outs = [torch.empty(hz.compress_bound(x.shape), dtype=torch.uint8, device=DEV) for x in xs]
    torch.cuda.synchronize()
    srv = hz.Server(0, slots=2, mem_budget=1 << 28, max_batch=4)
    for i, x in enumerate(xs):
        srv.submit_compress(i, fields[i].data_ptr(), x.shape, "rel", 1e-3, outs[i].data_ptr(),
                            outs[i].numel())
    got = _wait_all(srv, len(xs))
    lat = np.array([c["t_done"] - c["t_submit"] for c in got.values()])
    p50, p99 = np.percentile(lat, [50, 99])
    _say(f"p50 {p50 * 1e3:.3f} ms p99 {p99 * 1e3:.3f} ms")
    assert 0 < p50 <= p99 < 10.0
    assert all(c["batch_size"] <= 4 for c in got.values())
    srv.close()
