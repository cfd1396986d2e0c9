"""GPU: hiz_compress_noalloc (the allocation-free compression call) against
hiz_compress, through the C ABI.

Both calls take the same field and parameters; the streams must be identical
byte for byte. Two calls in a row, the second on a smaller field, show that
what the first call leaves in the shared scratch array does not leak into the
second. A field whose workspace exceeds the scratch array is refused before
any device work.
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


def _both(hz, ctx, x, eb, params):
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    cap = hz.compress_bound(x.shape)
    za = torch.zeros(cap, dtype=torch.uint8, device=dev)
    zb = torch.full((cap,), 0xA5, dtype=torch.uint8, device=dev)
    sh = hz.C.c_void_p(torch.cuda.current_stream().cuda_stream)
    na = ctx.compress_ptr(xd.data_ptr(), x.shape, "rel", eb, za.data_ptr(), cap, params, sh)
    nb = ctx.compress_noalloc_ptr(xd.data_ptr(), x.shape, "rel", eb, zb.data_ptr(), cap, params,
                                  sh)
    torch.cuda.synchronize()
    return za[:na].cpu().numpy(), zb[:nb].cpu().numpy()


@pytest.mark.parametrize("pipeline", [0, 1, 2])
def test_noalloc_equals_compress_two_calls(hz, pipeline):
    ctx = hz.Context(0)
    params = hz.make_params(tune=True, chunk=512, pipeline=pipeline)
    shapes = [(96, 80, 130), (40, 33, 50)]  # the second call is smaller
    for k, shape in enumerate(shapes):
        _say(f"noalloc pipeline={pipeline} call {k} shape={shape}")
        x = G.grf(shape, 3.0, 700 + 10 * pipeline + k)
        a, b = _both(hz, ctx, x, 1e-3, params)
        assert a.size == b.size and np.array_equal(a, b), f"call {k}: streams differ"
        if k == 1:
            ref = O.compress(x, O.REL, 1e-3, tune=True, chunk=512, debug=False,
                             pipeline=pipeline, reorder=(pipeline == 2))
            assert np.array_equal(b, ref.stream), "allocation-free stream differs from the oracle"
        y = ctx.decompress(torch.from_numpy(b).to("cuda:0")).cpu().numpy()
        info = hz.inspect(b[:512].tobytes())
        err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max()
        assert err <= info["eps"]
    ctx.close()


def test_noalloc_refuses_fields_beyond_its_scratch(hz):
    ctx = hz.Context(0)
    dev = torch.device("cuda:0")
    small = torch.zeros(16, dtype=torch.float32, device=dev)
    out = torch.zeros(1024, dtype=torch.uint8, device=dev)
    # 1024 x 1024 x 512 points need about 1 GB of workspace: refused on the
    # host before any launch (the buffers are never touched)
    with pytest.raises(hz.HizError) as e:
        ctx.compress_noalloc_ptr(small.data_ptr(), (1024, 1024, 512), "rel", 1e-3,
                                 out.data_ptr(), out.numel())
    assert e.value.status == hz.ERR_ARG
    assert "allocation-free" in str(e.value)
    # the context still works afterwards
    x = G.grf((20, 21, 22), 3.0, 5)
    a, b = _both(hz, ctx, x, 1e-2, hz.make_params(tune=True, chunk=256))
    assert np.array_equal(a, b)
    ctx.close()
