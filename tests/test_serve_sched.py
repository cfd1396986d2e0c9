"""Serving scheduler core (continuous batching) on a CPU mock device.

The scheduler template of the library's serving loop is compiled with g++
against a mock device with a simulated clock (tests/serve_mock.cpp) and replays
seeded Poisson traces. Checked: every request completes exactly once; a batch
holds one kind of request, at most max_batch of them, within the slot's
workspace; requests of one kind start in arrival order; batches on different
slots overlap; a request too large for any slot is rejected alone without
blocking the queue; latency percentiles come out of the completions.
"""
import json
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_mock.cpp")
INC = os.path.join(ROOT, "paper_2507_11165_amd", "csrc")


@pytest.fixture(scope="module")
def mock(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("serve") / "serve_mock")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-pthread", "-Wall", "-I", INC, SRC,
                           "-o", exe])

    def run(seed=1, rate=200.0, n=400, slots=4, max_batch=8, capacity=600_000_000,
            p_dec=0.3, oversize=0):
        out = subprocess.check_output([exe, str(seed), str(rate), str(n), str(slots),
                                       str(max_batch), str(capacity), str(p_dec),
                                       str(oversize)], timeout=120)
        return json.loads(out)
    return run


def _check_invariants(r, max_batch, capacity):
    n = r["n"]
    comp = r["completions"]
    ids = [c[0] for c in comp]
    assert sorted(ids) == list(range(n)), "every request completes exactly once"
    ops = r["ops"]
    for b in r["batches"]:
        assert 1 <= len(b["ids"]) <= max_batch
        assert all(ops[i] == b["op"] for i in b["ids"]), "one kind per batch"
        assert b["need"] <= capacity
    # same-kind requests start in arrival order
    start = {c[0]: c[4] for c in comp}
    for op in (0, 1):
        seq = [start[i] for i in range(n) if ops[i] == op and comp[ids.index(i)][1] == 0]
        assert all(a <= b for a, b in zip(seq, seq[1:])), f"op {op} served out of order"
    for c in comp:
        assert c[3] <= c[4] <= c[5], "submit <= start <= done"


def test_invariants_under_load(mock):
    r = mock(seed=3, rate=5000.0, n=600, slots=4, max_batch=8)
    _check_invariants(r, 8, 600_000_000)
    assert r["max_running"] >= 2, "batches on different slots overlap"
    sizes = [len(b["ids"]) for b in r["batches"]]
    assert max(sizes) > 1, "requests that wait together are batched"


def test_light_load_serves_singly(mock):
    r = mock(seed=5, rate=5.0, n=60, slots=2, max_batch=16)
    _check_invariants(r, 16, 600_000_000)
    lat = [c[5] - c[3] for c in r["completions"]]
    # arrivals 200 ms apart on average: almost no queueing
    assert np.median(lat) < 0.01


def test_capacity_limits_batches(mock):
    cap = 200_000_000
    r = mock(seed=7, rate=8000.0, n=500, slots=3, max_batch=64, capacity=cap)
    _check_invariants(r, 64, cap)
    assert max(b["need"] for b in r["batches"]) <= cap


def test_oversize_request_rejected_alone(mock):
    r = mock(seed=11, rate=300.0, n=300, slots=2, max_batch=8, oversize=25)
    comp = {c[0]: c for c in r["completions"]}
    assert sorted(comp) == list(range(300))
    for i in range(24, 300, 25):
        assert comp[i][1] == 5, "oversize request completes with ERR_NOMEM"
        assert comp[i][6] == 1, "and alone"
    others = [c for i, c in comp.items() if (i + 1) % 25]
    assert all(c[1] == 0 for c in others), "the queue behind it is served"


def test_latency_percentiles(mock):
    r = mock(seed=13, rate=200.0, n=800, slots=4, max_batch=16)
    lat = np.array([c[5] - c[3] for c in r["completions"]])
    p50, p99 = np.percentile(lat, [50, 99])
    assert 0 < p50 <= p99
    # the model serves 200 req/s of these sizes with room to spare
    assert p99 < 0.5


def test_deterministic(mock):
    a = mock(seed=17, n=200)
    b = mock(seed=17, n=200)
    assert a == b
