"""Benchmark: compress + decompress throughput of one FP32 3-D field on one GPU.

Headline workload: a 512^3 Gaussian random field with the Kolmogorov spectrum
k^-11/3 plus 1 % white noise (fieldgen.field_turb), value-range relative bound
1e-3, tuner on; input and output resident in HBM. A step is one compression
followed by one decompression of the field. `value` = (4N bytes in + 4N bytes
out) / (compress time + decompress time), i.e. 8N / (t_c + t_d).

The roofline entry covers the kernel with the largest share of the timed
region: its algorithmic bytes per launch (algorithmic_bytes below) divided by
its mean launch time, measured with HIP events on the launch stream inside the
timed region. `algorithmic_frac` is the whole step's algorithmic bytes over
the step time, as a fraction of the 8 TB/s peak; `traffic_ratio` is the HBM
bytes the kernels actually move (rocprofv3 FETCH_SIZE / WRITE_SIZE, from the
committed summary while the kernels' sources are unchanged) over those
algorithmic bytes. The CPU baseline is the oracle (single-threaded C, pinned
to one host core, median of 3) on a bounded slab of the same field.

After the headline line's measurements, the default run also measures, as
extra keys of the same JSON line:
  eb_sweep  the same field at rel eb 1e-2 and 1e-4;
  pipelines the same field at rel eb 1e-3 through the throughput mode
            (TCMS1-BIT1-RRE1) and the ratio mode (Huffman + RRE4-TCMS8-RZE1);
  forced_interp  the same field with the cubic (and the natural cubic) spline
            forced on every level, with the interpolation kernels' times;
  front     the anisotropic 100x500x500 field with a tanh front at rel eb 1e-3
            and 1e-4, with the tuner's per-level picks;
  batch64   64 uneven fields (sides 32..384, spectra k^-2..k^-4, rel eb 1e-3):
            64 plain per-field calls vs one batched call per direction, eager
            and replayed from a HIP graph;
  serve     the serving trace (Poisson arrivals at 200 requests/s, fields
            64^3..512^3, rel eb from 1e-2, 1e-3, 1e-4) through the
            continuous-batching server vs plain per-request calls: p50/p99
            latency paced by the trace, and throughput of all requests at once.
--headline-only skips them (profiling runs); --workload batch64|serve runs one
of them alone as the headline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--eb 1e-3]
                       [--workload turb512|batch64|serve] [--duration S]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(name, N, info, n_anchors):
    """Bytes the method itself must move per launch of a kernel: the field
    read once (and once more for the exact range in REL mode), the anchors,
    the outliers (index + value), the Huffman payload and its chunk table,
    and the reconstructed field written once. Intermediates of this
    implementation (the code array, the coarse pre-pass slots, tables) count
    zero. None for kernels that move no algorithmic bytes."""
    n_out = info["n_outliers"]
    pw = info["payload_words"]
    nch = info["n_chunks"]
    ob = ((4 if N < 2 ** 32 else 8) + 4) * n_out
    table = {
        "minmax": 4 * N,
        "predict_quant": 4 * N + 4 * n_anchors + ob,
        "encode": 4 * pw + 4 * nch,
        "decode": 4 * pw + 4 * nch,
        "scatter": ob,
        "reconstruct": 4 * N + 4 * n_anchors,
    }
    return table.get(name)


def step_algorithmic_bytes(N, info, n_anchors, rel=True):
    """Compress + decompress bytes of one step (the sum of the table above,
    plus the 384-byte header and code-length table written and read once)."""
    names = ["minmax"] if rel else []
    names += ["predict_quant", "encode", "decode", "scatter", "reconstruct"]
    return sum(algorithmic_bytes(k, N, info, n_anchors) for k in names) + 2 * 384


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "turb512_rel1e-3_hbm_traffic.md")


def measured_traffic(kernel):
    """HBM bytes per launch (read + write) of a kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the summary is missing or the
    kernel's sources changed since the counters were taken."""
    import hashlib
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    for line in lines:
        f = line.split()
        if len(f) < 6 or f[0] != "traffic" or f[1] != kernel:
            continue
        kv = dict(x.split("=", 1) for x in f[2:])
        for ref in (kv["src"], kv["hdr"]):
            fname, want = ref.split(":")
            path = os.path.join(ROOT, "paper_2507_11165_amd", "csrc", fname)
            try:
                have = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
            except OSError:
                return None
            if have != want:
                return None
        return int(kv["read"]) + int(kv["write"])
    return None


def host_cpu():
    """Model name and logical core count of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 0


def cpu_baseline(x, eb, planes, runs=3):
    """Oracle compress + decompress of the first `planes` x-planes, pinned to
    one host core, median of `runs` runs."""
    import oracle as O
    sample = np.ascontiguousarray(x[:planes])
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    os.sched_setaffinity(0, {core})  # this thread only: the oracle runs on it
    try:
        tc, td = [], []
        for _ in range(runs):
            t0 = time.perf_counter()
            r = O.compress(sample, O.REL, eb, tune=True, chunk=1024, debug=False)
            t1 = time.perf_counter()
            O.decompress(r.stream)
            t2 = time.perf_counter()
            tc.append(t1 - t0)
            td.append(t2 - t1)
    finally:
        os.sched_setaffinity(0, set(allowed))
    tot = sorted(a + b for a, b in zip(tc, td))[len(tc) // 2]
    gbs = 8.0 * sample.size / tot / 1e9
    model, ncores = host_cpu()
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first {planes} x-planes of the same field ({sample.shape}, "
                      f"{sample.nbytes / 1e6:.0f} MB), compress + decompress, single-threaded C "
                      f"pinned to core {core}, median of {runs}: compress "
                      f"{sorted(tc)[len(tc) // 2]:.2f} s, decompress {sorted(td)[len(td) // 2]:.2f} s",
            "host_cpu": model, "host_cores": ncores, "pinned_core": core,
            "runs_s": [round(a + b, 3) for a, b in zip(tc, td)]}


METRIC = "compress+decompress GB/s & % HBM peak at eb=1e-3; ratio; batched vs plain"


def base_line(value, steps, warmup, ms, config):
    return {"metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
            "steps": steps, "warmup": warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": config}


def measure_field(ctx, hiz, torch, xd, x, eb, params, steps, warmup, zbuf, ybuf, sh,
                  profile=True):
    """Time `steps` compress + decompress steps of one resident field, then the
    two directions apart; check the bound on every element."""
    N = x.size
    shape = x.shape
    cap = zbuf.numel()

    def step():
        size = ctx.compress_ptr(xd.data_ptr(), shape, "rel", eb, zbuf.data_ptr(), cap, params, sh)
        ctx.decompress_ptr(zbuf.data_ptr(), size, ybuf.data_ptr(), N, sh)
        return size

    for _ in range(warmup):
        size = step()
    torch.cuda.synchronize()
    if profile:
        ctx.reset_profile()
        ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        size = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = None
    if profile:
        ctx.set_profiling(False)
        prof = ctx.profile()
    elapsed = t1 - t0
    # compress and decompress timed apart (for the record, not the headline)
    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    for _ in range(steps):
        ctx.compress_ptr(xd.data_ptr(), shape, "rel", eb, zbuf.data_ptr(), cap, params, sh)
    torch.cuda.synchronize()
    tc1 = time.perf_counter()
    for _ in range(steps):
        ctx.decompress_ptr(zbuf.data_ptr(), size, ybuf.data_ptr(), N, sh)
    torch.cuda.synchronize()
    tc2 = time.perf_counter()
    info = hiz.inspect(zbuf[:512].cpu().numpy().tobytes())
    yv = ybuf.view(-1)[:N].view(shape)
    err = (xd.double() - yv.double()).abs()
    maxerr = float(err.max())
    mse = float((err * err).mean())
    del err
    rng = float(x.max()) - float(x.min())
    psnr = 20 * np.log10(rng) - 10 * np.log10(mse) if mse > 0 else float("inf")
    if maxerr > info["eps"]:
        raise SystemExit(f"error bound violated: {maxerr} > {info['eps']}")
    return {"size": size, "info": info, "elapsed": elapsed, "prof": prof,
            "t_c": (tc1 - tc0) / steps, "t_d": (tc2 - tc1) / steps, "maxerr": maxerr,
            "psnr": float(psnr)}


def field_summary(x, m):
    N = x.size
    info = m["info"]
    return {
        "compress_GBps": round(4.0 * N / m["t_c"] / 1e9, 2),
        "decompress_GBps": round(4.0 * N / m["t_d"] / 1e9, 2),
        "combined_GBps": round(8.0 * N / (m["t_c"] + m["t_d"]) / 1e9, 2),
        "ratio": round(4.0 * N / m["size"], 4),
        "bits_per_value": round(32.0 * m["size"] / (4.0 * N), 4),
        "psnr_db": round(m["psnr"], 3),
        "max_err_over_eps": round(m["maxerr"] / info["eps"], 6),
        "outlier_frac": round(info["n_outliers"] / N, 6),
        "level_cfg": info["level_cfg"],
        "chunk": info["chunk"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eb", type=float, default=1e-3)
    ap.add_argument("--tile-z", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--cpu-planes", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the extra workloads (eb sweep, front field, batch, serving)")
    ap.add_argument("--workload", choices=["turb512", "batch64", "serve"], default="turb512")
    ap.add_argument("--duration", type=float, default=2.0,
                    help="serve: seconds of the Poisson trace replayed")
    ap.add_argument("--graphs", type=int, default=0,
                    help="1: replay each call's launch sequence from a HIP graph")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run 3 plain device copies of this many MiB: the reference "
                         "kernel of known traffic that scales FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the compressor's data-parallel path runs on a "
              "single device here (multi-GPU sharding is described in DESIGN.md, not run)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import fieldgen
    from paper_2507_11165_amd import hiz

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.workload == "batch64":
        res = bench_batch(args, torch, fieldgen, hiz, args.steps, args.warmup)
        line = base_line(res["batched_graph_GBps"], args.steps, args.warmup,
                         res["ms_batched_graph"], res.pop("config"))
        line.update(res)
        print(json.dumps(line), flush=True)
        return
    if args.workload == "serve":
        res = bench_serve(args, torch, fieldgen, hiz)
        line = base_line(res["served_saturated_GBps"], 1, 1, None, res.pop("config"))
        line.update(res)
        print(json.dumps(line), flush=True)
        return

    dev = torch.device("cuda:0")
    log("generating 512^3 field (k^-11/3 + 1% noise)")
    t = time.time()
    x = fieldgen.field_turb()
    log(f"  generated in {time.time() - t:.1f}s")
    N = x.size
    shape = x.shape
    xd = torch.from_numpy(x).to(dev)
    ctx = hiz.Context(0)
    ctx.set_graphs(bool(args.graphs))
    params = hiz.make_params(tune=True, chunk=args.chunk, tile_z=args.tile_z)
    cap = 5 * N + (1 << 20)
    zbuf = torch.empty(cap, dtype=torch.uint8, device=dev)
    ybuf = torch.empty(shape, dtype=torch.float32, device=dev)
    sh = hiz.C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if args.copy_mib:
        src = torch.empty(args.copy_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log(f"headline: warmup {args.warmup}, {args.steps} timed steps")
    m = measure_field(ctx, hiz, torch, xd, x, args.eb, params, args.steps, args.warmup, zbuf,
                      ybuf, sh)
    elapsed, prof, info, size = m["elapsed"], m["prof"], m["info"], m["size"]
    log(f"timed {args.steps} steps in {elapsed:.3f}s")

    n_anchors = int(np.prod([-(-d // 16) for d in shape]))
    current = args.tile_z in (0, 2) and args.chunk in (0, 1024) and args.eb == 1e-3
    kernels = {}
    dom, dom_ms = None, -1.0
    for name, (launches, ms) in prof.items():
        mean_s = ms / max(launches, 1) / 1e3
        algo = algorithmic_bytes(name, N, info, n_anchors)
        kernels[name] = {"launches": launches, "mean_ms": round(mean_s * 1e3, 5)}
        if algo:
            kernels[name]["algorithmic_bytes"] = algo
            kernels[name]["achieved_GBps"] = round(algo / mean_s / 1e9, 1)
        tr = measured_traffic(name) if current else None
        if tr:
            kernels[name]["traffic"] = tr
        if ms > dom_ms:
            dom, dom_ms = name, ms
    launches, ms = prof[dom]
    mean_s = ms / launches / 1e3
    algo = algorithmic_bytes(dom, N, info, n_anchors)
    achieved = algo / mean_s / 1e9 if algo else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1) if achieved else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": measured_traffic(dom) if current else None,
                "algorithmic_bytes_per_launch": algo,
                "mean_launch_ms": round(mean_s * 1e3, 5)}
    step_bytes = step_algorithmic_bytes(N, info, n_anchors)
    step_s = elapsed / args.steps
    # measured HBM bytes of one step: every kernel's counted traffic (all of
    # them must have current counters; the coarse pre-pass kernels are listed
    # under their own names)
    traffic_names = ["minmax", "coarse", "predict_quant", "encode", "decode",
                     "coarse_rec", "reconstruct"]
    tr = [measured_traffic(k) if current else None for k in traffic_names]
    step_traffic = sum(tr) if all(tr) else None
    value = 8.0 * N * args.steps / elapsed / 1e9
    res = base_line(value, args.steps, args.warmup, round(step_s * 1e3, 4), {
        "workload": "single 512x512x512 FP32 field, GRF k^-11/3 + 1% white noise, rel eb 1e-3",
        "dims": list(shape), "eb_mode": "rel", "eb": args.eb,
        "chunk": info["chunk"], "tile_z": args.tile_z or "launch table (2 at 512^3)",
        "level_cfg": info["level_cfg"],
    })
    res.update(field_summary(x, m))
    res.pop("level_cfg")
    res.pop("chunk")
    res.update({
        "effective_hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_step": step_bytes,
        "algorithmic_GBps": round(step_bytes / step_s / 1e9, 1),
        "algorithmic_frac": round(step_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4),
        "traffic_bytes_per_step": step_traffic,
        "traffic_ratio": round(step_traffic / step_bytes, 3) if step_traffic else None,
        "kernels": kernels,
        "roofline": roofline,
    })
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_planes} planes, pinned, median of 3")
        res["cpu_baseline"] = cpu_baseline(x, args.eb, args.cpu_planes)

    if not args.headline_only:
        sweep = {}
        for eb in (1e-2, 1e-4):
            log(f"eb sweep: rel {eb}")
            me = measure_field(ctx, hiz, torch, xd, x, eb, params, 5, 2, zbuf, ybuf, sh,
                               profile=False)
            sweep[f"{eb:g}"] = field_summary(x, me)
        res["eb_sweep"] = sweep
        # the lossless pipelines beyond Huffman (Sec. 5.2.3) on the same field at rel 1e-3:
        # throughput mode (TCMS1-BIT1-RRE1 on the codes) and ratio mode (Huffman, then
        # RRE4-TCMS8-RZE1, codes reordered by level)
        pipes = {}
        for name, pipe in (("throughput_TCMS1-BIT1-RRE1", hiz.PIPE_TP),
                           ("ratio_HF-RRE4-TCMS8-RZE1", hiz.PIPE_CR)):
            log(f"pipeline: {name}")
            pp = hiz.make_params(tune=True, chunk=args.chunk, tile_z=args.tile_z, pipeline=pipe)
            me = measure_field(ctx, hiz, torch, xd, x, args.eb, pp, 5, 2, zbuf, ybuf, sh,
                               profile=False)
            pipes[name] = field_summary(x, me)
        res["pipelines"] = pipes
        # the interpolation kernels with the cubic splines forced on every level (the tuner
        # picks the linear spline on this field), multi-dimensional scheme (Sec. 5.1.1-5.1.2)
        forced = {}
        for name, spline in (("cubic_md", hiz.CUBIC), ("natural_cubic_md", hiz.NATURAL)):
            log(f"forced interpolation: {name}")
            pp = hiz.make_params(tune=False, level_cfg=((spline, hiz.MD, 0),) * 4,
                                 chunk=args.chunk, tile_z=args.tile_z)
            me = measure_field(ctx, hiz, torch, xd, x, args.eb, pp, 5, 2, zbuf, ybuf, sh,
                               profile=True)
            fs = field_summary(x, me)
            # mean launch time of each interpolation kernel (total / launches)
            fs["kernels_ms"] = {k: round(v[1] / max(v[0], 1), 5) for k, v in me["prof"].items()
                                if k in ("coarse", "predict_quant", "coarse_rec", "reconstruct")}
            forced[name] = fs
        res["forced_interp"] = forced
        del xd, zbuf, ybuf, x
        torch.cuda.empty_cache()
        log("front field 100x500x500")
        xf = fieldgen.field_front()
        xfd = torch.from_numpy(xf).to(dev)
        zf = torch.empty(5 * xf.size + (1 << 20), dtype=torch.uint8, device=dev)
        yf = torch.empty(xf.shape, dtype=torch.float32, device=dev)
        front = {"workload": "100x500x500 FP32, GRF k^-3 + tanh front of width 2 across a "
                             "random plane, tuner on"}
        for eb in (1e-3, 1e-4):
            me = measure_field(ctx, hiz, torch, xfd, xf, eb, params, 5, 2, zf, yf, sh,
                               profile=False)
            front[f"{eb:g}"] = field_summary(xf, me)
        res["front"] = front
        del xfd, zf, yf, xf
        torch.cuda.empty_cache()
        b = bench_batch(args, torch, fieldgen, hiz, 3, 1)
        b.pop("config")
        res["batch64"] = b
        torch.cuda.empty_cache()
        sv = bench_serve(args, torch, fieldgen, hiz)
        sv.pop("config")
        res["serve"] = sv
    print(json.dumps(res), flush=True)


def bench_batch(args, torch, fieldgen, hiz, steps, warmup):
    """64 uneven fields: plain per-field calls vs one batched call (eager / graph)."""
    dev = torch.device("cuda:0")
    specs = fieldgen.batch_specs()
    log(f"batch: generating {len(specs)} fields")
    t = time.time()
    fields = [torch.from_numpy(fieldgen.grf(sh, beta, seed)).to(dev) for sh, beta, seed in specs]
    log(f"  generated in {time.time() - t:.1f}s")
    n = len(fields)
    Ns = [f.numel() for f in fields]
    total = sum(Ns)
    caps = [2 * N + (1 << 20) for N in Ns]
    outs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    ys = [torch.empty_like(f) for f in fields]
    ctx = hiz.Context(0)
    sh = hiz.C.c_void_p(torch.cuda.current_stream().cuda_stream)
    fptr = [f.data_ptr() for f in fields]
    optr = [o.data_ptr() for o in outs]
    yptr = [y.data_ptr() for y in ys]
    shapes = [tuple(f.shape) for f in fields]
    modes = ["rel"] * n
    ebs = [args.eb] * n
    sizes = [0] * n

    def plain_step():
        for i in range(n):
            sizes[i] = ctx.compress_ptr(fptr[i], shapes[i], "rel", args.eb, optr[i], caps[i],
                                        None, sh)
        for i in range(n):
            ctx.decompress_ptr(optr[i], sizes[i], yptr[i], Ns[i], sh)

    def batch_step():
        sz, st = ctx.compress_batch_ptr(fptr, shapes, modes, ebs, optr, caps, None, sh)
        if any(st):
            raise SystemExit(f"batched compression failed: {st}")
        sizes[:] = sz
        _, st = ctx.decompress_batch_ptr(optr, sizes, yptr, Ns, sh)
        if any(st):
            raise SystemExit(f"batched decompression failed: {st}")

    def timed(step, graphs):
        ctx.set_graphs(graphs)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    log("batch: plain per-field calls")
    t_plain = timed(plain_step, False)
    plain_sizes = list(sizes)
    log("batch: batched, eager")
    t_eager = timed(batch_step, False)
    if sizes != plain_sizes:
        raise SystemExit("batched stream sizes differ from per-field calls")
    log("batch: batched, graph replay")
    t_graph = timed(batch_step, True)
    builds, replays = ctx.graph_stats()
    ctx.set_graphs(False)
    worst = 0.0
    for i in range(n):
        info = hiz.inspect(outs[i][:512].cpu().numpy().tobytes())
        err = float((fields[i].double() - ys[i].double()).abs().max())
        worst = max(worst, err / info["eps"])
    if worst > 1.0:
        raise SystemExit(f"error bound violated: max |err|/eps = {worst}")
    ctx.close()
    gbs = lambda sec: round(8.0 * total / sec / 1e9, 2)
    return {
        "config": {
            "workload": "batch of 64 FP32 fields, sides uniform 32..384, GRF k^-2..k^-4, "
                        "rel eb 1e-3; batched + HIP graph vs 64 plain per-field calls",
            "fields": n, "points": total, "eb_mode": "rel", "eb": args.eb,
        },
        "fields": n, "points": total, "steps": steps,
        "plain_GBps": gbs(t_plain),
        "batched_eager_GBps": gbs(t_eager),
        "batched_graph_GBps": gbs(t_graph),
        "speedup_vs_plain": round(t_plain / t_graph, 3),
        "ms_plain": round(t_plain * 1e3, 3),
        "ms_batched_eager": round(t_eager * 1e3, 3),
        "ms_batched_graph": round(t_graph * 1e3, 3),
        "graph_builds": builds, "graph_replays": replays,
        "ratio": round(4.0 * total / sum(sizes), 4),
        "max_err_over_eps": round(worst, 6),
    }


def bench_serve(args, torch, fieldgen, hiz):
    """Continuous-batching server vs plain per-request calls on the serving trace."""
    dev = torch.device("cuda:0")
    times, sides, ebs, pool = fieldgen.serving_trace(duration=args.duration)
    n = len(times)
    log(f"serve: {n} requests over {args.duration}s, sides {pool}")
    fields, nbytes = {}, {}
    for k, side in enumerate(pool):
        fields[side] = torch.from_numpy(fieldgen.grf((side,) * 3, 3.0, 1050 + k)).to(dev)
        nbytes[side] = 4 * side ** 3
    # output buffers: a free list per side, returned when a completion is polled
    free = {side: [] for side in pool}
    every = []

    def take(side):
        if not free[side]:
            buf = torch.empty(5 * side ** 3 + (1 << 20), dtype=torch.uint8, device=dev)
            every.append(buf)
            return buf
        return free[side].pop()

    torch.cuda.synchronize()
    srv = hiz.Server(0, slots=4, mem_budget=24 << 30, max_batch=16)
    ctx = hiz.Context(0)
    sh = hiz.C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def run_served(paced):
        inflight = {}
        lat, done_bytes = [], 0
        clock = hiz.Server.clock
        t0 = clock()
        first = None
        i = 0
        while i < n or inflight:
            now = clock() - t0
            # at most 64 requests in flight: bounds the output buffers held
            while i < n and (not paced or times[i] <= now) and len(inflight) < 64:
                side = int(sides[i])
                buf = take(side)
                inflight[i] = (side, buf)
                srv.submit_compress(i, fields[side].data_ptr(), (side,) * 3, "rel", float(ebs[i]),
                                    buf.data_ptr(), buf.numel())
                i += 1
            for c in srv.poll():
                side, buf = inflight.pop(c["id"])
                if c["status"] != 0:
                    raise SystemExit(f"served request {c['id']} failed: {c['status']}")
                lat.append(c["t_done"] - c["t_submit"])
                first = c["t_submit"] if first is None else min(first, c["t_submit"])
                done_bytes += nbytes[side]
                last = c["t_done"]
                free[side].append(buf)
            time.sleep(0.0002)
        return np.array(lat), done_bytes / (last - first) / 1e9

    def run_plain(paced):
        lat, done_bytes = [], 0
        t0 = time.perf_counter()
        for i in range(n):
            if paced:
                while time.perf_counter() - t0 < times[i]:
                    time.sleep(0.0001)
            ts = time.perf_counter() if paced else t0
            side = int(sides[i])
            buf = take(side)
            ctx.compress_ptr(fields[side].data_ptr(), (side,) * 3, "rel", float(ebs[i]),
                             buf.data_ptr(), buf.numel(), None, sh)
            free[side].append(buf)
            lat.append(time.perf_counter() - ts)
            done_bytes += nbytes[side]
        return np.array(lat), done_bytes / (time.perf_counter() - t0) / 1e9

    log("serve: warmup")
    for side in pool:
        b = take(side)
        ctx.compress_ptr(fields[side].data_ptr(), (side,) * 3, "rel", 1e-3, b.data_ptr(),
                         b.numel(), None, sh)
        free[side].append(b)
    log("serve: served, paced by the trace")
    lat_s, gbs_s_paced = run_served(True)
    log("serve: plain, paced by the trace")
    lat_p, gbs_p_paced = run_plain(True)
    log("serve: served, saturated")
    _, gbs_s_sat = run_served(False)
    log("serve: plain, saturated")
    _, gbs_p_sat = run_plain(False)
    st = srv.stats()
    srv.close()
    # the bound on one request of every size
    worst = 0.0
    for side in pool:
        b = take(side)
        size = ctx.compress_ptr(fields[side].data_ptr(), (side,) * 3, "rel", 1e-4, b.data_ptr(),
                                b.numel(), None, sh)
        y = ctx.decompress(b[:size])
        info = hiz.inspect(b[:512].cpu().numpy().tobytes())
        err = float((fields[side].double() - y.double()).abs().max())
        worst = max(worst, err / info["eps"])
    if worst > 1.0:
        raise SystemExit(f"error bound violated: {worst}")
    ctx.close()
    pct = lambda a, q: round(float(np.percentile(a, q)) * 1e3, 3)
    return {
        "config": {
            "workload": "serving trace: Poisson arrivals 200 req/s, FP32 fields 64^3..512^3 "
                        "(log-uniform volume, GRF k^-3), rel eb from {1e-2,1e-3,1e-4}; "
                        "compression requests, 4 slots, batches of up to 16",
            "requests": n, "duration_s": args.duration, "sides": pool,
        },
        "requests": n, "duration_s": args.duration,
        "served_p50_ms": pct(lat_s, 50), "served_p99_ms": pct(lat_s, 99),
        "plain_p50_ms": pct(lat_p, 50), "plain_p99_ms": pct(lat_p, 99),
        "served_paced_GBps": round(gbs_s_paced, 2), "plain_paced_GBps": round(gbs_p_paced, 2),
        "served_saturated_GBps": round(gbs_s_sat, 2), "plain_saturated_GBps": round(gbs_p_sat, 2),
        "served_vs_plain_saturated": round(gbs_s_sat / gbs_p_sat, 3),
        "server": st,
        "max_err_over_eps": round(worst, 6),
    }


if __name__ == "__main__":
    main()
