"""Measures the launch-shape table of the runtime: for fields of several sizes
and shapes, every Huffman chunk length and tile depth, the compress +
decompress time of one field on the GPU and the compression ratio.

The runtime's default chunk and tile depth per field (`default_launch` in
csrc/runtime.hip) are read off this table: the chunk with the highest
compress + decompress throughput among those whose ratio is within 1 % of the
best chunk's, and the fastest tile depth for it. The tile depth never changes
the output; the chunk is recorded in each stream.

Usage (on the GPU): python -m paper_2507_11165_amd.tune_table [--steps 5]
Prints one line per (shape, chunk, tile) and the pick per shape.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SHAPES = [(64, 64, 64), (128, 128, 128), (192, 192, 192), (256, 256, 256), (100, 500, 500),
          (384, 384, 384), (512, 512, 512), (384, 96, 48), (48, 96, 384)]
CHUNKS = [256, 512, 1024, 2048]
TILES = [1, 2, 4]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eb", type=float, default=1e-3)
    ap.add_argument("--shapes", type=str, default="",
                    help="only these shapes, e.g. 512x512x512,64x64x64")
    args = ap.parse_args()

    import numpy as np
    import torch

    import fieldgen
    from paper_2507_11165_amd import hiz

    dev = torch.device("cuda:0")
    ctx = hiz.Context(0)
    sh = hiz.C.c_void_p(torch.cuda.current_stream().cuda_stream)
    picks = []
    shapes = SHAPES
    if args.shapes:
        shapes = [tuple(int(v) for v in t.split("x")) for t in args.shapes.split(",")]
    for shape in shapes:
        x = fieldgen.grf(shape, 11.0 / 3.0, 9000 + shape[0])
        N = x.size
        xd = torch.from_numpy(x).to(dev)
        cap = 5 * N + (1 << 20)
        zb = torch.empty(cap, dtype=torch.uint8, device=dev)
        yb = torch.empty(shape, dtype=torch.float32, device=dev)
        rows = []
        for chunk in CHUNKS:
            for tz in TILES:
                p = hiz.make_params(tune=True, chunk=chunk, tile_z=tz)

                def step():
                    size = ctx.compress_ptr(xd.data_ptr(), shape, "rel", args.eb, zb.data_ptr(),
                                            cap, p, sh)
                    ctx.decompress_ptr(zb.data_ptr(), size, yb.data_ptr(), N, sh)
                    return size

                for _ in range(args.warmup):
                    size = step()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    size = step()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / args.steps * 1e3
                gbs = 8.0 * N / (ms * 1e-3) / 1e9
                ratio = 4.0 * N / size
                rows.append((chunk, tz, ms, gbs, ratio))
                # per-kernel means of two more (profiled, untimed) steps
                ctx.reset_profile()
                ctx.set_profiling(True)
                for _ in range(2):
                    step()
                torch.cuda.synchronize()
                ctx.set_profiling(False)
                prof = ctx.profile()
                ks = " ".join(f"{k}={v[1] / max(v[0], 1) * 1e3:.1f}us" for k, v in sorted(prof.items())
                              if k in ("encode", "decode", "predict_quant", "reconstruct", "coarse",
                                       "coarse_rec"))
                print(f"shape {shape} N {N} chunk {chunk} tile_z {tz} ms {ms:.4f} "
                      f"GBps {gbs:.1f} ratio {ratio:.4f} {ks}", flush=True)
        best_ratio = max(r[4] for r in rows)
        ok = [r for r in rows if r[4] >= 0.99 * best_ratio]
        best = max(ok, key=lambda r: r[3])
        picks.append((shape, N, best))
        print(f"pick {shape} N {N}: chunk {best[0]} tile_z {best[1]} ({best[3]:.1f} GB/s, "
              f"ratio {best[4]:.4f}; best ratio {best_ratio:.4f})", flush=True)
        del xd, zb, yb
        torch.cuda.empty_cache()
    print("summary")
    for shape, N, b in picks:
        print(f"  {shape} N={N}: chunk {b[0]} tile_z {b[1]}")


if __name__ == "__main__":
    main()
