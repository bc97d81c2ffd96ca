"""The benchmark's FP32 workload without its measurement code, for profilers.

    python -m paper_1611_02568_amd.profile_run [--n 1000000] [--steps 1000]

Runs what `bench.py` times on the FP32 path -- the 1,000,000 x 128 Zipf(1.1)
mixture, perplexity 50, screen 2048, the same initial embedding, 20 warm-up
iterations and then `--steps` iterations -- and finally copies a buffer of
`--copy-mib` MiB once, a kernel of known traffic for scaling hardware byte
counters.  The iterations are bit-reproducible, so iterations 21..20+steps
here are the benchmark's timed iterations.
"""
from __future__ import annotations

import argparse
import sys


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()

    import torch

    from . import datagen, pixelsne

    X, _, _ = datagen.zipf_mixture_1m(n=args.n)
    y0 = torch.as_tensor(datagen.initial_embedding(args.n, seed=datagen.seed_for(2, 1)))
    ctx = pixelsne.Context.from_data(torch.from_numpy(X).cuda(), 50.0, 2048, Y_init=y0,
                                     precision=pixelsne.FP32)
    print("setup done", flush=True)
    ctx.step(args.warmup)
    for done in range(0, args.steps, 100):
        ctx.step(min(100, args.steps - done))
        print(f"iterations {args.warmup + min(done + 100, args.steps)}", flush=True)
    if args.copy_mib:
        a = torch.ones(args.copy_mib * 2**18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
    torch.cuda.synchronize()
    print("done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
