"""The benchmark's workloads without their measurement code, for profilers.

    python -m paper_1611_02568_amd.profile_run [--what iter|knn] [--n 1000000]
                                               [--steps 1000] [--warmup 20] [--fp64]
                                               [--attract-side B --attract-help H]
                                           [--attract-fork snap|cells|auto]

--what iter (default): what `bench.py` times on the FP32 (or, with --fp64, the
FP64) path -- the 1,000,000 x 128 Zipf(1.1) mixture, perplexity 50, screen
2048, the same initial embedding, `--warmup` iterations and then `--steps`
iterations.  The iterations are bit-reproducible, so iterations
warmup+1 .. warmup+steps here are the benchmark's timed iterations.
--attract-side / --attract-help set the attraction's blocks per CU on the
second stream and in the helper after Z (defaults 2 and 3); 0 and 16 run all
of the attraction's row sums after the traversal, on the whole GPU, which
times that kernel alone.  --attract-fork fixes where the second stream takes
up the row sums (after the snap pass or after the cells) instead of the
device-side tuner's choice (auto, the default).  The results do not depend on
any of them.
--what knn: the brute-force kNN of the same 1,000,000 x 128 rows (k = 150),
the setup's MFMA kernel, alone.
Both finish by copying a buffer of `--copy-mib` MiB once, a kernel of known
traffic for scaling hardware byte counters.
"""
from __future__ import annotations

import argparse
import sys


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--what", choices=("iter", "knn"), default="iter")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--attract-side", type=int, default=2)
    ap.add_argument("--attract-help", type=int, default=3)
    ap.add_argument("--attract-fork", choices=("snap", "cells", "auto"), default="auto")
    args = ap.parse_args()

    import torch

    from . import datagen, pixelsne

    X, _, _ = datagen.zipf_mixture_1m(n=args.n)
    Xd = torch.from_numpy(X).cuda()
    if args.what == "knn":
        pixelsne.knn(Xd, 150)
        torch.cuda.synchronize()
        print("knn done", flush=True)
    else:
        y0 = torch.as_tensor(datagen.initial_embedding(args.n, seed=datagen.seed_for(2, 1)))
        ctx = pixelsne.Context.from_data(Xd, 50.0, 2048, Y_init=y0,
                                         precision=pixelsne.FP64 if args.fp64 else pixelsne.FP32,
                                         attract_blocks_per_cu=args.attract_side,
                                         attract_help_blocks_per_cu=args.attract_help,
                                         attract_fork={"snap": pixelsne.FORK_SNAP,
                                                       "cells": pixelsne.FORK_CELLS,
                                                       "auto": pixelsne.FORK_AUTO}[args.attract_fork])
        print("setup done", flush=True)
        for done in range(0, args.warmup, 100):
            ctx.step(min(100, args.warmup - done))
            print(f"warm-up {min(done + 100, args.warmup)}", flush=True)
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
