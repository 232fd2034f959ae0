"""Short runs of the hot path for hardware-counter profiling.

    python paper_1403_7394_amd/profile_run.py [--sweeps K] [--copy-gib G] [--n N] [--rows R] [--rb B]
    python paper_1403_7394_amd/profile_run.py --builds
    python paper_1403_7394_amd/profile_run.py --batch [--iters T] [--copy-gib G]

--builds: the similarity of the 32768-point, 64-dimensional workload built once in each
mode (direct, FP32 GEMM, BF16, BF16x3 on the matrix cores), nothing else.

--batch: the batched workload (512 problems, N ~ U{64..2048}, d = 16, L = 3, damping 0.8)
run once for T iterations (default 200) in the launch shape (1024 threads, 512 workgroups,
4 row groups), after the calibration copy.

Builds the FP32 similarity of the 8192-point, 64-blob 2-D workload on the GPU, runs K full
sweeps (all three levels, damping 0.9, no stop rule; the row pass in points mode unless
--read-s) and, before that, one device copy of
G GiB (read G GiB, write G GiB) whose counter readings calibrate the HBM byte counters.
--rows R updates rows [0, R) only (one device's block of a run split by rows, at its real
shape R x N); --rb B sets the rows per workgroup.
Every kernel runs on torch's current stream; a line is printed after each step.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--sweeps", type=int, default=4)
    ap.add_argument("--copy-gib", type=float, default=1.0)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--rows", type=int, default=0,
                    help="update rows [0, rows) only: one block of a run split by rows (0: all)")
    ap.add_argument("--rb", type=int, default=0, help="rows per workgroup (0: the default launch)")
    ap.add_argument("--read-s", action="store_true", help="row pass reads S (default: points mode)")
    ap.add_argument("--builds", action="store_true", help="profile the similarity builds instead")
    ap.add_argument("--batch", action="store_true", help="profile the batched form instead")
    ap.add_argument("--iters", type=int, default=200, help="--batch: iterations")
    args = ap.parse_args()

    import torch

    from paper_1403_7394_amd import hap, synth

    if not torch.cuda.is_available():
        print("profile_run needs a GPU", file=sys.stderr)
        return 2
    hap.load()
    dev = torch.device("cuda:0")
    if args.builds:
        blobs, _ = synth.workload_precision()
        n = blobs.X.shape[0]
        X = torch.from_numpy(blobs.X).to(dev)
        S = torch.empty((n, n), dtype=torch.float32, device=dev)
        for name, mode in (("direct", hap.BUILD_DIRECT), ("gemm_f32", hap.BUILD_GEMM), ("bf16", hap.BUILD_BF16),
                           ("bf16x3", hap.BUILD_BF16X3)):
            hap.build_similarity(X, S, mode=mode)
            torch.cuda.synchronize()
            print(f"build {name}: {n} x {n} from d = {blobs.X.shape[1]}", flush=True)
        return 0
    if args.copy_gib > 0:
        words = int(args.copy_gib * (1 << 30)) // 4
        src = torch.ones(words, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy: {words * 4} bytes read, {words * 4} bytes written", flush=True)
        del src, dst
    if args.batch:
        import numpy as np
        problems, rp = synth.workload_batched()
        sizes = [b.X.shape[0] for b in problems]
        X = torch.from_numpy(np.concatenate([b.X for b in problems])).to(dev)
        bt = hap.HapBatch(sizes, problems[0].X.shape[1], rp.levels)
        bt.set_launch(1024, 512, 4)
        out = bt.outputs(dev)
        torch.cuda.synchronize()
        print(f"batch ready: {len(sizes)} problems, sum n^2 = {sum(k * k for k in sizes)}", flush=True)
        bt.run(X, rp.damping, args.iters, out=out)
        torch.cuda.synchronize()
        print(f"batch done: {args.iters} iterations", flush=True)
        bt.close()
        return 0
    blobs, rp = synth.workload_plain_f32(n=args.n)
    n = blobs.X.shape[0]
    X = torch.from_numpy(blobs.X).to(dev)
    S = torch.empty((n, n), dtype=torch.float32, device=dev)
    hap.build_similarity(X, S)
    h = hap.Hap(S, rp.levels, rp.damping)
    if args.rows:
        h.set_row_count(args.rows)
    if args.rb:
        h.set_launch(rows_per_block=args.rb)
    if not args.read_s:
        h.set_points(X)
    torch.cuda.synchronize()
    print(f"similarity and state ready: n={n} levels={rp.levels}", flush=True)
    res = h.iterate(args.sweeps)
    torch.cuda.synchronize()
    print(f"sweeps done: {res.iters}; launch {h.get_launch()}; rows {h.get_row_count()}", flush=True)
    h.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
