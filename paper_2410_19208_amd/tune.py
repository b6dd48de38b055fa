"""Tile-shape tuner of libpsdproj: picks the split-K factor of the passes over A per (precision,
n bucket, padded width) by timing every candidate on the GPU, and writes the table the planner
compiles in (csrc/tile_table.inc).

    python -m paper_2410_19208_amd.tune [--out PATH] [--reps 3]

Run it on a GPU host, then rebuild the library (python paper_2410_19208_amd/build.py).  For
each bucket b (2^b <= n < 2^(b+1), b = 6 .. 14) the problem measured has n = 2^(b + 1/2)
(20000 for b = 14) and r = r_pad - 3; A is a symmetric Gaussian matrix (the pass time does not
depend on its values).  Each candidate factor s (1, 2, 4, 8, 16 with at least 64 rows per K
chunk) is set with psdproj_tile_override, and the device time of the pass and its fixed-order
reduction over `reps` plain q = 0 runs (two passes each) is read from the library's kernel
timers.  Each measurement is a batch of up to 16 problems of the bucket (at most 2^26 elements of
A in all) run as one grouped launch sequence, so the figure is the pass time per problem when the
GPU is shared with other problems' tiles, as in batched and served work; a single large problem
(the bucket of n = 20000) is a batch of one.  The fastest candidate is written to the table.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
PRECS = (("fp64", 0), ("fp32", 1), ("bf16x3", 2))
RPADS = (32, 64, 96, 128, 160, 224, 256)
BUCKETS = range(6, 15)
CANDIDATES = (1, 2, 4, 8, 16)


def batch_size(n):
    """Problems per measured batch: the grouped launches of a batch of small problems, as in
    batched and served work, where every problem's tiles share the GPU with the others'."""
    return max(1, min(16, (1 << 26) // (n * n)))


def measure(pp, BatchProjector, torch, A, n, r_pad, prec_name, prec, split, reps, kinds):
    pp.psdproj_tile_override(prec, split)
    try:
        k = r_pad - 3 - 10
        B = batch_size(n)
        bp = BatchProjector([dict(n=n, k=k, p=10, q=0, variant="plain", precision=prec_name, seed=i)
                             for i in range(B)], device=A.device)
        eff = pp.psdproj_plan_layout(bp.plans[0]).split_k
    finally:
        pp.psdproj_tile_override(prec, 0)
    As = [A] + [A.clone() for _ in range(B - 1)]   # distinct matrices, as in a real batch
    Ps = [torch.empty_like(A) for _ in range(B)]
    bp(As, Ps)   # warm-up (also the graph cache's first sighting)
    torch.cuda.synchronize()
    pp.psdproj_profile_select(kinds)
    pp.psdproj_profile_reset()
    pp.psdproj_profile_enable(True)
    for _ in range(reps):
        bp(As, Ps)
    torch.cuda.synchronize()
    pp.psdproj_profile_enable(False)
    pp.psdproj_profile_select(None)
    total = sum(pp.psdproj_profile_read(kd)[0] for kd in kinds)
    if any(r.status for r in bp.results()):
        raise RuntimeError(f"device status {[r.status for r in bp.results()]}")
    return 1e3 * total / (reps * B), eff   # microseconds per problem, effective factor


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=os.path.join(PKG, "csrc", "tile_table.inc"))
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()

    import torch

    import paper_2410_19208_amd as pp
    from paper_2410_19208_amd.torch_api import BatchProjector

    dev = torch.device("cuda:0")
    names = {pp.psdproj_kernel_name(i): i for i in range(pp.psdproj_kernel_kinds())}
    kinds = [names["k_pass"], names["k_pass_reduce"]]
    rows = []
    t0 = time.perf_counter()
    for b in BUCKETS:
        n = 20000 if b == 14 else int(round(2 ** (b + 0.5)))
        g = torch.Generator(device=dev)
        g.manual_seed(b)
        G = torch.randn((n, n), device=dev, generator=g, dtype=torch.float64)
        A64 = ((G + G.T) * (0.5 / math.sqrt(n))).contiguous()
        del G
        A32 = A64.to(torch.float32)
        for prec_name, prec in PRECS:
            A = A64 if prec == 0 else A32
            for r_pad in RPADS:
                if r_pad - 3 > n:
                    continue
                times = {}
                for s in CANDIDATES:
                    if s > 1 and n // s < 64:
                        continue
                    t, eff = measure(pp, BatchProjector, torch, A, n, r_pad, prec_name, prec, s, args.reps, kinds)
                    if eff not in times:   # K chunks are whole 64-row steps: factors can coincide
                        times[eff] = t
                best = min(times, key=times.get)
                rows.append((prec, b, r_pad, best, n, times))
                print(f"[tune] {prec_name} n={n} r_pad={r_pad}: " +
                      ", ".join(f"s={s} {t:.1f}us" for s, t in times.items()) + f" -> {best}", flush=True)
        del A64, A32
        torch.cuda.empty_cache()
    with open(args.out, "w") as f:
        f.write("// Pass split-K per (precision, n bucket, padded width): {precision, log2 bucket, r_pad, split}.\n")
        f.write("// Written by paper_2410_19208_amd/tune.py from GPU timings of the pass and its reduction\n")
        f.write("// (microseconds per problem of a plain q = 0 batch, two passes each, at the bucket's n) of every\n")
        f.write("// candidate.\n")
        for prec, b, r_pad, best, n, times in rows:
            t = " ".join(f"{s}:{v:.0f}" for s, v in times.items())
            f.write(f"{{{prec}, {b}, {r_pad}, {best}}},  // n={n} {t}\n")
    print(f"[tune] {len(rows)} entries written to {args.out} in {time.perf_counter() - t0:.0f}s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
