#!/usr/bin/env python3
"""Throughput of the randomized PSD projection on one MI355X.

Workload (the paper's large-matrix setting, Sec. 4, with a seeded synthetic stand-in for its
SuiteSparse matrices): n = 20000, A = U diag(lam) U^T stored in FP32 (1.6 GB), U Haar,
5% of lam decaying exponentially from 10 to 1e-4 and the rest uniform in [-1, 0];
k = 200, p = 20, q = 1.  One step = one plain projection (Alg. 2) and one scaled
projection (Alg. 3 with alpha estimated by Alg. 5, N = 10) of the same resident matrix,
run as one grouped launch sequence through the C ABI (psdproj_batch) with the split-BF16
(bf16x3) MFMA passes; the same two projections one after the other (psdproj_run each) are
timed beside it.  After the timed region (none of it counts towards `value`): the plain FP32
form of the same projections (latency, and parity with the oracle), a short serving leg
(Poisson arrivals at 200 and 1000 requests/s through the continuous-batching server, p50/p99
latency, against the FP32 form one request at a time), and the FP64 oracle (parity and the
host-core baseline).  The exit status is 1 when a parity check exceeds its tolerance.

Prints one JSON line (see the repository's design notes for the field definitions).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PSD projections/s + TFLOP/s & HBM GB/s at n=20K,k=200; p50/p99 latency @QPS"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
# relative Frobenius distance to the FP64 oracle on the same inputs
PARITY_TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-5}
# Alg. 5 with N <= PAIRED_MAX: both power iterations share each product (k_gemv2, N + 1 reads
# of A's upper triangle); otherwise they run one after the other (k_gemv, 2 (N + 1) reads).
PAIRED_MAX = 32


def alg5_products(N):
    """(kernel, products per scaled projection, algorithmic bytes per product beyond A's upper
    triangle) of Alg. 5 with N iterations."""
    if N <= PAIRED_MAX:
        return "k_gemv2", N + 1, 4 * 8.0     # two FP64 vectors in, two out, per row
    return "k_gemv", 2 * (N + 1), 2 * 8.0


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_large_20k_bf16x3.md")


def measured_traffic(kernel: str, problems_per_launch: float):
    """HBM bytes per launch (read + written) of `kernel` from the counter summary in profiles/:
    FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy.  None when there is no entry, when the
    launch covers a different number of problems, or when the kernel's source, or a file that
    shapes its launch (the entry's "also" list, e.g. the split-K table), has changed since the
    counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        ent = json.loads(block).get(kernel)
        if ent is None or abs(ent["problems_per_launch"] - problems_per_launch) > 1e-9:
            return None
        for src, digest in [(ent["source"], ent["sha1"])] + [tuple(x) for x in ent.get("also", [])]:
            with open(os.path.join(ROOT, src), "rb") as f:
                if hashlib.sha1(f.read()).hexdigest() != digest:
                    return None
        return float(ent["read_bytes"] + ent["write_bytes"])
    except (OSError, IndexError, ValueError, KeyError):
        return None


def rnd(x, nd):
    return None if x is None else round(x, nd)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--k", type=int, default=200)
    ap.add_argument("--p", type=int, default=20)
    ap.add_argument("--q", type=int, default=1)
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "fp32", "fp64"])
    ap.add_argument("--alpha-iters", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (parity and CPU timing)")
    ap.add_argument("--no-fp32-compare", action="store_true", help="skip timing the plain FP32 form")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-side-timings", action="store_true",
                    help="skip the untimed single-request, one-in-flight and sequential/grouped comparison "
                         "timings (profiler runs: only the warmup, kernel-table and timed steps launch "
                         "kernels, all with --inflight steps in flight)")
    ap.add_argument("--inflight", type=int, default=None,
                    help="steps in flight: consecutive steps go round-robin to this many HIP streams, each "
                         "with its own workspace and outputs, so one step's latency-bound eigensolve "
                         "overlaps the next steps' streaming kernels (1: one stream).  Default 3 for the "
                         "dense step (4 gives 1-2%% more projections/s, but the pass's launches then "
                         "overlap more and each takes longer), 4 for the sparse and structured-sketch "
                         "modes (4 matches the hardware queues HIP gives a process)")
    ap.add_argument("--sequential", action="store_true",
                    help="time the step as two psdproj_run calls instead of one grouped psdproj_batch")
    ap.add_argument("--mode", default="step",
                    choices=["step", "batch", "serve", "counters", "exact", "sdls", "sparse", "sketch", "configs"],
                    help="step: the headline n=20000 step (default); batch: 256 uneven problems in one "
                         "grouped launch sequence; serve: Poisson arrivals through the request server; "
                         "counters: a short run for hardware-counter profiles (symmetric Gaussian A, no QR "
                         "in the generator, two grouped steps, then one 1 GiB device copy for calibration); "
                         "exact: the exact projection (Thm 1) against the randomized ones at n=4096; sdls: "
                         "dual gradient descent (Alg. 6) iterations; sparse: the headline step on a sparse A; "
                         "sketch: the headline step with the structured test matrix; configs: per-projection "
                         "times of the small (n=512) and medium (n=4096) workloads with the oracle's beside them")
    ap.add_argument("--qps", default="50,100,200,500,1000,2000", help="serve mode: arrival rates")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="requests per arrival rate (at most) in serve mode and in the serving leg of the step")
    args = ap.parse_args()
    if args.inflight is None:
        args.inflight = 4 if args.mode in ("sparse", "sketch") else 3
    return args


def main() -> int:
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1; see the design notes for how the projection would shard).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2410_19208_amd as pp
    import workloads
    from paper_2410_19208_amd.torch_api import BatchProjector, Projector

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    if args.mode == "batch":
        return run_batch(args, dev)
    if args.mode == "serve":
        return run_serve(args, dev)
    if args.mode == "counters":
        return run_counters(args, dev)
    if args.mode == "exact":
        return run_exact(args, dev)
    if args.mode == "sdls":
        return run_sdls(args, dev)
    if args.mode == "sparse":
        return run_sparse(args, dev)
    if args.mode == "sketch":
        return run_sketch(args, dev)
    if args.mode == "configs":
        return run_configs(args, dev)
    n, k, p, q = args.n, args.k, args.p, args.q
    r = k + p

    # ---------------------------------------------------------------- workload
    t0 = time.perf_counter()
    U = workloads.haar_orthogonal(n, 3001, device="cuda")
    lam = workloads.spectrum_large(n, 0.05, 3001)
    A64 = workloads.from_spectrum(U, lam)
    A = A64.to(torch.float32) if args.precision != "fp64" else A64
    del A64
    pos = np.nonzero(lam > 0)[0]
    Upos = U[:, torch.as_tensor(pos, device=dev)].contiguous()
    del U
    torch.cuda.synchronize()
    log(f"workload n={n} generated on the GPU in {time.perf_counter() - t0:.1f}s")

    inflight = max(1, args.inflight)
    spec_plain = dict(n=n, k=k, p=p, q=q, variant="plain", precision=args.precision, seed=args.seed)
    spec_scaled = dict(n=n, k=k, p=p, q=q, variant="scaled", precision=args.precision, seed=args.seed,
                       alpha=0.0, alpha_iters=args.alpha_iters)

    class Slot:
        """One step's worth of projectors, workspaces and outputs, and its stream."""

        def __init__(self, stream):
            self.plain = Projector(n, k, p, q, "plain", args.precision, seed=args.seed, device=dev)
            self.scaled = Projector(n, k, p, q, "scaled", args.precision, seed=args.seed, alpha=0.0,
                                    alpha_iters=args.alpha_iters, device=dev)
            self.both = BatchProjector([spec_plain, spec_scaled], device=dev)
            self.P1 = torch.empty_like(A)
            self.P2 = torch.empty_like(A)
            self.stream = stream

        def sequential(self):
            self.plain(A, self.P1, stream=self.stream)
            self.scaled(A, self.P2, stream=self.stream)

        def grouped(self):
            self.both([A, A], [self.P1, self.P2], stream=self.stream)

        def results(self, sequential):
            return (self.plain.result(), self.scaled.result()) if sequential else tuple(self.both.results())

    # slot 0 runs on the current stream; further slots on streams of their own
    slots = [Slot(None)] + [Slot(torch.cuda.Stream(device=dev)) for _ in range(inflight - 1)]
    plain, scaled, both = slots[0].plain, slots[0].scaled, slots[0].both
    P1, P2 = slots[0].P1, slots[0].P2

    def step_sequential():
        slots[0].sequential()

    def step_grouped():
        slots[0].grouped()

    step = step_sequential if args.sequential else step_grouped

    def run_steps(count, nflight):
        """`count` steps, step i on slot i mod nflight; returns once all are enqueued."""
        if nflight > 1:
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream(dev))
            for sl in slots[1:nflight]:
                sl.stream.wait_event(ev)
        for i in range(count):
            sl = slots[i % nflight]
            sl.sequential() if args.sequential else sl.grouped()

    run_steps(max(args.warmup, inflight), inflight)
    torch.cuda.synchronize()
    for sl in slots:
        ra, rb = sl.results(args.sequential)
        if ra.status or rb.status:
            log(f"device status plain={ra.status} scaled={rb.status}")
            return 1
    r1, r2 = slots[0].results(args.sequential)
    # every slot computed the same two projections of the same A: their outputs agree bit for bit
    slots_equal = all(torch.equal(sl.P1, slots[0].P1) and torch.equal(sl.P2, slots[0].P2) for sl in slots[1:])
    if not slots_equal:
        log("outputs of the in-flight slots differ")

    # ---------------------------------------------------------------- per-kernel device times
    # Every launch bracketed by HIP events, over `args.steps` untimed steps run one at a time:
    # the kernel table, and which kernel dominates (the most device time of its own per step;
    # with steps overlapping, a launch's duration also counts the time it shares the GPU with
    # the other step, which favours the many short launches).  (Two event records per launch
    # lengthen a step of ~90 short launches by several per cent, so the timed region below
    # times the dominant kernel only.)
    def read_profile():
        out = {}
        for kind in range(pp.psdproj_kernel_kinds()):
            ms, cnt = pp.psdproj_profile_read(kind)
            if cnt:
                out[pp.psdproj_kernel_name(kind)] = {"kind": kind, "total_ms": ms, "launches": cnt,
                                                     "avg_us": 1e3 * ms / cnt}
        return out

    pp.psdproj_profile_select(None)
    pp.psdproj_profile_reset()
    pp.psdproj_profile_enable(True)
    run_steps(args.steps, 1)
    torch.cuda.synchronize()
    pp.psdproj_profile_enable(False)
    kern = read_profile()
    dom = max(kern, key=lambda kname: kern[kname]["total_ms"])

    # ---------------------------------------------------------------- timed region
    # `inflight` steps in flight; HIP events (on the stream of each launch) around the dominant
    # kernel's launches only
    pp.psdproj_profile_select([kern[dom]["kind"]])
    pp.psdproj_profile_reset()
    pp.psdproj_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(args.steps, inflight)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pp.psdproj_profile_enable(False)
    pp.psdproj_profile_select(None)
    dom_timed = read_profile()[dom]
    ms_per_step = 1e3 * elapsed / args.steps

    # the same steps one at a time on one stream (per-step time without overlap), the dominant
    # kernel timed the same way (a side timing: skipped with --no-side-timings)
    ms_one, dom_one = None, None
    if inflight > 1 and not args.no_side_timings:
        pp.psdproj_profile_select([kern[dom]["kind"]])
        pp.psdproj_profile_reset()
        pp.psdproj_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(args.steps, 1)
        torch.cuda.synchronize()
        ms_one = 1e3 * (time.perf_counter() - t0) / args.steps
        pp.psdproj_profile_enable(False)
        pp.psdproj_profile_select(None)
        dom_one = read_profile()[dom]
    value = 2.0 * args.steps / elapsed
    log(f"{args.steps} steps in {elapsed:.3f}s: {ms_per_step:.3f} ms/step, {value:.1f} projections/s")

    # per-variant latency (untimed region, after the measurement)
    def one(proj, P, reps=5):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            proj(A, P)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / reps

    ms_plain = ms_scaled = ms_other = None
    if not args.no_side_timings:
        ms_plain = one(plain, P1)
        ms_scaled = one(scaled, P2)
        other = step_grouped if args.sequential else step_sequential
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            other()
        torch.cuda.synchronize()
        ms_other = 1e3 * (time.perf_counter() - t) / 3
        step()
        torch.cuda.synchronize()

    # ---------------------------------------------------------------- algorithmic work
    es = 8 if args.precision == "fp64" else 4
    passes = 2 * q + 2
    nn = float(n) * n
    flops_plain = passes * 2 * nn * r + 2 * nn * r1.r_plus
    flops_scaled = passes * 2 * nn * r + 2 * nn * r2.r_plus + 2 * (args.alpha_iters + 1) * 2 * nn
    bytes_plain = (passes + 1) * nn * es
    gk, gprod, gvec = alg5_products(args.alpha_iters)
    # the method's algorithmic bytes: Alg. 5 as 2 (N + 1) products reading A in full, whatever
    # the kernels actually read (the upper triangle once per product pair)
    bytes_scaled = bytes_plain + 2 * (args.alpha_iters + 1) * nn * es
    step_s = ms_per_step / 1e3
    tflops = (flops_plain + flops_scaled) / step_s / 1e12
    gbs = (bytes_plain + bytes_scaled) / step_s / 1e9

    # roofline of the dominant kernel (largest device time per step, one step at a time), with its launches timed
    # in the timed region.  A grouped launch covers every problem active in its stage, so the
    # algorithmic work of one launch is the per-problem figure times the problem-launches of
    # the step over its launches.
    d = dom_timed
    bound, unit, peak = "hbm", "GB/s", HBM_PEAK_GBS
    launches_per_step = d["launches"] / args.steps
    if dom == gk:
        per_unit = n * (n + 1) / 2 * es + gvec * n
        units = gprod
        note = ("upper triangle of the symmetric A read once per product plus the FP64 vectors"
                + (" (both power iterations of Alg. 5 per product)" if gk == "k_gemv2" else ""))
    elif dom == "k_pass":
        # Algorithmic bytes: one read of A per problem-pass, n^2 s (the problems of a grouped
        # launch that stream the same A share its reads in L2, so the launch moves fewer bytes
        # than it is credited with).  The matrix-core work the precision's scheme issues is
        # reported beside it (BF16x3: three BF16 products of 2 n^2 r flops per problem-pass).
        per_unit = nn * es
        units = 2 * passes
        note = (f"one read of A (n^2 x {es} bytes) per pass and problem; a grouped launch covers both "
                f"problems of the step")
    elif dom == "k_rebuild":
        per_unit = nn * es
        units = 2
        note = "P written once per problem"
    else:
        per_unit, units = float("nan"), 1
        note = "no algorithmic byte model for this kernel"
    alg = per_unit * units / launches_per_step
    achieved = alg / (d["avg_us"] * 1e-6) / (1e12 if unit == "TFLOP/s" else 1e9)
    traffic = measured_traffic(dom, units / launches_per_step)
    roofline = {"bound": bound, "kernel": dom, "achieved": round(achieved, 1), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic,
                ("algorithmic_flops_per_launch" if unit == "TFLOP/s" else "algorithmic_bytes_per_launch"): alg,
                "problems_per_launch": round(units / launches_per_step, 3),
                "avg_launch_us": round(d["avg_us"], 2), "model": note,
                "timed_with": f"{inflight} step(s) in flight" + (
                    ": the kernel's launches overlap the other steps' kernels" if inflight > 1 else "")}
    if dom == "k_pass":
        nprod, mpeak = {"bf16x3": (3, BF16_PEAK_TFLOPS), "fp32": (1, FP32_PEAK_TFLOPS),
                        "fp64": (1, FP64_PEAK_TFLOPS)}[args.precision]
        fl = nprod * 2 * nn * r * units / launches_per_step
        tf = fl / (d["avg_us"] * 1e-6) / 1e12
        roofline["mfma_issued"] = {"flops_per_launch": fl, "achieved": round(tf, 1), "peak": mpeak,
                                   "unit": "TFLOP/s", "frac": round(tf / mpeak, 4),
                                   "model": f"{nprod} matrix-core product(s) of 2 n^2 r flops per pass and "
                                            f"problem, r = k + p = {r}"}
    if dom_one is not None:
        ach1 = alg / (dom_one["avg_us"] * 1e-6) / (1e12 if unit == "TFLOP/s" else 1e9)
        roofline["one_in_flight"] = {"avg_launch_us": round(dom_one["avg_us"], 2), "achieved": round(ach1, 1),
                                     "frac": round(ach1 / peak, 4)}

    # every A-streaming kernel against the HBM roofline (algorithmic bytes per launch: a pass is
    # credited with one read of A per problem it covers, although the two problems of the step
    # share their reads of A in L2).
    streaming = {}
    for kname, per_problem, problems_step in (
            ("k_pass", nn * es, 2 * passes),
            (gk, n * (n + 1) / 2 * es + gvec * n, gprod),
            ("k_rebuild", nn * es, 2)):
        if kname in kern:
            kd = kern[kname]
            lps = kd["launches"] / args.steps
            ppl = problems_step / lps
            b = per_problem * ppl
            kgbs = b / (kd["avg_us"] * 1e-6) / 1e9
            streaming[kname] = {"gb_per_launch": round(b / 1e9, 4), "avg_us": round(kd["avg_us"], 2),
                                "achieved_gbs": round(kgbs, 1), "frac_hbm": round(kgbs / HBM_PEAK_GBS, 4),
                                "traffic_bytes": measured_traffic(kname, ppl)}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "projections/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"large_20k: n={n}, k={k}, p={p}, q={q}; one plain (Alg. 2) + one scaled (Alg. 3, "
                               f"alpha by Alg. 5 with N={args.alpha_iters}) projection per step; A fp32 resident",
                   "n": n, "k": k, "p": p, "q": q, "precision": args.precision,
                   "step": "two psdproj_run calls" if args.sequential else "one grouped psdproj_batch of both",
                   "inflight": inflight},
        "slots_bitwise_equal": slots_equal,
        "ms_per_step_one_in_flight": rnd(ms_one, 4) if inflight > 1 else round(ms_per_step, 4),
        "ms_per_step_" + ("grouped" if args.sequential else "sequential"): rnd(ms_other, 4),
        "tflops": round(tflops, 2), "hbm_gbs": round(gbs, 1),
        "latency_ms": {"plain": rnd(ms_plain, 3), "scaled": rnd(ms_scaled, 3)},
        "r_plus": {"plain": r1.r_plus, "scaled": r2.r_plus}, "alpha": r2.alpha_used,
        "roofline": roofline,
        "a_streaming": streaming,
        "kernels_timed_with": "1 step in flight",
        "kernels": {kname: {"avg_us": round(v["avg_us"], 2), "launches_per_step": v["launches"] / args.steps,
                            "ms_per_step": round(v["total_ms"] / args.steps, 4)} for kname, v in kern.items()},
    }

    # ---------------------------------------------------------------- FP32 single-request comparison
    # the plain FP32 form of the same two projections, one request at a time; its outputs are kept
    # for the parity check against the oracle below
    Pf = None
    if not args.no_fp32_compare and not args.no_side_timings and args.precision == "bf16x3":
        f1 = Projector(n, k, p, q, "plain", "fp32", seed=args.seed, device=dev)
        f2 = Projector(n, k, p, q, "scaled", "fp32", seed=args.seed, alpha=0.0, alpha_iters=args.alpha_iters,
                       device=dev)
        f1(A, P1)
        f2(A, P2)
        out["fp32_latency_ms"] = {"plain": round(one(f1, P1, 3), 3), "scaled": round(one(f2, P2, 3), 3)}
        Pf = {"plain": f1(A, torch.empty_like(A)), "scaled": f2(A, torch.empty_like(A))}
        torch.cuda.synchronize()
        if f1.result().status or f2.result().status:
            log("FP32 comparison run reported a device error")
            return 1
        del f1, f2
        plain(A, P1)
        scaled(A, P2)

    # ---------------------------------------------------------------- serving leg
    # Poisson arrivals through the request server, requests drawn from a pool of leading
    # principal blocks of the resident matrix (symmetric, of the same spectral character),
    # against the plain FP32 form one request at a time at the same arrivals
    if not args.no_side_timings and args.precision == "bf16x3":
        buckets = [b for b in (256, 512, 1024, 2048, 4096, 8192, 16384) if b <= n]
        pool = {b: A[:b, :b] for b in buckets}
        serve_points(pool, buckets, [50.0], 40, "bf16x3", 64, dev, 99)   # warm-up
        out["serving"] = {
            "workload": "Poisson arrivals; n log-uniform in [256, 16384] snapped to log-spaced buckets, k in "
                        "{20,50,100,200}, p=10, q=1, plain/scaled 50/50 (alpha by Alg. 5, N=10); requests read "
                        "leading principal blocks of the resident matrix; latency = finish - submit",
            "bf16x3_continuous_batching": serve_points(pool, buckets, [200.0, 1000.0], args.serve_requests,
                                                       "bf16x3", 64, dev, 7000),
            "fp32_one_at_a_time": serve_points(pool, buckets, [200.0, 1000.0], args.serve_requests, "fp32", 1,
                                               dev, 7000)}
        if any(pt["errors"] for v in out["serving"].values() if isinstance(v, list) for pt in v):
            log("serving leg reported device errors")
            return 1

    # ---------------------------------------------------------------- oracle: parity and CPU baseline
    parity_ok = True
    if not args.no_cpu_baseline:
        from oracle import rnla
        try:
            import threadpoolctl
            cores = max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) or os.cpu_count()
        except Exception:
            cores = os.cpu_count()
        torch.cuda.synchronize()
        A_host = A.cpu().numpy().astype(np.float64)
        omega_dtype = np.float64 if args.precision == "fp64" else np.float32
        # the oracle pair (one plain, one scaled projection) repeated until about 10 s of host work
        t0 = time.perf_counter()
        reps = 0
        while True:
            log(f"oracle: plain + scaled projection on the host (pair {reps + 1})")
            o1 = rnla.project(A_host, k, p, q, "plain", seed=args.seed, omega_dtype=omega_dtype)
            o2 = rnla.project(A_host, k, p, q, "scaled", seed=args.seed, alpha_iters=args.alpha_iters,
                              omega_dtype=omega_dtype)
            reps += 1
            cpu_s = time.perf_counter() - t0
            if cpu_s >= 10.0 or reps >= 4:
                break
        out["cpu_baseline"] = {"value": round(2.0 * reps / cpu_s, 5), "unit": "projections/s", "cores": int(cores),
                               "kind": "oracle",
                               "sample": f"{reps} x (one plain + one scaled projection) of the same n={n} workload "
                                         f"(full FP64 oracle incl. Alg. 5 and the n x n rebuild), {cpu_s:.1f} s"}
        a_fro = float(np.linalg.norm(A_host))
        tol = PARITY_TOL[args.precision]
        par = {}
        for name, Pd, o in (("plain", P1, o1), ("scaled", P2, o2)):
            Ph = Pd.cpu().numpy().astype(np.float64)
            par[name] = rnla.parity_error(Ph, o.P, a_fro)
            del Ph
        out["parity"] = {"plain": par["plain"], "scaled": par["scaled"], "tol": tol,
                         "metric": "||P-P_oracle||_F / max(||P_oracle||_F, 1e-2 ||A||_F)",
                         "alpha_oracle": o2.alpha, "r_plus_oracle": {"plain": o1.r_plus, "scaled": o2.r_plus}}
        parity_ok = max(par.values()) < tol
        if Pf is not None:
            pf = {}
            for name, o in (("plain", o1), ("scaled", o2)):
                Ph = Pf[name].cpu().numpy().astype(np.float64)
                pf[name] = rnla.parity_error(Ph, o.P, a_fro)
                del Ph
            out["parity_fp32"] = {"plain": pf["plain"], "scaled": pf["scaled"], "tol": PARITY_TOL["fp32"]}
            parity_ok = parity_ok and max(pf.values()) < PARITY_TOL["fp32"]
        del A_host, o1, o2
    Pf = None
    # accuracy against the exact projection (closed form from the generator's spectrum)
    lam_pos = torch.as_tensor(lam[pos], device=dev)
    Apos = (Upos * lam_pos[None, :]) @ Upos.T
    ea = {}
    for name, Pd in (("plain", P1), ("scaled", P2)):
        ea[name] = float(torch.linalg.norm(Pd.double() - Apos) / torch.linalg.norm(Apos))
    out["e_alg"] = ea
    del Apos
    print(json.dumps(out), flush=True)
    if not parity_ok:
        log("parity against the oracle exceeds the tolerance")
        return 1
    return 0


def run_counters(args, dev) -> int:
    """The headline grouped step on a symmetric Gaussian matrix of the same size (the same kernels
    and bytes; the generator avoids the QR that counter collection does not survive), max(2,
    steps / 10) times, then one plain 1 GiB device-to-device copy whose FETCH_SIZE / WRITE_SIZE
    calibrate the counters."""
    import torch
    from paper_2410_19208_amd.torch_api import BatchProjector
    n, k, p, q = args.n, args.k, args.p, args.q
    g = torch.Generator(device=dev)
    g.manual_seed(args.seed + 1)
    G = torch.randn((n, n), device=dev, generator=g, dtype=torch.float32)
    A = (G + G.T).mul_(0.5 / math.sqrt(n)).contiguous()
    del G
    both = BatchProjector([dict(n=n, k=k, p=p, q=q, variant="plain", precision=args.precision, seed=args.seed),
                           dict(n=n, k=k, p=p, q=q, variant="scaled", precision=args.precision, seed=args.seed,
                                alpha=0.0, alpha_iters=args.alpha_iters)], device=dev)
    P1 = torch.empty_like(A)
    P2 = torch.empty_like(A)
    for _ in range(max(2, args.steps // 10)):   # two steps by default; more to let the clock settle
        both([A, A], [P1, P2])
    torch.cuda.synchronize()
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.add(src, 0.0, out=dst)   # one elementwise dispatch: reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    st = [r.status for r in both.results()]
    print(json.dumps({"mode": "counters", "n": n, "status": st, "copy_bytes": 1 << 30}), flush=True)
    return 0 if not any(st) else 1


def run_batch(args, dev) -> int:
    """256 uneven problems (n log-uniform in [64, 4096], k = min(n/8, 128), p = 10, q = 0,
    plain, BF16x3) through one psdproj_batch call, against a loop of single runs."""
    import torch

    import workloads
    from paper_2410_19208_amd.torch_api import BatchProjector, Projector

    t0 = time.perf_counter()
    sizes = workloads.batched_problem_sizes(256, 4000)
    As, specs = [], []
    for i, (n, k, p, f) in enumerate(sizes):
        U = workloads.haar_orthogonal(n, 4000 + i, device="cuda")
        lam = workloads.spectrum_batched(n, f, 4000 + i)
        As.append(workloads.from_spectrum(U, lam).to(torch.float32).contiguous())
        specs.append(dict(n=n, k=k, p=p, q=0, variant="plain", precision=args.precision, seed=i))
        del U
    torch.cuda.synchronize()
    log(f"256 batched matrices generated in {time.perf_counter() - t0:.1f}s "
        f"(sum n^2 = {sum(a.numel() for a in As) / 1e6:.0f}M elements)")
    bp = BatchProjector(specs, device=dev)
    Ps = [torch.empty_like(a) for a in As]
    singles = []
    for s_ in specs:
        s2 = dict(s_)
        singles.append(Projector(s2.pop("n"), s2.pop("k"), s2.pop("p"), device=dev, **s2))
    for _ in range(2):
        bp(As, Ps)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(reps):
        bp(As, Ps)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / reps
    bad = sum(1 for r in bp.results() if r.status)
    Q = [torch.empty_like(a) for a in As]
    for pr, a, q_ in zip(singles, As, Q):
        pr(a, q_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for pr, a, q_ in zip(singles, As, Q):
            pr(a, q_)
    torch.cuda.synchronize()
    loop_s = (time.perf_counter() - t0) / reps
    same = sum(1 for a, b in zip(Ps, Q) if torch.equal(a, b))
    out = {"metric": "batched PSD projections/s (256 uneven problems, one grouped launch sequence)",
           "value": round(256 / batch_s, 2), "unit": "projections/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": args.precision, "data": "synthetic",
           "config": {"workload": "batched_256: n log-uniform [64, 4096], k = min(n/8, 128), p = 10, q = 0, plain; "
                                  "positive fraction U[0.02, 0.3] geometric 1..1e-3, rest U[-0.1, 0]; seeds 4000+i"},
           "batch_ms": round(1e3 * batch_s, 3), "loop_of_single_runs_ms": round(1e3 * loop_s, 3),
           "speedup_vs_loop": round(loop_s / batch_s, 2), "bitwise_equal_to_single_runs": f"{same}/256",
           "device_errors": bad}
    print(json.dumps(out), flush=True)
    return 0 if (same == 256 and bad == 0) else 1


def serve_points(pool, buckets, qps_list, max_requests, precision, max_inflight, dev, seed0):
    """One serving measurement per arrival rate: Poisson arrivals (workloads.serving_requests),
    each request's n snapped to the nearest pool bucket (log scale), submitted to a fresh server
    (16 GiB budget, `max_inflight` requests in flight; 1 = the plain one-at-a-time FIFO form).
    Latency = finish - submit per request (host clock of the server)."""
    import numpy as np

    import workloads
    from paper_2410_19208_amd.torch_api import Server

    def snap(n):
        return min(buckets, key=lambda b: abs(math.log(b) - math.log(n)))

    out = []
    for i, qps in enumerate(qps_list):
        count = min(max_requests, max(20, int(qps * 3)))
        reqs = workloads.serving_requests(count, qps, seed0 + i)
        srv = Server(16 << 30, max_inflight, device=dev)
        tickets = []
        start = time.perf_counter()
        for (ta, n, k, p, q, variant) in reqs:
            delay = start + ta - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            nb = snap(n)
            kk = min(k, nb - p)
            t, _ = srv.submit(pool[nb], kk, p, q, variant, precision, seed=len(tickets))
            tickets.append(t)
        lat, fin, sub, errs = [], [], [], 0
        for t in tickets:
            r = srv.wait(t, 600.0)
            errs += int(r.status != 0)
            ts, _, tf = srv.times(t)
            lat.append(tf - ts)
            fin.append(tf)
            sub.append(ts)
        srv.close()
        lat = np.array(lat) * 1e3
        span = max(fin) - min(sub)
        out.append({"qps": qps, "requests": count, "achieved_rps": round(count / span, 1),
                    "p50_ms": round(float(np.percentile(lat, 50)), 2),
                    "p99_ms": round(float(np.percentile(lat, 99)), 2), "errors": errs})
        log(f"serve {precision} inflight<={max_inflight} at {qps:g} req/s: {out[-1]}")
    return out


def run_serve(args, dev) -> int:
    """Poisson arrivals through the request server: n from a device-resident pool of seven
    size buckets (256 .. 16384, log-spaced: a log-uniform draw is snapped to the nearest
    bucket), k uniform in {20, 50, 100, 200}, p = 10, q = 1, variant 50/50 (scaled with alpha
    from Alg. 5, N = 10), BF16x3; latency = finish - submit per request."""
    import torch

    import workloads

    buckets = [256, 512, 1024, 2048, 4096, 8192, 16384]
    t0 = time.perf_counter()
    pool = {}
    for n in buckets:
        U = workloads.haar_orthogonal(n, 5000 + n, device="cuda")
        lam = workloads.spectrum_large(n, 0.05, 5000 + n)
        pool[n] = workloads.from_spectrum(U, lam).to(torch.float32).contiguous()
        del U
    torch.cuda.synchronize()
    log(f"serving pool generated in {time.perf_counter() - t0:.1f}s")
    qps = [float(x) for x in args.qps.split(",")]
    serve_points(pool, buckets, [50.0], 40, args.precision, 64, dev, 99)   # warm-up
    points = serve_points(pool, buckets, qps, args.serve_requests, args.precision, 64, dev, 7000)
    # the plain FP32 form one request at a time (FIFO, nothing overlapped), same arrivals
    base = serve_points(pool, buckets, qps[:4], args.serve_requests, "fp32", 1, dev, 7000)
    out = {"metric": "PSD projection serving: throughput and p50/p99 latency at Poisson QPS",
           "value": max(pt["achieved_rps"] for pt in points), "unit": "requests/s (max achieved)", "n_gpus": 1,
           "higher_is_better": True, "dtype": args.precision, "data": "synthetic",
           "config": {"workload": "serving: n in {256..16384} log-spaced buckets, k in {20,50,100,200}, p=10, q=1, "
                                  "plain/scaled 50/50 (alpha by Alg. 5, N=10); continuous batching, max_inflight 64"},
           "points": points, "fp32_one_at_a_time": base}
    print(json.dumps(out), flush=True)
    return 0 if all(pt["errors"] == 0 for pt in points + base) else 1


# ------------------------------------------------------------------------------ helpers of the modes below
def kernel_table(pp, fn, reps):
    """Device time per kernel kind over `reps` calls of fn (every launch timed by the library)."""
    import torch
    pp.psdproj_profile_select(None)
    pp.psdproj_profile_reset()
    pp.psdproj_profile_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    pp.psdproj_profile_enable(False)
    out = {}
    for kind in range(pp.psdproj_kernel_kinds()):
        ms, cnt = pp.psdproj_profile_read(kind)
        if cnt:
            out[pp.psdproj_kernel_name(kind)] = {"avg_us": round(1e3 * ms / cnt, 2),
                                                  "launches_per_call": cnt / reps, "ms_per_call": round(ms / reps, 4)}
    return out


def timed(fn, reps, warm=1):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def host_cores():
    try:
        import threadpoolctl
        return max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) or os.cpu_count()
    except Exception:
        return os.cpu_count()


def roofline_entry(kernel, avg_us, work, bound, peak, unit, model):
    ach = work / (avg_us * 1e-6) / (1e12 if unit == "TFLOP/s" else 1e9)
    return {"bound": bound, "kernel": kernel, "achieved": round(ach, 1), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4), "traffic": None, "avg_launch_us": avg_us,
            ("algorithmic_flops_per_launch" if unit == "TFLOP/s" else "algorithmic_bytes_per_launch"): work,
            "model": model}


FP64_CU_TFLOPS = FP64_PEAK_TFLOPS / 256.0   # one compute unit's share of the FP64 vector peak


def tridiag_roofline(kern, r, problems_per_launch):
    """k_tridiag runs one workgroup (one CU) per problem: its work is the (4/3) r^3 flops of the
    Householder reduction, against the FP64 rate of the CUs it occupies."""
    d = kern["k_tridiag"]
    flops = 4.0 / 3.0 * r ** 3 * problems_per_launch
    e = roofline_entry("k_tridiag", d["avg_us"], flops, "alu", round(FP64_CU_TFLOPS * problems_per_launch, 4),
                       "TFLOP/s", "(4/3) r^3 flops per problem, one workgroup (one CU) per problem")
    return e


def run_exact(args, dev) -> int:
    """The exact projection (Thm 1; the scal = -1 branch of Alg. 6), computed on the GPU through
    the sign function (scaled Newton-Schulz, FP64 GEMMs on the matrix cores), against the
    randomized projections on the same n = 4096 matrix (the medium workload: 200 eigenvalues 1/i,
    the rest uniform in [-0.5, 0], Gaussian noise 1e-3/sqrt(n)): the O(n^3) versus O(k n^2) cost
    the paper states and does not time."""
    import numpy as np
    import torch

    import paper_2410_19208_amd as pp
    import workloads
    from oracle import rnla
    from paper_2410_19208_amd.torch_api import ExactProjector, Projector

    n = 4096
    U = workloads.haar_orthogonal(n, 0, device="cuda")
    lam = workloads.spectrum_medium(n, 200, 0)
    A64 = workloads.from_spectrum(U, lam)
    del U
    ex = ExactProjector(n, "fp64", device=dev)
    P = ex(A64)
    torch.cuda.synchronize()
    if ex.result().status:
        log(f"exact projection status {ex.result().status}")
        return 1
    reps = max(2, args.steps // 5)
    t_exact = timed(lambda: ex(A64, P), reps)
    kern = kernel_table(pp, lambda: ex(A64, P), 1)
    gemm = kern["k_gemm64"]
    rf = roofline_entry("k_gemm64", gemm["avg_us"], 2.0 * n ** 3, "mfma", FP64_PEAK_TFLOPS, "TFLOP/s",
                        "one n x n x n FP64 product (2 n^3 flops) per launch")
    A32 = A64.to(torch.float32)
    rnd = {}
    for prec, A in (("fp64", A64), ("fp32", A32), ("bf16x3", A32)):
        pr = Projector(n, 100, 10, 1, "scaled", prec, seed=0, alpha=0.0, device=dev)
        rnd[prec] = round(1e3 * timed(lambda: pr(A), reps), 3)
    # accuracy of the GPU exact projection against the oracle's eigendecomposition (host, FP64)
    A_host = A64.cpu().numpy()
    t0 = time.perf_counter()
    ref = rnla.exact_projection(A_host)
    cpu_s = time.perf_counter() - t0
    err = float(np.linalg.norm(P.cpu().numpy() - ref) / np.linalg.norm(ref))
    out = {"metric": "exact PSD projections/s (Thm 1 on the GPU) at n=4096, with the randomized ones beside it",
           "value": round(1.0 / t_exact, 3), "unit": "projections/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "medium_4096: n=4096, 200 eigenvalues 1/i, rest U[-0.5,0], noise 1e-3/sqrt(n); "
                                  "exact = sign-function iteration, FP64"},
           "ms_exact": round(1e3 * t_exact, 3), "gemms_per_projection": gemm["launches_per_call"],
           "ms_randomized_scaled_k100_p10_q1": rnd, "speedup_randomized_bf16x3": round(1e3 * t_exact / rnd["bf16x3"], 1),
           "parity_vs_eigendecomposition": err, "tol": PARITY_TOL["fp64"], "r_plus": ex.result().r_plus,
           "roofline": rf, "kernels": kern,
           "cpu_baseline": {"value": round(1.0 / cpu_s, 4), "unit": "projections/s", "cores": int(host_cores()),
                            "kind": "oracle", "sample": f"one exact projection (numpy eigh) of the same n={n} matrix, "
                                                        f"{cpu_s:.1f} s"}}
    print(json.dumps(out), flush=True)
    return 0 if err < PARITY_TOL["fp64"] else 1


def run_sdls(args, dev) -> int:
    """Dual gradient descent for an SDLS problem (Alg. 6) with the scaled randomized projection
    (scal = 1: Alg. 5 + Alg. 3 every iteration), n = 4096, m = 8 constraints, k = 100, l = 10,
    q = 1, BF16x3, after the synthetic recipe of the supplementary SDP section's first example
    (normalised symmetric Gaussian A_i, b from a random PSD X0, random symmetric C), a fixed number
    of iterations (eps = 0); the exact-projection descent (scal = -1) timed beside it."""
    import numpy as np
    import torch

    import paper_2410_19208_amd as pp
    import workloads
    from oracle import sdls
    from paper_2410_19208_amd.torch_api import SdlsSolver

    n, m, k, p, q, iters = 4096, 8, 100, 10, 1, 10
    C, A, b, y0 = workloads.sdls_problem(n, m, 77, dtype=np.float32)
    Cd, Ad = torch.from_numpy(C).to(dev), torch.from_numpy(A).to(dev)
    bt, yt = torch.from_numpy(b), torch.from_numpy(y0)
    solver = SdlsSolver(n, m, k, p, q, 1, "bf16x3", 10, iters, 1.0, 0.5, 0.0, 3, device=dev)
    y, X, info = solver.solve(Cd, Ad, bt, yt)
    t0 = time.perf_counter()
    y, X, info = solver.solve(Cd, Ad, bt, yt)
    t_solve = time.perf_counter() - t0
    if info.status:
        log(f"sdls status {info.status}")
        return 1
    kern = kernel_table(pp, lambda: solver.solve(Cd, Ad, bt, yt), 1)
    dom = max(kern, key=lambda kk: kern[kk]["ms_per_call"])
    per_iter = {kk: v["launches_per_call"] / iters for kk, v in kern.items()}
    es = 4
    models = {"k_pass": (n * n * es * 2 * (q + 1) / per_iter.get("k_pass", 1), "one read of A per pass"),
              "k_gemv": (n * (n + 1) / 2 * es + 2 * n * 8, "upper triangle of X per product"),
              "k_gemv2": (n * (n + 1) / 2 * es + 4 * n * 8, "upper triangle of X per product of both runs"),
              "k_rebuild": (n * n * es, "P written once"),
              "k_sdls_form": ((m + 2) * n * n * es, "C and the A_i read, X written"),
              "k_sdls_trace": ((m + 1) * n * n * es, "the A_i and P read")}
    if dom == "k_tridiag":
        rf = tridiag_roofline(kern, k + p, 1)
    else:
        work, model = models.get(dom, (float("nan"), "no byte model"))
        rf = roofline_entry(dom, kern[dom]["avg_us"], work, "hbm", HBM_PEAK_GBS, "GB/s", model)
    ex_solver = SdlsSolver(n, m, 0, 0, 0, -1, "bf16x3", 10, 2, 1.0, 0.5, 0.0, 3, device=dev)
    ex_solver.solve(Cd, Ad, bt, yt)
    t0 = time.perf_counter()
    _, _, info_ex = ex_solver.solve(Cd, Ad, bt, yt)
    t_ex = (time.perf_counter() - t0) / 2
    # oracle: one iteration on the host, and the GPU's first iterate against it
    one = SdlsSolver(n, m, k, p, q, 1, "bf16x3", 10, 1, 1.0, 0.5, 0.0, 3, device=dev)
    y1, _, _ = one.solve(Cd, Ad, bt, yt)
    t0 = time.perf_counter()
    ref = sdls.dual_gd(C, A, b, 1.0, k, p, q, 10, 1, 0.0, 0.5, 1, y0, seed=3, omega_dtype=np.float32,
                       storage_dtype=np.float32)
    cpu_s = time.perf_counter() - t0
    dy = float(np.max(np.abs(y1.cpu().numpy() - ref.y)))
    out = {"metric": "SDLS dual gradient descent iterations/s (Alg. 6, scaled randomized projection)",
           "value": round(iters / t_solve, 3), "unit": "iterations/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "bf16x3", "data": "synthetic",
           "config": {"workload": f"sdls: n={n}, m={m}, k={k}, l={p}, q={q}, scal=1 (alpha by Alg. 5, N=10), rho=1, "
                                  f"beta=0.5, {iters} iterations; A_i normalised symmetric Gaussian, b from a random "
                                  f"PSD X0"},
           "ms_per_iteration": round(1e3 * t_solve / iters, 3),
           "ms_per_iteration_exact_projection": round(1e3 * t_ex, 3), "grad_norm": info.grad_norm,
           "first_iterate_max_abs_diff_vs_oracle": dy, "roofline": rf, "kernels": kern,
           "cpu_baseline": {"value": round(1.0 / cpu_s, 4), "unit": "iterations/s", "cores": int(host_cores()),
                            "kind": "oracle", "sample": f"one iteration of the oracle's dual_gd on the same problem, "
                                                        f"{cpu_s:.1f} s"}}
    print(json.dumps(out), flush=True)
    return 0


def _pair_slots(args, dev, make_one, like):
    """`--inflight` slots of (plain projector, scaled projector, P1, P2, stream): slot 0 on the
    current stream, the others on streams of their own.  Returns the slots, step(slot, call),
    which runs one step (both projections, in order, on the slot's stream), and a round-robin
    counter: consecutive steps on different slots overlap, as in the headline step."""
    import torch
    inflight = max(1, args.inflight)
    slots = []
    for i in range(inflight):
        a, b = make_one()
        slots.append((a, b, torch.empty_like(like), torch.empty_like(like),
                      None if i == 0 else torch.cuda.Stream(device=dev)))
    ctr = [0]

    def step(slot, fn):
        a, b, P1, P2, st = slot
        fn(a, P1, st)
        fn(b, P2, st)

    return slots, step, ctr


def _step_pair_mode(args, dev, name, make_pair, bytes_model, note):
    """Shared body of the sparse and structured-sketch modes: steps of one plain + one scaled
    projection (two runs each, `--inflight` steps in flight on streams of their own, as in the
    headline step), the kernel table (one step at a time), the dominant kernel's roofline, parity
    with the oracle."""
    import numpy as np
    import torch

    import paper_2410_19208_amd as pp
    from oracle import rnla
    run, run_overlap, results, outputs, oracle_pair, dense_A = make_pair()
    run()
    torch.cuda.synchronize()
    st = [r.status for r in results()]
    if any(st):
        log(f"{name}: device status {st}")
        return 1
    t_one = timed(run, args.steps)
    t_step = timed(run_overlap, args.steps, warm=max(1, args.inflight))
    run()
    torch.cuda.synchronize()
    kern = kernel_table(pp, run, max(2, args.steps // 4))
    dom = max(kern, key=lambda kk: kern[kk]["ms_per_call"])
    if dom == "k_tridiag":
        rf = tridiag_roofline(kern, args.k + args.p, 1)
    else:
        work, model = bytes_model(dom, kern)
        rf = roofline_entry(dom, kern[dom]["avg_us"], work, "hbm", HBM_PEAK_GBS, "GB/s", model)
    # the streaming kernels against the HBM roofline as well
    stream = {}
    for kk in ("k_pass", "k_gemv", "k_gemv2", "k_rebuild"):
        if kk in kern:
            w, m = bytes_model(kk, kern)
            stream[kk] = roofline_entry(kk, kern[kk]["avg_us"], w, "hbm", HBM_PEAK_GBS, "GB/s", m)
    out = {"metric": f"PSD projections/s ({note})", "value": round(2.0 / t_step, 3), "unit": "projections/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": args.precision, "data": "synthetic",
           "config": {"workload": name, "inflight": max(1, args.inflight)}, "ms_per_step": round(1e3 * t_step, 3),
           "ms_per_step_one_in_flight": round(1e3 * t_one, 3),
           "r_plus": [r.r_plus for r in results()], "roofline": rf, "a_streaming": stream,
           "kernels_timed_with": "1 step in flight", "kernels": kern}
    if not args.no_cpu_baseline:
        A_host = dense_A()
        t0 = time.perf_counter()
        refs = oracle_pair(A_host)
        cpu_s = time.perf_counter() - t0
        a_fro = float(np.linalg.norm(A_host))
        par = [rnla.parity_error(o.cpu().numpy().astype(np.float64), r.P, a_fro) for o, r in zip(outputs(), refs)]
        out["parity"] = {"plain": par[0], "scaled": par[1], "tol": PARITY_TOL[args.precision]}
        out["cpu_baseline"] = {"value": round(2.0 / cpu_s, 5), "unit": "projections/s", "cores": int(host_cores()),
                               "kind": "oracle", "sample": f"one plain + one scaled projection, {cpu_s:.1f} s"}
        if max(par) >= PARITY_TOL[args.precision]:
            print(json.dumps(out), flush=True)
            return 1
    print(json.dumps(out), flush=True)
    return 0


def run_sparse(args, dev) -> int:
    """The headline parameters (n = 20000, k = 200, p = 20, q = 1, plain + scaled with alpha by
    Alg. 5) on a sparse symmetric A (CSR, about 32 stored entries per row, the spectral character
    of the dense stand-in on the diagonal): the paper's benchmark matrices are sparse."""
    import numpy as np
    import torch

    import workloads
    from oracle import rnla
    from paper_2410_19208_amd.torch_api import SparseProjector

    n, k, p, q, per_row = args.n, args.k, args.p, args.q, 32
    prec = args.precision
    dt = np.float64 if prec == "fp64" else np.float32
    rp, ci, v, D = workloads.sparse_symmetric(n, per_row, 8001, dt)
    nnz = len(ci)
    del D
    rpd, cid, vd = (torch.from_numpy(x).to(dev) for x in (rp, ci, v))
    like = torch.empty((n, n), dtype=vd.dtype, device=dev)
    slots, step, ctr = _pair_slots(args, dev, lambda: (
        SparseProjector(n, k, p, q, "plain", prec, seed=args.seed, device=dev),
        SparseProjector(n, k, p, q, "scaled", prec, seed=args.seed, alpha=0.0, alpha_iters=args.alpha_iters,
                        device=dev)), like)
    del like
    s1, s2, P1, P2 = slots[0][:4]

    def make_pair():
        def call(proj, P, st):
            proj(rpd, cid, vd, P, stream=st)

        def run():
            step(slots[0], call)

        def run_overlap():
            step(slots[ctr[0] % len(slots)], call)
            ctr[0] += 1

        def dense():
            return workloads.sparse_symmetric(n, per_row, 8001, dt)[3]

        def oracle_pair(Ah):
            return (rnla.project(Ah, k, p, q, "plain", seed=args.seed, omega_dtype=dt),
                    rnla.project(Ah, k, p, q, "scaled", seed=args.seed, alpha_iters=args.alpha_iters, omega_dtype=dt))
        return run, run_overlap, lambda: (s1.result(), s2.result()), lambda: (P1, P2), oracle_pair, dense

    es = 8 if prec == "fp64" else 4

    def bytes_model(dom, kern):
        per_problem = {"k_rebuild": (float(n) * n * es, "P written once"),
                       "k_pass": (nnz * (4 + es) + (n + 1) * 4 + n * (k + p) * es,
                                  "the CSR arrays and the panel read once per pass"),
                       "k_gemv": (nnz * (4 + es) + (n + 1) * 4 + 2 * n * 8, "the CSR arrays and two vectors"),
                       "k_gemv2": (nnz * (4 + es) + (n + 1) * 4 + 4 * n * 8, "the CSR arrays and four vectors")}
        w, m = per_problem.get(dom, (float("nan"), "no byte model"))
        lpc = kern[dom]["launches_per_call"]
        gk, gprod, _ = alg5_products(args.alpha_iters)
        problems = {"k_rebuild": 2, "k_pass": 2 * (2 * q + 2), gk: gprod}.get(dom, lpc)
        return w * problems / lpc, m
    return _step_pair_mode(args, dev, f"sparse_20k: n={n}, {nnz / n:.1f} stored entries per row (CSR, both "
                                      f"triangles), k={k}, p={p}, q={q}; one plain + one scaled projection per step",
                           make_pair, bytes_model, "sparse A, CSR")


def run_sketch(args, dev) -> int:
    """The headline step with the structured (subsampled randomized Hadamard) test matrix in place
    of the Gaussian one (Sec. 3.1's footnote): same matrix, same parameters."""
    import numpy as np
    import torch

    import workloads
    from oracle import rnla
    from paper_2410_19208_amd.torch_api import Projector

    n, k, p, q = args.n, args.k, args.p, args.q
    U = workloads.haar_orthogonal(n, 3001, device="cuda")
    lam = workloads.spectrum_large(n, 0.05, 3001)
    A = workloads.from_spectrum(U, lam).to(torch.float32 if args.precision != "fp64" else torch.float64)
    del U
    dt = np.float64 if args.precision == "fp64" else np.float32
    slots, step, ctr = _pair_slots(args, dev, lambda: (
        Projector(n, k, p, q, "plain", args.precision, seed=args.seed, device=dev, sketch="srht"),
        Projector(n, k, p, q, "scaled", args.precision, seed=args.seed, alpha=0.0, alpha_iters=args.alpha_iters,
                  device=dev, sketch="srht")), A)
    s1, s2, P1, P2 = slots[0][:4]

    def make_pair():
        def call(proj, P, st):
            proj(A, P, stream=st)

        def run():
            step(slots[0], call)

        def run_overlap():
            step(slots[ctr[0] % len(slots)], call)
            ctr[0] += 1

        def oracle_pair(Ah):
            return (rnla.project(Ah, k, p, q, "plain", seed=args.seed, omega_dtype=dt, sketch="srht"),
                    rnla.project(Ah, k, p, q, "scaled", seed=args.seed, alpha_iters=args.alpha_iters, omega_dtype=dt,
                                 sketch="srht"))
        return run, run_overlap, lambda: (s1.result(), s2.result()), lambda: (P1, P2), oracle_pair, \
            lambda: A.cpu().numpy().astype(np.float64)

    es = 8 if args.precision == "fp64" else 4

    def bytes_model(dom, kern):
        lpc = kern[dom]["launches_per_call"]
        per = {"k_pass": (float(n) * n * es, 2 * (2 * q + 2), "one read of A per pass and problem"),
               "k_rebuild": (float(n) * n * es, 2, "P written once")}
        gk, gprod, gvec = alg5_products(args.alpha_iters)
        per[gk] = (n * (n + 1) / 2 * es + gvec * n, gprod, "upper triangle per product")
        if dom not in per:
            return float("nan"), "no byte model"
        w, problems, m = per[dom]
        return w * problems / lpc, m
    return _step_pair_mode(args, dev, f"large_20k with the structured test matrix: n={n}, k={k}, p={p}, q={q}; "
                                      f"one plain + one scaled projection per step (two runs)",
                           make_pair, bytes_model, "structured subsampled-Hadamard test matrix")


def run_configs(args, dev) -> int:
    """Per-projection GPU times of the small workload (n = 512, k = 40, p = 10, q = 0, plain,
    FP64) and of the medium one (n = 4096, k = 100, p = 10, q in {0, 1}, plain and scaled with
    alpha by Alg. 5, FP32 and BF16x3), each a psdproj_run replayed from the graph cache, with the
    oracle's time for the same projection on the host."""
    import numpy as np
    import torch

    import workloads
    from oracle import rnla
    from paper_2410_19208_amd.torch_api import Projector

    rows = []
    A, _, _ = workloads.make_matrix("small", 512, 1001, storage="fp64")
    At = torch.from_numpy(A).to(dev)
    pr = Projector(512, 40, 10, 0, "plain", "fp64", seed=0, device=dev)
    t_gpu = timed(lambda: pr(At), 50, warm=3)
    t0 = time.perf_counter()
    for _ in range(5):
        rnla.project(A, 40, 10, 0, "plain", seed=0)
    t_cpu = (time.perf_counter() - t0) / 5
    rows.append({"config": "small n=512 k=40 p=10 q=0 plain fp64", "gpu_ms": round(1e3 * t_gpu, 4),
                 "oracle_ms": round(1e3 * t_cpu, 2)})
    A, _, _ = workloads.make_matrix("medium", 4096, 0, storage="fp32", noise=1e-3 / math.sqrt(4096))
    At = torch.from_numpy(A).to(dev)
    A64 = A.astype(np.float64)
    for q in (0, 1):
        for variant in ("plain", "scaled"):
            t0 = time.perf_counter()
            rnla.project(A64, 100, 10, q, variant, seed=0, omega_dtype=np.float32)
            t_cpu = time.perf_counter() - t0
            for prec in ("fp32", "bf16x3"):
                pr = Projector(4096, 100, 10, q, variant, prec, seed=0, device=dev)
                t_gpu = timed(lambda: pr(At), 20, warm=3)
                rows.append({"config": f"medium n=4096 k=100 p=10 q={q} {variant} {prec}",
                             "gpu_ms": round(1e3 * t_gpu, 4), "oracle_ms": round(1e3 * t_cpu, 1)})
    for r in rows:
        r["gpu_over_oracle_speedup"] = round(r["oracle_ms"] / r["gpu_ms"], 1)
    out = {"metric": "per-projection time of the small and medium workloads (single requests)", "rows": rows,
           "cores": int(host_cores()), "unit": "ms"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
