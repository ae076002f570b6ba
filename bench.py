#!/usr/bin/env python3
"""Benchmark of Fourier-accelerated steepest-descent Landau gauge fixing.

Workload: one 32^4 SU(3) lattice (V = 2^20 sites) from the seeded generator
(U = g exp(i eps H) g^dag(x+mu), eps for mean plaquette 0.6), alpha 0.08,
FP64, links stored as two rows (12 reals).  A "step" is one iteration of
Algorithm 1 (filter, g, gauge transform, Delta/F/theta), on links resident in
HBM.  Printed as one JSON line:

  value          iterations per second (K timed iterations, no profiling)
  roofline       the dominant kernel (fused transform + Delta + (x,y) FFT):
                 algorithmic bytes per launch / its mean duration from HIP
                 events on the library's stream in a second, profiled pass
  time_to_theta  wall time of lgf_fix to theta < 1e-15 for FP64 (12- and
                 18-real) and mixed FP32/FP64, from freshly loaded links:
                 best of three fixes on one context (the first, which also
                 captures the context's graphs, is reported beside it)
  mixed_16       16^4, seeds 1-4: plain FP64 against FP32 bulk + FP64 finish
  batch          64 lattices of three shapes in one lgf_batch (mixed), against
                 the same lattices fixed one by one in single contexts
  cpu_baseline   the FP64 oracle on this host's cores, a bounded sample

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
LEARNED_DIMS = (32, 32, 32, 64)
PAPER_C2070_ITERS_PER_S = 16.35    # 32^4, DP, 12-real, texture, ECC off (Table 3)


def alg_bytes(V, s, R):
    """Algorithmic HBM bytes: per iteration and per launch of each kernel.

    The links are G U0 G^dag(x+mu), formed where needed from the loaded links
    U0 (R reals per link) and the accumulated gauge G (kept as two rows, 12
    reals per site, for either link storage) and never stored.  Per site and
    iteration: U0 read once (4R) and G read once (12) by the transform; the
    packed Delta (8 reals) written once, read and written once by the (z, t)
    pass, and read once by the gauge kernel (32 reals); G read and written
    once by the gauge kernel (24).
    """
    return {
        "iteration": V * s * (4 * R + 12 + 32 + 24),
        "transform_measure": V * s * (4 * R + 12 + 8),
        "zt_fft_scale": V * s * 16,
        "gauge": V * s * (8 + 24),
    }


def source_digest():
    """Hash of the kernel and launch sources with comments and blank space
    removed: it changes when the code that was measured changes."""
    import re
    h = hashlib.sha256()
    for f in ("su3.hpp", "fft.hpp", "kernels.hpp", "runtime.hpp", "lgf.hip"):
        with open(os.path.join(ROOT, "paper_1206_0675_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, dims, storage):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    key = f"{kernel}@{'x'.join(map(str, dims))}/{storage}"
    e = rec.get(key)
    if not e or e.get("source_digest") != source_digest():
        return None
    return e.get("bytes_per_launch")


MIXED16_DIMS = (16, 16, 16, 16)


def batch_workload():
    """64 lattices of three shapes (24 x 8^4, 24 x 16^3 x 32, 16 x 16^4); lattice i
    has eps = 0.2 + 0.3 i / 63 and seed 1000 + i."""
    shapes = [(8, 8, 8, 8)] * 24 + [(16, 16, 16, 32)] * 24 + [(16, 16, 16, 16)] * 16
    return shapes, [0.2 + 0.3 * i / 63 for i in range(64)]


def fix_best(ctx, U, tries, torch):
    """Best of `tries` fixes from freshly loaded links (the first also
    captures the context's graphs)."""
    runs = []
    for _ in range(tries):
        ctx.load(U)
        ctx.measure()
        torch.cuda.synchronize()
        runs.append(ctx.fix())
    return min(runs, key=lambda r: r.seconds), runs[0]


def mixed_16(L, fields, torch):
    """16^4, four seeds: plain FP64 against FP32 bulk + FP64 finish."""
    from paper_1206_0675_amd import lgf
    out = []
    for seed, U in fields:
        rec = {"seed": seed}
        for label, kw in (("fp64", {}), ("mixed", {"precision": lgf.MIXED})):
            with lgf.Context(MIXED16_DIMS, lib=L, storage=12, poll_every=8, **kw) as ctx:
                s, _ = fix_best(ctx, U, 3, torch)
            rec[label] = {"seconds": round(s.seconds, 5), "iters": s.iter, "iters_fp32": s.iter_fp32, "F": s.F,
                          "theta": s.theta}
        rec["F_mixed_minus_fp64"] = rec["mixed"]["F"] - rec["fp64"]["F"]
        out.append(rec)
    return out


def batch_run(L, shapes, Us, torch):
    """The batch of 64 in one lgf_batch (mixed, 12-real, autotuned) against the
    same lattices fixed one by one in single contexts."""
    from paper_1206_0675_amd import lgf
    with lgf.Batch(shapes, lib=L, precision=lgf.MIXED, storage=12, poll_every=8, autotune=1) as b:
        best = None
        for _ in range(2):                 # the first fix also captures the graph
            for i, U in enumerate(Us):
                b.load(i, U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = b.fix()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        cfg = b.config()
    ok = all(x.status == lgf.OK and x.theta < 1e-15 for x in st)
    single = 0.0
    for d, U in zip(shapes, Us):
        with lgf.Context(d, lib=L, precision=lgf.MIXED, storage=12, poll_every=8) as ctx:
            s, _ = fix_best(ctx, U, 2, torch)
            single += s.seconds
    sites = sum(d[0] * d[1] * d[2] * d[3] for d in shapes)
    return {"configs": len(shapes), "sites": sites, "all_converged": ok, "seconds": round(best, 5),
            "configs_per_s": round(len(shapes) / best, 2), "iters_total": int(sum(x.iter for x in st)),
            "single_contexts_seconds": round(single, 5), "speedup_vs_single": round(single / best, 3),
            "launch_shape": {"plane_threads": cfg[0], "tile_bytes": cfg[1]}}


def shape_sweep(L, dims, R, U, args):
    """Force each candidate launch shape through the autotuner's cache file
    and time it like the main measurement."""
    import tempfile
    import torch
    from paper_1206_0675_amd import lgf
    cache = os.path.join(tempfile.mkdtemp(), "tune.txt")
    os.environ["LGF_TUNE_CACHE"] = cache
    with lgf.Context(dims, lib=L, storage=R, autotune=1) as ctx:
        print(f"# autotuner pick (threads, tile bytes): {ctx.config()}", flush=True)
    with open(cache) as fh:
        key = fh.read().split()[0]
    for nth in (64, 128, 256):
        for tb in (32, 64, 128):
            with open(cache, "w") as fh:
                fh.write(f"{key} {nth} {tb}\n")
            with lgf.Context(dims, lib=L, storage=R, autotune=1) as ctx:
                ctx.load(U)
                ctx.step(args.warmup)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.step(args.steps)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            with lgf.Context(dims, lib=L, storage=R, autotune=1, profile=1) as ctx:
                ctx.load(U)
                ctx.step(args.warmup)
                ctx.profile_reset()
                ctx.step(args.steps)
                prof = ctx.profile()
            us = {k: round(ms / n * 1e3, 1) for k, (n, ms) in prof.items() if n}
            print(f"threads {nth} tile_bytes {tb}: {args.steps / dt:.1f} iters/s, kernel us {us}", flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dims", type=int, nargs=4, default=[32, 32, 32, 32])
    ap.add_argument("--storage", type=int, default=12, choices=[12, 18])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the time-to-theta runs")
    ap.add_argument("--learned-seeds", type=int, default=4,
                    help="32^3x64 fields (seeds 3000...) for the learned-vs-plain comparison (0: skip)")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="for hardware counters: a few iterations, then one plain device copy of "
                         "--copy-mib MiB (a kernel of known traffic that scales FETCH_SIZE/WRITE_SIZE); no JSON")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--batch-sample", action="store_true",
                    help="run only the batch of 64 (one lgf_batch fix, then the lattices one by one) and print "
                         "its JSON; for profiling")
    ap.add_argument("--shape-sweep", action="store_true",
                    help="time every launch shape the autotuner chooses from (threads per plane block x tile "
                         "row bytes), one line each; no JSON")
    ap.add_argument("--gen-workers", type=int, default=1,
                    help="worker processes for input generation (fork + exec); leave at 1 under a profiler, "
                         "which sets up the GPU before this program starts")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              "there is no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import synth

    # All inputs are generated before this program touches the GPU (with
    # --gen-workers > 1 the generator starts worker processes by fork and exec).
    dims = tuple(args.dims)
    V = synth.volume(dims)
    t = time.time()
    U = None
    if not args.batch_sample:
        U = synth.random_links(dims, args.seed, workers=args.gen_workers)
        print(f"# generated {dims} seed {args.seed} in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    model_path = os.path.join(ROOT, "paper_1206_0675_amd", "models", "learned_step.bin")
    learned_fields = []
    if not (args.pmc_sample or args.shape_sweep or args.batch_sample or args.no_extras) and args.learned_seeds > 0 and os.path.exists(model_path):
        t = time.time()
        learned_fields = [(seed, synth.random_links(LEARNED_DIMS, seed, workers=args.gen_workers))
                          for seed in range(3000, 3000 + args.learned_seeds)]
        print(f"# generated {len(learned_fields)} fields {LEARNED_DIMS} in {time.time() - t:.1f}s", file=sys.stderr,
              flush=True)

    extra_inputs = not (args.pmc_sample or args.shape_sweep or args.no_extras) or args.batch_sample
    mixed16 = []
    batch_in = None
    if extra_inputs:
        t = time.time()
        mixed16 = [] if args.batch_sample else [(seed, synth.random_links(MIXED16_DIMS, seed)) for seed in (1, 2, 3, 4)]
        shapes, eps = batch_workload()
        batch_in = (shapes, [synth.random_links(d, 1000 + i, eps=e) for i, (d, e) in enumerate(zip(shapes, eps))])
        print(f"# generated the 16^4 seeds and the batch of {len(shapes)} in {time.time() - t:.1f}s", file=sys.stderr,
              flush=True)

    import torch

    from paper_1206_0675_amd import lgf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    L = lgf.load_library()
    R = args.storage
    ab = alg_bytes(V, 8, R)

    if args.pmc_sample:
        with lgf.Context(dims, lib=L, storage=R) as ctx:
            ctx.load(U)
            ctx.step(5)
        n = args.copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"# pmc sample: 5 iterations, then one copy of {args.copy_mib} MiB", file=sys.stderr, flush=True)
        return

    if args.shape_sweep:
        shape_sweep(L, dims, R, U, args)
        return
    if args.batch_sample:
        print(json.dumps(batch_run(L, batch_in[0], batch_in[1], torch)), flush=True)
        return

    # ---- timed iterations (no profiling) -----------------------------------
    with lgf.Context(dims, lib=L, storage=R) as ctx:
        launch_shape = dict(zip(("plane_threads", "tile_bytes"), ctx.config()))
        ctx.load(U)
        ctx.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    dt = t1 - t0
    iters_per_s = args.steps / dt
    print(f"# {args.steps} iterations in {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)

    # ---- profiled pass: per-kernel durations from HIP events ----------------
    with lgf.Context(dims, lib=L, storage=R, profile=1) as ctx:
        ctx.load(U)
        ctx.step(args.warmup)
        ctx.profile_reset()
        ctx.step(args.steps)
        prof = ctx.profile()
    kernels = {}
    for name in ("transform_measure", "zt_fft_scale", "gauge", "reduce"):
        n, ms = prof.get(name, (0, 0.0))
        if n:
            avg_s = ms / n / 1e3
            k = {"launches": n, "avg_us": round(avg_s * 1e6, 2)}
            if name in ab:
                k["alg_bytes"] = ab[name]
                k["gbps"] = round(ab[name] / avg_s / 1e9, 1)
                k["frac"] = round(ab[name] / avg_s / 1e9 / HBM_PEAK_GBPS, 4)
            kernels[name] = k
    dom = kernels["transform_measure"]
    achieved = dom["gbps"]
    traffic = measured_traffic("transform_measure", dims, R)

    # ---- time to theta < 1e-15 ---------------------------------------------
    extras = {}
    if not args.no_extras:
        for label, kw in (("fp64_12real", dict(storage=12)), ("fp64_18real", dict(storage=18)),
                          ("mixed_12real", dict(storage=12, precision=lgf.MIXED)),
                          ("mixed_18real", dict(storage=18, precision=lgf.MIXED))):
            with lgf.Context(dims, lib=L, poll_every=8, **kw) as ctx:
                runs = []
                for _ in range(3):         # the first fix also captures the context's graphs
                    ctx.load(U)
                    ctx.measure()
                    torch.cuda.synchronize()
                    runs.append(ctx.fix())
            s = min(runs, key=lambda r: r.seconds)
            extras[label] = {"seconds": round(s.seconds, 5), "first_seconds": round(runs[0].seconds, 5),
                             "iters": s.iter, "iters_fp32": s.iter_fp32, "F": s.F, "theta": s.theta}

    # ---- learned vs plain step: time to theta < 1e-15 on 32^3 x 64 ----------
    learned = None
    if learned_fields:
        with open(model_path, "rb") as fh:
            blob = fh.read()
        ld = LEARNED_DIMS
        runs = []
        for seed, Ul in learned_fields:
            rec = {"seed": seed}
            for label, kw in (("plain", {}), ("learned", {"step": lgf.STEP_LEARNED})):
                with lgf.Context(ld, lib=L, storage=12, poll_every=8, **kw) as ctx:
                    if kw:
                        ctx.set_model(blob)
                    tries = []
                    for _ in range(2):     # the first fix also captures the context's graphs
                        ctx.load(Ul)
                        ctx.measure()
                        torch.cuda.synchronize()
                        tries.append(ctx.fix())
                    s = min(tries, key=lambda r: r.seconds)
                rec[label] = {"seconds": round(s.seconds, 5), "iters": s.iter, "fallbacks": s.fallbacks, "F": s.F,
                              "theta": s.theta}
            rec["F_diff"] = abs(rec["learned"]["F"] - rec["plain"]["F"])
            runs.append(rec)
            print(f"# learned vs plain seed {seed}: {rec['plain']['iters']} -> {rec['learned']['iters']} iterations, "
                  f"{rec['plain']['seconds']:.4f} -> {rec['learned']['seconds']:.4f} s", file=sys.stderr, flush=True)
        tp = sum(r["plain"]["seconds"] for r in runs)
        tl = sum(r["learned"]["seconds"] for r in runs)
        learned = {"dims": list(ld), "storage": 12, "runs": runs, "plain_seconds": round(tp, 5),
                   "learned_seconds": round(tl, 5), "speedup": round(tp / tl, 4) if tl > 0 else None}

    # ---- 16^4 mixed precision, and the batch of 64 ----------------------------
    m16 = mixed_16(L, mixed16, torch) if mixed16 else None
    batch = batch_run(L, batch_in[0], batch_in[1], torch) if batch_in else None
    if batch:
        print(f"# batch of {batch['configs']}: {batch['seconds']:.4f} s, {batch['configs_per_s']} configs/s, "
              f"{batch['speedup_vs_single']}x one by one", file=sys.stderr, flush=True)

    # ---- CPU baseline: the FP64 oracle on this host -------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.opts(store12=(R == 12))
        n_a, n_b = 2, 32
        t = time.perf_counter()
        oracle.step(dims, U, n_a, o)
        t_a = time.perf_counter() - t
        t = time.perf_counter()
        oracle.step(dims, U, n_b, o)
        t_b = time.perf_counter() - t
        cpu = {"value": round((n_b - n_a) / (t_b - t_a), 4), "unit": "iters/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"FP64 oracle (plain C, OpenMP) on the same {'x'.join(map(str, dims))} lattice, "
                         f"{R}-real: rate = {n_b - n_a} / (t({n_b} updates) - t({n_a} updates)), "
                         f"{t_a + t_b:.1f}s of CPU work"}

    it_bytes = ab["iteration"]
    line = {
        "metric": "FA-SD iters/s and time to theta<1e-15 on 32^4 SU(3); HBM GB/s; learned vs plain",
        "value": round(iters_per_s, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} SU(3) FA-SD iteration, FP64, {R}-real links, alpha 0.08",
                   "dims": list(dims), "storage": R, "seed": args.seed, "generator": "g exp(i eps H) g^dag, plaquette 0.6"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "transform_measure", "alg_bytes_per_launch": ab["transform_measure"]},
        "iteration_alg_gbps": round(it_bytes * iters_per_s / 1e9, 1),
        "iteration_frac": round(it_bytes * iters_per_s / 1e9 / HBM_PEAK_GBPS, 4),
        "kernels": kernels,
        "time_to_theta": extras,
        "learned_vs_plain": learned,
        "mixed_16": m16,
        "batch": batch,
        "cpu_baseline": cpu,
        "context": {"paper_c2070_iters_per_s": PAPER_C2070_ITERS_PER_S,
                    "device": torch.cuda.get_device_name(0), "source_digest": source_digest(),
                    "launch_shape": launch_shape},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
