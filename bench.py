#!/usr/bin/env python3
"""Benchmark of Fourier-accelerated steepest-descent Landau gauge fixing.

Headline workload: one 32^4 SU(3) lattice (V = 2^20 sites) from the seeded
generator (U = g exp(i eps H) g^dag(x+mu), eps for mean plaquette 0.6),
alpha 0.08, FP64, links stored as two rows (12 reals).  A "step" is one
iteration of Algorithm 1 (filter, g, gauge transform, Delta/F/theta) on links
resident in HBM.  Printed as one JSON line:

  value            iterations per second (K timed iterations, no profiling)
  roofline         the dominant kernel (fused transform + Delta + (x,y) FFT):
                   algorithmic bytes per launch / its mean duration from HIP
                   events on the library's stream, in a second, profiled pass
  per_precision    32^4 iteration rate, kernel times and roofline fractions in
                   FP64 and FP32, 12- and 18-real links
  time_to_theta    32^4, seeds 1-4: wall time of lgf_fix to theta < 1e-15 from
                   freshly loaded links (Algorithm 1's first measurement
                   included) for FP64 and mixed FP32/FP64, 12- and 18-real,
                   and mixed 12-real with the switch to FP64 at theta 1e-12
  small_8          8^4: iteration rate and time to theta, F against the oracle
  mixed_16         16^4, seeds 1-4: plain FP64 against FP32 bulk + FP64 finish
  batch            64 lattices of three shapes in one lgf_batch (mixed), with
                   its aggregate algorithmic bandwidth, against the same
                   lattices fixed one by one in single contexts
  rate_32x32x32x64 the iteration rate and kernel times at 32^3x64 (seed 3000),
                   FP64, 12-real: the second HBM-resident shape
  learned_vs_plain 32^3x64, seeds 3000-3003: the committed learned step
                   against the plain step
  update_variants  16^4: iterations and time to theta for first-order and
                   exact-exponential updates over a sweep of alpha, and plain
                   steepest descent (no Fourier acceleration)
  wilson_32        the paper's workload class: Wilson-action fields at 32^4,
                   beta 5.8, 6.0, 6.2 (cold start, 102 updates of one heatbath
                   and four overrelaxation sweeps, all on the GPU), their
                   plaquette and time to theta for FP64, mixed (switch to
                   FP64 at theta 1e-6, 1e-10, 1e-12) and learned (and an
                   alpha sweep at beta 6.0), then three more fields
                   per beta in FP64 (four per beta, as in Table 3); heatbath and
                   overrelaxation sweep times with the
                   algorithmic bytes of a sweep (every link read and each
                   updated link written, per class launch)
  fft_study        32^4: the filter's 4D FFT as 1D x4, 2D+1D+1D and 2D+2D passes
                   over HBM, and 2D+1D+1D with the t DFTs on the matrix cores
                   (lgf_fft_study), ms per application
  rate_repeats     five more timed runs of K iterations: median, min, max
  copy_ceiling     a 1 GiB device copy's GB/s, and the transform kernel's and
                   the iteration's algorithmic GB/s as fractions of it
  cpu_baseline     the FP64 oracle on this host's cores, a bounded sample of
                   the headline workload; oracle_time_to_theta: full oracle
                   runs at 8^4, 16^4 and 32^4 with all cores, and at 8^4 with
                   one (16^4 per iteration)

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
HEADLINE_DIMS = (32, 32, 32, 32)
LEARNED_DIMS = (32, 32, 32, 64)
MIXED16_DIMS = (16, 16, 16, 16)
SMALL_DIMS = (8, 8, 8, 8)
PAPER_C2070_ITERS_PER_S = 16.35    # 32^4, DP, 12-real, texture, ECC off (Table 3)


def alg_bytes(V, s, R):
    """Algorithmic HBM bytes per iteration and per launch of each kernel.

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


def rewrite_design_bytes(V, s, R, with_G=False):
    """The reference byte count of one iteration of a design that reads and
    rewrites the links: V s (8R + 2R_g + 32), R_g = R; the FP32 phase of a
    mixed run adds the accumulated gauge (+2R_g)."""
    return V * s * (8 * R + (4 if with_G else 2) * R + 32)


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


def batch_workload():
    """64 lattices of three shapes (24 x 8^4, 24 x 16^3 x 32, 16 x 16^4); lattice i
    has eps = 0.2 + 0.3 i / 63 and seed 1000 + i."""
    shapes = [(8, 8, 8, 8)] * 24 + [(16, 16, 16, 32)] * 24 + [(16, 16, 16, 16)] * 16
    return shapes, [0.2 + 0.3 * i / 63 for i in range(64)]


def vol(d):
    return d[0] * d[1] * d[2] * d[3]


# ---------------------------------------------------------------------------
# GPU measurements
# ---------------------------------------------------------------------------
def fix_runs(ctx, U, tries, torch):
    """Fixes from freshly loaded links; each time includes Algorithm 1's first
    measurement.  Returns (best, first): the first also captures the
    context's graphs."""
    runs = []
    for _ in range(tries):
        ctx.load(U)
        torch.cuda.synchronize()
        runs.append(ctx.fix(raise_on_error=False))
    return min(runs, key=lambda r: r.seconds), runs[0]


def rate_and_kernels(L, dims, U, steps, warmup, torch, repeats=0, **kw):
    """Iteration rate over `steps` plain lgf_step iterations, then a profiled
    pass with per-kernel mean durations (HIP events).  With repeats > 0 the
    shape also carries the rates of that many further timed runs of `steps`
    (median, min, max), beside the one timed region the rate comes from."""
    from paper_1206_0675_amd import lgf
    with lgf.Context(dims, lib=L, **kw) as ctx:
        shape = dict(zip(("plane_threads", "tile_bytes"), ctx.config()))
        ctx.load(U)
        ctx.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if repeats:
            rates = []
            for _ in range(repeats):
                t1 = time.perf_counter()
                ctx.step(steps)
                torch.cuda.synchronize()
                rates.append(steps / (time.perf_counter() - t1))
            rates.sort()
            shape["repeats"] = {"n": repeats, "median_iters_per_s": round(rates[len(rates) // 2], 2),
                                "min": round(rates[0], 2), "max": round(rates[-1], 2)}
    with lgf.Context(dims, lib=L, profile=1, **kw) as ctx:
        ctx.load(U)
        ctx.step(warmup)
        ctx.profile_reset()
        ctx.step(steps)
        prof = ctx.profile()
    return steps / dt, dt / steps, prof, shape


def kernel_table(prof, ab):
    out = {}
    for name in ("transform_measure", "zt_fft_scale", "gauge", "reduce"):
        n, ms = prof.get(name, (0, 0.0))
        if n:
            avg_s = ms / n / 1e3
            k = {"launches": n, "avg_us": round(avg_s * 1e6, 2)}
            if name in ab:
                k["alg_bytes"] = ab[name]
                k["gbps"] = round(ab[name] / avg_s / 1e9, 1)
                k["frac"] = round(ab[name] / avg_s / 1e9 / HBM_PEAK_GBPS, 4)
            out[name] = k
    return out


def per_precision(L, U, args, torch):
    from paper_1206_0675_amd import lgf
    V = vol(HEADLINE_DIMS)
    out = {}
    for prec, pname, s in ((lgf.FP64, "fp64", 8), (lgf.FP32, "fp32", 4)):
        for R in (12, 18):
            rate, t_it, prof, _ = rate_and_kernels(L, HEADLINE_DIMS, U, args.steps, args.warmup, torch,
                                                   precision=prec, storage=R)
            ab = alg_bytes(V, s, R)
            sb = rewrite_design_bytes(V, s, R, with_G=(s == 4))
            out[f"{pname}_{R}real"] = {
                "iters_per_s": round(rate, 2), "ms_per_iter": round(t_it * 1e3, 4),
                "iteration_alg_bytes": ab["iteration"],
                "iteration_frac": round(ab["iteration"] / t_it / 1e9 / HBM_PEAK_GBPS, 4),
                "rewrite_design_bytes": sb, "rewrite_design_frac": round(sb / t_it / 1e9 / HBM_PEAK_GBPS, 4),
                "kernels": kernel_table(prof, ab)}
            print(f"# {pname} {R}-real: {rate:.1f} iters/s", file=sys.stderr, flush=True)
    return out


def rate_32x64(L, U, args, torch):
    """The other HBM point: iteration rate and kernel times at 32^3 x 64 (seed
    3000), FP64, 12-real, as the headline measures 32^4."""
    V = vol(LEARNED_DIMS)
    rate, t_it, prof, _ = rate_and_kernels(L, LEARNED_DIMS, U, args.steps, args.warmup, torch, storage=12)
    ab = alg_bytes(V, 8, 12)
    print(f"# 32^3x64 FP64 12-real: {rate:.1f} iters/s", file=sys.stderr, flush=True)
    return {"dims": list(LEARNED_DIMS), "storage": 12, "seed": 3000, "iters_per_s": round(rate, 2),
            "ms_per_iter": round(t_it * 1e3, 4), "iteration_alg_bytes": ab["iteration"],
            "iteration_frac": round(ab["iteration"] / t_it / 1e9 / HBM_PEAK_GBPS, 4),
            "kernels": kernel_table(prof, ab)}


def time_to_theta_32(L, fields, torch):
    from paper_1206_0675_amd import lgf
    modes = (("fp64_12real", dict(storage=12)), ("fp64_18real", dict(storage=18)),
             ("mixed_12real", dict(storage=12, precision=lgf.MIXED)),
             ("mixed_18real", dict(storage=18, precision=lgf.MIXED)),
             ("mixed_12real_switch_1e-12", dict(storage=12, precision=lgf.MIXED, theta_switch=1e-12)))
    out = {label: [] for label, _ in modes}
    for seed, U in fields:
        for label, kw in modes:
            with lgf.Context(HEADLINE_DIMS, lib=L, poll_every=8, **kw) as ctx:
                s, first = fix_runs(ctx, U, 2, torch)
            out[label].append({"seed": seed, "seconds": round(s.seconds, 5), "first_seconds": round(first.seconds, 5),
                               "iters": s.iter, "iters_fp32": s.iter_fp32, "F": s.F, "theta": s.theta})
        print(f"# 32^4 seed {seed}: " + ", ".join(f"{k} {v[-1]['seconds'] * 1e3:.2f} ms" for k, v in out.items()),
              file=sys.stderr, flush=True)
    for label in list(out):
        runs = out[label]
        out[label] = {"runs": runs, "mean_seconds": round(sum(r["seconds"] for r in runs) / len(runs), 5)}
    return out


def small_8(L, U, torch, oracle_F):
    from paper_1206_0675_amd import lgf
    rate, t_it, _, _ = rate_and_kernels(L, SMALL_DIMS, U, 500, 50, torch)
    with lgf.Context(SMALL_DIMS, lib=L, poll_every=8) as ctx:
        s, first = fix_runs(ctx, U, 5, torch)
    return {"dims": list(SMALL_DIMS), "iters_per_s": round(rate, 1), "ms_per_iter": round(t_it * 1e3, 4),
            "time_to_theta_s": round(s.seconds, 6), "first_seconds": round(first.seconds, 6), "iters": s.iter,
            "F": s.F, "F_minus_oracle": (s.F - oracle_F) if oracle_F is not None else None,
            "note": "cache resident (2 MB of links): launch and latency bound, not an HBM roofline point"}


def mixed_16(L, fields, torch):
    """16^4, four seeds: plain FP64 against FP32 bulk + FP64 finish."""
    from paper_1206_0675_amd import lgf
    out = []
    for seed, U in fields:
        rec = {"seed": seed}
        for label, kw in (("fp64", {}), ("mixed", {"precision": lgf.MIXED})):
            with lgf.Context(MIXED16_DIMS, lib=L, storage=12, poll_every=8, **kw) as ctx:
                s, _ = fix_runs(ctx, U, 3, torch)
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
            s, _ = fix_runs(ctx, U, 2, torch)
            single += s.seconds
    sites = sum(vol(d) for d in shapes)
    # algorithmic bytes of every iteration every member made, in its precision
    moved = sum(x.iter_fp32 * alg_bytes(vol(d), 4, 12)["iteration"] + x.iter_fp64 * alg_bytes(vol(d), 8, 12)["iteration"]
                for d, x in zip(shapes, st))
    return {"configs": len(shapes), "sites": sites, "all_converged": ok, "seconds": round(best, 5),
            "configs_per_s": round(len(shapes) / best, 2), "iters_total": int(sum(x.iter for x in st)),
            "alg_bytes_total": int(moved), "aggregate_alg_gbps": round(moved / best / 1e9, 1),
            "aggregate_frac": round(moved / best / 1e9 / HBM_PEAK_GBPS, 4),
            "single_contexts_seconds": round(single, 5), "speedup_vs_single": round(single / best, 3),
            "launch_shape": {"plane_threads": cfg[0], "tile_bytes": cfg[1]}}


def learned_vs_plain(L, fields, blob, torch):
    from paper_1206_0675_amd import lgf
    runs = []
    for seed, Ul in fields:
        rec = {"seed": seed}
        for label, kw in (("plain", {}), ("learned", {"step": lgf.STEP_LEARNED})):
            with lgf.Context(LEARNED_DIMS, lib=L, storage=12, poll_every=8, **kw) as ctx:
                if kw:
                    ctx.set_model(blob)
                s, _ = fix_runs(ctx, Ul, 2, torch)
            rec[label] = {"seconds": round(s.seconds, 5), "iters": s.iter, "fallbacks": s.fallbacks, "F": s.F,
                          "theta": s.theta}
        rec["F_diff"] = abs(rec["learned"]["F"] - rec["plain"]["F"])
        runs.append(rec)
        print(f"# learned vs plain seed {seed}: {rec['plain']['iters']} -> {rec['learned']['iters']} iterations, "
              f"{rec['plain']['seconds']:.4f} -> {rec['learned']['seconds']:.4f} s", file=sys.stderr, flush=True)
    tp = sum(r["plain"]["seconds"] for r in runs)
    tl = sum(r["learned"]["seconds"] for r in runs)
    return {"dims": list(LEARNED_DIMS), "storage": 12, "runs": runs, "plain_seconds": round(tp, 5),
            "learned_seconds": round(tl, 5), "speedup": round(tp / tl, 4) if tl > 0 else None}


def wilson_32(L, blob, torch):
    """Wilson-action fields at 32^4 from the GPU generator, then gauge fixing."""
    from paper_1206_0675_amd import lgf
    V = vol(HEADLINE_DIMS)
    sweep_bytes = 8 * (4 * V + V // 2) * 96           # 8 class launches: read all links, write half of one direction
    #                                                   (rows 0 and 1 of each link, as the sweeps store them)
    out = {"dims": list(HEADLINE_DIMS), "updates": 102, "or_per_update": 4, "runs": []}
    for i, beta in enumerate((5.8, 6.0, 6.2)):
        with lgf.WilsonGenerator(HEADLINE_DIMS, beta, 5000 + i, lib=L) as g:
            t = time.perf_counter()
            g.update(102, 4)
            t_gen = time.perf_counter() - t
            if i == 1:
                t = time.perf_counter()
                g.update(10, 0)
                t_hb = (time.perf_counter() - t) / 10
                t = time.perf_counter()
                for _ in range(10):
                    g.sweep(lgf.OVERRELAX)
                t_or = (time.perf_counter() - t) / 10
                out["heatbath_sweep_ms"] = round(t_hb * 1e3, 3)
                out["overrelax_sweep_ms"] = round(t_or * 1e3, 3)
                out["sweep_alg_bytes"] = sweep_bytes
                out["heatbath_alg_gbps"] = round(sweep_bytes / t_hb / 1e9, 1)
                out["heatbath_frac"] = round(sweep_bytes / t_hb / 1e9 / HBM_PEAK_GBPS, 4)
                out["overrelax_alg_gbps"] = round(sweep_bytes / t_or / 1e9, 1)
                g.sweep_index = 0
                g.cold()
                g.update(102, 4)
            rec = {"beta": beta, "seed": 5000 + i, "plaquette": round(g.plaquette(), 6),
                   "generate_s": round(t_gen, 3), "skipped": g.skipped()}
            modes = [("fp64_12real", dict(storage=12)), ("mixed_12real", dict(storage=12, precision=lgf.MIXED))]
            if blob is not None:
                modes.append(("learned_12real", dict(storage=12, step=lgf.STEP_LEARNED)))
            for label, kw in modes:
                with lgf.Context(HEADLINE_DIMS, lib=L, max_iter=100000, **kw) as ctx:
                    if "step" in kw:
                        ctx.set_model(blob)
                    ctx.load_device(g.device_links)
                    torch.cuda.synchronize()
                    s = ctx.fix(raise_on_error=False)
                rec[label] = {"status": s.status, "iters": s.iter, "seconds": round(s.seconds, 4),
                              "theta": s.theta, "F": s.F}
                if "step" in kw:
                    rec[label]["fallbacks"] = s.fallbacks
            # the mixed run's switch to FP64 taken later than the default theta = 1e-6
            for ts in (1e-10, 1e-12):
                with lgf.Context(HEADLINE_DIMS, lib=L, max_iter=100000, storage=12, precision=lgf.MIXED,
                                 theta_switch=ts) as ctx:
                    ctx.load_device(g.device_links)
                    torch.cuda.synchronize()
                    s = ctx.fix(raise_on_error=False)
                rec[f"mixed_12real_switch_{ts:g}"] = {"status": s.status, "iters": s.iter, "iters_fp32": s.iter_fp32,
                                                      "seconds": round(s.seconds, 4), "F": s.F}
            if i == 1:
                sweep = []
                for alpha in (0.06, 0.07, 0.075, 0.08):
                    with lgf.Context(HEADLINE_DIMS, lib=L, storage=12, max_iter=20000, alpha=alpha) as ctx:
                        ctx.load_device(g.device_links)
                        torch.cuda.synchronize()
                        s = ctx.fix(raise_on_error=False)
                    sweep.append({"alpha": alpha, "status": s.status, "iters": s.iter, "seconds": round(s.seconds, 4),
                                  "F": s.F})
                rec["alpha_sweep_fp64_12real"] = sweep
            # three more fields at this beta (Table 3 has four per beta), FP64 only
            more = []
            for k in range(3):
                seed = 5100 + 10 * i + k
                with lgf.WilsonGenerator(HEADLINE_DIMS, beta, seed, lib=L) as g2:
                    g2.update(102, 4)
                    P2 = g2.plaquette()
                    with lgf.Context(HEADLINE_DIMS, lib=L, max_iter=100000, storage=12) as ctx:
                        ctx.load_device(g2.device_links)
                        torch.cuda.synchronize()
                        s = ctx.fix(raise_on_error=False)
                more.append({"seed": seed, "plaquette": round(P2, 6), "status": s.status, "iters": s.iter,
                             "seconds": round(s.seconds, 4), "F": s.F})
            rec["more_fields_fp64_12real"] = more
            out["runs"].append(rec)
            print(f"# wilson beta {beta}: P {rec['plaquette']}, FP64 {rec['fp64_12real']['iters']} iterations "
                  f"{rec['fp64_12real']['seconds']} s, mixed {rec['mixed_12real']['seconds']} s", file=sys.stderr,
                  flush=True)
    return out


def fft_study_32(L, torch, kernels):
    """The filter's 4D FFT split three ways at 32^4 (four FP64 complex fields
    in the plain layout), ms per application and bandwidth on the passes'
    bytes (each pass reads and writes 64 V bytes); beside them, the
    iteration's own (z, t) kernel, which is all the filter adds to HBM traffic
    there (its (x, y) passes ride in the transform and gauge kernels)."""
    from paper_1206_0675_amd import lgf
    V = vol(HEADLINE_DIMS)
    g = torch.Generator(device="cpu").manual_seed(7)
    shape = (4, HEADLINE_DIMS[3], HEADLINE_DIMS[2], HEADLINE_DIMS[1], HEADLINE_DIMS[0])
    f = torch.complex(torch.randn(shape, dtype=torch.float64, generator=g),
                      torch.randn(shape, dtype=torch.float64, generator=g)).cuda()
    out = {"dims": list(HEADLINE_DIMS), "fields": 4, "reps": 20}
    for name, v, passes in (("1d_x4", lgf.FFT_1DX4, 7), ("2d_1d_1d", lgf.FFT_2D1D1D, 5), ("2d_2d", lgf.FFT_2D2D, 3),
                            ("2d_1d_1d_mfma_t", lgf.FFT_2D1D1D_MFMA, 5)):
        _, ms = lgf.fft_study(HEADLINE_DIMS, v, f, reps=20, lib=L)
        b = passes * 2 * 64 * V
        out[name] = {"ms": round(ms, 4), "passes": passes, "alg_bytes": b, "gbps": round(b / ms / 1e6, 1),
                     "frac": round(b / ms / 1e6 / HBM_PEAK_GBPS, 4)}
    out["2d_2d_faster_than_1d_x4"] = round(out["1d_x4"]["ms"] / out["2d_2d"]["ms"], 3)
    out["2d_2d_faster_than_2d_1d_1d"] = round(out["2d_1d_1d"]["ms"] / out["2d_2d"]["ms"], 3)
    out["mfma_t_vs_fft_t"] = round(out["2d_1d_1d"]["ms"] / out["2d_1d_1d_mfma_t"]["ms"], 3)
    zt = kernels.get("zt_fft_scale", {})
    out["iteration_zt_ms"] = round(zt.get("avg_us", 0.0) / 1e3, 4)
    del f
    print(f"# fft study 32^4: 1D x4 {out['1d_x4']['ms']} ms, 2D+1D+1D {out['2d_1d_1d']['ms']} ms, "
          f"2D+2D {out['2d_2d']['ms']} ms, 2D+1D+1D with MFMA t {out['2d_1d_1d_mfma_t']['ms']} ms", file=sys.stderr,
          flush=True)
    return out


def update_variants(L, U, torch):
    """16^4 seed 1: iterations and time to theta < 1e-15 over alpha, for the
    first-order update (the paper's) and the exact exponential; and plain
    steepest descent (no Fourier acceleration) at alpha = 0.08."""
    from paper_1206_0675_amd import lgf
    out = []
    for alpha in (0.04, 0.05, 0.0625, 0.07, 0.08, 0.10, 0.12):
        for label, upd in (("first_order", lgf.UPDATE_FIRST_ORDER), ("exp", lgf.UPDATE_EXP)):
            with lgf.Context(MIXED16_DIMS, lib=L, storage=12, poll_every=8, alpha=alpha, update=upd,
                             max_iter=3000) as ctx:
                s, _ = fix_runs(ctx, U, 2, torch)
            out.append({"alpha": alpha, "update": label, "converged": s.status == lgf.OK and s.theta < 1e-15,
                        "iters": s.iter, "seconds": round(s.seconds, 5), "F": s.F})
    with lgf.Context(MIXED16_DIMS, lib=L, storage=12, poll_every=64, accel=lgf.ACCEL_NONE, max_iter=20000) as ctx:
        ctx.load(U)
        s = ctx.fix(raise_on_error=False)
    out.append({"alpha": 0.08, "update": "first_order", "accel": "none", "converged": s.theta < 1e-15,
                "iters": s.iter, "seconds": round(s.seconds, 5), "F": s.F})
    return out


# ---------------------------------------------------------------------------
# CPU (oracle) measurements: run before the GPU is touched
# ---------------------------------------------------------------------------
def omp_threads(n):
    """Set the OpenMP thread count of the oracle's runtime (libgomp) in this
    process; returns the previous count."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(int(n))
    return prev


def cpu_baseline(U, R, dims):
    import oracle
    o = oracle.opts(store12=(R == 12))
    n_a, n_b = 2, 32
    t = time.perf_counter()
    oracle.step(dims, U, n_a, o)
    t_a = time.perf_counter() - t
    t = time.perf_counter()
    oracle.step(dims, U, n_b, o)
    t_b = time.perf_counter() - t
    return {"value": round((n_b - n_a) / (t_b - t_a), 4), "unit": "iters/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle (plain C, OpenMP) on the same {'x'.join(map(str, dims))} lattice, "
                      f"{R}-real: rate = {n_b - n_a} / (t({n_b} updates) - t({n_a} updates)), "
                      f"{t_a + t_b:.1f}s of CPU work"}


def copy_ceiling(torch, mib=1024, reps=5):
    """GB/s (bytes read + written) of a plain device-to-device copy of `mib`
    MiB, best of `reps`, timed with events on torch's stream, which the copy
    runs on: the stream-copy ceiling the kernels are set against."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return {"mib": mib, "gbps": round(2 * n * 8 / (best * 1e-3) / 1e9, 1)}


def oracle_time_to_theta(small, med, big=None, long_run=False):
    import oracle
    nproc = oracle.threads()
    out = {"nproc": nproc}
    try:
        import platform
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), platform.processor())
        out["cpu_model"] = model
    except OSError:
        pass
    cases = [("8^4", SMALL_DIMS, small), ("16^4", MIXED16_DIMS, med)]
    if big is not None:
        cases.append(("x".join(map(str, HEADLINE_DIMS)), HEADLINE_DIMS, big))
    if long_run:
        import synth
        cases.append(("x".join(map(str, LEARNED_DIMS)), LEARNED_DIMS, synth.random_links(LEARNED_DIMS, 3000)))
    for label, dims, U in cases:
        t = time.perf_counter()
        _, it, F, th, ok, _ = oracle.fix(dims, U)
        out[label] = {"threads": nproc, "seconds": round(time.perf_counter() - t, 3), "iters": it, "F": F,
                      "converged": ok}
    prev = omp_threads(1)
    try:
        t = time.perf_counter()
        _, it, F, th, ok, _ = oracle.fix(SMALL_DIMS, small)
        out["8^4_1thread"] = {"threads": 1, "seconds": round(time.perf_counter() - t, 3), "iters": it, "F": F,
                              "converged": ok}
        t = time.perf_counter()
        oracle.step(MIXED16_DIMS, med, 1)
        t1 = time.perf_counter() - t
        t = time.perf_counter()
        oracle.step(MIXED16_DIMS, med, 4)
        t4 = time.perf_counter() - t
        out["16^4_1thread_ms_per_iter"] = round((t4 - t1) / 3 * 1e3, 2)
    finally:
        omp_threads(prev)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", type=int, default=12, choices=[12, 18])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline line (rate and roofline)")
    ap.add_argument("--learned-seeds", type=int, default=4,
                    help="32^3x64 fields (seeds 3000...) for the learned-vs-plain comparison (0: skip)")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="for hardware counters: a few iterations, then one plain device copy of "
                         "--copy-mib MiB (a kernel of known traffic that scales FETCH_SIZE/WRITE_SIZE); no JSON")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--oracle-long", action="store_true",
                    help="also time the oracle's full fix at 32^3x64 (seed 3000, about 25 s of CPU work)")
    ap.add_argument("--batch-sample", action="store_true",
                    help="run only the batch of 64 (one lgf_batch fix, then the lattices one by one) and print "
                         "its JSON; for profiling")
    ap.add_argument("--wilson-sample", action="store_true",
                    help="run only a 32^4 beta 6.0 Wilson-action generation (20 updates of one heatbath and four "
                         "overrelaxation sweeps) and its FP64 gauge fixing; no JSON; for profiling")
    ap.add_argument("--fft-sample", action="store_true",
                    help="run only the 32^4 FFT decomposition study and print its JSON; for profiling")
    ap.add_argument("--gen-workers", type=int, default=min(8, os.cpu_count() or 1),
                    help="worker processes for input generation (started before this program touches the GPU; "
                         "use 1 under a profiler, which sets up the GPU before this program starts)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: "
              "there is no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import synth

    # ---- inputs, generated before this program touches the GPU -------------
    samples = args.pmc_sample or args.batch_sample or args.wilson_sample or args.fft_sample
    extras = not (args.no_extras or samples)
    gw = args.gen_workers
    t = time.time()
    U = None if (args.batch_sample or args.wilson_sample or args.fft_sample) else \
        synth.random_links(HEADLINE_DIMS, args.seed, workers=gw)
    seeds32 = []
    small = med = None
    mixed16 = []
    learned_fields = []
    batch_in = None
    model_path = os.path.join(ROOT, "paper_1206_0675_amd", "models", "learned_step.bin")
    if extras:
        seeds32 = [(args.seed, U)] + [(s, synth.random_links(HEADLINE_DIMS, s, workers=gw)) for s in (2, 3, 4)]
        small = synth.random_links(SMALL_DIMS, 1)
        mixed16 = [(seed, synth.random_links(MIXED16_DIMS, seed, workers=gw)) for seed in (1, 2, 3, 4)]
        med = mixed16[0][1]
        if args.learned_seeds > 0 and os.path.exists(model_path):
            learned_fields = [(seed, synth.random_links(LEARNED_DIMS, seed, workers=gw))
                              for seed in range(3000, 3000 + args.learned_seeds)]
    if extras or args.batch_sample:
        shapes, eps = batch_workload()
        batch_in = (shapes, [synth.random_links(d, 1000 + i, eps=e) for i, (d, e) in enumerate(zip(shapes, eps))])
    print(f"# inputs generated in {time.time() - t:.1f}s", file=sys.stderr, flush=True)

    # ---- CPU: the oracle on this host, before the GPU is touched ----------
    cpu = None
    oracle_ttt = None
    oracle_F8 = None
    if not args.no_cpu_baseline and not samples:
        cpu = cpu_baseline(U, args.storage, HEADLINE_DIMS)
        print(f"# cpu baseline: {cpu['value']} iters/s on {cpu['cores']} threads", file=sys.stderr, flush=True)
        if extras:
            oracle_ttt = oracle_time_to_theta(small, med, U, args.oracle_long)
            oracle_F8 = oracle_ttt["8^4"]["F"]
    elif extras:
        import oracle
        oracle_F8 = oracle.fix(SMALL_DIMS, small)[2]

    import torch

    from paper_1206_0675_amd import lgf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    L = lgf.load_library()
    R = args.storage
    V = vol(HEADLINE_DIMS)
    ab = alg_bytes(V, 8, R)

    if args.pmc_sample:
        with lgf.Context(HEADLINE_DIMS, lib=L, storage=R) as ctx:
            ctx.load(U)
            ctx.step(5)
        n = args.copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"# pmc sample: 5 iterations, then one copy of {args.copy_mib} MiB", file=sys.stderr, flush=True)
        return
    if args.batch_sample:
        print(json.dumps(batch_run(L, batch_in[0], batch_in[1], torch)), flush=True)
        return
    if args.fft_sample:
        print(json.dumps(fft_study_32(L, torch, {})), flush=True)
        return
    if args.wilson_sample:
        with lgf.WilsonGenerator(HEADLINE_DIMS, 6.0, 5001, lib=L) as g:
            g.update(20, 4)
            P = g.plaquette()
            with lgf.Context(HEADLINE_DIMS, lib=L, storage=R, max_iter=100000) as ctx:
                ctx.load_device(g.device_links)
                s = ctx.fix(raise_on_error=False)
        print(f"# wilson sample: P {P:.6f}, {s.iter} iterations, {s.seconds:.3f} s", file=sys.stderr, flush=True)
        return

    # ---- headline: timed iterations, then the profiled pass ---------------
    iters_per_s, t_it, prof, launch_shape = rate_and_kernels(L, HEADLINE_DIMS, U, args.steps, args.warmup, torch,
                                                             repeats=5 if extras else 0, storage=R)
    repeats = launch_shape.pop("repeats", None)
    print(f"# {args.steps} iterations at {t_it * 1e3:.4f} ms", file=sys.stderr, flush=True)
    kernels = kernel_table(prof, ab)
    copy = copy_ceiling(torch)
    dom = kernels["transform_measure"]
    traffic = measured_traffic("transform_measure", HEADLINE_DIMS, R)

    line_extra = {}
    if extras:
        line_extra["per_precision"] = per_precision(L, U, args, torch)
        line_extra["time_to_theta"] = time_to_theta_32(L, seeds32, torch)
        line_extra["small_8"] = small_8(L, small, torch, oracle_F8)
        line_extra["mixed_16"] = mixed_16(L, mixed16, torch)
        line_extra["update_variants"] = update_variants(L, med, torch)
        line_extra["fft_study"] = fft_study_32(L, torch, kernels)
        if learned_fields:
            line_extra["rate_32x32x32x64"] = rate_32x64(L, learned_fields[0][1], args, torch)
            with open(model_path, "rb") as fh:
                blob = fh.read()
            line_extra["learned_vs_plain"] = learned_vs_plain(L, learned_fields, blob, torch)
        blob = None
        if os.path.exists(model_path):
            with open(model_path, "rb") as fh:
                blob = fh.read()
        line_extra["wilson_32"] = wilson_32(L, blob, torch)
        b = batch_run(L, batch_in[0], batch_in[1], torch)
        line_extra["batch"] = b
        print(f"# batch of {b['configs']}: {b['seconds']:.4f} s, {b['configs_per_s']} configs/s, "
              f"{b['aggregate_alg_gbps']} GB/s aggregate, {b['speedup_vs_single']}x one by one", file=sys.stderr,
              flush=True)

    it_bytes = ab["iteration"]
    sb = rewrite_design_bytes(V, 8, R)
    line = {
        "metric": "FA-SD iters/s and time to theta<1e-15 on 32^4 SU(3); HBM GB/s; learned vs plain",
        "value": round(iters_per_s, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_it * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, HEADLINE_DIMS))} SU(3) FA-SD iteration, FP64, {R}-real links, "
                               "alpha 0.08",
                   "dims": list(HEADLINE_DIMS), "storage": R, "seed": args.seed,
                   "generator": "g exp(i eps H) g^dag, plaquette 0.6"},
        "roofline": {"bound": "hbm", "achieved": dom["gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": dom["frac"], "traffic": traffic,
                     "kernel": "transform_measure", "alg_bytes_per_launch": ab["transform_measure"]},
        "iteration_alg_gbps": round(it_bytes / t_it / 1e9, 1),
        "iteration_frac": round(it_bytes / t_it / 1e9 / HBM_PEAK_GBPS, 4),
        "iteration_rewrite_design_frac": round(sb / t_it / 1e9 / HBM_PEAK_GBPS, 4),
        "kernels": kernels,
        "rate_repeats": repeats,
        "copy_ceiling": {**copy, "transform_measure_frac": round(dom["gbps"] / copy["gbps"], 4),
                         "iteration_frac": round(it_bytes / t_it / 1e9 / copy["gbps"], 4)},
        **line_extra,
        "cpu_baseline": cpu,
        "oracle_time_to_theta": oracle_ttt,
        "context": {"paper_c2070_iters_per_s": PAPER_C2070_ITERS_PER_S,
                    "device": torch.cuda.get_device_name(0), "source_digest": source_digest(),
                    "launch_shape": launch_shape},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
