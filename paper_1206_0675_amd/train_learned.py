"""Train the learned spectral step on the GPU.

    python -m paper_1206_0675_amd.train_learned [--configs 256] [--rounds 1] [--out DIR]

1. Generate the training fields: seeds 2000, 2001, ... of the seeded
   synthetic generator (16^4, plaquette 0.6), and with --wilson N, N
   Wilson-action fields per beta of --betas from the library's heatbath
   generator (--wilson-dims, 32^4 by default; cold start, --updates updates
   of one heatbath and four overrelaxation sweeps, Philox seeds 7000 + 100 b
   + k), sampled every --wilson-every iterations.
2. Round 0: run the plain FP64 method on each; at every iteration until
   theta < 1e-14, record the band features of Delta and the log factor that
   minimises theta after one update (lgf_linesearch_bands, a golden-section
   search on the GPU).  An update's factors come from the band powers of the
   previous update's spectrum, so each sample pairs the features of iteration
   n - 1 with the target of iteration n.  Train the 16-64-64-16 network on
   these samples with the library's own forward, backward and Adam kernels
   (lgf_mlp_train).
3. Later rounds (--rounds > 1, off by default): collect the same way along
   the trajectories of the learned step with the current network, add them to
   the samples and train again.
4. Write the model blob and a JSON record of the run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1206_0675_amd import lgf  # noqa: E402

MODEL_DIR = os.path.join(HERE, "models")
MODEL_PATH = os.path.join(MODEL_DIR, "learned_step.bin")


def band_mask(dims):
    """Which of the 16 bands hold modes (the definition the library uses)."""
    L = np.array(dims, dtype=np.float64)
    axes = [4.0 * np.sin(np.pi * np.arange(int(n)) / n) ** 2 for n in L]
    p2 = (axes[3][:, None, None, None] + axes[2][None, :, None, None] + axes[1][None, None, :, None]
          + axes[0][None, None, None, :]).ravel()
    pmin = min(4.0 * np.sin(np.pi / n) ** 2 for n in L)
    pmax = sum(a.max() for a in axes)
    nz = p2[p2 > 0]
    b = np.clip(np.floor(16.0 * np.log(nz / pmin) / np.log(pmax / pmin)).astype(int), 0, 15)
    return np.bincount(b, minlength=16) > 0


def generate(dims, seeds, workers=8):
    """The training fields, generated in worker processes.  Call this before
    anything touches the GPU: the workers are started by fork and exec."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import synth
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(synth.random_links, [dims] * len(seeds), seeds))


def generate_wilson(dims, betas, per_beta, updates, lib=None):
    """Wilson-action fields from the GPU generator (cold start)."""
    out = []
    for b, beta in enumerate(betas):
        for k in range(per_beta):
            with lgf.WilsonGenerator(dims, beta, 7000 + 100 * b + k, lib=lib) as g:
                g.update(updates, 4)
                out.append(g.store())
    return out


def collect(dims, fields, every=1, theta_min=1e-14, lib=None, log=print, blob=None, max_iter=200):
    """Samples along the plain trajectories, or along those of the learned
    step with model `blob`.  The factors of an update come from the band
    powers of the previous update's spectrum, so a sample pairs the features
    of iteration n - 1 with the line-search target of iteration n."""
    X, Y = [], []
    mask = band_mask(dims)
    kw = {} if blob is None else {"step": lgf.STEP_LEARNED}
    for k, U in enumerate(fields):
        with lgf.Context(dims, lib=lib, **kw) as c:
            if blob is not None:
                c.set_model(blob)
            c.load(U)
            it, x_prev = 0, None
            while it < max_iter:
                st = c.measure()
                if st.theta < theta_min:
                    break
                x, ls = c.linesearch_bands()
                if x_prev is not None and it % every == 0:
                    X.append(x_prev)
                    Y.append(ls)
                x_prev = x
                c.step(1)
                it += 1
        if log and (k % 64 == 0 or k == len(fields) - 1 or len(fields) <= 64):
            log(f"# collected {len(X)} samples from {k + 1} fields")
    X, Y = np.array(X), np.array(Y)
    M = np.broadcast_to(mask.astype(np.float64), X.shape).copy()
    return X, Y, M


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--configs", type=int, default=256)
    ap.add_argument("--seed0", type=int, default=2000)
    ap.add_argument("--dims", type=int, nargs=4, default=[16, 16, 16, 16])
    ap.add_argument("--every", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--rounds", type=int, default=1)
    ap.add_argument("--wilson", type=int, default=0, help="Wilson-action fields per beta (0: none)")
    ap.add_argument("--betas", type=float, nargs="+", default=[5.8, 6.0, 6.2])
    ap.add_argument("--wilson-dims", type=int, nargs=4, default=[32, 32, 32, 32])
    ap.add_argument("--updates", type=int, default=100)
    ap.add_argument("--wilson-every", type=int, default=8, help="sample every n-th iteration of those runs")
    ap.add_argument("--wilson-max-iter", type=int, default=20000)
    ap.add_argument("--out", default=MODEL_DIR)
    args = ap.parse_args(argv)
    t0 = time.time()
    dims = tuple(args.dims)
    fields = generate(dims, list(range(args.seed0, args.seed0 + args.configs)))
    print(f"# generated {len(fields)} fields in {time.time() - t0:.1f}s", flush=True)
    L = lgf.load_library()
    say = lambda m: print(m, flush=True)    # noqa: E731
    wdims = tuple(args.wilson_dims)
    wfields = generate_wilson(wdims, args.betas, args.wilson, args.updates, lib=L) if args.wilson > 0 else []
    if wfields:
        say(f"# generated {len(wfields)} Wilson-action fields")
    Xs, Ys, Ms, blob, trace, rounds = [], [], [], None, None, []
    for r in range(args.rounds):
        t1 = time.time()
        X, Y, M = collect(dims, fields, args.every, lib=L, log=say, blob=blob)
        Xs.append(X), Ys.append(Y), Ms.append(M)
        if wfields:
            X, Y, M = collect(wdims, wfields, args.wilson_every, lib=L, log=say, blob=blob,
                              max_iter=args.wilson_max_iter)
            Xs.append(X), Ys.append(Y), Ms.append(M)
        X, Y, M = np.concatenate(Xs), np.concatenate(Ys), np.concatenate(Ms)
        t2 = time.time()
        blob, trace = lgf.mlp_train(X, Y, M, steps=args.steps, batch=args.batch, seed=1, lr=args.lr, lib=L)
        pred = lgf.mlp_eval(blob, X, lib=L)
        mse = float(np.sum(M * (pred - Y) ** 2) / np.sum(M))
        rounds.append({"round": r, "samples": int(X.shape[0]), "train_mse": mse,
                       "collect_seconds": round(t2 - t1, 1), "train_seconds": round(time.time() - t2, 2)})
        say(f"# round {r}: {X.shape[0]} samples, train mse {mse:.4g}")
    base = float(np.sum(M * Y ** 2) / np.sum(M))        # the plain step (all log factors 0)
    os.makedirs(args.out, exist_ok=True)
    with open(os.path.join(args.out, "learned_step.bin"), "wb") as f:
        f.write(blob)
    rec = {"dims": list(dims), "seeds": [args.seed0, args.seed0 + args.configs - 1], "every": args.every,
           "wilson": {"dims": list(wdims), "per_beta": args.wilson, "betas": args.betas, "updates": args.updates,
                      "every": args.wilson_every} if args.wilson > 0 else None,
           "samples": int(X.shape[0]), "steps": args.steps, "batch": args.batch, "lr": args.lr,
           "train_mse": rounds[-1]["train_mse"], "plain_step_mse": base, "loss_first": float(trace[0]),
           "loss_last": float(trace[-1]), "rounds": rounds, "seconds": round(time.time() - t0, 1),
           "mean_target_log_s": Y.mean(axis=0).round(4).tolist()}
    with open(os.path.join(args.out, "learned_step.json"), "w") as f:
        json.dump(rec, f, indent=1)
    np.savez_compressed(os.path.join(args.out, "learned_step_samples.npz"), X=X, Y=Y, M=M)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
