"""Benchmark of the Algorithm 6 hot path on one MI355X.

One step = one full iteration of Algorithm 6 (effective Hamiltonians, pair
update, pair PSD projections, cluster update, multiplier updates, X gradient
step, lattice DFT, momentum-block PSD projections, inverse DFT), with the FP64
diagnostics (Lagrangian bound, energy, feasibility) every ``--lb-every`` steps,
on synthetic input of the benchmark workload, all state resident in HBM.

Default workload: transverse-field Ising ring, N = 384 sites, J = 1, h = 1,
clusters of 3 sites (M = 128 clusters): 127 pair marginals of 64 x 64 and 65
unique 64 x 64 complex momentum blocks per step.

Prints ONE JSON line.  ``value`` = pair PSD projections per second (64 x 64).

The second half of the metric, time to a 1e-6 certified-bound gap with the learned
warm start against the cold start, is measured after the throughput run (object
``warm_start``): a parameter-sweep family (TFI or XXZ ring, N = 64, 2-site clusters,
seeded draws of model, h, J_z) provides solver-generated training states; the network
is trained with the library's kernels; held-out draws are then run cold and warm.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PSD projections/s (2^k×2^k) & time to 1e-6 SDP gap: warm-start vs cold"
# the eigensolver launches: the two projections, or both in one launch where the library fuses them
PROJ_KERNELS = ("pair_projection", "momentum_projection", "projections")
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}  # MI355X vector peaks: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz (f32 x2)


def flops_per_launch(kernel, info):
    """Algorithmic flops of one launch (Golub-Van Loan counts, no Jacobi overhead):
    pair projection 11 n^3 per matrix (9 n^3 eigendecomposition with vectors + 2 n^3
    rebuild); momentum projection 44 n_op^3 per complex block (4x real); the launch that
    runs both ("projections") the sum."""
    if kernel == "pair_projection":
        return 11.0 * info["n"] ** 3 * info["P"]
    if kernel == "momentum_projection":
        return 44.0 * info["n_op"] ** 3 * info["K_unique"]
    if kernel == "projections":
        return flops_per_launch("pair_projection", info) + flops_per_launch("momentum_projection", info)
    raise KeyError(kernel)


def source_digest():
    h = hashlib.sha256()
    for f in ("jacobi.hip", "jacobi_common.h"):  # the eigensolver kernels' sources
        with open(os.path.join(ROOT, "paper_2106_02682_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, precision, launches_bytes=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it is current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    entry = t.get(f"{kernel}/{precision}")
    if not entry or entry.get("source_digest") != source_digest():
        return None
    return entry.get("bytes_per_launch")


def cpu_baseline(workload, seconds):
    """The FP64 oracle (numpy / LAPACK) on this host's cores, on a bounded number of iterations."""
    import numpy as np  # noqa: F401
    from oracle import alg6

    threads = None
    try:
        from threadpoolctl import threadpool_info

        threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=None)
    except Exception:
        pass
    p = alg6.Problem.from_workload(workload)
    s = alg6.initial_state(p)
    s = alg6.step(p, s)  # warm-up
    t0 = time.perf_counter()
    it = 0
    while True:
        s = alg6.step(p, s)
        it += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {
        "value": p.P * it / dt,
        "unit": "projections/s",
        "cores": threads or os.cpu_count(),
        "kind": "oracle",
        "sample": f"{it} oracle iterations of the same workload ({p.P} pair projections each) after 1 warm-up, "
                  f"{dt:.1f} s",
    }


def log(msg):
    """Progress on stderr (the JSON line is the only stdout output)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def warm_start_leg(args):
    """Learned warm start vs cold start on held-out draws of one ring family (see module doc)."""
    import numpy as np
    import torch

    import synth
    from paper_2106_02682_amd import warmstart as ws

    N, L = 64, 2
    near = N // L // 2
    train = synth.family_draws(args.warm_train, N, L, split=0)
    held = synth.family_draws(args.warm_heldout, N, L, split=1)
    t0 = time.perf_counter()
    log(f"warm start: solving {len(train)} training draws for {args.warm_train_iters} iterations")
    X, T = ws.converged_targets(train, args.warm_train_iters, near, log=log)
    t_data = time.perf_counter() - t0
    net = ws.make_network(T.shape[1], max_batch=max(64, args.warm_heldout))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    log(f"warm start: training {args.warm_steps} steps")
    losses = ws.train(net, torch.from_numpy(X).cuda(), T, steps=args.warm_steps, batch=64, lr=2e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"warm start: {len(held)} held-out draws, cold {args.warm_ref} / warm {args.warm_horizon} iterations")
    res = ws.compare(held, net, near, iters=args.warm_horizon, ref_iters=args.warm_ref, every=50, tol=1e-6, log=log)
    net.close()
    out = {
        "family": f"TFI/XXZ ring N={N}, {L}-site clusters (M={N // L}); model, h, Jz from the seeded draws",
        "train_instances": args.warm_train, "train_solver_iters": args.warm_train_iters,
        "train_steps": args.warm_steps, "final_train_loss": losses[-1][1], "data_seconds": t_data,
        "train_seconds": t_train, "heldout": args.warm_heldout, "horizon_iters": args.warm_horizon,
        "reference_iters_cold": args.warm_ref, "predict_seconds": res["predict_seconds"],
        "median_first_gap_cold": float(np.median(res["first_gap_cold"])),
        "median_first_gap_warm": float(np.median(res["first_gap_warm"])),
    }
    for tol in (1e-6, 1e-5):
        r = ws.gap_report(res, tol, args.warm_horizon)
        out[f"gap_{tol:.0e}"] = {k: v for k, v in r.items() if k not in ("tol", "horizon_iters")}
    return out


def c4_leg(args):
    """The batched parameter sweep: 64 seeded instances (TFI or XXZ, N 32..512, clusters of 2..4
    sites, pair blocks 16x16 .. 256x256) stepped together, graph-replayed."""
    import torch

    import synth
    from paper_2106_02682_amd import vemb

    draws = synth.c4_instances(64)
    log(f"c4: creating {len(draws)} problems ({args.precision})")
    probs = [vemb.Problem.from_workload(synth.instance_workload(d, name=f"c4_{i}"), precision=args.precision)
             for i, d in enumerate(draws)]
    P_total = sum(p.info["P"] for p in probs)
    K_total = sum(p.info["K_unique"] for p in probs)
    sizes = {}
    for p in probs:
        sizes[p.info["n"]] = sizes.get(p.info["n"], 0) + p.info["P"]
    with vemb.Batch(probs) as b:
        info = b.info()
        log(f"c4: {P_total} pair and {K_total} momentum blocks per iteration; warm-up {args.warmup}")
        b.step(args.warmup)
        b.sync()
        log(f"c4: timing {args.steps} iterations")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(args.steps)
        b.sync()
        dt = time.perf_counter() - t0
        lbs = b.dual_bounds()
    for p in probs:
        p.close()
    return {
        "metric": METRIC,
        "value": P_total * args.steps / dt,
        "unit": "projections/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": f"batched sweep of 64 seeded ring instances (TFI or XXZ, N 32..512, 2..4-site "
                               f"clusters): {P_total} pair blocks {dict(sorted(sizes.items()))} by size and "
                               f"{K_total} momentum blocks per step, graph-replayed",
                   "precision": args.precision, "size_classes": info["classes"],
                   "launches_per_step": info["launches_per_iteration"]},
        "bounds_finite": bool(all(math.isfinite(x) for x in lbs)),
    }


def dense_leg(args):
    """Dense Algorithm 5 (no translation invariance) on a disordered ring: 120 pair marginals
    16 x 16 and one 256 x 256 dual per iteration (see synth.dense_bench)."""
    import torch

    import synth
    from paper_2106_02682_amd import vemb

    w, fields = synth.dense_bench()
    with vemb.Dense.from_workload(w, fields=fields, precision=args.precision) as g:
        info = g.info
        log(f"dense: {w.name}, {info['Q']} pairs of {info['n']}x{info['n']}, X {info['K']}x{info['K']}")
        g.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        lb = g.dual_bound()
        e, feas = g.primal_energy()
        sweeps = g.last_sweeps()
    return {
        "metric": METRIC,
        "value": info["Q"] * args.steps / dt,
        "unit": "projections/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": f"dense Algorithm 5, TFI ring N={w.extent[0]} J=1 h=1 with random transverse "
                               f"fields U[-0.5,0.5], 2-site clusters: {info['Q']} pair marginals "
                               f"{info['n']}x{info['n']} and one {info['K']}x{info['K']} dual projection per step",
                   "precision": args.precision},
        "max_sweeps_last_step": {"pair": sweeps[0], "x": sweeps[1]},
        "final": {"lb_per_site": lb, "energy_per_site": e, "feas": feas},
    }


def tune_leg(args):
    """Per-family parameter race (tuning.py) on the warm-start ring family (TFI / XXZ, N = 64, 2-site
    clusters): tune (mu = nu, eps) on 4 training draws, then compare the winner with the paper's
    choice on 8 held-out draws (iterations until the certified-bound gap stays below 1e-5 / 1e-6)."""
    import numpy as np

    from paper_2106_02682_amd import tuning

    iters = 30000
    best, table, secs = tuning.tune(tuning.family(4, split=0), iters=iters, every=100, tol=1e-5, log=log)
    log(f"tuning: winner {best} in {secs:.1f} s")
    t0 = time.perf_counter()
    its, lbs = tuning.run(tuning.family(8, split=1), [tuning.PAPER, best], iters, 100, log=log)
    secs_eval = time.perf_counter() - t0

    def summary(sc):
        v = [math.inf if x is None else x for x in sc]
        return {"reached": sum(x is not None for x in sc), "median_iters": float(np.median(v)), "iters": sc}

    out = {"family": "TFI/XXZ ring N=64, 2-site clusters, seeded draws", "candidates": [list(c) for c in tuning.CANDIDATES],
           "winner": list(best), "tuning_table_1e-5": {str(list(k)): v for k, v in table.items()},
           "tuning_seconds": secs, "heldout": 8, "horizon_iters": iters, "heldout_seconds": secs_eval}
    for tol in (1e-5, 1e-6):
        sc = tuning.scores_of(its, lbs, tol)
        out[f"heldout_{tol:.0e}"] = {"paper": summary(sc[0]), "tuned": summary(sc[1])}
    return {"metric": "iterations to the certified-bound gap, tuned vs the paper's (mu, nu, eps)", "value": None,
            "unit": "iterations", "n_gpus": 1, "data": "synthetic", "dtype": "f64",
            "config": {"workload": "parameter race on a ring family"}, "tuning": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--h", type=float, default=1.0)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--workload", choices=["c2b", "c4", "dense", "tune"], default="c2b",
                    help="c2b: the N=384 ring (default); c4: the 64-instance batched sweep; dense: Algorithm 5 "
                         "on a disordered ring; tune: the per-family parameter race")
    ap.add_argument("--lb-every", type=int, default=10)
    ap.add_argument("--prof-every", type=int, default=10, help="time the eigensolver launch on every N-th iteration")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample length (0 disables)")
    ap.add_argument("--warm", type=int, default=1, help="run the learned warm-start leg (0 skips it)")
    ap.add_argument("--warm-train", type=int, default=256)
    ap.add_argument("--warm-train-iters", type=int, default=30000)
    ap.add_argument("--warm-steps", type=int, default=20000)
    ap.add_argument("--warm-heldout", type=int, default=16)
    ap.add_argument("--warm-horizon", type=int, default=30000)
    ap.add_argument("--warm-ref", type=int, default=60000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2106_02682_amd import vemb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "c4":
        print(json.dumps(c4_leg(args)), flush=True)
        return
    if args.workload == "dense":
        print(json.dumps(dense_leg(args)), flush=True)
        return
    if args.workload == "tune":
        print(json.dumps(tune_leg(args)), flush=True)
        return
    w = synth.config_c2(args.h)[1]
    g = vemb.Problem.from_workload(w, precision=args.precision)
    info = g.info
    log(f"throughput: {w.name}, {args.warmup} warm-up + {args.steps} timed steps")
    g.step(args.warmup)
    torch.cuda.synchronize()
    # time the eigensolver launches (the roofline's candidates) with HIP events on every
    # prof_every-th iteration (each timed launch adds two event packets, ~8 us each on the GPU's
    # timeline); the diagnostics are queued on the stream and collected one interval later, so
    # the stream never drains inside the timed region
    g.set_profiling(True, kernels=list(PROJ_KERNELS))
    g.set_profiling_every(args.prof_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb = e = feas = None
    pending = False
    for i in range(args.steps):
        g.step(1)
        if args.lb_every and (i + 1) % args.lb_every == 0:
            if pending:
                lb, e, feas = g.diagnostics_collect()
            g.diagnostics_enqueue()
            pending = True
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if pending:
        lb, e, feas = g.diagnostics_collect()
    prof = g.get_profile()
    sweeps = g.last_sweeps()
    g.close()

    dtype = "f64" if args.precision == "fp64" else "f32"
    cand = {k: prof[k] for k in PROJ_KERNELS if prof[k][1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    ms_total, launches = prof[dom]
    avg_s = ms_total / launches * 1e-3
    achieved = flops_per_launch(dom, info) / avg_s / 1e12
    peak = PEAK_TFLOPS[dtype]
    roofline = {
        "bound": "alu",
        "kernel": dom,
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": measured_traffic(dom, args.precision),
        "avg_launch_ms": avg_s * 1e3,
        "timed_launches": launches,
        "timed_every": args.prof_every,
    }
    out = {
        "metric": METRIC,
        "value": info["P"] * args.steps / dt,
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": f"TFI ring N={w.extent[0]} J=1 h={args.h}, 3-site clusters (M={info['M']}): "
                        f"{info['P']} pair marginals {info['n']}x{info['n']}, {info['K_unique']} unique "
                        f"{info['n_op']}x{info['n_op']} complex momentum blocks per step",
            "precision": args.precision,
            "lb_every": args.lb_every,
        },
        "roofline": roofline,
        "kernels_avg_ms": {k: (v[0] / v[1] if v[1] else None) for k, v in prof.items()},
        "max_sweeps_last_step": {"pair": sweeps[0], "momentum": sweeps[1]},
        "final": {"lb_per_site": lb, "energy_per_site": e, "feas": feas},
    }
    if args.warm:
        out["warm_start"] = warm_start_leg(args)
    if args.cpu_seconds > 0:
        log(f"cpu baseline: the oracle for {args.cpu_seconds} s")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
