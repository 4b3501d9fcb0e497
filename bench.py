"""Benchmark of the Algorithm 6 hot path on one MI355X.

One step = one full iteration of Algorithm 6 (effective Hamiltonians, pair update, pair PSD
projections, cluster update, multiplier updates, X gradient step, lattice DFT, momentum-block PSD
projections, inverse DFT) over one batch of synthetic input, all state resident in HBM.

Default workload (the headline): the batched parameter sweep -- 64 seeded ring instances (TFI or XXZ,
N ~ U{32..512}, clusters of 2, 3 or 4 sites, h ~ U[0.2, 2], J_z ~ U[0, 2]) stepped together, one launch
per step kernel and per eigensolver size class, replayed from HIP graphs: ~5.8k pair marginals of
16 x 16, 64 x 64 and 256 x 256 and ~3k momentum blocks per step, FP64.  ``value`` = pair PSD
projections per second.  The kernels of every ``--prof-every``-th step are timed with HIP events (those
steps are enqueued directly instead of replayed) and give the ``roofline`` of the dominant kernel and the
figures of the HBM-bound step kernels.  The ``c2b`` object repeats the measurement on the N = 384 ring
with 3-site clusters (127 pair blocks and 65 complex momentum blocks of 64 x 64).

The second half of the metric, time to a 1e-6 gap with the learned warm start against the cold start,
is the ``warm_start`` object (see warm_start_leg).

Other legs: ``--workload c2b`` (the ring alone), ``dense`` (Algorithm 5), ``tune`` (parameter race),
``profile`` (a fixed run for rocprofv3, with a calibration copy) and ``--summarize-traffic`` (turns the
FETCH_SIZE / WRITE_SIZE counter runs of the profile leg into profiles/traffic.json).
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
# the eigensolver launches of one problem: the two projections, or both in one launch where fused
PROJ_KERNELS = ("pair_projection", "momentum_projection", "projections")
# MI355X published peaks: FP64 vector / matrix 78.6 TFLOP/s, FP32 157.3; HBM3E 8 TB/s
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
PEAK_HBM_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2106_02682_amd", "csrc")
# sources whose change makes a kernel's committed traffic counters stale
KERNEL_SOURCES = {
    "projections": ("jacobi.hip", "jacobi_common.h"), "pair_projection": ("jacobi.hip", "jacobi_common.h"),
    "momentum_projection": ("jacobi.hip", "jacobi_common.h"), "pair_jacobi": ("jacobi.hip", "jacobi_common.h"),
    "momentum_jacobi": ("jacobi.hip", "jacobi_common.h"),
    "sign_gemm_real": ("sign_batched.hip", "mfma_tile.h"), "sign_gemm_complex": ("sign_batched.hip", "mfma_tile.h"),
    "sign_load_real": ("sign_batched.hip",), "sign_load_complex": ("sign_batched.hip",),
    "sign_scale_real": ("sign_batched.hip",), "sign_scale_complex": ("sign_batched.hip",),
    "sign_store_real": ("sign_batched.hip",), "sign_store_complex": ("sign_batched.hip",),
    "pair_update": ("step_kernels.hip",), "pair_xstep": ("step_kernels.hip",), "cluster_update": ("step_kernels.hip",),
    "dft_forward": ("step_kernels.hip", "mfma_tile.h"), "dft_inverse": ("step_kernels.hip", "mfma_tile.h"),
}


def flops_per_launch(kernel, info):
    """Algorithmic flops of one launch of a single problem (Golub-Van Loan counts, no Jacobi overhead):
    pair projection 11 n^3 per matrix (9 n^3 eigendecomposition with vectors + 2 n^3 rebuild); momentum
    projection 44 n_op^3 per complex block (4x real); the launch that runs both ("projections") the sum."""
    if kernel == "pair_projection":
        return 11.0 * info["n"] ** 3 * info["P"]
    if kernel == "momentum_projection":
        return 44.0 * info["n_op"] ** 3 * info["K_unique"]
    if kernel == "projections":
        return flops_per_launch("pair_projection", info) + flops_per_launch("momentum_projection", info)
    raise KeyError(kernel)


def sign_gemm_flops(n, count, cplx):
    """One product launch of the sign-function projections over `count` blocks of size n: the
    upper-triangle 64 x 64 output tiles of each block (the product is symmetric / Hermitian and the
    mirror is copied), 2 flops per multiply-add, four real products per complex one."""
    t = n // 64
    return (4.0 if cplx else 1.0) * count * (t * (t + 1) / 2) * 64.0 * 64.0 * n * 2.0


def batch_work(infos):
    """Algorithmic work per launch of every batch kernel, summed over the instances of the launch.

    Bytes (FP64 words x 8) of the memory-bound step kernels, per instance:
      pair_update  per offset: read rho~, Lambda (2 n^2), X_0d (n_op^2), Lambda1, Lambda2 (2 m^2);
                   write rho (n^2), A_1 rho, A_2 rho (2 m^2); plus H_0d (n^2) for each bonded offset
                   (nearest-neighbour rings: d = 1 and M - 1)
      pair_xstep   per offset: read X_0d (n_op^2) and rho's realigned entries (n^2), write X'_0d (n_op^2)
      dft_forward  read X' (M n_op^2), write the K_u complex blocks (2 K_u n_op^2); dft_inverse the reverse
    Flops of the eigensolver launches: 11 n^3 per real pair block, 44 n^3 per complex block (LDS Jacobi
    classes, averaged over the class launches of one step) and sign_gemm_flops for the products of the
    256 x 256 blocks (one launch per product covers every block of the class)."""
    w = {"pair_update": 0.0, "pair_xstep": 0.0, "dft_forward": 0.0, "dft_inverse": 0.0}
    jac = {"pair_jacobi": [0.0, set()], "momentum_jacobi": [0.0, set()]}
    sign = {"sign_gemm_real": {}, "sign_gemm_complex": {}}
    for i in infos:
        n, m, k, P, M, Ku = i["n"], i["m"], i["n_op"], i["P"], i["M"], i["K_unique"]
        bonded = 2 if M > 2 else 1
        w["pair_update"] += 8.0 * (P * (3 * n * n + k * k + 4 * m * m) + bonded * n * n)
        w["pair_xstep"] += 8.0 * P * (2 * k * k + n * n)
        w["dft_forward"] += 8.0 * (M + 2 * Ku) * k * k
        w["dft_inverse"] += 8.0 * (M + 2 * Ku) * k * k
        if n > 64:  # 256 x 256 blocks: sign-function products in every precision
            sign["sign_gemm_real"][n] = sign["sign_gemm_real"].get(n, 0) + P
        else:
            jac["pair_jacobi"][0] += 11.0 * n ** 3 * P
            jac["pair_jacobi"][1].add(n)
        if k > 64:
            sign["sign_gemm_complex"][k] = sign["sign_gemm_complex"].get(k, 0) + Ku
        else:
            jac["momentum_jacobi"][0] += 44.0 * k ** 3 * Ku
            jac["momentum_jacobi"][1].add(k)
    out = {name: ("hbm", b) for name, b in w.items()}
    for name, (f, classes) in jac.items():
        if classes:
            out[name] = ("alu", f / len(classes))
    for name, by_n in sign.items():
        if by_n:
            f = sum(sign_gemm_flops(n, c, name.endswith("complex")) for n, c in by_n.items())
            out[name] = ("mfma", f / len(by_n))
    return out


def source_digest(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, ("jacobi.hip", "jacobi_common.h")):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel, precision):
    """Calibrated HBM bytes per launch from the committed rocprofv3 counter summary, if current."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    entry = t.get(f"{workload}/{kernel}/{precision}")
    if not entry or entry.get("source_digest") != source_digest(kernel):
        return None
    return entry.get("bytes_per_launch")


def roofline_entry(kernel, bound, work, ms_total, launches, dtype, workload, precision):
    avg_s = ms_total / launches * 1e-3
    if bound == "hbm":
        achieved, peak, unit = work / avg_s / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        achieved, peak, unit = work / avg_s / 1e12, PEAK_TFLOPS[dtype], "TFLOP/s"
    return {"bound": bound, "kernel": kernel, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": measured_traffic(workload, kernel, precision),
            "work_per_launch": work, "avg_launch_ms": avg_s * 1e3, "timed_launches": launches}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_steps(args):
    """Worker task: build one oracle problem (untimed), one warm-up step, then `iters` timed steps with one
    BLAS thread.  Returns (process id, pair projections done, seconds)."""
    w, iters = args
    from threadpoolctl import threadpool_limits

    from oracle import alg6

    with threadpool_limits(1):
        p = alg6.Problem.from_workload(w)
        s = alg6.step(p, alg6.initial_state(p))
        t0 = time.perf_counter()
        for _ in range(iters):
            s = alg6.step(p, s)
        dt = time.perf_counter() - t0
    return os.getpid(), p.P * iters, dt


def cpu_baseline(workloads, seconds, pool_workers):
    """The FP64 oracle (numpy / LAPACK) on this host, on a bounded sample of the workload.

    all cores: a process pool (fork, one BLAS thread per worker) runs one oracle iteration of every
    instance; the parallel time is the largest per-worker sum of iteration times (problem set-up and one
    warm-up iteration per instance excluded).  single core: the instances in order, one BLAS thread,
    one timed iteration each, until `seconds` have passed.  Runs before the GPU is touched."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import alg6

    t_wall = time.perf_counter()
    with mp.get_context("fork").Pool(pool_workers) as pool:
        res = pool.map(_oracle_steps, [(w, 1) for w in workloads], chunksize=1)
    per_pid = {}
    for pid, _, dt in res:
        per_pid[pid] = per_pid.get(pid, 0.0) + dt
    par_s = max(per_pid.values())
    proj = sum(r[1] for r in res)
    pool_wall = time.perf_counter() - t_wall
    done, dt_single = 0, 0.0
    with threadpool_limits(1):
        for w in workloads:
            p = alg6.Problem.from_workload(w)
            s = alg6.step(p, alg6.initial_state(p))
            t0 = time.perf_counter()
            alg6.step(p, s)
            dt_single += time.perf_counter() - t0
            done += p.P
            if dt_single >= seconds:
                break
    return {
        "value": proj / par_s, "unit": "projections/s", "cores": len(per_pid), "kind": "oracle",
        "sample": f"one oracle iteration of each of the {len(workloads)} instances ({proj} pair projections) in a "
                  f"pool of {pool_workers} processes with one BLAS thread each: {par_s:.2f} s of iteration time on "
                  f"the busiest worker ({pool_wall:.1f} s wall with set-up and one warm-up iteration each)",
        "cpu_model": cpu_model(),
        "single_core": {"value": done / dt_single, "unit": "projections/s", "cores": 1,
                        "sample": f"one oracle iteration each of the first instances in order, {done} pair "
                                  f"projections in {dt_single:.1f} s, one BLAS thread"},
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

    from paper_2106_02682_amd import vemb

    if args.warm_family == "cross":
        # one network for rings of 32..512 sites and clusters of the sizes in --warm-ls (k = 2L an input);
        # encodings of the `near` nearest distances exact and the rest averaged, so their size does not
        # depend on N
        near = args.warm_near
        Ls = tuple(int(x) for x in args.warm_ls.split(","))
        train = synth.cross_draws(args.warm_train, split=0, Ls=Ls)
        held = synth.cross_draws(args.warm_heldout, split=1, Ls=Ls)
        family = (f"TFI/XXZ rings, N ~ U{{32..512}}, clusters of {Ls} sites alternating, model, h, Jz from the "
                  f"seeded draws; one network, encodings with {near} exact distances"
                  + (", shorter targets zero-padded to the longest" if len(Ls) > 1 else ""))
    else:
        N, L = 64, 2
        near = N // L // 2
        train = synth.family_draws(args.warm_train, N, L, split=0)
        held = synth.family_draws(args.warm_heldout, N, L, split=1)
        family = f"TFI/XXZ ring N={N}, {L}-site clusters (M={N // L}); model, h, Jz from the seeded draws"
    t0 = time.perf_counter()
    log(f"warm start: solving {len(train)} training draws for {args.warm_train_iters} iterations "
        f"({args.warm_data_precision})")
    X, T = ws.converged_targets(train, args.warm_train_iters, near, log=log, precision=args.warm_data_precision)
    t_data = time.perf_counter() - t0
    net = ws.make_network(T.shape[1], max_batch=max(64, args.warm_heldout))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    log(f"warm start: training {args.warm_steps} steps")
    losses = ws.train(net, torch.from_numpy(X).cuda(), T, steps=args.warm_steps, batch=64, lr=2e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"warm start: {len(held)} held-out draws, cold {args.warm_ref} / warm {args.warm_horizon} iterations")
    res = ws.compare(held, net, near, iters=args.warm_horizon, ref_iters=args.warm_ref, every=50, tol=1e-6, log=log,
                     far_cold=bool(args.warm_far_cold))
    net.close()
    out = {
        "family": family, "outputs": int(T.shape[1]), "train_data_precision": args.warm_data_precision,
        "far_offsets": "cold" if args.warm_far_cold else "far slot",
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
    """The headline: 64 seeded instances (TFI or XXZ rings, N 32..512, clusters of 2..4 sites, pair blocks
    16 x 16 .. 256 x 256) stepped together, graph-replayed; kernels of every prof_every-th step timed."""
    import torch

    import synth
    from paper_2106_02682_amd import vemb

    draws = synth.c4_instances(64)
    log(f"c4: creating {len(draws)} problems ({args.precision})")
    probs = [vemb.Problem.from_workload(synth.instance_workload(d, name=f"c4_{i}"), precision=args.precision)
             for i, d in enumerate(draws)]
    infos = [dict(p.info, precision=args.precision) for p in probs]
    P_total = sum(i["P"] for i in infos)
    K_total = sum(i["K_unique"] for i in infos)
    sizes = {}
    for i in infos:
        sizes[i["n"]] = sizes.get(i["n"], 0) + i["P"]
    dtype = "f64" if args.precision == "fp64" else "f32"
    with vemb.Batch(probs) as b:
        info = b.info()
        log(f"c4: {P_total} pair and {K_total} momentum blocks per step; warm-up {args.warmup}")
        b.step(args.warmup)
        b.sync()
        b.set_profiling(args.prof_every)
        log(f"c4: timing {args.steps} steps (kernels of every {args.prof_every}-th step timed)")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(args.steps)
        b.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = b.get_profile()
        lbs, status = b.dual_bounds(check=False)
        e, feas = b.primal_energies()
    for p in probs:
        p.close()
    work = batch_work(infos)
    kernels = {}
    for k, (bound, wk) in work.items():
        ms, n = prof.get(k, (0.0, 0))
        if n > 0:
            kernels[k] = roofline_entry(k, bound, wk, ms, n, dtype, "c4", args.precision)
            kernels[k]["ms_per_step"] = ms / max(1, math.ceil(args.steps / args.prof_every))
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    out = {
        "metric": METRIC,
        "value": P_total * args.steps / dt,
        "unit": "projections/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"batched sweep of 64 seeded ring instances (TFI or XXZ, N 32..512, 2..4-site "
                               f"clusters): {P_total} pair blocks {dict(sorted(sizes.items()))} by size and "
                               f"{K_total} momentum blocks per step, graph-replayed",
                   "precision": args.precision, "size_classes": info["classes"],
                   "launches_per_step": info["launches_per_iteration"], "timed_every": args.prof_every},
        "roofline": kernels[dom],
        "kernel_rooflines": kernels,
        "final": {"bounds_finite": bool(all(math.isfinite(x) for x in lbs)), "status_ok": int(sum(s == 0 for s in status)),
                  "median_lb_per_site": float(sorted(lbs)[len(lbs) // 2]), "max_feas": float(max(feas))},
    }
    return out, [synth.instance_workload(d, name=f"c4_{i}") for i, d in enumerate(draws)]


def c2b_leg(args):
    """The N = 384 ring, 3-site clusters: 127 pair blocks and 65 complex momentum blocks of 64 x 64 per step,
    diagnostics queued every lb_every steps, the eigensolver launch timed on every prof_every-th step."""
    import torch

    import synth
    from paper_2106_02682_amd import vemb

    w = synth.config_c2(args.h)[1]
    g = vemb.Problem.from_workload(w, precision=args.precision)
    info = g.info
    steps = args.c2b_steps
    log(f"c2b: {w.name}, {args.warmup} warm-up + {steps} timed steps")
    g.step(args.warmup)
    torch.cuda.synchronize()
    # time the eigensolver launches with HIP events on every prof_every-th iteration (each timed launch
    # adds two event packets to the GPU's timeline); the diagnostics are queued on the stream and
    # collected one interval later, so the stream never drains inside the timed region
    g.set_profiling(True, kernels=list(PROJ_KERNELS))
    g.set_profiling_every(args.prof_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb = e = feas = None
    pending = False
    for i in range(steps):
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
    roof = roofline_entry(dom, "alu", flops_per_launch(dom, info), cand[dom][0], cand[dom][1], dtype, "c2b",
                          args.precision)
    return {
        "value": info["P"] * steps / dt, "unit": "projections/s", "steps": steps, "ms_per_step": dt / steps * 1e3,
        "dtype": dtype,
        "workload": f"TFI ring N={w.extent[0]} J=1 h={args.h}, 3-site clusters (M={info['M']}): {info['P']} pair "
                    f"marginals {info['n']}x{info['n']}, {info['K_unique']} unique {info['n_op']}x{info['n_op']} "
                    f"complex momentum blocks per step; diagnostics every {args.lb_every} steps",
        "roofline": roof,
        "kernels_avg_ms": {k: (v[0] / v[1] if v[1] else None) for k, v in prof.items()},
        "max_sweeps_last_step": {"pair": sweeps[0], "momentum": sweeps[1]},
        "final": {"lb_per_site": lb, "energy_per_site": e, "feas": feas},
    }, w


def precision_leg(args):
    """FP64 against MIXED (FP32 eigensolves: Jacobi sweeps, matrix-core rebuilds and sign-function products;
    FP64 state and diagnostics) on the batched sweep, the N = 384 ring and the 16 x 16 torus with 2 x 2
    clusters: ms per step of each, timed like the headline (warm-up, then synchronised steps)."""
    import torch

    import synth
    from paper_2106_02682_amd import vemb

    def time_problem(w, prec, steps):
        with vemb.Problem.from_workload(w, precision=prec) as g:
            g.step(args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / steps * 1e3, g.info["P"]

    def time_batch(prec, steps):
        probs = [vemb.Problem.from_workload(synth.instance_workload(d, name=f"c4_{i}"), precision=prec)
                 for i, d in enumerate(synth.c4_instances(64))]
        P = sum(p.info["P"] for p in probs)
        with vemb.Batch(probs) as b:
            b.step(args.warmup)
            b.sync()
            t0 = time.perf_counter()
            b.step(steps)
            b.sync()
            dt = (time.perf_counter() - t0) / steps * 1e3
        for p in probs:
            p.close()
        return dt, P

    out = {}
    log("precision modes: batched sweep in MIXED")
    ms, P = time_batch("mixed", args.steps)
    out["c4"] = {"mixed_ms_per_step": ms, "mixed_projections_per_s": P / ms * 1e3}
    for name, w, steps in (("c2b", synth.config_c2(args.h)[1], 300), ("c3b", synth.config_c3()[1], 20)):
        log(f"precision modes: {w.name}")
        m64, P = time_problem(w, "fp64", steps)
        m32, _ = time_problem(w, "mixed", steps)
        out[name] = {"fp64_ms_per_step": m64, "mixed_ms_per_step": m32, "speedup": m64 / m32,
                     "pair_blocks": P}
    return out


def profile_leg(args):
    """A fixed run for rocprofv3 (kernel traces and counters): the workload's steps after a warm-up, then one
    plain device-to-device copy of 256 MiB (the HIP runtime's copy kernel) whose FETCH_SIZE / WRITE_SIZE
    readings calibrate the byte counters."""
    import torch

    import synth
    from paper_2106_02682_amd import vemb

    if args.profile_workload == "c4":
        probs = [vemb.Problem.from_workload(synth.instance_workload(d, name=f"c4_{i}"), precision=args.precision)
                 for i, d in enumerate(synth.c4_instances(64))]
        with vemb.Batch(probs) as b:
            b.step(args.warmup)
            b.sync()
            print(f"profile: c4 {args.precision}, {args.warmup} warm-up steps done", flush=True)
            b.step(args.steps)
            b.sync()
            print(f"profile: c4 {args.steps} steps done", flush=True)
        for p in probs:
            p.close()
    else:
        w = {"c2b": lambda: synth.config_c2(1.0)[1], "c3a": lambda: synth.config_c3()[0],
             "c3b": lambda: synth.config_c3()[1]}[args.profile_workload]()
        with vemb.Problem.from_workload(w, precision=args.precision) as g:
            g.step(args.warmup)
            torch.cuda.synchronize()
            print(f"profile: {w.name} {args.precision}, {args.warmup} warm-up steps done", flush=True)
            g.step(args.steps)
            torch.cuda.synchronize()
            print(f"profile: {args.steps} steps done", flush=True)
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(f"profile: calibration copy of {COPY_BYTES} bytes done", flush=True)


COPY_BYTES = 256 << 20
# kernel name patterns of the iteration kernels (FP64 instantiations) in rocprofv3's CSV output
TRAFFIC_KERNELS = [
    ("momentum_projection", r"jacobi_kernel<vemb::cplx<double>, 64, 0, true, \d+, vemb::\(anonymous namespace\)::MomentumPolicy"),
    ("pair_projection", r"jacobi_kernel<double, 64, 0, true, \d+, vemb::\(anonymous namespace\)::PairPolicy"),
    ("projections", r"fused_projection_kernel<\d+, double>"),
    ("pair_update", r"pair_update_(kernel|batched)"), ("pair_xstep", r"pair_xstep_(kernel|batched)"),
    ("cluster_update", r"cluster_update_(kernel|batched)"),
    ("dft_forward", r"dft_mfma_kernel<true>|dft_forward_batched"),
    ("dft_inverse", r"dft_mfma_kernel<false>|dft_inverse_batched"),
    ("sign_gemm_real", r"sign_gemm_kernel<double>"), ("sign_gemm_complex", r"sign_gemm_kernel<vemb::cplx<double> >"),
    ("sign_load_real", r"sign_load_kernel<double,"), ("sign_load_complex", r"sign_load_kernel<vemb::cplx<double>,"),
    ("sign_scale_real", r"sign_scale_kernel<double,"), ("sign_scale_complex", r"sign_scale_kernel<vemb::cplx<double>,"),
    ("sign_store_real", r"sign_store_kernel<double,"), ("sign_store_complex", r"sign_store_kernel<vemb::cplx<double>,"),
    ("pair_jacobi", r"jacobi_kernel<double, \d+, 0, true, \d+, vemb::\(anonymous namespace\)::BatchedPairPolicy"),
    ("momentum_jacobi", r"jacobi_kernel<vemb::cplx<double>, \d+, 0, true, \d+, vemb::\(anonymous namespace\)::BatchedMomentumPolicy"),
]


def summarize_traffic(workload, precision, fetch_dir, write_dir):
    """Calibrated HBM bytes per launch from two rocprofv3 counter runs of the profile leg (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), each scaled by the same counter's reading for the calibration copy; written
    to profiles/traffic.json (tied to each kernel's source digest) and profiles/traffic_<workload>_<prec>.md."""
    import csv
    import re

    def rows(d, counter):
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    with open(os.path.join(root, f)) as fh:
                        return [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
        raise FileNotFoundError(f"no counter_collection.csv under {d}")

    def calib(rs):
        # the HIP runtime's device-to-device copy kernel of the 256 MiB copy: the largest grid of that name
        # (torch's fill of the source, an elementwise kernel, reads nothing and is not a calibration)
        copies = [r for r in rs if "copyBuffer" in r["Kernel_Name"]]
        return float(max(copies, key=lambda r: int(r["Grid_Size"]))["Counter_Value"])

    def mean(rs, pat):
        v = [float(r["Counter_Value"]) for r in rs if re.search(pat, r["Kernel_Name"])]
        return (sum(v) / len(v) if v else None), len(v)

    F, W = rows(fetch_dir, "FETCH_SIZE"), rows(write_dir, "WRITE_SIZE")
    copy_kib = COPY_BYTES / 1024
    fF, fW = copy_kib / calib(F), copy_kib / calib(W)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            out = json.load(fh)
    except (OSError, ValueError):
        out = {}
    cmd = (f"cd /tmp && timeout -s KILL 120 rocprofv3 --pmc {{}} -d <out> -o run --output-format csv -- python3 "
           f"/root/repo/bench.py --workload profile --profile-workload {workload} --precision {precision} "
           f"--steps 4 --warmup 2")
    out[f"calibration/{workload}/{precision}"] = {
        "copy_bytes": COPY_BYTES, "fetch_factor": fF, "write_factor": fW,
        "commands": [cmd.format("FETCH_SIZE"), cmd.format("WRITE_SIZE")]}
    lines = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated HBM MB / launch |",
             "|---|---|---|---|---|"]
    for name, pat in TRAFFIC_KERNELS:
        (f, nf), (w, _) = mean(F, pat), mean(W, pat)
        if f is None or w is None:
            continue
        b = (f * fF + w * fW) * 1024
        out[f"{workload}/{name}/{precision}"] = {"bytes_per_launch": b, "fetch_kib": f, "write_kib": w,
                                                 "source_digest": source_digest(name), "dispatches": nf}
        lines.append(f"| {name} | {nf} | {f:.1f} | {w:.1f} | {b / 1e6:.2f} |")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    md = [f"# HBM traffic per launch, workload {workload} ({precision})", "",
          f"Counters: `{cmd.format('FETCH_SIZE')}` and `{cmd.format('WRITE_SIZE')}` (one counter per run).", "",
          f"Calibration: the plain 256 MiB device copy at the end of the run reads FETCH_SIZE {calib(F):.0f} KiB and "
          f"WRITE_SIZE {calib(W):.0f} KiB against {copy_kib:.0f} KiB moved: factors {fF:.3f} (fetch) and {fW:.3f} "
          f"(write) are applied below.", ""] + lines + [
          "", f"Summarised by `python bench.py --summarize-traffic <fetch out> <write out> --profile-workload "
              f"{workload} --precision {precision}`; each entry of profiles/traffic.json carries the digest of its "
              f"kernel's sources and is ignored once they change."]
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


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


def summarize_stats(stats_dir, title, command, out_name):
    """profiles/<out_name>.md from the kernel statistics CSV of a `rocprofv3 --kernel-trace --stats` run:
    calls, average / min / max microseconds and share of every kernel (the top 25 by total time)."""
    import csv

    path = None
    for root, _, files in os.walk(stats_dir):
        for f in files:
            if f.endswith("kernel_stats.csv"):
                path = os.path.join(root, f)
    if path is None:
        raise FileNotFoundError(f"no kernel_stats.csv under {stats_dir}")
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics: {title}", "", f"Command: `{command}`", "",
             "| kernel | calls | average µs | min µs | max µs | share % |", "|---|---|---|---|---|---|"]
    for r in rows[:25]:
        name = r["Name"].replace("|", "\\|")
        if len(name) > 150:
            name = name[:147] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    with open(os.path.join(ROOT, "profiles", f"{out_name}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_counters(counter_dirs, title, commands, out_name, kernels):
    """profiles/<out_name>.md from `rocprofv3 --pmc` runs: the average of each counter per dispatch for the
    kernels named by the (label, regex) pairs, plus ratios the design notes use."""
    import csv
    import re

    vals = {}
    for d in counter_dirs:
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    with open(os.path.join(root, f)) as fh:
                        for r in csv.DictReader(fh):
                            for label, pat in kernels:
                                if re.search(pat, r["Kernel_Name"]):
                                    vals.setdefault((label, r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    counters = sorted({c for _, c in vals})
    labels = [k for k, _ in kernels]
    lines = [f"# Hardware counters per dispatch: {title}", "", "Commands (one pass each):", ""]
    lines += [f"* `{c}`" for c in commands]
    lines += ["", "| counter | " + " | ".join(labels) + " |", "|---|" + "---|" * len(labels)]
    for c in counters:
        row = []
        for k in labels:
            v = vals.get((k, c))
            row.append(f"{sum(v) / len(v):.4g}" if v else "")
        lines.append(f"| {c} | " + " | ".join(row) + " |")
    with open(os.path.join(ROOT, "profiles", f"{out_name}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--c2b-steps", type=int, default=500, help="timed steps of the c2b object")
    ap.add_argument("--h", type=float, default=1.0)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--workload", choices=["c4", "c2b", "dense", "tune", "profile", "warm"], default="c4",
                    help="c4: the 64-instance batched sweep (default, with the c2b object); c2b: the N=384 ring alone; "
                         "dense: Algorithm 5 on a disordered ring; tune: the per-family parameter race; profile: a "
                         "fixed run for rocprofv3; warm: the learned warm-start leg alone")
    ap.add_argument("--profile-workload", choices=["c4", "c2b", "c3a", "c3b"], default="c4")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-stats", nargs=4, metavar=("STATS_DIR", "TITLE", "COMMAND", "OUT_NAME"),
                    help="write profiles/OUT_NAME.md from a rocprofv3 --stats run")
    ap.add_argument("--lb-every", type=int, default=10)
    ap.add_argument("--prof-every", type=int, default=5, help="time the kernels of every N-th step")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="single-core oracle sample length (0 disables "
                                                                    "the CPU baseline)")
    ap.add_argument("--cpu-workers", type=int, default=16, help="processes of the all-cores oracle baseline")
    ap.add_argument("--c2b", type=int, default=1, help="add the c2b object to the c4 line (0 skips it)")
    ap.add_argument("--mixed", type=int, default=1, help="add the FP64-vs-MIXED timings to the c4 line (0 skips)")
    ap.add_argument("--warm", type=int, default=1, help="run the learned warm-start leg (0 skips it)")
    ap.add_argument("--warm-train", type=int, default=256)
    ap.add_argument("--warm-train-iters", type=int, default=30000)
    ap.add_argument("--warm-steps", type=int, default=20000)
    ap.add_argument("--warm-heldout", type=int, default=16)
    ap.add_argument("--warm-horizon", type=int, default=30000)
    ap.add_argument("--warm-ref", type=int, default=60000)
    ap.add_argument("--warm-family", choices=("ring64", "cross"), default="ring64",
                    help="ring64: the N=64, 2-site family; cross: rings of 32..512 sites, 2- and 3-site clusters")
    ap.add_argument("--warm-data-precision", choices=("fp64", "mixed"), default="fp64",
                    help="precision of the solves that produce the training states")
    ap.add_argument("--warm-ls", default="2,3", help="cluster sizes of the cross family")
    ap.add_argument("--warm-near", type=int, default=3, help="exact distances of the cross family's encoding")
    ap.add_argument("--warm-far-cold", type=int, default=0,
                    help="1: the warm start's offsets beyond the exact distances start cold (else the far slot)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.summarize_traffic:
        summarize_traffic(args.profile_workload, args.precision, *args.summarize_traffic)
        return
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats)
        return

    import synth

    # the oracle baseline runs first, in a process that has not touched the GPU (its pool forks)
    cpu = None
    if args.workload in ("c4", "c2b") and args.cpu_seconds > 0:
        workers = max(1, min(args.cpu_workers, len(os.sched_getaffinity(0))))
        wl = ([synth.instance_workload(d, name=f"c4_{i}") for i, d in enumerate(synth.c4_instances(64))]
              if args.workload == "c4" else [synth.config_c2(args.h)[1]] * workers)
        log(f"cpu baseline: the oracle on {len(wl)} instances, {workers} processes, then one core for "
            f"{args.cpu_seconds} s")
        cpu = cpu_baseline(wl, args.cpu_seconds, workers)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "profile":
        profile_leg(args)
        return
    if args.workload == "dense":
        print(json.dumps(dense_leg(args)), flush=True)
        return
    if args.workload == "tune":
        print(json.dumps(tune_leg(args)), flush=True)
        return
    if args.workload == "warm":
        print(json.dumps({"warm_start": warm_start_leg(args)}), flush=True)
        return
    if args.workload == "c4":
        out, _ = c4_leg(args)
        if args.c2b:
            out["c2b"], _ = c2b_leg(args)
        if args.mixed and args.precision == "fp64":
            out["precision_modes"] = precision_leg(args)
            out["precision_modes"]["c4"]["fp64_ms_per_step"] = out["ms_per_step"]
            out["precision_modes"]["c4"]["speedup"] = out["ms_per_step"] / out["precision_modes"]["c4"]["mixed_ms_per_step"]
    else:
        c2, _ = c2b_leg(args)
        out = {"metric": METRIC, "value": c2["value"], "unit": "projections/s", "n_gpus": 1, "steps": c2["steps"],
               "warmup": args.warmup, "ms_per_step": c2["ms_per_step"], "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": c2["dtype"], "data": "synthetic",
               "config": {"workload": c2["workload"], "precision": args.precision, "lb_every": args.lb_every},
               "roofline": c2["roofline"], "kernels_avg_ms": c2["kernels_avg_ms"],
               "max_sweeps_last_step": c2["max_sweeps_last_step"], "final": c2["final"]}
    if args.warm:
        out["warm_start"] = warm_start_leg(args)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
