"""Learned warm start: training data from the solver, training, and the cold / warm comparison.

Every numerical step runs in the library's kernels (batched Algorithm 6 iterations,
state encoding and decoding, the network's forward / backward / Adam); this module
only sequences the calls and keeps the host-side bookkeeping (which instance is in
which row, when each run reached the gap).

Two convergence rules are reported.
* SDP gap: the first check at which the primal-dual gap of the iterate, (E_p - LB) / |LB|, and the
  equality residual (eq. feasErr) are both at or below the tolerance (E_p the energy of the iterate's
  marginals, LB its Lagrangian bound).
* Bound gap: the Lagrangian bound LB_t of every iterate is a certified lower bound (X PSD).  For an
  instance, LB_ref is the best bound seen over a long cold reference run and the warm run; the relative
  gap of iterate t is (LB_ref - LB_t) / |LB_ref|, and a run has converged when it stays at or below the
  tolerance from then on (every later check).
"""
from __future__ import annotations

import math
import time

import numpy as np

import synth
from . import vemb

HIDDEN = (256, 256, 256)


def _torch():
    import torch

    return torch


def open_problems(draws, precision="fp64"):
    return [vemb.Problem.from_workload(synth.instance_workload(d, name=f"i{k}"), precision=precision)
            for k, d in enumerate(draws)]


def features(draws) -> np.ndarray:
    return np.stack([synth.mlp_features(d) for d in draws]).astype(np.float32)


def encoding_size(L, near):
    """Warm-start encoding length of a ring with clusters of L sites (independent of the ring's size once
    M > 2 near + 1), read from the library on a small ring."""
    with vemb.Problem.from_workload(synth.tfi_ring((2 * near + 2) * L, L, 1.0)) as p:
        return vemb.warm_size(p.h, near)


def converged_targets(draws, iters, near, chunk=64, log=None, precision="fp64"):
    """Solve every draw for `iters` iterations (batched, graph-replayed) and encode its state
    (`near` distances exact).  Returns (features, targets), targets a device float32 tensor whose rows
    are the encodings, zero-padded to the longest one when the draws mix cluster sizes (each problem
    decodes its own prefix)."""
    torch = _torch()
    size = max(encoding_size(L, near) for L in sorted({d["L"] for d in draws}))
    rows = []
    for c0 in range(0, len(draws), chunk):
        part = draws[c0:c0 + chunk]
        probs = open_problems(part, precision)
        try:
            with vemb.Batch(probs) as b:
                done = 0
                while done < iters:
                    k = min(2000, iters - done)
                    b.step(k)
                    b.sync()
                    done += k
                    if log:
                        log(f"training data: instances {c0}..{c0 + len(part) - 1}: {done}/{iters} iterations")
            for p in probs:
                v = torch.zeros(size, dtype=torch.float32, device="cuda")
                vemb.warm_encode(p.h, v[:vemb.warm_size(p.h, near)], near)
                rows.append(v)
            torch.cuda.synchronize()
        finally:
            for p in probs:
                p.close()
    return features(draws), torch.stack(rows)


STD_REL_FLOOR = 1e-3


def make_network(n_out, max_batch=512, tag=0):
    dims = [synth.N_FEATURES, *HIDDEN, n_out]
    return vemb.MLP(dims, synth.mlp_init(dims, tag=tag), max_batch=max_batch)


def train(net, X, T, steps=3000, batch=64, lr=1e-3, lr_min=1e-5, seed=0, log=None):
    """Adam on random minibatches (seeded), cosine learning-rate decay.  X, T device tensors."""
    torch = _torch()
    count = X.shape[0]
    batch = min(batch, count)
    net.fit_normalization(T, STD_REL_FLOOR)
    rng = np.random.default_rng([synth.BASE_SEED, 15, seed])
    losses = []
    for s in range(steps):
        rows = torch.from_numpy(rng.choice(count, size=batch, replace=False).astype(np.int32)).cuda()
        lr_s = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * s / max(1, steps - 1)))
        want = (s % 250 == 0) or s == steps - 1
        loss = net.train_step(X, T, rows=rows, lr=lr_s, want_loss=want)
        if want:
            losses.append((s, loss))
            if log:
                log(f"train step {s}: loss {loss:.3e} lr {lr_s:.2e}")
    return losses


def predict(net, X):
    torch = _torch()
    Y = torch.empty((X.shape[0], net.dims[-1]), dtype=torch.float32, device="cuda")
    net.forward(X, Y)
    return Y


def bound_trajectory(probs, iters, every, warm_vecs=None, near=None, log=None, tag="", far_cold=False):
    """Step a batch of problems `iters` iterations, reading the bounds, energies and feasibility errors
    every `every`.  Returns (its, lbs[len(its), count], secs[len(its)], es, fs) with wall-clock seconds
    since the start (the start includes decoding the warm vectors, if given; the energies are read after
    each time stamp)."""
    torch = _torch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if warm_vecs is not None:
        for p, v in zip(probs, warm_vecs):
            vemb.warm_start(p.h, v, near, far_cold=far_cold)
    its, lbs, secs, es, fs = [], [], [], [], []
    with vemb.Batch(probs) as b:
        done = 0
        while done < iters:
            b.step(every)
            done += every
            lbs.append(b.dual_bounds())
            secs.append(time.perf_counter() - t0)
            e, f = b.primal_energies()
            es.append(e)
            fs.append(f)
            its.append(done)
            if log and done % 2000 == 0:
                log(f"{tag}: {done}/{iters} iterations")
    return np.array(its), np.array(lbs), np.array(secs), np.array(es), np.array(fs)


def first_sdp_gap(its, lbs, es, fs, secs, tol):
    """Per instance: (iterations, seconds) of the first check with (E_p - LB) / |LB| <= tol and
    feasErr <= tol, or (None, None)."""
    gap = np.abs(es - lbs) / np.abs(lbs)
    out = []
    for j in range(lbs.shape[1]):
        ok = np.nonzero((gap[:, j] <= tol) & (fs[:, j] <= tol))[0]
        out.append((int(its[ok[0]]), float(secs[ok[0]])) if len(ok) else (None, None))
    return out


def first_converged(its, lbs, secs, lb_ref, tol):
    """Per instance: (iterations, seconds) from which the gap stays <= tol, or (None, None)."""
    gap = (lb_ref[None, :] - lbs) / np.abs(lb_ref)[None, :]
    out = []
    for j in range(lbs.shape[1]):
        ok = gap[:, j] <= tol
        if not ok[-1]:
            out.append((None, None))
            continue
        k = len(ok) - 1
        while k > 0 and ok[k - 1]:
            k -= 1
        out.append((int(its[k]), float(secs[k])))
    return out


def compare(draws, net, near, iters, ref_iters, every=20, tol=1e-6, log=None, far_cold=False):
    """Cold reference run (ref_iters) and warm run (iters) on the same instances; far_cold starts the
    warm run's offsets beyond `near` cold."""
    torch = _torch()
    probs = open_problems(draws)
    try:
        c_its, c_lbs, c_secs, c_es, c_fs = bound_trajectory(probs, ref_iters, every, log=log, tag="cold")
    finally:
        for p in probs:
            p.close()
    probs = open_problems(draws)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xh = torch.from_numpy(features(draws)).cuda()
        V = predict(net, Xh)
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - t0
        vecs = [V[i, :vemb.warm_size(p.h, near)] for i, p in enumerate(probs)]
        w_its, w_lbs, w_secs, w_es, w_fs = bound_trajectory(probs, iters, every, warm_vecs=vecs, near=near,
                                                            log=log, tag="warm", far_cold=far_cold)
        w_secs = w_secs + t_pred
    finally:
        for p in probs:
            p.close()
    lb_ref = np.maximum(c_lbs.max(axis=0), w_lbs.max(axis=0))
    cold = first_converged(c_its[c_its <= iters], c_lbs[c_its <= iters], c_secs[c_its <= iters], lb_ref, tol)
    warm = first_converged(w_its, w_lbs, w_secs, lb_ref, tol)
    w0 = (lb_ref - w_lbs[0]) / np.abs(lb_ref)
    c0 = (lb_ref - c_lbs[0]) / np.abs(lb_ref)
    return {
        "lb_ref": lb_ref, "cold": cold, "warm": warm, "predict_seconds": t_pred,
        "first_gap_cold": c0, "first_gap_warm": w0,
        "cold_traj": (c_its, c_lbs, c_secs), "warm_traj": (w_its, w_lbs, w_secs),
        "cold_primal": (c_es, c_fs), "warm_primal": (w_es, w_fs),
    }


def gap_report(res, tol, horizon):
    """Counts and medians of (iterations, seconds) to the gap `tol` within `horizon`
    iterations for the cold and warm runs of `compare`; None where the median run never
    reached it (censored)."""
    c_its, c_lbs, c_secs = res["cold_traj"]
    w_its, w_lbs, w_secs = res["warm_traj"]
    kc, kw = c_its <= horizon, w_its <= horizon
    cold = first_converged(c_its[kc], c_lbs[kc], c_secs[kc], res["lb_ref"], tol)
    warm = first_converged(w_its[kw], w_lbs[kw], w_secs[kw], res["lb_ref"], tol)

    def med(pairs, k):
        v = float(np.median([p[k] if p[k] is not None else math.inf for p in pairs]))
        return v if math.isfinite(v) else None

    def sdp(traj, primal, limit):
        its, lbs, secs = traj
        es, fs = primal
        k = its <= limit
        return first_sdp_gap(its[k], lbs[k], es[k], fs[k], secs[k], tol)

    sdp_cold = sdp(res["cold_traj"], res["cold_primal"], c_its[-1])  # the whole cold reference run
    sdp_warm = sdp(res["warm_traj"], res["warm_primal"], horizon)
    return {
        "tol": tol, "horizon_iters": horizon,
        "sdp_gap": {"rule": "first check with (E_p - LB)/|LB| <= tol and feasErr <= tol",
                    "cold_horizon_iters": int(c_its[-1]), "warm_horizon_iters": horizon,
                    "cold_reached": sum(p[0] is not None for p in sdp_cold),
                    "warm_reached": sum(p[0] is not None for p in sdp_warm),
                    "median_iters_cold": med(sdp_cold, 0), "median_iters_warm": med(sdp_warm, 0),
                    "median_seconds_cold": med(sdp_cold, 1), "median_seconds_warm": med(sdp_warm, 1),
                    "iters_cold": [p[0] for p in sdp_cold], "iters_warm": [p[0] for p in sdp_warm]},
        "bound_gap_rule": "the gap (LB_ref - LB_t)/|LB_ref| stays <= tol from this check on",
        "cold_reached": sum(p[0] is not None for p in cold), "warm_reached": sum(p[0] is not None for p in warm),
        "median_iters_cold": med(cold, 0), "median_iters_warm": med(warm, 0),
        "median_seconds_cold": med(cold, 1), "median_seconds_warm": med(warm, 1),
        "iters_cold": [p[0] for p in cold], "iters_warm": [p[0] for p in warm],
    }


