"""Per-family choice of the penalty and step parameters (mu = nu, eps) of Algorithm 6.

Section 4 fixes mu = nu = 10, eps = 2 for every problem and remarks that tuning them per problem
and cluster choice could smooth convergence.  For a family of problems (a parameter sweep: one
lattice and cluster choice, several couplings), every candidate runs on a few tuning instances,
all together in one graph-replayed batch, and the certified Lagrangian bound of every run is read
every `every` iterations.  For each instance LB_ref is the best bound any run reached; a run's
score is the first check from which its relative gap (LB_ref - LB_t) / |LB_ref| stays at or below
the tolerance (never: infinite).  The candidate with the smallest median score wins; ties go to the
smaller mean of the finite scores, then to the paper's choice.  A candidate whose iterates stop
being finite ranks last on that instance.

Every numerical step runs in the library's kernels; this module sequences the calls and keeps the
bookkeeping.
"""
from __future__ import annotations

import math
import time

import numpy as np

import synth
from . import vemb

PAPER = (10.0, 2.0)
# (mu = nu, eps): the paper's choice and scalings of it with eps / mu in {0.2, 0.4}
CANDIDATES = ((5.0, 1.0), (10.0, 2.0), (10.0, 4.0), (20.0, 4.0), (20.0, 8.0), (40.0, 8.0), (40.0, 16.0))


def converged_index(gaps: np.ndarray, tol: float):
    """Index of the first check from which every later gap is <= tol (None if the last is not)."""
    ok = np.isfinite(gaps) & (gaps <= tol)
    if len(ok) == 0 or not ok[-1]:
        return None
    k = len(ok) - 1
    while k > 0 and ok[k - 1]:
        k -= 1
    return k


def select(scores: dict):
    """scores: candidate -> list of iterations to the gap (None = never), one per instance."""
    def key(c):
        v = np.array([math.inf if x is None else float(x) for x in scores[c]])
        finite = v[np.isfinite(v)]
        return (float(np.median(v)), float(finite.mean()) if len(finite) else math.inf, 0 if c == PAPER else 1)

    return min(scores, key=key)


def run(workloads, candidates, iters: int, every: int, precision: str = "fp64", log=None):
    """Every (instance, candidate) pair as one batch.  Returns (its, lbs[checks, instances, candidates])
    with non-finite bounds (diverged runs) as -inf."""
    probs = []
    try:
        for w in workloads:
            for mu, eps in candidates:
                probs.append(vemb.Problem.from_workload(w, mu=mu, nu=mu, eps=eps, precision=precision))
        its, rows = [], []
        with vemb.Batch(probs) as b:
            done = 0
            while done < iters:
                b.step(every)
                done += every
                lb, status = b.dual_bounds(check=False)
                lb = np.where((np.asarray(status) == 0) & np.isfinite(lb), lb, -np.inf)
                rows.append(lb.reshape(len(workloads), len(candidates)))
                its.append(done)
                if log and done % 10000 == 0:
                    log(f"parameter race: {done}/{iters} iterations")
        return np.array(its), np.stack(rows)
    finally:
        for p in probs:
            p.close()


def scores_of(its, lbs, tol):
    """candidate index -> iterations to the gap per instance, LB_ref the best bound of any run."""
    ref = np.max(np.where(np.isfinite(lbs), lbs, -np.inf), axis=(0, 2))  # per instance
    out = {}
    for c in range(lbs.shape[2]):
        per = []
        for i in range(lbs.shape[1]):
            gaps = (ref[i] - lbs[:, i, c]) / abs(ref[i])
            k = converged_index(gaps, tol)
            per.append(None if k is None else int(its[k]))
        out[c] = per
    return out


def tune(workloads, candidates=CANDIDATES, iters: int = 6000, every: int = 50, tol: float = 1e-6,
         precision: str = "fp64", log=None):
    """Returns (best (mu, eps), {candidate: iterations per instance}, seconds)."""
    t0 = time.perf_counter()
    its, lbs = run(workloads, candidates, iters, every, precision, log)
    sc = scores_of(its, lbs, tol)
    table = {candidates[c]: v for c, v in sc.items()}
    return select(table), table, time.perf_counter() - t0


def family(count: int, N: int = 64, L: int = 2, split: int = 0):
    """Workloads of the ring parameter sweep used by the learned warm start (TFI or XXZ draws)."""
    return [synth.instance_workload(d, name=f"f{split}_{k}") for k, d in enumerate(synth.family_draws(count, N, L, split))]
