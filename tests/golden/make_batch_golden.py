"""Writes tests/golden/c4_t20.json: the FP64 oracle's Lagrangian bound, energy and feasibility error per
site after 20 iterations of Algorithm 6 for each of the 64 seeded instances of the batched parameter
sweep (TFI or XXZ rings, N 32..512, clusters of 2..4 sites), from the initialisation of Section 4.

Only the oracle is called.  Run from the repository root (a pool of processes, one BLAS thread each;
about ten minutes of CPU):  python tests/golden/make_batch_golden.py [--processes 8]
"""
import argparse
import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

ITERS = 20


def _run(i):
    from threadpoolctl import threadpool_limits

    from oracle import alg6

    d = synth.c4_instances(64)[i]
    w = synth.instance_workload(d, name=f"c4_{i}")
    with threadpool_limits(1):
        p = alg6.Problem.from_workload(w)
        s, _ = alg6.solve(p, ITERS)
        out = {"draw": d, "N_eff": w.extent[0], "L": w.cluster[0], "P": p.P, "n": p.n,
               "lb": alg6.lower_bound(p, s), "energy": alg6.energy_per_site(p, s),
               "feas": alg6.feasibility_error(p, s)}
    print(f"instance {i}: {w.name}, P {p.P} of {p.n}: lb {out['lb']:.15f}", flush=True)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--processes", type=int, default=8)
    args = ap.parse_args()
    with Pool(args.processes) as pool:
        res = pool.map(_run, range(64), chunksize=1)
    doc = {"_source": "oracle.alg6 (FP64), 20 iterations from the Section 4 initialisation, mu = nu = 10, eps = 2; "
                      "instances synth.c4_instances(64) (draws default_rng([210602682, 4, i]))",
           "iters": ITERS, "instances": res}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_t20.json"), "w") as f:
        json.dump(doc, f, indent=1)
