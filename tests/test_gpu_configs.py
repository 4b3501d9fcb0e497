"""The workloads at their full sizes against the FP64 oracle.

* 16x16 torus, 2x2 clusters (63 pair blocks and 34 complex momentum blocks of 256 x 256, matrix-sign
  projections on matrix cores), 20 iterations: FP64 to 1e-10 relative on the bound and energy and 1e-9 of
  each state array's largest entry; MIXED (FP32 eigensolves, FP32 sign-function products) to 2e-5 on
  the bound, its FP32 drift over 20 iterations (printed).
* The 64-instance batched sweep in the benchmark's launch configuration (graph-replayed), 20 iterations:
  every instance's bound, energy and feasibility error against the oracle values that
  tests/golden/make_batch_golden.py wrote (oracle only), and the full states of a sample of instances
  (the smallest of each model and cluster size) against oracle runs made here, element by element.
* The same sweep in MIXED against the same oracle values, to the FP32 drift (2e-5).
* An uneven batch (pair blocks 16, 64, 256 and a torus) against the oracle, instance by instance.
* The 8-site ring with 4-site clusters (one pair marginal spans the ring): the bound and the energy
  approach the exact ground-state energy (tightness) at a step that converges for this instance.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import alg6, exact

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden")
STATE_KEYS = ("X", "rho0", "rho", "rho_t", "Lam", "Lam1", "Lam2")


@pytest.fixture(scope="module")
def vemb():
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a GPU")
    from paper_2106_02682_amd import vemb as v

    v.lib()
    return v


def _state_errors(st, s):
    ref = {"X": s.X, "rho0": s.rho0, "rho": s.rho, "rho_t": s.rho_t, "Lam": s.Lam, "Lam1": s.Lam1, "Lam2": s.Lam2}
    return {k: float(np.abs(st[k] - ref[k]).max() / max(1.0, np.abs(ref[k]).max())) for k in STATE_KEYS}


@pytest.fixture(scope="module")
def c3b_oracle():
    w = synth.config_c3()[1]
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, 20)
    return w, p, s


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 2e-5)])
def test_torus_2x2_clusters_20_iterations(vemb, c3b_oracle, precision, tol):
    w, p, s = c3b_oracle
    print(f"{w.name} {precision}: 20 iterations", flush=True)
    with vemb.Problem.from_workload(w, precision=precision) as g:
        g.step(20)
        st = g.get_state()
        lb = g.dual_bound()
        e, feas = g.primal_energy()
    lb_o, e_o = alg6.lower_bound(p, s), alg6.energy_per_site(p, s)
    errs = _state_errors(st, s)
    print(f"{w.name} {precision}: lb {lb:.15f} oracle {lb_o:.15f} (rel {abs(lb - lb_o) / abs(lb_o):.2e}); "
          f"energy rel {abs(e - e_o) / abs(e_o):.2e}; state errors {errs}")
    assert abs(lb - lb_o) <= tol * abs(lb_o)
    assert abs(e - e_o) <= tol * abs(e_o)
    if precision == "fp64":
        assert max(errs.values()) <= 1e-9


def _sample(instances):
    """Smallest instance (by N) of each (model, L)."""
    best = {}
    for i, d in enumerate(instances):
        key = (d["model"], d["L"])
        if key not in best or d["N"] < instances[best[key]]["N"]:
            best[key] = i
    return sorted(best.values())


def test_batched_sweep_64_instances_against_oracle(vemb):
    with open(os.path.join(GOLD, "c4_t20.json")) as f:
        gold = json.load(f)
    iters = gold["iters"]
    draws = synth.c4_instances(64)
    ws = [synth.instance_workload(d, name=f"c4_{i}") for i, d in enumerate(draws)]
    print(f"batched sweep: {len(ws)} instances, {iters} iterations, graph-replayed", flush=True)
    probs = [vemb.Problem.from_workload(w) for w in ws]
    try:
        with vemb.Batch(probs) as b:
            b.step(iters)
            lbs, status = b.dual_bounds(check=False)
            es, feas = b.primal_energies()
        assert all(rc == 0 for rc in status), status
        worst = 0.0
        for i, (g, lb, e, f) in enumerate(zip(gold["instances"], lbs, es, feas)):
            assert g["draw"]["N"] == draws[i]["N"] and g["draw"]["L"] == draws[i]["L"]
            rel = max(abs(lb - g["lb"]) / abs(g["lb"]), abs(e - g["energy"]) / abs(g["energy"]))
            worst = max(worst, rel)
            assert rel <= 1e-10, (i, lb, g["lb"], e, g["energy"])
            assert abs(f - g["feas"]) <= 1e-8 * max(g["feas"], 1e-3), (i, f, g["feas"])
        print(f"batched sweep: worst relative bound / energy error over 64 instances {worst:.2e}")
        for i in _sample(draws):
            op = alg6.Problem.from_workload(ws[i])
            s, _ = alg6.solve(op, iters)
            errs = _state_errors(probs[i].get_state(), s)
            print(f"  instance {i} ({ws[i].name}, pair blocks {op.n}): state errors {errs}", flush=True)
            assert max(errs.values()) <= 1e-9, (i, errs)
    finally:
        for p in probs:
            p.close()


def test_batched_sweep_mixed_against_oracle(vemb):
    """The same 64 instances in MIXED (FP32 eigensolves, FP32 sign products for the 256-blocks) against the
    FP64 oracle values at t = 20: the FP32 trajectory drifts by rounding, held to 2e-5 relative on every
    bound and energy (measured: median 1.6e-6, worst 1.7e-5 on the XXZ ring of 469 sites with 3-site
    clusters; the torus with 2x2 clusters drifts 3e-7 over the same count)."""
    with open(os.path.join(GOLD, "c4_t20.json")) as f:
        gold = json.load(f)
    iters = gold["iters"]
    draws = synth.c4_instances(64)
    probs = [vemb.Problem.from_workload(synth.instance_workload(d, name=f"c4_{i}"), precision="mixed")
             for i, d in enumerate(draws)]
    try:
        with vemb.Batch(probs) as b:
            b.step(iters)
            lbs, status = b.dual_bounds(check=False)
            es, feas = b.primal_energies()
        assert all(rc == 0 for rc in status), status
        errs = [max(abs(lb - g["lb"]) / abs(g["lb"]), abs(e - g["energy"]) / abs(g["energy"]))
                for g, lb, e in zip(gold["instances"], lbs, es)]
        worst = int(np.argmax(errs))
        print(f"batched sweep MIXED: worst relative bound / energy error {errs[worst]:.2e} (instance {worst}, "
              f"{draws[worst]['model']} N {draws[worst]['N']} L {draws[worst]['L']}); median {np.median(errs):.1e}")
        assert max(errs) <= 2e-5
    finally:
        for p in probs:
            p.close()


def test_uneven_batch_against_oracle(vemb):
    ws = [synth.tfi_ring(12, 2, 0.5), synth.tfi_ring(12, 3, 1.0), synth.xxz_ring(10, 2, 0.5),
          synth.tfi_ring(8, 4, 1.0), synth.tfi_torus(4, 4, 2, 1, 3.0), synth.xxz_ring(16, 4, 1.3)]
    iters = 9
    probs = [vemb.Problem.from_workload(w) for w in ws]
    try:
        with vemb.Batch(probs) as b:
            b.step(iters)
            lbs = b.dual_bounds()
        for w, p, lb in zip(ws, probs, lbs):
            op = alg6.Problem.from_workload(w)
            s, _ = alg6.solve(op, iters)
            lb_o = alg6.lower_bound(op, s)
            errs = _state_errors(p.get_state(), s)
            print(f"{w.name}: lb rel {abs(lb - lb_o) / abs(lb_o):.2e}, state errors {errs}")
            assert abs(lb - lb_o) <= 1e-10 * abs(lb_o)
            assert max(errs.values()) <= 1e-9
    finally:
        for p in probs:
            p.close()


def test_ring_spanned_by_one_pair_is_tight(vemb):
    """N = 8, 4-site clusters (M = 2): the single pair marginal is the whole state, so the relaxation is
    exact.  At the paper's step eps = 2 this instance does not converge (the bound stays ~9 per site
    below E_0 after 30,000 iterations, on the GPU as in the oracle); the relaxation's value does not
    depend on the step, and with eps = 0.5 bound and energy approach E_0 / N of exact diagonalisation
    sublinearly (1e-5 by 10,000 iterations), the bound staying below it."""
    w = synth.tfi_ring(8, 4, 1.0)
    E0, _ = exact.ground_state(w.terms, w.extent)
    with vemb.Problem.from_workload(w, eps=0.5) as g:
        g.step(10000)
        lb = g.dual_bound()
        e, feas = g.primal_energy()
    print(f"{w.name} eps 0.5: lb - E0/N {lb - E0 / 8:.2e}, energy - E0/N {e - E0 / 8:.2e}, feas {feas:.1e}")
    assert lb <= E0 / 8 + 1e-12
    assert abs(lb - E0 / 8) <= 2e-5
    assert abs(e - E0 / 8) <= 3e-5
