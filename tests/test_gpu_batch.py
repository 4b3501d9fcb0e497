"""Batches of independent problems (parameter sweeps, uneven cluster sizes).

* A batch computes for each instance what stepping it alone computes (the same
  arithmetic, in separately compiled kernels, so contraction of products into
  FMAs may differ): states compared element by element to 1e-12 of each
  array's largest entry.
* The captured graphs are replayed several times with eager work and
  synchronisations in between (diagnostics on the problems' own streams, torch
  work on the current stream); every replay is checked against a batch of
  identical problems launched without graphs, across cold refreshes.
* One batch is checked against the FP64 oracle directly.
"""
import numpy as np
import pytest

import synth
from oracle import alg6

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

STATE_KEYS = ("X", "rho0", "rho", "rho_t", "Lam", "Lam1", "Lam2")


@pytest.fixture(scope="module")
def vemb():
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a GPU")
    from paper_2106_02682_amd import vemb as v

    v.lib()
    return v


def _uneven():
    # pair sizes 16, 64, 16, 256 (M = 2 ring of 4-site clusters) and a torus
    return [synth.tfi_ring(12, 2, 0.5), synth.tfi_ring(12, 3, 1.0), synth.xxz_ring(10, 2, 0.5),
            synth.tfi_ring(8, 4, 1.0), synth.tfi_torus(4, 4, 2, 1, 3.0)]


def _open(vemb, ws, **kw):
    return [vemb.Problem.from_workload(w, **kw) for w in ws]


def _assert_same_state(a, b, what, rtol=0.0):
    sa, sb = a.get_state(), b.get_state()
    worst = 0.0
    for k in STATE_KEYS:
        d = np.abs(sa[k] - sb[k]).max() / max(np.abs(sa[k]).max(), 1e-300)
        worst = max(worst, d)
        if d > rtol:
            raise AssertionError(f"{what}: state {k} differs (max rel {d:.3e} > {rtol:.1e})")
    return worst


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_equals_individual_stepping(vemb, use_graph):
    ws = _uneven()
    iters = 7
    alone = _open(vemb, ws, tpb=256, warm_refresh=4)
    batched = _open(vemb, ws, tpb=256, warm_refresh=4)
    try:
        for p in alone:
            p.step(iters)
        with vemb.Batch(batched, use_graph=use_graph) as b:
            info = b.info()
            print(f"batch of {len(ws)}: {info}")
            assert info["classes"] >= 4
            b.step(iters)
            b.sync()
            lbs = b.dual_bounds()
        for w, p, q, lb in zip(ws, alone, batched, lbs):
            d = _assert_same_state(p, q, w.name, rtol=1e-12)
            lb_alone = p.dual_bound()
            print(f"{w.name}: batch vs alone, max rel state difference {d:.2e}, lb {lb:.15f} vs {lb_alone:.15f}")
            assert abs(lb - lb_alone) <= 1e-12 * abs(lb_alone)
    finally:
        for p in alone + batched:
            p.close()


def test_graph_replays_match_eager_batch(vemb):
    ws = [synth.tfi_ring(12, 3, h) for h in (0.5, 1.0, 2.0)] + [synth.tfi_ring(8, 2, 1.5)]
    g_probs = _open(vemb, ws, warm_refresh=3)
    e_probs = _open(vemb, ws, warm_refresh=3)
    try:
        with vemb.Batch(g_probs, use_graph=True) as bg, vemb.Batch(e_probs, use_graph=False) as be:
            junk = torch.randn(1 << 20, device="cuda")
            for replay in range(7):  # crosses cold refreshes at t = 3 and 6
                bg.step(1)
                be.step(1)
                # eager work between replays: torch on the current stream, diagnostics
                # on the problems' streams, host synchronisation
                junk.mul_(0.5).add_(1.0)
                lb_g = bg.dual_bounds()
                lb_e = be.dual_bounds()
                torch.cuda.synchronize()
                assert np.array_equal(lb_g, lb_e), f"replay {replay}: bounds differ {lb_g - lb_e}"
                for w, p, q in zip(ws, g_probs, e_probs):
                    _assert_same_state(p, q, f"replay {replay} {w.name}")
    finally:
        for p in g_probs + e_probs:
            p.close()


def test_batch_parity_with_oracle(vemb):
    hs = (0.5, 1.0, 3.0)
    ws = [synth.tfi_ring(12, 3, h) for h in hs]
    iters = 30
    probs = _open(vemb, ws)
    try:
        with vemb.Batch(probs) as b:
            b.step(iters)
            lbs = b.dual_bounds()
            es, feas = b.primal_energies()
        for w, p, lb, e in zip(ws, probs, lbs, es):
            op = alg6.Problem.from_workload(w)
            s, _ = alg6.solve(op, iters)
            lb_o = alg6.lower_bound(op, s)
            e_o = alg6.energy_per_site(op, s)
            st = p.get_state()
            err_x = np.abs(st["X"] - s.X).max() / np.abs(s.X).max()
            print(f"{w.name}: lb {lb:.12f} oracle {lb_o:.12f}; X rel {err_x:.2e}")
            assert abs(lb - lb_o) <= 1e-10 * abs(lb_o)
            assert abs(e - e_o) <= 1e-10 * abs(e_o)
            assert err_x < 1e-9
    finally:
        for p in probs:
            p.close()


def test_batch_then_individual_continue(vemb):
    """A problem leaves the batch and continues alone: same as never batching."""
    w = synth.tfi_ring(12, 3, 1.0)
    a, b = _open(vemb, [w, w], tpb=256)
    try:
        a.step(5)
        with vemb.Batch([b]) as bt:
            bt.step(3)
        b.step(2)
        _assert_same_state(a, b, w.name, rtol=1e-12)
    finally:
        a.close()
        b.close()


def test_batch_rejects_mixed_settings(vemb):
    ws = [synth.tfi_ring(8, 2, 1.0)] * 2
    p = vemb.Problem.from_workload(ws[0], warm_refresh=4)
    q = vemb.Problem.from_workload(ws[1], warm_refresh=8)
    try:
        with pytest.raises(vemb.VembError):
            vemb.Batch([p, q])
        with pytest.raises(vemb.VembError):
            vemb.Batch([p, p])
    finally:
        p.close()
        q.close()
