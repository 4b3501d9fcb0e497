"""The per-family parameter race (tuning.py) on the GPU: iterates at non-default (mu = nu, eps)
against the FP64 oracle, and a small race whose bounds are finite, below the exact energies, and
whose winner follows the selection rule."""
import numpy as np
import pytest

import synth
from oracle import alg6, exact

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vemb():
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a GPU")
    from paper_2106_02682_amd import vemb as v

    v.lib()
    return v


@pytest.mark.parametrize("mu,eps", [(5.0, 1.0), (20.0, 8.0), (40.0, 16.0)])
def test_iterates_at_other_parameters_match_oracle(vemb, mu, eps):
    w = synth.tfi_ring(16, 2, 0.8)
    p = alg6.Problem(w.terms, w.extent, w.cluster, w.opset, mu, mu, eps)
    s, _ = alg6.solve(p, 10)
    with vemb.Problem.from_workload(w, mu=mu, nu=mu, eps=eps) as g:
        g.step(10)
        st = g.get_state()
        lb = g.dual_bound()
    for k, ref in [("X", s.X), ("rho0", s.rho0), ("rho_t", s.rho_t), ("Lam", s.Lam), ("Lam1", s.Lam1)]:
        assert np.abs(st[k] - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max()), k
    lb_o = alg6.lower_bound(p, s)
    assert abs(lb - lb_o) <= 1e-10 * abs(lb_o)


def test_small_race(vemb):
    from paper_2106_02682_amd import tuning

    ws = [synth.tfi_ring(8, 2, 1.0), synth.tfi_ring(8, 2, 0.6)]
    e0 = [exact.tfi_ring_energy_jw(8, 1.0), exact.tfi_ring_energy_jw(8, 0.6)]
    cands = [(5.0, 1.0), (10.0, 2.0), (20.0, 8.0)]
    its, lbs = tuning.run(ws, cands, 3000, 100)
    assert lbs.shape == (30, 2, 3)
    assert np.isfinite(lbs).all()
    for i in range(2):
        assert (lbs[:, i, :] <= e0[i] + 1e-12).all()
    sc = tuning.scores_of(its, lbs, 1e-5)
    table = {cands[c]: v for c, v in sc.items()}
    best = tuning.select(table)
    print("race:", table, "->", best)
    assert best in cands
    assert any(x is not None for v in table.values() for x in v)
