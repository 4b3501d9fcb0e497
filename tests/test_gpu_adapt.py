"""The adaptive mode (vemb_options.adapt_every: (mu, nu, eps) scaled together, the scale following
feasErr of eq. feasErr and the primal-dual gap) against the oracle's adaptive mode (oracle/adapt.py),
element by element, on the three projection routes (16 x 16 blocks, 64 x 64 blocks in the fused launch,
256 x 256 blocks through the sign function); resuming an adaptive run; the batch and dense constructors
refuse the mode."""
import numpy as np
import pytest

import synth
from oracle import adapt, alg6

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("X", "rho0", "rho", "rho_t", "Lam", "Lam1", "Lam2")


@pytest.fixture(scope="module")
def vemb():
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a GPU")
    from paper_2106_02682_amd import vemb as v

    v.lib()
    return v


def _errors(st, s):
    return {k: float(np.abs(st[k] - getattr(s, k)).max() / max(1.0, np.abs(getattr(s, k)).max())) for k in KEYS}


CASES = [
    ("xxz_ring_8_L2", lambda: synth.xxz_ring(8, 2, 0.5), 600, 50),
    ("tfi_ring_12_L3", lambda: synth.tfi_ring(12, 3, 1.0), 150, 25),
    ("tfi_ring_8_L4", lambda: synth.tfi_ring(8, 4, 1.0), 60, 20),
]


@pytest.mark.parametrize("name,make,iters,every", CASES, ids=[c[0] for c in CASES])
def test_adaptive_run_matches_oracle(vemb, name, make, iters, every):
    w = make()
    op = alg6.Problem.from_workload(w)
    s_o, hist, q = adapt.solve(op, iters, every)
    print(f"{name}: {iters} iterations, checks every {every}; oracle scales {[round(c, 4) for *_, c in hist]}",
          flush=True)
    got = []
    with vemb.Problem.from_workload(w, adapt_every=every) as g:
        for _ in range(iters // every):
            g.step(every)
            pen = g.penalties()
            got.append((g.get_state()["t"], pen["last_feas"], pen["last_gap"], pen["scale"]))
        st = g.get_state()
        pen = g.penalties()
    assert len(got) == len(hist)
    for (t, f, gp, c), (tg, fg, gg, cg) in zip(hist, got):
        assert t == tg
        assert abs(fg - f) <= 1e-9 * f + 1e-13, (t, fg, f)
        assert abs(gg - gp) <= 1e-8 * gp + 1e-13, (t, gg, gp)
        assert cg == c, (t, cg, c)
    assert (pen["mu"], pen["nu"], pen["eps"]) == pytest.approx((q.mu, q.nu, q.eps), rel=1e-15)
    errs = _errors(st, s_o)
    print(f"{name}: state errors {errs}")
    assert max(errs.values()) <= 1e-9


def test_adaptive_run_resumes(vemb):
    """get_state / set_state with the kept eigenvectors and vemb_set_penalty_scale continue an adaptive run
    as if it had not stopped."""
    w = synth.xxz_ring(8, 2, 0.5)
    with vemb.Problem.from_workload(w, adapt_every=50) as a:
        a.step(300)
        mid, pen = a.get_state(with_eigvecs=True), a.penalties()
        a.step(300)
        ref, pref = a.get_state(), a.penalties()
    with vemb.Problem.from_workload(w, adapt_every=50) as b:
        b.set_state(mid)
        b.set_penalty_scale(pen["scale"], pen["last_feas"], pen["last_gap"])
        b.step(300)
        st, pb = b.get_state(), b.penalties()
    assert pb["scale"] == pref["scale"] and pb["mu"] == pref["mu"]
    assert pb["last_feas"] == pytest.approx(pref["last_feas"], rel=1e-10)
    assert pb["last_gap"] == pytest.approx(pref["last_gap"], rel=1e-8)
    for k in KEYS:
        assert np.abs(st[k] - ref[k]).max() <= 1e-12 * max(1.0, np.abs(ref[k]).max()), k


def test_batch_and_dense_refuse_adaptive_problems(vemb):
    w = synth.tfi_ring(8, 2, 1.0)
    probs = [vemb.Problem.from_workload(w, adapt_every=10), vemb.Problem.from_workload(w)]
    try:
        with pytest.raises(vemb.VembError, match="single problems"):
            vemb.Batch(probs)
    finally:
        for p in probs:
            p.close()
    with pytest.raises(vemb.VembError, match="translation-invariant"):
        vemb.Dense.from_workload(w, adapt_every=10)
    with pytest.raises(vemb.VembError):
        vemb.Problem.from_workload(w, adapt_every=-1)
    with vemb.Problem.from_workload(w) as g:
        with pytest.raises(vemb.VembError):
            g.set_penalty_scale(0.5)
        g.set_penalty_scale(2.0)
        pen = g.penalties()
        assert (pen["mu"], pen["nu"], pen["eps"], pen["scale"], pen["last_feas"], pen["last_gap"]) == \
            (20.0, 20.0, 4.0, 2.0, -1.0, -1.0)
