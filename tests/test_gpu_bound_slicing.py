"""The bound of problems with 256 x 256 pair blocks (4-site clusters) against the FP64 oracle.

lambda_min of every pair matrix of the Lagrangian bound is found above 128 by spectral slicing: the
sign function of sigma I - K on FP64 matrix cores (in every precision mode: the bound is an FP64
diagnostic), then a Rayleigh-Ritz step in FP64 on K itself.  Each evaluation is compared with the oracle's
bound of the library's own state (its eigendecompositions, Section 2.4's bound), so both precision modes
are held to 1e-10.  The instances include the SU(2)-symmetric
XXZ ring at J_z = 1, whose pair matrices have degenerate low spectra, a torus, the ring spanned by one
pair, the first evaluation (no Ritz vector yet: smallest diagonal shift, several passes), and a state
replaced under the kept Ritz vectors."""
import numpy as np
import pytest

import synth
from oracle import alg6

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


def _oracle_bound(op, st):
    s = alg6.State(t=int(st["t"]), **{k: np.array(st[k]) for k in KEYS})
    return alg6.lower_bound(op, s)


CASES = [
    ("tfi_ring_8_L4", lambda: synth.tfi_ring(8, 4, 1.0)),
    ("xxz_ring_16_L4_jz1", lambda: synth.xxz_ring(16, 4, 1.0)),
    ("xxz_ring_12_L4_jz05", lambda: synth.xxz_ring(12, 4, 0.5)),
    ("tfi_torus_8x4_2x2", lambda: synth.tfi_torus(8, 4, 2, 2, 3.0)),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_bound_by_slicing_matches_oracle(vemb, name, make, precision):
    w = make()
    op = alg6.Problem.from_workload(w)
    print(f"{name} {precision}: pair blocks {op.n}", flush=True)
    assert op.n == 256
    worst = 0.0
    with vemb.Problem.from_workload(w, precision=precision) as g:
        for k in (0, 3, 10, 30):
            if k > g.get_state()["t"]:
                g.step(k - g.get_state()["t"])
            lb = g.dual_bound()
            lb_o = _oracle_bound(op, g.get_state())
            rel = abs(lb - lb_o) / abs(lb_o)
            worst = max(worst, rel)
            print(f"  t={k}: lb {lb:.15f} oracle {lb_o:.15f} rel {rel:.1e}", flush=True)
            assert rel <= 1e-10, (k, lb, lb_o)
    print(f"{name} {precision}: worst {worst:.1e}")


def test_bound_after_state_replaced(vemb):
    """A state from elsewhere under Ritz vectors kept from another state: the shifts start high and the
    flagged blocks take further passes; the value still matches the oracle."""
    w = synth.xxz_ring(16, 4, 1.0)
    op = alg6.Problem.from_workload(w)
    with vemb.Problem.from_workload(w) as g:
        s0 = g.get_state()
        g.step(40)
        lb40 = g.dual_bound()
        assert abs(lb40 - _oracle_bound(op, g.get_state())) <= 1e-10 * abs(lb40)
        g.set_state(s0)
        lb0 = g.dual_bound()
        lb0_o = _oracle_bound(op, g.get_state())
        print(f"after set_state: lb {lb0:.15f} oracle {lb0_o:.15f}")
        assert abs(lb0 - lb0_o) <= 1e-10 * abs(lb0_o)


def test_diagnostics_queue_with_slicing(vemb):
    """The queued diagnostics (the watchdog's path) give the same bound as the synchronous call."""
    w = synth.tfi_torus(8, 4, 2, 2, 3.0)
    op = alg6.Problem.from_workload(w)
    with vemb.Problem.from_workload(w) as g:
        g.step(5)
        g.diagnostics_enqueue()
        lb_q, e_q, f_q = g.diagnostics_collect()
        lb_o = _oracle_bound(op, g.get_state())
        lb_s = g.dual_bound()
        print(f"queued {lb_q:.15f} sync {lb_s:.15f} oracle {lb_o:.15f}")
        assert abs(lb_q - lb_o) <= 1e-10 * abs(lb_o)
        assert abs(lb_s - lb_o) <= 1e-10 * abs(lb_o)
