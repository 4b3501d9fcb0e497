"""The divergence watchdog's rule (vemb_divergence_check) decided on the host, no GPU: non-finite
values give VEMB_E_NUMERIC; a feasibility error above 1e3, or one that rose at each of the last five
checks to 100 times its smallest value, gives VEMB_E_DIVERGED; ordinary histories (decreasing, noisy,
or briefly rising, as ADMM residuals do) pass.  The allocator hook's argument checks need no GPU either."""
import math

import numpy as np
import pytest

from paper_2106_02682_amd import vemb

NUMERIC, DIVERGED, INVALID = -5, -6, -1


def test_numeric():
    assert vemb.divergence_check([1e-3, math.nan], -1.0, -1.0) == NUMERIC
    assert vemb.divergence_check([1e-3], math.inf, -1.0) == NUMERIC
    assert vemb.divergence_check([1e-3], -1.0, -math.inf) == NUMERIC


def test_diverged():
    assert vemb.divergence_check([1e-3, 2e3], -1.0, -1.0) == DIVERGED
    rise = list(np.geomspace(1e-4, 1e-1, 8))  # rising every check, 1000x overall
    assert vemb.divergence_check(rise, -1.0, -1.0) == DIVERGED
    # the printed "+ eps G" iteration of the oracle's 8-ring: feasibility history every 10 iterations
    from oracle import alg6
    import synth

    p = alg6.Problem.from_workload(synth.tfi_ring(8, 1, 1.0))
    s = alg6.initial_state(p)
    hist, fired = [], None
    with np.errstate(all="ignore"):
        for t in range(1, 301):
            s = alg6.step(p, s, sign=+1)
            if t % 10 == 0:
                hist.append(alg6.feasibility_error(p, s))
                rc = vemb.divergence_check(hist, alg6.lower_bound(p, s), alg6.energy_per_site(p, s))
                if rc != 0:
                    fired = (t, rc)
                    break
    assert fired is not None and fired[1] in (NUMERIC, DIVERGED), fired


def test_ordinary_histories_pass():
    assert vemb.divergence_check([0.5], -1.0, -1.0) == 0
    dec = list(np.geomspace(1e-1, 1e-9, 40))
    assert vemb.divergence_check(dec, -1.2, -1.1) == 0
    noisy = [1e-3 * (1 + 0.5 * np.sin(i)) for i in range(30)]
    assert vemb.divergence_check(noisy, -1.2, -1.1) == 0
    # five rises but only 4x growth: ADMM residuals do rise for a while
    brief = [1e-4, 1e-4, 1.2e-4, 1.6e-4, 2e-4, 3e-4, 4e-4]
    assert vemb.divergence_check(brief, -1.2, -1.1) == 0
    # the oracle's ordinary iteration never fires
    from oracle import alg6
    import synth

    p = alg6.Problem.from_workload(synth.tfi_ring(8, 2, 1.0))
    s = alg6.initial_state(p)
    hist = []
    for t in range(1, 601):
        s = alg6.step(p, s)
        if t % 10 == 0:
            hist.append(alg6.feasibility_error(p, s))
            assert vemb.divergence_check(hist, alg6.lower_bound(p, s), alg6.energy_per_site(p, s)) == 0


def test_invalid_arguments():
    lib = vemb.lib()
    assert lib.vemb_divergence_check(None, 3, -1.0, -1.0) == INVALID
    f = np.zeros(1)
    assert lib.vemb_divergence_check(f.ctypes.data_as(vemb._DP), 0, -1.0, -1.0) == INVALID


def test_allocator_needs_both_functions_or_neither():
    lib = vemb.lib()
    a = vemb.ALLOC_FN(lambda n, c: None)
    assert lib.vemb_set_allocator(a, vemb.FREE_FN(), None) == INVALID
    assert lib.vemb_set_allocator(vemb.ALLOC_FN(), vemb.FREE_FN(), None) == 0  # back to hipMalloc
