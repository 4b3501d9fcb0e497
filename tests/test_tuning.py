"""Host logic of the per-family parameter choice (no GPU): the convergence index of a gap trace,
the scores against the best bound of any run, and the selection rule."""
import math

import numpy as np

from paper_2106_02682_amd import tuning


def test_converged_index_needs_the_gap_to_stay_small():
    g = np.array([1e-2, 1e-7, 1e-3, 1e-7, 1e-8, 1e-9])
    assert tuning.converged_index(g, 1e-6) == 3
    assert tuning.converged_index(np.array([1e-7, 1e-7]), 1e-6) == 0
    assert tuning.converged_index(np.array([1e-7, 1e-3]), 1e-6) is None
    assert tuning.converged_index(np.array([1e-7, np.nan]), 1e-6) is None


def test_scores_use_the_best_bound_of_any_run():
    its = np.array([50, 100, 150])
    # 2 instances x 2 candidates; instance 0: candidate 1 reaches the best bound first
    lbs = np.array([
        [[-1.10, -1.01], [-2.2, -2.0000001]],
        [[-1.02, -1.0000001], [-2.0000001, -2.0]],
        [[-1.0000001, -1.0], [-2.0, -np.inf]],
    ])
    sc = tuning.scores_of(its, lbs, 1e-6)
    assert sc[0] == [150, 100]
    assert sc[1] == [100, None]  # diverged at the last check: never converged


def test_selection_rule():
    p = tuning.PAPER
    a, b = (20.0, 8.0), (5.0, 1.0)
    assert tuning.select({p: [300, 400], a: [200, 250], b: [None, 100]}) == a
    # equal medians: smaller mean of the finite scores, then the paper's choice
    assert tuning.select({p: [200, 300], a: [100, 400]}) == p
    assert tuning.select({a: [200, 300], p: [200, 300]}) == p
    assert tuning.select({a: [None, None], p: [None, None]}) == p
    assert math.isinf(float(np.median([math.inf, math.inf])))
