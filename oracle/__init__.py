"""FP64 CPU oracle of the translation-invariant two-marginal SDP iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links
or executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library and imports nothing from it; the two meet only through the seeded
input generators in ``synth``.

Contents
--------
``model``    lattice / cluster geometry and the local Hamiltonians H_0, H_{0,d}
             (Sections 2.1-2.3 and 3.3 of the paper).
``maps``     operator-collection maps: partial traces A_1, A_2 and adjoints,
             the global-matrix blocks G_{0,0}, G_{0,d}, the effective
             Hamiltonians (eq. effHam), the closed-form inverse of the pair
             system (eq. rhoijUpdate), the PSD projection (Section 3).
``alg6``     Algorithm 6 step by step, plus the diagnostics (energy, eq.
             feasErr, the Lagrangian lower bound).
``alg5``     tiny dense non-translation-invariant Algorithm 5, used only to
             pin the translation-invariant reduction.
``exact``    exact diagonalisation and the Jordan-Wigner closed form.
``mlp``      FP64 forward/backward of the warm-start network (gradient pin).
``warm``     the warm-start state encoding and decoding.
``adapt``    Algorithm 6 with the joint scale of (mu, nu, eps) adapted during
             the run (Section 4's remark on tuning them).
``fermion``  Jordan-Wigner operators and Hamiltonians of spinless fermions.

Readings of the paper that the oracle fixes are listed in the header of
``alg6``; every function cites the passage it follows.
"""
from . import model, maps, alg6, exact  # noqa: F401
