"""PSD projection of one large symmetric matrix by the matrix-sign route (scaled Newton-Schulz on
matrix cores), the dense solver's X projection for K > 64, against the oracle's eigendecomposition
projection: ADMM-shaped inputs from 16 to 1024, and degenerate spectra (zero, PSD, NSD, identities,
a rank-deficient spectrum, eigenvalues at the resolution limit), an asymmetric input (its symmetric
part is projected) and in-place use.  Tolerance: 1e-12 ||A||_F (the schedule resolves every
eigenvalue above 1e-14 ||A||_F; products add rounding of order n u ||A||)."""
import numpy as np
import pytest

import synth
from oracle.maps import psd_project

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vemb():
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a GPU")
    from paper_2106_02682_amd import vemb as v

    v.lib()
    return v


def _project(vemb, C, inplace=False):
    x = torch.from_numpy(np.ascontiguousarray(C)).cuda()
    out = x if inplace else torch.empty_like(x)
    vemb.psd_project_sign(x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n", [16, 48, 96, 256, 512, 1024])
def test_matches_oracle(vemb, n):
    C = synth.admm_like_batch(n, 1, tag=81)[0]
    got = _project(vemb, C)
    want = psd_project(C)
    err = np.abs(got - want).max()
    print(f"n {n}: max error {err:.2e}, ||C||_F {np.linalg.norm(C):.2e}")
    assert err <= 1e-12 * np.linalg.norm(C)
    assert np.array_equal(got, got.T)


def test_degenerate_spectra(vemb):
    n = 64
    rng = np.random.default_rng([synth.BASE_SEED, 82])
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = rng.standard_normal((n, n))
    S = B @ B.T / n
    spectra = {
        "rank deficient": np.r_[np.ones(20), np.zeros(24), -np.ones(20)],
        "resolution limit": np.r_[np.ones(8), 1e-16 * np.ones(24), -1e-16 * np.ones(24), -np.ones(8)],
        "graded": np.r_[np.logspace(0, -12, 32), -np.logspace(0, -12, 32)],
    }
    cases = {"zero": np.zeros((n, n)), "psd": S, "nsd": -S, "identity": np.eye(n), "minus identity": -np.eye(n)}
    for k, lam in spectra.items():
        cases[k] = (Qm * lam) @ Qm.T
    for name, C in cases.items():
        got = _project(vemb, C)
        want = psd_project(C)
        err = np.abs(got - want).max()
        print(f"{name}: {err:.2e}")
        assert err <= 1e-12 * max(np.linalg.norm(C), 1e-300), name
    assert np.abs(_project(vemb, np.zeros((n, n)))).max() == 0.0


def test_asymmetric_input_and_in_place(vemb):
    n = 96
    rng = np.random.default_rng([synth.BASE_SEED, 83])
    C = rng.standard_normal((n, n))
    want = psd_project(0.5 * (C + C.T))
    assert np.abs(_project(vemb, C) - want).max() <= 1e-12 * np.linalg.norm(C)
    assert np.abs(_project(vemb, C, inplace=True) - want).max() <= 1e-12 * np.linalg.norm(C)
