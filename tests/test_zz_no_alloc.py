"""The allocation-free sign projection (static device scratch) against the allocating entry point.

Two calls in a row on the same GPU, the second with a smaller matrix (the static array keeps the
first call's contents, which the second must not read), each compared with vemb_psd_project_sign on
the same input: the kernels and their order are the same, so the results agree bit for bit; the
bar of the projection tests (1e-12 ||C||_F against the oracle's eigendecomposition) is checked too.
Sizes above the static limit are rejected with VEMB_E_INVALID before any device work."""
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


def _both(vemb, C):
    x = torch.from_numpy(np.ascontiguousarray(C)).cuda()
    ref = torch.empty_like(x)
    got = torch.full_like(x, float("nan"))
    vemb.psd_project_sign(x, ref)
    vemb.psd_project_sign_noalloc(x, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_matches_allocating_entry_point_twice(vemb):
    for n, tag in ((512, 91), (96, 92)):  # second call smaller than the first
        C = synth.admm_like_batch(n, 1, tag=tag)[0]
        print(f"noalloc sign projection: n {n}, tag {tag}", flush=True)
        got, ref = _both(vemb, C)
        assert np.array_equal(got, ref), f"n {n}: max difference {np.abs(got - ref).max():.3e}"
        err = np.abs(got - psd_project(C)).max()
        assert err <= 1e-12 * np.linalg.norm(C), f"n {n}: error {err:.3e} against the oracle"


def test_noalloc_in_place_and_limits(vemb):
    n = 64
    C = synth.admm_like_batch(n, 1, tag=93)[0]
    x = torch.from_numpy(C.copy()).cuda()
    vemb.psd_project_sign_noalloc(x, x)
    torch.cuda.synchronize()
    assert np.abs(x.cpu().numpy() - psd_project(C)).max() <= 1e-12 * np.linalg.norm(C)
    big = torch.zeros((528, 528), dtype=torch.float64, device="cuda")
    with pytest.raises(vemb.VembError) as ei:
        vemb.psd_project_sign_noalloc(big, big)
    assert ei.value.code == -1  # VEMB_E_INVALID
    odd = torch.zeros((40, 40), dtype=torch.float64, device="cuda")
    with pytest.raises(vemb.VembError) as ei:
        vemb.psd_project_sign_noalloc(odd, odd)
    assert ei.value.code == -1  # VEMB_E_INVALID
