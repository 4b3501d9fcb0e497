"""Reduced-precision modes against the FP64 oracle; the error is stated for every result.

* ``mixed``: FP32 Jacobi sweeps find the eigenvectors, one FP64 sweep warm-started from them and
  an FP64 rebuild finish each projection.  Target: 1e-6 relative on the lower bound at equal
  iteration counts.
* ``fp32``: FP32 sweeps and rebuilds throughout; state, diagnostics and ``refine`` stay FP64.
  Its error is reported (about 1e-4 after tens of iterations), not held to 1e-6.
"""
import numpy as np
import pytest

import synth
from oracle import alg6
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


def _interleave(c):
    return np.stack([c.real, c.imag], axis=-1)


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
@pytest.mark.parametrize("n,cplx", [(16, False), (64, False), (256, False), (16, True), (64, True), (256, True)])
def test_projection_error(vemb, n, cplx, precision):
    tol = 5e-4 if precision == "fp32" else (1e-9 if n <= 64 else 5e-8)
    batch = 4
    C = synth.hermitian_batch(n, batch, tag=21) if cplx else synth.admm_like_batch(n, batch, tag=21)
    inp = torch.from_numpy(np.ascontiguousarray(_interleave(C) if cplx else C)).cuda()
    out = torch.empty_like(inp)
    vemb.psd_project_batched(inp, out, is_complex=cplx, precision=precision)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1] if cplx else got
    want = psd_project(C)
    rel = np.abs(got - want).max() / np.abs(want).max()
    print(f"{precision} projection n={n} complex={cplx}: max relative error {rel:.2e}")
    assert rel < tol


@pytest.mark.parametrize("w,iters", [(synth.config_c2(1.0)[1], 60), (synth.config_c3()[0], 60),
                                     (synth.tfi_ring(8, 2, 1.0), 300), (synth.tfi_ring(8, 4, 1.0), 8)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_mixed_iteration_error_vs_fp64_oracle(vemb, w, iters):
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, iters)
    lb_o = alg6.lower_bound(p, s)
    e_o = alg6.energy_per_site(p, s)
    with vemb.Problem.from_workload(w, precision="mixed") as g:
        g.step(iters)
        lb = g.dual_bound()
        e, _ = g.primal_energy()
        st = g.get_state()
    err_lb = abs(lb - lb_o) / abs(lb_o)
    err_e = abs(e - e_o) / abs(e_o)
    err_x = np.abs(st["X"] - s.X).max() / np.abs(s.X).max()
    print(f"{w.name}: mixed vs FP64 oracle after {iters} iterations: lb rel {err_lb:.2e}, energy rel {err_e:.2e}, "
          f"X rel {err_x:.2e}")
    assert err_lb < 1e-6
    assert err_e < 1e-6


@pytest.mark.parametrize("w,iters", [(synth.config_c2(1.0)[1], 60), (synth.config_c3()[0], 60)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_fp32_iteration_error_is_reported(vemb, w, iters):
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, iters + 1)
    lb_o = alg6.lower_bound(p, s)
    with vemb.Problem.from_workload(w, precision="fp32") as g:
        g.step(iters)
        g.refine(1)
        lb = g.dual_bound()
    err_lb = abs(lb - lb_o) / abs(lb_o)
    print(f"{w.name}: fp32 + one FP64 refinement iteration vs FP64 oracle after {iters}+1 iterations: "
          f"lb rel {err_lb:.2e}")
    assert err_lb < 1e-3
