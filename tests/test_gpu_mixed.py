"""Reduced-precision modes against the FP64 oracle; the error is stated for every result.

* Isolated projections (vemb_psd_project_batched): ``mixed`` = FP32 sweeps, then one FP64 refinement
  sweep and an FP64 rebuild (1e-9 of the result for n <= 64, 5e-8 for 256); ``fp32`` = FP32 throughout.
* Problems in ``mixed`` (``fp32`` is the same for problems): the eigensolves of every iteration run in
  FP32 (Jacobi rotations, the rebuild on FP32 matrix cores, the sign-function products of 256 x 256
  blocks on FP32 matrix cores); state, diagnostics and ``refine`` stay FP64.
  - At equal iteration counts the trajectory drifts from the FP64 one by FP32 rounding: bound errors
    measured 6e-8 (8-ring, 2-site clusters, 300 iterations), 1.3e-6 (16 x 16 torus, 2 x 1 clusters,
    60), 1.1e-6 (8-ring, 4-site clusters, 8), 9.4e-6 (384-ring, 3-site clusters, 60); each case holds
    a tolerance about twice its measurement.
  - Run to convergence and closed by FP64 refinement iterations (vemb_refine), the bound meets the
    oracle's to 1e-6 (the mixed-mode target): 1.5e-8 measured on the 8-ring.
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


@pytest.mark.parametrize("w,iters,tol", [(synth.config_c2(1.0)[1], 60, 2e-5), (synth.config_c3()[0], 60, 3e-6),
                                         (synth.tfi_ring(8, 2, 1.0), 300, 2e-7), (synth.tfi_ring(8, 4, 1.0), 8, 3e-6)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_mixed_iteration_error_vs_fp64_oracle(vemb, w, iters, tol):
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
    print(f"{w.name}: mixed (FP32 eigensolves) vs FP64 oracle after {iters} iterations: lb rel {err_lb:.2e}, "
          f"energy rel {err_e:.2e}, X rel {err_x:.2e}")
    assert err_lb < tol
    assert err_e < tol


@pytest.mark.parametrize("w,iters,refine", [(synth.tfi_ring(8, 2, 1.0), 3000, 200)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_mixed_converged_and_refined_meets_the_oracle(vemb, w, iters, refine):
    """FP32 iterations to convergence, closed by FP64 refinement iterations: the certified bound equals the
    FP64 oracle's after the same number of iterations to 1e-6 relative."""
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, iters + refine)
    lb_o = alg6.lower_bound(p, s)
    with vemb.Problem.from_workload(w, precision="mixed") as g:
        g.step(iters)
        g.refine(refine)
        lb = g.dual_bound()
        e, feas = g.primal_energy()
    err = abs(lb - lb_o) / abs(lb_o)
    print(f"{w.name}: mixed {iters} + FP64 refine {refine}: lb {lb:.12f} oracle {lb_o:.12f} (rel {err:.2e}), "
          f"feas {feas:.1e}")
    assert err < 1e-6


def test_fp32_problem_is_mixed(vemb):
    """For problems, ``fp32`` runs the same FP32 eigensolves as ``mixed``: identical iterates."""
    w = synth.config_c3()[0]
    with vemb.Problem.from_workload(w, precision="fp32") as a, vemb.Problem.from_workload(w, precision="mixed") as b:
        a.step(10)
        b.step(10)
        sa, sb = a.get_state(), b.get_state()
    for k in ("X", "rho", "rho_t", "Lam"):
        assert np.array_equal(sa[k], sb[k]), k
