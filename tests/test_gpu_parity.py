"""GPU parity of the HIP path against the FP64 oracle (calls go through the C ABI).

* batched PSD projection and eigenvalues vs the oracle's projection / numpy,
  real and Hermitian, sizes spanning every LDS size class, odd sizes (padding
  column) and degenerate inputs (zero, PSD, NSD, repeated eigenvalues);
* full iterations of Algorithm 6 vs the oracle at equal iteration counts:
  the Lagrangian bound to 1e-10 relative (FP64), energies, feasibility and
  every state array element by element;
* the bench workload (N=384 ring, 3-site clusters, 64 x 64 marginals) at the
  launch configuration the benchmark times, compared after a few iterations.
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _interleave(c):
    return np.stack([c.real, c.imag], axis=-1)


def _deinterleave(a):
    return a[..., 0] + 1j * a[..., 1]


@pytest.mark.parametrize("n,batch", [(2, 5), (3, 7), (4, 64), (7, 9), (8, 33), (16, 130), (33, 5), (64, 127),
                                     (128, 3)])
def test_projection_real_fp64(vemb, n, batch):
    C = synth.admm_like_batch(n, batch, tag=11)
    out = torch.empty(C.shape, dtype=torch.float64, device="cuda")
    vemb.psd_project_batched(_dev(C), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = psd_project(C)
    scale = np.abs(C).max()
    assert np.abs(got - want).max() <= 1e-12 * max(scale, 1.0) * max(1, n / 16)


@pytest.mark.parametrize("n,batch", [(3, 8), (4, 8), (9, 6), (16, 65), (64, 65)])
def test_projection_complex_fp64(vemb, n, batch):
    C = synth.hermitian_batch(n, batch, tag=12)
    out = torch.empty(C.shape + (2,), dtype=torch.float64, device="cuda")
    vemb.psd_project_batched(_dev(_interleave(C)), out, is_complex=True)
    torch.cuda.synchronize()
    got = _deinterleave(out.cpu().numpy())
    want = psd_project(C)
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(C).max()) * max(1, n / 16)


@pytest.mark.parametrize("n,batch,cplx", [(256, 3, False), (160, 2, False), (256, 2, True), (128, 3, True)])
def test_projection_streamed_solver(vemb, n, batch, cplx):
    """Matrices above the LDS capacity go through the block-streamed solver."""
    C = synth.hermitian_batch(n, batch, tag=15) if cplx else synth.admm_like_batch(n, batch, tag=15)
    inp = _dev(_interleave(C) if cplx else C)
    out = torch.empty_like(inp)
    sw = torch.zeros(batch, dtype=torch.int32, device="cuda")
    vemb.psd_project_batched_ex(inp, out, is_complex=cplx, sweeps=sw)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    got = _deinterleave(got) if cplx else got
    assert np.abs(got - psd_project(C)).max() <= 1e-12 * max(1.0, np.abs(C).max()) * n / 16
    assert int(sw.max()) < 40
    w = torch.empty((batch, n), dtype=torch.float64, device="cuda")
    vemb.eigvalsh_batched(inp, w, is_complex=cplx)
    torch.cuda.synchronize()
    want = np.linalg.eigvalsh(C)
    assert np.abs(w.cpu().numpy() - want).max() <= 1e-12 * max(1.0, np.abs(want).max()) * n / 16


def test_projection_degenerate_inputs(vemb):
    n = 16
    rng = np.random.default_rng(3)
    B = rng.standard_normal((n, n))
    S = B @ B.T / n
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    rep = Q @ np.diag([1.0] * 5 + [-1.0] * 5 + [0.0] * 6) @ Q.T  # +-1 pairs and a zero block
    cases = np.stack([np.zeros((n, n)), S, -S, rep, np.eye(n), -np.eye(n)])
    out = torch.empty(cases.shape, dtype=torch.float64, device="cuda")
    vemb.psd_project_batched(_dev(cases), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = psd_project(cases)
    assert np.abs(got - want).max() < 1e-12
    assert np.abs(got[0]).max() == 0.0


@pytest.mark.parametrize("n,cplx", [(5, False), (16, False), (64, False), (128, False), (16, True), (64, True)])
def test_eigenvalues(vemb, n, cplx):
    if cplx:
        C = synth.hermitian_batch(n, 9, tag=13)
        inp = _dev(_interleave(C))
    else:
        C = synth.admm_like_batch(n, 9, tag=13)
        inp = _dev(C)
    w = torch.empty((9, n), dtype=torch.float64, device="cuda")
    vemb.eigvalsh_batched(inp, w, is_complex=cplx)
    torch.cuda.synchronize()
    want = np.linalg.eigvalsh(C)
    assert np.abs(w.cpu().numpy() - want).max() <= 1e-12 * max(1.0, np.abs(want).max()) * max(1, n / 16)


def _tight_gershgorin_cases(complex_phases):
    """Singlet/triplet matrices x P_s + y P_t (x > 0 > y): the Gershgorin shift equals -lambda_min, so
    B = C + s I is exactly singular with a triple (or larger) zero eigenvalue -- rounding-noise columns."""
    v = np.array([0.0, 1.0, -1.0, 0.0]) / np.sqrt(2.0)
    Ps = np.outer(v, v)
    out = []
    for x, y in [(0.238, -1.61), (0.9, -0.3), (1.0, -1.0)]:
        C = x * Ps + y * (np.eye(4) - Ps)
        for blk in (C, np.kron(C, np.eye(4)), np.kron(np.eye(2), C)):
            if complex_phases:
                th = np.linspace(0.3, 2.9, blk.shape[0])
                D = np.diag(np.exp(1j * th))
                blk = D @ blk @ D.conj().T
            out.append(blk)
    return out


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("max_sweeps", [40, 400])
def test_projection_exactly_singular_shift(vemb, cplx, max_sweeps):
    """Regression: noise columns of an exactly singular B must not be rotated forever (the complex
    phase of an underflowing inner product rescaled the surviving column)."""
    for C in _tight_gershgorin_cases(cplx):
        n = C.shape[0]
        inp = _dev(_interleave(C[None]) if cplx else C[None])
        out = torch.empty_like(inp)
        sw = torch.zeros(1, dtype=torch.int32, device="cuda")
        vemb.psd_project_batched_ex(inp, out, is_complex=cplx, max_sweeps=max_sweeps, sweeps=sw)
        torch.cuda.synchronize()
        got = out.cpu().numpy()[0]
        got = _deinterleave(got) if cplx else got
        assert np.abs(got - psd_project(C)).max() < 1e-14 * n
        assert int(sw.cpu()[0]) < 10


def test_projection_inplace_alias(vemb):
    C = synth.admm_like_batch(32, 10, tag=14)
    buf = _dev(C)
    vemb.psd_project_batched(buf, buf)
    torch.cuda.synchronize()
    assert np.abs(buf.cpu().numpy() - psd_project(C)).max() < 1e-12


# ---------------------------------------------------------------------------
# Full iterations
# ---------------------------------------------------------------------------

def _compare(w, iters, rel_lb=1e-10, atol_state=1e-9):
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, iters)
    from paper_2106_02682_amd import vemb as v

    with v.Problem.from_workload(w) as g:
        worst = (0, 0)
        for _ in range(iters):
            g.step(1)
            sw = g.last_sweeps()
            worst = (max(worst[0], sw[0]), max(worst[1], sw[1]))
        assert max(worst) < 40, f"an eigensolve hit the sweep cap: {worst}"
        st = g.get_state()
        lb = g.dual_bound()
        e, feas = g.primal_energy()
    assert st["t"] == iters
    lb_o = alg6.lower_bound(p, s)
    assert abs(lb - lb_o) <= rel_lb * abs(lb_o), (lb, lb_o)
    assert abs(e - alg6.energy_per_site(p, s)) <= rel_lb * abs(lb_o)
    fo = alg6.feasibility_error(p, s)
    assert abs(feas - fo) <= 1e-8 * max(fo, 1e-3)
    for key, ref in [("X", s.X), ("rho0", s.rho0), ("rho", s.rho), ("rho_t", s.rho_t), ("Lam", s.Lam),
                     ("Lam1", s.Lam1), ("Lam2", s.Lam2)]:
        err = np.abs(st[key] - ref).max()
        assert err <= atol_state * max(1.0, np.abs(ref).max()), (key, err)
    return lb, lb_o


@pytest.mark.parametrize("w,iters", [
    (synth.tfi_ring(8, 1, 1.0), 300),
    (synth.tfi_ring(8, 1, 1.0, "pauli1"), 300),
    (synth.tfi_ring(8, 2, 1.0), 200),
    (synth.tfi_ring(6, 1, 0.5), 200),
    (synth.tfi_ring(9, 3, 1.5), 60),
    (synth.xxz_ring(8, 2, 0.7), 150),
    (synth.tfi_ring(4, 2, 1.0), 200),
    (synth.tfi_torus(4, 4, 2, 1, 1.0), 80),
    (synth.tfi_torus(6, 4, 1, 2, 3.0), 40),
    (synth.afh_torus(4, 4, 1, 1), 100),
    (synth.tfi_ring(8, 4, 1.0), 12),
    (synth.tfi_torus(4, 4, 2, 2, 3.0), 6),
], ids=lambda x: getattr(x, "name", str(x)))
def test_iteration_parity_fp64(vemb, w, iters):
    _compare(w, iters)


def test_bench_workload_parity(vemb):
    """N = 384 ring, L = 3 (127 pair marginals 64 x 64, 65 unique momentum blocks 64 x 64)."""
    w = synth.config_c2(1.0)[1]
    _compare(w, 5, rel_lb=1e-10, atol_state=1e-9)


@pytest.mark.parametrize("w", [synth.tfi_ring(8, 2, 1.0), synth.config_c2(0.5)[1]], ids=lambda w: w.name)
def test_state_roundtrip_and_resume(vemb, w):
    """Resuming from a checkpoint that includes the kept eigenvectors is bit-identical to running through;
    without them the resumed run starts its eigensolves cold and agrees to rounding."""
    from paper_2106_02682_amd import vemb as v

    with v.Problem.from_workload(w) as a, v.Problem.from_workload(w) as b, v.Problem.from_workload(w) as c:
        a.step(30)
        mid = a.get_state(with_eigvecs=True)
        a.step(20)
        b.set_state(mid)
        b.step(20)
        c.set_state({k: mid[k] for k in mid if k not in ("Vpair", "Vmom")})
        c.step(20)
        sa, sb, sc = a.get_state(), b.get_state(), c.get_state()
    for k in ("X", "rho0", "rho_t", "Lam", "Lam1", "Lam2"):
        assert np.array_equal(sa[k], sb[k]), k
        assert np.abs(sa[k] - sc[k]).max() < 1e-11, k
    assert sb["t"] == 50


def test_sampled_kernel_timing(vemb):
    """With timing on every 5th iteration, 20 iterations time 4 launches of each timed kernel;
    a step count below 1 is rejected."""
    from paper_2106_02682_amd import vemb as v

    with v.Problem.from_workload(synth.tfi_ring(8, 2, 1.0)) as g:
        g.step(3)
        g.set_profiling(True, kernels=["pair_update", "cluster_update"])
        g.set_profiling_every(5)
        g.step(20)  # iterations 3..22: t = 5, 10, 15, 20 are timed
        prof = g.get_profile()
        with pytest.raises(v.VembError):
            g.set_profiling_every(0)
    assert prof["pair_update"][1] == 4 and prof["cluster_update"][1] == 4
    assert prof["pair_xstep"][1] == 0
    assert prof["pair_update"][0] > 0


def test_fused_projections_match_separate_launches(vemb):
    """With both eigensolvers on 512 threads the pair and momentum projections run as one launch on one
    stream; forced to 1024 threads they run as two launches on two streams.  The iterates agree to the
    rounding of the different lane groupings."""
    from paper_2106_02682_amd import vemb as v

    w = synth.config_c2(1.0)[1]
    with v.Problem.from_workload(w, tpb=512) as a, v.Problem.from_workload(w, tpb=1024) as b:
        a.set_profiling(True)
        b.set_profiling(True)
        a.step(20)
        b.step(20)
        pa, pb = a.get_profile(), b.get_profile()
        sa, sb = a.get_state(), b.get_state()
        la, lb = a.dual_bound(), b.dual_bound()
    assert pa["projections"][1] == 20 and pa["pair_projection"][1] == 0 and pa["momentum_projection"][1] == 0
    assert pb["projections"][1] == 0 and pb["pair_projection"][1] == 20 and pb["momentum_projection"][1] == 20
    for k in ("X", "rho0", "rho_t", "Lam", "Lam1", "Lam2"):
        assert np.abs(sa[k] - sb[k]).max() < 1e-9, k
    assert abs(la - lb) < 1e-10 * abs(lb)


@pytest.mark.parametrize("w", [synth.tfi_ring(8, 2, 1.0), synth.afh_torus(4, 4, 1, 1), synth.config_c2(1.0)[1]],
                         ids=lambda w: w.name)
def test_kept_eigenvectors_orthonormal(vemb, w):
    """The eigenvectors kept for the next warm start (the normalised columns of the converged W, or the
    identity for a block with a noise-floor column) are orthonormal in every block up to the residual
    non-orthogonality of the converged W, which also bounds the error of the projection built from that W:
    the sweep that ends a solve rotated by less than sqrt(tol) / 16 (~7e-9 at n = 64), and after it the
    residual is far smaller except inside clusters of nearly equal eigenvalues (measured: 3.4e-12 on the
    N = 384 ring after 30 iterations)."""
    from paper_2106_02682_amd import vemb as v

    with v.Problem.from_workload(w) as g:
        g.step(30)
        st = g.get_state(with_eigvecs=True)
    vp = st["Vpair"]
    vm = st["Vmom"][..., 0] + 1j * st["Vmom"][..., 1]
    for name, V in (("pair", vp), ("momentum", vm)):
        eye = np.eye(V.shape[1])
        dev = max(np.abs(b @ b.conj().T - eye).max() for b in V)
        assert dev < 1e-10, (name, dev)


@pytest.mark.parametrize("w", [synth.tfi_ring(8, 2, 1.0), synth.afh_torus(4, 4, 1, 1), synth.config_c2(1.5)[1]],
                         ids=lambda w: w.name)
def test_warm_started_eigensolves_match_cold(vemb, w):
    """Eigensolves started from the previous eigenvectors give the same iterates as cold solves.  Both
    stop a solve once the next sweep would rotate nothing above the tolerance, after different numbers
    of sweeps; their iterates agree to a few 1e-11 after 40 iterations."""
    from paper_2106_02682_amd import vemb as v

    with v.Problem.from_workload(w) as a, v.Problem.from_workload(w, warm_refresh=-1) as b:
        for _ in range(40):
            a.step(1)
            b.step(1)
        sa, sb = a.get_state(), b.get_state()
        assert max(a.last_sweeps()) <= max(b.last_sweeps())
    for k in ("X", "rho0", "rho_t", "Lam", "Lam1", "Lam2"):
        assert np.abs(sa[k] - sb[k]).max() < 3e-11 * max(1.0, np.abs(sb[k]).max()), k


def test_set_state_rejects_nonfinite(vemb):
    w = synth.tfi_ring(8, 1, 1.0)
    from paper_2106_02682_amd import vemb as v

    with v.Problem.from_workload(w) as g:
        st = g.get_state()
        st["Lam"][0, 0, 0] = np.nan
        with pytest.raises(v.VembError) as ei:
            g.set_state(st)
        assert ei.value.code == -5


def test_repeated_bounds_and_diagnostics(vemb):
    """The bound's eigensolves start from the previous evaluation's eigenvectors (every 16th cold):
    each of 20 evaluations, 3 iterations apart, against the oracle; vemb_diagnostics against the
    separate calls."""
    from paper_2106_02682_amd import vemb as v

    w = synth.tfi_ring(12, 3, 0.7)
    p = alg6.Problem.from_workload(w)
    s = alg6.initial_state(p)
    with v.Problem.from_workload(w) as g:
        for k in range(20):
            g.step(3)
            for _ in range(3):
                s = alg6.step(p, s)
            if k % 2:
                lb, e, feas = g.diagnostics()
            else:
                lb = g.dual_bound()
                e, feas = g.primal_energy()
            lb_o = alg6.lower_bound(p, s)
            assert abs(lb - lb_o) <= 1e-10 * abs(lb_o), (k, lb, lb_o)
            assert abs(e - alg6.energy_per_site(p, s)) <= 1e-10 * abs(lb_o)
        lb2 = g.dual_bound()
        e2, f2 = g.primal_energy()
        lb3, e3, f3 = g.diagnostics()
    assert lb3 == pytest.approx(lb2, rel=1e-13) and e3 == e2 and f3 == f2


def test_async_diagnostics_match_synchronous(vemb):
    """Diagnostics queued without draining the stream report the state at their place in the
    stream, whatever was queued after them."""
    from paper_2106_02682_amd import vemb as v

    w = synth.tfi_ring(12, 3, 0.7)
    with v.Problem.from_workload(w) as a, v.Problem.from_workload(w) as b:
        a.step(7)
        a.diagnostics_enqueue()
        a.step(5)  # queued after the diagnostics
        got = a.diagnostics_collect()
        b.step(7)
        want = b.diagnostics()
        with pytest.raises(v.VembError):
            a.diagnostics_collect()  # nothing pending
    assert got[0] == pytest.approx(want[0], rel=1e-13)
    assert got[1] == want[1] and got[2] == want[2]
