"""Failure handling and memory ownership on the GPU, every kernel exiting normally:

* the printed "+ eps G" step diverges; with lb_every the watchdog stops vemb_step with
  VEMB_E_DIVERGED or VEMB_E_NUMERIC, while the ordinary iteration with the same setting runs on;
* with a 3-sweep cap, warm-started iterations follow cold-started ones to 1e-10 on the 384-ring, and every
  kept basis is orthonormal or the identity on the AFH 48-ring;
* an eigensolve stopped by a (deliberately small) sweep cap is reported as VEMB_E_NOCONV and its kept
  eigenvectors are reset to the identity, so the next solve starts cold;
* with torch's caching allocator installed (the binding's default on a GPU), every device allocation
  of problems, batches, dense problems, networks and isolated entry points goes through it and comes
  back at destruction, and the results equal those of hipMalloc'd runs bit for bit.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vemb():
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a GPU")
    from paper_2106_02682_amd import vemb as v

    v.lib()
    return v


def test_watchdog_stops_the_printed_sign(vemb):
    w = synth.tfi_ring(8, 1, 1.0)
    with vemb.Problem.from_workload(w, sign=+1, lb_every=10) as g:
        with pytest.raises(vemb.VembError) as ei:
            for _ in range(60):
                g.step(10)
        print(f"watchdog: {ei.value}")
        assert ei.value.code in (-5, -6)
    with vemb.Problem.from_workload(w, lb_every=10) as g:
        g.step(600)
        lb, e, feas = g.diagnostics_collect()
        assert np.isfinite(lb) and feas < 1e-3


def test_unconverged_solves_reset_their_eigenvectors(vemb):
    w = synth.tfi_ring(24, 3, 1.0)  # 64 x 64 blocks: a cold solve of a dense block needs about 10 sweeps
    with vemb.Problem.from_workload(w, tpb=256) as ref:
        ref.step(30)
        st0 = ref.get_state()  # without eigenvectors: the next solve starts cold
    with vemb.Problem.from_workload(w, max_sweeps=3, tpb=256) as g:
        g.set_state(st0)
        g.step(1)
        a, b, rc = g.last_sweeps(check=False)
        assert rc == -7 and max(a, b) == 4, (a, b, rc)
        st = g.get_state(with_eigvecs=True)
        n = g.info["n"]
        V = st["Vpair"].reshape(-1, n, n)
        assert np.array_equal(V, np.broadcast_to(np.eye(n), V.shape))
        with pytest.raises(vemb.VembError):
            g.last_sweeps()


def test_capped_warm_solves_match_cold_solves(vemb):
    """A sweep cap of 3 stops every solve of the 384-ring's dense 64 x 64 blocks unconverged; they keep
    the identity instead of a non-orthonormal basis, so the warm-started iterations follow the always-cold
    ones (warm_refresh < 0) to 1e-10 instead of drifting with an unconverged basis."""
    w = synth.tfi_ring(384, 3, 1.0)
    out = {}
    for refresh in (64, -1):
        with vemb.Problem.from_workload(w, max_sweeps=3, warm_refresh=refresh) as g:
            g.step(20)
            out[refresh] = g.get_state()
    keys = ("X", "rho0", "rho", "rho_t", "Lam", "Lam1", "Lam2")
    errs = {k: float(np.abs(out[64][k] - out[-1][k]).max() / max(1.0, np.abs(out[-1][k]).max())) for k in keys}
    print(f"warm vs cold with a 3-sweep cap {errs}")
    assert max(errs.values()) <= 1e-10


def test_capped_solves_keep_orthonormal_bases(vemb):
    """Where some solves do converge within a 3-sweep cap from a warm start (the degenerate spectra of the
    AFH 48-ring with 3-site clusters), warm and cold runs differ by the cold run's truncation (4e-3 after
    20 iterations), so the property checked is the kept bases themselves: after every iteration each
    kept pair and momentum basis is orthonormal (a converged solve) or exactly the identity (an
    unconverged one)."""
    w = synth.xxz_ring(48, 3, 1.0)
    with vemb.Problem.from_workload(w, max_sweeps=3) as g:
        n, k = g.info["n"], g.info["n_op"]
        ident = converged = 0
        for _ in range(20):
            g.step(1)
            st = g.get_state(with_eigvecs=True)
            Vp = st["Vpair"].reshape(-1, n, n)
            Vm = st["Vmom"].reshape(-1, k, k, 2)
            Vm = Vm[..., 0] + 1j * Vm[..., 1]
            for V in list(Vp) + list(Vm):
                if np.array_equal(V, np.eye(V.shape[0])):
                    ident += 1
                    continue
                converged += 1
                err = np.abs(V.conj().T @ V - np.eye(V.shape[0])).max()
                assert err <= 1e-9, err
    print(f"kept bases: {ident} identities, {converged} orthonormal")
    assert ident > 0 and converged > 0


def _run_all(vemb):
    out = {}
    w = synth.tfi_ring(12, 3, 1.0)
    with vemb.Problem.from_workload(w) as g:
        g.step(5)
        out["lb"] = g.dual_bound()
        out["X"] = g.get_state()["X"]
    probs = [vemb.Problem.from_workload(x) for x in (synth.tfi_ring(12, 2, 0.5), synth.tfi_ring(8, 4, 1.0))]
    with vemb.Batch(probs) as b:
        b.step(3)
        out["batch"] = b.dual_bounds()
    for p in probs:
        p.close()
    with vemb.Dense.from_workload(synth.tfi_ring(8, 2, 1.0)) as d:
        d.step(3)
        out["dense"] = d.dual_bound()
    C = torch.from_numpy(synth.admm_like_batch(96, 1, tag=95)[0]).cuda()
    Y = torch.empty_like(C)
    vemb.psd_project_sign(C, Y)
    torch.cuda.synchronize()
    out["sign"] = Y.cpu().numpy()
    net = vemb.MLP([4, 8, 3])
    net.close()
    return out


def test_torch_allocator_sees_every_allocation(vemb):
    ta = vemb.torch_allocator()
    assert ta is not None, "the binding installs torch's allocator on a GPU"
    c0, b0 = ta.count, ta.bytes
    w = synth.tfi_ring(12, 3, 1.0)
    with vemb.Problem.from_workload(w) as g:
        i = g.info
        # the iteration state alone: X, X' and the momentum blocks, rho, rho~, Lambda, the kept eigenvectors
        state = 8 * (2 * i["M"] * i["n_op"] ** 2 + 4 * i["K_unique"] * i["n_op"] ** 2 + 4 * i["P"] * i["n"] ** 2)
        assert ta.count > c0 and ta.bytes - b0 >= state
        assert len(ta.live) > 0
    assert not ta.live, "every allocation returned at destruction"
    got = _run_all(vemb)
    assert not ta.live and ta.frees == ta.count
    # the same computations with hipMalloc / hipFree
    vemb.TorchAllocator.uninstall()
    try:
        ref = _run_all(vemb)
    finally:
        ta.install()
    assert got["lb"] == ref["lb"] and np.array_equal(got["X"], ref["X"])
    assert np.array_equal(got["batch"], ref["batch"]) and got["dense"] == ref["dense"]
    assert np.array_equal(got["sign"], ref["sign"])


def test_allocator_cannot_change_while_objects_live(vemb):
    with vemb.Problem.from_workload(synth.tfi_ring(8, 2, 1.0)):
        with pytest.raises(vemb.VembError):
            vemb.TorchAllocator.uninstall()
