"""Register-resident Jacobi variants for 64 x 64 matrices (solver codes 64 and 128) against the
FP64 oracle, next to the LDS variant (256): projections of ADMM-shaped and degenerate inputs in
every precision, exactly singular shifts, and whole iterations of the benchmark ring with warm
starts.  Tolerances as for the LDS solver (FP64 1e-12 relative, FP32 5e-4, mixed 1e-9)."""
import numpy as np
import pytest

import synth
from oracle import alg6
from oracle.maps import psd_project

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VARIANTS = [64, 128, 256]
TOL = {"fp64": 1e-12, "mixed": 1e-9, "fp32": 5e-4}


@pytest.fixture(scope="module")
def vemb():
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a GPU")
    from paper_2106_02682_amd import vemb as v

    v.lib()
    return v


def _interleave(c):
    return np.stack([c.real, c.imag], axis=-1)


def _project(vemb, C, cplx, precision, tpb, max_sweeps=0):
    inp = torch.from_numpy(np.ascontiguousarray(_interleave(C) if cplx else C)).cuda()
    out = torch.empty_like(inp)
    sw = torch.zeros(C.shape[0], dtype=torch.int32, device="cuda")
    vemb.psd_project_batched_ex(inp, out, is_complex=cplx, precision=precision, max_sweeps=max_sweeps, sweeps=sw,
                                tpb=tpb)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    return (got[..., 0] + 1j * got[..., 1] if cplx else got), sw.cpu().numpy()


@pytest.mark.parametrize("tpb", VARIANTS)
@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
@pytest.mark.parametrize("cplx", [False, True])
def test_projection_variants(vemb, tpb, precision, cplx):
    C = synth.hermitian_batch(64, 33, tag=71) if cplx else synth.admm_like_batch(64, 33, tag=71)
    got, sw = _project(vemb, C, cplx, precision, tpb)
    want = psd_project(C)
    rel = np.abs(got - want).max() / np.abs(want).max()
    print(f"tpb {tpb} {precision} complex={cplx}: rel error {rel:.2e}, sweeps max {sw.max()}")
    assert rel < TOL[precision] * (4 if precision == "fp64" else 1)
    assert sw.max() < 40


@pytest.mark.parametrize("tpb", [64, 128])
def test_degenerate_inputs(vemb, tpb):
    n = 64
    rng = np.random.default_rng([synth.BASE_SEED, 72])
    B = rng.standard_normal((n, n))
    S = B @ B.T / n
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    rep = Q @ np.diag([1.0] * 20 + [-1.0] * 20 + [0.0] * 24) @ Q.T
    cases = np.stack([np.zeros((n, n)), S, -S, rep, np.eye(n), -np.eye(n)])
    got, _ = _project(vemb, cases, False, "fp64", tpb)
    assert np.abs(got - psd_project(cases)).max() < 1e-12 * 4
    assert np.abs(got[0]).max() == 0.0


@pytest.mark.parametrize("tpb", [64, 128])
@pytest.mark.parametrize("cplx", [False, True])
def test_exactly_singular_shift(vemb, tpb, cplx):
    """x P_singlet + y P_triplet blocks (the Gershgorin shift equals -lambda_min) tiled to 64 x 64."""
    v = np.array([0.0, 1.0, -1.0, 0.0]) / np.sqrt(2.0)
    Ps = np.outer(v, v)
    cases = []
    for x, y in [(0.238, -1.61), (1.0, -1.0)]:
        C = np.kron(np.eye(16), x * Ps + y * (np.eye(4) - Ps))
        if cplx:
            D = np.diag(np.exp(1j * np.linspace(0.3, 2.9, 64)))
            C = D @ C @ D.conj().T
        cases.append(C)
    cases = np.stack(cases)
    got, sw = _project(vemb, cases, cplx, "fp64", tpb, max_sweeps=400)
    assert np.abs(got - psd_project(cases)).max() < 1e-14 * 64
    assert sw.max() < 10


@pytest.mark.parametrize("tpb", [64, 128])
def test_bench_ring_iterations(vemb, tpb):
    """5 iterations of the N = 384, L = 3 ring (pair and momentum blocks 64 x 64) against the oracle,
    then 40 warm-started iterations against cold-started ones."""
    w = synth.config_c2(1.0)[1]
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, 5)
    with vemb.Problem.from_workload(w, tpb=tpb) as g:
        assert vemb.problem_threads(g.h) == (tpb, tpb)
        g.step(5)
        st = g.get_state()
        lb = g.dual_bound()
    lb_o = alg6.lower_bound(p, s)
    assert abs(lb - lb_o) <= 1e-10 * abs(lb_o)
    for k, ref in [("X", s.X), ("rho_t", s.rho_t), ("Lam", s.Lam), ("Lam1", s.Lam1)]:
        assert np.abs(st[k] - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max()), k
    with vemb.Problem.from_workload(w, tpb=tpb) as a, vemb.Problem.from_workload(w, tpb=tpb, warm_refresh=-1) as b:
        a.step(40)
        b.step(40)
        sa, sb = a.get_state(), b.get_state()
        print(f"tpb {tpb}: sweeps warm {a.last_sweeps()} cold {b.last_sweeps()}")
        assert max(a.last_sweeps()) < max(b.last_sweeps())
    for k in ("X", "rho0", "rho_t", "Lam", "Lam1", "Lam2"):
        assert np.abs(sa[k] - sb[k]).max() < 1e-11 * max(1.0, np.abs(sb[k]).max()), k
