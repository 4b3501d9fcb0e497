"""Learned warm start on the GPU against the FP64 oracles (oracle/mlp.py, oracle/warm.py).

* Network forward, gradients and Adam: FP32 kernels with bfloat16-read weights against FP64
  on the same rounded weights.  Tolerances: outputs 1e-5 and gradients 1e-4 of each
  layer's largest entry (FP32 accumulation over at most a few hundred terms), parameters
  after Adam 1e-6 of the learning rate.
* State encoding / decoding: the GPU's encoding of its own state against the oracle's
  encoding of the same state (FP32 rounding, 1e-6 relative); decoding a seeded vector
  against the oracle's decoding, 1e-10 of each array's largest entry (FP64 after the
  FP32 input; the X projection by Jacobi against LAPACK).
* The learned start on a small family: a network trained by these kernels on solver
  states reaches a fixed certified-bound gap in fewer iterations than the cold start.
"""
import numpy as np
import pytest

import synth
from oracle import alg6, mlp, warm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vemb():
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a GPU")
    from paper_2106_02682_amd import vemb as v

    v.lib()
    return v


def _rel(a, b):
    return np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("dims,B", [([37, 70], 19), ([7, 256, 256, 256, 300], 130), ([9, 64, 1], 65)])
def test_forward_matches_oracle(vemb, dims, B):
    flat = synth.mlp_init(dims, tag=31)
    x = synth.mlp_batch(dims[0], B, tag=32)
    with vemb.MLP(dims, flat, max_batch=256) as net:
        mean = np.linspace(-1, 1, dims[-1]).astype(np.float32)
        std = np.linspace(0.5, 2, dims[-1]).astype(np.float32)
        net.set_normalization(mean, std)
        xd = torch.from_numpy(x).cuda()
        y = torch.empty((B, dims[-1]), dtype=torch.float32, device="cuda")
        net.forward(xd, y)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
    want = mlp.predict(mlp.unflatten(flat, dims), x, mean.astype(np.float64), std.astype(np.float64))
    err = _rel(got, want)
    print(f"forward {dims} B={B}: max rel error {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("dims,B", [([5, 64, 48, 33], 37), ([7, 256, 256, 256, 520], 96), ([7, 64, 64, 2600], 40)])
def test_gradients_match_oracle(vemb, dims, B):
    flat = synth.mlp_init(dims, tag=41)
    x = synth.mlp_batch(dims[0], B, tag=42)
    t = synth.mlp_batch(dims[-1], B, tag=43) * 0.5 + 0.1
    t[:, 3] = 0.25  # a constant output: std from the floor (the K = 2600 case exercises split-K)
    with vemb.MLP(dims, flat, max_batch=128) as net:
        td = torch.from_numpy(t).cuda()
        net.fit_normalization(td, 1e-2)
        mean, std = net.get_normalization()
        g = torch.empty(net.num_params, dtype=torch.float32, device="cuda")
        loss = net.gradients(torch.from_numpy(x).cuda(), td, g)
        got = g.cpu().numpy()
    m_o, s_o = mlp.normalisation(t, 1e-2)
    assert _rel(mean, m_o) < 1e-6 and _rel(std, s_o) < 1e-6 and std[3] == pytest.approx(1e-2 * s_o.max(), rel=1e-6)
    loss_o, grads = mlp.loss_and_grads(mlp.unflatten(flat, dims), x, t, mean.astype(np.float64),
                                       std.astype(np.float64))
    assert abs(loss - loss_o) <= 1e-5 * loss_o
    gl = mlp.unflatten(got, dims)
    for l, ((gW, gb), (oW, ob)) in enumerate(zip(gl, grads)):
        eW, eb = _rel(gW, oW), _rel(gb, ob)
        print(f"gradients {dims} layer {l}: W rel {eW:.2e}, b rel {eb:.2e}")
        assert eW < 1e-4 and eb < 1e-4


def test_adam_matches_oracle(vemb):
    dims = [5, 32, 17]
    flat = synth.mlp_init(dims, tag=51)
    x = torch.from_numpy(synth.mlp_batch(5, 24, tag=52)).cuda()
    t = torch.from_numpy(synth.mlp_batch(17, 24, tag=53)).cuda()
    lr = 3e-3
    with vemb.MLP(dims, flat, max_batch=32) as net:
        opt = mlp.Adam(flat.size)
        theta = flat.astype(np.float64)
        for step in range(3):
            g = torch.empty(net.num_params, dtype=torch.float32, device="cuda")
            net.gradients(x, t, g)
            net.adam_step(lr)
            theta = opt.step(theta, g.cpu().numpy(), lr)
            got = net.get_params()
            err = np.abs(got - theta).max() / lr
            print(f"Adam step {step + 1}: max |theta - oracle| / lr = {err:.2e}")
            assert err < 1e-4


def test_train_step_gathers_rows_and_descends(vemb):
    dims = [5, 64, 64, 40]
    flat = synth.mlp_init(dims, tag=61)
    X = torch.from_numpy(synth.mlp_batch(5, 50, tag=62)).cuda()
    T = torch.from_numpy(np.tanh(synth.mlp_batch(40, 50, tag=63))).cuda()
    rows = torch.tensor([3, 7, 7, 49, 0, 12, 31, 44], dtype=torch.int32, device="cuda")
    with vemb.MLP(dims, flat, max_batch=64) as a, vemb.MLP(dims, flat, max_batch=64) as b:
        a.fit_normalization(T)
        b.fit_normalization(T)
        la = a.train_step(X, T, rows=rows, lr=1e-3, want_loss=True)
        lb = b.gradients(X[rows.long()].contiguous(), T[rows.long()].contiguous())
        b.adam_step(1e-3)
        assert la == pytest.approx(lb, rel=1e-12)
        assert np.array_equal(a.get_params(), b.get_params())
        first = a.train_step(X, T, lr=3e-3, want_loss=True)
        for _ in range(200):
            last = a.train_step(X, T, lr=3e-3, want_loss=True)
        print(f"full-batch loss {first:.3e} -> {last:.3e}")
        assert last < 0.5 * first


@pytest.mark.parametrize("N,near", [(16, 3), (22, 3), (32, 3), (22, 5), (32, 8), (32, 12)])
def test_encode_matches_oracle(vemb, N, near):
    w = synth.tfi_ring(N, 2, 0.8)
    p = alg6.Problem.from_workload(w)
    with vemb.Problem.from_workload(w) as g:
        g.step(40)
        st = g.get_state()
        v = torch.empty(vemb.warm_size(g.h, near), dtype=torch.float32, device="cuda")
        vemb.warm_encode(g.h, v, near)
        torch.cuda.synchronize()
        got = v.cpu().numpy()
    s = alg6.State(40, st["X"], st["rho0"], st["rho"], st["rho_t"], st["Lam"], st["Lam1"], st["Lam2"])
    want = warm.encode(p, s, near)
    assert got.size == want.size == warm.sizes(p, near)[0]
    assert np.abs(got - want).max() <= 1e-6 * np.abs(want).max()


@pytest.mark.parametrize("N,L,near,far_cold", [(16, 2, 3, False), (22, 2, 3, False), (32, 2, 3, False),
                                                (24, 3, 3, False), (22, 2, 5, False), (32, 2, 8, False),
                                                (32, 2, 3, True), (24, 3, 2, True), (22, 2, 5, True)])
def test_decode_matches_oracle(vemb, N, L, near, far_cold):
    w = synth.tfi_ring(N, L, 1.0)
    p = alg6.Problem.from_workload(w)
    vec = (np.random.default_rng([synth.BASE_SEED, 16, N, L]).standard_normal(warm.sizes(p, near)[0]) * 0.2)
    vec = vec.astype(np.float32)
    with vemb.Problem.from_workload(w) as g:
        vemb.warm_start(g.h, torch.from_numpy(vec).cuda(), near, far_cold=far_cold)
        st = g.get_state()
        lb = g.dual_bound()
    s = warm.decode(p, vec.astype(np.float64), near, far_cold=far_cold)
    for k in ("X", "rho0", "rho_t", "rho", "Lam", "Lam1", "Lam2"):
        err = np.abs(st[k] - getattr(s, k)).max() / max(np.abs(getattr(s, k)).max(), 1e-30)
        assert err < 1e-10, (k, err)
    assert lb == pytest.approx(alg6.lower_bound(p, s), rel=1e-10)
