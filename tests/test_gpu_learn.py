"""Warm-start network kernels (ws_*) vs the FP64 oracle MLP (oracle/mlp.py), feature matching vs a brute-force
nearest-centroid search, and the residual guard inside bem_solve."""
import numpy as np
import pytest
import torch

from oracle import mlp as om
from workloads import geometry as geo

pytestmark = pytest.mark.gpu


def _oracle_params_from_flat(flat, din=16, W=128):
    o = 0
    p = {}
    for name, shape in (("W1", (din, W)), ("b1", (W,)), ("W2", (W, W)), ("b2", (W,)), ("W3", (W, 3)), ("b3", (3,))):
        size = int(np.prod(shape))
        p[name] = flat[o:o + size].astype(np.float64).reshape(shape)
        o += size
    return p


def _flat(p):
    return np.concatenate([p[k].reshape(-1) for k in om.PARAM_NAMES]).astype(np.float32)


@pytest.fixture
def net(cuda):
    from paper_1612_04082_amd import kfmm
    n = kfmm.WarmStartNet(seed=1)
    p = om.init_params(16, 128, seed=3)
    rng = np.random.default_rng(4)
    for k in p:  # non-zero biases and last layer so every gradient is exercised
        p[k] = p[k] + 0.05 * rng.normal(size=p[k].shape)
    n.set_params(_flat(p))
    yield n, _oracle_params_from_flat(_flat(p))
    n.close()


def _batch(n=3000, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 16)).astype(np.float32)
    R = (0.3 * rng.normal(size=(n, 3))).astype(np.float32)
    return X, R


def test_loss_and_gradient_match_oracle(net):
    g_net, p = net
    X, R = _batch()
    L, g = g_net.loss_grad(torch.tensor(X, device="cuda"), torch.tensor(R, device="cuda"))
    Lo, go = om.loss_and_grad(p, X.astype(np.float64), R.astype(np.float64))
    gflat = np.concatenate([go[k].reshape(-1) for k in om.PARAM_NAMES])
    print(f"loss gpu {L:.8f} oracle {Lo:.8f}; grad rel err {np.linalg.norm(g - gflat) / np.linalg.norm(gflat):.2e}")
    assert abs(L - Lo) <= 1e-5 * abs(Lo)
    assert np.linalg.norm(g - gflat) <= 1e-4 * np.linalg.norm(gflat)
    for k in om.PARAM_NAMES:  # every block, not only the norm
        a = g[_slice(k)]
        b = go[k].reshape(-1)
        assert np.linalg.norm(a - b) <= 2e-4 * max(np.linalg.norm(b), 1e-12), k


def _slice(name, din=16, W=128):
    sizes = {"W1": din * W, "b1": W, "W2": W * W, "b2": W, "W3": W * 3, "b3": 3}
    o = 0
    for k in om.PARAM_NAMES:
        if k == name:
            return slice(o, o + sizes[k])
        o += sizes[k]


def test_adam_steps_match_oracle(net):
    g_net, p = net
    X, R = _batch(2000, seed=1)
    scale = 2.0
    xm = np.random.default_rng(5).normal(size=(2000, 3))
    xt = xm + scale * R.astype(np.float64)
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")
    g_net.train(dev(X, torch.float32), dev(xm, torch.float64), dev(xt, torch.float64), scale, epochs=3, lr=1e-2)
    opt = om.Adam(p, lr=1e-2)
    Rr = ((xt - xm) / scale).astype(np.float32).astype(np.float64)
    for _ in range(3):
        _, g = om.loss_and_grad(p, X.astype(np.float64), Rr)
        p = opt.step(p, g)
    got = g_net.get_params()
    ref = _flat(p).astype(np.float64)
    err = np.abs(got - ref).max()
    print(f"after 3 Adam steps: max |param - oracle| = {err:.2e}")
    assert err < 2e-4  # steps are lr-sized (1e-2); FP32 gradients agree to ~1e-4 relative


def test_bf16_inference_matches_fp32_forward(net):
    g_net, p = net
    X, _ = _batch(5000, seed=2)
    xm = np.random.default_rng(6).normal(size=(5000, 3))
    scale = 0.7
    x0 = g_net.predict(torch.tensor(X, device="cuda"), torch.tensor(xm, device="cuda"), scale).cpu().numpy()
    y, _ = om.forward(p, X.astype(np.float64))
    ref = xm + scale * y
    err = np.linalg.norm((x0 - xm) - (ref - xm)) / np.linalg.norm(ref - xm)
    print(f"BF16 inference vs FP64 forward: rel err of the correction {err:.2e}")
    assert err < 2e-2


def test_features_match_brute_force(cuda):
    from paper_1612_04082_amd import kfmm
    M = np.ones((12, 4, 4), bool)
    M2 = M.copy()
    M2[5:7, 1:3, 3] = False  # a notch: new faces appear, some vanish
    p1 = geo.cantilever_problem(M, 0.5)
    p2 = geo.cantilever_problem(M2, 0.5)
    rng = np.random.default_rng(7)
    T1 = p1["tri"].shape[0]
    u1 = rng.normal(size=(T1, 3))
    t1 = rng.normal(size=(T1, 3))
    d = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    prev = dict(tri=d(p1["tri"]), bc_type=d(p1["bc_type"], torch.int8), bc_val=d(p1["bc_val"]))
    nxt = dict(tri=d(p2["tri"]), bc_type=d(p2["bc_type"], torch.int8), bc_val=d(p2["bc_val"]))
    feat, xm, scale = kfmm.ws_features(prev, d(u1), d(t1), nxt)
    feat, xm = feat.cpu().numpy(), xm.cpu().numpy()
    c1 = p1["tri"].mean(1)
    c2 = p2["tri"].mean(1)
    D = np.linalg.norm(c2[:, None, :] - c1[None, :, :], axis=2)
    j = np.argmin(D, axis=1)
    dist = D[np.arange(len(c2)), j]
    exact = dist == 0
    assert exact.sum() > 0.8 * len(c2)
    expect = np.where(p2["bc_type"] == 0, t1[j], u1[j])
    # elements with a unique nearest neighbour must map exactly
    second = np.partition(D, 1, axis=1)[:, 1]
    uniq = second > dist + 1e-9
    assert np.array_equal(xm[uniq], expect[uniq])
    assert np.allclose(feat[:, 3], dist / np.mean(np.linalg.norm(p2["tri"] - np.roll(p2["tri"], -1, 1), axis=2)),
                       rtol=1e-5, atol=1e-6)
    assert np.isclose(scale, np.sqrt(np.mean(xm ** 2)), rtol=1e-12)
    assert np.allclose(feat[:, 10:13], xm / scale, rtol=1e-6, atol=1e-6)


def test_guard_picks_better_start_and_save_load(cuda, tmp_path):
    from paper_1612_04082_amd import kfmm
    p = geo.cube_tension_problem(2)
    d = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    args = (d(p["tri"]), d(p["bc_type"], torch.int8), d(p["bc_val"]))
    x, u, t, st = kfmm.bem_solve(*args, tol=1e-8, precision=0)
    bad = torch.full_like(x, 1e3)
    # the minimal-residual combination of the two starts recovers the solution: no iteration needed
    x2, _, _, st2 = kfmm.bem_solve(*args, tol=1e-8, precision=0, x0=bad, x0_alt=x)
    assert st2["iters"] == 0 and abs(st2["start_coef"][1] - 1.0) < 1e-6 and abs(st2["start_coef"][0]) < 1e-6
    x3, _, _, st3 = kfmm.bem_solve(*args, tol=1e-8, precision=0, x0=x, x0_alt=bad)
    assert st3["iters"] == 0 and st3["rel_res_alt"] > 1.0
    # a scaled solution is rescaled by the projection
    x4, _, _, st4 = kfmm.bem_solve(*args, tol=1e-8, precision=0, x0=3.0 * x)
    assert st4["iters"] == 0 and abs(st4["start_coef"][0] - 1.0 / 3.0) < 1e-8
    n1 = kfmm.WarmStartNet(seed=5)
    n1.save(tmp_path / "net.bin")
    n2 = kfmm.WarmStartNet(seed=9)
    assert not np.array_equal(n1.get_params(), n2.get_params())
    n2.load(tmp_path / "net.bin")
    assert np.array_equal(n1.get_params(), n2.get_params())
