"""Pins of the MLP oracle (finite differences, Adam closed forms) and of the TD oracle (special cases)."""
import numpy as np

from oracle import mlp, td


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(7, 16, seed=1)
    for k in p:
        p[k] = p[k] + 0.1 * rng.normal(size=p[k].shape)
    X = rng.normal(size=(11, 7)); Y = rng.normal(size=(11, 3))
    L, g = mlp.loss_and_grad(p, X, Y)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h; Lp, _ = mlp.loss_and_grad(p, X, Y)
            flat[idx] = old - h; Lm, _ = mlp.loss_and_grad(p, X, Y)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-7 * max(1e-3, abs(fd)) + 1e-10


def test_mlp_forward_closed_form():
    """A hand-built network whose pre-activations land on 0 and +-ln 3, where silu is exact:
    silu(0) = 0, silu(ln 3) = (3/4) ln 3 (sigmoid(ln 3) = 3/4), silu(-ln 3) = -(1/4) ln 3.  Pins the
    composition (bias after each product, silu on the hidden layers only, X W row convention)."""
    l3 = np.log(3.0)
    p = dict(W1=np.eye(2), b1=np.array([1.0, -2.0]),
             W2=np.array([[(l3 - 1) / (0.75 * l3), (1 - l3) / (0.75 * l3)], [5.0, 7.0]]), b2=np.array([1.0, -1.0]),
             W3=np.array([[1.0, 0.0, 2.0], [0.0, 1.0, 2.0]]), b3=np.array([0.5, 0.0, -1.0]))
    X = np.array([[l3 - 1.0, 2.0]])     # z1 = (ln 3, 0), h1 = ((3/4) ln 3, 0)
    y, (_, z1, h1, z2, h2) = mlp.forward(p, X)
    assert np.allclose(z1, [[l3, 0.0]], rtol=1e-15, atol=1e-15)
    assert np.allclose(z2, [[l3, -l3]], rtol=1e-14, atol=1e-15)
    assert np.allclose(h2, [[0.75 * l3, -0.25 * l3]], rtol=1e-14)
    assert np.allclose(y, [[0.75 * l3 + 0.5, -0.25 * l3, l3 - 1.0]], rtol=1e-14)


def test_silu_grad():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.silu_grad(z)).max() < 1e-9


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g, bias-corrected moments are exactly g and g^2 at every step,
    so each step moves a parameter by -lr g / (|g| + eps)."""
    p = {"w": np.array([0.5, -1.0, 2.0])}
    g = {"w": np.array([0.3, -2.0, 1e-3])}
    opt = mlp.Adam(p, lr=0.01, eps=1e-8)
    w0 = p["w"].copy()
    for t in range(1, 6):
        p = opt.step(p, g)
        expect = w0 - t * 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
        assert np.allclose(p["w"], expect, rtol=1e-12, atol=1e-14)


def test_td_special_cases():
    E, nu, s = 2.6, 0.3, 1.7
    hyd = np.array([s, s, s, 0, 0, 0])
    assert np.isclose(td.topological_derivative(hyd, E, nu), 9 * (1 - nu) * s * s / (4 * E), rtol=1e-14)
    uni = np.array([s, 0, 0, 0, 0, 0])
    assert np.isclose(td.topological_derivative(uni, E, nu),
                      3 * (1 - nu) * (9 + 5 * nu) * s * s / (4 * E * (7 - 5 * nu)), rtol=1e-14)
    # pure shear tau: sig:sig = 2 tau^2, tr = 0
    sh = np.array([0, 0, 0, 0, 0, s])
    assert np.isclose(td.topological_derivative(sh, E, nu),
                      3 * (1 - nu) * 20 * (1 + nu) * s * s / (4 * E * (7 - 5 * nu)), rtol=1e-14)
    # invariance under rotation of the stress tensor
    rng = np.random.default_rng(2)
    A = rng.normal(size=(3, 3)); S = A + A.T
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    S2 = Q @ S @ Q.T
    v = lambda M: np.array([M[0, 0], M[1, 1], M[2, 2], M[1, 2], M[0, 2], M[0, 1]])
    assert np.isclose(td.topological_derivative(v(S), E, nu), td.topological_derivative(v(S2), E, nu), rtol=1e-12)


def test_removal_rule_strict():
    t = np.array([0.0, 1.0, 2.0, 10.0])
    assert list(td.removal_mask(t, 0.1)) == [True, False, False, False]  # threshold 1.0, strict
    assert list(td.removal_mask(t, 0.0)) == [False, False, False, False]
