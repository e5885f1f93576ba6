"""Pins of the FP64 direct-summation oracle against facts the mathematics fixes.

Each kernel of the oracle (eqs. disp_1, disp_2, stress_2, stress_3) is checked against a
relation that does not restate its formula:
  * U: symmetry, reciprocity, 1/r homogeneity, Navier's equation (finite differences);
  * D = C : grad_target U and S = C : grad_target P (finite differences, eq. elast for C);
  * P = traction, at the source point, of the point-force field whose stress is D;
  * the double-layer jump identity  int_Gamma P = -I inside, 0 outside (Sec. 2.1, eq. BIE with
    a rigid translation);
  * Somigliana reproduction of rigid motions and uniform strain, in displacement (eq. BIE, interior
    form) and in stress (eq. stress_1);
  * zero divergence of the stress field of a random source set (first line of eq. elast).
A dropped term, a wrong sign, a swapped index or a wrong prefactor in any kernel fails at least one.
"""
import numpy as np
import pytest

from oracle import direct as od
from tests.quadrature import sphere_rule, stiffness, VOIGT

G = 1.0
NU = 0.3
K = od.moduli(G, NU)


def _fd(fun, x, h=1e-3):
    """Fourth-order central differences of fun at x along each axis -> list of 3 arrays."""
    out = []
    for m in range(3):
        e = np.zeros(3); e[m] = h
        out.append((-fun(x + 2 * e) + 8 * fun(x + e) - 8 * fun(x - e) + fun(x - 2 * e)) / (12 * h))
    return out


def _one(trg, src, nrm):
    return od.pair_kernels(trg[None], src[None], nrm[None], K, G)


@pytest.fixture(scope="module")
def pairs():
    rng = np.random.default_rng(11)
    trg = rng.normal(size=(6, 3))
    src = trg + rng.normal(size=(6, 3)) * 0.8 + 0.3
    nrm = rng.normal(size=(6, 3)); nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    return trg, src, nrm


def test_U_symmetric_reciprocal_homogeneous(pairs):
    trg, src, nrm = pairs
    U, _, _, _ = od.pair_kernels(trg, src, nrm, K, G)
    U2, _, _, _ = od.pair_kernels(src, trg, nrm, K, G)
    assert np.allclose(U, np.transpose(U, (0, 2, 1)), rtol=1e-14, atol=0)
    assert np.allclose(U, U2, rtol=1e-14, atol=0)
    U3, _, _, _ = od.pair_kernels(2.5 * trg, 2.5 * src, nrm, K, G)
    assert np.allclose(U3 * 2.5, U, rtol=1e-13)


def test_U_solves_navier(pairs):
    """(K + G/3) grad div u + G lap u = 0 for each column of U, away from the source."""
    trg, src, nrm = pairs
    h = 2e-3
    for t, s, n in zip(trg, src, nrm):
        def Ufun(x):
            return _one(x, s, n)[0][0]  # U[i, j]: column j is the field of a force along j

        # second derivatives by nested 5-point differences
        H = np.zeros((3, 3, 3, 3))  # [m, q, i, j] = d2 U_ij / dx_m dx_q
        for m in range(3):
            em = np.zeros(3); em[m] = h
            for q in range(3):
                eq = np.zeros(3); eq[q] = h
                f = lambda a, b: Ufun(t + a * em + b * eq)
                H[m, q] = (f(1, 1) - f(1, -1) - f(-1, 1) + f(-1, -1)) / (4 * h * h)
        lap = H[0, 0] + H[1, 1] + H[2, 2]
        grad_div = np.einsum("mqqj->mj", H)  # d/dx_m sum_q dU_qj/dx_q
        res = (K + G / 3.0) * grad_div + G * lap
        scale = np.abs(G * lap).max()
        assert np.abs(res).max() < 1e-4 * scale


def test_D_is_stiffness_times_grad_U(pairs):
    trg, src, nrm = pairs
    C = stiffness(K, G)
    for t, s, n in zip(trg, src, nrm):
        dU = _fd(lambda x: _one(x, s, n)[0][0], t)  # dU[m][l,k]
        gradU = np.stack(dU, axis=-1)  # [l,k,m]
        D_fd = np.einsum("ijlm,lkm->kij", C, gradU)
        D = _one(t, s, n)[2][0]
        assert np.abs(D - D_fd).max() < 1e-9 * np.abs(D).max()


def test_S_is_stiffness_times_grad_P(pairs):
    trg, src, nrm = pairs
    C = stiffness(K, G)
    for t, s, n in zip(trg, src, nrm):
        dP = _fd(lambda x: _one(x, s, n)[1][0], t)
        gradP = np.stack(dP, axis=-1)
        S_fd = np.einsum("ijlm,lkm->kij", C, gradP)
        S = _one(t, s, n)[3][0]
        assert np.abs(S - S_fd).max() < 1e-8 * np.abs(S).max()


def test_P_is_traction_of_point_force_field(pairs):
    """P_ij(xi, x; n) = sigma^(i)_jk(x) n_k where sigma^(i) is the stress at x of a unit force e_i at xi."""
    trg, src, nrm = pairs
    _, P, _, _ = od.pair_kernels(trg, src, nrm, K, G)
    # stress at x (target) of a point force at xi (source): D with the roles swapped
    _, _, Dsw, _ = od.pair_kernels(src, trg, nrm, K, G)  # Dsw[p, i, j, k]: force direction i
    trac = np.einsum("pijk,pk->pij", Dsw, nrm)
    assert np.allclose(P, trac, rtol=1e-12, atol=1e-14)


def test_double_layer_jump_identity():
    pts, nrm, w = sphere_rule(R=1.0, n_theta=48, n_phi=96)
    inside = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1], [0.0, 0.45, -0.3]])
    outside = np.array([[2.0, 0.0, 0.0], [1.5, 1.5, -0.5]])
    for k in range(3):
        b = np.zeros_like(pts); b[:, k] = 1.0
        vin = od.direct(od.DISP, inside, pts, w, b=b, nrm=nrm, K=K, G=G)
        vout = od.direct(od.DISP, outside, pts, w, b=b, nrm=nrm, K=K, G=G)
        e = np.zeros(3); e[k] = 1.0
        assert np.abs(vin + e[None, :]).max() < 1e-12
        assert np.abs(vout).max() < 1e-12


@pytest.mark.parametrize("case", ["translation", "rotation", "strain"])
def test_somigliana_displacement_and_stress(case):
    rng = np.random.default_rng(3)
    pts, nrm, w = sphere_rule(R=1.3, n_theta=48, n_phi=96, center=(0.2, -0.1, 0.05))
    C = stiffness(K, G)
    if case == "translation":
        A = np.zeros((3, 3)); c = rng.normal(size=3)
    elif case == "rotation":
        Wm = rng.normal(size=(3, 3)); A = Wm - Wm.T; c = np.zeros(3)
    else:
        A = rng.normal(size=(3, 3)); c = rng.normal(size=3)
    eps = 0.5 * (A + A.T)
    sig = np.einsum("ijkl,kl->ij", C, eps)
    u = pts @ A.T + c
    t = nrm @ sig.T  # t_i = sig_ij n_j
    xi = np.array([[0.2, -0.1, 0.05], [0.6, 0.2, -0.3], [-0.3, 0.1, 0.5]])
    v = od.direct(od.DISP, xi, pts, w, a=t, b=-u, nrm=nrm, K=K, G=G)
    assert np.abs(v - (xi @ A.T + c)).max() < 1e-11 * max(1.0, np.abs(u).max())
    s = od.direct(od.STRESS, xi, pts, w, a=t, b=-u, nrm=nrm, K=K, G=G)
    s_ref = np.array([sig[i, j] for (i, j) in VOIGT])
    assert np.abs(s - s_ref[None, :]).max() < 1e-10 * max(1.0, np.abs(sig).max())


def test_stress_divergence_free():
    rng = np.random.default_rng(5)
    src = rng.normal(size=(20, 3)) * 0.5
    nrm = rng.normal(size=(20, 3)); nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    w = rng.random(20); a = rng.normal(size=(20, 3)); b = rng.normal(size=(20, 3))
    x0 = np.array([2.0, 1.5, -1.0])

    def sig(x):
        s = od.direct(od.STRESS, x[None], src, w, a=a, b=b, nrm=nrm, K=K, G=G)[0]
        M = np.zeros((3, 3))
        for v, (i, j) in enumerate(VOIGT):
            M[i, j] = M[j, i] = s[v]
        return M

    d = _fd(sig, x0)  # d[m][i,j]
    div = sum(d[j][:, j] for j in range(3))
    assert np.abs(div).max() < 1e-8 * np.abs(sig(x0)).max()


def test_self_pair_skipped_and_kinds_linear():
    rng = np.random.default_rng(9)
    src = rng.normal(size=(30, 3))
    nrm = rng.normal(size=(30, 3)); nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    w = rng.random(30); a = rng.normal(size=(30, 3)); b = rng.normal(size=(30, 3))
    for kind in (od.DISP, od.STRESS):
        full = od.direct(kind, src, src, w, a=a, b=b, nrm=nrm, K=K, G=G)
        assert np.all(np.isfinite(full))
        sa = od.direct(kind, src, src, w, a=a, nrm=nrm, K=K, G=G)
        sb = od.direct(kind, src, src, w, b=b, nrm=nrm, K=K, G=G)
        assert np.allclose(full, sa + sb, rtol=1e-13, atol=1e-13)
        # target 0 against all other sources only, explicitly
        one = od.direct(kind, src[:1], src[1:], w[1:], a=a[1:], b=b[1:], nrm=nrm[1:], K=K, G=G)
        assert np.allclose(full[0], one[0], rtol=1e-14, atol=1e-14)
