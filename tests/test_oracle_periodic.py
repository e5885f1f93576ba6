"""Pins of the periodic (Ewald) oracle, oracle/periodic.py, against facts that do not come from it.

  * the tensor algebra that builds U, P, D, S from the two radial families equals the free-space oracle
    (oracle/direct.c, itself pinned by tests/test_oracle_kernels.py) when the radial functions are the
    plain 1/r and r;
  * the Ewald splitting parameter drops out (real-space and reciprocal parts, and the constant of the left
    out k = 0 term, must fit together);
  * periodicity in every lattice direction;
  * closed forms of the periodic field of a closed surface in the cell (Sec. 4.3: integrals over the
    infinite periodic surface).  A compactly supported free-space field F has the periodic sum
    "periodised F minus its cell mean" under the k = 0 reading.  For a sphere of volume |O| in a cell of
    volume V: a constant double-layer density gives -e_k (1 - |O|/V) inside and e_k |O|/V outside, and
    the Somigliana data of a linear field u = A x + c gives chi (A xi + c) - (|O|/V)(A x_O + c) in
    displacement (x_O the centre) and exactly chi sigma in stress (the distributional gradient of a
    periodic field has zero mean);
  * Navier's equation with the uniform balancing body force: for one point force F, away from it,
    G lap v + (K + G/3) grad div v = F / V;
  * the coincident source: the periodic field minus the free-space kernel tends to the value with the
    n = 0 image left out.
"""
import numpy as np
import pytest

from oracle import direct as od
from oracle import periodic as op
from tests.quadrature import VOIGT, sphere_rule, stiffness

G = 1.0
K = od.moduli(G, 0.3)


@pytest.fixture(scope="module")
def cloud():
    rng = np.random.default_rng(1)
    N = 60
    src = rng.uniform(size=(N, 3)) * 1.3
    nrm = rng.normal(size=(N, 3))
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    return dict(src=src, nrm=nrm, w=rng.uniform(size=N), a=rng.normal(size=(N, 3)), b=rng.normal(size=(N, 3)),
                trg=rng.uniform(size=(7, 3)) * 1.3)


@pytest.mark.parametrize("kind", [od.DISP, od.STRESS])
def test_free_space_algebra_equals_direct(cloud, kind):
    c = cloud
    f = op.periodic(kind, c["trg"], c["src"], c["w"], a=c["a"], b=c["b"], nrm=c["nrm"], K=K, G=G, L=1.3,
                    free_space=True)
    g = od.direct(kind, c["trg"], c["src"], c["w"], a=c["a"], b=c["b"], nrm=c["nrm"], K=K, G=G)
    assert np.abs(f - g).max() < 1e-13 * np.abs(g).max()


@pytest.mark.parametrize("kind", [od.DISP, od.STRESS])
def test_splitting_parameter_drops_out_and_lattice_period(cloud, kind):
    """Densities with a net force per cell included (the balancing body force is part of the definition)."""
    c = cloud
    L = 1.3
    r = [op.periodic(kind, c["trg"], c["src"], c["w"], a=c["a"], b=c["b"], nrm=c["nrm"], K=K, G=G, L=L, alpha_L=aL)
         for aL in (3.5, 5.0, 7.0)]
    scale = np.abs(r[1]).max()
    assert np.abs(r[0] - r[1]).max() < 1e-12 * scale
    assert np.abs(r[2] - r[1]).max() < 1e-12 * scale
    for shift in ([L, 0, 0], [0, -L, 0], [0, 0, 2 * L], [L, L, -L]):
        s = op.periodic(kind, c["trg"] + np.array(shift), c["src"], c["w"], a=c["a"], b=c["b"], nrm=c["nrm"], K=K,
                        G=G, L=L)
        assert np.abs(s - r[1]).max() < 1e-12 * scale


@pytest.fixture(scope="module")
def sphere_in_cell():
    L, R = 2.0, 0.55
    c = np.array([1.0, 0.9, 1.1])
    pts, nrm, w = sphere_rule(R=R, n_theta=48, n_phi=96, center=tuple(c))
    inside = c + np.array([[0, 0, 0], [0.2, -0.1, 0.15], [0.0, 0.3, -0.2]])
    outside = np.array([[0.1, 0.1, 0.1], [1.9, 0.2, 1.0], [1.0, 1.8, 0.1], [2.3, 2.2, 2.1]])
    return dict(L=L, c=c, pts=pts, nrm=nrm, w=w, inside=inside, outside=outside,
                frac=4.0 / 3.0 * np.pi * R ** 3 / L ** 3)


def test_periodic_double_layer_jump(sphere_in_cell):
    s = sphere_in_cell
    for k in range(3):
        b = np.zeros_like(s["pts"])
        b[:, k] = 1.0
        e = np.zeros(3)
        e[k] = 1.0
        vin = op.periodic(od.DISP, s["inside"], s["pts"], s["w"], b=b, nrm=s["nrm"], K=K, G=G, L=s["L"])
        vout = op.periodic(od.DISP, s["outside"], s["pts"], s["w"], b=b, nrm=s["nrm"], K=K, G=G, L=s["L"])
        assert np.abs(vin + e * (1.0 - s["frac"])).max() < 1e-12
        assert np.abs(vout - e * s["frac"]).max() < 1e-12


@pytest.mark.parametrize("case", ["translation", "rotation", "strain"])
def test_periodic_somigliana(sphere_in_cell, case):
    s = sphere_in_cell
    rng = np.random.default_rng(3)
    if case == "translation":
        A = np.zeros((3, 3)); c0 = rng.normal(size=3)
    elif case == "rotation":
        Wm = rng.normal(size=(3, 3)); A = Wm - Wm.T; c0 = np.zeros(3)
    else:
        A = rng.normal(size=(3, 3)); c0 = rng.normal(size=3)
    C = stiffness(K, G)
    sig = np.einsum("ijkl,kl->ij", C, 0.5 * (A + A.T))
    u = s["pts"] @ A.T + c0
    t = s["nrm"] @ sig.T
    xi = np.vstack([s["inside"], s["outside"]])
    chi = np.r_[np.ones(len(s["inside"])), np.zeros(len(s["outside"]))]
    v = op.periodic(od.DISP, xi, s["pts"], s["w"], a=t, b=-u, nrm=s["nrm"], K=K, G=G, L=s["L"])
    ref = chi[:, None] * (xi @ A.T + c0) - s["frac"] * (A @ s["c"] + c0)
    assert np.abs(v - ref).max() < 1e-12 * max(1.0, np.abs(u).max())
    st = op.periodic(od.STRESS, xi, s["pts"], s["w"], a=t, b=-u, nrm=s["nrm"], K=K, G=G, L=s["L"])
    sv = np.array([sig[i, j] for (i, j) in VOIGT])
    assert np.abs(st - chi[:, None] * sv[None]).max() < 1e-11 * max(1.0, np.abs(sig).max())


def test_navier_with_balancing_body_force():
    L = 2.0
    y = np.array([[0.3, 0.4, 0.5]])
    F = np.array([[0.2, -1.0, 0.5]])
    x0 = np.array([1.3, 1.1, 0.9])
    h = 1e-3

    def v(x):
        return op.periodic(od.DISP, x[None], y, np.ones(1), a=F, K=K, G=G, L=L)[0]

    H = np.zeros((3, 3, 3))
    for m in range(3):
        for q in range(3):
            em = np.zeros(3); em[m] = h
            eq = np.zeros(3); eq[q] = h
            H[m, q] = (v(x0 + em + eq) - v(x0 + em - eq) - v(x0 - em + eq) + v(x0 - em - eq)) / (4 * h * h)
    res = (K + G / 3.0) * np.einsum("mqq->m", H) + G * (H[0, 0] + H[1, 1] + H[2, 2])
    assert np.abs(res - F[0] / L ** 3).max() < 1e-4 * np.abs(F).max() / L ** 3  # second-order differences


@pytest.mark.parametrize("kind,layer,d", [(od.DISP, "a", 1e-2), (od.DISP, "b", 1e-3), (od.STRESS, "a", 1e-3),
                                          (od.STRESS, "b", 1e-2)])
def test_coincident_source_limit(kind, layer, d):
    """One source and its images: periodic(xi) - free(xi) -> periodic(y) (n = 0 image left out) as xi -> y.
    The difference is smooth; its even parts (U, and the second derivatives in S) close like d^2, its odd
    parts (P, D, zero at the source) like d: the gap must fall at least 8-fold from d to d/10."""
    rng = np.random.default_rng(4)
    L = 2.0
    y = rng.uniform(size=(1, 3)) * L
    w = np.array([0.7])
    dens = rng.normal(size=(1, 3))
    n = rng.normal(size=(1, 3)); n /= np.linalg.norm(n)
    kw = dict(a=dens) if layer == "a" else dict(b=dens, nrm=n)
    e = rng.normal(size=3); e /= np.linalg.norm(e)
    pc = op.periodic(kind, y, y, w, K=K, G=G, L=L, **kw)
    gaps = []
    for dd in (d, d / 10):
        xt = y + dd * e
        pn = op.periodic(kind, xt, y, w, K=K, G=G, L=L, **kw)
        fr = od.direct(kind, xt, y, w, K=K, G=G, **kw)
        gaps.append(np.abs(pn - fr - pc).max())
    assert gaps[1] < gaps[0] / 8 and gaps[1] < 1e-4
