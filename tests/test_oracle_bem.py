"""Pins of the dense BEM oracle (oracle/bem.py) against facts fixed by the mathematics.

  * the 4-point rule on 4 sub-triangles integrates all cubics exactly (reading of Sec. 2.2);
  * closed-form self integrals: int_T 1/r from the centroid of an equilateral triangle equals
    sqrt(3) a ln(2 + sqrt(3)); U_self equals a brute-force Duffy-transformed quadrature of U;
    P_self equals a brute-force polar quadrature of P over the triangle minus a small disk (the
    principal value), and vanishes for an equilateral triangle (symmetry);
  * the discrete system reproduces a rigid translation (Dirichlet u = c gives t ~ 0);
  * LU, the oracle's plain GMRES and scipy's GMRES agree on the rearranged system (eq. num2);
  * the unit cube in uniaxial tension (Sec. 3 benchmark shape) reproduces the uniform stress at
    interior points through eq. stress_1, converging under refinement.
"""
import numpy as np
import pytest

from oracle import bem as ob
from oracle import direct as od
from workloads import geometry as geo

G = 1.0
NU = 0.3
K = od.moduli(G, NU)


def test_quadrature_exact_for_cubics():
    rng = np.random.default_rng(0)
    tri = rng.normal(size=(1, 3, 3))
    pts, nrm, w = ob.quadrature(tri)[:3]
    area = ob.tri_geometry(tri)[2][0]
    # barycentric coordinates of the points
    Tm = np.stack([tri[0, 0] - tri[0, 2], tri[0, 1] - tri[0, 2]], axis=1)
    lam01 = np.linalg.lstsq(Tm, (pts - tri[0, 2]).T, rcond=None)[0].T
    lam = np.column_stack([lam01, 1 - lam01.sum(1)])
    from math import factorial
    for a in range(4):
        for b in range(4 - a):
            for c in range(4 - a - b):
                exact = 2 * area * factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 2)
                approx = np.sum(w * lam[:, 0] ** a * lam[:, 1] ** b * lam[:, 2] ** c)
                assert abs(approx - exact) < 1e-13 * max(1, abs(exact))
    assert abs(w.sum() - area) < 1e-14 * area


def _equilateral(a=1.0):
    return np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * np.sqrt(3) / 2, 0]], float)


def _int_inv_r(tri):
    Us, _ = ob.self_integrals(tri, K, G)
    c = 1.0 / (16 * np.pi * (1 - NU) * G)
    return np.trace(Us) / (c * (3 * (3 - 4 * NU) + 1))


def test_inv_r_equilateral_closed_form():
    for a in (1.0, 0.37):
        assert abs(_int_inv_r(_equilateral(a)) - np.sqrt(3) * a * np.log(2 + np.sqrt(3))) < 1e-13


def _subtris(tri):
    xi = tri.mean(0)
    return xi, [(tri[e], tri[(e + 1) % 3]) for e in range(3)]


def _duffy_U(tri, n=40):
    """Brute force int_T U(xi, x) dS by the Duffy map on the 3 sub-triangles (xi, a, b)."""
    g, gw = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1); gw = 0.5 * gw
    xi, sub = _subtris(tri)
    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0]); nrm /= np.linalg.norm(nrm)
    total = np.zeros((3, 3))
    for a, b in sub:
        J = np.linalg.norm(np.cross(a - xi, b - a))
        U_, V_ = np.meshgrid(g, g, indexing="ij")
        W = np.outer(gw, gw) * U_ * J
        X = xi[None] + U_.reshape(-1, 1) * (a - xi)[None] + (U_ * V_).reshape(-1, 1) * (b - a)[None]
        Uk = od.pair_kernels(np.repeat(xi[None], X.shape[0], 0), X, np.repeat(nrm[None], X.shape[0], 0), K, G)[0]
        total += np.einsum("p,pij->ij", W.reshape(-1), Uk)
    return total


def _polar_P(tri, n_th=96, n_s=24, eps_frac=0.05):
    """Brute force PV int_T P(xi, x) dS: polar quadrature over T minus a disk of radius eps about xi.

    The excluded disk contributes nothing to the principal value (the in-plane kernel is odd in r_hat).
    """
    xi, sub = _subtris(tri)
    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0]); nrm /= np.linalg.norm(nrm)
    e1 = (tri[0] - xi) / np.linalg.norm(tri[0] - xi); e2 = np.cross(nrm, e1)
    gt, gtw = np.polynomial.legendre.leggauss(n_th)
    gs, gsw = np.polynomial.legendre.leggauss(n_s)
    gs = 0.5 * (gs + 1); gsw = 0.5 * gsw
    inr = min(abs(np.dot(np.cross(b - a, xi - a), nrm)) / np.linalg.norm(b - a) for a, b in sub)
    eps = eps_frac * inr
    total = np.zeros((3, 3))
    for a, b in sub:
        ta = np.arctan2(np.dot(a - xi, e2), np.dot(a - xi, e1))
        tb = np.arctan2(np.dot(b - xi, e2), np.dot(b - xi, e1))
        if tb < ta:
            tb += 2 * np.pi
        th = ta + (tb - ta) * 0.5 * (gt + 1); thw = (tb - ta) * 0.5 * gtw
        for t, tw in zip(th, thw):
            d = np.cos(t) * e1 + np.sin(t) * e2
            # distance to edge (a,b) along d
            m = np.cross(b - a, nrm)
            R = np.dot(a - xi, m) / np.dot(d, m)
            rho = eps * (R / eps) ** gs
            wts = tw * gsw * rho * rho * np.log(R / eps)
            X = xi[None] + rho[:, None] * d[None]
            Pk = od.pair_kernels(np.repeat(xi[None], len(rho), 0), X, np.repeat(nrm[None], len(rho), 0), K, G)[1]
            total += np.einsum("p,pij->ij", wts, Pk)
    return total


@pytest.mark.parametrize("which", ["equilateral", "voxel", "random"])
def test_self_blocks_match_brute_force(which):
    if which == "equilateral":
        tri = _equilateral(0.8)
    elif which == "voxel":
        tri = geo.cube_mesh(1)["tri"][1]
    else:
        tri = np.random.default_rng(4).normal(size=(3, 3))
    Us, Ps = ob.self_integrals(tri, K, G)
    Ub = _duffy_U(tri)
    assert np.abs(Us - Ub).max() < 1e-11 * np.abs(Ub).max()
    Pb = _polar_P(tri)
    assert np.abs(Ps - Pb).max() < 1e-9 * max(1e-3, np.abs(Pb).max())
    if which == "equilateral":
        assert np.abs(Ps).max() < 1e-14
    else:
        assert np.abs(Ps).max() > 1e-6  # the antisymmetric coupling is present


@pytest.fixture(scope="module")
def tension2():
    p = geo.cube_tension_problem(2)
    return ob.DenseBEM(p["tri"], p["bc_type"], p["bc_val"], K, G)


def _refine(t):
    v0, v1, v2 = t[:, 0], t[:, 1], t[:, 2]
    m01, m12, m20 = (v0 + v1) / 2, (v1 + v2) / 2, (v2 + v0) / 2
    return np.concatenate([np.stack(s, 1) for s in [(v0, m01, m20), (m01, v1, m12), (m20, m12, v2),
                                                      (m01, m12, m20)]])


def test_rigid_translation_identity():
    """(1/2 I + P^D) c = 0 for a constant c on a closed surface (eq. BIE with u = c, t = 0).

    With the 16-point rule the residual is the near-singular quadrature error of the neighbours
    (Sec. 2.2 notes this limitation); evaluating the same integrals with refined quadrature drives it
    to zero, which pins the assembly, the self blocks and the free term.
    """
    tri = geo.cube_mesh(3)["tri"]
    T = tri.shape[0]
    c = np.array([0.3, -0.7, 0.2])
    sysm = ob.DenseBEM(tri, np.zeros((T, 3), np.int8), np.zeros((T, 3)), K, G)
    r0 = np.abs(sysm.H @ np.tile(c, T)).max()
    assert r0 < 1e-2 * np.linalg.norm(c)
    cen = ob.tri_geometry(tri)[0]
    res = []
    for lev in (1, 2, 3):
        sub, parent = tri.copy(), np.arange(T)
        for _ in range(lev):
            sub, parent = _refine(sub), np.concatenate([parent] * 4)
        qp, qn, qw, qe = ob.quadrature(sub)
        _, Pm = od.quad_blocks(cen, qp, qn, qw, parent[qe], T, K, G)
        for k in range(T):
            Pm[3 * k:3 * k + 3, 3 * k:3 * k + 3] = ob.self_integrals(tri[k], K, G)[1]
        res.append(np.abs((Pm + 0.5 * np.eye(3 * T)) @ np.tile(c, T)).max())
    assert res[0] < r0 and res[1] < res[0] and res[2] < res[1]
    assert res[2] < 1e-6 * np.linalg.norm(c)


def test_lu_gmres_scipy_agree(tension2):
    import scipy.sparse.linalg as sla
    A, b = tension2.A, tension2.b
    x_lu = np.linalg.solve(A, b)
    x_g, it, ok, rr = ob.gmres(lambda v: A @ v, b, tol=1e-12, restart=30, max_iter=2000)
    assert ok and rr <= 1e-12
    assert np.linalg.norm(x_g - x_lu) <= 1e-9 * np.linalg.norm(x_lu)
    x_s, info = sla.gmres(A, b, rtol=1e-12, restart=30, maxiter=200)
    assert info == 0
    assert np.linalg.norm(x_s - x_lu) <= 1e-8 * np.linalg.norm(x_lu)
    # warm start from the solution: zero iterations
    _, it0, ok0, _ = ob.gmres(lambda v: A @ v, b, x0=x_lu, tol=1e-10)
    assert ok0 and it0 == 0


def test_uniaxial_tension_interior_stress():
    errs = []
    for N in (2, 4):
        p = geo.cube_tension_problem(N)
        sys = ob.DenseBEM(p["tri"], p["bc_type"], p["bc_val"], K, G)
        u, t = sys.split(sys.solve_lu())
        qp, qn, qw, qe = ob.quadrature(sys.tri)
        a = t[qe]; b = -u[qe]
        xi = np.array([[0.5, 0.5, 0.5], [0.3, 0.6, 0.4]])
        s = od.direct(od.STRESS, xi, qp, qw, a=a, b=b, nrm=qn, K=K, G=G)
        ref = np.array([1.0, 0, 0, 0, 0, 0])
        errs.append(np.abs(s - ref[None]).max())
        # displacement along x on the loaded face ~ 1/E
        E = 2 * G * (1 + NU)
        loaded = (p["bc_val"][:, 0] == 1.0)
        assert abs(u[loaded, 0].mean() - 1.0 / E) < 0.1 / E
    assert errs[1] < errs[0] and errs[1] < 0.05


def test_matvec_rows_equals_dense():
    p = geo.cube_tension_problem(2)
    s = ob.DenseBEM(p["tri"], p["bc_type"], p["bc_val"], K, G)
    x = np.random.default_rng(1).normal(size=s.A.shape[0])
    rows = np.array([0, 5, 17, 40, 95])
    got = ob.matvec_rows(p["tri"], p["bc_type"], x, rows, K, G)
    ref = (s.A @ x).reshape(-1, 3)[rows]
    assert np.abs(got - ref).max() < 1e-12 * np.abs(s.A @ x).max()


def test_rhs_rows_equals_dense():
    """Right-hand side by direct sums equals the dense B y of eq. num2 (columns of the prescribed values)."""
    p = geo.cube_tension_problem(2)
    s = ob.DenseBEM(p["tri"], p["bc_type"], p["bc_val"], K, G)
    rows = np.array([0, 3, 22, 41, 95])
    got = ob.rhs_rows(p["tri"], p["bc_type"], p["bc_val"], rows, K, G)
    ref = s.b.reshape(-1, 3)[rows]
    assert np.abs(got - ref).max() < 1e-12 * np.abs(s.b).max()


# ------------------------------------------------------------------ near-singular (upsampled) quadrature

def _gl_triangle(x, v, n_gl, K, G):
    """U and P blocks of triangle v at point x by a tensor Gauss-Legendre rule on the collapsed square
    (Duffy map (s, t) -> v0 + s (v1 - v0) + s t (v2 - v1), Jacobian 2 A s): a quadrature family
    independent of the midpoint-split rules."""
    g, gw = np.polynomial.legendre.leggauss(n_gl)
    g = 0.5 * (g + 1.0)
    gw = 0.5 * gw
    S, Tt = np.meshgrid(g, g, indexing="ij")
    W = np.outer(gw, gw)
    v0, v1, v2 = v
    pts = v0[None, None] + S[..., None] * (v1 - v0)[None, None] + (S * Tt)[..., None] * (v2 - v1)[None, None]
    cr = np.cross(v1 - v0, v2 - v0)
    A2 = np.linalg.norm(cr)
    w = (W * S * A2).reshape(-1)
    pts = pts.reshape(-1, 3)
    nrm = np.repeat((cr / A2)[None], pts.shape[0], axis=0)
    U = np.zeros((3, 3))
    P = np.zeros((3, 3))
    for j in range(3):
        a = np.zeros((pts.shape[0], 3))
        a[:, j] = 1.0
        U[:, j] = od.direct(od.DISP, x[None], pts, w, a=a, K=K, G=G)[0]
        P[:, j] = od.direct(od.DISP, x[None], pts, w, b=a, nrm=nrm, K=K, G=G)[0]
    return U, P


def test_upsampled_blocks_converge_to_an_independent_rule():
    """Nearest neighbour of a collocation point on the cube mesh (a triangle of the same face, centroids 0.11
    longest edges apart): the upsampled blocks converge to a 64 x 64 Gauss-Legendre rule on the collapsed
    square (itself unchanged from 48 to 160 points), past the first split by more than 10x per level (the
    rule's fourth order gives 16x asymptotically); level 4 agrees to 1e-8 of the self-block size."""
    tri = geo.cube_mesh(3)["tri"]
    cen = ob.tri_geometry(tri)[0]
    t = 40
    d = np.linalg.norm(cen - cen[t], axis=1)
    d[t] = np.inf
    e = int(np.argmin(d))
    Uref, Pref = _gl_triangle(cen[t], tri[e], 64, K, G)
    scale = np.abs(ob.self_integrals(tri[t], K, G)[0]).max()
    errs = []
    for L in range(5):
        U, P = od.near_blocks(cen, tri, [[t, e]], L, K, G)
        errs.append(max(np.abs(U[0] - Uref).max() / scale, np.abs(P[0] - Pref).max()))
    assert errs[1] < errs[0] and all(errs[k + 1] < errs[k] / 10 for k in range(1, 4)), errs
    assert errs[4] < 1e-8 and errs[0] > 3e-4, errs


def test_upsampled_level0_is_the_element_rule():
    """Level 0 of the upsampled rule is the element's own 16-point rule: the blocks equal the dense
    quadrature blocks of the same pairs."""
    p = geo.cube_tension_problem(2)
    s = ob.DenseBEM(p["tri"], p["bc_type"], p["bc_val"], K, G)
    pairs = ob.near_pairs(s.tri)[:40]
    qp, qn, qw, qe = ob.quadrature(s.tri)
    Um, Pm = od.quad_blocks(s.colloc, qp, qn, qw, qe, s.T, K, G)
    U, P = od.near_blocks(s.colloc, s.tri, pairs, 0, K, G)
    for (t, e), u, pp in zip(pairs, U, P):
        assert np.allclose(u, Um[3 * t:3 * t + 3, 3 * e:3 * e + 3], rtol=1e-12, atol=1e-16)
        assert np.allclose(pp, Pm[3 * t:3 * t + 3, 3 * e:3 * e + 3], rtol=1e-12, atol=1e-16)


def test_near_pairs_use_the_source_edge():
    """Two triangles of different sizes: the pair (t, e) is near when c_t lies within 1.5 longest edges of
    e, so a small triangle next to a large one is near the large one's collocation point's view of it only
    one way round."""
    big = np.array([[0.0, 0.0, 0.0], [4.0, 0.0, 0.0], [0.0, 4.0, 0.0]])  # longest edge 4 sqrt 2
    small = np.array([[6.0, 0.0, 0.0], [6.5, 0.0, 0.0], [6.0, 0.5, 0.0]])  # longest edge sqrt(0.5)
    tri = np.stack([big, small])
    c = ob.tri_geometry(tri)[0]
    dist = np.linalg.norm(c[0] - c[1])  # 4.8 > 1.5 sqrt(0.5), < 1.5 * 4 sqrt 2
    assert 1.5 * np.sqrt(0.5) < dist < 1.5 * 4 * np.sqrt(2)
    got = {tuple(x) for x in ob.near_pairs(tri)}
    assert got == {(1, 0)}


def test_rigid_translation_identity_with_upsampling():
    """On a closed surface a rigid translation is annihilated by 1/2 I + P (interior Somigliana identity at
    a smooth boundary point).  The discrete residual max |H u_rigid| is set by the near-singular quadrature:
    1e-2 with the 16-point rule, falling with each upsampling level to below 1e-5 at level 3, on two mesh
    sizes alike (the error is local to the neighbours of each collocation point)."""
    for N in (3, 4):
        tri = geo.cube_mesh(N)["tri"]
        bc = np.ones((tri.shape[0], 3), np.int8)
        res = []
        for L in (0, 1, 2, 3):
            s = ob.DenseBEM(tri, bc, np.zeros((tri.shape[0], 3)), K, G, near_levels=L)
            r = 0.0
            for k in range(3):
                u = np.zeros(3 * s.T)
                u[k::3] = 1.0
                r = max(r, np.abs(s.H @ u).max())
            res.append(r)
        assert res[0] > 5e-3 and res[3] < 1e-5, res
        assert all(res[k + 1] < res[k] for k in range(3)), res


def test_upsampling_restores_convergence_under_refinement():
    """Cube in uniaxial tension (exact u = (x, -nu y, -nu z) / E): with the 16-point rule the displacement error
    does not fall as the mesh is refined (each row keeps O(1) near-singular quadrature errors on its
    neighbours), with the neighbours upsampled (level 3) it falls with every refinement."""
    E = 2 * G * (1 + NU)
    err = {0: [], 3: []}
    for N in (2, 3, 4):
        p = geo.cube_tension_problem(N)
        cen = ob.tri_geometry(p["tri"])[0]
        uex = np.stack([cen[:, 0], -NU * cen[:, 1], -NU * cen[:, 2]], axis=1) / E
        for L in (0, 3):
            s = ob.DenseBEM(p["tri"], p["bc_type"], p["bc_val"], K, G, near_levels=L)
            u, _ = s.split(s.solve_lu())
            err[L].append(np.abs(u - uex).max() / np.abs(uex).max())
    assert err[3][0] > err[3][1] > err[3][2] and err[3][2] < 0.5 * err[0][2], err
    assert err[0][2] > err[0][0], err


def _periodic_surface():
    M = geo.cavity_cell(6, 0.25, center=(0.05, 0.5, 0.5))  # the cavity crosses the x faces
    return geo.periodic_voxel_surface(M, 1.0 / 6.0)["tri"]


@pytest.mark.parametrize("radius", [ob.NEAR_RADIUS, 4.1])
def test_periodic_near_pairs_match_the_tiled_surface(radius):
    """Near pairs of a periodic surface (cell side 1) against the free-space near pairs of its 3 x 3 x 3 tiling:
    the rows of the centre copy, each element of copy s mapped back to (e, code of s).  At 4.1 edges of 1/6 the
    near distance lies between half a side and a side, so some element pairs are near through two images.
    (Not at 4 edges: centroid distances of exactly 2/3 exist on this voxel grid, and such ties are decided by
    rounding, which differs between c_e + s and the centroid of the shifted vertices; with face centres as
    vertices the centroids lie on a 1/36 grid, so squared centroid distances are multiples of 1/1296, and the
    threshold at 4.1 edges is 605.16/1296.)"""
    tri = _periodic_surface()
    T = tri.shape[0]
    shifts = [(sx, sy, sz) for sz in (-1, 0, 1) for sy in (-1, 0, 1) for sx in (-1, 0, 1)]
    tiled = np.concatenate([tri + np.array(s, dtype=np.float64) for s in shifts])
    free = ob.near_pairs(tiled, radius)
    centre = 13 * T
    want = sorted((int(t) - centre, int(e) % T, int(e) // T) for t, e in free if centre <= t < centre + T)
    got = [tuple(int(v) for v in row) for row in ob.near_pairs(tri, radius, cell_L=1.0)]
    assert got == want
    assert any(c != 13 for _, _, c in got)  # pairs across the faces exist
    twice = len(got) - len({(t, e) for t, e, _ in got})
    assert (twice > 0) == (radius == 4.1)


def test_periodic_near_block_is_the_shifted_element_seen_from_the_point():
    """The block of e's image shifted by L s at c_t equals the block of e at c_t - L s (translation
    invariance), which is how the near correction of a periodic row is computed."""
    tri = _periodic_surface()
    pairs = ob.near_pairs(tri, cell_L=1.0)
    cen = ob.tri_geometry(tri)[0]
    k = next(i for i in range(pairs.shape[0]) if pairs[i, 2] != 13)
    t, e, code = (int(v) for v in pairs[k])
    s = ob.shift_of(code)
    K = od.moduli(1.0, 0.3)
    U1, P1 = od.near_blocks(cen[t][None, :], tri[e][None] + s, np.array([[0, 0]]), 2, K, 1.0)
    U2, P2 = od.near_blocks((cen[t] - s)[None, :], tri, np.array([[0, e]]), 2, K, 1.0)
    assert np.allclose(U1, U2, rtol=1e-12, atol=1e-14) and np.allclose(P1, P2, rtol=1e-12, atol=1e-14)


def test_matvec_rows_with_upsampling_equals_dense():
    """Rows by direct sums with the near pairs' 16-point terms replaced by the upsampled blocks equal the dense
    matrix built with the same blocks (the correction added in the rows is the block swap of DenseBEM)."""
    p = geo.cube_tension_problem(2)
    s = ob.DenseBEM(p["tri"], p["bc_type"], p["bc_val"], K, G, near_levels=2)
    x = np.random.default_rng(4).normal(size=s.A.shape[0])
    rows = np.array([0, 5, 17, 40, 95])
    got = ob.matvec_rows(p["tri"], p["bc_type"], x, rows, K, G, near_levels=2)
    ref = (s.A @ x).reshape(-1, 3)[rows]
    assert np.abs(got - ref).max() < 1e-12 * np.abs(s.A @ x).max()
    gotb = ob.rhs_rows(p["tri"], p["bc_type"], p["bc_val"], rows, K, G, near_levels=2)
    assert np.abs(gotb - s.b.reshape(-1, 3)[rows]).max() < 1e-12 * np.abs(s.b).max()
