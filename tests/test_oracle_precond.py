"""Pins of the two-level preconditioner oracle (oracle/precond.py), checked against constructions written
independently here: the Morton order of a regular grid by string interleaving of the bits, the
preconditioner as an explicit dense matrix from selection matrices and the raw coarse columns (the coarse
term depends only on their span), the exactness of each level on its own subspace, reproduction of rigid
motions by the coarse space, and right-preconditioned GMRES on small systems."""
import numpy as np

from oracle import precond as op


def _zorder_by_strings(q, bits):
    """Morton keys by writing the bits out: for bit b from high to low, the characters z, y, x."""
    keys = []
    for x, y, z in q:
        s = "".join(f"{(z >> b) & 1}{(y >> b) & 1}{(x >> b) & 1}" for b in range(bits - 1, -1, -1))
        keys.append(int(s, 2))
    return np.argsort(np.array(keys), kind="stable")


def test_morton_order_of_a_grid():
    """16^3 grid points at i/16 plus one point at (1, 1, 1): the extent is 1, so q = 1024 i exactly and the
    order is the Z-order of the integer grid (the extra point clamps to the last cell and comes last)."""
    g = np.arange(16)
    I = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(0)
    perm = rng.permutation(I.shape[0])
    I = I[perm]
    cen = np.vstack([I / 16.0, [[1.0, 1.0, 1.0]]])
    got = op.morton_order(cen)
    ref = _zorder_by_strings(I, 4)
    assert np.array_equal(got[:-1], ref) and got[-1] == I.shape[0]


def _rigid_columns(els, cen, disp, n):
    """Raw columns of one aggregate written out independently: translations of every unknown, and the
    rotation fields w x (x - c) (w = e_x, e_y, e_z) at the displacement unknowns."""
    c = cen[els].mean(axis=0)
    cols = []
    for k in range(3):
        z = np.zeros(n)
        z[3 * els + k] = 1.0
        cols.append(z)
    for k in range(3):
        z = np.zeros(n)
        for e in els:
            x, y, zz = cen[e] - c
            rot = [np.array([0.0, -zz, y]), np.array([zz, 0.0, -x]), np.array([-y, x, 0.0])][k]
            for comp in range(3):
                if disp[3 * e + comp]:
                    z[3 * e + comp] = rot[comp]
        cols.append(z)
    return cols


def _explicit(A, cen, disp, order, fine, coarse):
    """M^-1 as a dense matrix from selection matrices R_b (3|b| x 3T) and a basis of the raw columns."""
    n = A.shape[0]
    T = n // 3
    M = np.zeros((n, n))
    eye = np.eye(n)
    for s in range(0, T, fine):
        els = order[s:s + fine]
        R = np.vstack([eye[3 * e + c] for e in els for c in range(3)])
        M += R.T @ np.linalg.solve(R @ A @ R.T, R)
    basis = []
    for s in range(0, T, coarse):
        C = np.array(_rigid_columns(order[s:s + coarse], cen, disp, n)).T
        U, sv, _ = np.linalg.svd(C, full_matrices=False)
        basis.append(U[:, sv > 1e-10 * sv.max()])
    Z = np.hstack(basis)
    M += Z @ np.linalg.solve(Z.T @ A @ Z, Z.T)
    return M


def _system(T, seed):
    rng = np.random.default_rng(seed)
    n = 3 * T
    A = rng.normal(size=(n, n)) / np.sqrt(n) + 3.0 * np.eye(n)
    cen = rng.uniform(0, 5, size=(T, 3))
    disp = rng.uniform(size=n) < 0.8
    return A, cen, disp, rng


def test_matches_explicit_construction():
    """T = 150 elements: 5 fine blocks (the last of 22 elements) and 3 aggregates (the last of 22); 20% of
    the unknowns are tractions, and the second aggregate has no displacement unknown (its rotations are dropped)."""
    A, cen, disp, rng = _system(150, 1)
    order = op.morton_order(cen)
    disp[op.unknowns(order[64:128])] = False
    pc = op.TwoLevel(A, cen, disp)
    assert pc.Z.shape[1] == 3 * 6 - 3
    M = _explicit(A, cen, disp, order, op.FINE, op.COARSE)
    for _ in range(3):
        v = rng.normal(size=A.shape[0])
        assert np.allclose(pc(v), M @ v, rtol=1e-10, atol=1e-10 * np.abs(M @ v).max())


def test_each_level_is_exact_on_its_subspace():
    A, cen, disp, rng = _system(130, 2)
    pc = op.TwoLevel(A, cen, disp)
    # fine level: with A replaced by its block-diagonal part, M_f^-1 A = I
    Ab = np.zeros_like(A)
    for idx, _ in pc.fine:
        Ab[np.ix_(idx, idx)] = A[np.ix_(idx, idx)]
    pcb = op.TwoLevel(Ab, cen, disp)
    v = rng.normal(size=A.shape[0])
    assert np.allclose(pcb.apply_fine(Ab @ v), v, rtol=1e-11, atol=1e-11)
    # coarse level: Z^T A (Z E^-1 Z^T u) = Z^T u (Galerkin projection)
    u = rng.normal(size=A.shape[0])
    assert np.allclose(pc.Z.T @ (A @ pc.apply_coarse(u)), pc.Z.T @ u, rtol=1e-11, atol=1e-11)
    # orthonormal columns, each supported on one aggregate
    assert np.allclose(pc.Z.T @ pc.Z, np.eye(pc.Z.shape[1]), atol=1e-13)


def test_coarse_space_reproduces_rigid_motions():
    """With every unknown a displacement, a global rigid motion u(x) = a + w x x at the centroids lies in
    the coarse space (each aggregate's translations and rotations about its own centre span it): the
    orthogonal projector Z Z^T leaves it unchanged, and a random field is not."""
    T = 200
    rng = np.random.default_rng(7)
    cen = rng.uniform(-1, 1, size=(T, 3))
    disp = np.ones(3 * T, bool)
    pc = op.TwoLevel(np.eye(3 * T), cen, disp)
    a, w = rng.normal(size=3), rng.normal(size=3)
    u = (a[None, :] + np.cross(w[None, :], cen)).reshape(-1)
    assert np.allclose(pc.Z @ (pc.Z.T @ u), u, rtol=1e-12, atol=1e-12)
    v = rng.normal(size=3 * T)
    assert np.linalg.norm(pc.Z @ (pc.Z.T @ v) - v) > 0.5 * np.linalg.norm(v)
    assert pc.Z.shape[1] == 6 * 4


def test_identity_operator_closed_form():
    """A = I: M^-1 v = v + (per aggregate, the least-squares projection of v onto its raw columns)."""
    T = 100
    cen = np.random.default_rng(3).uniform(size=(T, 3))
    disp = np.random.default_rng(5).uniform(size=3 * T) < 0.7
    pc = op.TwoLevel(np.eye(3 * T), cen, disp)
    v = np.random.default_rng(4).normal(size=3 * T)
    expect = v.copy()
    order = op.morton_order(cen)
    for s in range(0, T, op.COARSE):
        C = np.array(_rigid_columns(order[s:s + op.COARSE], cen, disp, 3 * T)).T
        coef = np.linalg.lstsq(C, v, rcond=None)[0]
        expect += C @ coef
    assert np.allclose(pc(v), expect, rtol=1e-12, atol=1e-12)


def test_right_preconditioned_gmres():
    A, cen, disp, rng = _system(90, 5)
    b = rng.normal(size=A.shape[0])
    x_ref = np.linalg.solve(A, b)
    Ainv = np.linalg.inv(A)
    x, it, ok, rel = op.gmres_right(A, b, lambda v: Ainv @ v, tol=1e-10)
    assert ok and it == 1 and np.allclose(x, x_ref, rtol=1e-8)
    x, it, ok, rel = op.gmres_right(A, b, lambda v: v, tol=1e-10, restart=20)
    assert ok and np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    x, it2, ok, rel = op.gmres_right(A, b, op.TwoLevel(A, cen, disp), tol=1e-10, restart=20)
    assert ok and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
