"""Pins of the two-level preconditioner oracle (oracle/precond.py), checked against constructions written
independently here: the Morton order of a regular grid by string interleaving of the bits, the
preconditioner as an explicit dense matrix from selection matrices, the exactness of each level on its
own subspace, and right-preconditioned GMRES on small systems."""
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


def _explicit(A, order, fine, coarse):
    """M^-1 as a dense matrix from selection matrices R_b (3|b| x 3T) and the indicator matrix Z."""
    n = A.shape[0]
    T = n // 3
    M = np.zeros((n, n))
    eye = np.eye(n)
    for s in range(0, T, fine):
        els = order[s:s + fine]
        R = np.vstack([eye[3 * e + c] for e in els for c in range(3)])
        M += R.T @ np.linalg.solve(R @ A @ R.T, R)
    cols = []
    for s in range(0, T, coarse):
        els = order[s:s + coarse]
        for c in range(3):
            z = np.zeros(n)
            z[3 * els + c] = 1.0
            cols.append(z)
    Z = np.array(cols).T
    M += Z @ np.linalg.solve(Z.T @ A @ Z, Z.T)
    return M


def _system(T, seed):
    rng = np.random.default_rng(seed)
    n = 3 * T
    A = rng.normal(size=(n, n)) / np.sqrt(n) + 3.0 * np.eye(n)
    cen = rng.uniform(0, 5, size=(T, 3))
    return A, cen, rng


def test_matches_explicit_construction():
    """T = 150 elements: 5 fine blocks (the last of 22 elements) and 3 aggregates (the last of 22)."""
    A, cen, rng = _system(150, 1)
    pc = op.TwoLevel(A, cen)
    M = _explicit(A, op.morton_order(cen), op.FINE, op.COARSE)
    for _ in range(3):
        v = rng.normal(size=A.shape[0])
        assert np.allclose(pc(v), M @ v, rtol=1e-12, atol=1e-12 * np.abs(M @ v).max())


def test_each_level_is_exact_on_its_subspace():
    A, cen, rng = _system(130, 2)
    pc = op.TwoLevel(A, cen)
    # fine level: with A replaced by its block-diagonal part, M_f^-1 A = I
    Ab = np.zeros_like(A)
    for idx, _ in pc.fine:
        Ab[np.ix_(idx, idx)] = A[np.ix_(idx, idx)]
    pcb = op.TwoLevel(Ab, cen)
    v = rng.normal(size=A.shape[0])
    assert np.allclose(pcb.apply_fine(Ab @ v), v, rtol=1e-11, atol=1e-11)
    # coarse level: Z^T A (Z E^-1 Z^T u) = Z^T u (Galerkin projection)
    u = rng.normal(size=A.shape[0])
    assert np.allclose(pc.Z.T @ (A @ pc.apply_coarse(u)), pc.Z.T @ u, rtol=1e-11, atol=1e-11)
    # the aggregates partition the unknowns: every row of Z has exactly one 1
    assert np.array_equal(pc.Z.sum(axis=1), np.ones(A.shape[0]))


def test_identity_operator_closed_form():
    """A = I: M^-1 v = v + (per aggregate and component, the mean of v over its elements)."""
    T = 100
    cen = np.random.default_rng(3).uniform(size=(T, 3))
    pc = op.TwoLevel(np.eye(3 * T), cen)
    v = np.random.default_rng(4).normal(size=3 * T)
    expect = v.copy()
    order = op.morton_order(cen)
    for s in range(0, T, op.COARSE):
        els = order[s:s + op.COARSE]
        for c in range(3):
            expect[3 * els + c] += v[3 * els + c].mean()
    assert np.allclose(pc(v), expect, rtol=1e-14, atol=1e-14)


def test_right_preconditioned_gmres():
    A, cen, rng = _system(90, 5)
    b = rng.normal(size=A.shape[0])
    x_ref = np.linalg.solve(A, b)
    Ainv = np.linalg.inv(A)
    x, it, ok, rel = op.gmres_right(A, b, lambda v: Ainv @ v, tol=1e-10)
    assert ok and it == 1 and np.allclose(x, x_ref, rtol=1e-8)
    x, it, ok, rel = op.gmres_right(A, b, lambda v: v, tol=1e-10, restart=20)
    assert ok and np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    x, it2, ok, rel = op.gmres_right(A, b, op.TwoLevel(A, cen), tol=1e-10, restart=20)
    assert ok and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
