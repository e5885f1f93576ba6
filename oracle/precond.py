"""Oracle (test infrastructure only): two-level additive Schwarz preconditioner of the collocation BEM
system, FP64, dense.

The paper leaves the preconditioning of mixed boundary-value problems open (Sec. 5, "Discussion and
future work"); this is the non-learned competitor of the learned warm start.  For the rearranged system
A x = b of eq. num2 (the dense matrix of oracle.bem.DenseBEM, solver units):

    M^-1 v = sum_b R_b^T (R_b A R_b^T)^-1 R_b v  +  Z (Z^T A Z)^-1 Z^T v

  * elements are ordered along a Morton curve of their centroids: each coordinate is mapped to
    q = floor((c - lo) / ext * 2^14) (lo: per-axis minimum of the centroids, ext: the largest per-axis
    extent), clamped to [0, 2^14 - 1], and the bits of (qx, qy, qz) are interleaved with x in the lowest
    position of each triple; ties keep the element order;
  * fine blocks R_b: consecutive runs of 32 elements of that order (the last one shorter), each with
    the 3 unknowns of every element;
  * coarse space Z: consecutive runs of 64 elements ("aggregates").  Per aggregate six raw columns, in
    this order: the three translations (component k of every unknown of its elements, displacement and
    traction unknowns alike) and the three infinitesimal rotations about the mean centroid c_a of its
    elements (the value (e_k x (c_e - c_a))_c at the displacement unknown (e, c), zero at traction
    unknowns).  Local rigid motions are the near-null space of 1/2 I + P (on a closed surface a rigid
    displacement gives zero traction), which is what makes the slender cantilevers converge slowly.
    The six are orthonormalised by modified Gram-Schmidt, two passes, in that order; a column whose
    norm after the passes is at most 1e-8 of its raw norm (or whose raw norm is zero: an aggregate with
    no displacement unknown, or collinear ones) is dropped.

GMRES is run on A M^-1 (right preconditioning), so the residual it reduces is the true ||b - A x||.
Parity pinned by tests/test_oracle_precond.py (an explicit dense construction from the raw columns,
the exactness of each level on its own subspace, reproduction of rigid motions, and the Morton order of
a regular grid).
"""
import numpy as np

QBITS = 14
FINE = 32
COARSE = 64
DROP = 1e-8


def morton_order(cen):
    """Element order along the Morton curve of the centroids (see the module docstring)."""
    cen = np.asarray(cen, dtype=np.float64)
    lo = cen.min(axis=0)
    ext = float((cen.max(axis=0) - lo).max())
    if ext == 0.0:
        ext = 1.0
    q = np.floor((cen - lo) / ext * float(1 << QBITS)).astype(np.int64)
    q = np.clip(q, 0, (1 << QBITS) - 1)
    key = np.zeros(cen.shape[0], dtype=np.int64)
    for bit in range(QBITS):
        for axis in range(3):
            key |= ((q[:, axis] >> bit) & 1) << (3 * bit + axis)
    return np.argsort(key, kind="stable")


def blocks(order, size):
    """Consecutive runs of `size` elements of the order (the last may be shorter)."""
    return [order[i:i + size] for i in range(0, order.size, size)]


def unknowns(elems):
    """Indices of the 3 unknowns of each element, element by element."""
    elems = np.asarray(elems)
    return (3 * elems[:, None] + np.arange(3)[None, :]).reshape(-1)


def raw_columns(elems, cen, disp):
    """The six raw coarse columns of one aggregate, restricted to its unknowns (3|a| x 6)."""
    elems = np.asarray(elems)
    ca = cen[elems].mean(axis=0)
    d = cen[elems] - ca
    m = disp[unknowns(elems)].reshape(-1, 3)
    C = np.zeros((3 * elems.size, 6))
    for k in range(3):
        tr = np.zeros((elems.size, 3))
        tr[:, k] = 1.0
        C[:, k] = tr.reshape(-1)
        e = np.zeros(3)
        e[k] = 1.0
        C[:, 3 + k] = (np.cross(e, d) * m).reshape(-1)
    return C


def orthonormal_columns(C):
    """Modified Gram-Schmidt, two passes, in column order; dropped columns are left out."""
    kept = []
    for j in range(C.shape[1]):
        v = C[:, j].copy()
        raw = np.linalg.norm(v)
        for _ in range(2):
            for q in kept:
                v = v - np.dot(q, v) * q
        nv = np.linalg.norm(v)
        if raw == 0.0 or nv <= DROP * raw:
            continue
        kept.append(v / nv)
    return np.array(kept).T if kept else np.zeros((C.shape[0], 0))


class TwoLevel:
    """M^-1 of the module docstring for a dense A (3T x 3T), the element centroids and the mask of
    displacement unknowns (True where the traction is prescribed)."""

    def __init__(self, A, cen, disp, fine=FINE, coarse=COARSE):
        self.A = np.asarray(A, dtype=np.float64)
        T = self.A.shape[0] // 3
        cen = np.asarray(cen, dtype=np.float64)
        disp = np.asarray(disp, dtype=bool).reshape(-1)
        self.order = morton_order(cen)
        self.fine = []
        for bl in blocks(self.order, fine):
            idx = unknowns(bl)
            self.fine.append((idx, np.linalg.inv(self.A[np.ix_(idx, idx)])))
        cols = []
        for bl in blocks(self.order, coarse):
            Q = orthonormal_columns(raw_columns(bl, cen, disp))
            for j in range(Q.shape[1]):
                z = np.zeros(3 * T)
                z[unknowns(bl)] = Q[:, j]
                cols.append(z)
        self.Z = np.array(cols).T
        self.E = self.Z.T @ self.A @ self.Z
        self.Einv = np.linalg.inv(self.E)

    def apply_fine(self, v):
        y = np.zeros_like(v)
        for idx, Binv in self.fine:
            y[idx] = Binv @ v[idx]
        return y

    def apply_coarse(self, v):
        return self.Z @ (self.Einv @ (self.Z.T @ v))

    def __call__(self, v):
        v = np.asarray(v, dtype=np.float64)
        return self.apply_fine(v) + self.apply_coarse(v)


def gmres_right(A, b, Minv, tol=1e-6, restart=50, max_iter=3000):
    """Restarted GMRES(m) on A M^-1 (right preconditioning), MGS Arnoldi applied twice, FP64.

    Stops when the true ||b - A x|| / ||b|| <= tol (checked at every restart).  Returns (x, iterations,
    converged, rel_res)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    it = 0
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta / bn <= tol or it >= max_iter:
            return x, it, beta / bn <= tol, beta / bn
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        V[0] = r / beta
        k = 0
        for j in range(restart):
            w = A @ Minv(V[j])
            it += 1
            for _ in range(2):
                for i in range(j + 1):
                    h = np.dot(w, V[i])
                    H[i, j] += h
                    w = w - h * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            if H[j + 1, j] == 0.0:
                break
            V[j + 1] = w / H[j + 1, j]
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            if np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y) / bn <= tol or it >= max_iter:
                break
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
        x = x + Minv(y @ V[:k])
