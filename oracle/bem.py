"""Oracle (test infrastructure only): dense collocation BEM for 3D elastostatics, FP64.

Follows Sec. 2.2 ("Discretization of BIE", "Matrix-vector products"):
  * piecewise-constant displacement u and traction t per flat triangle, collocation at the
    triangle centroid, free term 1/2 I (smooth point of the boundary, eq. BIE);
  * eq. num / eq. coef: (1/2 I + P^D) u = U^D t, with off-diagonal blocks by quadrature and
    the self (diagonal) blocks evaluated in closed form;
  * eq. num2: columns rearranged so that every unknown is in x and every prescribed value in
    y (per element and component: u unknown where t is prescribed, t unknown where u is);
  * quadrature: each triangle is split at its edge midpoints into four equal triangles, each
    carrying a 4-point rule; a quadrature source carries (value) x (area) x (weight).

Readings where the paper is silent (all listed with the design notes):
  * the 4-point rule is the symmetric degree-3 rule (centroid weight -27/48, three points at
    barycentric (3/5, 1/5, 1/5) with weight 25/48);
  * "analytic" self integrals are done fully in closed form in polar coordinates about the
    centroid (radial integral exact, angular integral exact per edge);
  * traction unknowns are column-scaled by -G / l (l = mean element edge): the magnitude balances the
    single-layer columns against the 1/2 I + P columns, the sign turns the columns -U (negative
    definite) into +U so that the spectrum lies in the right half-plane (GMRES stalls otherwise);
  * GMRES stops on the true relative residual ||b - A x|| / ||b||.

The matrices come from oracle.direct.quad_blocks (plain FP64 sums, coincident pairs skipped).
"""
import numpy as np

from . import direct as od

# symmetric degree-3 four-point rule on a triangle: (barycentric, weight)
RULE_BARY = np.array([[1.0 / 3, 1.0 / 3, 1.0 / 3], [0.6, 0.2, 0.2], [0.2, 0.6, 0.2], [0.2, 0.2, 0.6]])
RULE_W = np.array([-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48])


def poisson(K, G):
    return (3.0 * K - 2.0 * G) / (2.0 * (3.0 * K + G))


def tri_geometry(tri):
    """Centroids, unit normals (right-hand rule on vertex order) and areas of triangles (T,3,3)."""
    v0, v1, v2 = tri[:, 0], tri[:, 1], tri[:, 2]
    cen = (v0 + v1 + v2) / 3.0
    cr = np.cross(v1 - v0, v2 - v0)
    area2 = np.linalg.norm(cr, axis=1)
    return cen, cr / area2[:, None], 0.5 * area2


def quadrature(tri):
    """16 quadrature points per triangle: returns points (16T,3), normals, weights, element index.

    Sub-triangles (v0,m01,m20), (m01,v1,m12), (m20,m12,v2), (m01,m12,m20); in each the rule above.
    The centroid of the central sub-triangle is the collocation point itself: it is set to the
    collocation point's own value so that the coincident pair is recognised exactly.
    """
    T = tri.shape[0]
    cen, nrm, area = tri_geometry(tri)
    v0, v1, v2 = tri[:, 0], tri[:, 1], tri[:, 2]
    m01, m12, m20 = 0.5 * (v0 + v1), 0.5 * (v1 + v2), 0.5 * (v2 + v0)
    subs = [(v0, m01, m20), (m01, v1, m12), (m20, m12, v2), (m01, m12, m20)]
    pts = np.empty((T, 4, 4, 3))
    for s, (a, b, c) in enumerate(subs):
        for q in range(4):
            l0, l1, l2 = RULE_BARY[q]
            pts[:, s, q] = l0 * a + l1 * b + l2 * c
    pts[:, 3, 0] = cen
    w = (area / 4.0)[:, None, None] * RULE_W[None, None, :] * np.ones((T, 4, 4))
    elem = np.repeat(np.arange(T), 16)
    return pts.reshape(-1, 3), np.repeat(nrm, 16, axis=0), w.reshape(-1), elem


def _edge_frames(tri_k, xi, n):
    """Per edge (a->b): perpendicular distance h, in-plane outward normal m, tangent t, angles (phi_a, phi_b)."""
    out = []
    for e in range(3):
        a, b = tri_k[e], tri_k[(e + 1) % 3]
        t = (b - a) / np.linalg.norm(b - a)
        m = np.cross(t, n)  # in-plane, perpendicular to the edge
        h = np.dot(a - xi, m)
        if h < 0:
            m, h = -m, -h
        pa, pb = np.arctan2(np.dot(a - xi, t), h), np.arctan2(np.dot(b - xi, t), h)
        out.append((h, m, t, pa, pb))
    return out


def self_integrals(tri_k, K, G):
    """Closed-form self blocks (3x3) at the centroid of one flat triangle: U_self, P_self (principal value).

    Polar coordinates about the centroid xi: per edge, R(phi) = h / cos(phi), r_hat = cos(phi) m + sin(phi) t.
      int 1/r           = sum_e h [L]                          L(phi) = ln(sec phi + tan phi)
      int r_i r_j / r   = sum_e h [m m sin - (m t + t m) cos + t t (L - sin)]
      PV int r_hat/r^2  = sum_e [m (sin (ln h - ln cos + 1) - L) - t cos (ln h - ln cos + 1)]
    U_self = ((3-4nu) I int 1/r + int r r / r) / (16 pi (1-nu) G)            (eq. disp_1)
    P_self = (1-2nu)/(8 pi (1-nu)) (V n^T - n V^T), V = PV int r_hat / r^2   (eq. disp_2, dr/dn = 0 in plane)
    """
    nu = poisson(K, G)
    cen = tri_k.mean(axis=0)
    cr = np.cross(tri_k[1] - tri_k[0], tri_k[2] - tri_k[0])
    n = cr / np.linalg.norm(cr)
    inv_r = 0.0
    rr = np.zeros((3, 3))
    V = np.zeros(3)
    L = lambda p: np.log(1.0 / np.cos(p) + np.tan(p))
    for (h, m, t, pa, pb) in _edge_frames(tri_k, cen, n):
        inv_r += h * (L(pb) - L(pa))
        mm, tt, mt = np.outer(m, m), np.outer(t, t), np.outer(m, t) + np.outer(t, m)
        F = lambda p: (mm * np.sin(p) - mt * np.cos(p) + tt * (L(p) - np.sin(p)))
        rr += h * (F(pb) - F(pa))
        Fm = lambda p: np.sin(p) * (np.log(h) - np.log(np.cos(p)) + 1.0) - L(p)
        Ft = lambda p: -np.cos(p) * (np.log(h) - np.log(np.cos(p)) + 1.0)
        V += m * (Fm(pb) - Fm(pa)) + t * (Ft(pb) - Ft(pa))
    Us = ((3.0 - 4.0 * nu) * np.eye(3) * inv_r + rr) / (16.0 * np.pi * (1.0 - nu) * G)
    Ps = (1.0 - 2.0 * nu) / (8.0 * np.pi * (1.0 - nu)) * (np.outer(V, n) - np.outer(n, V))
    return Us, Ps


def mean_edge(tri):
    return float(np.mean(np.linalg.norm(tri - np.roll(tri, -1, axis=1), axis=2)))


NEAR_RADIUS = 1.5


def near_pairs(tri, radius=NEAR_RADIUS, cell_L=None):
    """Pairs (t, e), t != e, whose collocation point lies within `radius` longest edges of triangle e:
    |c_t - c_e|^2 < radius^2 l_e^2, with squared distances summed as dx*dx + dy*dy + dz*dz and l_e^2 the
    largest squared edge of e (brute force over all pairs).  Sorted by t, then e.  Reading: the paper names
    'triangles close to the triangle with singularity' (Sec. 2.2) without a distance; at 1.5 edges the
    16-point rule is within about 2e-6 of the exact block on voxel surfaces.

    cell_L: the surface repeats with period cell_L (Sec. 4.3); the pairs are then (t, e, code) with e's image
    shifted by cell_L (sx, sy, sz), s in {-1, 0, 1}^3, code = (sx+1) + 3 (sy+1) + 9 (sz+1), the image tested
    as c_e + cell_L s (only the element itself at s = 0 is left out); sorted by t, e, code."""
    tri = np.asarray(tri, dtype=np.float64)
    cen = tri_geometry(tri)[0]
    l2 = np.zeros(tri.shape[0])
    for a in range(3):
        d = tri[:, (a + 1) % 3] - tri[:, a]
        l2 = np.maximum(l2, d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
    thr = (radius * radius) * l2
    out = []
    shifts = [(0, 0, 0)] if cell_L is None else [(sx, sy, sz) for sz in (-1, 0, 1) for sy in (-1, 0, 1)
                                                   for sx in (-1, 0, 1)]
    for t in range(tri.shape[0]):
        for sx, sy, sz in shifts:
            code = (sx + 1) + 3 * (sy + 1) + 9 * (sz + 1)
            img = cen if cell_L is None else cen + cell_L * np.array([sx, sy, sz], dtype=np.float64)
            d = img - cen[t]
            d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
            es = np.nonzero(d2 < thr)[0]
            if cell_L is None:
                out.extend((t, e) for e in es if e != t)
            else:
                out.extend((t, e, code) for e in es if e != t or code != 13)
    if cell_L is None:
        return np.array(out, dtype=np.int64).reshape(-1, 2)
    out = sorted(out)
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def shift_of(code):
    """(sx, sy, sz) of a shift code (sx+1) + 3 (sy+1) + 9 (sz+1)."""
    return np.array([code % 3 - 1, (code // 3) % 3 - 1, code // 9 - 1], dtype=np.float64)


class DenseBEM:
    """Dense H = 1/2 I + P^D and Gm = U^D (eq. num) and the rearranged system A x = b (eq. num2)."""

    def __init__(self, tri, bc_type, bc_val, K, G, nthreads=0, near_levels=0, near_radius=NEAR_RADIUS):
        """near_levels > 0: the blocks of every near pair (near_pairs(tri, near_radius)) use the upsampled
        rule with that many extra midpoint splits (oracle.direct.near_blocks) instead of the 16-point rule."""
        self.tri = np.ascontiguousarray(tri, dtype=np.float64)
        self.T = self.tri.shape[0]
        self.bc_type = np.asarray(bc_type, dtype=np.int8).reshape(self.T, 3)
        self.bc_val = np.asarray(bc_val, dtype=np.float64).reshape(self.T, 3)
        self.K, self.G = K, G
        cen, _, _ = tri_geometry(self.tri)
        self.colloc = cen
        qp, qn, qw, qe = quadrature(self.tri)
        Um, Pm = od.quad_blocks(cen, qp, qn, qw, qe, self.T, K, G, nthreads)
        self.near = np.zeros((0, 2), dtype=np.int64)
        if near_levels > 0:
            self.near = near_pairs(self.tri, near_radius)
            Un, Pn = od.near_blocks(cen, self.tri, self.near, near_levels, K, G, nthreads)
            for (t, e), u, p in zip(self.near, Un, Pn):
                Um[3 * t:3 * t + 3, 3 * e:3 * e + 3] = u
                Pm[3 * t:3 * t + 3, 3 * e:3 * e + 3] = p
        for k in range(self.T):
            Us, Ps = self_integrals(self.tri[k], K, G)
            Um[3 * k:3 * k + 3, 3 * k:3 * k + 3] = Us
            Pm[3 * k:3 * k + 3, 3 * k:3 * k + 3] = Ps
        self.H = Pm + 0.5 * np.eye(3 * self.T)
        self.Gm = Um
        self.scale_t = -G / mean_edge(self.tri)
        flat = self.bc_type.reshape(-1)
        self.u_unknown = flat == 1  # traction prescribed -> displacement unknown
        self.t_unknown = flat == 0
        # A x = b with x = u (where unknown) and x = t / scale_t (where t unknown)
        self.A = np.where(self.u_unknown[None, :], self.H, -self.Gm * self.scale_t)
        y = self.bc_val.reshape(-1)
        self.b =(self.Gm[:, self.u_unknown] @ y[self.u_unknown]) - (self.H[:, self.t_unknown] @ y[self.t_unknown])

    def split(self, x):
        """Physical (u, t) per element from the unknown vector x and the prescribed values."""
        y = self.bc_val.reshape(-1)
        u = np.where(self.u_unknown, x, y)
        t = np.where(self.t_unknown, x * self.scale_t, y)
        return u.reshape(-1, 3), t.reshape(-1, 3)

    def solve_lu(self):
        return np.linalg.solve(self.A, self.b)


def gmres(matvec, b, x0=None, tol=1e-6, restart=50, max_iter=2000):
    """Plain restarted GMRES(m) (Saad & Schultz) with modified Gram-Schmidt, FP64.

    Stops when the true residual ||b - A x|| / ||b|| <= tol, checked at every restart and at the end.
    Returns (x, iterations, converged, rel_res).
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, True, 0.0
    it = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            return x, it, True, beta / bnorm
        if it >= max_iter:
            return x, it, False, beta / bnorm
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = matvec(V[j])
            it += 1
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # apply previous rotations
                a, c = H[i, j], H[i + 1, j]
                H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j], H[j + 1, j] = den, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            if abs(g[j + 1]) / bnorm <= tol or it >= max_iter or H[j, j] == 0.0:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + V[:k].T @ y


def _rows(tri, a_el, b_el, rows, K, G, nthreads, cell_L=None, near_levels=0, near_radius=NEAR_RADIUS):
    """Rows of U(a) + P(b) + 1/2 b at the collocation points `rows`, element densities a_el, b_el (T x 3):
    the quadrature sum over every element's 16 points (coincident pair skipped), with the element's own
    quadrature terms replaced by its closed-form self block, plus the free term.  cell_L: the surface
    repeats with period cell_L (Sec. 4.3): the quadrature sum runs over every lattice image (oracle.periodic,
    the k = 0 reading) and only the element's own n = 0 terms are replaced.  near_levels > 0: the 16-point
    terms of every near pair (near_pairs; with cell_L, of the near image) are replaced by the upsampled
    blocks, as in DenseBEM."""
    qp, qn, qw, qe = quadrature(tri)
    cen = tri_geometry(tri)[0]
    rows = np.asarray(rows)
    if cell_L is None:
        out = od.direct(od.DISP, cen[rows], qp, qw, a=a_el[qe], b=b_el[qe], nrm=qn, K=K, G=G, nthreads=nthreads)
    else:
        from . import periodic as opd
        out = opd.periodic(od.DISP, cen[rows], qp, qw, a=a_el[qe], b=b_el[qe], nrm=qn, K=K, G=G, L=cell_L,
                           nthreads=nthreads)
    for i, r in enumerate(rows):
        sl = slice(16 * r, 16 * r + 16)
        own = od.direct(od.DISP, cen[r:r + 1], qp[sl], qw[sl], a=a_el[qe[sl]], b=b_el[qe[sl]], nrm=qn[sl], K=K, G=G)
        Us, Ps = self_integrals(tri[r], K, G)
        out[i] += -own[0] + Us @ a_el[r] + Ps @ b_el[r] + 0.5 * b_el[r]
    if near_levels > 0:
        pairs = near_pairs(tri, near_radius, cell_L)
        pos = {int(r): i for i, r in enumerate(rows)}
        sel = [k for k in range(pairs.shape[0]) if int(pairs[k, 0]) in pos]
        for k in sel:
            t, e = int(pairs[k, 0]), int(pairs[k, 1])
            # the image of e shifted by cell_L s seen from c_t is e itself seen from c_t - cell_L s
            x = cen[t] - (0.0 if cell_L is None else cell_L * shift_of(int(pairs[k, 2])))
            Un, Pn = od.near_blocks(x[None, :], tri, np.array([[0, e]]), near_levels, K, G)
            sl = slice(16 * e, 16 * e + 16)
            q16 = od.direct(od.DISP, x[None, :], qp[sl], qw[sl], a=a_el[qe[sl]], b=b_el[qe[sl]], nrm=qn[sl], K=K,
                            G=G)
            out[pos[t]] += Un[0] @ a_el[e] + Pn[0] @ b_el[e] - q16[0]
    return out


def matvec_rows(tri, bc_type, x, rows, K, G, nthreads=0, cell_L=None, near_levels=0, near_radius=NEAR_RADIUS):
    """Rows of A x (eq. num2, solver units as in DenseBEM) by direct FP64 sums, for large meshes (cell_L: the
    periodic surface of a cell of that side, see _rows).

    Unknown layout as DenseBEM: u where the traction is prescribed, t / scale_t where the displacement is
    prescribed, scale_t = -G / l; A x = 1/2 u_unk + P u_unk - U t_unk.
    """
    tri = np.ascontiguousarray(tri, dtype=np.float64)
    T = tri.shape[0]
    bc = np.asarray(bc_type).reshape(T, 3)
    x = np.asarray(x, dtype=np.float64).reshape(T, 3)
    scale_t = -G / mean_edge(tri)
    t_unk = bc == 0
    a_el = np.where(t_unk, -scale_t * x, 0.0)   # -t for traction unknowns
    b_el = np.where(t_unk, 0.0, x)              #  u for displacement unknowns
    return _rows(tri, a_el, b_el, rows, K, G, nthreads, cell_L, near_levels, near_radius)


def rhs_rows(tri, bc_type, bc_val, rows, K, G, nthreads=0, cell_L=None, near_levels=0, near_radius=NEAR_RADIUS):
    """Rows of the right-hand side b = U t_known - P u_known - 1/2 u_known (eq. num2) by direct FP64 sums
    (cell_L as in matvec_rows)."""
    tri = np.ascontiguousarray(tri, dtype=np.float64)
    T = tri.shape[0]
    bc = np.asarray(bc_type).reshape(T, 3)
    y = np.asarray(bc_val, dtype=np.float64).reshape(T, 3)
    u_known = bc == 0
    a_el = np.where(u_known, 0.0, y)    # t where the traction is prescribed
    b_el = np.where(u_known, -y, 0.0)   # -u where the displacement is prescribed
    return _rows(tri, a_el, b_el, rows, K, G, nthreads, cell_L, near_levels, near_radius)
