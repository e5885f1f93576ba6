"""Seeded synthetic inputs shaped like the paper's workloads (Sec. 3 and Sec. 4).

This module only generates inputs (points, normals, weights, densities, triangles, boundary
conditions) and is shared by tests, the benchmark and the oracle-side checks.  It holds no kernel, FMM
or solver arithmetic.  One piece of the method's discretisation does live here: quadrature_cloud places
the 16 quadrature points of a triangle (4 midpoint sub-triangles x the symmetric 4-point rule, Sec. 2.2
"Matrix-vector products") to turn a surface into an FMM source cloud (the box beam and the periodic
cells).  Those clouds are plain inputs of fmm_eval, so the FMM parity tests do not depend on the rule;
the BEM tests never take their quadrature from here: oracle/bem.py and the library each place the points
with their own code, and a GPU test compares the two.  Every generator takes an explicit seed and uses
numpy.random.default_rng.

Shapes:
  * sphere cloud            -- the plain KIFMM check (uniform points on the unit sphere);
  * voxel surfaces          -- boundary faces of a voxel array, each square face split through its
                               centre into 4 triangles (Sec. 3: 24 N^2 triangles for the N-cube);
  * box beam                -- the 120 x 20 x 20 beam tiled by squares of side 20/11;
  * cantilever with holes   -- 8:1:1 beam voxelised, random spherical holes (Sec. 4.1 shape family);
  * periodic-cell bodies    -- unit cube minus random ellipsoidal inclusions (Sec. 4.3 shape family);
  * periodic cavity surface -- the void/solid faces of a voxel cell repeated over the lattice (Sec. 4.3:
                               the cell's own faces are not boundary), with a spherical cavity as the
                               paper's initial guess.
"""
import numpy as np

# ----------------------------------------------------------------------------- point clouds


def sphere_cloud(n=4096, seed=1):
    """n points uniform on the unit sphere, normals = positions, weights 4 pi / n, densities U[-1,1]^3."""
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(n, 3))
    x = g / np.linalg.norm(g, axis=1)[:, None]
    a = rng.uniform(-1.0, 1.0, size=(n, 3))
    w = np.full(n, 4.0 * np.pi / n)
    return dict(src=x, nrm=x.copy(), w=w, a=a, b=None)


# ----------------------------------------------------------------------------- voxel surfaces


def voxel_boundary_quads(M, h=1.0, origin=(0.0, 0.0, 0.0)):
    """Boundary faces of the filled voxels of M (bool, shape (nx,ny,nz)).

    Returns quads (F,4,3) ordered counter-clockwise seen from outside the material, the face
    axis (F,), the face sign (F,) (+1: normal along +axis) and the voxel index (F,3) that owns it.
    """
    M = np.asarray(M, dtype=bool)
    origin = np.asarray(origin, dtype=np.float64)
    P = np.pad(M, 1)
    quads, axes, signs, owners = [], [], [], []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for s in (+1, -1):
            nb = np.roll(P, -s, axis=a)[1:-1, 1:-1, 1:-1]  # neighbour across the face
            face = M & ~nb
            idx = np.argwhere(face)
            if idx.size == 0:
                continue
            base = idx.astype(np.float64)
            base[:, a] += 1.0 if s > 0 else 0.0
            corners = np.zeros((idx.shape[0], 4, 3))
            offs = [(0, 0), (1, 0), (1, 1), (0, 1)]
            if s < 0:
                offs = offs[::-1]
            for q, (db, dc) in enumerate(offs):
                p = base.copy()
                p[:, b] += db
                p[:, c] += dc
                corners[:, q] = origin + h * p
            quads.append(corners)
            axes.append(np.full(idx.shape[0], a))
            signs.append(np.full(idx.shape[0], s))
            owners.append(idx)
    return (np.concatenate(quads), np.concatenate(axes), np.concatenate(signs), np.concatenate(owners))


def quads_to_tris(quads):
    """Split each quad through its centre into 4 triangles (both diagonals), keeping the orientation."""
    C = quads.mean(axis=1)
    tris = np.empty((quads.shape[0], 4, 3, 3))
    for e in range(4):
        tris[:, e, 0] = quads[:, e]
        tris[:, e, 1] = quads[:, (e + 1) % 4]
        tris[:, e, 2] = C
    return tris.reshape(-1, 3, 3)


def surface_from_voxels(M, h=1.0, origin=(0.0, 0.0, 0.0)):
    quads, axes, signs, owners = voxel_boundary_quads(M, h, origin)
    tris = quads_to_tris(quads)
    rep = lambda x: np.repeat(x, 4, axis=0)
    return dict(tri=tris, axis=rep(axes), sign=rep(signs), owner=rep(owners))


def periodic_voxel_surface(M, h=1.0, origin=(0.0, 0.0, 0.0)):
    """Faces between filled and empty voxels of a cell repeated periodically (neighbours wrap around), split
    into 4 triangles each, counter-clockwise seen from the void (normals point out of the material).  A
    face on the upper plane of an axis (between the last layer and the first layer's image) is placed on
    the lower plane, so every face lies in [origin, origin + n h) up to its edges."""
    M = np.asarray(M, dtype=bool)
    origin = np.asarray(origin, dtype=np.float64)
    quads, axes, signs, owners = [], [], [], []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for s in (+1, -1):
            nb = np.roll(M, -s, axis=a)  # periodic neighbour across the face
            idx = np.argwhere(M & ~nb)
            if idx.size == 0:
                continue
            base = idx.astype(np.float64)
            base[:, a] += 1.0 if s > 0 else 0.0
            base[:, a] = np.where(base[:, a] >= M.shape[a], base[:, a] - M.shape[a], base[:, a])
            corners = np.zeros((idx.shape[0], 4, 3))
            offs = [(0, 0), (1, 0), (1, 1), (0, 1)]
            if s < 0:
                offs = offs[::-1]
            for q, (db, dc) in enumerate(offs):
                p = base.copy()
                p[:, b] += db
                p[:, c] += dc
                corners[:, q] = origin + h * p
            quads.append(corners)
            axes.append(np.full(idx.shape[0], a))
            signs.append(np.full(idx.shape[0], s))
            owners.append(idx)
    quads = np.concatenate(quads)
    rep = lambda x: np.repeat(np.concatenate(x), 4, axis=0)
    return dict(tri=quads_to_tris(quads), axis=rep(axes), sign=rep(signs), owner=rep(owners))


def cavity_cell(n, radius, center=(0.5, 0.5, 0.5)):
    """n^3 voxels of a unit cell, solid except a ball of the given radius (voxel centres inside it are
    void; the ball wraps around the cell faces when it crosses them)."""
    xs = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
    d = [np.abs(P - c) for P, c in zip((X, Y, Z), center)]
    d = [np.minimum(q, 1.0 - q) for q in d]  # periodic distance
    return (d[0] ** 2 + d[1] ** 2 + d[2] ** 2) > radius * radius


def cube_mesh(N):
    """Unit cube of N^3 voxels: 24 N^2 triangles (Sec. 3 benchmark)."""
    return surface_from_voxels(np.ones((N, N, N), bool), h=1.0 / N)


# ----------------------------------------------------------------------------- quadrature clouds

_RULE_BARY = np.array([[1.0 / 3, 1.0 / 3, 1.0 / 3], [0.6, 0.2, 0.2], [0.2, 0.6, 0.2], [0.2, 0.2, 0.6]])
_RULE_W = np.array([-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48])


def quadrature_cloud(tri):
    """16 points per triangle (4 midpoint sub-triangles x symmetric 4-point rule), as a source cloud.

    Returns points, unit normals and area weights (value x area x rule weight), as the paper's
    matrix-vector products feed them to the fast summation (Sec. 2.2).
    """
    v0, v1, v2 = tri[:, 0], tri[:, 1], tri[:, 2]
    cr = np.cross(v1 - v0, v2 - v0)
    a2 = np.linalg.norm(cr, axis=1)
    nrm = cr / a2[:, None]
    area = 0.5 * a2
    m01, m12, m20 = 0.5 * (v0 + v1), 0.5 * (v1 + v2), 0.5 * (v2 + v0)
    subs = [(v0, m01, m20), (m01, v1, m12), (m20, m12, v2), (m01, m12, m20)]
    T = tri.shape[0]
    pts = np.empty((T, 4, 4, 3))
    for s, (a, b, c) in enumerate(subs):
        for q in range(4):
            l0, l1, l2 = _RULE_BARY[q]
            pts[:, s, q] = l0 * a + l1 * b + l2 * c
    w = (area / 4.0)[:, None, None] * _RULE_W[None, None, :] * np.ones((T, 4, 4))
    return pts.reshape(-1, 3), np.repeat(nrm, 16, axis=0), w.reshape(-1)


def box_beam_cloud(seed=2, L=120.0, W=20.0, n_w=11):
    """The 120 x 20 x 20 beam, faces tiled by squares of side W/n_w: 201,344 quadrature points.

    Densities a, b ~ N(0,1)^3 independent.
    """
    h = W / n_w
    nx = int(round(L / h))
    surf = surface_from_voxels(np.ones((nx, n_w, n_w), bool), h=h)
    pts, nrm, w = quadrature_cloud(surf["tri"])
    rng = np.random.default_rng(seed)
    a = rng.normal(size=pts.shape)
    b = rng.normal(size=pts.shape)
    return dict(src=pts, nrm=nrm, w=w, a=a, b=b, tri=surf["tri"])


# ----------------------------------------------------------------------------- cantilever with holes


def cantilever_voxels(L=32.0, Wd=4.0, h=2.0 / 9.0, n_holes=64, r_lo=0.3, r_hi=0.8, seed=3, max_tries=200000,
                      margin=None):
    """Beam [0,L]x[0,Wd]^2 voxelised at spacing h, with random non-overlapping spherical holes.

    With m = margin (default 2h): hole centres lie in x in [2+r+m, L-2-r-m], y,z in [r+m, Wd-r-m]; a
    candidate is rejected if within r_i + r_j + m of an accepted hole.  Voxels whose centre lies inside a
    hole are empty.
    """
    rng = np.random.default_rng(seed)
    m = 2 * h if margin is None else margin
    nx, ny = int(round(L / h)), int(round(Wd / h))
    holes = []
    tries = 0
    while len(holes) < n_holes and tries < max_tries:
        tries += 1
        r = rng.uniform(r_lo, r_hi)
        c = np.array([rng.uniform(2 + r + m, L - 2 - r - m),
                      rng.uniform(r + m, Wd - r - m), rng.uniform(r + m, Wd - r - m)])
        if all(np.linalg.norm(c - c2) >= r + r2 + m for (c2, r2) in holes):
            holes.append((c, r))
    xs = (np.arange(nx) + 0.5) * h
    ys = (np.arange(ny) + 0.5) * h
    X, Y, Z = np.meshgrid(xs, ys, ys, indexing="ij")
    M = np.ones((nx, ny, ny), bool)
    for c, r in holes:
        M &= (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 > r * r
    return M, holes


def cantilever_problem(M, h, load=(0.0, 0.0, -1.0)):
    """Mixed BVP on the voxel surface: u = 0 on the x = 0 face, t = load on the x = max face, t = 0 elsewhere.

    bc_type per element and component: 0 = displacement prescribed, 1 = traction prescribed.
    """
    surf = surface_from_voxels(M, h)
    tri = surf["tri"]
    T = tri.shape[0]
    bc_type = np.ones((T, 3), np.int8)
    bc_val = np.zeros((T, 3))
    nx = M.shape[0]
    clamp = (surf["axis"] == 0) & (surf["sign"] < 0) & (surf["owner"][:, 0] == 0)
    loaded = (surf["axis"] == 0) & (surf["sign"] > 0) & (surf["owner"][:, 0] == nx - 1)
    bc_type[clamp] = 0
    bc_val[loaded] = np.asarray(load)[None, :]
    return dict(tri=tri, bc_type=bc_type, bc_val=bc_val, surf=surf)


def interior_lattice(M, h, n=128, holes=(), margin=None):
    """Cell-centred n^3 lattice over the beam shrunk by h/2, keeping points in material and at least
    `margin` (default h/2) away from the hole surfaces."""
    margin = 0.5 * h if margin is None else margin
    ext = np.array(M.shape) * h
    axes = [np.linspace(margin, e - margin, n) for e in ext]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    keep = np.ones(P.shape[0], bool)
    for c, r in holes:
        keep &= np.linalg.norm(P - c[None, :], axis=1) >= r + margin
    idx = np.floor(P / h).astype(int)
    idx = np.minimum(idx, np.array(M.shape) - 1)
    keep &= M[idx[:, 0], idx[:, 1], idx[:, 2]]
    return P[keep]


# ----------------------------------------------------------------------------- periodic-cell bodies


def _largest_component(M):
    from scipy import ndimage
    lab, n = ndimage.label(M)
    if n <= 1:
        return M
    sizes = ndimage.sum(M, lab, index=np.arange(1, n + 1))
    return lab == (1 + int(np.argmax(sizes)))


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def cell_voxels(g, n_vox, seed_base=4000):
    """Unit cube at n_vox^3 voxels minus 1-8 random ellipsoids (semi-axes U[0.05,0.25], random rotation,
    centres U[0.25,0.75]^3); the largest face-connected component is kept."""
    rng = np.random.default_rng(seed_base + g)
    n_inc = int(rng.integers(1, 9))
    h = 1.0 / n_vox
    xs = (np.arange(n_vox) + 0.5) * h
    X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    M = np.ones((n_vox,) * 3, bool)
    for _ in range(n_inc):
        ax = rng.uniform(0.05, 0.25, size=3)
        R = _rotation(rng)
        c = rng.uniform(0.25, 0.75, size=3)
        loc = (P - c) @ R
        M &= ((loc / ax) ** 2).sum(-1) > 1.0
    return _largest_component(M), h


def cell_batch(n_cells=64, seed_base=4000, lo=20000, hi=200000, seed=4):
    """n_cells periodic-cell bodies with uneven sizes: each cell draws a target point count in [lo, hi]
    and the voxel resolution closest to it.  Returns a list of dicts with src, nrm, w, a, b."""
    out = []
    for g in range(n_cells):
        rng = np.random.default_rng(seed_base + 1000 + g)
        target = rng.uniform(lo, hi)
        # a full cube at n voxels has 6 n^2 faces * 64 points
        n_vox = int(np.clip(round(np.sqrt(target / 384.0)), 7, 22))
        while True:  # inclusions add surface: step the resolution down until the cell is within [lo, hi]
            M, h = cell_voxels(g, n_vox, seed_base)
            surf = surface_from_voxels(M, h)
            if surf["tri"].shape[0] * 16 <= hi or n_vox <= 7:
                break
            n_vox -= 1
        pts, nrm, w = quadrature_cloud(surf["tri"])
        r2 = np.random.default_rng(seed * 100000 + g)
        out.append(dict(src=pts, nrm=nrm, w=w, a=r2.normal(size=pts.shape), b=r2.normal(size=pts.shape)))
    return out


def periodic_cell_batch(n_cells=64, seed_base=4000, lo=20000, hi=200000, seed=4):
    """n_cells periodic metamaterial cells (Sec. 4.3): the unit cell of cell_voxels repeated over the lattice,
    the surface the void/material faces only (periodic_voxel_surface; the cell's own faces are no boundary),
    the voxel resolution chosen so that each cell's quadrature point count falls near a target drawn in
    [lo, hi].  Returns a list of dicts with src, nrm, w, a, b (densities with zero net single-layer force
    per cell, the case of a closed surface's tractions)."""
    out = []
    for g in range(n_cells):
        rng = np.random.default_rng(seed_base + 1000 + g)
        target = rng.uniform(lo, hi)
        n_vox, pts = 8, None
        while n_vox <= 96:
            M, h = cell_voxels(g, n_vox, seed_base)
            surf = periodic_voxel_surface(M, h)
            npts = surf["tri"].shape[0] * 16
            if npts >= target or n_vox == 96:
                if npts > hi and n_vox > 8:  # one step back stays within [lo, hi]
                    M, h = cell_voxels(g, n_vox - 1, seed_base)
                    surf = periodic_voxel_surface(M, h)
                break
            n_vox += max(1, int(n_vox * (np.sqrt(target / max(npts, 1)) - 1.0) * 0.5))
        pts, nrm, w = quadrature_cloud(surf["tri"])
        r2 = np.random.default_rng(seed * 100000 + g)
        a = r2.normal(size=pts.shape)
        a -= (w[:, None] * a).sum(0) / w.sum()
        out.append(dict(src=pts, nrm=nrm, w=w, a=a, b=r2.normal(size=pts.shape)))
    return out


# ----------------------------------------------------------------------------- cube in uniaxial tension


def cube_tension_problem(N, traction=1.0):
    """Unit cube (Sec. 3 benchmark shape) in uniaxial tension along x with symmetry rollers.

    x = 0: u_x = 0, t_y = t_z = 0;  y = 0: u_y = 0, t_x = t_z = 0;  z = 0: u_z = 0, t_x = t_y = 0;
    x = 1: t = (traction, 0, 0);  y = 1, z = 1: t = 0.
    Exact solution: sigma = traction e_x e_x, u = traction (x, -nu y, -nu z) / E.
    """
    surf = cube_mesh(N)
    tri = surf["tri"]
    T = tri.shape[0]
    bc_type = np.ones((T, 3), np.int8)
    bc_val = np.zeros((T, 3))
    ax, sg = surf["axis"], surf["sign"]
    for a in range(3):
        sym = (ax == a) & (sg < 0)
        bc_type[sym, a] = 0
    bc_val[(ax == 0) & (sg > 0), 0] = traction
    return dict(tri=tri, bc_type=bc_type, bc_val=bc_val)
