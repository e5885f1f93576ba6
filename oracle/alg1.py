"""Oracle (test infrastructure only): the voxel steps of Algorithm 1 (Sec. 2.3, "hard-kill" topology
optimisation) and the adaptive sampling of the interior (Sec. 2.2 end, Sec. 5 "adaptive grid").

A design is a boolean voxel array M (nx, ny, nz) of voxels of edge h with the origin at 0; voxel (i, j, k)
spans [i h, (i + 1) h] x [j h, (j + 1) h] x [k h, (k + 1) h].  Linear voxel order is C order (i slowest).

surface(M, h, load)
    Boundary of the material: every face of a filled voxel whose neighbour across it is empty (or outside the
    array).  Faces come in six classes, axis a = 0, 1, 2 and for each the sign s = +1 then -1 (the outward
    normal is s e_a); inside a class in linear voxel order.  A face's corners, counter-clockwise seen from
    outside, are the points h p with p = the voxel's index (+1 along a when s = +1) plus (0,0), (1,0), (1,1),
    (0,1) along the axes b = a + 1, c = a + 2 (mod 3), in reverse order when s = -1.  Each face gives four
    triangles (q_e, q_{e+1}, centre), e = 0..3, centre = (((q0 + q1) + q2) + q3) / 4 (the paper's 24 N^2
    triangles for an N^3 cube, Sec. 3).  Boundary conditions of the cantilever: the x = 0 faces of the
    voxels with i = 0 are clamped (displacement 0 prescribed), the x = +L faces of the voxels with
    i = nx - 1 carry the traction `load`, every other face is traction-free.
centres(M, h)
    Centres (idx + 1/2) h of the filled voxels, linear order (the interior points of eq. stress_1).
update(M, td, C)
    The removal rule of Algorithm 1: a filled voxel becomes empty when td < D_min + C (D_max - D_min)
    (strict; td per filled voxel in linear order), except in the first and last layers along x (the
    supports; the paper is silent, reading); then only the voxels face-connected to both of those layers
    are kept (a floating piece would make the elastic problem singular; reading of "post-processing").
adaptive sampling with blocks of b^3 voxels (the paper's two-scale grid, coarse then fine):
    coarse_blocks(M, b)   blocks of the block grid (ceil(n / b) per axis, linear order) all of whose voxels
                          are filled; their centres are evaluated first.
    refine_mask(M, b, td_coarse, C)
                          a block is refined (evaluated voxel by voxel) unless it is fully filled and each of
                          its six face neighbours is a fully filled block with the same coarse decision
                          (td < lo + C (hi - lo) over the coarse values: the paper's refinement criterion,
                          different threshold values in neighbouring cells).
    fine_voxels(M, b, refined)
                          filled voxels of refined blocks (linear order): the second round of targets.
    expand(M, b, td_coarse, refined, td_fine)
                          one value per filled voxel: its own fine value in a refined block, else its block's
                          coarse value; update() then applies the rule to this field.
Periodic cell of a metamaterial (Sec. 4.3; the cell repeats over the lattice and its own faces are no
boundary):
cell_surface(M, h, sig_h)
    The faces of surface() with the neighbour across a face taken periodically (index modulo the cell size),
    a face on the upper plane of an axis emitted on the lower plane (coordinate 0; the same face of the
    periodic surface), and every element loaded with the superposition traction -sig_h n (sig_h a 3 x 3
    stress, n = s e_a the normal out of the material): the problem of the fluctuation field.
cell_update(M, td, alpha)
    The single-iteration rule of the paper's metamaterial example (reading: the volume fraction alpha_c is
    met exactly): the filled voxels sorted by (td, linear index), the first ones removed until
    round(alpha n) stay filled (none when no more are filled).
"""
from collections import deque

import numpy as np


def surface(M, h, load=(0.0, 0.0, -1.0)):
    M = np.asarray(M, dtype=bool)
    nx, ny, nz = M.shape
    dims = (nx, ny, nz)
    tris, bct, bcv, axes, signs, owners = [], [], [], [], [], []

    def filled(i, j, k):
        return 0 <= i < nx and 0 <= j < ny and 0 <= k < nz and M[i, j, k]

    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for s in (1, -1):
            for i in range(nx):
                for j in range(ny):
                    for k in range(nz):
                        if not M[i, j, k]:
                            continue
                        idx = [i, j, k]
                        nb = list(idx)
                        nb[a] += s
                        if filled(*nb):
                            continue
                        base = list(idx)
                        if s > 0:
                            base[a] += 1
                        offs = [(0, 0), (1, 0), (1, 1), (0, 1)]
                        if s < 0:
                            offs = offs[::-1]
                        q = []
                        for db, dc in offs:
                            p = list(base)
                            p[b] += db
                            p[c] += dc
                            q.append(np.array([h * float(p[0]), h * float(p[1]), h * float(p[2])]))
                        cen = (((q[0] + q[1]) + q[2]) + q[3]) / 4.0
                        typ, val = [1, 1, 1], [0.0, 0.0, 0.0]
                        if a == 0 and s < 0 and i == 0:
                            typ = [0, 0, 0]
                        if a == 0 and s > 0 and i == dims[0] - 1:
                            val = list(load)
                        for e in range(4):
                            tris.append(np.array([q[e], q[(e + 1) % 4], cen]))
                            bct.append(typ)
                            bcv.append(val)
                            axes.append(a)
                            signs.append(s)
                            owners.append(idx)
    return dict(tri=np.array(tris).reshape(-1, 3, 3), bc_type=np.array(bct, dtype=np.int8).reshape(-1, 3),
                bc_val=np.array(bcv, dtype=np.float64).reshape(-1, 3), axis=np.array(axes), sign=np.array(signs),
                owner=np.array(owners).reshape(-1, 3))


def centres(M, h):
    idx = np.argwhere(np.asarray(M, dtype=bool))
    return (idx + 0.5) * h, idx


def components(M):
    """Face-connected components by breadth-first search; label = smallest linear index of the component,
    -1 on empty voxels."""
    M = np.asarray(M, dtype=bool)
    nx, ny, nz = M.shape
    lab = -np.ones(M.shape, dtype=np.int64)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                if not M[i, j, k] or lab[i, j, k] >= 0:
                    continue
                root = (i * ny + j) * nz + k
                lab[i, j, k] = root
                queue = deque([(i, j, k)])
                while queue:
                    x, y, z = queue.popleft()
                    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                        u, v, w = x + dx, y + dy, z + dz
                        if 0 <= u < nx and 0 <= v < ny and 0 <= w < nz and M[u, v, w] and lab[u, v, w] < 0:
                            lab[u, v, w] = root
                            queue.append((u, v, w))
    return lab


def update(M, td, C):
    M = np.asarray(M, dtype=bool)
    idx = np.argwhere(M)
    td = np.asarray(td, dtype=np.float64)
    lo, hi = td.min(), td.max()
    thr = lo + C * (hi - lo)
    out = M.copy()
    for (i, j, k), d in zip(idx, td):
        if d < thr and 0 < i < M.shape[0] - 1:
            out[i, j, k] = False
    lab = components(out)
    first = set(lab[0][lab[0] >= 0].tolist())
    last = set(lab[-1][lab[-1] >= 0].tolist())
    keep = first & last
    return out & np.isin(lab, sorted(keep))


def _block_grid(M, b):
    return tuple(-(-n // b) for n in M.shape)


def _block_full(M, b):
    nb = _block_grid(M, b)
    full = np.zeros(nb, dtype=bool)
    for I in range(nb[0]):
        for J in range(nb[1]):
            for K in range(nb[2]):
                blk = M[I * b:(I + 1) * b, J * b:(J + 1) * b, K * b:(K + 1) * b]
                full[I, J, K] = blk.size == b ** 3 and blk.all()
    return full


def coarse_blocks(M, b, h):
    """Fully filled blocks (block indices, linear order) and their centres ((idx + 1/2) b h)."""
    full = _block_full(np.asarray(M, dtype=bool), b)
    bidx = np.argwhere(full)
    return bidx, (bidx + 0.5) * (b * h)


def refine_mask(M, b, td_coarse, C):
    M = np.asarray(M, dtype=bool)
    full = _block_full(M, b)
    nb = full.shape
    bidx = np.argwhere(full)
    kill = np.zeros(nb, dtype=bool)
    if len(bidx):
        td_coarse = np.asarray(td_coarse, dtype=np.float64)
        lo, hi = td_coarse.min(), td_coarse.max()
        for (I, J, K), d in zip(bidx, td_coarse):
            kill[I, J, K] = d < lo + C * (hi - lo)
    refined = np.ones(nb, dtype=bool)
    for I, J, K in bidx:
        settled = True
        for dI, dJ, dK in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            u, v, w = I + dI, J + dJ, K + dK
            if not (0 <= u < nb[0] and 0 <= v < nb[1] and 0 <= w < nb[2]) or not full[u, v, w] or \
                    kill[u, v, w] != kill[I, J, K]:
                settled = False
        refined[I, J, K] = not settled
    return refined


def fine_voxels(M, b, refined):
    idx = np.argwhere(np.asarray(M, dtype=bool))
    sel = np.array([refined[i // b, j // b, k // b] for i, j, k in idx], dtype=bool)
    return idx[sel]


def expand(M, b, td_coarse, refined, td_fine):
    M = np.asarray(M, dtype=bool)
    full = _block_full(M, b)
    coarse_val = {}
    for (I, J, K), d in zip(np.argwhere(full), td_coarse):
        coarse_val[(I, J, K)] = d
    out = []
    it = iter(td_fine)
    for i, j, k in np.argwhere(M):
        blk = (i // b, j // b, k // b)
        out.append(next(it) if refined[blk] else coarse_val[blk])
    return np.array(out, dtype=np.float64)


def cell_surface(M, h, sig_h):
    M = np.asarray(M, dtype=bool)
    sig_h = np.asarray(sig_h, dtype=np.float64).reshape(3, 3)
    dims = M.shape
    tris, vals, owners = [], [], []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for s in (1, -1):
            for i in range(dims[0]):
                for j in range(dims[1]):
                    for k in range(dims[2]):
                        if not M[i, j, k]:
                            continue
                        idx = [i, j, k]
                        nb = list(idx)
                        nb[a] = (nb[a] + s) % dims[a]
                        if M[nb[0], nb[1], nb[2]]:
                            continue
                        base = list(idx)
                        if s > 0:
                            base[a] += 1
                            if base[a] == dims[a]:
                                base[a] = 0
                        offs = [(0, 0), (1, 0), (1, 1), (0, 1)]
                        if s < 0:
                            offs = offs[::-1]
                        q = []
                        for db, dc in offs:
                            p = list(base)
                            p[b] += db
                            p[c] += dc
                            q.append(np.array([h * float(p[0]), h * float(p[1]), h * float(p[2])]))
                        cen = (((q[0] + q[1]) + q[2]) + q[3]) / 4.0
                        n = np.zeros(3)
                        n[a] = float(s)
                        t = -(sig_h @ n)
                        for e in range(4):
                            tris.append([q[e], q[(e + 1) % 4], cen])
                            vals.append(t)
                            owners.append(idx)
    T = len(tris)
    return dict(tri=np.array(tris).reshape(T, 3, 3), bc_type=np.ones((T, 3), np.int8),
                bc_val=np.array(vals).reshape(T, 3), owner=np.array(owners, dtype=np.int64).reshape(T, 3))


def cell_update(M, td, alpha):
    M = np.asarray(M, dtype=bool)
    td = np.asarray(td, dtype=np.float64)
    lin = np.flatnonzero(M.reshape(-1))
    assert td.shape == lin.shape
    keep = int(round(alpha * M.size))
    n_remove = max(0, lin.size - keep)
    order = np.lexsort((np.arange(lin.size), td))  # by td, then linear order
    out = M.reshape(-1).copy()
    out[lin[order[:n_remove]]] = False
    return out.reshape(M.shape)
