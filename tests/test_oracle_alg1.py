"""Pins of the Algorithm 1 voxel oracle (oracle/alg1.py) against facts that do not come from it: the paper's
triangle count, the divergence theorem, outward orientation, an independently written surface generator,
scipy's connected-component labelling, hand-made designs for the removal rule, and properties the adaptive
sampling must have (block size 1, and TD fields constant on blocks, reproduce the uniform result)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import alg1 as oa
from workloads import geometry as geo


def _random_design(shape, seed, fill=0.7):
    rng = np.random.default_rng(seed)
    M = rng.uniform(size=shape) < fill
    M[0] = True
    M[-1] = True
    return M


@pytest.mark.parametrize("N", [1, 2, 3])
def test_cube_surface_counts_and_divergence(N):
    h = 1.0 / N
    s = oa.surface(np.ones((N, N, N), bool), h)
    tri = s["tri"]
    assert tri.shape[0] == 24 * N * N  # Sec. 3
    cr = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    area_n = 0.5 * cr
    assert np.allclose(area_n.sum(axis=0), 0.0, atol=1e-14)
    cen = tri.mean(axis=1)
    assert np.isclose((cen * area_n).sum(), 3.0 * 1.0, rtol=1e-13)  # int x . n dA = 3 V
    assert np.isclose(np.linalg.norm(cr, axis=1).sum() / 2, 6.0, rtol=1e-13)


def test_surface_orientation_and_boundary_conditions():
    M = _random_design((6, 4, 5), 1)
    h = 0.5
    s = oa.surface(M, h, load=(0.0, 0.3, -1.0))
    tri = s["tri"]
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    n /= np.linalg.norm(n, axis=1)[:, None]
    probe = tri.mean(axis=1) + 0.25 * h * n  # just outside the material
    ijk = np.floor(probe / h).astype(int)
    inside = (ijk >= 0).all(1) & (ijk < np.array(M.shape)).all(1)
    assert not M[tuple(ijk[inside].T)].any()
    own = s["owner"]
    assert M[tuple(own.T)].all()
    back = np.floor((tri.mean(axis=1) - 0.25 * h * n) / h).astype(int)
    assert np.array_equal(back, own)
    clamp = (s["axis"] == 0) & (s["sign"] < 0) & (own[:, 0] == 0)
    loaded = (s["axis"] == 0) & (s["sign"] > 0) & (own[:, 0] == M.shape[0] - 1)
    assert clamp.sum() == 4 * M[0].sum() and loaded.sum() == 4 * M[-1].sum()
    assert (s["bc_type"][clamp] == 0).all() and (s["bc_type"][~clamp] == 1).all()
    assert np.allclose(s["bc_val"][loaded], [0.0, 0.3, -1.0]) and (s["bc_val"][~loaded] == 0).all()


def test_surface_equals_the_independent_generator():
    """workloads.geometry builds the same faces with array operations (written separately): the same
    triangles in the same order."""
    M = _random_design((5, 4, 3), 2)
    s = oa.surface(M, 0.25)
    g = geo.surface_from_voxels(M, 0.25)
    assert s["tri"].shape == g["tri"].shape
    assert np.allclose(s["tri"], g["tri"], rtol=0, atol=1e-15)
    assert np.array_equal(s["owner"], g["owner"]) and np.array_equal(s["axis"], g["axis"])


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_components_equal_scipy_labels(seed):
    M = _random_design((7, 5, 6), seed, fill=0.45)
    lab = oa.components(M)
    ref, n = ndimage.label(M)  # face connectivity (the default structure)
    assert (lab >= 0).sum() == M.sum()
    # the same partition: a one-to-one map between labels
    pairs = set(zip(lab[M].tolist(), ref[M].tolist()))
    assert len(pairs) == len(set(lab[M].tolist())) == n
    # canonical label: the smallest linear index of the component
    lin = np.arange(M.size).reshape(M.shape)
    for l in set(lab[M].tolist()):
        assert l == lin[lab == l].min()


def test_update_rule_on_hand_made_designs():
    M = np.zeros((6, 3, 3), bool)
    M[:, 1, 1] = True          # a bar from end to end
    M[2, 0, 0] = True          # floating voxel
    M[0:2, 2, 2] = True        # stub attached to one end only (not face-connected to the bar)
    idx = np.argwhere(M)
    td = np.ones(len(idx))     # nothing below the threshold (ties keep material)
    out = oa.update(M, td, 0.5)
    assert out[:, 1, 1].all() and not out[2, 0, 0] and not out[0:2, 2, 2].any()
    # the lowest TD in the interior of the bar cuts it: nothing connects both ends any more
    td2 = td.copy()
    td2[[k for k, (i, j, l) in enumerate(idx) if (i, j, l) == (3, 1, 1)][0]] = 0.0
    assert not oa.update(M, td2, 0.5).any()
    # the end layers are protected even at the lowest TD
    td3 = td.copy()
    td3[[k for k, (i, j, l) in enumerate(idx) if (i, j, l) == (0, 1, 1)][0]] = 0.0
    assert oa.update(M, td3, 0.5)[0, 1, 1]
    # strict rule on a solid slab: td below the threshold goes, td equal to it (0 + 0.5 (1 - 0)) stays
    S = np.ones((6, 3, 3), bool)
    sidx = np.argwhere(S)
    td5 = np.array([0.0 if (i, j, l) == (3, 1, 1) else 0.5 if (i, j, l) == (2, 1, 1) else 1.0 for i, j, l in sidx])
    out5 = oa.update(S, td5, 0.5)
    assert not out5[3, 1, 1] and out5[2, 1, 1] and out5.sum() == S.sum() - 1


def test_adaptive_block_one_is_uniform():
    """Blocks of one voxel: every coarse centre is a voxel centre, so with the fine values taken at the same
    points the expanded field is the uniform one and the update is identical."""
    M = _random_design((6, 4, 4), 6, fill=0.8)
    rng = np.random.default_rng(7)
    td_all = rng.uniform(size=M.sum())
    idx = np.argwhere(M)
    val = {tuple(v): d for v, d in zip(idx, td_all)}
    bidx, _ = oa.coarse_blocks(M, 1, 0.5)
    td_c = np.array([val[tuple(v)] for v in bidx])
    ref = oa.refine_mask(M, 1, td_c, 0.3)
    fine = oa.fine_voxels(M, 1, ref)
    td_f = np.array([val[tuple(v)] for v in fine])
    field = oa.expand(M, 1, td_c, ref, td_f)
    assert np.array_equal(field, td_all)
    assert np.array_equal(oa.update(M, field, 0.3), oa.update(M, td_all, 0.3))


def test_adaptive_matches_uniform_for_block_constant_fields():
    """A TD field constant on every block of b^3 voxels: settled blocks carry exactly their voxels' value and
    refined blocks their own, so the adaptive update equals the uniform one; far from the surface and from
    the threshold front the blocks are settled (fewer evaluations)."""
    b = 2
    M = np.ones((12, 6, 6), bool)
    M[4:6, 2:4, 0:2] = False  # a notch
    idx = np.argwhere(M)
    blockval = lambda i, j, k: float((i // b) * 10 + (j // b) + 0.1 * (k // b))
    td_all = np.array([blockval(*v) for v in idx])
    bidx, _ = oa.coarse_blocks(M, b, 1.0)
    td_c = np.array([blockval(*(v * b)) for v in bidx])
    ref = oa.refine_mask(M, b, td_c, 0.35)
    fine = oa.fine_voxels(M, b, ref)
    td_f = np.array([blockval(*v) for v in fine])
    field = oa.expand(M, b, td_c, ref, td_f)
    assert np.array_equal(field, td_all)
    assert np.array_equal(oa.update(M, field, 0.35), oa.update(M, td_all, 0.35))
    assert len(fine) < M.sum()


@pytest.mark.parametrize("center", [(0.5, 0.5, 0.5), (0.05, 0.5, 0.9)])
def test_cell_surface_closed_and_equal_to_independent_generator(center):
    """Periodic cell (Sec. 4.3): the void/material faces of the repeated cell form closed surfaces (area
    normals sum to zero), equal the separately written generator, and carry -sig_h n."""
    M = geo.cavity_cell(8, 0.3, center=center)
    h = 0.125
    sig = np.array([[1.0, 0.2, -0.3], [0.2, 2.0, 0.5], [-0.3, 0.5, -1.0]])
    s = oa.cell_surface(M, h, sig)
    g = geo.periodic_voxel_surface(M, h)
    assert np.allclose(s["tri"], g["tri"], rtol=0, atol=1e-15) and np.array_equal(s["owner"], g["owner"])
    tri = s["tri"]
    cr = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    assert np.abs(cr.sum(axis=0)).max() < 1e-13
    n = cr / np.linalg.norm(cr, axis=1)[:, None]
    assert np.allclose(s["bc_val"], -n @ sig.T, atol=1e-15) and (s["bc_type"] == 1).all()
    cen = tri.mean(axis=1)
    assert (cen >= 0).all() and (cen < 1.0).all()  # every element inside the half-open cell
    if center == (0.5, 0.5, 0.5):  # divergence theorem: the normals point into the cavity
        assert np.isclose((cen * 0.5 * cr).sum() / 3.0, -(~M).sum() * h ** 3, rtol=1e-12)
    # a face whose neighbour across the cell face is void: emitted on the lower plane
    M2 = np.ones((3, 3, 3), bool)
    M2[0, 1, 1] = False
    s2 = oa.cell_surface(M2, 1.0, np.eye(3))
    up = s2["owner"][:, 0] == 2  # voxel (2, 1, 1) faces the void (0, 1, 1) through the cell face x = 3 = 0
    assert up.any() and np.allclose(s2["tri"][up][:, :, 0], 0.0)


def test_cell_update_volume_fraction_and_ties():
    M = np.ones((4, 3, 2), bool)
    M[0, 0, 0] = False
    lin = np.flatnonzero(M.reshape(-1))
    td = np.array([5.0, 1.0, 1.0, 3.0] + [9.0] * (len(lin) - 4))
    out = oa.cell_update(M, td, alpha=20.0 / 24.0)  # 23 filled, keep 20: remove the three smallest
    removed = set(lin) - set(np.flatnonzero(out.reshape(-1)))
    assert removed == {lin[1], lin[2], lin[3]}
    out2 = oa.cell_update(M, td, alpha=21.0 / 24.0)  # remove two: the tied pair, by linear order
    assert set(lin) - set(np.flatnonzero(out2.reshape(-1))) == {lin[1], lin[2]}
    out3 = oa.cell_update(M, td, alpha=1.0)  # already below the target: nothing removed
    assert np.array_equal(out3, M)
