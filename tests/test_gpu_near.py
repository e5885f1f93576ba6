"""Near-singular (upsampled) quadrature of the BEM system on the GPU against the oracle (oracle/bem.py
DenseBEM with near_levels, oracle/direct.c oracle_near_blocks).

  * the near pairs equal the oracle's brute-force list exactly (index work: bit-exact), on a voxel cube
    surface whose structured distances make ties of the distance test likely, and on the cantilever;
  * the correction alone (product with near_levels minus product without, the fast summation cancelling
    exactly) equals (A_near - A_16) x of the dense oracle to rounding;
  * the full product with the correction matches the dense oracle to the fast-summation error;
  * the preconditioner built on the corrected system matches the oracle's;
  * on the cube in uniaxial tension the corrected solve is closer to the exact displacement than the
    uncorrected one, as the oracle's LU solutions are.
"""
import numpy as np
import pytest
import torch

from oracle import bem as ob
from oracle import direct as od
from oracle import precond as op
from workloads import geometry as geo

pytestmark = pytest.mark.gpu

G = 1.0
NU = 0.3
K = od.moduli(G, NU)


def dev(x, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def _args(prob):
    return dev(prob["tri"]), dev(prob["bc_type"], torch.int8), dev(prob["bc_val"])


@pytest.fixture(scope="module")
def cantilever():
    M, holes = geo.cantilever_voxels(L=16.0, Wd=2.0, h=0.5, n_holes=4, r_lo=0.3, r_hi=0.5, seed=3, margin=0.25)
    return geo.cantilever_problem(M, 0.5)


@pytest.mark.parametrize("case", ["cube", "cantilever"])
@pytest.mark.parametrize("radius", [1.5, 0.8])
def test_near_pairs_match_oracle(cuda, cantilever, case, radius):
    from paper_1612_04082_amd import kfmm
    tri = geo.cube_mesh(4)["tri"] if case == "cube" else cantilever["tri"]
    got = kfmm.bem_near_pairs(dev(tri), near_radius=radius).cpu().numpy().astype(np.int64)
    ref = ob.near_pairs(tri, radius)
    print(f"{case} radius {radius}: {tri.shape[0]} triangles, {ref.shape[0]} near pairs")
    assert got.shape == ref.shape and np.array_equal(got, ref)


def test_correction_matches_oracle(cuda, cantilever):
    from paper_1612_04082_amd import kfmm
    prob = cantilever
    s0 = ob.DenseBEM(prob["tri"], prob["bc_type"], prob["bc_val"], K, G)
    s3 = ob.DenseBEM(prob["tri"], prob["bc_type"], prob["bc_val"], K, G, near_levels=3)
    x = np.random.default_rng(31).normal(size=3 * s0.T)
    kw = dict(x=dev(x.reshape(-1, 3)), which=0, K=K, G=G, p=6, precision=0)
    y3 = kfmm.bem_matvec(*_args(prob), near_levels=3, **kw).cpu().numpy().reshape(-1)
    y0 = kfmm.bem_matvec(*_args(prob), **kw).cpu().numpy().reshape(-1)
    ref = (s3.A - s0.A) @ x
    err = np.linalg.norm((y3 - y0) - ref) / np.linalg.norm(ref)
    full = np.linalg.norm(y3 - s3.A @ x) / np.linalg.norm(s3.A @ x)
    print(f"correction rel err {err:.2e} (|correction| / |A x| = {np.linalg.norm(ref) / np.linalg.norm(s3.A @ x):.2e}); "
          f"corrected product vs dense {full:.2e}")
    assert err < 1e-11
    assert full < 2e-4  # the p = 6 fast-summation error (1.6e-4 on the box beam, 6e-5 here)


def test_corrected_product_matches_dense_p8(cuda, cantilever):
    from paper_1612_04082_amd import kfmm
    prob = cantilever
    s3 = ob.DenseBEM(prob["tri"], prob["bc_type"], prob["bc_val"], K, G, near_levels=3)
    x = np.random.default_rng(32).normal(size=3 * s3.T)
    y = kfmm.bem_matvec(*_args(prob), x=dev(x.reshape(-1, 3)), which=0, K=K, G=G, p=8, precision=0,
                        near_levels=3).cpu().numpy().reshape(-1)
    ref = s3.A @ x
    e2 = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"p=8 corrected product vs dense: {e2:.2e}")
    assert e2 < 5e-6


def test_preconditioner_with_correction(cuda, cantilever):
    from paper_1612_04082_amd import kfmm
    prob = cantilever
    s3 = ob.DenseBEM(prob["tri"], prob["bc_type"], prob["bc_val"], K, G, near_levels=3)
    cen = ob.tri_geometry(prob["tri"])[0]
    pc = op.TwoLevel(s3.A, cen, s3.u_unknown)
    v = np.random.default_rng(33).normal(size=3 * s3.T)
    y, info = kfmm.bem_precond_apply(*_args(prob), dev(v.reshape(-1, 3)), K=K, G=G, p=6, precision=0,
                                     near_levels=3)
    ref = pc(v)
    err = np.linalg.norm(y.cpu().numpy().reshape(-1) - ref) / np.linalg.norm(ref)
    print(f"M^-1 v with the near correction: rel err {err:.2e}")
    assert err < 1e-9


def test_cube_tension_closer_to_exact(cuda):
    from paper_1612_04082_amd import kfmm
    prob = geo.cube_tension_problem(4)
    E = 2 * G * (1 + NU)
    cen = ob.tri_geometry(prob["tri"])[0]
    uex = np.stack([cen[:, 0], -NU * cen[:, 1], -NU * cen[:, 2]], axis=1) / E
    errs = {}
    for L in (0, 3):
        _, u, _, st = kfmm.bem_solve(*_args(prob), K=K, G=G, tol=1e-9, restart=50, max_iter=500, precision=0, p=8,
                                     near_levels=L)
        assert st["converged"]
        errs[L] = np.abs(u.cpu().numpy() - uex).max() / np.abs(uex).max()
        s = ob.DenseBEM(prob["tri"], prob["bc_type"], prob["bc_val"], K, G, near_levels=L)
        u_lu, _ = s.split(s.solve_lu())
        e_lu = np.abs(u_lu - uex).max() / np.abs(uex).max()
        print(f"near_levels {L}: GPU displacement error {errs[L]:.3e}, oracle LU {e_lu:.3e}")
        assert abs(errs[L] - e_lu) < 1e-4
    assert errs[3] < 0.5 * errs[0]
