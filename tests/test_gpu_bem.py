"""bem_solve / bem_stress / bem_quadrature (through the C ABI) vs the dense FP64 BEM oracle.

The GPU solver and oracle/bem.py discretise eq. BIE identically (16-point rule, closed-form self integrals,
column rearrangement of eq. num2, traction columns scaled by G/l), so:
  * the quadrature points of the HIP expansion equal the oracle's;
  * the GPU solution reaches the requested residual when the residual is recomputed with the oracle's
    dense FP64 matrix (fast-summation error aside), and agrees with the LU solution;
  * a warm start at the LU solution needs no iteration; max_iter = 1 returns E_NOCONV with stats;
  * interior stress from a boundary solution matches the oracle's direct FP64 sum (eq. stress_1).
"""
import numpy as np
import pytest
import torch

from oracle import bem as ob
from oracle import direct as od
from workloads import geometry as geo

pytestmark = pytest.mark.gpu

G = 1.0
NU = 0.3
K = od.moduli(G, NU)


def dev(x, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def _solve(prob, **kw):
    from paper_1612_04082_amd import kfmm
    return kfmm.bem_solve(dev(prob["tri"]), dev(prob["bc_type"], torch.int8), dev(prob["bc_val"]), K=K, G=G, **kw)


@pytest.fixture(scope="module")
def coarse_cantilever():
    M, holes = geo.cantilever_voxels(L=16.0, Wd=2.0, h=0.5, n_holes=4, r_lo=0.3, r_hi=0.5, seed=3, margin=0.25)
    prob = geo.cantilever_problem(M, 0.5)
    sysm = ob.DenseBEM(prob["tri"], prob["bc_type"], prob["bc_val"], K, G)
    x_lu = sysm.solve_lu()
    return prob, sysm, x_lu, M, holes


def test_quadrature_matches_oracle(cuda):
    from paper_1612_04082_amd import kfmm
    tri = geo.cube_mesh(3)["tri"]
    qp, qn, qw, cen = kfmm.bem_quadrature(dev(tri))
    p2, n2, w2, _ = ob.quadrature(tri)
    assert np.abs(qp.cpu().numpy() - p2).max() < 1e-15
    assert np.abs(qn.cpu().numpy() - n2).max() < 1e-15
    assert np.abs(qw.cpu().numpy() - w2).max() < 1e-17
    c2 = ob.tri_geometry(tri)[0]
    assert np.array_equal(cen.cpu().numpy(), c2)
    # the central sub-triangle centroid is the collocation point, bit for bit
    assert np.array_equal(qp.cpu().numpy().reshape(-1, 16, 3)[:, 12], cen.cpu().numpy())


@pytest.mark.parametrize("N", [2, 3])
def test_cube_tension_matches_lu_fp64(cuda, N):
    prob = geo.cube_tension_problem(N)
    sysm = ob.DenseBEM(prob["tri"], prob["bc_type"], prob["bc_val"], K, G)
    x_lu = sysm.solve_lu()
    x, u, t, st = _solve(prob, tol=1e-9, restart=50, max_iter=500, precision=0, p=8)
    x = x.cpu().numpy().reshape(-1).copy()
    x[sysm.t_unknown] /= sysm.scale_t  # oracle unknowns are in solver units
    err = np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu)
    print(f"N={N}: iters {st['iters']} rel_res {st['rel_res']:.2e} |x - x_lu|/|x_lu| = {err:.2e}")
    # the fast summation differs from the dense quadrature by ~1e-6 (p = 8); cond(A) ~ 20
    assert st["converged"] and err < 1e-4
    u_o, t_o = sysm.split(x_lu)
    assert np.abs(u.cpu().numpy() - u_o).max() < 1e-4 * np.abs(u_o).max()


def test_cantilever_converges_and_matches_oracle(cuda, coarse_cantilever):
    """Mixed BVP on the slender cantilever: the GPU residual (recomputed through bem_matvec) meets the
    tolerance; measured with the oracle's dense matrix the residual and the distance to the LU solution
    are bounded by the fast-summation error amplified by ||A|| ||x|| / ||b|| ~ 1e4 and cond(A) ~ 1.3e4."""
    from paper_1612_04082_amd import kfmm
    prob, sysm, x_lu, _, _ = coarse_cantilever
    # FP64: the solution is ~1e4 times larger than ||b|| / ||A||, so FP32 products carry ~1e-3 relative
    # noise on this problem and GMRES stalls there; FP64 products converge like the dense oracle (~300 steps)
    x, u, t, st = _solve(prob, tol=1e-6, restart=50, max_iter=2000, precision=0, p=8, leaf_max=128)
    args = (dev(prob["tri"]), dev(prob["bc_type"], torch.int8), dev(prob["bc_val"]))
    xs = x.cpu().numpy().reshape(-1).copy()
    xs[sysm.t_unknown] /= sysm.scale_t  # solver units
    Ax = kfmm.bem_matvec(*args, x=dev(xs.reshape(-1, 3)), which=0, K=K, G=G, p=8, precision=0).cpu().numpy()
    bb = kfmm.bem_matvec(*args, which=1, K=K, G=G, p=8, precision=0).cpu().numpy()
    res_gpu = np.linalg.norm(bb - Ax) / np.linalg.norm(bb)
    res_or = np.linalg.norm(sysm.b - sysm.A @ xs) / np.linalg.norm(sysm.b)
    err = np.linalg.norm(xs - x_lu) / np.linalg.norm(x_lu)
    print(f"T={sysm.T}: iters {st['iters']} gpu rel_res {st['rel_res']:.2e} recomputed {res_gpu:.2e} "
          f"oracle-matrix residual {res_or:.2e} |x - x_lu| {err:.2e}")
    assert st["converged"] and st["rel_res"] <= 1e-6 and res_gpu < 2e-6
    assert res_or < 5e-2 and err < 5e-2


def test_warm_start_and_noconv(cuda, coarse_cantilever):
    prob, sysm, x_lu, _, _ = coarse_cantilever
    x, _, _, st = _solve(prob, tol=1e-5, restart=50, max_iter=2000, precision=0, p=8)
    assert st["converged"]
    x2, _, _, st2 = _solve(prob, tol=1e-5, x0=x, precision=0, p=8, max_iter=100)
    assert st2["iters"] == 0 and st2["rel_res0"] <= 1e-5
    x3, _, _, st3 = _solve(prob, tol=1e-9, max_iter=1, precision=0, p=8, allow_noconv=True)
    assert st3["converged"] == 0 and st3["iters"] == 1 and st3["rel_res"] < 1.0


def test_interior_stress_matches_oracle(cuda, coarse_cantilever):
    from paper_1612_04082_amd import kfmm
    prob, sysm, x_lu, M, holes = coarse_cantilever
    u_o, t_o = sysm.split(x_lu)
    trg = geo.interior_lattice(M, 0.5, n=24, holes=holes)
    out = kfmm.bem_stress(dev(prob["tri"]), dev(prob["bc_type"], torch.int8), dev(prob["bc_val"]), dev(u_o),
                          dev(t_o), dev(trg), K=K, G=G, p=8, precision=1).cpu().numpy()
    qp, qn, qw, qe = ob.quadrature(sysm.tri)
    ref = od.direct(od.STRESS, trg, qp, qw, a=t_o[qe], b=-u_o[qe], nrm=qn, K=K, G=G)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    print(f"{trg.shape[0]} interior points: stress rel err {err:.2e}")
    assert err < 2e-5
