"""Two-level preconditioner of the BEM system on the GPU (bem_precond_apply, bem_solve with KFMM_PC_TWO_LEVEL)
against oracle/precond.py built on the oracle's dense FP64 matrix.

  * M^-1 v element by element: the fine blocks are the exact blocks of A (same quadrature, closed-form self
    blocks, free term), the coarse matrix is Z^T A Z summed directly, all in FP64; the two sides differ by
    rounding amplified by the conditioning of the blocks and of E (bound 1e-9 relative);
  * ragged fine blocks and aggregates (sizes that divide nothing), and the dropped rotation columns of
    aggregates without displacement unknowns (the clamped end), counted like the oracle;
  * right-preconditioned GMRES reaches the tolerance in about as many steps as the oracle's dense
    right-preconditioned GMRES, and far fewer than without the preconditioner.
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


@pytest.fixture(scope="module")
def cantilever():
    M, holes = geo.cantilever_voxels(L=16.0, Wd=2.0, h=0.5, n_holes=4, r_lo=0.3, r_hi=0.5, seed=3, margin=0.25)
    prob = geo.cantilever_problem(M, 0.5)
    sysm = ob.DenseBEM(prob["tri"], prob["bc_type"], prob["bc_val"], K, G)
    cen = ob.tri_geometry(prob["tri"])[0]
    return prob, sysm, cen


def _args(prob):
    return dev(prob["tri"]), dev(prob["bc_type"], torch.int8), dev(prob["bc_val"])


@pytest.mark.parametrize("fine,coarse", [(32, 64), (7, 50)])
def test_apply_matches_oracle(cuda, cantilever, fine, coarse):
    from paper_1612_04082_amd import kfmm
    prob, sysm, cen = cantilever
    pc = op.TwoLevel(sysm.A, cen, sysm.u_unknown, fine=fine, coarse=coarse)
    T = sysm.T
    na = -(-T // coarse)
    rng = np.random.default_rng(11)
    for trial in range(2):
        v = rng.normal(size=3 * T)
        y, info = kfmm.bem_precond_apply(*_args(prob), dev(v.reshape(-1, 3)), K=K, G=G, p=8, precision=0,
                                         pc_fine=fine, pc_coarse=coarse)
        y = y.cpu().numpy().reshape(-1)
        ref = pc(v)
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        einf = np.abs(y - ref).max() / np.abs(ref).max()
        print(f"T={T} fine={fine} coarse={coarse}: M^-1 v rel err {err:.2e}, max {einf:.2e}; "
              f"coarse dim {info['n_coarse'] - info['n_dropped']} (dropped {info['n_dropped']}), "
              f"set-up {info['t_setup_s'] * 1e3:.1f} ms")
        assert err < 1e-9 and einf < 1e-9
    assert info["n_fine_blocks"] == -(-T // fine) and info["n_aggregates"] == na
    assert info["n_coarse"] == 6 * na and info["n_coarse"] - info["n_dropped"] == pc.Z.shape[1]


def test_dropped_columns_of_the_clamped_end(cuda, cantilever):
    """Aggregates of 16 elements: the clamped face (displacement prescribed everywhere, so no displacement
    unknown) fills whole aggregates whose rotation columns are dropped; the coarse space still matches."""
    from paper_1612_04082_amd import kfmm
    prob, sysm, cen = cantilever
    pc = op.TwoLevel(sysm.A, cen, sysm.u_unknown, fine=16, coarse=16)
    na = -(-sysm.T // 16)
    assert 6 * na - pc.Z.shape[1] >= 3
    v = np.random.default_rng(12).normal(size=3 * sysm.T)
    y, info = kfmm.bem_precond_apply(*_args(prob), dev(v.reshape(-1, 3)), K=K, G=G, p=8, precision=0,
                                     pc_fine=16, pc_coarse=16)
    ref = pc(v)
    err = np.linalg.norm(y.cpu().numpy().reshape(-1) - ref) / np.linalg.norm(ref)
    print(f"dropped {info['n_dropped']} of {info['n_coarse']}; rel err {err:.2e}")
    assert info["n_dropped"] == 6 * na - pc.Z.shape[1] and err < 1e-9


def test_preconditioned_gmres(cuda, cantilever):
    """Coarse cantilever, FP64 products at p = 8: right-preconditioned GMRES reaches 1e-6 (true residual of
    its own operator) in about the oracle's number of steps (dense operator, same preconditioner), against
    ~300 without; the solution agrees with the unpreconditioned one to the tolerance's reach."""
    from paper_1612_04082_amd import kfmm
    prob, sysm, cen = cantilever
    pc = op.TwoLevel(sysm.A, cen, sysm.u_unknown)
    _, it_or, ok_or, _ = op.gmres_right(sysm.A, sysm.b, pc, tol=1e-6, restart=50)
    args = _args(prob)
    x1, _, _, st1 = kfmm.bem_solve(*args, K=K, G=G, tol=1e-6, restart=50, max_iter=2000, precision=0, p=8,
                                   precond=kfmm.PC_TWO_LEVEL)
    x0, _, _, st0 = kfmm.bem_solve(*args, K=K, G=G, tol=1e-6, restart=50, max_iter=2000, precision=0, p=8)
    d = (torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0)).item()
    print(f"oracle {it_or} steps; GPU preconditioned {st1['iters']} steps (rel_res {st1['rel_res']:.2e}, "
          f"set-up {st1['t_precond_s'] * 1e3:.0f} ms, coarse dim {st1['pc_coarse_dim']}), plain {st0['iters']}; "
          f"|x_pc - x| / |x| = {d:.2e}")
    assert ok_or and st1["converged"] and st1["rel_res"] <= 1e-6
    assert st1["iters"] <= it_or + 10 and 3 * st1["iters"] < st0["iters"]
    assert st1["pc_coarse_dim"] == pc.Z.shape[1]
    assert d < 3e-2  # cond(A) ~ 1.3e4 times residuals of 1e-6 on both sides
