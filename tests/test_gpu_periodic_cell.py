"""The metamaterial cell of Sec. 4.3 end to end on the device (paper_1612_04082_amd.alg1.PeriodicCell): a
16^3 voxel cell with a central spherical cavity (the paper's initial guess) under hydrostatic stress,
the single-iteration solution at volume fraction alpha_c = 0.7, and the effective bulk modulus of both
designs against the Hashin-Shtrikman upper bound (a rigorous bound for any porous material of the same
void fraction; the paper's cells come within 95% of it).  The steps themselves are pinned elsewhere: the
voxel steps bit for bit against oracle/alg1.py, the periodic solve and stress against the Ewald oracle."""
import numpy as np
import pytest

from workloads import geometry as geo

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("near_levels", [0, 2])
def test_single_iteration_cell(cuda, near_levels):
    """One single-iteration step of the cell (Sec. 4.3), with the 16-point rule everywhere and with the
    near-singular quadrature on the periodic surface."""
    from paper_1612_04082_amd.alg1 import PeriodicCell
    n = 16
    M0 = geo.cavity_cell(n, 0.3)
    cell = PeriodicCell(n, p=6, tol=1e-6, near_levels=near_levels)
    new, rec = cell.single_iteration(M0, alpha_c=0.7)
    print({k: (round(v, 4) if isinstance(v, float) else v) for k, v in rec.items()})
    assert rec["converged"] and rec["gmres"] <= 60
    assert rec["kept"] == round(0.7 * n ** 3) and int(new.sum().item()) == rec["kept"]
    assert rec["K_eff"] <= 1.01 * rec["K_hs"] and rec["K_eff"] > 0.8 * rec["K_hs"]
    out = cell.bulk_modulus(new)
    print(f"after one iteration: void fraction {out['void_fraction']:.3f}, K_eff/K_HS {out['K_eff'] / out['K_hs']:.3f}, "
          f"GMRES {out['gmres']}, T {out['T']}")
    assert out["converged"]
    assert abs(out["void_fraction"] - 0.3) < 1e-3
    assert 0.5 * out["K_hs"] < out["K_eff"] <= 1.01 * out["K_hs"]
