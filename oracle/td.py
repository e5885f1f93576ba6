"""Oracle (test infrastructure only): topological derivative and the removal rule.

eq. deriv (Sec. 2): D^T = 3 (1 - nu) / (4 E (7 - 5 nu)) [10 (1 + nu) sig:sig - (1 + 5 nu) (tr sig)^2],
reading "tr sigma_ij(p)^2" as the square of the trace.  Stress given in the order xx, yy, zz, yz, xz, xy.
Removal rule (Sec. 2.3, Algorithm 1): a voxel becomes void when D^T < D_min + C (D_max - D_min) (strict).
Pinned by closed-form special cases (hydrostatic and uniaxial stress) in tests/test_oracle_mlp_td.py.
"""
import numpy as np


def topological_derivative(sig6, E, nu):
    s = np.asarray(sig6, dtype=np.float64)
    ss = (s[..., 0] ** 2 + s[..., 1] ** 2 + s[..., 2] ** 2
          + 2.0 * (s[..., 3] ** 2 + s[..., 4] ** 2 + s[..., 5] ** 2))
    tr = s[..., 0] + s[..., 1] + s[..., 2]
    return 3.0 * (1.0 - nu) / (4.0 * E * (7.0 - 5.0 * nu)) * (10.0 * (1.0 + nu) * ss - (1.0 + 5.0 * nu) * tr * tr)


def removal_mask(td, C):
    lo, hi = np.min(td), np.max(td)
    return td < lo + C * (hi - lo)
