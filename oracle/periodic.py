"""Periodic sums of the Kelvin kernels (oracle/ewald.c): the boundary integrals of eq. fmm_summation over
every lattice image of the sources of a cubic cell of side L (Sec. 4.3, periodic cell of a metamaterial).

Test infrastructure only.  Definition (a reading; the paper names no summation order): the Fourier series
over the reciprocal lattice with the k = 0 term left out -- the periodic field of zero cell mean.  The
image n = 0 of a source that coincides with a target is left out, every other image is kept.  Evaluated
by Ewald summation with splitting parameter alpha; the real-space and reciprocal cut-offs below keep
both truncation errors under about 1e-15 of the leading terms.
"""
import math

import numpy as np

from .direct import DISP, STRESS, _f64, _p, lib, moduli  # noqa: F401


def cutoffs(L, alpha_L=5.0, digits=15.5):
    """Splitting parameter and cut-offs for a cell of side L: erfc(alpha rcut) and exp(-k^2/(4 alpha^2))
    both below 10^-digits."""
    alpha = alpha_L / L
    x = math.sqrt(digits * math.log(10.0)) + 0.5
    rcut = x / alpha
    nreal = int(math.ceil(rcut / L)) + 1
    kmax = int(math.ceil(2.0 * alpha * x * L / (2.0 * math.pi)))
    return alpha, nreal, rcut, kmax


def periodic(kind, trg, src, w, a=None, b=None, nrm=None, K=None, G=1.0, L=1.0, alpha_L=5.0, free_space=False,
             nthreads=0):
    """Periodic (or, with free_space=True, plain free-space through the same tensor algebra) sum.
    Returns (M, 3) for DISP or (M, 6) for STRESS (xx, yy, zz, yz, xz, xy)."""
    if K is None:
        K = moduli(G, 0.3)
    trg = _f64(trg).reshape(-1, 3)
    src = _f64(src).reshape(-1, 3)
    w = _f64(w).reshape(-1)
    a = None if a is None else _f64(a).reshape(-1, 3)
    b = None if b is None else _f64(b).reshape(-1, 3)
    nrm = None if nrm is None else _f64(nrm).reshape(-1, 3)
    M, N = trg.shape[0], src.shape[0]
    out = np.zeros((M, 3 if kind == DISP else 6))
    alpha, nreal, rcut, kmax = cutoffs(L, alpha_L)
    rc = lib().oracle_periodic(kind, K, G, L, _p(trg), M, _p(src), _p(nrm), _p(w), _p(a), _p(b), N, alpha, nreal,
                               rcut, kmax, 1 if free_space else 0, _p(out), nthreads)
    if rc != 0:
        raise ValueError("oracle_periodic: bad arguments")
    return out
