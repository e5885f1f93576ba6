"""Oracle: plain, slow, FP64 CPU implementations of what the KIFMM/BEM hot path computes.

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the HIP path
(``paper_1612_04082_amd``) and imports nothing from it.

Modules
-------
direct   FP64 direct sums of the Kelvin kernels U, P, D, S (C, OpenMP) -- eq. fmm_summation.
periodic FP64 periodic (Ewald) sums of the same kernels over a cubic lattice of cells (C) -- Sec. 4.3.
bem      dense collocation BEM: quadrature, closed-form self integrals, LU and plain GMRES.
mlp      FP64 point-MLP forward / backward / Adam for the warm-start network.
td       topological derivative (eq. deriv) and the threshold rule of Algorithm 1.
"""
