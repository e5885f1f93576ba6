"""Test-side quadrature rules used to pin the oracle (independent of oracle/ and of the HIP path)."""
import numpy as np


def sphere_rule(R=1.0, n_theta=40, n_phi=80, center=(0.0, 0.0, 0.0)):
    """Gauss-Legendre in cos(theta) x trapezoid in phi: spectrally accurate for smooth integrands.

    Returns points (n,3), outward unit normals (n,3) and area weights (n,) that sum to 4 pi R^2.
    """
    mu, wmu = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    MU, PHI = np.meshgrid(mu, phi, indexing="ij")
    W = np.repeat(wmu[:, None], n_phi, axis=1) * (2.0 * np.pi / n_phi) * R * R
    s = np.sqrt(1.0 - MU * MU)
    nrm = np.stack([s * np.cos(PHI), s * np.sin(PHI), MU], axis=-1).reshape(-1, 3)
    pts = np.asarray(center)[None, :] + R * nrm
    return pts, nrm, W.reshape(-1)


def stiffness(K, G):
    """C_ijkl of eq. elast (bulk K, shear G)."""
    d = np.eye(3)
    C = (K * np.einsum("ij,kl->ijkl", d, d)
         + G * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)
                - 2.0 / 3.0 * np.einsum("ij,kl->ijkl", d, d)))
    return C


VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def to_voigt(sig):
    return np.array([sig[..., i, j] for (i, j) in VOIGT]).T if sig.ndim == 3 else np.array(
        [sig[i, j] for (i, j) in VOIGT])
