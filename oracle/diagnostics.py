"""Oracle: axial modal kinetic energy of a toroidal-poloidal state.

Test infrastructure only (see the package header).

Sec. 5.3 (Results and validation) measures the growth of a seeded axial wave through the
kinetic energy E_k held by axial wavenumber k.  The paper does not state the normalisation (a
growth rate does not depend on it); the reading used here: with the nodal velocity u of
(psi, chi) and its axial Fourier coefficients u_k(r, phi) = (1/N_z) sum_l u(z_l) exp(-i kappa_k z_l),
    E_k = (L_z / 2) int_0^{2 pi} int_0^inf |u_k|^2 r dr dphi,
so that the sum of E_k over all k is the kinetic energy of one axial period.  The area integral
uses the Gauss-Legendre rule in the mapped variable (r dr = ell^2 / (1-x)^2 dx) and the
trapezoidal rule in phi.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid
from .rhs import VecTables, synthesize


def axial_modal_energy(psi: np.ndarray, chi: np.ndarray, g: Grid, vt: VecTables) -> np.ndarray:
    """E per axial FFT slot (length N_z, slot order of numpy's fft)."""
    u, _ = synthesize(psi, chi, g, vt)
    E = np.zeros(g.nz)
    for c in u:
        uk = np.fft.fft(c, axis=0) / g.nz                      # (N_z, N_r, N_phi)
        E += (np.abs(uk) ** 2 * g.area_w[None, :, None]).sum(axis=(1, 2)) * (2 * np.pi / g.nphi)
    return 0.5 * g.lz * E


def kinetic_energy(psi: np.ndarray, chi: np.ndarray, g: Grid, vt: VecTables) -> float:
    """(1/2) int |u|^2 dV over one axial period, summed directly on the physical grid."""
    u, _ = synthesize(psi, chi, g, vt)
    tot = sum((c ** 2 * g.area_w[None, :, None]).sum() for c in u)
    return 0.5 * tot * (g.lz / g.nz) * (2 * np.pi / g.nphi)
