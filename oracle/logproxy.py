"""Oracle: potentials with a logarithmic far field (Eq. logproxy) and the enstrophy diagnostic.

Test infrastructure only (see the package header).

Sec. 3.1: a source with a nonzero integral gives a two-dimensional Poisson solution a logarithmic
far field, which no combination of the decaying basis functions represents; the potential then
carries one extra real amplitude c of the proxy Lambda(r) = ln(r^2 + ell^2), whose horizontal
Laplacian lies in the m = 0 basis (Eq. logproxy):
    grad_h^2 Lambda = (1/ell^2)(4/3 P_0 - 2 P_1 + 2/3 P_2)(x) = (1 - x)^2 / ell^2 = 4 ell^2 / (r^2 + ell^2)^2.
Here both potentials may carry one: psi = psi~ + c_psi Lambda, chi = chi~ + c_chi Lambda (m = 0, k = 0).
With Eq. tp (u = curl(psi z) + curl curl(chi z)) the proxy parts contribute, at every node,
    u_phi = -c_psi dLambda/dr = -2 c_psi r / (r^2 + ell^2),     u_z = -c_chi grad_h^2 Lambda,
    w_phi = c_chi d(grad_h^2 Lambda)/dr = -16 c_chi ell^2 r / (r^2 + ell^2)^3,
    w_z = -c_psi grad_h^2 Lambda,                              u_r = w_r = 0.
The amplitudes are constants of the motion: the circulation at infinity is -4 pi c_psi and the axial
volume flux -4 pi c_chi, both conserved.  The evolution of the regular parts therefore gains the
dissipation of the proxy parts as a constant forcing of the m = 0, k = 0 column:
    d psi~ / dt = psi_N + L psi~ + c_psi L Lambda,   L Lambda = nu g + nu_h (-Dbar_0)^{p/2 - 1} g,
g the coefficient vector of grad_h^2 Lambda in the normalised basis (Pbar_n^0 = sqrt((2n+1)/2) P_n)
and Dbar_0 the truncated horizontal Laplacian of Eq. del2h-entries, its power the matrix power as in
the dissipation of Eq. dissipation; the same for chi~ with c_chi.

Enstrophy: (1/2) int |w|^2 dV over one axial period, by the area quadrature of the nodes and the
trapezoidal rule in phi and z (the reading of the paper's enstrophy used here).
"""
from __future__ import annotations

import numpy as np

from .basis import laplacian_matrix
from .grid import Grid
from .rhs import (VecTables, apply_mask, cross_with_background, dealias_mask, projection_sources,
                  solve_projection, synthesize)


def laplacian_image(nrc: int, ell: float) -> np.ndarray:
    """g: coefficients of grad_h^2 Lambda on Pbar_0^0 .. Pbar_{N_r^c - 1}^0 (Eq. logproxy)."""
    g = np.zeros(nrc)
    unnorm = [4.0 / 3.0, -2.0, 2.0 / 3.0]          # on the unnormalised P_0, P_1, P_2
    for n, a in enumerate(unnorm[:nrc]):
        g[n] = a / np.sqrt((2 * n + 1) / 2.0) / ell ** 2
    return g


def proxy_fields(r: np.ndarray, ell: float, c_psi: float, c_chi: float):
    """(u_phi, u_z, w_phi, w_z) of c_psi Lambda and c_chi Lambda at the radii r."""
    d = r ** 2 + ell ** 2
    lap = 4.0 * ell ** 2 / d ** 2
    return (-2.0 * c_psi * r / d, -c_chi * lap, -16.0 * c_chi * ell ** 2 * r / d ** 3, -c_psi * lap)


def synthesize_log(psi, chi, g: Grid, vt: VecTables, c_psi: float, c_chi: float):
    """Nodal u and w of (psi~ + c_psi Lambda, chi~ + c_chi Lambda)."""
    u, w = synthesize(psi, chi, g, vt)
    up, uz, wp, wz = (f[None, :, None] for f in proxy_fields(g.r, g.ell, c_psi, c_chi))
    return [u[0], u[1] + up, u[2] + uz], [w[0], w[1] + wp, w[2] + wz]


def rhs_tp_log(psi, chi, g: Grid, vt: VecTables, U=(0.0, 0.0, 0.0), dealias: bool = True, c_psi: float = 0.0,
               c_chi: float = 0.0, taps: dict | None = None):
    """rhs_tp of the regular parts when the potentials carry proxy amplitudes (the projection keeps
    the decay gauge: the amplitudes do not change).  Dealiasing masks the regular parts on the way
    in, as in rhs_tp; the proxies are axisymmetric and axially uniform (m = 0, k = 0)."""
    if dealias:
        psi, chi = apply_mask(psi, g), apply_mask(chi, g)
    u, w = synthesize_log(psi, chi, g, vt, c_psi, c_chi)
    Nr_, Np_, Nz_ = cross_with_background(u, w, U, g)
    C, K, Z = projection_sources(Nr_, Np_, Nz_, g, vt)
    if dealias:
        mk = dealias_mask(g)[:, None, :]
        C, K, Z = C * mk, K * mk, Z * mk
    if taps is not None:
        taps.update(u=u, w=w, N=(Nr_, Np_, Nz_), C=C, K=K, Z=Z)
    return solve_projection(C, K, Z, g, dealias)


def proxy_forcing(g: Grid, nu: float, nu_h: float = 0.0, p: int = 8) -> np.ndarray:
    """L Lambda on the m = 0, k = 0 column: nu g + nu_h (-Dbar_0)^{p/2 - 1} g."""
    gv = laplacian_image(g.nrc, g.ell)
    out = nu * gv
    if nu_h != 0.0:
        D = laplacian_matrix(0, g.nrc, g.ell)
        out = out + nu_h * np.linalg.matrix_power(-D, p // 2 - 1) @ gv
    return out


def add_forcing(N: np.ndarray, f: np.ndarray, c: float) -> np.ndarray:
    """Dense (M, N_r^c, N_z) with c f added to the m = 0, k = 0 column."""
    out = N.copy()
    out[0, :, 0] += c * f
    return out


def enstrophy(psi, chi, g: Grid, vt: VecTables, c_psi: float = 0.0, c_chi: float = 0.0) -> float:
    """(1/2) int |w|^2 dV over one axial period."""
    _, w = synthesize_log(psi, chi, g, vt, c_psi, c_chi)
    tot = sum((c ** 2 * g.area_w[None, :, None]).sum() for c in w)
    return 0.5 * tot * (g.lz / g.nz) * (2 * np.pi / g.nphi)
