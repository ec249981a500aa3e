"""Oracle: the Fisher-KPP front of Sec. 5.2 (Example 2): closed form, error norm, front radius.

Test infrastructure only (see the package header).

Eq. kpp: u_t = D grad^2 u + gamma u (1 - u) on the unbounded plane, seeded by the axisymmetric
Gaussian u(r, 0) = A exp(-r^2 / (2 sigma^2)).  While u << 1 the reaction is linear and
Eq. kpp-linear gives the exact solution
    u(r, t) = A sigma^2 / (sigma^2 + 2 D t) e^{gamma t} exp(-r^2 / (2 (sigma^2 + 2 D t))).
The front radius is the largest radius at which the azimuthal average of u exceeds one half; the
average of a field is its m = 0 harmonic, evaluated here from the spectral coefficients at any
radius through the normalised functions of the basis module and located by bisection.

Readings: the "relative weighted L2 error" is taken with the area quadrature of the grid
(Gauss-Legendre in the mapped variable, r dr = ell^2 / (1 - x)^2 dx, trapezoidal in phi) over the
collocation nodes; the front radius is bracketed on a uniform radial scan of step h and then bisected.
"""
from __future__ import annotations

import numpy as np

from .basis import pbar
from .grid import Grid


def linear_solution(r: np.ndarray, t: float, A: float = 1e-6, sigma: float = 1.0, D: float = 1.0,
                    gamma: float = 0.25) -> np.ndarray:
    """Eq. kpp-linear."""
    s2 = sigma ** 2 + 2.0 * D * t
    return A * sigma ** 2 / s2 * np.exp(gamma * t) * np.exp(-r ** 2 / (2.0 * s2))


def weighted_rel_error(u: np.ndarray, u_ref: np.ndarray, g: Grid) -> float:
    """sqrt(sum W (u - u_ref)^2 / sum W u_ref^2) over the physical nodes (N_z, N_r, N_phi)."""
    W = g.area_w[None, :, None]
    return float(np.sqrt((W * (u - u_ref) ** 2).sum() / (W * u_ref ** 2).sum()))


def harmonic_at(S: np.ndarray, g: Grid, m: int, kk: int, r: np.ndarray) -> np.ndarray:
    """sum_n S[m, n, kk] Pbar_n^m(x(r)) for the dense oracle layout (M, N_r^c, N_z)."""
    r = np.atleast_1d(np.asarray(r, dtype=np.longdouble))
    ell = np.longdouble(g.ell)
    x = (r ** 2 - ell ** 2) / (r ** 2 + ell ** 2)
    P = pbar(m, g.nrc, x)[m:]           # degrees n = m .. N_r^c - 1 (rows), radii (columns)
    Sc = S[m, m:, kk].astype(np.clongdouble)
    return (Sc @ P).astype(np.complex128)


def front_radius(S: np.ndarray, g: Grid, r_max: float, h: float = 0.25, level: float = 0.5) -> float:
    """Largest r in [0, r_max] with Re f_00(r) > level (nan if there is none)."""
    r = np.arange(0.0, r_max + h, h)
    f = harmonic_at(S, g, 0, 0, r).real
    above = np.nonzero(f > level)[0]
    if above.size == 0:
        return float("nan")
    i = above[-1]
    if i + 1 >= r.size:
        return float(r[-1])
    a, b = r[i], r[i + 1]
    for _ in range(60):
        c = 0.5 * (a + b)
        if harmonic_at(S, g, 0, 0, np.array([c])).real[0] > level:
            a = c
        else:
            b = c
    return 0.5 * (a + b)
