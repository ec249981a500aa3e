"""Oracle: the mapped radial grid and the periodic grids (Sec. 3.1, Eq. map).

Test infrastructure only (see the package header).

Radial collocation uses the N_r Gauss-Legendre nodes x_i in [-1, 1) (the roots
of P_{N_r}), ordered ascending, with quadrature weights w_i.  The algebraic map
of Eq. map sends them to r_i = ell * sqrt((1 + x_i) / (1 - x_i)), so exactly
half of the nodes lie inside r < ell (Sec. 1, Fig. grid caption).

The nodes are found here by Golub-Welsch (eigenvalues of the Jacobi matrix of
the Legendre polynomials) followed by Newton polishing on P_{N_r} in extended
precision; the HIP library uses an unrelated Newton iteration in theta.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LD = np.longdouble


def _legendre_and_derivative(n: int, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """P_n(x) and P_n'(x) by the Bonnet three-term recurrence, in long double."""
    x = np.asarray(x, dtype=LD)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # (x^2 - 1) P_n' = n (x P_n - P_{n-1})
    dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def gauss_legendre(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre nodes (ascending) and weights on [-1, 1], returned in long double.

    Golub-Welsch gives the starting values (the Jacobi matrix of the monic
    Legendre recurrence has zero diagonal and off-diagonal k / sqrt(4k^2 - 1));
    three Newton steps on P_n in long double then fix the nodes to ~1e-19, and
    the weights follow from w = 2 / ((1 - x^2) P_n'(x)^2).
    """
    if n < 1:
        raise ValueError("need at least one node")
    k = np.arange(1, n, dtype=np.float64)
    off = k / np.sqrt(4.0 * k * k - 1.0)
    jac = np.diag(off, 1) + np.diag(off, -1)
    x = np.sort(np.linalg.eigvalsh(jac)).astype(LD)
    for _ in range(4):
        p, dp = _legendre_and_derivative(n, x)
        x = x - p / dp
    _, dp = _legendre_and_derivative(n, x)
    w = 2 / ((1 - x * x) * dp * dp)
    return x, w


@dataclass
class Grid:
    """Collocation grid and chops of one scalar field.

    Chops follow Sec. 3.1: N_r^c <= N_r, N_phi^c <= N_phi/2 + 1,
    N_z^c <= N_z/2 + 1.  Defaults: N_r^c = N_r, M = N_phi^c = N_phi/2
    (the azimuthal Nyquist order is not kept), N_z^c = N_z/2 (so |k| <= N_z/2 - 1;
    for N_z = 1 only k = 0).
    """

    nr: int
    nphi: int
    nz: int
    ell: float
    lz: float = 2 * np.pi
    nrc: int = 0
    nphic: int = 0
    nzc: int = 0

    def __post_init__(self):
        if self.nr < 2 or self.nphi < 1 or self.nz < 1:
            raise ValueError("bad grid size")
        if not (self.ell > 0 and self.lz > 0):
            raise ValueError("ell and L_z must be positive")
        if self.nrc == 0:
            self.nrc = self.nr
        if self.nphic == 0:
            self.nphic = max(1, self.nphi // 2)
        if self.nzc == 0:
            self.nzc = max(1, self.nz // 2)
        if self.nrc > self.nr or self.nphic > self.nphi // 2 + 1 or self.nzc > self.nz // 2 + 1:
            raise ValueError("chop exceeds its bound")
        xl, wl = gauss_legendre(self.nr)
        self.x_ld = xl
        self.x = xl.astype(np.float64)
        self.w = wl.astype(np.float64)
        one_minus = (1 - xl)
        one_plus = (1 + xl)
        self.one_minus_x = one_minus.astype(np.float64)
        self.one_plus_x = one_plus.astype(np.float64)
        self.sin_theta = np.sqrt(one_minus * one_plus).astype(np.float64)
        # Eq. map, inverted: r = ell sqrt((1+x)/(1-x))
        self.r = (LD(self.ell) * np.sqrt(one_plus / one_minus)).astype(np.float64)
        # q = (1-x)^2 / ell^2 appears in the nodal horizontal Laplacian
        self.q = (one_minus * one_minus / LD(self.ell) ** 2).astype(np.float64)
        # area element r dr dphi = ell^2/(1-x)^2 dx dphi  (dx = r (1-x)^2/ell^2 dr)
        self.area_w = (wl * LD(self.ell) ** 2 / (one_minus * one_minus)).astype(np.float64)
        self.phi = 2 * np.pi * np.arange(self.nphi) / self.nphi
        self.z = self.lz * np.arange(self.nz) / self.nz

    @property
    def M(self) -> int:
        """Number of stored azimuthal orders m = 0 .. M-1."""
        return self.nphic

    def kvals(self) -> np.ndarray:
        """Signed axial index k for each slot of a length-N_z FFT-ordered axis."""
        return np.fft.fftfreq(self.nz, d=1.0 / self.nz).round().astype(int)

    def kappa(self) -> np.ndarray:
        """Axial wavenumbers kappa_k = 2 pi k / L_z per FFT slot (Sec. 3.1)."""
        return 2 * np.pi * self.kvals() / self.lz

    def kmask(self) -> np.ndarray:
        """True for FFT slots kept by the axial chop: |k| < N_z^c and not Nyquist."""
        k = self.kvals()
        keep = np.abs(k) < self.nzc
        if self.nz % 2 == 0 and self.nz > 1:
            keep &= k != -(self.nz // 2)
        return keep

    def dealias_m(self) -> int:
        """Largest azimuthal order kept by the two-thirds mask (Sec. 3.3)."""
        return (self.nphi - 1) // 3

    def dealias_k(self) -> int:
        """Largest |k| kept by the two-thirds mask (Sec. 3.3)."""
        return (self.nz - 1) // 3
