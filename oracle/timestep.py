"""Oracle: semi-implicit time integration of ds/dt = A(s) + L s (Sec. 3.3).

Test infrastructure only (see the package header).

* Eq. dissipation: L = nu grad^2 - nu_h (-grad^2)^{p/2}, p in {4, 6, 8}; per
  harmonic grad^2 = Dbar_m - kappa_k^2 I with the truncated Dbar_m of
  Eq. del2h-entries, and the power is the matrix power of that truncated matrix.
* FE-BE: s <- (I - h L)^{-1} (s + h A(s)).
* AB-CN, Eq. abcn:
  (I - dt/2 L) s^{j+1} = (I + dt/2 L) s^j + dt/2 (3 A^j - A^{j-1}).
* Start-up: Richardson extrapolation from FE-BE sub-steps (Sec. 3.3),
  s^1 = 2 S_{dt/2}(S_{dt/2}(s^0)) - S_dt(s^0), S_h the FE-BE step; A^0 = A(s^0).

Spectral states use the oracle layout (M, N_r^c, N_z); each (m, k) column is
advanced with dense matrices.

Pins: the printed Table tab:oseen and the manufactured mode (nu only, no axial
dependence); the -kappa^2 shift and the hyperviscous power against symbolic
(-grad^2)^{p/2} of fields in the retained span, and AB-CN with kappa != 0 against
the three-dimensional heat kernel (tests/test_oracle_dissipation_pins.py).
"""
from __future__ import annotations

from typing import Callable

import numpy as np

from .basis import laplacian_matrix
from .grid import Grid


class Dissipation:
    """Dense per-(m, k) matrices of L and the factors the integrators need."""

    def __init__(self, g: Grid, nu: float, nu_h: float = 0.0, p: int = 8):
        if p not in (4, 6, 8):
            raise ValueError("p must be 4, 6 or 8")
        if nu_h < 0:
            raise ValueError("nu_h must be non-negative")
        self.g = g
        kap = g.kappa()
        self.L = {}
        for m in range(min(g.M, g.nrc)):
            D = laplacian_matrix(m, g.nrc, g.ell)
            eye = np.eye(D.shape[0])
            for kk in range(g.nz):
                lap = D - kap[kk] ** 2 * eye
                op = nu * lap
                if nu_h != 0.0:
                    op = op - nu_h * np.linalg.matrix_power(-lap, p // 2)
                self.L[(m, kk)] = op

    def apply_inverse(self, S: np.ndarray, h: float) -> np.ndarray:
        """(I - h L)^{-1} S, column by column."""
        out = np.zeros_like(S)
        for (m, kk), op in self.L.items():
            a = np.eye(op.shape[0]) - h * op
            out[m, m:, kk] = np.linalg.solve(a, S[m, m:, kk])
        return out

    def apply(self, S: np.ndarray, h: float) -> np.ndarray:
        """(I + h L) S."""
        out = np.zeros_like(S)
        for (m, kk), op in self.L.items():
            out[m, m:, kk] = S[m, m:, kk] + h * (op @ S[m, m:, kk])
        return out


NonLinear = Callable[[np.ndarray], np.ndarray]


def fe_be_step(S: np.ndarray, h: float, diss: Dissipation, A: NonLinear) -> np.ndarray:
    """S_h(s) = (I - h L)^{-1} (s + h A(s))."""
    return diss.apply_inverse(S + h * A(S), h)


def richardson_start(S0: np.ndarray, dt: float, diss: Dissipation, A: NonLinear) -> np.ndarray:
    """s^1 = 2 S_{dt/2}(S_{dt/2}(s^0)) - S_dt(s^0)."""
    half = fe_be_step(fe_be_step(S0, dt / 2, diss, A), dt / 2, diss, A)
    full = fe_be_step(S0, dt, diss, A)
    return 2 * half - full


def abcn_step(S: np.ndarray, A_now: np.ndarray, A_prev: np.ndarray, dt: float,
              diss: Dissipation) -> np.ndarray:
    """Eq. abcn."""
    rhs = diss.apply(S, dt / 2) + dt / 2 * (3 * A_now - A_prev)
    return diss.apply_inverse(rhs, dt / 2)


def integrate_abcn(S0: np.ndarray, dt: float, nsteps: int, diss: Dissipation, A: NonLinear) -> np.ndarray:
    """Richardson start then nsteps-1 AB-CN steps (nsteps total steps of size dt)."""
    A_prev = A(S0)
    S = richardson_start(S0, dt, diss, A)
    for _ in range(nsteps - 1):
        A_now = A(S)
        S = abcn_step(S, A_now, A_prev, dt, diss)
        A_prev = A_now
    return S


def integrate_febe(S0: np.ndarray, dt: float, nsteps: int, diss: Dissipation, A: NonLinear) -> np.ndarray:
    S = S0
    for _ in range(nsteps):
        S = fe_be_step(S, dt, diss, A)
    return S
