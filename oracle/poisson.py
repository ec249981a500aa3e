"""Oracle: inversion of the Laplacian with the logarithmic proxy, and removal of the far-field level
of axisymmetric components (Sec. 3.1: the far-field paragraph, Eq. laplacian, Eq. logproxy).

Test infrastructure only (see the package header).

* Far-field level (Sec. 3.1): every basis function of order m != 0 decays as r -> infinity, but
  Pbar_n^0 tends to Pbar_n^0(1) = sqrt((2n + 1)/2), so an m = 0 harmonic has the free level
  sum_n sqrt((2n + 1)/2) shat_n at infinity.  Removing it adjusts the regular coefficients so that
  the limit vanishes.  Reading: the adjustment is made through the constant basis function
  Pbar_0^0 = 1/sqrt(2) alone (shat_0 -= level / Pbar_0^0(1)), i.e. the constant at infinity is
  subtracted from the component everywhere, which leaves every derivative of the field unchanged.
* Inversion (Eq. laplacian): per harmonic, (Dbar_m - kappa_k^2 I) shat = fhat with the truncated
  Dbar_m of Eq. del2h-entries (dense here).  The m = k = 0 block is singular (Dbar_0 annihilates the
  constant); a scalar may carry one extra real amplitude c of Lambda = ln(r^2 + ell^2), whose
  horizontal Laplacian has the coefficient vector g (Eq. logproxy), and the paper gives two
  variants that differ only in that block:
  - 'prescribe': c is given; the first row of Dbar_0 is replaced by a constraint and the system
    Dbar_0 shat = fhat - c g is solved.  Reading: the constraint is the decay gauge
    sum_n Pbar_n^0(1) shat_n = 0 (the regular part vanishes at infinity), with right-hand side 0.
  - 'solve': the first column of Dbar_0 is replaced by g, so that the unknown that multiplied
    Pbar_0^0 becomes c; [g | Dbar_0[:, 1:]] (c, shat_1, ...) = fhat.  The constant shat_0 that the
    Laplacian cannot see is then fixed by the same decay gauge (reading).
  The potential is s = c Lambda + sum shat_n Pbar_n^0 in both variants.  The m = k = 0 column of a
  real field is real: the block uses the real part of fhat there and returns a real column and a
  real c.
"""
from __future__ import annotations

import numpy as np

from .basis import laplacian_matrix
from .grid import Grid
from .logproxy import laplacian_image


def far_field_weights(nrc: int) -> np.ndarray:
    """Pbar_n^0(1) = sqrt((2n + 1) / 2), n = 0 .. N_r^c - 1."""
    return np.sqrt((2 * np.arange(nrc) + 1) / 2.0)


def far_field_level(S: np.ndarray, g: Grid) -> np.ndarray:
    """Level at r -> infinity of the m = 0 harmonic of every axial slot: sum_n Pbar_n^0(1) shat_n."""
    return far_field_weights(g.nrc) @ S[0]


def remove_far_field(S: np.ndarray, g: Grid) -> np.ndarray:
    """S with the far-field level of each m = 0 harmonic removed through shat_0."""
    out = S.copy()
    v = far_field_weights(g.nrc)
    out[0, 0, :] -= far_field_level(S, g) / v[0]
    return out


def laplacian_solve(F: np.ndarray, g: Grid, variant: str = "solve", c: float = 0.0):
    """(grad^2)^{-1} F for a scalar in the oracle layout (M, N_r^c, N_z); returns (S, c).

    variant 'prescribe' uses the given c; 'solve' returns the c it solves for."""
    if variant not in ("prescribe", "solve"):
        raise ValueError("variant must be 'prescribe' or 'solve'")
    S = np.zeros_like(F)
    kap = g.kappa()
    keep = g.kmask()
    for m in range(min(g.M, g.nrc)):
        D = laplacian_matrix(m, g.nrc, g.ell)
        for kk in range(g.nz):
            if not keep[kk]:
                continue
            f = F[m, m:, kk]
            if m == 0 and kap[kk] == 0.0:
                continue
            S[m, m:, kk] = np.linalg.solve(D - kap[kk] ** 2 * np.eye(D.shape[0]), f)
    if not keep[0]:
        return S, c
    D0 = laplacian_matrix(0, g.nrc, g.ell)
    gv = laplacian_image(g.nrc, g.ell)
    v = far_field_weights(g.nrc)
    f = F[0, :, 0].real
    if variant == "prescribe":
        A = D0.copy()
        A[0, :] = v
        b = f - c * gv
        b[0] = 0.0
        S[0, :, 0] = np.linalg.solve(A, b)
        return S, float(c)
    A = D0.copy()
    A[:, 0] = gv
    x = np.linalg.solve(A, f)
    c_out = float(x[0])
    reg = x.copy()
    reg[0] = 0.0
    reg[0] = -(v @ reg) / v[0]
    S[0, :, 0] = reg
    return S, c_out
