"""Oracle: the bounded adaptive modal filter of Sec. 3.3 (the paragraph on aliasing and dissipation).

Test infrastructure only (see the package header).

The paper's filter, applied to a field between time steps: every retained coefficient s_{n m k}
whose normalised index zeta (the largest of its radial, azimuthal and axial indices, each divided
by its own truncation) lies above a cutoff zeta_c is multiplied by
    sigma = exp(-eps ((zeta - zeta_c) / (1 - zeta_c))^8).
The amplitude eps is not fixed: it follows the fraction f of the field's coefficient energy held
above the cutoff, stays zero while f is below a target tau (2e-2 by default), grows as f passes
tau and saturates from f = 2 tau on; it is bounded, relaxed from one application to the next, and
every field keeps its own.

Readings (the paper fixes none of these numbers or forms):
* zeta = max(n / N_r^c, m / N_phi^c, |k| / N_z^c) over the stored coefficients (n the degree,
  0 <= m < N_phi^c, |k| < N_z^c), so the last retained index of each direction sits just below 1;
* coefficient energy: the plain sum of |s|^2 over the stored coefficients (m >= 0);
* the response: target eps* = eps_max * clip((f - tau) / tau, 0, 1), a linear ramp between tau and
  2 tau, with eps_max = 36 (exp(-36) ~ 2e-16: full damping of the last retained index);
* relaxation: eps <- eps + r (eps* - eps), r = 0.1 per application, starting from eps = 0;
* zeta_c = 2/3 (the fraction the periodic directions keep under the two-thirds mask);
* one application measures f on the incoming field, updates eps, then applies sigma with the
  updated eps.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .grid import Grid


@dataclass
class FilterConfig:
    zeta_c: float = 2.0 / 3.0
    tau: float = 2e-2
    eps_max: float = 36.0
    relax: float = 0.1


def normalized_index(g: Grid) -> np.ndarray:
    """zeta for the dense oracle layout (M, N_r^c, N_z); entries n < m (not coefficients) are -1."""
    n = np.arange(g.nrc)[None, :, None].astype(float)
    m = np.arange(g.M)[:, None, None].astype(float)
    kk = np.arange(g.nz)
    k = np.where(2 * kk < g.nz, kk, kk - g.nz)
    kz = (np.abs(k) / g.nzc)[None, None, :]
    zeta = np.maximum(np.maximum(n / g.nrc, m / g.M), kz)
    valid = (np.arange(g.nrc)[None, :] >= np.arange(g.M)[:, None])[:, :, None]
    return np.where(valid, zeta, -1.0)


def tail_fraction(S: np.ndarray, g: Grid, cfg: FilterConfig) -> float:
    """Fraction of sum |s|^2 held by the coefficients with zeta > zeta_c (0 for a zero field)."""
    zeta = normalized_index(g)
    e = np.abs(S) ** 2
    total = e[zeta >= 0].sum()
    if total == 0.0:
        return 0.0
    return float(e[zeta > cfg.zeta_c].sum() / total)


def target_amplitude(f: float, cfg: FilterConfig) -> float:
    return cfg.eps_max * min(max((f - cfg.tau) / cfg.tau, 0.0), 1.0)


def relaxed_amplitude(eps_prev: float, f: float, cfg: FilterConfig) -> float:
    return eps_prev + cfg.relax * (target_amplitude(f, cfg) - eps_prev)


def transfer(zeta: np.ndarray, eps: float, cfg: FilterConfig) -> np.ndarray:
    """sigma(zeta): 1 at and below the cutoff, exp(-eps ((zeta - zeta_c) / (1 - zeta_c))^8) above."""
    t = (zeta - cfg.zeta_c) / (1.0 - cfg.zeta_c)
    return np.where(zeta > cfg.zeta_c, np.exp(-eps * t ** 8), 1.0)


def apply(S: np.ndarray, g: Grid, cfg: FilterConfig, eps_prev: float):
    """One application: (filtered S, updated eps, measured f)."""
    f = tail_fraction(S, g, cfg)
    eps = relaxed_amplitude(eps_prev, f, cfg)
    return S * transfer(normalized_index(g), eps, cfg), eps, f
