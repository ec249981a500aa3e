"""Oracle: normalised associated Legendre functions and radial operators.

Test infrastructure only (see the package header).

* ``pbar(m, nmax, x)``: the normalised functions Pbar_n^m = N_n^m P_n^m of
  Eq. norm (Sec. 3.1), no Condon-Shortley phase (Pbar_m^m > 0), evaluated by
  the normalised three-term recurrence in long double.  The recurrence ratios
  are exactly the ones the paper writes for ln N_n^m, so no factorial is formed.
* ``tbar(m, nmax, x)``: (1 - x^2) dPbar_n^m/dx = r d/dr Pbar_n^m (the radial
  derivative through the map of Eq. map), from the recurrence differentiated
  term by term.
* ``laplacian_matrix(m, nrc, ell)``: the pentadiagonal horizontal Laplacian of
  Eq. del2h-entries, written for the unnormalised P_n^m and rescaled to the
  normalised basis by exp(ln N_j - ln N_i) with ln N accumulated from the
  ratio given after Eq. norm.
"""
from __future__ import annotations

import numpy as np

LD = np.longdouble


def pbar(m: int, nmax: int, x: np.ndarray) -> np.ndarray:
    """Pbar_n^m(x) for n = 0 .. nmax-1 (rows); rows n < m are zero.  Long double."""
    x = np.asarray(x, dtype=LD)
    out = np.zeros((nmax, x.size), dtype=LD)
    if m >= nmax:
        return out
    s = np.sqrt((1 - x) * (1 + x))
    # Pbar_m^m = sqrt(1/2) prod_{j=1..m} sqrt((2j+1)/(2j)) sin^m(theta)
    c = np.sqrt(LD(0.5))
    pmm = np.full_like(x, c)
    for j in range(1, m + 1):
        pmm = pmm * np.sqrt(LD(2 * j + 1) / LD(2 * j)) * s
    out[m] = pmm
    if m + 1 < nmax:
        out[m + 1] = np.sqrt(LD(2 * m + 3)) * x * pmm
    for n in range(m + 2, nmax):
        a = np.sqrt(LD(4 * n * n - 1) / LD(n * n - m * m))
        b = np.sqrt(LD((2 * n + 1) * (n - 1 - m) * (n - 1 + m)) / LD((2 * n - 3) * (n * n - m * m)))
        out[n] = a * x * out[n - 1] - b * out[n - 2]
    return out


def tbar(m: int, nmax: int, x: np.ndarray) -> np.ndarray:
    """(1 - x^2) dPbar_n^m/dx for n = 0 .. nmax-1, by differentiating the recurrence.

    With T_n := (1-x^2) Pbar_n':  T_m = -m x Pbar_m^m (from d sin^m/dx), then
    T_{m+1} = sqrt(2m+3) [(1-x^2) Pbar_m + x T_m] and
    T_n = a_n [(1-x^2) Pbar_{n-1} + x T_{n-1}] - b_n T_{n-2}.
    """
    x = np.asarray(x, dtype=LD)
    p = pbar(m, nmax, x)
    out = np.zeros_like(p)
    if m >= nmax:
        return out
    one_m_x2 = (1 - x) * (1 + x)
    out[m] = -m * x * p[m]
    if m + 1 < nmax:
        out[m + 1] = np.sqrt(LD(2 * m + 3)) * (one_m_x2 * p[m] + x * out[m])
    for n in range(m + 2, nmax):
        a = np.sqrt(LD(4 * n * n - 1) / LD(n * n - m * m))
        b = np.sqrt(LD((2 * n + 1) * (n - 1 - m) * (n - 1 + m)) / LD((2 * n - 3) * (n * n - m * m)))
        out[n] = a * (one_m_x2 * p[n - 1] + x * out[n - 1]) - b * out[n - 2]
    return out


def log_norm(m: int, nmax: int) -> np.ndarray:
    """ln N_n^m up to an m-dependent constant, for n = m .. nmax-1 (index n; rows n<m unused).

    Accumulated from 2 ln(N_n/N_{n-1}) = ln[(2n+1)(n-|m|)] - ln[(2n-1)(n+|m|)]
    (Sec. 3.1, after Eq. norm).  Only differences are ever used.
    """
    out = np.zeros(nmax + 2, dtype=np.float64)
    for n in range(m + 1, nmax + 2):
        out[n] = out[n - 1] + 0.5 * (np.log((2 * n + 1) * (n - m)) - np.log((2 * n - 1) * (n + m)))
    return out


def _del2h_unnormalised_row(n: int, m: int) -> dict[int, float]:
    """Eq. del2h-entries: ell^2 (grad_h^2 s)_n as coefficients on s_{n-2..n+2} (unnormalised P)."""
    am = abs(m)
    return {
        n - 2: -((n - am - 1) * (n - am) * (n - 2) * (n - 1)) / ((2 * n - 3) * (2 * n - 1)),
        n - 1: (2 * n * (n - 1) * (n - am)) / (2 * n - 1),
        n: -(2 * n * (n + 1) * (3 * n * n + 3 * n - m * m - 2)) / ((2 * n - 1) * (2 * n + 3)),
        n + 1: (2 * (n + 1) * (n + 2) * (n + am + 1)) / (2 * n + 3),
        n + 2: -((n + 2) * (n + 3) * (n + am + 1) * (n + am + 2)) / ((2 * n + 3) * (2 * n + 5)),
    }


def laplacian_matrix(m: int, nrc: int, ell: float) -> np.ndarray:
    """Dbar_m: the truncated normalised horizontal Laplacian on n = m .. nrc-1.

    Dbar[i, j] = D[i, j] exp(ln N_j - ln N_i) / ell^2 with D from
    Eq. del2h-entries; entries with an index < |m| or >= nrc are dropped
    (truncated matrix, Sec. 3.1).  Returned as a dense (nrc-m) x (nrc-m) array.
    """
    size = nrc - m
    lnn = log_norm(m, nrc)
    d = np.zeros((size, size))
    for n in range(m, nrc):
        for j, v in _del2h_unnormalised_row(n, m).items():
            if m <= j < nrc:
                d[n - m, j - m] = v * np.exp(lnn[j] - lnn[n]) / ell ** 2
    return d

