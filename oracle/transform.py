"""Oracle: the physical <-> spectral transform pair of Eq. expansion (Sec. 3.1, Sec. 4.1).

Test infrastructure only (see the package header).

Layouts used by the oracle (the HIP library uses its own; tests convert
between the two by pure index permutation):

* physical real field  s[l, i, j] = s(r_i, phi_j, z_l), shape (N_z, N_r, N_phi);
* spectral complex     S[m, n, kk] = shat_{n m k}, shape (M, N_r^c, N_z), with
  kk the FFT slot of k (numpy ``fftfreq`` order); rows n < m, slots outside the
  axial chop and the Nyquist slot are zero.

Forward (physical -> spectral), the plain sum
    shat_{nmk} = sum_i w_i Pbar_n^m(x_i) (1/(N_phi N_z)) sum_{j,l} s_{ijl} exp(-i m phi_j - i kappa_k z_l)
for 0 <= m < M, |k| < N_z^c, m <= n < N_r^c (quadrature orthonormality of
Pbar makes this the inverse of the expansion on band-limited data).

Backward (spectral -> physical), Eq. expansion with shat_{n,-m,-k} = conj(shat_{nmk}):
    s_{ijl} = sum_k sum_{|m| < M} sum_n shat_{n|m|k}^(*) Pbar_n^|m|(x_i) exp(i m phi_j + i kappa_k z_l).
The m = 0 harmonic enters through its real part (a real field has a Hermitian
m = 0 column; the transform does not enforce it).

FFTs (numpy) serve as single steps; ``*_bruteforce`` evaluate the same sums by
explicit loops over every index and are used by the pins on tiny grids.
"""
from __future__ import annotations

import numpy as np

from .basis import pbar
from .grid import Grid


class Tables:
    """Pbar_n^m(x_i) for every stored m, rounded to double: P[m] has shape (N_r^c, N_r)."""

    def __init__(self, g: Grid):
        self.g = g
        self.P = [pbar(m, g.nrc, g.x_ld).astype(np.float64) for m in range(g.M)]


def _spectral_zero(g: Grid) -> np.ndarray:
    return np.zeros((g.M, g.nrc, g.nz), dtype=np.complex128)


def azimuthal_forward(s: np.ndarray, g: Grid) -> np.ndarray:
    """(1/N_phi) sum_j s[..., j] exp(-i m phi_j) for m = 0..M-1; real last axis -> complex."""
    f = np.fft.rfft(s, axis=-1) / g.nphi
    out = np.zeros(s.shape[:-1] + (g.M,), dtype=np.complex128)
    mm = min(g.M, f.shape[-1])
    out[..., :mm] = f[..., :mm]
    if g.nphi % 2 == 0 and g.M > g.nphi // 2:
        out[..., g.nphi // 2] = 0.0  # the Nyquist order is never kept
    return out


def azimuthal_backward(f: np.ndarray, g: Grid) -> np.ndarray:
    """Re f_0 + 2 Re sum_{1<=m<M} f_m exp(i m phi_j): the Hermitian synthesis in phi."""
    s = np.zeros(f.shape[:-1] + (g.nphi,), dtype=np.float64)
    for m in range(g.M):
        if g.nphi % 2 == 0 and m == g.nphi // 2:
            continue
        e = np.exp(1j * m * g.phi)
        term = f[..., m, None] * e
        s += term.real if m == 0 else 2.0 * term.real
    return s


def axial_forward(a: np.ndarray, g: Grid, axis: int) -> np.ndarray:
    """(1/N_z) sum_l a_l exp(-i kappa_k z_l), zeroing slots outside the chop and Nyquist."""
    out = np.fft.fft(a, axis=axis) / g.nz
    shape = [1] * out.ndim
    shape[axis] = g.nz
    return out * g.kmask().reshape(shape)


def axial_backward(a: np.ndarray, g: Grid, axis: int) -> np.ndarray:
    """sum_{kept k} a_k exp(+i kappa_k z_l)."""
    shape = [1] * a.ndim
    shape[axis] = g.nz
    return np.fft.ifft(a * g.kmask().reshape(shape), axis=axis) * g.nz


def radial_forward(f_m: np.ndarray, P_m: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum_i w_i Pbar_n(x_i) f[i, ...]  (Gauss-Legendre projection onto Pbar_n)."""
    return (P_m * w[None, :]) @ f_m


def radial_backward(c_m: np.ndarray, P_m: np.ndarray) -> np.ndarray:
    """sum_n Pbar_n(x_i) c[n, ...]."""
    return P_m.T @ c_m


def forward(s: np.ndarray, g: Grid, t: Tables) -> np.ndarray:
    """Physical (N_z, N_r, N_phi) real -> spectral (M, N_r^c, N_z) complex."""
    f = azimuthal_forward(s, g)            # (N_z, N_r, M)
    S = _spectral_zero(g)
    for m in range(g.M):
        S[m] = radial_forward(f[:, :, m].T, t.P[m], g.w)   # (N_r^c, N_z)
    return axial_forward(S, g, axis=2)


def backward(S: np.ndarray, g: Grid, t: Tables) -> np.ndarray:
    """Spectral (M, N_r^c, N_z) -> physical (N_z, N_r, N_phi) real."""
    a = axial_backward(S, g, axis=2)       # (M, N_r^c, N_z) in physical z
    f = np.zeros((g.nz, g.nr, g.M), dtype=np.complex128)
    for m in range(g.M):
        f[:, :, m] = radial_backward(a[m], t.P[m]).T
    return azimuthal_backward(f, g)


def mixed_backward(S: np.ndarray, g: Grid, t: Tables) -> np.ndarray:
    """Spectral -> harmonics at the radial nodes, (M, N_r, N_z) complex in spectral k."""
    out = np.zeros((g.M, g.nr, g.nz), dtype=np.complex128)
    for m in range(g.M):
        out[m] = radial_backward(S[m] * g.kmask()[None, :], t.P[m])
    return out


def forward_bruteforce(s: np.ndarray, g: Grid) -> np.ndarray:
    """The forward sum with explicit loops (tiny grids only)."""
    S = _spectral_zero(g)
    kap = g.kappa()
    keep = g.kmask()
    for m in range(g.M):
        P = pbar(m, g.nrc, g.x_ld).astype(np.float64)
        for kk in range(g.nz):
            if not keep[kk]:
                continue
            for n in range(m, g.nrc):
                acc = 0j
                for i in range(g.nr):
                    inner = 0j
                    for j in range(g.nphi):
                        for l in range(g.nz):
                            inner += s[l, i, j] * np.exp(-1j * m * g.phi[j] - 1j * kap[kk] * g.z[l])
                    acc += g.w[i] * P[n, i] * inner / (g.nphi * g.nz)
                S[m, n, kk] = acc
    return S


def backward_bruteforce(S: np.ndarray, g: Grid) -> np.ndarray:
    """Eq. expansion summed term by term over m in (-M, M), all kept k and n (tiny grids only)."""
    s = np.zeros((g.nz, g.nr, g.nphi), dtype=np.complex128)
    kv = g.kvals()
    keep = g.kmask()
    Ps = [pbar(m, g.nrc, g.x_ld).astype(np.float64) for m in range(g.M)]
    slot = {int(k): kk for kk, k in enumerate(kv)}
    for l in range(g.nz):
        for i in range(g.nr):
            for j in range(g.nphi):
                acc = 0j
                for m in range(-(g.M - 1), g.M):
                    if g.nphi % 2 == 0 and abs(m) == g.nphi // 2:
                        continue
                    for kk in range(g.nz):
                        if not keep[kk]:
                            continue
                        k = int(kv[kk])
                        for n in range(abs(m), g.nrc):
                            if m >= 0:
                                c = S[m, n, kk]
                            else:  # shat_{n,-m,-k} = conj(shat_{n,m,k})
                                c = np.conj(S[-m, n, slot[-k]])
                            acc += c * Ps[abs(m)][n, i] * np.exp(1j * m * g.phi[j] + 2j * np.pi * k * g.z[l] / g.lz)
                s[l, i, j] = acc
    # m = 0 enters through its real part; for m != 0 the (m, -m) pairs are conjugate
    return s.real


# ----------------------------------------------------------------- sampled evaluation
# The same sums for a few output columns or points, for checks at sizes where the full
# transform is slow on the host.

def forward_columns(s: np.ndarray, g: Grid, cols):
    """The forward sum for selected (m, kk) columns: {(m, kk): complex (N_r^c,)}."""
    kap = g.kappa()
    keep = g.kmask()
    out = {}
    for m, kk in cols:
        col = np.zeros(g.nrc, dtype=np.complex128)
        if keep[kk]:
            e_z = np.exp(-1j * kap[kk] * g.z)
            e_p = np.exp(-1j * m * g.phi)
            f = np.einsum("lij,l,j->i", s, e_z, e_p) / (g.nphi * g.nz)
            P = pbar(m, g.nrc, g.x_ld).astype(np.float64)
            col = (P * g.w[None, :]) @ f
            col[:m] = 0.0
        out[(m, kk)] = col
    return out


def backward_points(S: np.ndarray, g: Grid, pts):
    """Eq. expansion at grid points pts = [(l, i, j)], summed over m, n and kept k."""
    kap = g.kappa()
    keep = g.kmask()
    nodes = sorted({i for _, i, _ in pts})
    P = [pbar(m, g.nrc, g.x_ld[nodes]).astype(np.float64) for m in range(g.M)]
    where = {i: a for a, i in enumerate(nodes)}
    vals = []
    for l, i, j in pts:
        ez = np.exp(1j * kap * g.z[l]) * keep
        acc = 0.0
        for m in range(g.M):
            if g.nphi % 2 == 0 and m == g.nphi // 2:
                continue
            v = (P[m][:, where[i]] @ S[m]) @ ez
            term = v * np.exp(1j * m * g.phi[j])
            acc += term.real if m == 0 else 2.0 * term.real
        vals.append(acc)
    return np.array(vals)
