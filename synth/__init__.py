"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds no arithmetic of the spectral method: it draws seeded
random numbers, evaluates closed-form initial conditions at caller-supplied
points, and permutes array indices between the oracle's dense spectral layout
and the library's packed triangular layout.  Both the oracle and the HIP path
receive exactly these arrays.

Workload recipes (the paper runs only analytic initial conditions, so no
dataset is replaced):

* ``geometric_spectrum``: coefficients (g1 + i g2)/sqrt(2) * a^n * b^m * c^|k|
  with g ~ N(0, 1), Hermitian in k for m = 0 and real at (m, k) = (0, 0),
  n >= m; the m = 0 real part of k = 0 is drawn real.  For the 2D polar case
  (N_z = 1) a = 0.7, b = 0.8; for 3D toroidal-poloidal pairs a = 0.9,
  b = c = 0.85 unless stated.
* ``vortex_pair_psi``: the stream function of two counter-rotating Lamb-Oseen
  vortices (circulations +-Gamma, core radius a, centres (+-b/2, 0)) whose
  centres are displaced along a plane inclined at 48 degrees by
  delta sin(2 pi z / L_z), mirror-symmetric about x = 0 (Sec. 5.3).
* ``gaussian_bump``: A exp(-|X - X0|^2 / (2 sigma^2)) in the plane (Sec. 5.2 seeds).
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def kvals(nz: int) -> np.ndarray:
    """Signed axial index per FFT slot (numpy fftfreq order)."""
    return np.fft.fftfreq(nz, d=1.0 / nz).round().astype(int)


def geometric_spectrum(M: int, nrc: int, nz: int, nzc: int, seed: int,
                       a: float = 0.9, b: float = 0.85, c: float = 0.85) -> np.ndarray:
    """Dense oracle-layout coefficients S[m, n, kk] of shape (M, nrc, nz), complex128."""
    g = rng(seed)
    kv = kvals(nz)
    keep = np.abs(kv) < nzc
    if nz % 2 == 0 and nz > 1:
        keep &= kv != -(nz // 2)
    re = g.standard_normal((M, nrc, nz))
    im = g.standard_normal((M, nrc, nz))
    n = np.arange(nrc)[None, :, None]
    m = np.arange(M)[:, None, None]
    decay = a ** n * b ** m * c ** np.abs(kv)[None, None, :]
    S = (re + 1j * im) / np.sqrt(2.0) * decay
    S[:, :, ~keep] = 0.0
    for mm in range(M):
        S[mm, :mm, :] = 0.0
    # a real field: m = 0 column Hermitian in k, (0, 0) real
    slot = {int(k): i for i, k in enumerate(kv)}
    for i, k in enumerate(kv):
        if k < 0 and keep[i] and (-k) in slot:
            S[0, :, i] = np.conj(S[0, :, slot[-k]])
    S[0, :, slot[0]] = S[0, :, slot[0]].real
    return S


def tri_offsets(M: int, nrc: int) -> np.ndarray:
    """Row offset of each m block in the packed triangular layout (rows n = m .. nrc-1)."""
    sizes = np.array([max(nrc - m, 0) for m in range(M)], dtype=np.int64)
    return np.concatenate([[0], np.cumsum(sizes)])


def to_packed(S: np.ndarray) -> np.ndarray:
    """Dense (M, nrc, nz) -> packed triangular (tau, nz): row off[m] + (n - m) holds S[m, n]."""
    M, nrc, nz = S.shape
    off = tri_offsets(M, nrc)
    out = np.zeros((off[-1], nz), dtype=S.dtype)
    for m in range(M):
        out[off[m]:off[m + 1]] = S[m, m:]
    return out


def from_packed(P: np.ndarray, M: int, nrc: int) -> np.ndarray:
    """Packed triangular (tau, nz) -> dense (M, nrc, nz) with zero rows n < m."""
    nz = P.shape[1]
    off = tri_offsets(M, nrc)
    out = np.zeros((M, nrc, nz), dtype=P.dtype)
    for m in range(M):
        out[m, m:] = P[off[m]:off[m + 1]]
    return out


def _ein(s: np.ndarray) -> np.ndarray:
    """Ein(s) = int_0^s (1 - e^-t)/t dt (entire), by its series for s < 2, else ln s + gamma_E + E1(s)."""
    from scipy.special import exp1
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    small = s < 2.0
    ss = s[small]
    term = ss.copy()
    acc = ss.copy()
    for k in range(2, 40):
        term = -term * ss * (k - 1) / (k * k)
        acc = acc + term
    out[small] = acc
    big = ~small
    out[big] = np.log(s[big]) + np.euler_gamma + exp1(s[big])
    return out


def vortex_pair_psi(r: np.ndarray, phi: np.ndarray, z: np.ndarray, *, gamma: float = 2 * np.pi,
                    a: float = 0.1, b: float = 1.0, delta: float = 0.01, lz: float = 8.6,
                    incline_deg: float = 48.0, phase: float = 0.0) -> np.ndarray:
    """psi(z, r, phi) on the tensor grid, shape (len(z), len(r), len(phi)).

    Each Lamb-Oseen vortex of circulation G has omega = G/(pi a^2) exp(-rho^2/a^2) and
    stream function -(G / 4 pi) Ein(rho^2 / a^2); the pair has +Gamma at x > 0 and
    -Gamma at x < 0, so psi decays like a dipole.  Both cores are displaced by
    delta sin(2 pi z / L_z + phase) along (+-cos incline, sin incline), mirror-symmetric.
    """
    ang = np.deg2rad(incline_deg)
    Z, R, P = np.meshgrid(z, r, phi, indexing="ij")
    X = R * np.cos(P)
    Y = R * np.sin(P)
    disp = delta * np.sin(2 * np.pi * Z / lz + phase)
    x1 = b / 2 + disp * np.cos(ang)
    y1 = disp * np.sin(ang)
    x2 = -b / 2 - disp * np.cos(ang)
    y2 = disp * np.sin(ang)
    rho1 = ((X - x1) ** 2 + (Y - y1) ** 2) / a ** 2
    rho2 = ((X - x2) ** 2 + (Y - y2) ** 2) / a ** 2
    return -(gamma / (4 * np.pi)) * (_ein(rho1) - _ein(rho2))


def gaussian_bump(r: np.ndarray, phi: np.ndarray, amp: float, sigma: float,
                  x0: float, y0: float) -> np.ndarray:
    """amp * exp(-((x - x0)^2 + (y - y0)^2) / (2 sigma^2)) on the polar grid, shape (len(r), len(phi))."""
    R, P = np.meshgrid(r, phi, indexing="ij")
    X = R * np.cos(P)
    Y = R * np.sin(P)
    return amp * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * sigma ** 2))


def batched_instances(count: int, seed: int):
    """Uneven 2D reaction-diffusion instances: (nr, nphi, ell, amp, sigma, x0, y0) per instance.

    N_r ~ U{48..256}; N_phi ~ U over the even 5-smooth integers in [32, 256];
    ell ~ U[0.5, 2]; A ~ U[0.5, 1.5]; sigma ~ U[0.5, 1.5] ell; |x0| ~ U[0, ell] at a uniform angle.
    """
    smooth = [n for n in range(32, 257, 2) if _is_5smooth(n)]
    g = rng(seed)
    out = []
    for _ in range(count):
        nr = int(g.integers(48, 257))
        nphi = int(smooth[int(g.integers(0, len(smooth)))])
        ell = float(g.uniform(0.5, 2.0))
        amp = float(g.uniform(0.5, 1.5))
        sigma = float(g.uniform(0.5, 1.5) * ell)
        rad = float(g.uniform(0.0, ell))
        ang = float(g.uniform(0.0, 2 * np.pi))
        out.append(dict(nr=nr, nphi=nphi, ell=ell, amp=amp, sigma=sigma,
                        x0=rad * np.cos(ang), y0=rad * np.sin(ang)))
    return out


def _is_5smooth(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def closure_init(seed: int, nin: int = 258, hidden: int = 256, nout: int = 256,
                 last_gain: float = 0.1) -> np.ndarray:
    """Initial closure weights, float32, in the order W1 [h][nin], b1, W2 [h][h], b2, W3 [nout][h], b3.

    Glorot-uniform weights (the last layer scaled by last_gain) and zero biases.
    """
    g = rng(seed)

    def glorot(fo, fi, gain=1.0):
        a = gain * np.sqrt(6.0 / (fi + fo))
        return g.uniform(-a, a, (fo, fi))

    parts = [glorot(hidden, nin), np.zeros(hidden), glorot(hidden, hidden), np.zeros(hidden),
             glorot(nout, hidden, last_gain), np.zeros(nout)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def batch_indices(count: int, nb: int, steps: int, seed: int) -> np.ndarray:
    """steps x nb int32 row indices: consecutive slices of seeded permutations of range(count)."""
    g = rng(seed)
    out = np.empty((steps, nb), dtype=np.int32)
    perm, pos = g.permutation(count), 0
    for s in range(steps):
        if pos + nb > count:
            perm, pos = g.permutation(count), 0
        out[s] = perm[pos:pos + nb]
        pos += nb
    return out
