"""Oracle: the learned coarse-grid closure network (an addition to the paper's method).

Test infrastructure only (see the package header).  There is no paper passage for this part:
the network, its training and its rounding points are defined here and in the library's
header, and the oracle mirrors them in FP64:

* features x (258 per (m, k) column, zero-padded to 288): coarse psi and chi coefficients for
  n < 64 (real, imaginary), then m / M_c and k / K_c, each multiplied by a feature scale;
* z1 = x W1^T + b1, h1 = tanh(z1); z2 = h1 W2^T + b2, h2 = tanh(z2); y = h2 W3^T + b3;
* loss = mean((y - t)^2) over the batch and the 256 outputs;
* bfloat16 rounding (round to nearest even) is applied where the GPU stores bfloat16: the inputs
  x, the weights used by the products, h1 and h2, and the gradients dy, dz2, dz1 that enter
  products; every product and sum is otherwise exact (FP64 here, FP32 accumulation on the GPU);
* Adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction, on FP32-held master
  weights.

Pinned by: the FP64 gradients (no rounding) against central differences of the loss, and the
bfloat16 rounding against exact representable values.  Parity of the trained network's accuracy
is unpinned (no paper value): its gain is judged against the plain solver on held-out runs.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), via float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(x, W1, b1, W2, b2, W3, b3, rounding: bool = True):
    r = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    xr = r(x)
    z1 = xr @ r(W1).T + b1
    h1 = np.tanh(z1)
    h1r = r(h1)
    z2 = h1r @ r(W2).T + b2
    h2 = np.tanh(z2)
    h2r = r(h2)
    y = h2r @ r(W3).T + b3
    return dict(x=xr, h1=h1, h1r=h1r, h2=h2, h2r=h2r, y=y)


def loss_and_grads(x, t, W1, b1, W2, b2, W3, b3, rounding: bool = True):
    """MSE loss and gradients of all parameters (the GPU's backward pass, mirrored)."""
    r = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    f = forward(x, W1, b1, W2, b2, W3, b3, rounding)
    y = f["y"]
    n = y.size
    loss = np.mean((y - t) ** 2)
    dy = r(2.0 * (y - t) / n)
    gW3 = dy.T @ f["h2r"]
    gb3 = dy.sum(0)
    dh2 = dy @ r(W3)
    dz2 = r(dh2 * (1.0 - f["h2"] ** 2))
    gW2 = dz2.T @ f["h1r"]
    gb2 = dz2.sum(0)
    dh1 = dz2 @ r(W2)
    dz1 = r(dh1 * (1.0 - f["h1"] ** 2))
    gW1 = dz1.T @ f["x"]
    gb1 = dz1.sum(0)
    return loss, dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, W3=gW3, b3=gb3)


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (returns new p, m, v); step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------- index definitions
# Spectral arrays here use the oracle layout S[m, n, kk] of shape (M, N_r^c, N_z) (zero for n < m).

NCOEF = 64
NIN = 4 * NCOEF + 2
NOUT = 4 * NCOEF


def _kvals(nz: int) -> np.ndarray:
    return np.fft.fftfreq(nz, d=1.0 / nz).round().astype(int)


def _kept(nz: int, nzc: int) -> np.ndarray:
    k = _kvals(nz)
    keep = np.abs(k) < nzc
    if nz % 2 == 0 and nz > 1:
        keep &= k != -(nz // 2)
    return keep


def truncate(S: np.ndarray, nzc_from: int, M_to: int, nrc_to: int, nz_to: int, nzc_to: int) -> np.ndarray:
    """Move coefficients to another grid (Sec. 3.1, Eq. expansion: Pbar_n^m does not depend on N_r).

    Every (m, n, k) stored by both grids and kept by both axial chops is copied; the rest is 0.
    """
    M_from, nrc_from, nz_from = S.shape
    out = np.zeros((M_to, nrc_to, nz_to), dtype=S.dtype)
    kf, kt = _kvals(nz_from), _kvals(nz_to)
    keep_f, keep_t = _kept(nz_from, nzc_from), _kept(nz_to, nzc_to)
    src_slot = {int(k): i for i, k in enumerate(kf) if keep_f[i]}
    for j, k in enumerate(kt):
        if not keep_t[j] or int(k) not in src_slot:
            continue
        i = src_slot[int(k)]
        for m in range(min(M_from, M_to)):
            for n in range(m, min(nrc_from, nrc_to)):
                out[m, n, j] = S[m, n, i]
    return out


def columns(M: int, nz: int, nzc: int):
    """(m, slot) of every closure column, m-major, kept slots in FFT order."""
    slots = [i for i in range(nz) if _kept(nz, nzc)[i]]
    return [(m, s) for m in range(M) for s in slots], slots


def features(Sp: np.ndarray, Sc: np.ndarray, nzc: int) -> np.ndarray:
    """Raw features (ncols, 258): Re/Im psi, Re/Im chi for n < 64 at offsets 0/64/128/192, m/M, k/k_max."""
    M, nrc, nz = Sp.shape
    cols, slots = columns(M, nz, nzc)
    kv = _kvals(nz)
    kmax = max([abs(int(kv[s])) for s in slots] + [0])
    X = np.zeros((len(cols), NIN), dtype=np.float32)
    for c, (m, s) in enumerate(cols):
        for n in range(m, min(nrc, NCOEF)):
            X[c, n] = Sp[m, n, s].real
            X[c, NCOEF + n] = Sp[m, n, s].imag
            X[c, 2 * NCOEF + n] = Sc[m, n, s].real
            X[c, 3 * NCOEF + n] = Sc[m, n, s].imag
        X[c, 4 * NCOEF] = np.float32(m) / np.float32(M)
        X[c, 4 * NCOEF + 1] = np.float32(kv[s]) / np.float32(kmax) if kmax > 0 else 0.0
    return X


def targets(Rp, Rc, Np, Nc, nzc: int) -> np.ndarray:
    """Raw targets (ncols, 256): (reference - coarse term) at the output positions."""
    M, nrc, nz = Rp.shape
    cols, _ = columns(M, nz, nzc)
    Y = np.zeros((len(cols), NOUT), dtype=np.float32)
    for c, (m, s) in enumerate(cols):
        for n in range(m, min(nrc, NCOEF)):
            dp = Rp[m, n, s] - Np[m, n, s]
            dc = Rc[m, n, s] - Nc[m, n, s]
            Y[c, n], Y[c, NCOEF + n] = dp.real, dp.imag
            Y[c, 2 * NCOEF + n], Y[c, 3 * NCOEF + n] = dc.real, dc.imag
    return Y


def correction(Y: np.ndarray, M: int, nrc: int, nz: int, nzc: int):
    """Spectral correction (Cpsi, Cchi) from per-column outputs; m = 0 made Hermitian in k."""
    cols, _ = columns(M, nz, nzc)
    col_of = {ms: c for c, ms in enumerate(cols)}
    Cp = np.zeros((M, nrc, nz), dtype=np.complex128)
    Cc = np.zeros((M, nrc, nz), dtype=np.complex128)
    for (m, s), c in col_of.items():
        for n in range(m, min(nrc, NCOEF)):
            vp = complex(float(Y[c, n]), float(Y[c, NCOEF + n]))
            vc = complex(float(Y[c, 2 * NCOEF + n]), float(Y[c, 3 * NCOEF + n]))
            if m == 0:
                cn = col_of[(0, (nz - s) % nz)]
                vp = 0.5 * (vp + complex(float(Y[cn, n]), -float(Y[cn, NCOEF + n])))
                vc = 0.5 * (vc + complex(float(Y[cn, 2 * NCOEF + n]), -float(Y[cn, 3 * NCOEF + n])))
            Cp[m, n, s], Cc[m, n, s] = vp, vc
    return Cp, Cc


def judge(Cp, Cc, Rp, Rc, beta: float, ref=None) -> bool:
    """True when the correction is accepted: finite norms and ||C|| <= beta ||RHS|| and, with a
    reference term ref = (Ar_psi, Ar_chi) (the plain term on a finer grid), ||RHS + C - Ar|| <=
    ||RHS - Ar||."""
    cn = np.sqrt(np.sum(np.abs(Cp) ** 2) + np.sum(np.abs(Cc) ** 2))
    rn = np.sqrt(np.sum(np.abs(Rp) ** 2) + np.sum(np.abs(Rc) ** 2))
    ok = bool(np.isfinite(cn) and np.isfinite(rn) and cn <= beta * rn)
    if ref is not None:
        Ap, Ac = ref
        a = np.sqrt(np.sum(np.abs(Rp + Cp - Ap) ** 2) + np.sum(np.abs(Rc + Cc - Ac) ** 2))
        b = np.sqrt(np.sum(np.abs(Rp - Ap) ** 2) + np.sum(np.abs(Rc - Ac) ** 2))
        ok = ok and bool(np.isfinite(a) and np.isfinite(b) and a <= b)
    return ok


def network_params(params: np.ndarray):
    """Split the flat parameter vector (W1 [256][258], b1, W2, b2, W3, b3) into arrays (FP64)."""
    p = np.asarray(params, dtype=np.float64)
    h = 256
    sizes = [(h, NIN), (h,), (h, h), (h,), (NOUT, h), (NOUT,)]
    out, o = [], 0
    for sz in sizes:
        n = int(np.prod(sz))
        out.append(p[o:o + n].reshape(sz))
        o += n
    return out


def flatten_grads(g: dict) -> np.ndarray:
    return np.concatenate([g[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
