"""Oracle: pseudospectral nonlinear terms and the toroidal-poloidal projection.

Test infrastructure only (see the package header).

Scalar (Sec. 3.3; Sec. 5.2, Eq. kpp):
    R(shat) = Mask( F( g( B( Mask(shat) ) ) ) ),  g(u) = u^2  or  g(u) = gamma u (1 - u),
with the conventional two-thirds mask in phi and z (keep m <= floor((N_phi-1)/3),
|k| <= floor((N_z-1)/3)); no radial margin (N_r^c = N_r in the paper's runs).  The mask is
the dealiasing margin between the periodic chops and the collocation counts (Sec. 3.3): the
fields that enter the product hold no mode in the margin, and the product keeps none there, so
it applies on the way in as well as on the way out.

Vector (Sec. 3.2 Eq. tp, Sec. 5.3 Eq. tp-evolution):
    (psi_N, chi_N) = Mask( P[ (U + u) x omega ] ),  u = curl(psi z) + curl curl(chi z),
    omega = curl u of the masked potentials (Mask(psi), Mask(chi)), U a uniform Cartesian
    background (the moving frame of Sec. 5.3).
The velocity and vorticity harmonics at the nodes are the plain curl formulas
in cylindrical coordinates; r d/dr of a harmonic is Tbar = (1-x^2) dPbar/dx, and
the horizontal Laplacian of Pbar_n^m(x(r)) is -n(n+1) (1-x)^2/ell^2 Pbar_n^m, which
follows from the mapped Legendre equation (Eq. mapped-legendre).

The projection P (Eq. tp-poisson) is taken in its gradient-removing curl form
(Sec. 3.2: the potentials follow from the axial curl and curl-curl, which
annihilate gradients):
    -grad_h^2 psi_N = z . curl N,     grad^2 grad_h^2 chi_N = z . curl curl N,
with z . curl N = (1/r) d_r(r N_phi) - (1/r) d_phi N_r and
z . curl curl N = d_z (1/r) d_r(r N_r) + (1/r) d_phi d_z N_phi - grad_h^2 N_z.
The cylindrical components of N enter coefficient space by Gauss-Legendre
projection of N/r and of N_z, and the divergence-form radial term by its
integration-by-parts (weak) form
    [(1/r) d_r(r f)]^_n = - sum_i w_i [Tbar_n(x_i) - 2 (1 + x_i) Pbar_n(x_i)] f_i / r_i,
whose boundary terms vanish for bounded f decaying at infinity.  The elliptic
problems are solved with the truncated Dbar_m of Eq. del2h-entries by dense LU
with partial pivoting; the singular m = 0 blocks take the decay gauge
sum_n Pbar_n^0(1) shat_n = 0 (psi, chi -> 0 as r -> infinity, Sec. 3.2) in
place of their first row.  At k = 0 the curl-curl equation reduces to
grad_h^2 chi_N = -N_z (the first Poisson equation of Eq. tp-poisson).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .basis import laplacian_matrix, pbar, tbar
from .grid import Grid
from .transform import (Tables, axial_backward, axial_forward, azimuthal_backward,
                        azimuthal_forward, backward, forward)


# ----------------------------------------------------------------- masks

def dealias_mask(g: Grid) -> np.ndarray:
    """Boolean (M, N_z) mask of the (m, k slot) pairs the two-thirds rule keeps."""
    mkeep = np.arange(g.M) <= g.dealias_m()
    kkeep = (np.abs(g.kvals()) <= g.dealias_k()) & g.kmask()
    return mkeep[:, None] & kkeep[None, :]


def apply_mask(S: np.ndarray, g: Grid) -> np.ndarray:
    return S * dealias_mask(g)[:, None, :]


# ----------------------------------------------------------------- scalar

def rhs_scalar(S: np.ndarray, g: Grid, t: Tables, kind: str, gamma: float = 0.25,
               dealias: bool = True) -> np.ndarray:
    """R = Mask(F(g(B(Mask(S))))) with g = u^2 ('u2') or gamma u (1 - u) ('kpp'); without
    dealiasing, R = F(g(B(S)))."""
    u = backward(apply_mask(S, g) if dealias else S, g, t)
    if kind == "u2":
        v = u * u
    elif kind == "kpp":
        v = gamma * u * (1.0 - u)
    else:
        raise ValueError(kind)
    out = forward(v, g, t)
    return apply_mask(out, g) if dealias else out


# ----------------------------------------------------------------- vector tables

class VecTables:
    """Pbar, Tbar and Qbar = Tbar - 2(1+x)Pbar at the nodes, double, per m: (N_r^c, N_r)."""

    def __init__(self, g: Grid):
        self.g = g
        self.P, self.T, self.Q = [], [], []
        for m in range(g.M):
            p = pbar(m, g.nrc, g.x_ld)
            tt = tbar(m, g.nrc, g.x_ld)
            self.P.append(p.astype(np.float64))
            self.T.append(tt.astype(np.float64))
            self.Q.append((tt - 2 * (1 + g.x_ld)[None, :] * p).astype(np.float64))
        self.L = np.arange(g.nrc, dtype=np.float64) * (np.arange(g.nrc) + 1.0)


def velocity_vorticity_harmonics(psi: np.ndarray, chi: np.ndarray, g: Grid, vt: VecTables, nodes=None):
    """Harmonics (M, N_r, N_z) in spectral k of u_r, u_phi, u_z, w_r, w_phi, w_z at the nodes
    (at the radial nodes listed in ``nodes`` only, if given).

    u = (1/r d_phi psi + d_r d_z chi,  -d_r psi + (1/r) d_phi d_z chi,  -grad_h^2 chi)
    w = (d_r d_z psi - (1/r) d_phi grad^2 chi,  (1/r) d_phi d_z psi + d_r grad^2 chi,  -grad_h^2 psi)
    per harmonic (d_phi -> i m, d_z -> i kappa, grad^2 = grad_h^2 - kappa^2).
    """
    sel = np.arange(g.nr) if nodes is None else np.asarray(nodes)
    M, nr, nz = g.M, len(sel), g.nz
    kap = g.kappa()
    keep = g.kmask()
    r = g.r[sel]
    q = g.q[sel]
    x = g.x[sel]
    outs = [np.zeros((M, nr, nz), dtype=np.complex128) for _ in range(6)]
    for m in range(M):
        P, T = vt.P[m][:, sel], vt.T[m][:, sel]
        ps = psi[m] * keep[None, :]
        ch = chi[m] * keep[None, :]
        A1 = P.T @ ps                         # psi
        A2 = T.T @ ps                         # r d_r psi
        lap_psi = -q[:, None] * (P.T @ (vt.L[:, None] * ps))       # grad_h^2 psi
        B1 = P.T @ ch                         # chi
        B2 = T.T @ ch                         # r d_r chi
        lap_chi = -q[:, None] * (P.T @ (vt.L[:, None] * ch))       # grad_h^2 chi
        rdr_lap_chi_h = -(T.T @ (vt.L[:, None] * ch))              # r d_r (Lchi) part, times q below
        im = 1j * m
        ik = 1j * kap[None, :]
        rr = r[:, None]
        # grad^2 chi = grad_h^2 chi - kappa^2 chi ; r d_r of it:
        # r d_r(-q Pbar(L chi)) = -q Tbar(L chi) - (r d_r q) Pbar(L chi), r d_r q = -2(1+x) q
        rdr_lap_chi = q[:, None] * rdr_lap_chi_h + 2 * (1 + x)[:, None] * q[:, None] * (P.T @ (vt.L[:, None] * ch))
        lap3_chi = lap_chi - (kap ** 2)[None, :] * B1
        rdr_lap3_chi = rdr_lap_chi - (kap ** 2)[None, :] * B2
        outs[0][m] = (im * A1 + ik * B2) / rr                          # u_r
        outs[1][m] = (-A2 + im * ik * B1) / rr                         # u_phi
        outs[2][m] = -lap_chi                                           # u_z
        outs[3][m] = (ik * A2 - im * lap3_chi) / rr                     # w_r
        outs[4][m] = (im * ik * A1 + rdr_lap3_chi) / rr                 # w_phi
        outs[5][m] = -lap_psi                                           # w_z
    return outs


def synthesize(psi: np.ndarray, chi: np.ndarray, g: Grid, vt: VecTables):
    """Nodal u and omega (each a list of 3 real (N_z, N_r, N_phi) arrays)."""
    h = velocity_vorticity_harmonics(psi, chi, g, vt)
    nodal = []
    for f in h:
        a = axial_backward(f, g, axis=2)                   # (M, N_r, N_z) physical z
        nodal.append(azimuthal_backward(np.transpose(a, (2, 1, 0)), g))
    return nodal[:3], nodal[3:]


def synthesize_points(psi: np.ndarray, chi: np.ndarray, g: Grid, vt: VecTables, pts):
    """Nodal u and omega at grid points pts = [(l, i, j)]: the harmonics at those radial nodes,
    summed over m and kept k (Eq. expansion); returns an array (6, len(pts))."""
    nodes = sorted({i for _, i, _ in pts})
    where = {i: a for a, i in enumerate(nodes)}
    h = velocity_vorticity_harmonics(psi, chi, g, vt, nodes=nodes)
    kap = g.kappa()
    keep = g.kmask()
    out = np.zeros((6, len(pts)))
    for c, (l, i, j) in enumerate(pts):
        ez = np.exp(1j * kap * g.z[l]) * keep
        for f in range(6):
            acc = 0.0
            for m in range(g.M):
                if g.nphi % 2 == 0 and m == g.nphi // 2:
                    continue
                term = (h[f][m, where[i]] @ ez) * np.exp(1j * m * g.phi[j])
                acc += term.real if m == 0 else 2.0 * term.real
            out[f, c] = acc
    return out


def cross_with_background(u, w, U, g: Grid):
    """N = (U + u) x w in cylindrical components; U = (U_x, U_y, U_z) Cartesian."""
    cphi = np.cos(g.phi)[None, None, :]
    sphi = np.sin(g.phi)[None, None, :]
    ur = u[0] + U[0] * cphi + U[1] * sphi
    up = u[1] - U[0] * sphi + U[1] * cphi
    uz = u[2] + U[2]
    nr_ = up * w[2] - uz * w[1]
    np_ = uz * w[0] - ur * w[2]
    nz_ = ur * w[1] - up * w[0]
    return nr_, np_, nz_


def _mixed_forward(f: np.ndarray, g: Grid) -> np.ndarray:
    """Physical (N_z, N_r, N_phi) -> harmonics (M, N_r, N_z) in spectral k (phi then z)."""
    a = azimuthal_forward(f, g)                             # (N_z, N_r, M)
    return axial_forward(np.transpose(a, (2, 1, 0)), g, axis=2)


def projection_sources(Nr_, Np_, Nz_, g: Grid, vt: VecTables):
    """Galerkin sources C = [z.curl N]^, K = [z.curl curl N]^ and Zhat = [N_z]^, shape (M, N_r^c, N_z)."""
    a = _mixed_forward(Nr_ / g.r[None, :, None], g)
    b = _mixed_forward(Np_ / g.r[None, :, None], g)
    c = _mixed_forward(Nz_, g)
    kap = g.kappa()
    C = np.zeros((g.M, g.nrc, g.nz), dtype=np.complex128)
    K = np.zeros_like(C)
    Z = np.zeros_like(C)
    for m in range(min(g.M, g.nrc)):   # orders m >= N_r^c have no coefficients
        C[m], K[m], Z[m] = _sources(a[m], b[m], c[m], m, kap[None, :], g, vt)
    keep = g.kmask()[None, None, :]
    return C * keep, K * keep, Z * keep


def _sources(a_m, b_m, c_m, m, kap, g: Grid, vt: VecTables):
    """C, K, Zhat of order m from the harmonics of N_r/r, N_phi/r, N_z at the nodes."""
    WP = vt.P[m] * g.w[None, :]
    WQ = vt.Q[m] * g.w[None, :]
    Pa, Qa = WP @ a_m, WQ @ a_m
    Pb, Qb = WP @ b_m, WQ @ b_m
    Zm = WP @ c_m
    # z.curl N = (1/r) d_r(r N_phi) - i m N_r / r ; weak form of the first term is -Q^T W (N_phi/r)
    C = -Qb - 1j * m * Pa
    # z.curl curl N = i kappa (1/r) d_r(r N_r) - m kappa N_phi / r - grad_h^2 N_z
    D = np.zeros((g.nrc, g.nrc))
    D[m:, m:] = laplacian_matrix(m, g.nrc, g.ell)
    K = 1j * kap * (-Qa) - m * kap * Pb - D @ Zm
    return C, K, Zm


def projection_sources_columns(Nr_, Np_, Nz_, g: Grid, vt: VecTables, cols):
    """C, K, Zhat for selected (m, kk) columns: the harmonics by the plain sums over phi and z,
    then the Galerkin projections of ``projection_sources``; {(m, kk): (C, K, Z)}."""
    kap = g.kappa()
    keep = g.kmask()
    out = {}
    for m, kk in cols:
        e_z = np.exp(-1j * kap[kk] * g.z)
        e_p = np.exp(-1j * m * g.phi)

        def harm(f):
            return np.einsum("lij,l,j->i", f, e_z, e_p) / (g.nphi * g.nz)

        a = harm(Nr_ / g.r[None, :, None])
        b = harm(Np_ / g.r[None, :, None])
        c = harm(Nz_)
        if keep[kk] and m < g.nrc:
            out[(m, kk)] = _sources(a, b, c, m, kap[kk], g, vt)
        else:
            z = np.zeros(g.nrc, dtype=np.complex128)
            out[(m, kk)] = (z, z.copy(), z.copy())
    return out


def _gauge_row(nrc: int) -> np.ndarray:
    """Pbar_n^0(1) = sqrt((2n+1)/2): the value at r = infinity of each m = 0 basis function."""
    n = np.arange(nrc)
    return np.sqrt((2 * n + 1) / 2.0)


def solve_projection(C, K, Z, g: Grid, dealias: bool = True):
    """Dbar psi = -C ; (Dbar - kappa^2) q = K (q = -Zhat at k = 0) ; Dbar chi = q (gauge at m = 0)."""
    kap = g.kappa()
    keep = g.kmask()
    mask = dealias_mask(g) if dealias else np.ones((g.M, g.nz), bool) & keep[None, :]
    psi = np.zeros_like(C)
    chi = np.zeros_like(C)
    for m in range(min(g.M, g.nrc)):
        cols = np.nonzero(mask[m] & keep)[0]
        if cols.size == 0:
            continue
        D = laplacian_matrix(m, g.nrc, g.ell)
        Dg = D.copy()
        if m == 0:
            Dg[0, :] = _gauge_row(g.nrc)
        lu = sla.lu_factor(Dg)
        rhs_psi = -C[m, m:, :][:, cols]
        rhs_q = -Z[m, m:, :][:, cols]
        nz_cols = np.nonzero(kap[cols] != 0.0)[0]
        if nz_cols.size:
            eye = np.eye(g.nrc - m)
            mats = D[None, :, :] - (kap[cols[nz_cols]] ** 2)[:, None, None] * eye[None, :, :]
            sol = np.linalg.solve(mats, K[m, m:, :][:, cols[nz_cols]].T[:, :, None])[:, :, 0]
            rhs_q[:, nz_cols] = sol.T
        if m == 0:
            rhs_psi[0, :] = 0.0
            rhs_q[0, :] = 0.0
        psi[m, m:, cols] = sla.lu_solve(lu, rhs_psi).T
        chi[m, m:, cols] = sla.lu_solve(lu, rhs_q).T
    return psi, chi


def rhs_tp(psi: np.ndarray, chi: np.ndarray, g: Grid, vt: VecTables, U=(0.0, 0.0, 0.0),
           dealias: bool = True, taps: dict | None = None):
    """(psi_N, chi_N) = Mask(P[(U+u) x omega]) for the toroidal-poloidal pair (psi, chi), u and
    omega those of (Mask(psi), Mask(chi)) when dealiasing.

    ``taps``, if given, receives the intermediate quantities the parity tests
    compare: nodal u, omega, N and the sources C, K, Zhat.
    """
    if dealias:
        psi, chi = apply_mask(psi, g), apply_mask(chi, g)
    u, w = synthesize(psi, chi, g, vt)
    Nr_, Np_, Nz_ = cross_with_background(u, w, U, g)
    C, K, Z = projection_sources(Nr_, Np_, Nz_, g, vt)
    if dealias:
        mk = dealias_mask(g)[:, None, :]
        C, K, Z = C * mk, K * mk, Z * mk
    if taps is not None:
        taps.update(u=u, w=w, N=(Nr_, Np_, Nz_), C=C, K=K, Z=Z)
    return solve_projection(C, K, Z, g, dealias)


def velocity_from_potentials(psi, chi, g: Grid, vt: VecTables):
    """Nodal velocity only (used by the projection pins)."""
    u, _ = synthesize(psi, chi, g, vt)
    return u
