"""Pins of the oracle's toroidal-poloidal synthesis and projection (Sec. 3.2, Sec. 5.3).

* The nodal velocity and vorticity are checked against the curl of Eq. tp
  taken symbolically in Cartesian coordinates (sympy), for single modes whose
  basis functions are written out as rational functions of (X, Y).
* The projection is checked on its defining properties: it inverts the
  synthesis on potentials that satisfy the decay gauge, it annihilates
  gradients, and it is linear.
"""
import numpy as np
import pytest

from oracle.grid import Grid
from oracle.rhs import (VecTables, cross_with_background, projection_sources, rhs_tp,
                        solve_projection, synthesize)
from oracle.transform import Tables, forward
import synth

sp = pytest.importorskip("sympy")


def _mode_expr(n, m, kap, c, ell, X, Y, Z):
    """2 Re[c Pbar_n^m(x(r)) e^{i m phi + i kappa z}] as a sympy expression in Cartesian X, Y, Z.

    Pbar_n^m = N_n^m (1-x^2)^{m/2} d^m P_n/dx^m with (1-x^2)^{1/2} = 2 ell r/(r^2+ell^2) and
    r^m e^{i m phi} = (X + iY)^m, so the mode is rational in X, Y.
    """
    t = sp.Symbol("t")
    r2 = X ** 2 + Y ** 2
    x = (r2 - ell ** 2) / (r2 + ell ** 2)
    dmP = sp.diff(sp.legendre(n, t), t, m).subs(t, x)
    norm = sp.sqrt(sp.Rational(2 * n + 1, 2) * sp.factorial(n - m) / sp.factorial(n + m))
    radial = norm * (2 * ell / (r2 + ell ** 2)) ** m * dmP
    cr, ci = sp.nsimplify(c.real), sp.nsimplify(c.imag)
    ang_re, ang_im = sp.expand((X + sp.I * Y) ** m, complex=True).as_real_imag()
    ez_re, ez_im = sp.cos(kap * Z), sp.sin(kap * Z)
    # e^{i m phi} r^m e^{i kappa z} = (ang_re + i ang_im)(ez_re + i ez_im)
    e_re = ang_re * ez_re - ang_im * ez_im
    e_im = ang_re * ez_im + ang_im * ez_re
    val_re = cr * e_re - ci * e_im
    fac = 1 if (m == 0 and kap == 0) else 2
    return fac * radial * val_re


def test_synthesis_matches_symbolic_cartesian_curl():
    ell, lz = sp.Rational(13, 10), sp.Rational(5, 2)
    g = Grid(10, 8, 4, 1.3, lz=2.5)
    vt = VecTables(g)
    X, Y, Z = sp.symbols("X Y Z", real=True)
    kap1 = 2 * sp.pi / lz
    psi = np.zeros((g.M, g.nrc, g.nz), complex)
    chi = np.zeros_like(psi)
    slot = {int(k): i for i, k in enumerate(g.kvals())}
    # psi: (n, m, k) = (3, 2, 1) and (1, 0, 0);  chi: (2, 1, -1) and (2, 0, +-1) (Hermitian m = 0)
    modes_psi = [(3, 2, 1, 0.6 - 0.3j), (1, 0, 0, 0.3 + 0j)]
    modes_chi = [(2, 1, -1, 0.4 + 0.5j), (2, 0, 1, 0.2 - 0.7j)]
    psi_e = 0
    chi_e = 0
    for n, m, k, c in modes_psi:
        psi[m, n, slot[k]] = c
        psi_e += _mode_expr(n, m, k * kap1, c, ell, X, Y, Z)
    for n, m, k, c in modes_chi:
        chi[m, n, slot[k]] = c
        if m == 0 and k != 0:
            chi[m, n, slot[-k]] = np.conj(c)
        chi_e += _mode_expr(n, m, k * kap1, c, ell, X, Y, Z)
    d = sp.diff
    ux = d(psi_e, Y) + d(chi_e, X, Z)
    uy = -d(psi_e, X) + d(chi_e, Y, Z)
    uz = -(d(chi_e, X, 2) + d(chi_e, Y, 2))
    wx = d(uz, Y) - d(uy, Z)
    wy = d(ux, Z) - d(uz, X)
    wz = d(uy, X) - d(ux, Y)
    f = sp.lambdify((X, Y, Z), [ux, uy, uz, wx, wy, wz], "numpy")
    Zg, Rg, Pg = np.meshgrid(g.z, g.r, g.phi, indexing="ij")
    vals = [np.broadcast_to(np.asarray(v, float), Zg.shape) for v in f(Rg * np.cos(Pg), Rg * np.sin(Pg), Zg)]
    c, s = np.cos(Pg), np.sin(Pg)
    ref_u = [vals[0] * c + vals[1] * s, -vals[0] * s + vals[1] * c, vals[2]]
    ref_w = [vals[3] * c + vals[4] * s, -vals[3] * s + vals[4] * c, vals[5]]
    u, w = synthesize(psi, chi, g, vt)
    scale = max(np.abs(a).max() for a in ref_u + ref_w)
    for a, b in zip(u + w, ref_u + ref_w):
        assert np.abs(a - b).max() < 1e-12 * scale


def _gauged(S, g):
    """Band-limit to n < N_r - 3 and adjust n = 0 of every m = 0 column so that
    sum_n sqrt((2n+1)/2) S_n = 0 (psi -> 0 at infinity).

    With three empty top degrees every Galerkin integrand of P(V(psi, chi)) is a polynomial of degree
    below 2 N_r, so Gauss-Legendre quadrature makes the discrete projection an exact inverse.
    """
    S = S.copy()
    S[:, g.nrc - 3:, :] = 0.0
    n = np.arange(g.nrc)
    v = np.sqrt((2 * n + 1) / 2.0)
    S[0, 0, :] = -(v[1:, None] * S[0, 1:, :]).sum(0) / v[0]
    return S


def test_projection_inverts_synthesis():
    g = Grid(24, 12, 8, 0.9, lz=3.0)
    vt = VecTables(g)
    psi = _gauged(synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=21, a=0.8, b=0.8, c=0.8), g)
    chi = _gauged(synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=22, a=0.8, b=0.8, c=0.8), g)
    u, _ = synthesize(psi, chi, g, vt)
    C, K, Z = projection_sources(u[0], u[1], u[2], g, vt)
    p2, c2 = solve_projection(C, K, Z, g, dealias=False)
    # chi passes through two solves with Dbar (cond ~1e5 at N_r = 24), so rounding is amplified
    # more than for psi; a wrong term or sign would give an O(1) difference.
    assert np.abs(p2 - psi).max() < 1e-11 * np.abs(psi).max()
    assert np.abs(c2 - chi).max() < 1e-9 * np.abs(chi).max()


def _gradient_projection(nr, nphi):
    g = Grid(nr, nphi, 8, 1.0, lz=2 * np.pi)
    vt = VecTables(g)
    Zg, Rg, Pg = np.meshgrid(g.z, g.r, g.phi, indexing="ij")
    X, Y = Rg * np.cos(Pg), Rg * np.sin(Pg)
    s2 = 0.5
    gauss = np.exp(-((X - 0.3) ** 2 + (Y + 0.1) ** 2) / (2 * s2))
    zf = 1 + 0.3 * np.cos(Zg) + 0.2 * np.sin(2 * Zg)
    dzf = -0.3 * np.sin(Zg) + 0.4 * np.cos(2 * Zg)
    px = -(X - 0.3) / s2 * gauss * zf
    py = -(Y + 0.1) / s2 * gauss * zf
    pz = gauss * dzf
    c, s = np.cos(Pg), np.sin(Pg)
    C, K, Z = projection_sources(px * c + py * s, -px * s + py * c, pz, g, vt)
    p2, c2 = solve_projection(C, K, Z, g, dealias=False)
    scale = np.abs(forward(gauss * zf, g, Tables(g))).max()
    return np.abs(p2).max() / scale, np.abs(c2).max() / scale


def test_projection_annihilates_gradients():
    # P(grad p) = 0 up to the representation error of p, which falls spectrally with resolution.
    coarse = _gradient_projection(32, 12)
    fine = _gradient_projection(64, 24)
    assert fine[0] < 1e-10 and fine[1] < 1e-8
    assert fine[0] < 1e-3 * coarse[0] and fine[1] < 1e-2 * coarse[1]


def test_rhs_tp_is_quadratic_and_background_linear():
    # N = (U + u) x w is quadratic in (psi, chi) for U = 0 and affine in U.
    g = Grid(16, 8, 4, 1.0, lz=2 * np.pi)
    vt = VecTables(g)
    psi = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=31, a=0.6, b=0.7, c=0.7)
    chi = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=32, a=0.6, b=0.7, c=0.7)
    a1, b1 = rhs_tp(psi, chi, g, vt)
    a2, b2 = rhs_tp(2 * psi, 2 * chi, g, vt)
    assert np.abs(a2 - 4 * a1).max() < 1e-12 * np.abs(a2).max()
    assert np.abs(b2 - 4 * b1).max() < 1e-12 * np.abs(b2).max()
    U = (0.3, -0.2, 0.5)
    aU, bU = rhs_tp(psi, chi, g, vt, U=U)
    aU2, bU2 = rhs_tp(psi, chi, g, vt, U=tuple(2 * x for x in U))
    assert np.abs((aU2 - aU) - (aU - a1)).max() < 1e-12 * np.abs(aU).max()
    assert np.abs((bU2 - bU) - (bU - b1)).max() < 1e-12 * np.abs(bU).max()


def test_cross_product_orientation():
    # e_r x e_phi = e_z, e_phi x e_z = e_r, e_z x e_r = e_phi
    g = Grid(4, 4, 1, 1.0)
    one = np.ones((1, 4, 4))
    zero = np.zeros((1, 4, 4))
    N = cross_with_background([one, zero, zero], [zero, one, zero], (0, 0, 0), g)
    assert np.all(N[2] == 1) and np.all(N[0] == 0) and np.all(N[1] == 0)
    N = cross_with_background([zero, one, zero], [zero, zero, one], (0, 0, 0), g)
    assert np.all(N[0] == 1)
    N = cross_with_background([zero, zero, one], [one, zero, zero], (0, 0, 0), g)
    assert np.all(N[1] == 1)
    # a uniform Cartesian U_x seen in cylindrical components at phi = 0 and phi = pi/2
    N = cross_with_background([zero, zero, zero], [zero, zero, one], (1.0, 0, 0), g)
    # U x e_z with U = e_x gives -e_y: radial part -sin(phi), azimuthal part -cos(phi)
    assert np.allclose(N[0][0, 0], -np.sin(g.phi)) and np.allclose(N[1][0, 0], -np.cos(g.phi))


def test_sampled_evaluations_agree_with_the_full_oracle():
    """The column / point forms used for checks at full size equal the full transforms."""
    from oracle.rhs import projection_sources_columns, synthesize_points
    from oracle.transform import Tables, backward, backward_points, forward, forward_columns
    g = Grid(18, 12, 10, 0.9, lz=3.0)
    t = Tables(g)
    vt = VecTables(g)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((g.nz, g.nr, g.nphi))
    S = forward(f, g, t)
    cols = [(0, 0), (0, 3), (1, 9), (4, 2), (5, 5), (3, 7)]
    fc = forward_columns(f, g, cols)
    for (m, kk), v in fc.items():
        np.testing.assert_allclose(v, S[m, :, kk], rtol=0, atol=1e-13 * np.abs(S).max())
    pts = [(0, 0, 0), (3, 17, 5), (9, 8, 11), (5, 2, 6)]
    bp = backward_points(S, g, pts)
    full = backward(S, g, t)
    np.testing.assert_allclose(bp, [full[l, i, j] for l, i, j in pts], rtol=0, atol=1e-13 * np.abs(full).max())
    psi = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=7, a=0.8)
    chi = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=8, a=0.8)
    u, w = synthesize(psi, chi, g, vt)
    sp = synthesize_points(psi, chi, g, vt, pts)
    ref = np.array([[x[l, i, j] for l, i, j in pts] for x in list(u) + list(w)])
    np.testing.assert_allclose(sp, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    N = cross_with_background(u, w, (0.1, 0.4, -0.2), g)
    C, K, Z = projection_sources(*N, g, vt)
    pc = projection_sources_columns(*N, g, vt, cols)
    for (m, kk), (c, k, z) in pc.items():
        for got, want in ((c, C), (k, K), (z, Z)):
            np.testing.assert_allclose(got, want[m, :, kk], rtol=0, atol=1e-12 * np.abs(want).max())


def test_rhs_tp_two_thirds_rule_is_alias_free():
    # as the scalar pin: the masked (psi_N, chi_N) on (N_phi, N_z) equal those of the masked
    # potentials on (2 N_phi, 2 N_z) on every kept (m, k), though the input populates the margin
    from oracle.rhs import apply_mask
    gc = Grid(10, 12, 6, 1.1, lz=4.0)
    gf = Grid(10, 24, 12, 1.1, lz=4.0)
    psi = synth.geometric_spectrum(gc.M, gc.nrc, gc.nz, gc.nzc, seed=43, a=0.7, b=0.9, c=0.9)
    chi = synth.geometric_spectrum(gc.M, gc.nrc, gc.nz, gc.nzc, seed=44, a=0.7, b=0.9, c=0.9)
    U = (0.2, -0.1, 0.3)
    ac, bc = rhs_tp(psi, chi, gc, VecTables(gc), U=U)

    def embed(S):
        Sf = np.zeros((gf.M, gc.nrc, gf.nz), complex)
        for kk, k in enumerate(gc.kvals()):
            Sf[:gc.M, :, k % gf.nz] = S[:, :, kk]
        return Sf

    af, bf = rhs_tp(embed(apply_mask(psi, gc)), embed(apply_mask(chi, gc)), gf, VecTables(gf), U=U)
    kept = (np.arange(gc.M)[:, None] <= gc.dealias_m()) & \
        ((np.abs(gc.kvals()) <= gc.dealias_k()) & gc.kmask())[None, :]
    big = max(np.abs(ac).max(), np.abs(bc).max())
    for m in range(gc.M):
        for kk, k in enumerate(gc.kvals()):
            if kept[m, kk]:
                assert np.abs(ac[m, :, kk] - af[m, :, k % gf.nz]).max() < 1e-12 * big, (m, k)
                assert np.abs(bc[m, :, kk] - bf[m, :, k % gf.nz]).max() < 1e-12 * big, (m, k)
            else:
                assert np.abs(ac[m, :, kk]).max() == 0.0 and np.abs(bc[m, :, kk]).max() == 0.0
    # margin-only potentials produce nothing (the background alone carries no gradient-free part)
    a0, b0 = rhs_tp(psi - apply_mask(psi, gc), chi - apply_mask(chi, gc), gc, VecTables(gc), U=U)
    assert np.abs(a0).max() == 0.0 and np.abs(b0).max() == 0.0
