"""Pins of the FP64 oracle against the paper's printed numbers and closed forms.

Each test ties an oracle function to something other than itself: a value the
paper prints (fixtures under tests/golden/), a closed form, a mathematical
invariant, or a brute-force sum on a tiny grid.
"""
import os

import numpy as np
import pytest

from oracle import timestep as ts
from oracle.basis import laplacian_matrix, pbar, tbar
from oracle.grid import Grid, gauss_legendre
from oracle.rhs import rhs_scalar
from oracle.transform import (Tables, backward, backward_bruteforce, forward,
                              forward_bruteforce)
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _area_rel(g, a, b):
    aw = g.area_w[None, :, None]
    return np.sqrt(np.sum(aw * (a - b) ** 2) / np.sum(aw * b ** 2))


# ------------------------------------------------------------------ grid

@pytest.mark.parametrize("n", [2, 7, 24, 64, 96])
def test_gauss_legendre_exactness(n):
    x, w = gauss_legendre(n)
    x = x.astype(float)
    w = w.astype(float)
    assert np.all(np.diff(x) > 0)
    for j in range(2 * n):
        exact = 2.0 / (j + 1) if j % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** j) - exact) < 2e-15 * max(1, n / 8)


def test_half_nodes_inside_ell_and_outer_radius():
    # Sec. 1 / Fig. grid: half of the radial nodes lie inside r = ell; for N_r = 24 the
    # outermost node sits between 20 and 81 radii (20.36 ell at the smallest map scale).
    for ell in (0.5, 1.0, 4.0):
        g = Grid(24, 16, 1, ell)
        assert np.sum(g.r < ell) == 12
        assert abs(g.r.max() / ell - 20.3608) < 1e-4
    # the node on the other side of the mid-point mirrors: r_i r_{N-1-i} = ell^2
    g = Grid(24, 16, 1, 2.0)
    assert np.allclose(g.r * g.r[::-1], 4.0, rtol=1e-14)


# ------------------------------------------------------------------ basis

def test_low_order_closed_forms():
    x = np.linspace(-0.95, 0.95, 9)
    s = np.sqrt(1 - x * x)
    assert np.allclose(pbar(0, 3, x)[0].astype(float), np.sqrt(0.5), rtol=1e-15)
    assert np.allclose(pbar(0, 3, x)[1].astype(float), np.sqrt(1.5) * x, rtol=1e-15, atol=1e-16)
    assert np.allclose(pbar(1, 3, x)[1].astype(float), np.sqrt(3) / 2 * s, rtol=1e-15)
    assert np.allclose(pbar(2, 3, x)[2].astype(float), np.sqrt(15) / 4 * s * s, rtol=1e-15)
    # Pbar_2^0 = sqrt(5/2) (3x^2 - 1)/2
    assert np.allclose(pbar(0, 3, x)[2].astype(float), np.sqrt(2.5) * (3 * x * x - 1) / 2, atol=1e-15)


@pytest.mark.parametrize("m", [0, 1, 5, 40, 127, 255])
def test_discrete_orthonormality(m):
    # Gauss-Legendre quadrature integrates Pbar_n^m Pbar_n'^m (a polynomial of degree n + n') exactly,
    # and Eq. norm makes the family orthonormal on [-1, 1].
    n = 256
    x, w = gauss_legendre(n)
    P = pbar(m, n, x).astype(float)
    G = (P * w.astype(float)) @ P.T
    E = np.eye(n)
    E[:m, :m] = 0
    assert np.abs(G - E).max() < 5e-14


def test_pbar_against_multiprecision():
    # Reference from the definition: Pbar_n^m = N_n^m (1-x^2)^{m/2} d^m/dx^m P_n(x) with Rodrigues'
    # explicit sum P_n(x) = 2^-n sum_k (-1)^k C(n,k) C(2n-2k,n) x^{n-2k}, in 400-digit arithmetic.
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 400
    xs = [-0.73, 0.1, 0.999]
    for (n, m) in [(5, 2), (60, 17), (200, 100), (255, 127)]:
        P = pbar(m, n + 1, np.array(xs))[n]
        for xi, val in zip(xs, P):
            x = mp.mpf(xi)
            acc = mp.mpf(0)
            for k in range(n // 2 + 1):
                e = n - 2 * k
                if e < m:
                    continue
                acc += ((-1) ** k * mp.binomial(n, k) * mp.binomial(2 * n - 2 * k, n)
                        * mp.factorial(e) / mp.factorial(e - m) * x ** (e - m))
            ref = acc / mp.mpf(2) ** n * (1 - x * x) ** (mp.mpf(m) / 2)
            ref *= mp.sqrt((2 * n + 1) * mp.factorial(n - m) / (2 * mp.factorial(n + m)))
            assert abs(float(val) - float(ref)) <= 2e-15 * max(1.0, abs(float(ref))) + 1e-300, (n, m, xi)


@pytest.mark.parametrize("m", [0, 1, 3, 10])
def test_tbar_is_r_d_dr(m):
    # T = (1-x^2) dPbar/dx: check against a 4th-order finite difference and against the
    # three-term derivative identity (1-x^2) Pbar_n' = (n+1) e_n Pbar_{n-1} - n e_{n+1} Pbar_{n+1}.
    n = 20
    x = np.linspace(-0.9, 0.9, 11)
    h = 1e-4
    P = lambda xx: pbar(m, n, xx).astype(float)
    fd = (-P(x + 2 * h) + 8 * P(x + h) - 8 * P(x - h) + P(x - 2 * h)) / (12 * h)
    T = tbar(m, n, x).astype(float)
    assert np.abs(T - (1 - x * x) * fd).max() < 1e-8 * np.abs(T).max()
    Pn = pbar(m, n + 1, x).astype(float)
    for nn in range(m, n):
        e = lambda k: np.sqrt((k * k - m * m) / (4.0 * k * k - 1)) if k > 0 else 0.0
        ident = -nn * e(nn + 1) * Pn[nn + 1]
        if nn - 1 >= m:
            ident = ident + (nn + 1) * e(nn) * Pn[nn - 1]
        assert np.abs(T[nn] - ident).max() < 1e-12


@pytest.mark.parametrize("m", [0, 1, 2, 7])
def test_laplacian_matches_nodal_identity(m):
    # grad_h^2 [Pbar_n^m(x(r)) e^{i m phi}] = -n(n+1) (1-x)^2/ell^2 Pbar_n^m e^{i m phi}, so the
    # Galerkin matrix is -n(n+1)/ell^2 <Pbar_j, (1-x)^2 Pbar_n>; quadrature is exact for n + j <= 2N - 3.
    N = 24
    ell = 1.7
    g = Grid(N, 4, 1, ell)
    P = pbar(m, N, g.x_ld).astype(float)
    n = np.arange(N)
    G = (P * (g.w * g.one_minus_x ** 2)) @ P.T
    ref = -G * (n * (n + 1))[None, :] / ell ** 2
    D = laplacian_matrix(m, N, ell)
    sub = ref[m:, m:]
    mask = (np.add.outer(n[m:], n[m:]) <= 2 * N - 3)
    assert np.abs((D - sub)[mask]).max() < 1e-11 * np.abs(sub).max()
    # pentadiagonal
    i, j = np.nonzero(D)
    assert np.all(np.abs(i - j) <= 2)


# ------------------------------------------------------------------ transforms

@pytest.mark.parametrize("shape", [(6, 4, 1), (5, 6, 4), (8, 8, 2)])
def test_transforms_match_bruteforce(shape):
    nr, nphi, nz = shape
    g = Grid(nr, nphi, nz, 1.3, lz=3.0)
    t = Tables(g)
    rs = np.random.default_rng(7)
    s = rs.standard_normal((nz, nr, nphi))
    S = forward(s, g, t)
    Sb = forward_bruteforce(s, g)
    assert np.abs(S - Sb).max() < 1e-13
    C = synth.geometric_spectrum(g.M, g.nrc, nz, g.nzc, seed=3, a=0.8, b=0.9, c=0.9)
    assert np.abs(backward(C, g, t) - backward_bruteforce(C, g)).max() < 1e-13


@pytest.mark.parametrize("shape", [(32, 16, 1), (24, 12, 8), (16, 10, 6)])
def test_round_trip_exact_on_band_limited(shape):
    nr, nphi, nz = shape
    g = Grid(nr, nphi, nz, 0.8)
    t = Tables(g)
    C = synth.geometric_spectrum(g.M, g.nrc, nz, g.nzc, seed=11, a=0.95, b=0.95, c=0.95)
    C2 = forward(backward(C, g, t), g, t)
    assert np.abs(C2 - C).max() < 1e-14 * np.abs(C).max() * nr


def test_azimuthal_purity():
    # Sec. 5.1: a single-order field keeps its order under the transform pair; with an input that is
    # exactly pi-periodic in phi the odd orders vanish to rounding and the mean stays at rounding level.
    g = Grid(32, 16, 1, 1.0)
    t = Tables(g)
    c2 = np.cos(2 * g.phi[:8])
    cos2 = np.concatenate([c2, c2])
    s = (g.r ** 2 * np.exp(-g.r ** 2 / 2))[None, :, None] * cos2[None, None, :]
    S = forward(s, g, t)
    scale = np.abs(S).max()
    assert np.all(S[1::2] == 0.0)                 # odd orders identically zero
    assert np.abs(S[0]).max() <= 8.5e-17          # the paper's bound on the azimuthal mean
    assert np.abs(S[4:]).max() <= 1e-16 * scale


def test_representation_errors_match_paper():
    sA = lambda r, p: r * np.cos(p) / (r ** 2 + 1.7 ** 2) + r ** 2 * np.cos(2 * p) / (r ** 2 + 1.7 ** 2) ** 2
    sB = lambda r, p: r ** 2 * np.exp(-r ** 2 / 2) * np.cos(2 * p)
    for name, ell, nr, val, how in _rows("representation.txt"):
        ell, nr, val = float(ell), int(nr), float(val)
        g = Grid(nr, 8, 1, ell)
        t = Tables(g)
        R, P = np.meshgrid(g.r, g.phi, indexing="ij")
        s = ({"sA": sA, "sB": sB}[name])(R, P)[None]
        err = _area_rel(g, backward(forward(s, g, t), g, t), s)
        if how == "at_most":
            assert err <= val
        else:
            assert float(f"{err:.1e}") == val, (name, ell, nr, err)


# ------------------------------------------------------------------ scalar nonlinear term

def test_u2_closed_form_axisymmetric():
    # u = 1 - x = sqrt2 Pbar_0^0 - sqrt(2/3) Pbar_1^0  =>  u^2 = (1-x)^2 has coefficients
    # (4 sqrt2/3, -2 sqrt(2/3), (2/3) sqrt(2/5)) on Pbar_0..2 (same polynomial as Eq. logproxy).
    g = Grid(16, 8, 1, 1.0)
    t = Tables(g)
    S = np.zeros((g.M, g.nrc, 1), complex)
    S[0, 0, 0] = np.sqrt(2)
    S[0, 1, 0] = -np.sqrt(2 / 3)
    R = rhs_scalar(S, g, t, "u2")
    ref = np.zeros_like(R)
    ref[0, 0, 0] = 4 * np.sqrt(2) / 3
    ref[0, 1, 0] = -2 * np.sqrt(2 / 3)
    ref[0, 2, 0] = 2 / 3 * np.sqrt(2 / 5)
    assert np.abs(R - ref).max() < 1e-14


def test_u2_closed_form_m1():
    # u = sin(theta) cos(phi) = 2 ell r cos(phi)/(r^2+ell^2): stored m = 1 coefficient 1/sqrt3 on Pbar_1^1.
    # u^2 = (1-x^2)(1 + cos 2phi)/2: m = 0 part (P_0 - P_2)/3, m = 2 part P_2^2/12 (half of the cos).
    g = Grid(12, 8, 1, 0.7)
    t = Tables(g)
    S = np.zeros((g.M, g.nrc, 1), complex)
    S[1, 1, 0] = 1 / np.sqrt(3)
    R = rhs_scalar(S, g, t, "u2")
    ref = np.zeros_like(R)
    ref[0, 0, 0] = np.sqrt(2) / 3
    ref[0, 2, 0] = -np.sqrt(2 / 5) / 3
    ref[2, 2, 0] = (1 / 12) * np.sqrt(48 / 5)
    assert np.abs(R - ref).max() < 1e-14


def test_kpp_term_equals_quadratic_combination():
    # gamma u (1 - u) = gamma u - gamma u^2, with u = B(S): the forward transform is linear
    g = Grid(20, 12, 4, 1.1)
    t = Tables(g)
    S = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=5, a=0.7, b=0.8, c=0.8)
    from oracle.rhs import apply_mask
    lhs = rhs_scalar(S, g, t, "kpp", 0.25)
    rhs = apply_mask(0.25 * forward(backward(S, g, t), g, t), g) - 0.25 * rhs_scalar(S, g, t, "u2")
    assert np.abs(lhs - rhs).max() < 1e-14


# ------------------------------------------------------------------ time stepping

@pytest.mark.parametrize("row", _rows("oseen_table.txt"))
def test_oseen_table(row):
    scheme, dt, err_p, gam_p, m2_p = row
    dt = float(dt)
    nu, tf, nr = 0.1, 10.0, 96
    g = Grid(nr, 2, 1, 1.0)
    t = Tables(g)
    B = lambda tt: 1 + 2 * nu * tt
    om = lambda r, tt: np.exp(-r ** 2 / (2 * B(tt))) / (2 * np.pi * B(tt))
    s0 = np.broadcast_to(om(g.r, 0)[None, :, None], (1, nr, 2)).copy()
    S0 = forward(s0, g, t)
    diss = ts.Dissipation(g, nu)
    A = lambda S: np.zeros_like(S)
    n = int(round(tf / dt))
    integ = ts.integrate_febe if scheme == "febe" else ts.integrate_abcn
    s = backward(integ(S0, dt, n, diss, A), g, t)[0, :, 0]
    ex = om(g.r, tf)
    aw = g.area_w
    err = np.sqrt(np.sum(aw * (s - ex) ** 2) / np.sum(aw * ex ** 2))
    gam = 2 * np.pi * np.sum(aw * s)
    m2 = 2 * np.pi * np.sum(aw * g.r ** 2 * s)
    assert f"{err:.3e}" == f"{float(err_p):.3e}"
    assert f"{gam:.7f}" == gam_p
    assert f"{m2:.4f}" == m2_p


@pytest.mark.parametrize("row", _rows("kpp_linear.txt"))
def test_kpp_linearised(row):
    dt, err_p, digits = float(row[0]), float(row[1]), int(row[2])
    nr, ell, T = 96, 4.0, 20.0
    g = Grid(nr, 2, 1, ell)
    t = Tables(g)
    A0, D, gam = 1e-6, 1.0, 0.25
    s0 = np.broadcast_to((A0 * np.exp(-g.r ** 2 / 2))[None, :, None], (1, nr, 2)).copy()
    diss = ts.Dissipation(g, D)
    S = ts.integrate_abcn(forward(s0, g, t), dt, int(round(T / dt)), diss,
                          lambda S: rhs_scalar(S, g, t, "kpp", gam))
    s = backward(S, g, t)[0, :, 0]
    sig2 = 1 + 2 * D * T
    ex = A0 / sig2 * np.exp(gam * T) * np.exp(-g.r ** 2 / (2 * sig2))
    aw = g.area_w
    err = np.sqrt(np.sum(aw * (s - ex) ** 2) / np.sum(aw * ex ** 2))
    # the paper prints 3 or 4 significant digits (5.806e-6 appears as 5.80e-6): allow one unit
    # in the last printed digit
    unit = 10.0 ** (np.floor(np.log10(err_p)) - (digits - 1))
    assert abs(err - err_p) <= unit, (dt, err)


def _heat_mode_error(nr, dt, nu=0.1):
    g = Grid(nr, 8, 1, 1.0)
    t = Tables(g)
    R, P = np.meshgrid(g.r, g.phi, indexing="ij")
    Bt = lambda tt: 1 + 2 * nu * tt
    sm = lambda tt: Bt(tt) ** -3 * R ** 2 * np.exp(-R ** 2 / (2 * Bt(tt))) * np.cos(2 * P)
    diss = ts.Dissipation(g, nu)
    S = ts.integrate_abcn(forward(sm(0)[None], g, t), dt, int(round(1 / dt)), diss, lambda S: np.zeros_like(S))
    return _area_rel(g, backward(S, g, t), sm(1.0)[None])


@pytest.mark.parametrize("row", _rows("manufactured_mode.txt"))
def test_manufactured_mode_spatial_error(row):
    nr, val = int(row[0]), float(row[1])
    err = _heat_mode_error(nr, 1e-3)
    assert float(f"{err:.1e}") == val, err


def test_abcn_second_order_on_heat_mode():
    # Sec. 5.1 (Fig. manufactured b): refining dt recovers second order with AB-CN once the spatial
    # error (2.7e-7 at N_r = 96) is below the temporal one.
    errs = [_heat_mode_error(96, dt) for dt in (0.1, 0.05, 0.025)]
    p = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((p > 1.7) & (p < 2.2)), p


# ------------------------------------------------------------------ two-thirds rule

def _embed(S, gc, gf):
    """Spectrum S of grid gc placed on the finer periodic grid gf (same radial grid and chop)."""
    Sf = np.zeros((gf.M, gc.nrc, gf.nz), complex)
    for kk, k in enumerate(gc.kvals()):
        Sf[:gc.M, :, k % gf.nz] = S[:, :, kk]
    return Sf


def _kept_pairs(gc):
    keep = np.arange(gc.M)[:, None] <= gc.dealias_m()
    keep = keep & ((np.abs(gc.kvals()) <= gc.dealias_k()) & gc.kmask())[None, :]
    return [(m, kk, k) for m in range(gc.M) for kk, k in enumerate(gc.kvals()) if keep[m, kk]]


@pytest.mark.parametrize("kind", ["u2", "kpp"])
def test_scalar_rhs_two_thirds_rule_is_alias_free(kind):
    # Sec. 3.3: the periodic directions are dealiased by the two-thirds margin.  The input carries
    # modes in the margin as well; the masked RHS on (N_phi, N_z) must equal the RHS of the masked
    # input on (2 N_phi, 2 N_z), where the product of the kept modes does not alias in phi or z,
    # on every kept (m, k).  A mask applied only to the output lets the margin modes alias into
    # the kept ones and fails this.
    gc = Grid(10, 12, 6, 0.9, lz=3.0)
    gf = Grid(10, 24, 12, 0.9, lz=3.0)
    S = synth.geometric_spectrum(gc.M, gc.nrc, gc.nz, gc.nzc, seed=41, a=0.8, b=0.9, c=0.9)
    from oracle.rhs import apply_mask
    assert np.abs(S - apply_mask(S, gc)).max() > 0.05  # the margin is populated
    Rc = rhs_scalar(S, gc, Tables(gc), kind, 0.3)
    Rf = rhs_scalar(_embed(apply_mask(S, gc), gc, gf), gf, Tables(gf), kind, 0.3)
    big = np.abs(Rc).max()
    for m, kk, k in _kept_pairs(gc):
        assert np.abs(Rc[m, :, kk] - Rf[m, :, k % gf.nz]).max() < 1e-13 * big, (m, k)
    # nothing leaves the mask, and margin-only input has no product
    assert np.abs(Rc - apply_mask(Rc, gc)).max() == 0.0
    margin = S - apply_mask(S, gc)
    assert np.abs(rhs_scalar(margin, gc, Tables(gc), kind, 0.3)).max() == 0.0
