"""Pins of the oracle's dissipation operator (Eq. dissipation) with an axial wavenumber and
hyperviscosity, and of the constant forcing that the logarithmic proxy's dissipation adds
(Eq. logproxy), against the mathematics rather than the oracle's own matrices.

* The time integration with kappa != 0: a three-dimensional heat-kernel solution (an m = 0 and an
  m = 2 Gaussian mode times cos(kappa z)) advanced by the oracle's AB-CN with nu only, against the
  closed form e^{-nu kappa^2 t} x (the two-dimensional solution).
* The operator itself for p = 4, 6, 8 (nu = 0, nu_h = 1): applied to a field that lies in the
  span of the retained basis and stays there under p/2 Laplacians, against the coefficients of
  -(-grad^2)^{p/2} of that field, formed symbolically (sympy) from the cylindrical Laplacian
  d^2/dr^2 + (1/r) d/dr - m^2/r^2 - kappa^2 in r, evaluated at the nodes and transformed.
* The proxy forcing nu grad^2 Lambda - nu_h (-grad^2)^{p/2} Lambda for Lambda = ln(r^2 + ell^2),
  formed the same way.

The symbolic route shares nothing with the oracle's Eq. del2h-entries matrices: a dropped
kappa^2, a sign or power slip in the hyperviscosity, or a wrong power in the proxy forcing fails
one of these tests.
"""
import numpy as np
import pytest
import sympy as sp

from oracle import timestep as ts
from oracle.grid import Grid
from oracle.logproxy import proxy_forcing
from oracle.transform import Tables, backward, forward

_r = sp.symbols("r", positive=True)


def _cyl_laplacian(expr, m, kappa):
    """grad^2 of expr(r) e^{i m phi} e^{i kappa z}, divided by the exponentials."""
    return sp.together(sp.diff(expr, _r, 2) + sp.diff(expr, _r) / _r - m ** 2 * expr / _r ** 2
                       - kappa ** 2 * expr)


def _neg_lap_power(expr, m, kappa, j):
    out = expr
    for _ in range(j):
        out = sp.cancel(-_cyl_laplacian(out, m, kappa))
    return out


def _nodal(g, radial, m, kk):
    """Real field radial(r_i) cos(m phi_j) cos(kappa_k z_l) in the oracle's (N_z, N_r, N_phi) layout."""
    kap = 2 * np.pi * kk / g.lz
    return (np.cos(kap * g.z)[:, None, None] * radial[None, :, None]
            * np.cos(m * g.phi)[None, None, :])


# ------------------------------------------------------------------ heat kernel with kappa

def _heat_kernel(r, phi, z, t, m, nu, t0, kap):
    """r^m cos(m phi) exp(-r^2 / (4 nu (t0 + t))) / (t0 + t)^{m+1} cos(kappa z) e^{-nu kappa^2 t}:
    the m-th azimuthal derivative of the 2D heat kernel times a decaying axial mode."""
    T = t0 + t
    rad = r ** m * np.exp(-r ** 2 / (4 * nu * T)) / T ** (m + 1)
    return (np.cos(kap * z)[:, None, None] * rad[None, :, None] * np.cos(m * phi)[None, None, :]
            * np.exp(-nu * kap ** 2 * t))


def _heat_error(m, dt, nu=0.05, t0=5.0, tf=4.0, with_kappa_factor=True):
    g = Grid(48, 8, 4, 2.0, lz=2 * np.pi * 0.7)
    t = Tables(g)
    kap = 2 * np.pi / g.lz
    s0 = _heat_kernel(g.r, g.phi, g.z, 0.0, m, nu, t0, kap)
    diss = ts.Dissipation(g, nu)
    S = ts.integrate_abcn(forward(s0, g, t), dt, int(round(tf / dt)), diss, lambda S: np.zeros_like(S))
    ex = _heat_kernel(g.r, g.phi, g.z, tf, m, nu, t0, kap)
    if not with_kappa_factor:
        ex = ex * np.exp(nu * kap ** 2 * tf)
    aw = g.area_w[None, :, None]
    s = backward(S, g, t)
    return np.sqrt(np.sum(aw * (s - ex) ** 2) / np.sum(aw * ex ** 2))


@pytest.mark.parametrize("m", [0, 2])
def test_abcn_heat_kernel_with_axial_mode(m):
    # nu kappa^2 t = 0.41: the axial factor e^{-nu kappa^2 t} is a 34% effect, so a dropped or
    # misplaced kappa^2 cannot hide in the tolerance
    # (the spatial error on 48 nodes at ell = 2 is below 1e-8; what remains is AB-CN's O(dt^2))
    errs = [_heat_error(m, dt) for dt in (0.1, 0.05)]
    assert errs[1] < 5e-5, errs
    order = np.log2(errs[0] / errs[1])
    assert 1.8 < order < 2.2, (errs, order)
    assert _heat_error(m, 0.05, with_kappa_factor=False) > 0.3


# ------------------------------------------------------------------ hyperviscosity and kappa shift

# exact rationals, so that sympy's cancellation of (1 + x) is exact
_ELL = sp.Rational(13, 10)
_POLY = (sp.Integer(1), sp.Rational(1, 2), sp.Rational(-3, 10))          # 1 + x/2 - 3x^2/10
_x = sp.symbols("x")


def _x_laplacian(expr, m, kappa, ell):
    """The same cylindrical Laplacian written in the mapped coordinate of Eq. map: with
    r d/dr = (1 - x^2) d/dx and 1/r^2 = (1 - x) / (ell^2 (1 + x)),
    grad^2 = (1 - x) / (ell^2 (1 + x)) [((1 - x^2) d/dx)^2 - m^2] - kappa^2."""
    rdr = lambda f: (1 - _x ** 2) * sp.diff(f, _x)
    return sp.cancel((1 - _x) / (ell ** 2 * (1 + _x)) * (rdr(rdr(expr)) - m ** 2 * expr) - kappa ** 2 * expr)


def _poly_mode_x(m):
    """sin^m(theta) P(x): a field in the span of Pbar_m^m .. Pbar_{m+2}^m."""
    return sp.sqrt(1 - _x ** 2) ** m * sum(c * _x ** i for i, c in enumerate(_POLY))


def test_mapped_laplacian_equals_cylindrical_laplacian():
    # the x form above is the r form after the change of variables of Eq. map
    m, kap = 2, sp.Rational(3, 4)
    f = _poly_mode_x(m)
    lx = _x_laplacian(f, m, kap, _ELL)
    x_of_r = (_r ** 2 - _ELL ** 2) / (_r ** 2 + _ELL ** 2)
    fr = sp.simplify(f.subs(_x, x_of_r))
    lr = _cyl_laplacian(fr, m, kap)
    for rv in (0.3, 1.0, 2.7, 11.0):
        a = float(lx.subs(_x, x_of_r).subs(_r, rv))
        b = float(lr.subs(_r, rv))
        assert abs(a - b) <= 1e-12 * max(abs(b), 1.0), (rv, a, b)


@pytest.mark.parametrize("p", [4, 6, 8])
@pytest.mark.parametrize("m,kk", [(0, 0), (0, 1), (2, 1), (3, -1)])
def test_hyperviscous_operator_against_symbolic_powers(p, m, kk):
    g = Grid(28, 8, 4, float(_ELL), lz=2 * np.pi * 0.8)
    t = Tables(g)
    kap = sp.Rational(5 * kk, 4)                                 # 2 pi k / L_z
    assert abs(float(kap) - 2 * np.pi * kk / g.lz) < 1e-15
    f = _poly_mode_x(m)
    lf = f
    for _ in range(p // 2):
        lf = -_x_laplacian(lf, m, kap, _ELL)
    lf = -lf                                                     # -(-grad^2)^{p/2} f
    xs = g.x_ld.astype(np.float64)
    rad_f = np.array([float(f.subs(_x, sp.Float(str(v), 30))) for v in g.x_ld])
    rad_lf = np.array([float(lf.subs(_x, sp.Float(str(v), 30))) for v in g.x_ld])
    assert rad_f.shape == xs.shape
    S = forward(_nodal(g, rad_f, m, kk), g, t)
    E = forward(_nodal(g, rad_lf, m, kk), g, t)
    diss = ts.Dissipation(g, 0.0, 1.0, p)
    slot = kk % g.nz
    # the field's exact coefficients vanish above degree m + 2; its transform holds rounding noise
    # there, which p/2 Laplacians would amplify by ~n^p, so the input is cut to its exact support
    s = S[m, m:, slot].copy()
    assert np.abs(s[3:]).max() <= 1e-14 * np.abs(s).max()
    s[3:] = 0.0
    got = diss.L[(m, slot)] @ s
    want = E[m, m:, slot]
    assert np.linalg.norm(got - want) <= 1e-11 * np.linalg.norm(want), (
        np.linalg.norm(got - want) / np.linalg.norm(want))
    # the result stays in the retained span: the highest degree reached is m + 2 + p
    assert np.abs(want[2 + p + 1:]).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("p", [4, 6, 8])
def test_viscous_part_and_shift_combine_linearly(p):
    # L(nu, nu_h) = nu (Dbar - kappa^2) - nu_h (-(Dbar - kappa^2))^{p/2}: the two parts add
    g = Grid(20, 6, 4, 0.9)
    a = ts.Dissipation(g, 0.3, 0.0, p)
    b = ts.Dissipation(g, 0.0, 0.7, p)
    c = ts.Dissipation(g, 0.3, 0.7, p)
    for key in c.L:
        assert np.allclose(c.L[key], a.L[key] + b.L[key], rtol=1e-13, atol=0.0)


# ------------------------------------------------------------------ proxy forcing

@pytest.mark.parametrize("p", [4, 6, 8])
@pytest.mark.parametrize("nu,nu_h", [(1.0, 0.0), (0.0, 1.0), (0.37, 2.5)])
def test_proxy_forcing_against_symbolic_dissipation_of_lambda(p, nu, nu_h):
    ell = 1.7
    g = Grid(24, 2, 1, ell)
    t = Tables(g)
    lam = sp.log(_r ** 2 + ell ** 2)
    lap = sp.cancel(_cyl_laplacian(lam, 0, 0))                    # 4 ell^2 / (r^2 + ell^2)^2
    assert sp.simplify(lap - 4 * ell ** 2 / (_r ** 2 + ell ** 2) ** 2) == 0
    # L Lambda = nu grad^2 Lambda - nu_h (-grad^2)^{p/2} Lambda; Lambda itself is not in the span,
    # but grad^2 Lambda is, and (-grad^2)^{p/2} Lambda = -(-grad^2)^{p/2 - 1} grad^2 Lambda
    hyper = _neg_lap_power(lap, 0, 0, p // 2 - 1)
    expr = nu * lap + nu_h * hyper
    rad = sp.lambdify(_r, expr, "numpy")(g.r)
    want = forward(_nodal(g, rad, 0, 0), g, t)[0, :, 0].real
    got = proxy_forcing(g, nu, nu_h, p)
    assert np.linalg.norm(got - want) <= 1e-11 * np.linalg.norm(want), (
        np.linalg.norm(got - want) / np.linalg.norm(want))
