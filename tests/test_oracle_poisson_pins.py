"""Pins of the oracle's inverse Laplacian with the logarithmic proxy and of the far-field level
removal (Sec. 3.1, Eq. laplacian, Eq. logproxy), against closed forms:

* a field with a known constant at infinity (a polynomial in x plus a constant, exact in the basis);
* Poisson problems with a net source: a normalised Gaussian source, whose amplitude c = 1/(4 pi) and
  regular part (1/(4 pi)) [ln(r^2/(r^2 + ell^2)) + E1(r^2/sigma^2)] follow from the two-dimensional
  Green's function, and an exact-in-the-basis source a grad_h^2 Lambda + grad_h^2 ((1 - x)/2) formed
  symbolically, whose solution is c = a and (1 - x)/2;
* the ordinary harmonics (m, k) != (0, 0): Gaussian modes whose Laplacian is formed symbolically.
"""
import numpy as np
import pytest
import sympy as sp
from scipy.special import exp1

from oracle.basis import pbar
from oracle.grid import Grid
from oracle.poisson import far_field_level, laplacian_solve, remove_far_field
from oracle.transform import Tables, backward, forward

_r, _x = sp.symbols("r x", positive=True)


def _nodal(g, radial, m=0, kk=0):
    kap = 2 * np.pi * kk / g.lz
    return (np.cos(kap * g.z)[:, None, None] * radial[None, :, None] * np.cos(m * g.phi)[None, None, :])


def _at_x(expr, g):
    return np.array([float(expr.subs(_x, sp.Float(str(v), 30))) for v in g.x_ld])


# ------------------------------------------------------------------ far-field level

def test_far_field_level_of_known_constants_and_its_removal():
    g = Grid(20, 4, 4, 1.3, lz=3.0)
    t = Tables(g)
    x = g.x
    s = _nodal(g, 3.0 + (1 - x) ** 2) + _nodal(g, 2.0 + (1 - x) ** 2, kk=1) \
        + _nodal(g, np.sqrt(1 - x ** 2) * (1 + x), m=1)
    S = forward(s, g, t)
    lev = far_field_level(S, g)
    assert abs(lev[0] - 3.0) < 1e-13 and abs(lev[1] - 1.0) < 1e-13 and abs(lev[-1] - 1.0) < 1e-13
    R = remove_far_field(S, g)
    # the result is the decaying polynomial part; m = 1 and the degrees n >= 1 are untouched
    want = forward(_nodal(g, (1 - x) ** 2) + _nodal(g, (1 - x) ** 2, kk=1)
                   + _nodal(g, np.sqrt(1 - x ** 2) * (1 + x), m=1), g, t)
    assert np.abs(R - want).max() < 1e-13
    assert np.array_equal(R[0, 1:], S[0, 1:]) and np.array_equal(R[1:], S[1:])
    # the series evaluated at x = 1 (r = infinity) by the basis functions themselves vanishes
    p1 = pbar(0, g.nrc, np.array([1.0])).astype(np.float64)[:, 0]
    assert np.abs(p1 @ R[0]).max() < 1e-13
    assert abs(p1 @ S[0, :, 0] - 3.0) < 1e-13


# ------------------------------------------------------------------ net-source Poisson problems

@pytest.mark.parametrize("nr,ell,sigma", [(96, 1.0, 1.0), (128, 2.0, 1.5)])
def test_gaussian_source_amplitude_and_regular_part(nr, ell, sigma):
    g = Grid(nr, 4, 1, ell)
    t = Tables(g)
    f = np.exp(-g.r ** 2 / sigma ** 2) / (np.pi * sigma ** 2)          # unit integral over the plane
    F = forward(_nodal(g, f), g, t)
    S, c = laplacian_solve(F, g, "solve")
    # spectral convergence: 1.9e-7, 8.8e-9, 2.3e-11, 2.2e-13 at N_r = 32, 48, 64, 96 (ell = sigma = 1)
    assert abs(c - 1.0 / (4 * np.pi)) < 2e-12, c
    u = g.r ** 2 / sigma ** 2
    reg = (np.log(g.r ** 2 / (g.r ** 2 + ell ** 2)) + exp1(u)) / (4 * np.pi)
    got = backward(S, g, t)[0, :, 0]
    assert np.abs(got - reg).max() < 2e-10 * np.abs(reg).max(), np.abs(got - reg).max()
    # the prescribe variant with the true amplitude gives the same potential
    S2, _ = laplacian_solve(F, g, "prescribe", c=1.0 / (4 * np.pi))
    # (the two variants reach shat_0 through different rounding: the gauge sums degrees weighted by
    # sqrt((2n + 1)/2))
    assert np.abs(S2 - S).max() < 5e-10 * np.abs(S).max()


def _lap_h_x(expr, ell):
    """grad_h^2 of an axisymmetric function of x through Eq. map: (1 - x)/(ell^2 (1 + x)) ((1 - x^2) d/dx)^2."""
    rdr = lambda f: (1 - _x ** 2) * sp.diff(f, _x)
    return sp.cancel((1 - _x) / (ell ** 2 * (1 + _x)) * rdr(rdr(expr)))


@pytest.mark.parametrize("a", [0.0, 1.0, -2.5])
def test_exact_source_with_amplitude(a):
    ell = sp.Rational(7, 5)
    g = Grid(24, 2, 1, float(ell))
    t = Tables(g)
    lam = sp.log((1 + _x) / (1 - _x) * ell ** 2 + ell ** 2)       # ln(r^2 + ell^2) written in x
    img = _lap_h_x(lam, ell)                                       # = (1 - x)^2 / ell^2 (Eq. logproxy)
    assert sp.simplify(img - (1 - _x) ** 2 / ell ** 2) == 0
    reg = (1 - _x) / 2                                             # decays: 0 at x = 1
    f = sp.Rational(a).limit_denominator(10) * img + _lap_h_x(reg, ell)
    F = forward(_nodal(g, _at_x(f, g)), g, t)
    S, c = laplacian_solve(F, g, "solve")
    tol = 2e-12 * max(1.0, abs(a))
    assert abs(c - a) < tol, c
    want = forward(_nodal(g, _at_x(reg, g)), g, t)
    assert np.abs(S - want).max() < tol
    Sp, _ = laplacian_solve(F, g, "prescribe", c=a)
    assert np.abs(Sp - want).max() < tol


# ------------------------------------------------------------------ other harmonics

@pytest.mark.parametrize("m,kk", [(2, 1), (0, 1), (1, 0), (3, -1)])
def test_ordinary_harmonics_against_symbolic_laplacian(m, kk):
    # (spectral convergence in N_r: up to 6.9e-9 at 64 nodes, 4.5e-12 at 96, 1.2e-13 at 128)
    g = Grid(128, 8, 4, 1.0, lz=2 * np.pi * 0.8)
    t = Tables(g)
    kap = sp.Rational(5 * kk, 4)
    s = _r ** m * sp.exp(-_r ** 2)
    lap = sp.diff(s, _r, 2) + sp.diff(s, _r) / _r - m ** 2 * s / _r ** 2 - kap ** 2 * s
    fs = sp.lambdify(_r, s, "numpy")
    fl = sp.lambdify(_r, lap, "numpy")
    S0 = forward(_nodal(g, fs(g.r), m, kk), g, t)
    F = forward(_nodal(g, fl(g.r), m, kk), g, t)
    S, _ = laplacian_solve(F, g, "solve")
    slot = kk % g.nz
    got, want = S[m, m:, slot], S0[m, m:, slot]
    assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want), np.linalg.norm(got - want) / np.linalg.norm(want)
