"""Pins of the oracle's Fisher-KPP pieces (Sec. 5.2, Eq. kpp, Eq. kpp-linear).

The closed form is checked against the linearised equation itself (finite-difference residual),
its initial value and its exact mass 2 pi A sigma^2 e^{gamma t}; the pointwise evaluation of a
harmonic against the forward transform of a known field (spectral interpolation reproduces the
nodal values and an analytic field between nodes); the front radius against a field whose
half-level crossing is known in closed form.
"""
import numpy as np

from oracle.grid import Grid
from oracle.kpp import front_radius, harmonic_at, linear_solution, weighted_rel_error
from oracle.transform import Tables, forward


def test_linear_solution_solves_the_linearised_equation():
    D, gam, A, sig = 1.0, 0.25, 1e-6, 1.0
    r = np.linspace(0.5, 12.0, 47)
    for t in (0.5, 5.0, 20.0):
        h = 1e-3
        u = linear_solution(r, t, A, sig, D, gam)
        ut = (linear_solution(r, t + h, A, sig, D, gam) - linear_solution(r, t - h, A, sig, D, gam)) / (2 * h)
        ur = (linear_solution(r + h, t, A, sig, D, gam) - linear_solution(r - h, t, A, sig, D, gam)) / (2 * h)
        urr = (linear_solution(r + h, t, A, sig, D, gam) - 2 * u + linear_solution(r - h, t, A, sig, D, gam)) / h ** 2
        res = ut - D * (urr + ur / r) - gam * u
        assert np.abs(res).max() < 1e-6 * np.abs(u).max()
    assert np.allclose(linear_solution(r, 0.0, A, sig, D, gam), A * np.exp(-r ** 2 / (2 * sig ** 2)), rtol=1e-15)


def test_linear_solution_mass():
    # int u dA = 2 pi A sigma^2 e^{gamma t} for every t (diffusion conserves it, the reaction grows it)
    g = Grid(96, 4, 1, 8.0)
    for t in (0.0, 7.0, 20.0):
        u = linear_solution(g.r, t, 2.0, 1.3, 1.0, 0.25)
        mass = 2 * np.pi * (g.area_w * u).sum()
        assert abs(mass / (2 * np.pi * 2.0 * 1.3 ** 2 * np.exp(0.25 * t)) - 1) < 1e-10


def test_harmonic_evaluation_interpolates_the_field():
    g = Grid(64, 8, 1, 4.0)
    t = Tables(g)
    f = lambda r: np.exp(-r ** 2 / 8.0) * (1 + 0.3 * r ** 2 / (1 + r ** 2))
    phys = np.broadcast_to(f(g.r)[None, :, None], (1, g.nr, g.nphi)).copy()
    S = forward(phys, g, t)
    # at the nodes the expansion reproduces the nodal values; between them the analytic field
    assert np.abs(harmonic_at(S, g, 0, 0, g.r).real - f(g.r)).max() < 1e-13
    rr = np.linspace(0.0, 20.0, 201)
    assert np.abs(harmonic_at(S, g, 0, 0, rr).real - f(rr)).max() < 1e-10
    assert np.abs(harmonic_at(S, g, 0, 0, rr).imag).max() < 1e-15


def test_front_radius_of_a_known_profile():
    # u = 1 / (1 + exp((r - R0) / w)) crosses one half at r = R0 exactly
    g = Grid(160, 4, 1, 16.0)
    t = Tables(g)
    R0, w = 23.7, 1.5
    prof = 1 / (1 + np.exp(np.minimum((g.r - R0) / w, 700.0)))
    phys = np.broadcast_to(prof[None, :, None], (1, g.nr, g.nphi)).copy()
    S = forward(phys, g, t)
    assert abs(front_radius(S, g, 60.0) - R0) < 1e-7


def test_weighted_error_norm():
    g = Grid(32, 4, 1, 2.0)
    u = np.ones((1, 32, 4))
    assert abs(weighted_rel_error(1.01 * u, u, g) - 0.01) < 1e-14
    assert weighted_rel_error(u, u, g) == 0.0
