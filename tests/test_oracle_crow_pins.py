"""Pins of the oracle's Crow dispersion relation (Sec. 5.3, Eq. crow-dispersion) and of its
axial modal energy (the diagnostic from which Sec. 5.3 reads the growth rate).

* K_0, K_1 and Ci, written from their series, against scipy's implementations.
* The values the paper prints for the relation (tests/golden/crow_dispersion.txt): the Lamb-Oseen
  cutoff, the growth rate at the simulated wavenumber, and the most-amplified point.  The paper
  does not state the cutoff ratio behind its most-amplified point; the pin takes the ratio at which
  the maximum sits at the printed beta_max and checks the three other printed numbers there.
* The modal energy against closed forms (a Gaussian stream function, with and without an axial
  wave) and against the kinetic energy summed directly on the physical grid (Parseval).
"""
import math
import os

import numpy as np
import pytest

from oracle import crow
from oracle.diagnostics import axial_modal_energy, kinetic_energy
from oracle.grid import Grid
from oracle.rhs import VecTables
from oracle.transform import Tables, forward
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    out = {}
    with open(os.path.join(HERE, "golden", "crow_dispersion.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val, digits = line.split()
            out[name] = (float(val), int(digits))
    return out


def _within_print(x, val, digits):
    # the printed value has `digits` significant figures: half a unit in the last place
    q = 10 ** (math.floor(math.log10(abs(val))) - digits + 1)
    return abs(x - val) <= 0.5 * q * (1 + 1e-9)


@pytest.mark.parametrize("x", [0.01, 0.08, 0.3, 0.7306, 1.0, 1.7])
def test_special_functions_against_scipy(x):
    sc = pytest.importorskip("scipy.special")
    assert abs(crow.bessel_k0(x) - sc.k0(x)) < 1e-13 * max(1.0, abs(sc.k0(x)))
    assert abs(crow.bessel_k1(x) - sc.k1(x)) < 1e-13 * max(1.0, abs(sc.k1(x)))
    assert abs(crow.cosine_integral(x) - sc.sici(x)[1]) < 1e-13 * max(1.0, abs(sc.sici(x)[1]))


def test_lamb_oseen_cutoff_and_rate_at_the_simulated_wavenumber():
    g = _golden()
    ratio = crow.lamb_oseen_cutoff(1.0)
    assert _within_print(ratio, *g["cutoff_over_a"])
    beta = 2 * math.pi / 8.6  # L_z = 8.6 b
    assert _within_print(beta, 0.7306, 4)
    alpha = crow.growth_rate(beta, 0.125 * ratio)
    assert _within_print(alpha, *g["alpha_at_beta_0.7306_a_over_b_0.125"])


def test_most_amplified_point_is_consistent():
    g = _golden()
    target = g["beta_max"][0]
    # bisect the cutoff ratio for which the maximum sits at the printed beta_max
    lo, hi = 0.03, 0.08   # beta_max decreases as d / b decreases
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if crow.most_amplified(mid)[0] > target:
            hi = mid
        else:
            lo = mid
    db = 0.5 * (lo + hi)
    bmax, amax = crow.most_amplified(db)
    assert abs(bmax - target) < 1e-6
    assert _within_print(amax, *g["alpha_max"])
    assert _within_print(crow.inclination_deg(bmax, db), *g["inclination_deg"])
    assert _within_print(2 * math.pi / bmax, *g["lambda_max_over_b"])


def test_long_wave_limit_and_stability_band():
    # far above the band the symmetric mode is stable; the maximum is interior to (0, 1.5)
    assert crow.growth_rate(1.4, 0.1) == 0.0
    b, a = crow.most_amplified(0.1)
    assert 0.3 < b < 1.2 and a > crow.growth_rate(0.3, 0.1) and a > crow.growth_rate(1.2, 0.1)


def _gaussian_psi(g, axial):
    R = g.r[None, :, None]
    Z = g.z[:, None, None]
    f = np.exp(-R ** 2) * np.ones((g.nz, g.nr, g.nphi))
    if axial:
        f = f * np.cos(2 * np.pi * Z / g.lz)
    return forward(f, g, Tables(g))


def test_modal_energy_of_a_gaussian_stream_function():
    # psi = exp(-r^2): u_phi = 2 r exp(-r^2), int |u|^2 r dr dphi = 2 pi * 4 int r^3 exp(-2 r^2) dr = pi
    g = Grid(40, 8, 4, 1.0, lz=3.0)
    vt = VecTables(g)
    S = _gaussian_psi(g, False)
    E = axial_modal_energy(S, np.zeros_like(S), g, vt)
    assert abs(E[0] - 0.5 * g.lz * math.pi) < 1e-9
    assert np.all(np.abs(E[1:]) < 1e-12)
    # with cos(2 pi z / L_z) the energy halves and splits equally over k = +1 and -1
    S = _gaussian_psi(g, True)
    E = axial_modal_energy(S, np.zeros_like(S), g, vt)
    kv = g.kvals()
    for k, e in zip(kv, E):
        want = g.lz * math.pi / 8 if abs(k) == 1 else 0.0
        assert abs(e - want) < 1e-9, (k, e, want)


def test_modal_energy_sums_to_the_kinetic_energy():
    g = Grid(24, 12, 8, 0.9, lz=3.0)
    vt = VecTables(g)
    psi = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=4, a=0.8, b=0.8, c=0.8)
    chi = 0.3 * synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=5, a=0.8, b=0.8, c=0.8)
    E = axial_modal_energy(psi, chi, g, vt)
    tot = kinetic_energy(psi, chi, g, vt)
    assert abs(E.sum() - tot) < 1e-12 * tot
    # real fields: k and -k carry the same energy
    kv = g.kvals()
    for k in range(1, g.nz // 2):
        assert abs(E[list(kv).index(k)] - E[list(kv).index(-k)]) < 1e-12 * tot
