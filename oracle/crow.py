"""Oracle: Crow's dispersion relation for the symmetric mode of a counter-rotating vortex pair.

Test infrastructure only (see the package header).

Sec. 5.3 (Results and validation), Eq. crow-dispersion: with beta = kappa b, delta = kappa d
(kappa the axial wavenumber, b the separation, d the cutoff distance of the core),
    xi(beta)    = beta K_1(beta),
    eta(beta)   = beta^2 K_0(beta) + beta K_1(beta),
    varpi(delta) = [(cos delta - 1)/delta^2 + sin(delta)/delta - Ci(delta)] / 2,
the symmetric mode grows at alpha_S (units Gamma / (2 pi b^2)) with
    alpha_S^2 = (1 - eta + beta^2 varpi) (1 + xi - beta^2 varpi).
For a Lamb-Oseen core of radius a the cutoff is d = a exp((1 - gamma_E - ln 2) / 2).

K_0, K_1 and Ci are written from their ascending series (small arguments: beta < 2 and
delta < 1 here), with the Euler-Mascheroni constant gamma_E and the harmonic numbers H_k:
    I_0(x) = sum_k (x^2/4)^k / (k!)^2,
    K_0(x) = -(ln(x/2) + gamma_E) I_0(x) + sum_{k>=1} H_k (x^2/4)^k / (k!)^2,
    K_1(x) = 1/x + ln(x/2) I_1(x) - (x/4) sum_{k>=0} (psi(k+1) + psi(k+2)) (x^2/4)^k / (k! (k+1)!),
             with I_1(x) = (x/2) sum_k (x^2/4)^k / (k! (k+1)!) and psi(k+1) = H_k - gamma_E,
    Ci(x)  = gamma_E + ln x + sum_{k>=1} (-1)^k x^(2k) / (2k (2k)!).
The inclination of the symmetric mode's displacement plane follows from the same two factors:
tan^2(theta) = (1 + xi - beta^2 varpi) / (1 - eta + beta^2 varpi).
"""
from __future__ import annotations

import math

EULER_GAMMA = 0.57721566490153286060651209008240243


def _harmonic(k: int) -> float:
    return sum(1.0 / j for j in range(1, k + 1))


def bessel_k0(x: float, terms: int = 40) -> float:
    q = x * x / 4.0
    i0 = 0.0
    s = 0.0
    t = 1.0  # q^k / (k!)^2
    for k in range(terms):
        if k > 0:
            t *= q / (k * k)
        i0 += t
        s += _harmonic(k) * t
    return -(math.log(x / 2.0) + EULER_GAMMA) * i0 + s


def bessel_k1(x: float, terms: int = 40) -> float:
    q = x * x / 4.0
    i1 = 0.0
    s = 0.0
    t = 1.0  # q^k / (k! (k+1)!)
    for k in range(terms):
        if k > 0:
            t *= q / (k * (k + 1))
        i1 += t
        psi1 = _harmonic(k) - EULER_GAMMA
        psi2 = _harmonic(k + 1) - EULER_GAMMA
        s += (psi1 + psi2) * t
    i1 *= x / 2.0
    return 1.0 / x + math.log(x / 2.0) * i1 - (x / 4.0) * s


def cosine_integral(x: float, terms: int = 40) -> float:
    s = 0.0
    t = 1.0  # x^(2k) / (2k)!
    for k in range(1, terms):
        t *= x * x / ((2 * k - 1) * (2 * k))
        s += (-1) ** k * t / (2 * k)
    return EULER_GAMMA + math.log(x) + s


def lamb_oseen_cutoff(a: float) -> float:
    """Cutoff distance d of a Lamb-Oseen core of radius a (Sec. 5.3)."""
    return a * math.exp((1.0 - EULER_GAMMA - math.log(2.0)) / 2.0)


def symmetric_factors(beta: float, d_over_b: float) -> tuple[float, float]:
    """The two factors (1 - eta + beta^2 varpi, 1 + xi - beta^2 varpi) of Eq. crow-dispersion."""
    delta = beta * d_over_b
    k0, k1 = bessel_k0(beta), bessel_k1(beta)
    xi = beta * k1
    eta = beta * beta * k0 + beta * k1
    varpi = 0.5 * ((math.cos(delta) - 1.0) / (delta * delta) + math.sin(delta) / delta - cosine_integral(delta))
    return 1.0 - eta + beta * beta * varpi, 1.0 + xi - beta * beta * varpi


def growth_rate(beta: float, d_over_b: float) -> float:
    """alpha_S of the symmetric mode (0 where the mode is stable)."""
    a, b = symmetric_factors(beta, d_over_b)
    return math.sqrt(a * b) if a * b > 0 else 0.0


def inclination_deg(beta: float, d_over_b: float) -> float:
    a, b = symmetric_factors(beta, d_over_b)
    return math.degrees(math.atan(math.sqrt(b / a)))


def most_amplified(d_over_b: float, lo: float = 0.2, hi: float = 1.5, tol: float = 1e-12) -> tuple[float, float]:
    """(beta_max, alpha_max) by golden-section search of alpha_S over [lo, hi]."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = growth_rate(c, d_over_b), growth_rate(d, d_over_b)
    while b - a > tol:
        if fc > fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = growth_rate(c, d_over_b)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = growth_rate(d, d_over_b)
    x = 0.5 * (a + b)
    return x, growth_rate(x, d_over_b)
