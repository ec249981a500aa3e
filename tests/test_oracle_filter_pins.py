"""Pins of the oracle's adaptive modal filter (Sec. 3.3) against its definition.

The normalised index and the tail fraction are checked against brute-force loops over the
coefficients; the transfer function, the amplitude ramp and its relaxation against closed forms.
"""
import math

import numpy as np

import synth
from oracle.filter import (FilterConfig, apply, normalized_index, relaxed_amplitude, tail_fraction,
                           target_amplitude, transfer)
from oracle.grid import Grid


def _brute_zeta(g):
    out = {}
    for m in range(g.M):
        for n in range(m, g.nrc):
            for kk in range(g.nz):
                k = kk if 2 * kk < g.nz else kk - g.nz
                out[(m, n, kk)] = max(n / g.nrc, m / g.M, abs(k) / g.nzc)
    return out


def test_normalized_index_brute_force():
    for args in ((5, 6, 4), (7, 10, 1), (6, 8, 6)):
        g = Grid(*args, 1.0)
        z = normalized_index(g)
        ref = _brute_zeta(g)
        for (m, n, kk), v in ref.items():
            assert z[m, n, kk] == v
        mask = np.zeros(z.shape, bool)
        for (m, n, kk) in ref:
            mask[m, n, kk] = True
        assert np.all(z[~mask] == -1.0)


def test_tail_fraction_brute_force():
    g = Grid(9, 12, 8, 1.0)
    cfg = FilterConfig(zeta_c=0.5)
    S = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=4, a=0.95, b=0.95, c=0.95)
    tail = total = 0.0
    for (m, n, kk), zeta in _brute_zeta(g).items():
        e = abs(S[m, n, kk]) ** 2
        total += e
        if zeta > cfg.zeta_c:
            tail += e
    assert abs(tail_fraction(S, g, cfg) - tail / total) < 1e-14
    assert tail_fraction(np.zeros_like(S), g, cfg) == 0.0


def test_amplitude_ramp_and_relaxation():
    cfg = FilterConfig()
    assert target_amplitude(0.0, cfg) == 0.0
    assert target_amplitude(cfg.tau, cfg) == 0.0
    assert abs(target_amplitude(1.5 * cfg.tau, cfg) - cfg.eps_max / 2) < 1e-12
    assert target_amplitude(2 * cfg.tau, cfg) == cfg.eps_max
    assert target_amplitude(0.9, cfg) == cfg.eps_max
    # from eps = 0 at a fixed saturating fraction: eps_j = eps_max (1 - (1 - r)^j)
    eps = 0.0
    for j in range(1, 40):
        eps = relaxed_amplitude(eps, 0.5, cfg)
        assert abs(eps - cfg.eps_max * (1 - (1 - cfg.relax) ** j)) < 1e-12
    # and back down once the tail is gone: eps_j = eps_0 (1 - r)^j
    e0 = eps
    for j in range(1, 10):
        eps = relaxed_amplitude(eps, 0.0, cfg)
        assert abs(eps - e0 * (1 - cfg.relax) ** j) < 1e-12


def test_transfer_closed_forms():
    cfg = FilterConfig()
    z = np.linspace(0, 1, 301)
    s = transfer(z, cfg.eps_max, cfg)
    assert np.all(s[z <= cfg.zeta_c] == 1.0)
    assert abs(transfer(np.array([1.0]), cfg.eps_max, cfg)[0] - math.exp(-36.0)) < 1e-30
    mid = cfg.zeta_c + 0.5 * (1 - cfg.zeta_c)
    assert abs(transfer(np.array([mid]), 10.0, cfg)[0] - math.exp(-10.0 / 256)) < 1e-15
    assert np.all(np.diff(s) <= 0)
    assert np.all(transfer(z, 0.0, cfg) == 1.0)


def test_apply_inactive_below_target_and_untouched_below_cutoff():
    g = Grid(24, 16, 12, 1.0)
    cfg = FilterConfig()
    smooth = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=5, a=0.5, b=0.5, c=0.5)
    assert tail_fraction(smooth, g, cfg) < cfg.tau
    out, eps, f = apply(smooth, g, cfg, 0.0)
    assert eps == 0.0 and np.array_equal(out, smooth)
    # a flat spectrum has most of its energy above the cutoff: the filter acts above it only
    flat = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=6, a=1.0, b=1.0, c=1.0)
    f0 = tail_fraction(flat, g, cfg)
    assert f0 > 2 * cfg.tau
    out, eps, f = apply(flat, g, cfg, 20.0)
    assert f == f0 and abs(eps - (20.0 + cfg.relax * (cfg.eps_max - 20.0))) < 1e-12
    zeta = normalized_index(g)
    below = zeta <= cfg.zeta_c
    assert np.array_equal(out[below], flat[below])
    above = zeta > cfg.zeta_c
    ratio = np.abs(out[above]) / np.where(np.abs(flat[above]) > 0, np.abs(flat[above]), 1.0)
    expect = np.exp(-eps * ((zeta[above] - cfg.zeta_c) / (1 - cfg.zeta_c)) ** 8)
    nz = np.abs(flat[above]) > 0
    assert np.allclose(ratio[nz], expect[nz], rtol=1e-14, atol=0)
