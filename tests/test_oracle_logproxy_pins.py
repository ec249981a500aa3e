"""Pins of the oracle's logarithmic-proxy pieces (Eq. logproxy, Eq. tp) and of its enstrophy.

The image g of grad_h^2 Lambda is checked against the closed form 4 ell^2 / (r^2 + ell^2)^2 and the
truncated Laplacian applied to it against the closed-form Laplacian of that function; a single
columnar q-vortex on the axis (V_phi = (1 - e^{-r^2}) / r, V_z = e^{-r^2} / q), written as regular
potentials plus proxy amplitudes, synthesises its exact velocity and vorticity, is a steady Euler
solution (the projected nonlinear term vanishes), and has the closed-form enstrophy
(1/2)(2 pi + pi / q^2) L_z.
"""
import numpy as np

import synth
from oracle.basis import laplacian_matrix, pbar
from oracle.grid import Grid
from oracle.logproxy import (enstrophy, laplacian_image, proxy_fields, proxy_forcing, rhs_tp_log,
                             synthesize_log)
from oracle.rhs import VecTables
from oracle.transform import Tables, forward

EULER = 0.57721566490153286060651209008240243


def _eval0(coef, g, x):
    return coef @ pbar(0, g.nrc, x).astype(np.float64)


def test_laplacian_image_and_its_laplacian():
    g = Grid(24, 4, 1, 1.7)
    gv = laplacian_image(g.nrc, g.ell)
    assert np.count_nonzero(gv) == 3
    x = np.linspace(-0.999, 0.999, 41)
    r = g.ell * np.sqrt((1 + x) / (1 - x))
    assert np.allclose(_eval0(gv, g, x), 4 * g.ell ** 2 / (r ** 2 + g.ell ** 2) ** 2, rtol=1e-13, atol=1e-15)
    lap = laplacian_matrix(0, g.nrc, g.ell) @ gv
    exact = g.ell ** 2 * (64 * r ** 2 - 32 * g.ell ** 2) / (r ** 2 + g.ell ** 2) ** 4
    assert np.allclose(_eval0(lap, g, x), exact, rtol=1e-11, atol=1e-13)
    assert np.allclose(proxy_forcing(g, 0.3), 0.3 * gv, rtol=0, atol=0)
    f = proxy_forcing(g, 0.3, 1e-3, 4)
    assert np.allclose(f, 0.3 * gv + 1e-3 * (-laplacian_matrix(0, g.nrc, g.ell)) @ gv, rtol=1e-15)


def _axial_q_vortex(g, q):
    """Regular parts and amplitudes of the columnar q-vortex on the axis."""
    t = Tables(g)
    r = g.r
    ein = synth._ein(r ** 2)
    psit = 0.5 * (np.log(r ** 2 + g.ell ** 2) - ein + EULER)     # -> 0 as r -> infinity
    chit = psit / (2 * q)
    shape = (g.nz, g.nr, g.nphi)
    P = forward(np.broadcast_to(psit[None, :, None], shape).copy(), g, t)
    C = forward(np.broadcast_to(chit[None, :, None], shape).copy(), g, t)
    return P, C, -0.5, -0.25 / q


def test_axial_q_vortex_fields_steadiness_and_enstrophy():
    q = 1.3
    g = Grid(48, 8, 4, 2.0, lz=2 * np.pi)
    vt = VecTables(g)
    P, C, cp, cc = _axial_q_vortex(g, q)
    u, w = synthesize_log(P, C, g, vt, cp, cc)
    r = g.r[None, :, None]
    e = np.exp(-r ** 2)
    assert np.abs(u[0]).max() < 1e-10 and np.abs(w[0]).max() < 1e-10
    assert np.abs(u[1] - (1 - e) / r).max() < 1e-9
    assert np.abs(u[2] - e / q).max() < 1e-9
    assert np.abs(w[1] - 2 * r * e / q).max() < 1e-9
    assert np.abs(w[2] - 2 * e).max() < 1e-9
    # a columnar vortex is a steady solution: its nonlinear term is a pure gradient
    pn, cn = rhs_tp_log(P, C, g, vt, U=(0.0, 0.0, 0.0), dealias=False, c_psi=cp, c_chi=cc)
    assert np.abs(pn).max() < 1e-9 and np.abs(cn).max() < 1e-9
    Z = enstrophy(P, C, g, vt, cp, cc)
    assert abs(Z / (0.5 * (2 * np.pi + np.pi / q ** 2) * g.lz) - 1) < 1e-9
    # the proxy parts alone: closed forms
    up, uz, wp, wz = proxy_fields(np.array([0.0, 1.0, 3.0]), 2.0, 1.0, 1.0)
    assert np.allclose(up, [0.0, -2 / 5, -6 / 13]) and np.allclose(wz, uz) and wp[0] == 0.0


def test_viscous_q_vortex_decay_with_proxy_forcing():
    """With the proxy forcing, the AB-CN loop reproduces the viscous columnar q-vortex: the nonlinear
    term vanishes and the profiles diffuse as V_phi = (1 - e^{-r^2/s}) / r, V_z = e^{-r^2/s} / (q s),
    w_z = (2 / s) e^{-r^2/s}, s = 1 + 4 nu t (to the O(dt^2) error of the scheme)."""
    from oracle import timestep as ts
    from oracle.logproxy import add_forcing
    q, nu, dt, n = 1.0, 0.05, 0.01, 100
    g = Grid(40, 8, 2, 2.0, lz=2 * np.pi)
    vt = VecTables(g)
    P, C, cp, cc = _axial_q_vortex(g, q)
    diss = ts.Dissipation(g, nu)
    f = proxy_forcing(g, nu)

    def A(p, c):
        pn, cn = rhs_tp_log(p, c, g, vt, dealias=False, c_psi=cp, c_chi=cc)
        return add_forcing(pn, f, cp), add_forcing(cn, f, cc)

    A0 = A(P, C)
    full = [ts.fe_be_step(s, dt, diss, lambda _s, a=a: a) for s, a in zip((P, C), A0)]
    h1 = [ts.fe_be_step(s, dt / 2, diss, lambda _s, a=a: a) for s, a in zip((P, C), A0)]
    Ah = A(*h1)
    h2 = [ts.fe_be_step(s, dt / 2, diss, lambda _s, a=a: a) for s, a in zip(h1, Ah)]
    S = [2 * a - b for a, b in zip(h2, full)]
    prev = A0
    for _ in range(n - 1):
        now = A(*S)
        S = [ts.abcn_step(s, an, ap, dt, diss) for s, an, ap in zip(S, now, prev)]
        prev = now
    u, w = synthesize_log(S[0], S[1], g, vt, cp, cc)
    s = 1 + 4 * nu * n * dt
    r = g.r[None, :, None]
    e = np.exp(-r ** 2 / s)
    assert np.abs(w[2] - 2 / s * e).max() < 1e-6
    assert np.abs(u[1] - (1 - e) / r).max() < 1e-6
    assert np.abs(u[2] - e / (q * s)).max() < 1e-6
