"""GPU parity of the axial modal kinetic energy (mlg_tp_energy): the diagnostic from which Sec. 5.3
reads the Crow growth rate.  Against the oracle's energy of the same seeded spectra (1e-12
normwise over the axial slots), and against the closed form of a Gaussian stream function
(psi = exp(-r^2): E_0 = pi L_z / 2)."""
import math

import numpy as np
import pytest

import synth
from helpers import rel, to_lib
from oracle.diagnostics import axial_modal_energy
from oracle.grid import Grid
from oracle.rhs import VecTables
from oracle.transform import Tables, forward

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [
    # nr, nphi, nz, ell, lz
    (24, 12, 8, 0.9, 3.0),
    (25, 12, 8, 0.8, 3.0),       # odd N_r: unfolded synthesis
    (32, 16, 1, 1.0, 2 * np.pi),  # 2D
    (48, 32, 32, 4.0, 34.4),      # the counter-rotating pair's map scale and axial period
    (16, 256, 256, 1.0, 8.6),     # 256-point kernels
]


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_18026_amd import Plan
    return Plan


@pytest.mark.parametrize("case", CASES)
def test_energy_parity(case):
    Plan = _gpu()
    nr, nphi, nz, ell, lz = case
    print("energy parity", case, flush=True)
    g = Grid(nr, nphi, nz, ell, lz=lz)
    vt = VecTables(g)
    psi = synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=7, a=0.85, b=0.8, c=0.8)
    chi = 0.3 * synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=8, a=0.85, b=0.8, c=0.8)
    want = axial_modal_energy(psi, chi, g, vt)
    plan = Plan(nr, nphi, nz, ell, lz, dealias=1)
    P = torch.from_numpy(to_lib(psi)).cuda()
    C = torch.from_numpy(to_lib(chi)).cuda()
    got = plan.energy(P, C).cpu().numpy()
    err = rel(got, want)
    print("  rel", err, flush=True)
    assert err < 1e-12, err


def test_energy_of_a_gaussian_stream_function():
    Plan = _gpu()
    nr, nphi, nz, ell, lz = 40, 8, 4, 1.0, 3.0
    plan = Plan(nr, nphi, nz, ell, lz, dealias=1)
    g = Grid(nr, nphi, nz, ell, lz=lz)
    f = np.exp(-g.r[None, :, None] ** 2) * np.ones((nz, nr, nphi))
    phys = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    psi = plan.empty_spec()
    plan.forward(phys, psi)
    E = plan.energy(psi, torch.zeros_like(psi)).cpu().numpy()
    assert abs(E[0] - 0.5 * lz * math.pi) < 1e-9, E[0]
    assert np.all(np.abs(E[1:]) < 1e-12)
