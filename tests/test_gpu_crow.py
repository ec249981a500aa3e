"""The linear stage of the Crow instability on the GPU (Sec. 5.3, Results and validation).

The paper's counter-rotating pair (Gamma = +-2 pi, a = 0.5, b = 4, L_z = 8.6 b, seed 0.002 b,
nu = 1e-4, nu_h = 5e-8, p = 8) advanced in the moving frame by the AB-CN loop of mlg_tp_advance on a
96 x 64 x 32 grid; the growth rate alpha = (pi b^2 / Gamma) d ln E_1 / dt of the seeded fundamental,
fitted over t = 28..38 from mlg_tp_energy, is compared with the oracle's evaluation of Crow's
dispersion relation at beta = 0.7306, a / b = 0.125 (0.798; the paper measures 0.8197, 2.7% above
it).  The measured rate is the same to three digits on grids up to 160 x 128 x 48 and for time steps
from 1e-3 to 5e-3; the bound here (4%) is wider than that spread and than the paper's own gap.
"""
import math

import pytest

from oracle import crow as crow_theory

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.timeout(300)
def test_crow_growth_rate():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_18026_amd.crow import CrowSpec, run
    spec = CrowSpec(nr=96, nphi=64, nz=32, dt=5e-3, t_end=38.0)
    print("crow run", spec, flush=True)
    res = run(spec)
    assert res["stable"], "the run became non-finite"
    alpha = res["alpha_fit_28_38"]
    theory = crow_theory.growth_rate(2 * math.pi / spec.lz_over_b, spec.a / spec.b * crow_theory.lamb_oseen_cutoff(1.0))
    print("alpha", alpha, "theory", theory, "ms/step", res["ms_per_step"], flush=True)
    assert abs(alpha - theory) < 0.04 * theory, (alpha, theory)
    # the energy of the axisymmetric-in-z base flow decays slowly (diffusion only)
    assert res["E0"][-1] < res["E0"][0] and res["E0"][-1] > 0.95 * res["E0"][0]


@pytest.mark.timeout(300)
def test_crow_to_t60_with_radial_margin():
    """Without a radial margin every grid breaks down after t ~ 27..52 (radial aliasing of the
    quadratic products into the retained degrees); with 96 degrees on 128 nodes the run reaches
    t = 60, the k = 2 energy stays the quadratic harmonic of the fundamental, and the rate over the
    paper's window t = 33..60 stays within 4% of the relation."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import numpy as np
    from paper_2609_18026_amd.crow import CrowSpec, run
    spec = CrowSpec(nr=128, nrc=96, nphi=64, nz=32, dt=5e-3, t_end=60.0)
    print("crow run with a radial margin", spec, flush=True)
    res = run(spec)
    assert res["stable"] and res["steps"] == 12000
    t, E1, E2 = np.array(res["t"]), np.array(res["E1"]), np.array(res["E2"])
    ratio = E2 / E1 ** 2
    r30 = ratio[np.argmin(abs(t - 30.0))]
    sel = (t >= 30.0) & (t <= 55.0)
    assert np.all(np.abs(ratio[sel] / r30 - 1.0) < 0.1), ratio[sel] / r30
    theory = crow_theory.growth_rate(2 * math.pi / spec.lz_over_b, spec.a / spec.b * crow_theory.lamb_oseen_cutoff(1.0))
    alpha = res["alpha_fit_33_60"]
    print("alpha 33..60", alpha, "33..50", res["alpha_fit_33_50"], "theory", theory, flush=True)
    assert abs(alpha - theory) < 0.04 * theory, (alpha, theory)
