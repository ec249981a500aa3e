"""Co-rotating q-vortex pair of Sec. 5.3 (Example 3): the enstrophy ladder at t = 10.

Two parallel q-vortices (V_phi = (1 - e^{-rho^2}) / rho, V_z = e^{-rho^2} / q, circulation 2 pi each)
at (x, y) = (+-b/2, 0) with b = 4, q = 1, a uniform axial background U_z = -0.5, ell = 4, L_z = 2 pi
and nu = 1e-4 (Gamma / nu = 6.3e4), nu_h = 5e-7 with p = 8, advanced by the Richardson start-up and
AB-CN loop of mlg_tp_advance.  The pair has a net circulation 4 pi and a net axial volume flux
2 pi / q, so its potentials carry logarithmic proxies (Eq. logproxy, mlg_set_log_proxy): with the
stream function of one vortex -(1/2) Ein(rho^2) (Ein(s) = int_0^s (1 - e^{-t}) / t dt) and
chi = psi / (2 q),
    c_psi = -1,  c_chi = -1 / (2 q),
    psi~ = ln(r^2 + ell^2) - (1/2) sum_i Ein(rho_i^2) + gamma_E,   chi~ = psi~ / (2 q)
(the regular parts, which vanish as r -> infinity).  The enstrophy (1/2) int |omega|^2 dV comes from
mlg_tp_enstrophy.

    python -m paper_2609_18026_amd.qvortex --nr 128 --nphi 64 --nz 64 --dt 5e-3
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import asdict, dataclass

import numpy as np

EULER_GAMMA = 0.57721566490153286060651209008240243


@dataclass
class QVortexSpec:
    nr: int = 128
    nphi: int = 64
    nz: int = 64
    ell: float = 4.0
    b: float = 4.0
    q: float = 1.0
    uz: float = -0.5
    lz: float = 2 * math.pi
    nu: float = 1e-4
    nu_h: float = 5e-7        # the paper's hyperviscosity for this pair (p = 8); without it the
                              # margin-free runs gain spurious enstrophy after t ~ 4
    p: int = 8
    dt: float = 5e-3
    t_end: float = 10.0
    sample_every: float = 0.5


def run(spec: QVortexSpec, log=None) -> dict:
    import torch

    import synth
    from .binding import Plan

    plan = Plan(spec.nr, spec.nphi, spec.nz, spec.ell, spec.lz, dealias=1)
    plan.step_setup(spec.nu, spec.nu_h, spec.p, spec.dt)
    c_psi, c_chi = -1.0, -1.0 / (2 * spec.q)
    plan.set_log_proxy(c_psi, c_chi)
    x, w, r = plan.nodes()
    phi = 2 * np.pi * np.arange(spec.nphi) / spec.nphi
    R, PH = np.meshgrid(r, phi, indexing="ij")
    X, Y = R * np.cos(PH), R * np.sin(PH)
    rho1 = (X - spec.b / 2) ** 2 + Y ** 2
    rho2 = (X + spec.b / 2) ** 2 + Y ** 2
    psit = np.log(R ** 2 + spec.ell ** 2) - 0.5 * (synth._ein(rho1) + synth._ein(rho2)) + EULER_GAMMA
    shape = (spec.nz, spec.nr, spec.nphi)
    psi, chi = plan.empty_spec(), plan.empty_spec()
    plan.forward(torch.from_numpy(np.ascontiguousarray(np.broadcast_to(psit[None], shape))).cuda(), psi)
    plan.forward(torch.from_numpy(np.ascontiguousarray(np.broadcast_to(psit[None] / (2 * spec.q), shape))).cuda(), chi)
    hp, hc = plan.empty_spec(), plan.empty_spec()
    U = (0.0, 0.0, spec.uz)
    every = max(1, int(round(spec.sample_every / spec.dt)))
    nsteps = int(round(spec.t_end / spec.dt))
    times, Z = [0.0], [float(plan.enstrophy(psi, chi).sum())]
    done, tmp = 0, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < nsteps:
        n = min(every, nsteps - done)
        tmp = plan.advance(psi, chi, hp, hc, n, start=1 if done == 0 else 0, U=U, tmp=tmp)
        done += n
        times.append(done * spec.dt)
        Z.append(float(plan.enstrophy(psi, chi).sum()))
        if not math.isfinite(Z[-1]):
            break
        if log and len(times) % 4 == 0:
            log(f"qvortex: t = {times[-1]:.2f}, enstrophy = {Z[-1]:.7f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"spec": asdict(spec), "steps": done, "wall_s": round(wall, 3),
            "ms_per_step_including_samples": round(wall / max(done, 1) * 1e3, 4),
            "t": times, "enstrophy": Z, "enstrophy_t_end": Z[-1], "c_psi": c_psi, "c_chi": c_chi}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    d = QVortexSpec()
    for k, v in asdict(d).items():
        ap.add_argument("--" + k.replace("_", "-"), type=type(v), default=v)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    spec = QVortexSpec(**{k: getattr(args, k) for k in asdict(d)})
    res = run(spec, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    print(json.dumps({k: v for k, v in res.items() if k not in ("t", "enstrophy")}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
