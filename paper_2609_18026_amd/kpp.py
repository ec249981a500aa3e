"""The Fisher-KPP front of Sec. 5.2 (Example 2) on one GPU.

u_t = D grad^2 u + gamma u (1 - u) (Eq. kpp) on the unbounded plane with D = 1, gamma = 1/4 (planar
front speed 2 sqrt(D gamma) = 1), seeded by the axisymmetric Gaussian u(r, 0) = A exp(-r^2 / (2 sigma^2)),
sigma = 1.  Diffusion is implicit and the reaction explicit: the Richardson start-up and AB-CN loop
of Sec. 3.3 in mlg_scalar_advance (L = D grad^2 from mlg_step_setup, the reaction from
mlg_rhs_scalar with MLG_RHS_KPP).  Two measurements, as in the paper:
* the linear stage (A = 1e-6): the relative weighted L2 error against the closed form of
  Eq. kpp-linear at t_end (area quadrature over the collocation nodes);
* the front: R(t), the largest radius at which the azimuthal mean of u exceeds one half (the m = 0
  harmonic, evaluated at any radius by mlg_eval_harmonic, bracketed on a radial scan and refined by
  multisection), and the speed dR/dt against the log-corrected law c* - (N + 2) / (2 lambda* t).

Every step runs in the library's kernels; this module sequences the calls, locates the crossing
and fits.

    python -m paper_2609_18026_amd.kpp --nr 768 --ell 32 --t-end 80
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import asdict, dataclass

import numpy as np


@dataclass
class KppSpec:
    nr: int = 768
    nphi: int = 4           # the seed is axisymmetric: only m = 0 is excited
    ell: float = 32.0
    D: float = 1.0
    gamma: float = 0.25
    A: float = 1.0
    sigma: float = 1.0
    dt: float = 1e-2
    t_end: float = 80.0
    sample_every: float = 1.0
    r_scan: float = 0.0     # radial scan range of the front search (0: 1.5 t_end + 20)


def _front(plan, spec_u, r_max, torch, level=0.5, h=0.25):
    """Largest r with the m = 0 mean above 'level' (nan if none): scan, then multisection."""
    r = torch.arange(0.0, r_max + h, h, dtype=torch.float64, device="cuda")
    f = plan.eval_harmonic(spec_u, 0, 0, r).real.cpu().numpy()
    above = np.nonzero(f > level)[0]
    if above.size == 0:
        return float("nan")
    i = int(above[-1])
    if i + 1 >= f.size:
        return float(r[-1])
    a, b = i * h, (i + 1) * h
    for _ in range(8):                      # 32 intervals per pass: 32^8 ~ 1e12 shrink
        rr = torch.linspace(a, b, 33, dtype=torch.float64, device="cuda")
        v = plan.eval_harmonic(spec_u, 0, 0, rr).real.cpu().numpy()
        j = int(np.nonzero(v > level)[0][-1])
        a, b = float(rr[j]), float(rr[j + 1])
    return 0.5 * (a + b)


def run(spec: KppSpec, log=None) -> dict:
    import torch

    from .binding import MLG_RHS_KPP, Plan

    plan = Plan(spec.nr, spec.nphi, 1, spec.ell, dealias=1)
    plan.step_setup(spec.D, 0.0, 8, spec.dt)
    x, w, r = plan.nodes()
    u0 = spec.A * np.exp(-r ** 2 / (2 * spec.sigma ** 2))
    phys = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(u0[None, :, None], (1, spec.nr, spec.nphi)))).cuda()
    s = plan.empty_spec()
    plan.forward(phys, s)
    hist = plan.empty_spec()
    every = max(1, int(round(spec.sample_every / spec.dt)))
    nsteps = int(round(spec.t_end / spec.dt))
    r_max = spec.r_scan if spec.r_scan > 0 else 1.5 * spec.t_end + 20.0
    times, radii = [0.0], [_front(plan, s, r_max, torch)]
    done, tmp = 0, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < nsteps:
        n = min(every, nsteps - done)
        tmp = plan.advance_scalar(MLG_RHS_KPP, spec.gamma, s, hist, n, start=1 if done == 0 else 0, tmp=tmp)
        done += n
        times.append(done * spec.dt)
        radii.append(_front(plan, s, r_max, torch))
        if log and len(times) % 20 == 0:
            log(f"kpp: t = {times[-1]:.2f}, R = {radii[-1]:.6f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t = np.array(times)
    R = np.array(radii)
    # the linear stage against Eq. kpp-linear (meaningful while u << 1)
    plan.backward(s, phys)
    u = phys.cpu().numpy()
    s2 = spec.sigma ** 2 + 2 * spec.D * t[-1]
    uex = spec.A * spec.sigma ** 2 / s2 * math.exp(spec.gamma * t[-1]) * np.exp(-r ** 2 / (2 * s2))
    W = (w * spec.ell ** 2 / (1 - x) ** 2)[None, :, None]
    uexg = np.broadcast_to(uex[None, :, None], u.shape)
    lin_err = float(np.sqrt((W * (u - uexg) ** 2).sum() / (W * uexg ** 2).sum()))
    out = {"spec": asdict(spec), "steps": done, "wall_s": round(wall, 3),
           "ms_per_step_including_samples": round(wall / max(done, 1) * 1e3, 4),
           "t": t.tolist(), "R": R.tolist(), "linear_rel_err": lin_err}
    cstar = 2 * math.sqrt(spec.D * spec.gamma)
    lam = math.sqrt(spec.gamma / spec.D)
    for tt in (32.0, 80.0):
        k = int(np.argmin(abs(t - tt)))
        if abs(t[k] - tt) > 1e-9 or k < 2:
            continue
        if k < len(t) - 1:
            speed = (R[k + 1] - R[k - 1]) / (t[k + 1] - t[k - 1])
        else:  # one-sided, second order
            speed = (3 * R[k] - 4 * R[k - 1] + R[k - 2]) / (t[k] - t[k - 2])
        out[f"R_{int(tt)}"] = float(R[k])
        out[f"speed_{int(tt)}"] = float(speed)
        # log-corrected law in N = 2 dimensions: dR/dt = c* - (N + 2) / (2 lambda* t)
        out[f"speed_theory_{int(tt)}"] = cstar - 4.0 / (2.0 * lam * tt)
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    d = KppSpec()
    for k, v in asdict(d).items():
        ap.add_argument("--" + k.replace("_", "-"), type=type(v), default=v)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    spec = KppSpec(**{k: getattr(args, k) for k in asdict(d)})
    res = run(spec, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    print(json.dumps({k: v for k, v in res.items() if k not in ("t", "R")}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
