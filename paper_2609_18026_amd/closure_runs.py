"""Fine / coarse run pairs for the learned closure, driven entirely through the C ABI.

A fine run advances (psi, chi) with mlg_tp_advance; at every snapshot the fine nonlinear term
is truncated to the coarse grid (mlg_truncate) and compared with the coarse term of the
truncated state, giving one (features, target) row per (m, k) column:
    features = F(T s_f),  target = T A_f(s_f) - A_c(T s_f).
The network is trained with mlg_closure_train_step on index batches supplied by the caller, and
judged a priori by the residual ratio
    gain = ||T A_f - (A_c + C)|| / ||T A_f - A_c||
over held-out snapshots, and a posteriori by coarse roll-outs with and without the closure
against the truncated fine run.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .binding import Closure, Plan


@dataclass
class RunSpec:
    """Dissipation and time step shared by the fine and coarse runs (Eq. dissipation, Eq. abcn)."""
    nu: float = 1e-4
    nu_h: float = 0.0
    p: int = 8
    dt: float = 1e-3
    U: tuple = (0.0, 1.0, 0.0)


@dataclass
class Snapshots:
    """Per-snapshot device tensors on the coarse grid."""
    psi: list = field(default_factory=list)    # T s_f
    chi: list = field(default_factory=list)
    ref_psi: list = field(default_factory=list)  # T A_f(s_f)
    ref_chi: list = field(default_factory=list)


def setup(plan: Plan, spec: RunSpec) -> None:
    plan.step_setup(spec.nu, spec.nu_h, spec.p, spec.dt)


def fine_run(fine: Plan, coarse: Plan, spec: RunSpec, psi0, chi0, nsnap: int, every: int) -> Snapshots:
    """Advance the fine state nsnap * every steps; keep T s_f and T A_f(s_f) every 'every' steps
    (first snapshot at t = 0)."""
    import torch
    psi, chi = psi0.clone(), chi0.clone()
    hp, hc = fine.empty_spec(), fine.empty_spec()
    Ap, Ac = fine.empty_spec(), fine.empty_spec()
    tmp = torch.empty(6 * fine.layout.spec_elems, dtype=torch.complex128, device=psi.device)
    out = Snapshots()
    for s in range(nsnap):
        if s > 0:
            fine.advance(psi, chi, hp, hc, every, start=(s == 1), U=spec.U, tmp=tmp)
        fine.rhs_tp(psi, chi, Ap, Ac, U=spec.U)
        tp, tc, rp, rc = (coarse.empty_spec() for _ in range(4))
        fine.truncate_to(coarse, psi, tp)
        fine.truncate_to(coarse, chi, tc)
        fine.truncate_to(coarse, Ap, rp)
        fine.truncate_to(coarse, Ac, rc)
        out.psi.append(tp)
        out.chi.append(tc)
        out.ref_psi.append(rp)
        out.ref_chi.append(rc)
    return out


def dataset(coarse: Plan, closure: Closure, snaps: Snapshots, spec: RunSpec):
    """Raw features [n * ncols, 258] and targets [n * ncols, 256] (device float32)."""
    import torch
    n, nc = len(snaps.psi), closure.ncols
    dev = snaps.psi[0].device
    X = torch.empty((n * nc, 258), dtype=torch.float32, device=dev)
    Y = torch.empty((n * nc, 256), dtype=torch.float32, device=dev)
    Np, Nc = coarse.empty_spec(), coarse.empty_spec()
    for i in range(n):
        coarse.rhs_tp(snaps.psi[i], snaps.chi[i], Np, Nc, U=spec.U)
        closure.features(snaps.psi[i], snaps.chi[i], X[i * nc:(i + 1) * nc])
        closure.targets(snaps.ref_psi[i], snaps.ref_chi[i], Np, Nc, Y[i * nc:(i + 1) * nc])
    return X, Y


def fit(closure: Closure, X, Y, batches, lr: float, lr_final: float | None = None, report_every: int = 0):
    """One Adam step per row of 'batches' (device int32 [steps, nb]); returns the recorded losses.

    The learning rate decays geometrically from lr to lr_final (if given)."""
    steps, nb = batches.shape
    losses = []
    for s in range(steps):
        rate = lr if lr_final is None else lr * (lr_final / lr) ** (s / max(1, steps - 1))
        want = report_every > 0 and (s % report_every == 0 or s == steps - 1)
        loss = closure.train_step(X, Y, batches[s], nb, rate, want_loss=want)
        if want:
            losses.append((s, loss))
    return losses


def a_priori(coarse: Plan, closure: Closure, snaps: Snapshots, spec: RunSpec):
    """Per snapshot: (||T A_f - A_c||, ||T A_f - (A_c + C)||, fallback flag)."""
    import torch
    out = []
    Np, Nc = coarse.empty_spec(), coarse.empty_spec()
    for i in range(len(snaps.psi)):
        coarse.rhs_tp(snaps.psi[i], snaps.chi[i], Np, Nc, U=spec.U)
        before = torch.sqrt(torch.sum(torch.abs(snaps.ref_psi[i] - Np) ** 2) +
                            torch.sum(torch.abs(snaps.ref_chi[i] - Nc) ** 2)).item()
        fb = closure.infer(snaps.psi[i], snaps.chi[i], Np, Nc, want_flag=True)
        after = torch.sqrt(torch.sum(torch.abs(snaps.ref_psi[i] - Np) ** 2) +
                           torch.sum(torch.abs(snaps.ref_chi[i] - Nc) ** 2)).item()
        out.append((before, after, fb))
    return out


def rollout(coarse: Plan, spec: RunSpec, psi0, chi0, nsnap: int, every: int, closure: Closure | None = None):
    """Coarse roll-out from T s_f(0); returns the states at the snapshot times."""
    import torch
    psi, chi = psi0.clone(), chi0.clone()
    hp, hc = coarse.empty_spec(), coarse.empty_spec()
    tmp = torch.empty(6 * coarse.layout.spec_elems, dtype=torch.complex128, device=psi.device)
    states = [(psi.clone(), chi.clone())]
    for s in range(1, nsnap):
        coarse.advance(psi, chi, hp, hc, every, start=(s == 1), U=spec.U, closure=closure, tmp=tmp)
        states.append((psi.clone(), chi.clone()))
    return states
