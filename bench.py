"""Benchmark: toroidal-poloidal nonlinear RHS at N_r = N_phi = N_z = 256 on one MI355X.

One step = one mlg_rhs_tp call on the resident 256^3 vortex-pair state (FP64): radial
synthesis of u and omega, inverse z and phi FFTs, (U + u) x omega, forward FFTs,
Galerkin projection and the per-(m, k) elliptic solves (the whole transform round trip
plus the nonlinear term).  value = N_r N_phi N_z / (seconds per step) / 1e9 [GDOF/s].

Further sections of the same JSON line: per-kernel times and roofline fractions, the transform
pair, the FP32 and split-bfloat16 RHS (float data) with their bytes and errors, the batched 2D launch, whole AB-CN time steps, the
learned closure (training / inference cost, held-out gain, roll-outs) and the oracle timed on
the host.  --gpus N with N > 1 exits: the benchmark runs on exactly one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spectral transform+RHS GDOF/s at 256^3 on 1 MI355X; rel. error vs FP64 oracle"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# vortex pair (Sec. 5.3): Gamma = +-2 pi, core radius 0.1, separation 1, displacement 0.01,
# axial period 8.6 (the Crow wavelength in units of the separation), moving frame U = (0, 1, 0)
PAIR = dict(gamma=2 * np.pi, a=0.1, b=1.0, delta=0.01, lz=8.6)
U_FRAME = (0.0, 1.0, 0.0)


# HBM traffic per RHS step of each kernel family from two rocprofv3 --pmc runs (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0: the factors of a plain 256 MiB copy) at 256^3; a record is used only while the
# kernel source hashes to the one that was measured (profiles/rhs_tp_256cubed_kernels.md).
_SUMMARY = "profiles/rhs_tp_256cubed_kernels.md"
MEASURED_TRAFFIC = {
    "synth_gemm": {"bytes": 570752743, "launches": 1, "n": 256,
                   "source": "paper_2609_18026_amd/csrc/gemm_fold.hip",
                   "sha256": "f4a0f702484fbf98751cd20659c2689655334ac4627dbb4ccb4332c7beeb5fcc",
                   "profile_avg_ms": 0.2729, "mfma_counter_flops": 11.77e9, "mfma_busy_pct": 59.1},
    "proj_gemm": {"bytes": 408833265, "launches": 1, "n": 256,
                  "source": "paper_2609_18026_amd/csrc/gemm_fold.hip",
                  "sha256": "f4a0f702484fbf98751cd20659c2689655334ac4627dbb4ccb4332c7beeb5fcc",
                  "profile_avg_ms": 0.2119, "mfma_counter_flops": 8.82e9, "mfma_busy_pct": 56.5},
    "phi_fft": {"bytes": 811893208, "launches": 1, "n": 256,
                "source": "paper_2609_18026_amd/csrc/fft256.hip",
                "sha256": "0af234d19557e3211f2e7bfc0a1f1dad41c5692ef4e35003d44cebef8e25ce03",
                "profile_avg_ms": 0.221},
    "z_fft": {"bytes": 913157899 + 452430330, "launches": 2, "n": 256,
              "source": "paper_2609_18026_amd/csrc/fft256.hip",
              "sha256": "0af234d19557e3211f2e7bfc0a1f1dad41c5692ef4e35003d44cebef8e25ce03"},
    "projection": {"bytes": 510715433, "launches": 1, "n": 256,
                   "source": "paper_2609_18026_amd/csrc/kernels.hip",
                   "sha256": "0c6f72ebed826dbc463c4d0594ca884358824ecb775e6435952dbab288e27a90",
                   "profile_avg_ms": 0.1415},
}


def measured_record(kernel, n):
    """The profiled record of a kernel family (profiles/rhs_tp_256cubed_kernels.md) while its source
    hashes to the one that was measured, else None."""
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
    if not rec or rec["n"] != n:
        return None
    try:
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
                return None
    except OSError:
        return None
    return rec


def measured_traffic(kernel, n, per_launch=True):
    """Measured HBM bytes of a kernel family (per launch, or per RHS step), or None when no record
    matches the current source."""
    rec = measured_record(kernel, n)
    if rec is None:
        return None
    return rec["bytes"] / rec["launches"] if per_launch else rec["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def active_columns(nphi, nz, M, nrc, dealias=True):
    """Orders and k slots the projection computes: m < mmax, |k| <= kmax (two-thirds mask)."""
    kmax = min(max(nz // 2, 1) - 1, nz // 2 - 1) if nz > 1 else 0
    mmax = min(M, nrc)
    if dealias:
        kmax = min(kmax, (nz - 1) // 3)
        mmax = min(mmax, (nphi - 1) // 3 + 1)
    nkact = 1 if nz == 1 else 2 * kmax + 1
    return mmax, nkact


def radial_folded(nr):
    """Even N_r: the library folds the radial products over the node symmetry (half the flops),
    unless MLG_RADIAL_FOLD=0 was set when the plan was created."""
    return nr % 2 == 0 and os.environ.get("MLG_RADIAL_FOLD", "1") != "0"


def kernel_work(nr, nphi, nz, M, nrc):
    """Algorithmic flops / HBM bytes per RHS step for each kernel family (FP64); with parity
    folding the radial products count half the flops and read half of each table.  Under the
    two-thirds mask (the RHS workload) the potentials enter through it: the synthesis covers the
    kept orders and axial slots, the inverse z transforms the kept orders (reading the kept slots,
    writing every z), the phi stage reads and writes the kept orders, and the forward z transforms
    write the kept slots only (the projection products read no others)."""
    mmax, nkact = active_columns(nphi, nz, M, nrc)
    mk = min(M, (nphi - 1) // 3 + 1)             # orders kept by the mask
    tau_k = sum(max(nrc - m, 0) for m in range(mk))
    tau_a = sum(max(nrc - m, 0) for m in range(mmax))
    tau = sum(max(nrc - m, 0) for m in range(M))
    kept = mk * nr * nz * 16                     # one harmonic field on the kept orders, complex
    f = 0.5 if radial_folded(nr) else 1.0
    w = {}
    w["synth_gemm"] = dict(flops=f * 7 * 2.0 * nr * tau_k * 2 * nkact,
                           bytes=f * 2 * tau_k * nr * 8 + 2 * tau_k * nkact * 16 + 6 * mk * nr * nkact * 16)
    w["proj_gemm"] = dict(flops=f * 5 * 2.0 * nr * tau_a * 2 * nkact,
                          bytes=f * 2 * tau_a * nr * 8 + 3 * mmax * nr * nkact * 16 + 3 * tau_a * nkact * 16)
    w["phi_fft"] = dict(flops=None, bytes=9 * kept)
    # forward: the three fields of the active orders, read whole, written on the kept slots only
    w["z_fft"] = dict(flops=None, bytes=6 * mk * nr * (nkact + nz) * 16 + 3 * mmax * nr * (nz + nkact) * 16)
    # the solves: sources, potentials (zeros outside the solved columns) and, like the radial
    # products' tables, their plan operators: the q-operator factors (l1, l2 and a pivot, 24 B per
    # solved entry) and 11 per-order Gram and factor tables (8 B per solved degree)
    w["projection"] = dict(flops=None, bytes=3 * tau_a * nkact * 16 + 2 * tau * nz * 16 + 24 * tau_a * nkact
                           + 11 * 8 * tau_a)
    return w


def build_state(plan, n, torch):
    import synth
    x, w, r = plan.nodes()
    phi = 2 * np.pi * np.arange(n) / n
    z = PAIR["lz"] * np.arange(n) / n
    psi = synth.vortex_pair_psi(r, phi, z, gamma=PAIR["gamma"], a=PAIR["a"], b=PAIR["b"],
                                delta=PAIR["delta"], lz=PAIR["lz"])
    phys = torch.from_numpy(psi).cuda()
    psi_hat = plan.empty_spec()
    plan.forward(phys, psi_hat)
    chi_hat = torch.zeros_like(psi_hat)
    torch.cuda.synchronize()
    return phys, psi_hat, chi_hat


def _host_cpu():
    """CPU model name and the number of cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return model, ncpu


def _timed(fn, warmup, reps):
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def sample_rhs_256(torch, plan, psi, n, npts=16, seed=11):
    """The library's RHS at n^3 with its taps, cut down to what a sampled oracle comparison needs:
    u, omega at npts seeded nodes (l, i, j), the full nodal N, the sources C, K, Zhat (packed) and
    the potentials (host copies).  The state is the headline vortex pair psi with a small geometric
    poloidal part chi = 1e-2 S (seed 9), as in the full-size parity test: with chi = 0 the nearly
    columnar pair has N_z ~ 0, and K and Zhat are then cancelling residuals whose normwise error
    measures rounding against a vanishing column rather than the path's accuracy."""
    import synth
    lay = plan.layout
    chi = torch.from_numpy(synth.to_packed(1e-2 * synth.geometric_spectrum(
        lay.M, lay.nrc, n, lay.nzc, seed=9, a=0.9, b=0.85, c=0.85))).to(psi.device)
    tp = plan.taps_buffer()
    po, co = plan.empty_spec(), plan.empty_spec()
    plan.rhs_tp(psi, chi, po, co, U=U_FRAME, taps=tp)
    torch.cuda.synchronize()
    pe = plan.layout.phys_elems
    r = np.random.default_rng(seed)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 3, n // 2, 0), (n // 2, n // 4, n // 2)]
    while len(pts) < npts:
        pts.append((int(r.integers(n)), int(r.integers(n)), int(r.integers(n))))
    idx = torch.tensor([(l * n + i) * n + j for l, i, j in pts], device=tp.device)
    uw = tp[:6 * pe].view(6, pe)[:, idx].cpu().numpy()
    N = tp[6 * pe:9 * pe].view(3, n, n, n).cpu().numpy()
    src = tp[9 * pe:].cpu().numpy().view(np.complex128).reshape(3, plan.tau, n)
    out = {"pts": pts, "uw": uw, "N": N, "src": src, "psi": psi.cpu().numpy(), "chi": chi.cpu().numpy(),
           "psi_n": po.cpu().numpy(), "chi_n": co.cpu().numpy(), "M": plan.layout.M, "nrc": plan.layout.nrc, "n": n}
    del tp, po, co
    return out


def parity_256_sampled(s256):
    """The library's 256^3 RHS stages against the oracle at sampled nodes and columns: u, omega
    from the (masked) potentials at the sampled nodes; N = (U + u) x omega there from the library's
    u, omega; the sources C, K, Zhat at 12 seeded active (m, k) columns (with (0, 0) and the highest
    kept order) from the library's nodal N."""
    import synth
    from oracle.grid import Grid
    from oracle.rhs import VecTables, apply_mask, dealias_mask, projection_sources_columns, synthesize_points
    n, M, nrc = s256["n"], s256["M"], s256["nrc"]
    g = Grid(n, n, n, 1.0, lz=PAIR["lz"])
    vt = VecTables(g)
    rel = lambda a, b: float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))
    P = synth.from_packed(s256["psi"].reshape(-1, n), M, nrc)
    C = synth.from_packed(s256["chi"].reshape(-1, n), M, nrc)
    pts = s256["pts"]
    ref_uw = synthesize_points(apply_mask(P, g), apply_mask(C, g), g, vt, pts)
    uw = s256["uw"]
    # the cross product at the sampled nodes from the library's u, omega (U Cartesian)
    cph = np.array([np.cos(g.phi[j]) for _, _, j in pts])
    sph = np.array([np.sin(g.phi[j]) for _, _, j in pts])
    U = U_FRAME
    ur, up, uz = uw[0] + U[0] * cph + U[1] * sph, uw[1] - U[0] * sph + U[1] * cph, uw[2] + U[2]
    ref_N = np.stack([up * uw[5] - uz * uw[4], uz * uw[3] - ur * uw[5], ur * uw[4] - up * uw[3]])
    Nl = s256["N"]
    got_N = np.stack([[Nl[f][l, i, j] for l, i, j in pts] for f in range(3)])
    src = [synth.from_packed(s256["src"][i], M, nrc) for i in range(3)]
    allowed = dealias_mask(g)
    nrm = np.where(allowed, np.linalg.norm(src[0], axis=1), -1.0)
    order = np.argsort(nrm, axis=None)[::-1]
    cols = [tuple(int(v) for v in np.unravel_index(o, nrm.shape)) for o in order[:6]]
    r = np.random.default_rng(6)
    cand = np.argwhere(allowed)
    for c in [(0, 0), (int(cand[:, 0].max()), 0)]:
        if c not in cols:
            cols.append(c)
    while len(cols) < 12:
        c = tuple(int(v) for v in cand[r.integers(len(cand))])
        if c not in cols:
            cols.append(c)
    pc = projection_sources_columns(Nl[0], Nl[1], Nl[2], g, vt, cols)
    srcerr = {}
    for i, name in enumerate(("C", "K", "Zhat")):
        srcerr[name] = rel(np.concatenate([src[i][m, :, kk] for m, kk in cols]),
                           np.concatenate([pc[c][i] for c in cols]))
    # the solves: backward error ||A x - b|| / (||A|| ||x|| + ||b||) of the library's potentials at the
    # columns against the library's sources, with the oracle's truncated Laplacian (Eq. del2h-entries)
    # and, at m = 0, its gauge row (Sec. 3.2: D psi_N = -C, (D - kappa^2) q = K, D chi_N = q)
    from oracle.basis import laplacian_matrix
    Po = synth.from_packed(s256["psi_n"].reshape(-1, n), M, nrc)
    Co = synth.from_packed(s256["chi_n"].reshape(-1, n), M, nrc)
    kap = g.kappa()
    worst = 0.0
    for m, kk in cols:
        D = laplacian_matrix(m, nrc, g.ell)
        Dg = D.copy()
        if m == 0:
            Dg[0, :] = np.sqrt((2 * np.arange(nrc) + 1) / 2.0)
        nA = np.linalg.norm(Dg, 2)
        b = -src[0][m, m:, kk].copy()
        q = -src[2][m, m:, kk] if kap[kk] == 0 else np.linalg.solve(D - kap[kk] ** 2 * np.eye(D.shape[0]), src[1][m, m:, kk])
        for x, rhs in ((Po[m, m:, kk], b), (Co[m, m:, kk], q.copy())):
            if m == 0:
                rhs[0] = 0
            worst = max(worst, float(np.linalg.norm(Dg @ x - rhs) / (nA * np.linalg.norm(x) + np.linalg.norm(rhs))))
    return {"workload": f"vortex pair psi with chi = 1e-2 x a geometric spectrum at {n}^3, FP64, sampled",
            "nodes": len(pts), "columns": [list(c) for c in cols],
            "rel_err_u_omega_at_nodes": rel(uw, ref_uw), "rel_err_N_at_nodes": rel(got_N, ref_N),
            "rel_err_sources_at_columns": srcerr, "solve_backward_error_at_columns": worst,
            "solve_backward_error_bound": 2 * nrc * float(np.finfo(np.float64).eps)}


def cpu_baseline(n_sample: int, gpu_small: dict):
    """The oracle timed on the host (1 warm-up, median of 5 unless stated): the headline workload's
    rhs_tp on a bounded sample (the vortex pair at n_sample^3) with all BLAS threads and with one, its
    growth with the grid (48^3 vs n_sample^3) and the 256^3 rate that growth implies, and the other
    workloads: the 32 x 16 x 1 scalar term and transform pair, the 128^3 vector RHS (median of 3) and
    the 64 batched 2D KPP terms (median of 3).  gpu_small: the library's outputs on the sampled and
    small workloads, compared here with the oracle's (the FP64 parity of the bench path)."""
    import synth
    from oracle.grid import Grid
    from oracle.rhs import VecTables, rhs_scalar, rhs_tp, synthesize
    from oracle.transform import Tables, backward, forward
    from threadpoolctl import threadpool_info, threadpool_limits
    model, ncpu = _host_cpu()
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])

    def pair_case(n):
        g = Grid(n, n, n, 1.0, lz=PAIR["lz"])
        psi = synth.vortex_pair_psi(g.r, g.phi, g.z, gamma=PAIR["gamma"], a=PAIR["a"], b=PAIR["b"],
                                    delta=PAIR["delta"], lz=PAIR["lz"])
        S = forward(psi, g, Tables(g))
        return g, S, VecTables(g)

    res = {"kind": "oracle", "unit": "GDOF/s", "cpu_model": model, "host_cpus": ncpu, "warmup": 1, "median_of": 5}
    g, S, vt = pair_case(n_sample)
    Z = np.zeros_like(S)
    run = lambda: rhs_tp(S, Z, g, vt, U=U_FRAME, dealias=True)
    g2, S2, vt2 = pair_case(48)
    Z2 = np.zeros_like(S2)
    run48 = lambda: rhs_tp(S2, Z2, g2, vt2, U=U_FRAME, dealias=True)
    t_all, t48_all = _timed(run, 1, 5), _timed(run48, 1, 5)
    with threadpool_limits(limits=1):
        t_one, t48_one = _timed(run, 1, 5), _timed(run48, 1, 5)
    # the reported value is the faster of the two thread settings ('cores' = its thread count)
    best_all = t_all <= t_one
    t_best, t48 = (t_all, t48_all) if best_all else (t_one, t48_one)
    res["cores"] = int(threads) if best_all else 1
    res["value"] = round(n_sample ** 3 / t_best / 1e9, 7)
    res["seconds"] = round(t_best, 4)
    res["threads"] = {f"{threads}": {"value": round(n_sample ** 3 / t_all / 1e9, 7), "seconds": round(t_all, 4)},
                      "1": {"value": round(n_sample ** 3 / t_one / 1e9, 7), "seconds": round(t_one, 4)}}
    res["sample"] = (f"oracle rhs_tp on the vortex-pair state at N_r=N_phi=N_z={n_sample} "
                     f"(1/{(256 // n_sample) ** 3} of the 256^3 grid points)")
    # growth with the grid, and the 256^3 rate it implies (an extrapolation, not a measurement)
    e = float(np.log(t_best / t48) / np.log(n_sample / 48))
    t256 = t_best * (256 / n_sample) ** e
    res["scaling"] = {"seconds_48": round(t48, 4), f"seconds_{n_sample}": round(t_best, 4), "exponent": round(e, 3),
                      "extrapolated_256_seconds": round(t256, 2),
                      "extrapolated_256_gdofs": round(256 ** 3 / t256 / 1e9, 7)}
    # parity of the bench path: the library's RHS at n_sample^3 (same workload) against the oracle's
    ref_p, ref_c = run()
    gp, gc = gpu_small["pair_psi_n"], gpu_small["pair_chi_n"]
    rel = lambda a, b: float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
    v_ref, _ = synthesize(ref_p, ref_c, g, vt)
    v_got, _ = synthesize(gp, gc, g, vt)
    res["parity"] = {"workload": f"vortex pair at {n_sample}^3, FP64",
                     "rel_err_psi_n": rel(gp, ref_p), "rel_err_chi_n": rel(gc, ref_c),
                     "rel_err_velocity_of_output": rel(np.stack(v_got), np.stack(v_ref))}
    cfg = {}
    # config 1: 32 x 16 x 1 scalar, u^2 term and round trip
    g1 = Grid(32, 16, 1, 1.0)
    t1 = Tables(g1)
    S1 = synth.geometric_spectrum(g1.M, g1.nrc, 1, g1.nzc, seed=1, a=0.7, b=0.8, c=1.0)
    tr = _timed(lambda: rhs_scalar(S1, g1, t1, "u2"), 1, 5)
    tp = _timed(lambda: forward(backward(S1, g1, t1), g1, t1), 1, 5)
    cfg["scalar_32x16x1"] = {"rhs_u2_ms": round(tr * 1e3, 4), "transform_pair_ms": round(tp * 1e3, 4),
                             "rhs_gdofs": round(512 / tr / 1e9, 7)}
    r1 = rhs_scalar(S1, g1, t1, "u2")
    cfg["scalar_32x16x1"]["parity_rel_err"] = rel(gpu_small["cfg1_u2"], r1)
    # config 2: 128^3 geometric potentials, vector RHS (1 warm-up, median of 3)
    g3 = Grid(128, 128, 128, 1.0)
    vt3 = VecTables(g3)
    P3 = synth.geometric_spectrum(g3.M, g3.nrc, 128, g3.nzc, seed=2, a=0.9, b=0.85, c=0.85)
    C3 = synth.geometric_spectrum(g3.M, g3.nrc, 128, g3.nzc, seed=3, a=0.9, b=0.85, c=0.85)
    t3 = _timed(lambda: rhs_tp(P3, C3, g3, vt3, U=(0.0, 0.0, 0.0), dealias=True), 1, 3)
    cfg["vector_128cubed"] = {"seconds": round(t3, 3), "gdofs": round(128 ** 3 / t3 / 1e9, 7), "median_of": 3}
    # config 3: the 64 batched 2D KPP terms (tables built outside the timed region; median of 3)
    insts = synth.batched_instances(64, 3)
    cases = []
    for k, d in enumerate(insts):
        gk = Grid(d["nr"], d["nphi"], 1, d["ell"])
        Sk = synth.geometric_spectrum(gk.M, gk.nrc, 1, gk.nzc, seed=1000 + k, a=0.9, b=0.85, c=1.0)
        cases.append((gk, Tables(gk), Sk))
    t4 = _timed(lambda: [rhs_scalar(Sk, gk, tk, "kpp", 0.25) for gk, tk, Sk in cases], 0, 3)
    dofs = sum(d["nr"] * d["nphi"] for d in insts)
    cfg["batched_2d_kpp"] = {"seconds": round(t4, 4), "gdofs": round(dofs / t4 / 1e9, 7), "median_of": 3,
                             "warmup": 0}
    res["configs"] = cfg
    return res


def bench_batched(torch, args, stream, e0, e1, count=64, seed=3):
    """64 uneven 2D KPP instances (the batched reaction-diffusion recipe: Gaussian bumps u on uneven
    grids, transformed by per-instance FP64 plans of the library) in three persistent launches
    (autotuned), FP64 and FP32."""
    import synth
    from paper_2609_18026_amd import MLG_FP32, Batch, Plan, mlg_grid
    insts = synth.batched_instances(count, seed)
    grids = [mlg_grid(d["nr"], d["nphi"], 1, 0, 0, 0, d["ell"], 2 * np.pi, 1) for d in insts]
    dofs = sum(d["nr"] * d["nphi"] for d in insts)
    res = {"instances": count, "grid_points": dofs,
           "input": "Gaussian bumps u = A exp(-|x - x0|^2 / (2 sigma^2)) per instance, forward-transformed in FP64"}
    spectra = []
    for d in insts:
        with Plan(d["nr"], d["nphi"], 1, d["ell"], 2 * np.pi) as pk:
            x, w, r = pk.nodes()
            phi = 2 * np.pi * np.arange(d["nphi"]) / d["nphi"]
            u = synth.gaussian_bump(r, phi, d["amp"], d["sigma"], d["x0"], d["y0"])[None]
            sk = pk.empty_spec()
            pk.forward(torch.from_numpy(np.ascontiguousarray(u)).cuda(), sk)
            torch.cuda.synchronize()
            spectra.append(sk[:, 0].clone())
    outs = {}
    for prec, name in ((0, "fp64"), (MLG_FP32, "fp32")):
        b = Batch(grids, prec=prec)
        sin = b.empty_spec()
        for k, sk in enumerate(spectra):
            sin[int(b.offsets[k]):int(b.offsets[k + 1])] = sk.to(sin.dtype)
        sout = b.empty_spec()
        chosen, tune_ms = b.autotune(0.25, sin, sout)
        for _ in range(args.warmup):
            b.rhs_kpp(0.25, sin, sout)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            b.rhs_kpp(0.25, sin, sout)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        outs[name] = sout.to(torch.complex128)
        res[name] = {"ms_per_launch": round(ms, 4), "gdofs": round(dofs / (ms / 1e3) / 1e9, 4),
                     "autotuned": b.get_config()}
        b.close()
    res["fp32_rel_err_vs_fp64"] = float(torch.linalg.vector_norm(outs["fp32"] - outs["fp64"]) /
                                        torch.linalg.vector_norm(outs["fp64"]))
    log(f"bench: batched 2D fp64 {res['fp64']['ms_per_launch']:.3f} ms, fp32 {res['fp32']['ms_per_launch']:.3f} ms")
    return res


def reduced_work(nr, nphi, nz, M, nrc, skip=True):
    """Algorithmic HBM bytes per RHS step of each kernel family on a reduced-precision plan: float
    data and intermediates (8-byte complex), 4-byte synthesis tables (FP32, or bfloat16 hi + lo),
    FP64 projection tables and sources.  skip: the synthesis covers only the orders and axial
    slots the mask keeps (as both reduced-precision syntheses do at 256^3)."""
    tau = sum(max(nrc - m, 0) for m in range(M))
    mmax, nkact = active_columns(nphi, nz, M, nrc)
    mk = min(M, (nphi - 1) // 3 + 1)
    tau_k = sum(max(nrc - m, 0) for m in range(mk))
    tau_a = sum(max(nrc - m, 0) for m in range(mmax))
    kept = mk * nr * nz * 8
    f = 0.5 if nr % 2 == 0 else 1.0
    synth = (f * 2 * tau_k * nr * 4 + 2 * tau_k * nkact * 8 + 6 * mk * nr * nkact * 8) if skip else \
        (f * 2 * tau * nr * 4 + 2 * tau * nz * 8 + 6 * M * nr * nz * 8)
    return {"synth_gemm": synth,
            "proj_gemm": f * 2 * tau_a * nr * 8 + 3 * mmax * nr * nkact * 8 + 3 * tau_a * nkact * 16,
            "phi_fft": 9 * kept,
            "z_fft": 6 * mk * nr * (nkact + nz) * 8 + 3 * mmax * nr * (nz + nkact) * 8,
            "projection": 3 * tau_a * nkact * 16 + 2 * tau * nz * 8 + 24 * tau_a * nkact + 11 * 8 * tau_a}


def bench_reduced(torch, prec, plan, psi, chi, fp64_kernels, args, stream, e0, e1):
    """An MLG_FP32 or MLG_SPLIT_BF16 plan (float data) on the same state rounded to complex64: RHS and
    transform-pair times and per-kernel times beside FP64, the algorithmic bytes of both, and the
    errors against the FP64 library result on the same rounded inputs (that result is itself within
    1e-12 of the oracle), so that they are the reduced arithmetic's own: the nodal taps u, omega, N
    and the sources C, K, Zhat, the output coefficients, and the velocity V(psi_N, chi_N) they
    represent (plain and area-weighted node norms, and relative to the nodal N)."""
    from paper_2609_18026_amd import MLG_FP32, Plan, mlg_timing_enable, mlg_timing_read
    name = "fp32" if prec == MLG_FP32 else "split-bf16"
    n = plan.nr
    pe = plan.layout.phys_elems
    se = plan.layout.spec_elems
    rp = Plan(n, n, n, 1.0, PAIR["lz"], dealias=1, prec=prec)
    p32, c32 = psi.to(torch.complex64), chi.to(torch.complex64)
    psi_r, chi_r = p32.to(torch.complex128), c32.to(torch.complex128)   # the rounded state in FP64
    sp, sc = rp.empty_spec(), rp.empty_spec()
    for _ in range(args.warmup):
        rp.rhs_tp(p32, c32, sp, sc, U=U_FRAME)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        rp.rhs_tp(p32, c32, sp, sc, U=U_FRAME)
    e1.record(stream)
    torch.cuda.synchronize()
    rms = e0.elapsed_time(e1) / args.steps
    families = ["synth_gemm", "proj_gemm", "phi_fft", "z_fft", "projection", "radial_gemm"]
    mlg_timing_enable(rp.handle, True)
    for f in families:
        mlg_timing_read(rp.handle, f)
    for _ in range(args.steps):
        rp.rhs_tp(p32, c32, sp, sc, U=U_FRAME)
    torch.cuda.synchronize()
    kern = {f: mlg_timing_read(rp.handle, f) for f in families}
    mlg_timing_enable(rp.handle, False)
    bytes_r = reduced_work(n, n, n, plan.layout.M, plan.layout.nrc)
    bytes_64 = {f: w["bytes"] for f, w in kernel_work(n, n, n, plan.layout.M, plan.layout.nrc).items()}
    per_kernel = {}
    for f in families[:5]:
        t = kern[f][0] / args.steps
        per_kernel[f] = {"ms_per_step": round(t, 4), "fp64_ms_per_step": fp64_kernels[f]["ms_per_step"],
                         "algorithmic_bytes_per_step": bytes_r[f], "fp64_algorithmic_bytes_per_step": bytes_64[f],
                         "gbs": round(bytes_r[f] / (t / 1e3) / 1e9, 1) if t > 0 else None}
    # transform pair (float physical field)
    rphys, rspec = rp.empty_phys(), rp.empty_spec()
    rp.backward(p32, rphys)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        rp.backward(p32, rphys)
        rp.forward(rphys, rspec)
    e1.record(stream)
    torch.cuda.synchronize()
    pair_ms = e0.elapsed_time(e1) / args.steps
    rel = lambda x, y: float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y))
    # FP64 references on the rounded inputs
    phys64, spec64 = plan.empty_phys(), plan.empty_spec()
    plan.backward(psi_r, phys64)
    plan.forward(rphys.to(torch.float64), spec64)
    torch.cuda.synchronize()
    perr = rel(rphys.to(torch.float64), phys64)
    serr = rel(rspec.to(torch.complex128), spec64)
    del rphys, rspec, phys64, spec64
    t64, tr = plan.taps_buffer(), rp.taps_buffer()
    a, b = plan.empty_spec(), plan.empty_spec()
    plan.rhs_tp(psi_r, chi_r, a, b, U=U_FRAME, taps=t64)
    rp.rhs_tp(p32, c32, sp, sc, U=U_FRAME, taps=tr)
    torch.cuda.synchronize()
    rp.close()
    taps = {"u": rel(tr[:3 * pe], t64[:3 * pe]), "omega": rel(tr[3 * pe:6 * pe], t64[3 * pe:6 * pe]),
            "N": rel(tr[6 * pe:9 * pe], t64[6 * pe:9 * pe])}
    for j, nm in enumerate(("C", "K", "Zhat")):
        o = 9 * pe + 2 * j * se
        taps[nm] = rel(tr[o:o + 2 * se], t64[o:o + 2 * se])
    Nn = t64[6 * pe:9 * pe].view(3, n, n, n).clone()
    del t64, tr
    spd, scd = sp.to(torch.complex128), sc.to(torch.complex128)
    uw_ref = torch.empty(6 * pe, dtype=torch.float64, device="cuda")
    uw_red = torch.empty_like(uw_ref)
    plan.synthesize(a, b, uw_ref)
    plan.synthesize(spd, scd, uw_red)
    torch.cuda.synchronize()
    x, w, r = plan.nodes()
    area = torch.from_numpy(w / (1 - x) ** 2).cuda()
    vr = uw_ref[:3 * pe].view(3, n, n, n)
    vs = uw_red[:3 * pe].view(3, n, n, n)
    d2 = ((vs - vr) ** 2).sum(dim=(0, 1, 3))
    r2 = (vr ** 2).sum(dim=(0, 1, 3))
    n2 = (Nn ** 2).sum(dim=(0, 1, 3))
    vel = {"plain": rel(vs, vr), "area_weighted": float(torch.sqrt((d2 * area).sum() / (r2 * area).sum())),
           "plain_rel_to_N": float(torch.sqrt(d2.sum() / n2.sum())),
           "area_weighted_rel_to_N": float(torch.sqrt((d2 * area).sum() / (n2 * area).sum()))}
    res = {"ms_per_step": round(rms, 4), "gdofs": round(n ** 3 / (rms / 1e3) / 1e9, 4),
           "algorithmic_bytes_per_step": sum(bytes_r.values()),
           "fp64_algorithmic_bytes_per_step": sum(bytes_64.values()),
           "data": "float / complex64 arrays; the state is the FP64 state rounded to complex64",
           "stages": ("FP32 MFMA" if prec == MLG_FP32 else "split bfloat16 MFMA (hi/lo, FP32 accumulation)") +
                     ": synthesis and transform-pair radial products" +
                     ("" if prec == MLG_FP32 else ", inverse z DFT products") +
                     "; FP64 arithmetic on float-stored data: phi FFTs, cross product, z FFTs; FP64: projection "
                     "source products and solves",
           "kernels": per_kernel,
           "rel_err_vs_fp64_same_inputs": {"velocity_of_output": vel, "psi_coefficients": rel(spd, a),
                                           "chi_coefficients": rel(scd, b), "taps": taps},
           "input_rounding_rel": rel(psi_r, psi),
           "transform_pair_ms": round(pair_ms, 4), "transform_pair_gdofs": round(n ** 3 / (pair_ms / 1e3) / 1e9, 4),
           "rel_err_pair_backward_vs_fp64": perr, "rel_err_pair_forward_vs_fp64": serr}
    log(f"bench: {name} {rms:.3f} ms/step, velocity rel err {vel['plain']:.2e} (area {vel['area_weighted']:.2e}, "
        f"vs |N| {vel['plain_rel_to_N']:.2e}); taps {taps}; pair {pair_ms:.3f} ms, rel err {perr:.2e} / {serr:.2e}; "
        f"kernels {per_kernel}")
    return res


def bench_small(torch, args, stream, e0, e1):
    """The other workloads on the GPU: the 32 x 16 x 1 scalar term and transform pair, the 128^3 vector
    RHS of geometric potentials, and the vortex-pair RHS at the oracle's sample size (for the parity
    figure of the bench path).  Returns host copies of the outputs the oracle leg compares, and
    timings."""
    import synth
    from paper_2609_18026_amd import MLG_RHS_U2, Plan

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    outs, res = {}, {}
    p1 = Plan(32, 16, 1, 1.0)
    S1 = synth.geometric_spectrum(p1.layout.M, p1.layout.nrc, 1, p1.layout.nzc, seed=1, a=0.7, b=0.8, c=1.0)
    d1 = torch.from_numpy(synth.to_packed(S1)).cuda()
    o1, ph = p1.empty_spec(), p1.empty_phys()
    ms_u2 = timed(lambda: p1.rhs_scalar(MLG_RHS_U2, 0.25, d1, o1))
    ms_pair = timed(lambda: (p1.backward(d1, ph), p1.forward(ph, o1)))
    p1.rhs_scalar(MLG_RHS_U2, 0.25, d1, o1)
    torch.cuda.synchronize()
    outs["cfg1_u2"] = synth.from_packed(o1.cpu().numpy(), p1.layout.M, p1.layout.nrc)
    res["scalar_32x16x1"] = {"rhs_u2_us": round(ms_u2 * 1e3, 2), "transform_pair_us": round(ms_pair * 1e3, 2),
                             "rhs_gdofs": round(512 / (ms_u2 / 1e3) / 1e9, 5)}
    p1.close()
    p3 = Plan(128, 128, 128, 1.0)
    L3 = p3.layout
    P3 = torch.from_numpy(synth.to_packed(synth.geometric_spectrum(L3.M, L3.nrc, 128, L3.nzc, seed=2, a=0.9, b=0.85,
                                                                     c=0.85))).cuda()
    C3 = torch.from_numpy(synth.to_packed(synth.geometric_spectrum(L3.M, L3.nrc, 128, L3.nzc, seed=3, a=0.9, b=0.85,
                                                                     c=0.85))).cuda()
    a3, b3 = p3.empty_spec(), p3.empty_spec()
    ms3 = timed(lambda: p3.rhs_tp(P3, C3, a3, b3))
    res["vector_128cubed"] = {"ms_per_step": round(ms3, 4), "gdofs": round(128 ** 3 / (ms3 / 1e3) / 1e9, 4)}
    p3.close()
    n = args.cpu_sample
    ps = Plan(n, n, n, 1.0, PAIR["lz"], dealias=1)
    _, psi, chi = build_state(ps, n, torch)
    a, b = ps.empty_spec(), ps.empty_spec()
    ps.rhs_tp(psi, chi, a, b, U=U_FRAME)
    torch.cuda.synchronize()
    L = ps.layout
    outs["pair_psi_n"] = synth.from_packed(a.cpu().numpy(), L.M, L.nrc)
    outs["pair_chi_n"] = synth.from_packed(b.cpu().numpy(), L.M, L.nrc)
    ps.close()
    log(f"bench: 32x16x1 u^2 term {ms_u2 * 1e3:.1f} us, 128^3 vector RHS {ms3:.3f} ms")
    return outs, res


def bench_no_mask(torch, n, psi, chi, args, stream, e0, e1):
    """The same RHS on a plan without dealiasing (dealias = 0): every mode of the input is synthesized
    and every output mode kept, so none of the work the two-thirds mask removes is skipped."""
    from paper_2609_18026_amd import Plan
    pn = Plan(n, n, n, 1.0, PAIR["lz"], dealias=0)
    a, b = pn.empty_spec(), pn.empty_spec()
    for _ in range(args.warmup):
        pn.rhs_tp(psi, chi, a, b, U=U_FRAME)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        pn.rhs_tp(psi, chi, a, b, U=U_FRAME)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    pn.close()
    log(f"bench: RHS without dealiasing {ms:.3f} ms/step")
    return {"ms_per_step": round(ms, 4), "gdofs": round(n ** 3 / (ms / 1e3) / 1e9, 4),
            "note": "dealias = 0: every input mode synthesized, every output mode kept"}


def bench_time_step(torch, plan, psi, chi, args, stream, e0, e1):
    """Whole AB-CN steps of (psi, chi) at the bench size: one RHS plus the implicit update of both
    potentials per step (Eq. abcn), through mlg_tp_advance on resident state."""
    from paper_2609_18026_amd import mlg_timing_enable, mlg_timing_read
    plan.step_setup(1e-4, 1e-14, 8, 5e-4)
    p, c = psi.clone(), chi.clone()
    hp, hc = plan.empty_spec(), plan.empty_spec()
    tmp = torch.empty(6 * plan.layout.spec_elems, dtype=torch.complex128, device="cuda")
    plan.advance(p, c, hp, hc, 1 + args.warmup, start=1, U=U_FRAME, tmp=tmp)
    torch.cuda.synchronize()
    e0.record(stream)
    plan.advance(p, c, hp, hc, args.steps, start=0, U=U_FRAME, tmp=tmp)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # the implicit part from a second, instrumented pass (events around every launch)
    mlg_timing_enable(plan.handle, True)
    mlg_timing_read(plan.handle, "step")
    plan.advance(p, c, hp, hc, args.steps, start=0, U=U_FRAME, tmp=tmp)
    torch.cuda.synchronize()
    step_ms, launches = mlg_timing_read(plan.handle, "step")
    mlg_timing_enable(plan.handle, False)
    nrc, M, nz = plan.layout.nrc, plan.layout.M, plan.nz
    ksq = sum((nrc - m - (1 if m == 0 else 0)) ** 2 for m in range(min(M, nrc)))
    flops = 2 * 12.0 * nz * ksq          # two potentials; V^-1 [s | a] (2 products) and V W per m
    impl_ms = step_ms / args.steps
    finite = bool(torch.isfinite(torch.view_as_real(p)).all().item())
    res = {"ms_per_step": round(ms, 4), "implicit_ms_per_step": round(impl_ms, 4),
           "implicit_tflops": round(flops / (impl_ms / 1e3) / 1e12, 3),
           "implicit_frac_fp64_peak": round(flops / (impl_ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4),
           "gdofs": round(plan.nr * plan.nphi * nz / (ms / 1e3) / 1e9, 4), "state_finite": finite,
           "params": {"nu": 1e-4, "nu_h": 1e-14, "p": 8, "dt": 5e-4},
           "paper_context": "the paper's 256^3 run (a different vortex, ell=4, p=8) takes 78.9 s per 30 steps on "
                            "128 EPYC 7763 cores (Table tab:scaling), 2.63 s per step"}
    log(f"bench: AB-CN time step {ms:.3f} ms (implicit part {impl_ms:.3f} ms)")
    return res


def bench_closure_cost(torch, args, stream, e0, e1):
    """Cost of the closure's kernels alone (for profiling): training steps of 4096 rows and inferences
    on the 64^3 coarse grid, with random data and weights (no fine runs)."""
    import synth
    from paper_2609_18026_amd import Closure, Plan
    coarse = Plan(64, 64, 64, 1.0, PAIR["lz"])
    cl = Closure(coarse, max_batch=4096, beta=1e30)
    r = np.random.default_rng(7)
    rows = 4 * 4096
    X = torch.from_numpy(r.standard_normal((rows, 258)).astype(np.float32)).cuda()
    Y = torch.from_numpy(r.standard_normal((rows, 256)).astype(np.float32)).cuda()
    cl.set_params(synth.closure_init(1))
    batches = torch.from_numpy(synth.batch_indices(rows, 4096, args.steps + args.warmup, seed=3)).cuda()
    for s_ in range(args.warmup):
        cl.train_step(X, Y, batches[s_], 4096, 1e-4)
    torch.cuda.synchronize()
    e0.record(stream)
    for s_ in range(args.steps):
        cl.train_step(X, Y, batches[args.warmup + s_], 4096, 1e-4)
    e1.record(stream)
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / args.steps
    _, psi, chi = build_state(coarse, 64, torch)
    Np, Nc = coarse.empty_spec(), coarse.empty_spec()
    coarse.rhs_tp(psi, chi, Np, Nc, U=U_FRAME)
    e0.record(stream)
    for _ in range(args.steps):
        cl.infer(psi, chi, Np, Nc)
    e1.record(stream)
    torch.cuda.synchronize()
    inf_ms = e0.elapsed_time(e1) / args.steps
    flops = 3 * 2.0 * 4096 * (288 * 256 + 256 * 256 + 256 * 256)
    cl.close()
    coarse.close()
    log(f"bench: closure train step {train_ms:.3f} ms, inference {inf_ms:.3f} ms (random data)")
    return {"train_step_ms": round(train_ms, 4), "train_tflops": round(flops / (train_ms / 1e3) / 1e12, 3),
            "infer_ms": round(inf_ms, 4)}


def bench_closure(torch, args, stream, e0, e1):
    """Learned closure at the coarse 64^3 grid: cost of a training step (4096 columns) and of an
    inference next to the coarse RHS, then the held-out gain of a network trained on fine 256^3
    runs and coarse roll-outs with and without it (the recipe of the gain test)."""
    import synth
    from paper_2609_18026_amd import Closure, Plan
    from paper_2609_18026_amd import closure_runs as cr
    n_c, n_f = 64, 256
    coarse = Plan(n_c, n_c, n_c, 1.0, PAIR["lz"])
    fine = Plan(n_f, n_f, n_f, 1.0, PAIR["lz"])
    spec = cr.RunSpec(nu=1e-4, nu_h=1e-14, p=8, dt=5e-4, U=U_FRAME)
    cr.setup(fine, spec)
    cr.setup(coarse, spec)

    def init(plan, delta, phase):
        x, w, r = plan.nodes()
        phi = 2 * np.pi * np.arange(plan.nphi) / plan.nphi
        z = PAIR["lz"] * np.arange(plan.nz) / plan.nz
        f = synth.vortex_pair_psi(r, phi, z, gamma=PAIR["gamma"], a=PAIR["a"], b=PAIR["b"], delta=delta,
                                  lz=PAIR["lz"], phase=phase)
        psi = plan.empty_spec()
        plan.forward(torch.from_numpy(np.ascontiguousarray(f)).cuda(), psi)
        return psi, torch.zeros_like(psi)

    nsnap, every = 12, 40
    runs = []
    for i in range(8):
        phase = float(synth.rng(5 + i).uniform(0, 2 * np.pi))
        runs.append(cr.fine_run(fine, coarse, spec, *init(fine, (0.005, 0.01, 0.02)[i % 3], phase), nsnap, every))
    torch.cuda.synchronize()

    def merge(rs):
        out = cr.Snapshots()
        for r in rs:
            out.psi += r.psi
            out.chi += r.chi
            out.ref_psi += r.ref_psi
            out.ref_chi += r.ref_chi
        return out

    train, held = merge(runs[:6]), merge(runs[6:])
    cl = Closure(coarse, max_batch=4096, beta=1.0)
    X, Y = cr.dataset(coarse, cl, train, spec)
    xr = torch.sqrt(torch.mean(X.double() ** 2, 0)).cpu().numpy()
    yr = torch.sqrt(torch.mean(Y.double() ** 2, 0)).cpu().numpy()
    xs = np.where(xr > 0, 1.0 / np.maximum(xr, 1e-300), 1.0).astype(np.float32)
    ys = np.where(yr > 0, yr, 1.0).astype(np.float32)
    cl.set_scales(xs, ys)
    cl.set_params(synth.closure_init(1))
    nb, steps = 4096, 3000
    batches = torch.from_numpy(synth.batch_indices(X.shape[0], nb, steps, seed=3)).cuda()
    torch.cuda.synchronize()
    e0.record(stream)
    cr.fit(cl, X, Y, batches, 1e-3, 5e-5)
    e1.record(stream)
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / steps
    flops_train = 3 * 2.0 * nb * (288 * 256 + 256 * 256 + 256 * 256)
    # inference and the coarse RHS on one held-out snapshot
    p, c = held.psi[6], held.chi[6]
    Np, Nc = coarse.empty_spec(), coarse.empty_spec()
    reps = 50
    e0.record(stream)
    for _ in range(reps):
        coarse.rhs_tp(p, c, Np, Nc, U=U_FRAME)
    e1.record(stream)
    torch.cuda.synchronize()
    rhs_ms = e0.elapsed_time(e1) / reps
    free = Closure(coarse, max_batch=4096, beta=1e30)
    free.set_scales(xs, ys)
    free.set_params(cl.get_params())
    e0.record(stream)
    for _ in range(reps):
        free.infer(p, c, Np, Nc)
    e1.record(stream)
    torch.cuda.synchronize()
    inf_ms = e0.elapsed_time(e1) / reps

    def gain(closure, snaps):
        res = cr.a_priori(coarse, closure, snaps, spec)
        return sum(a for _, a, _ in res) / sum(b for b, _, _ in res), int(sum(f for *_, f in res))

    g_tr, _ = gain(free, train)
    g_free, _ = gain(free, held)
    g_jud, nfb = gain(cl, held)
    # a posteriori: roll-outs of both held-out runs against their truncated fine runs

    def nrm(*ts):
        return float(np.sqrt(sum(torch.linalg.vector_norm(t).item() ** 2 for t in ts)))

    ref = Plan(96, 96, 96, 1.0, PAIR["lz"], nrc=n_c, nphic=n_c // 2, nzc=n_c // 2)
    rj = Closure(coarse, max_batch=4096, beta=1.0)
    rj.set_scales(xs, ys)
    rj.set_params(cl.get_params())
    rj.set_reference(ref, spec.U)
    roll = {}
    for ri in (6, 7):
        sn = runs[ri]
        for name, clo in (("plain", None), ("closure_judged", cl), ("closure_unjudged", free),
                          ("closure_reference_judge", rj)):
            st = cr.rollout(coarse, spec, sn.psi[0], sn.chi[0], nsnap, every, closure=clo)
            roll[f"run{ri}_{name}"] = [round(nrm(a - sn.psi[j], b - sn.chi[j]) / nrm(sn.psi[j], sn.chi[j]), 6)
                                       for j, (a, b) in enumerate(st)][1:]
    calls, fbs = cl.stats()
    rcalls, rfbs = rj.stats()
    res = {"coarse": f"{n_c}^3", "fine": f"{n_f}^3", "columns": cl.ncols, "train_rows": int(X.shape[0]),
           "train_step_ms": round(train_ms, 4), "train_batch": nb,
           "train_tflops": round(flops_train / (train_ms / 1e3) / 1e12, 3),
           "train_frac_bf16_peak": round(flops_train / (train_ms / 1e3) / 1e12 / 2500.0, 5),
           "infer_ms": round(inf_ms, 4), "coarse_rhs_ms": round(rhs_ms, 4),
           "infer_overhead_vs_rhs": round(inf_ms / rhs_ms, 4),
           "a_priori_gain": {"train": round(g_tr, 4), "held_out_unjudged": round(g_free, 4),
                             "held_out_judged": round(g_jud, 4), "held_out_fallbacks": nfb,
                             "held_out_snapshots": len(held.psi)},
           "rollout_rel_field_error": roll, "rollout_judge_calls_fallbacks": [calls, fbs],
           "rollout_reference_judge_calls_fallbacks": [rcalls, rfbs],
           "reference_judge": "plain term of the coarse state on 96^3 nodes (64^3 coefficients), corrections kept "
                              "only when they move the coarse term towards it",
           "recipe": "8 fine 256^3 vortex-pair runs (delta 0.005/0.01/0.02, phases from seeds 5..12), nu=1e-4, "
                     "nu_h=1e-14, p=8, dt=5e-4, 12 snapshots 40 steps apart; runs 0-5 train, 6-7 held out; "
                     "coarse 64^3"}
    log(f"bench: closure train step {train_ms:.3f} ms, inference {inf_ms:.3f} ms vs coarse RHS {rhs_ms:.3f} ms, "
        f"held-out gain {g_free:.3f} (judged {g_jud:.3f})")
    torch.cuda.synchronize()
    for h in (rj, free, cl, ref, fine, coarse):
        h.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=25)  # ~25 ms of untimed RHS steps: the GPU clocks settle
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure section")
    ap.add_argument("--sections", default="all",
                    help="comma list of the sections after the headline RHS and transform pair to run: no_mask "
                         "(the RHS without dealiasing), fp32, split, batched, step, closure, closure_cost (training "
                         "and inference cost on random data only, for profiling), small (and the oracle leg); "
                         "default all but closure_cost")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain device copy of 256 MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported (the library has no "
              "multi-GPU path: its kernels work on one GPU's share of the grid)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2609_18026_amd import Plan, mlg_timing_enable, mlg_timing_read
    # a plain 256 MiB device copy: the HBM counter reference (--calibrate-copy) and the practical
    # read + write rate the streaming kernels are compared with
    src = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    if args.calibrate_copy:
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: calibration copy of 268435456 bytes x3 done")
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_ms = c0.elapsed_time(c1) / 10
    copy_ref = {"bytes_read_plus_written": 2 * 2 ** 28, "ms": round(copy_ms, 4),
                "gbs": round(2 * 2 ** 28 / (copy_ms / 1e3) / 1e9, 1),
                "frac_hbm_peak": round(2 * 2 ** 28 / (copy_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
    log(f"bench: plain 256 MiB device copy {copy_ref['gbs']:.0f} GB/s (read + write)")
    del src, dst
    n = args.n
    plan = Plan(n, n, n, 1.0, PAIR["lz"], dealias=1)
    log(f"bench: plan {n}^3 ready, workspace {plan.layout.workspace_bytes / 2**30:.2f} GiB")
    _, psi, chi = build_state(plan, n, torch)
    po, co = plan.empty_spec(), plan.empty_spec()
    for _ in range(args.warmup):
        plan.rhs_tp(psi, chi, po, co, U=U_FRAME)
    torch.cuda.synchronize()
    log("bench: warmup done")
    families = ["synth_gemm", "proj_gemm", "phi_fft", "z_fft", "projection"]
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # the timed steps run uninstrumented; a second pass of the same steps then times every kernel
    # launch with HIP events on the stream it runs on (the per-kernel figures and the roofline):
    # bracketing each launch with events adds about 0.1 ms to a step
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.rhs_tp(psi, chi, po, co, U=U_FRAME)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    mlg_timing_enable(plan.handle, True)
    for f in families + ["radial_gemm", "mask"]:
        mlg_timing_read(plan.handle, f)
    for _ in range(args.steps):
        plan.rhs_tp(psi, chi, po, co, U=U_FRAME)
    torch.cuda.synchronize()
    kern = {f: mlg_timing_read(plan.handle, f) for f in families}
    mlg_timing_enable(plan.handle, False)
    log(f"bench: {ms:.3f} ms/step (wall {wall / args.steps * 1e3:.3f})")
    value = n ** 3 / (ms / 1e3) / 1e9
    work = kernel_work(n, n, n, plan.layout.M, plan.layout.nrc)
    per_kernel = {}
    for f in families:
        tot_ms, launches = kern[f]
        step_ms = tot_ms / args.steps
        wk = work[f]
        ent = {"ms_per_step": round(step_ms, 4), "launches_per_step": launches / args.steps,
               "avg_launch_ms": round(tot_ms / max(launches, 1), 4)}
        if wk["flops"]:
            ent["tflops"] = round(wk["flops"] / (step_ms / 1e3) / 1e12, 3)
            ent["frac_fp64_peak"] = round(ent["tflops"] / PEAK_FP64_TFLOPS, 4)
        ent["gbs"] = round(wk["bytes"] / (step_ms / 1e3) / 1e9, 1)
        ent["frac_hbm_peak"] = round(ent["gbs"] / PEAK_HBM_GBS, 4)
        ent["algorithmic_bytes_per_step"] = wk["bytes"]
        ent["measured_hbm_bytes_per_step"] = measured_traffic(f, n, per_launch=False)
        per_kernel[f] = ent
    dom = max(families, key=lambda f: kern[f][0])
    d = per_kernel[dom]
    if work[dom]["flops"]:
        launches = max(kern[dom][1], 1)
        roofline = dict(bound="mfma", kernel=dom, achieved=d["tflops"], peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                        frac=d["frac_fp64_peak"], traffic=measured_traffic(dom, n),
                        algorithmic_bytes_per_launch=work[dom]["bytes"],
                        work_per_launch=work[dom]["flops"] * args.steps / launches, avg_launch_ms=d["avg_launch_ms"])
        rec = measured_record(dom, n)
        if rec is not None and "profile_avg_ms" in rec:
            wl = work[dom]["flops"] * args.steps / launches
            roofline["profile"] = {"avg_launch_ms": rec["profile_avg_ms"],
                                   "frac": round(wl / (rec["profile_avg_ms"] / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4),
                                   "mfma_counter_flops": rec.get("mfma_counter_flops"),
                                   "mfma_busy_pct": rec.get("mfma_busy_pct"),
                                   "source": _SUMMARY}
    else:
        launches = max(kern[dom][1], 1)
        roofline = dict(bound="hbm", kernel=dom, achieved=d["gbs"], peak=PEAK_HBM_GBS, unit="GB/s",
                        frac=d["frac_hbm_peak"], traffic=measured_traffic(dom, n),
                        work_per_launch=work[dom]["bytes"] * args.steps / launches, avg_launch_ms=d["avg_launch_ms"])
    # transform pair of one scalar on the same plan (extra figure)
    phys = plan.empty_phys()
    spec = plan.empty_spec()
    plan.backward(psi, phys)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        plan.backward(psi, phys)
        plan.forward(phys, spec)
    e1.record(stream)
    torch.cuda.synchronize()
    pair_ms = e0.elapsed_time(e1) / args.steps
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"toroidal-poloidal RHS P[(U+u) x omega] of a counter-rotating Lamb-Oseen vortex "
                               f"pair at N_r=N_phi=N_z={n}, ell=1, L_z=8.6, two-thirds dealiasing, FP64",
                   "nr": n, "nphi": n, "nz": n, "ell": 1.0, "lz": PAIR["lz"], "U": list(U_FRAME)},
        "roofline": roofline,
        "kernels": per_kernel,
        "kernel_timing": "a second pass of the same steps after the timed one, with HIP events around every "
                         "launch on the stream it runs on (the timed pass runs without them)",
        "transform_pair": {"ms": round(pair_ms, 4), "gdofs": round(n ** 3 / (pair_ms / 1e3) / 1e9, 4)},
        "hbm_copy_reference": copy_ref,
    }
    sections = set(args.sections.split(",")) if args.sections != "all" else None
    want = lambda name: (sections is None and name != "closure_cost") or (sections is not None and name in sections)
    if want("no_mask"):  # a section of its own: its phi stage shares the kernel and grid of the headline's
        out["no_mask"] = bench_no_mask(torch, n, psi, chi, args, stream, e0, e1)
    # reduced-precision plans on the same state: time, bytes, and the errors against the FP64 result
    if want("fp32"):
        from paper_2609_18026_amd import MLG_FP32
        out["fp32"] = bench_reduced(torch, MLG_FP32, plan, psi, chi, per_kernel, args, stream, e0, e1)
        out["fp32"]["fp64_ms_per_step"] = round(ms, 4)
    if want("split"):
        from paper_2609_18026_amd import MLG_SPLIT_BF16
        out["split_bf16"] = bench_reduced(torch, MLG_SPLIT_BF16, plan, psi, chi, per_kernel, args, stream, e0, e1)
        out["split_bf16"]["fp64_ms_per_step"] = round(ms, 4)
    if want("batched"):
        out["batched_2d"] = bench_batched(torch, args, stream, e0, e1)
    if want("step"):
        out["time_step"] = bench_time_step(torch, plan, psi, chi, args, stream, e0, e1)
    if want("closure") and not args.no_closure:
        out["closure"] = bench_closure(torch, args, stream, e0, e1)
    if want("closure_cost"):
        out["closure_cost"] = bench_closure_cost(torch, args, stream, e0, e1)
    torch.cuda.synchronize()
    s256 = None
    if want("small") and not args.no_cpu_baseline and n == 256:
        s256 = sample_rhs_256(torch, plan, psi, n)
    plan.close()                 # every native handle is released before the interpreter shuts down
    gpu_small = None
    if want("small"):
        gpu_small, out["small_workloads"] = bench_small(torch, args, stream, e0, e1)
    if not args.no_cpu_baseline and gpu_small is not None:
        log("bench: timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample, gpu_small)
        out["rel_err_vs_fp64_oracle"] = out["cpu_baseline"]["parity"]
        if s256 is not None:
            log("bench: sampled 256^3 oracle comparison")
            t0 = time.perf_counter()
            out["cpu_baseline"]["parity_256_sampled"] = parity_256_sampled(s256)
            out["cpu_baseline"]["parity_256_sampled"]["oracle_seconds"] = round(time.perf_counter() - t0, 2)
            out["rel_err_vs_fp64_oracle"] = dict(out["cpu_baseline"]["parity"],
                                                 sampled_256cubed=out["cpu_baseline"]["parity_256_sampled"])
            del s256
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
