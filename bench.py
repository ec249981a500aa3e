"""Benchmark: toroidal-poloidal nonlinear RHS at N_r = N_phi = N_z = 256 on one MI355X.

One step = one mlg_rhs_tp call on the resident 256^3 vortex-pair state (FP64): radial
synthesis of u and omega, inverse z and phi FFTs, (U + u) x omega, forward FFTs,
Galerkin projection and the per-(m, k) elliptic solves (the whole transform round trip
plus the nonlinear term).  value = N_r N_phi N_z / (seconds per step) / 1e9 [GDOF/s].

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
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


def kernel_work(nr, nphi, nz, M, nrc):
    """Algorithmic flops / HBM bytes per RHS step for each kernel family (FP64)."""
    tau = sum(max(nrc - m, 0) for m in range(M))
    mmax, nkact = active_columns(nphi, nz, M, nrc)
    tau_a = sum(max(nrc - m, 0) for m in range(mmax))
    mixed = M * nr * nz * 16                     # one harmonic field, complex
    w = {}
    w["synth_gemm"] = dict(flops=7 * 2.0 * nr * tau * 2 * nz,
                           bytes=2 * tau * nr * 8 + 2 * tau * nz * 16 + 6 * mixed)
    w["proj_gemm"] = dict(flops=5 * 2.0 * nr * tau_a * 2 * nkact,
                          bytes=2 * tau_a * nr * 8 + 3 * mmax * nr * nkact * 16 + 3 * tau_a * nkact * 16)
    w["phi_fft"] = dict(flops=None, bytes=9 * mixed)
    w["z_fft"] = dict(flops=None, bytes=6 * 2 * mixed + 3 * 2 * mmax * nr * nz * 16)
    w["projection"] = dict(flops=None, bytes=3 * tau_a * nkact * 16 + 2 * tau * nz * 16)
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


def cpu_baseline(n_sample: int):
    """Oracle rhs_tp on the same vortex-pair workload at n_sample^3 (host cores)."""
    import synth
    from oracle.grid import Grid
    from oracle.rhs import VecTables, rhs_tp
    from oracle.transform import Tables, forward
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    g = Grid(n_sample, n_sample, n_sample, 1.0, lz=PAIR["lz"])
    psi = synth.vortex_pair_psi(g.r, g.phi, g.z, gamma=PAIR["gamma"], a=PAIR["a"], b=PAIR["b"],
                                delta=PAIR["delta"], lz=PAIR["lz"])
    S = forward(psi, g, Tables(g))
    vt = VecTables(g)
    t0 = time.perf_counter()
    rhs_tp(S, np.zeros_like(S), g, vt, U=U_FRAME, dealias=True)
    dt = time.perf_counter() - t0
    return dict(value=round(n_sample ** 3 / dt / 1e9, 6), unit="GDOF/s", cores=int(threads), kind="oracle",
                sample=f"one oracle rhs_tp on the vortex-pair state at N_r=N_phi=N_z={n_sample} "
                       f"(1/{(256 // n_sample) ** 3} of the 256^3 grid points), {dt:.1f} s")


def bench_batched(torch, args, stream, e0, e1, count=64, seed=3):
    """64 uneven 2D KPP instances in one persistent launch (autotuned), FP64 and FP32."""
    import synth
    from paper_2609_18026_amd import MLG_FP32, Batch, mlg_grid
    insts = synth.batched_instances(count, seed)
    grids = [mlg_grid(d["nr"], d["nphi"], 1, 0, 0, 0, d["ell"], 2 * np.pi, 1) for d in insts]
    dofs = sum(d["nr"] * d["nphi"] for d in insts)
    res = {"instances": count, "grid_points": dofs}
    outs = {}
    for prec, name in ((0, "fp64"), (MLG_FP32, "fp32")):
        b = Batch(grids, prec=prec)
        sin = b.empty_spec()
        for k, d in enumerate(insts):
            M = d["nphi"] // 2
            S = synth.geometric_spectrum(M, d["nr"], 1, 1, seed=1000 + k, a=0.9, b=0.85, c=1.0)
            sin[int(b.offsets[k]):int(b.offsets[k + 1])] = torch.from_numpy(synth.to_packed(S)[:, 0]).to(sin.dtype).cuda()
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=128)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain device copy of 256 MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported by this build "
              "(the single-GPU kernels and a sharding design are described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2609_18026_amd import Plan, mlg_timing_enable, mlg_timing_read
    if args.calibrate_copy:
        src = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: calibration copy of 268435456 bytes x3 done")
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
    mlg_timing_enable(plan.handle, True)
    for f in families + ["radial_gemm", "mask"]:
        mlg_timing_read(plan.handle, f)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.rhs_tp(psi, chi, po, co, U=U_FRAME)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
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
        per_kernel[f] = ent
    dom = max(families, key=lambda f: kern[f][0])
    d = per_kernel[dom]
    if work[dom]["flops"]:
        launches = max(kern[dom][1], 1)
        roofline = dict(bound="mfma", kernel=dom, achieved=d["tflops"], peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                        frac=d["frac_fp64_peak"], traffic=None,
                        work_per_launch=work[dom]["flops"] * args.steps / launches, avg_launch_ms=d["avg_launch_ms"])
    else:
        launches = max(kern[dom][1], 1)
        roofline = dict(bound="hbm", kernel=dom, achieved=d["gbs"], peak=PEAK_HBM_GBS, unit="GB/s",
                        frac=d["frac_hbm_peak"], traffic=None,
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
        "transform_pair": {"ms": round(pair_ms, 4), "gdofs": round(n ** 3 / (pair_ms / 1e3) / 1e9, 4)},
    }
    # split-bfloat16 radial products on the same state: time, and the error against the FP64 result
    # at the tap that is well conditioned: the velocity V(psi_N, chi_N) the potentials represent
    from paper_2609_18026_amd import MLG_SPLIT_BF16
    ref_p, ref_c = po.clone(), co.clone()
    splan = Plan(n, n, n, 1.0, PAIR["lz"], dealias=1, prec=MLG_SPLIT_BF16)
    sp, sc = splan.empty_spec(), splan.empty_spec()
    for _ in range(args.warmup):
        splan.rhs_tp(psi, chi, sp, sc, U=U_FRAME)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        splan.rhs_tp(psi, chi, sp, sc, U=U_FRAME)
    e1.record(stream)
    torch.cuda.synchronize()
    sms = e0.elapsed_time(e1) / args.steps
    del splan
    uw_ref = torch.empty(6 * plan.layout.phys_elems, dtype=torch.float64, device="cuda")
    uw_spl = torch.empty_like(uw_ref)
    plan.synthesize(ref_p, ref_c, uw_ref)
    plan.synthesize(sp, sc, uw_spl)
    torch.cuda.synchronize()
    pe = plan.layout.phys_elems
    verr = float(torch.linalg.vector_norm(uw_spl[:3 * pe] - uw_ref[:3 * pe]) / torch.linalg.vector_norm(uw_ref[:3 * pe]))
    cerr = float(torch.linalg.vector_norm(sp - ref_p) / torch.linalg.vector_norm(ref_p))
    out["split_bf16"] = {"ms_per_step": round(sms, 4), "gdofs": round(n ** 3 / (sms / 1e3) / 1e9, 4),
                         "rel_err_velocity_of_output_vs_fp64": verr, "rel_err_psi_coefficients_vs_fp64": cerr}
    log(f"bench: split-bf16 {sms:.3f} ms/step, velocity rel err {verr:.2e} (coefficients {cerr:.2e})")
    out["batched_2d"] = bench_batched(torch, args, stream, e0, e1)
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
