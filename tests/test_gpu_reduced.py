"""Reduced-precision plans (MLG_FP32, MLG_SPLIT_BF16) against the FP64 oracle, at the 256-point
azimuthal and axial sizes they support.

Both keep their data as float / complex64 (half the bytes of every stage).  The radial products of
the transform pair, the scalar term and the vector synthesis run on FP32 MFMA with FP32 tables
(MLG_FP32) or as hi_a hi_b + hi_a lo_b + lo_a hi_b of bfloat16 parts with FP32 accumulation
(MLG_SPLIT_BF16, whose z transforms of those stages are radix-16 DFT products in the same
arithmetic); the FFTs and pointwise products compute in FP64 on float-stored intermediates; the
projection's source products and elliptic solves compute in FP64 from the float-stored N (the
solves are ill-conditioned along the far-field directions of the Gram matrices, cond ~1e9 at
N_r = 256, and reduced-precision source products there were amplified into O(1) output errors).

The oracle runs on the float-rounded inputs the library sees, so every error below is the library's
own arithmetic.  Bounds (normwise relative; measured values in brackets):
  * transforms, scalar RHS, nodal u, omega and N: 1e-6 for FP32 [<= 1.9e-7], 3e-5 for split
    [<= 9.3e-6];
  * nonlinear term: its velocity V(psi_N, chi_N) relative to |N| (the projection is a contraction
    in the continuous L2 norm, so it does not enlarge the error of N): 1e-5 [<= 4.9e-6]; relative
    to V itself the error grows by |N| / |P N|: 1e-4 [<= 1.4e-5].
At 256^3 (the bench plan) the oracle checks sampled outputs stage by stage as for FP64 plans: forward
columns, backward points, nodal u and omega at points, N at every node from the library's u and
omega, the Galerkin sources at columns from the library's N, and the backward error of the solves
from the library's sources and float outputs (2.5e-7: rounding the FP64 solution to float moves
it by at most 2^-24 of its norm, which bounds the backward error by the same).  The sources are a
cancelling residual of N for this near-steady pair (|C| ~ |N| / 90), so the float storage of the
harmonics of N (2^-24) reaches them amplified: 2e-5 [4.7e-6 FP32, 3.7e-6 split].
"""
import functools

import numpy as np
import pytest

import synth
from helpers import from_lib, rel, to_lib
from oracle.grid import Grid
from oracle.rhs import (VecTables, cross_with_background, dealias_mask, projection_sources_columns, rhs_scalar, rhs_tp,
                        synthesize, synthesize_points)
from oracle.transform import Tables, backward, backward_points, forward, forward_columns

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (MLG_FP32 = 1, MLG_SPLIT_BF16 = 2) -> bound of the transform-type stages
STAGE_TOL = {1: 1e-6, 2: 3e-5}
NAMES = {1: "fp32", 2: "split-bf16"}


def _say(*a):
    print(*a, flush=True)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_18026_amd as m
    return m


def _c64(S):
    """Round an oracle spectrum to complex64 and back: the values a float plan is given."""
    return S.astype(np.complex64).astype(np.complex128)


SCALAR_CASES = [
    # nr, ell, lz, nrc, dealias, kind
    (24, 1.1, 3.0, 0, 1, "u2"),
    (40, 0.8, 5.0, 36, 0, "kpp"),     # radial chop; 20 folded rows: one full 16-row tile and a tail
]


@functools.lru_cache(maxsize=None)
def _scalar_oracle(case):
    nr, ell, lz, nrc, dealias, kind = case
    g = Grid(nr, 256, 256, ell, lz=lz, nrc=nrc)
    t = Tables(g)
    s = np.random.default_rng(200 + nr).standard_normal((256, nr, 256)).astype(np.float32)
    C = _c64(synth.geometric_spectrum(g.M, g.nrc, 256, g.nzc, seed=8, a=0.9, b=0.9, c=0.9))
    return g, s, forward(s.astype(np.float64), g, t), C, backward(C, g, t), \
        rhs_scalar(C, g, t, kind, 0.25, dealias=bool(dealias))


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("case", SCALAR_CASES)
def test_reduced_transforms_and_scalar(case, prec):
    m = _gpu()
    nr, ell, lz, nrc, dealias, kind = case
    _say(NAMES[prec], "transforms and scalar RHS", case)
    g, s, F, C, B, R = _scalar_oracle(case)
    plan = m.Plan(nr, 256, 256, ell, lz, nrc=nrc, dealias=dealias, prec=prec)
    try:
        assert plan.rdtype == torch.float32 and plan.cdtype == torch.complex64
        errs = {}
        spec = plan.empty_spec()
        plan.forward(torch.from_numpy(s).cuda(), spec)
        phys = plan.empty_phys()
        Cd = torch.from_numpy(to_lib(C).astype(np.complex64)).cuda()
        plan.backward(Cd, phys)
        out = plan.empty_spec()
        plan.rhs_scalar(m.MLG_RHS_U2 if kind == "u2" else m.MLG_RHS_KPP, 0.25, Cd, out)
        torch.cuda.synchronize()
        errs["forward"] = rel(from_lib(spec.cpu().numpy().astype(np.complex128), g.M, g.nrc), F)
        errs["backward"] = rel(phys.cpu().numpy().astype(np.float64), B)
        got = from_lib(out.cpu().numpy().astype(np.complex128), g.M, g.nrc)
        errs["rhs_scalar"] = rel(got, R)
    finally:
        plan.close()
    _say("  relative errors:", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < STAGE_TOL[prec], (k, v)
    if dealias:
        assert np.all(got[g.dealias_m() + 1:] == 0)


TP_CASES = [
    # nr, ell, lz, U, dealias, nrc
    (24, 0.9, 3.0, (0.3, -0.2, 0.5), 1, 0),
    (40, 1.2, 8.6, (0.0, 1.0, 0.0), 0, 36),
]


@functools.lru_cache(maxsize=None)
def _tp_oracle(case):
    nr, ell, lz, U, dealias, nrc = case
    g = Grid(nr, 256, 256, ell, lz=lz, nrc=nrc)
    vt = VecTables(g)
    psi = _c64(synth.geometric_spectrum(g.M, g.nrc, 256, g.nzc, seed=2, a=0.9, b=0.85, c=0.85))
    chi = _c64(synth.geometric_spectrum(g.M, g.nrc, 256, g.nzc, seed=3, a=0.9, b=0.85, c=0.85))
    taps = {}
    ref_psi, ref_chi = rhs_tp(psi, chi, g, vt, U=U, dealias=bool(dealias), taps=taps)
    v_ref, _ = synthesize(ref_psi, ref_chi, g, vt)
    return g, vt, psi, chi, taps, ref_psi, ref_chi, np.stack(v_ref)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("case", TP_CASES)
def test_reduced_rhs_tp(case, prec):
    m = _gpu()
    nr, ell, lz, U, dealias, nrc = case
    _say(NAMES[prec], "rhs_tp", case)
    g, vt, psi, chi, taps, ref_psi, ref_chi, v_ref = _tp_oracle(case)
    plan = m.Plan(nr, 256, 256, ell, lz, nrc=nrc, dealias=dealias, prec=prec)
    try:
        tp = plan.taps_buffer()
        po, co = plan.empty_spec(), plan.empty_spec()
        plan.rhs_tp(torch.from_numpy(to_lib(psi).astype(np.complex64)).cuda(),
                    torch.from_numpy(to_lib(chi).astype(np.complex64)).cuda(), po, co, U=U, taps=tp)
        torch.cuda.synchronize()
        pe = plan.layout.phys_elems
        tn = tp.cpu().numpy()
        gp = from_lib(po.cpu().numpy().astype(np.complex128), g.M, g.nrc)
        gc = from_lib(co.cpu().numpy().astype(np.complex128), g.M, g.nrc)
    finally:
        plan.close()
    nodal = tn[:9 * pe].reshape(9, 256, nr, 256)
    errs = {}
    names = ["u_r", "u_phi", "u_z", "w_r", "w_phi", "w_z", "N_r", "N_phi", "N_z"]
    refs = list(taps["u"]) + list(taps["w"]) + list(taps["N"])
    for i, nm in enumerate(names):
        errs[nm] = rel(nodal[i], refs[i])
    errs["psi_N"] = rel(gp, ref_psi)
    errs["chi_N"] = rel(gc, ref_chi)
    v_got = np.stack(synthesize(gp, gc, g, vt)[0])
    errs["V(psi_N,chi_N)"] = rel(v_got, v_ref)
    nN = np.linalg.norm(np.stack(list(taps["N"])).ravel())
    errs["V err / |N|"] = np.linalg.norm((v_got - v_ref).ravel()) / nN
    _say("  relative errors:", {k: f"{v:.2e}" for k, v in errs.items()})
    for nm in names:
        assert errs[nm] < STAGE_TOL[prec], (nm, errs[nm])
    assert errs["V err / |N|"] < 1e-5, errs["V err / |N|"]
    assert errs["V(psi_N,chi_N)"] < 1e-4, errs["V(psi_N,chi_N)"]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [1, 2])
def test_reduced_full_size_256_sampled(prec):
    m = _gpu()
    from test_gpu_full_size import ELL, LZ, N, U, _column_backward_error, _pick_columns, _points
    tol = STAGE_TOL[prec]
    _say(NAMES[prec], "256^3 sampled parity: setup")
    g = Grid(N, N, N, ELL, lz=LZ)
    plan = m.Plan(N, N, N, ELL, LZ, dealias=1, prec=prec)
    try:
        f = synth.vortex_pair_psi(g.r, g.phi, g.z, lz=LZ).astype(np.float32)
        psi = plan.empty_spec()
        plan.forward(torch.from_numpy(np.ascontiguousarray(f)).cuda(), psi)
        chi_host = _c64(1e-2 * synth.geometric_spectrum(g.M, g.nrc, g.nz, g.nzc, seed=9, a=0.9, b=0.85, c=0.85))
        chi = torch.from_numpy(to_lib(chi_host).astype(np.complex64)).cuda()
        torch.cuda.synchronize()
        psi_host = from_lib(psi.cpu().numpy().astype(np.complex128), g.M, g.nrc)
        f64 = f.astype(np.float64)

        cols = _pick_columns(psi_host, 6, 4, seed=5)
        _say("  forward columns", cols)
        fc = forward_columns(f64, g, cols)
        err = rel(np.concatenate([psi_host[mm, :, kk] for mm, kk in cols]), np.concatenate([fc[c] for c in cols]))
        _say("  forward columns rel", err)
        assert err < tol

        pts = _points(g, 16, seed=11)
        phys = plan.empty_phys()
        plan.backward(psi, phys)
        torch.cuda.synchronize()
        ph = phys.cpu().numpy()
        del phys
        err = rel(np.array([ph[l, i, j] for l, i, j in pts], dtype=np.float64), backward_points(psi_host, g, pts))
        _say("  backward points rel", err)
        assert err < tol
        del ph

        _say("  rhs_tp with taps")
        tp = plan.taps_buffer()
        po, co = plan.empty_spec(), plan.empty_spec()
        plan.rhs_tp(psi, chi, po, co, U=U, taps=tp)
        torch.cuda.synchronize()
        pe = plan.layout.phys_elems
        tn = tp.cpu().numpy()
        del tp
        pl = from_lib(po.cpu().numpy().astype(np.complex128), g.M, g.nrc)
        cl = from_lib(co.cpu().numpy().astype(np.complex128), g.M, g.nrc)
        tau = plan.tau
    finally:
        plan.close()
    nodal = tn[:9 * pe].reshape(9, N, N, N)
    src = tn[9 * pe:].view(np.complex128).reshape(3, tau, N)
    vt = VecTables(g)
    # the RHS synthesizes the potentials through the two-thirds mask (the fields entering the product)
    from oracle.rhs import apply_mask
    sp = synthesize_points(apply_mask(psi_host, g), apply_mask(chi_host, g), g, vt, pts)
    err = rel(np.array([[nodal[f][l, i, j] for l, i, j in pts] for f in range(6)]), sp)
    _say("  nodal u, w at points rel", err)
    assert err < tol
    Nref = cross_with_background(nodal[0:3], nodal[3:6], U, g)
    for c in range(3):
        e = rel(nodal[6 + c], Nref[c])
        _say("  N", c, "rel", e)
        assert e < 1e-12
    del Nref
    Cl, Kl, Zl = (from_lib(src[i], g.M, g.nrc) for i in range(3))
    acols = _pick_columns(Cl, 5, 4, seed=6, allowed=dealias_mask(g)) + [(0, 0), (85, 85)]
    _say("  sources at columns", acols)
    pc = projection_sources_columns(nodal[6], nodal[7], nodal[8], g, vt, acols)
    for i, name in enumerate(("C", "K", "Z")):
        e = rel(np.concatenate([(Cl, Kl, Zl)[i][mm, :, kk] for mm, kk in acols]),
                np.concatenate([pc[c][i] for c in acols]))
        _say("  source", name, "rel", e)
        assert e < 2e-5
    worst = max(_column_backward_error(g, mm, kk, pl[mm, :, kk], cl[mm, :, kk], Cl[mm, :, kk], Kl[mm, :, kk],
                                       Zl[mm, :, kk]) for mm, kk in acols)
    _say("  solve backward error", worst)
    assert worst < 2.5e-7


def test_reduced_plan_limits():
    m = _gpu()
    for prec in (1, 2):
        for shape in ((24, 128, 256), (24, 256, 64), (25, 256, 256)):
            with pytest.raises(m.MlgError) as ei:
                m.Plan(*shape, prec=prec)
            assert ei.value.status == 4, (prec, shape)
        plan = m.Plan(16, 256, 256, prec=prec)
        try:
            a, b = plan.empty_spec(), plan.empty_spec()
            a.zero_()
            with pytest.raises(m.MlgError) as ei:
                plan.remove_far_field(a)
            assert ei.value.status == 4
            with pytest.raises(m.MlgError) as ei:
                plan.laplacian_solve(a, b)
            assert ei.value.status == 4
            # the logarithmic proxy fields are added in FP64 kernels: nonzero amplitudes are refused
            with pytest.raises(m.MlgError):
                plan.set_log_proxy(1.0, 0.0)
        finally:
            plan.close()
