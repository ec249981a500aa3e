"""mlg_rhs_tp_noalloc (the entry point for callers that cannot allocate) against mlg_rhs_tp.

Both run the same kernels, the first on the library's fixed per-GPU workspace and the second on a
caller workspace, so the outputs must agree exactly (the FP64 bar of 1e-12 is met with zero
difference).  Two calls in a row on the same GPU, the second on a smaller grid, check that the fixed
workspace carries nothing from one call into the next; a plan whose workspace exceeds the fixed size
and a plan with timing enabled are refused with an error.
"""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_18026_amd import binding as B
    return B


def _spectra(plan, seed):
    L = plan.layout
    S1 = synth.geometric_spectrum(L.M, L.nrc, plan.nz, L.nzc, seed=seed, a=0.8, b=0.8, c=0.8)
    S2 = synth.geometric_spectrum(L.M, L.nrc, plan.nz, L.nzc, seed=seed + 1, a=0.8, b=0.8, c=0.8)
    return (torch.from_numpy(synth.to_packed(S1)).cuda(), torch.from_numpy(synth.to_packed(S2)).cuda())


def _both(B, plan, psi, chi, U, with_taps):
    a, b = plan.empty_spec(), plan.empty_spec()
    c, d = torch.full_like(a, np.nan), torch.full_like(b, np.nan)
    ta = plan.taps_buffer() if with_taps else None
    tb = plan.taps_buffer() if with_taps else None
    plan.rhs_tp(psi, chi, a, b, U=U, taps=ta)
    s = torch.cuda.current_stream().cuda_stream
    B.mlg_rhs_tp_noalloc(plan.handle, U, plan._spec(psi, "psi"), plan._spec(chi, "chi"), plan._spec(c, "psi_n"),
                         plan._spec(d, "chi_n"), 0 if tb is None else tb.data_ptr(), s)
    torch.cuda.synchronize()
    return (a, b, ta), (c, d, tb)


def test_noalloc_matches_rhs_tp_on_two_calls_the_second_smaller():
    B = _mods()
    U = (0.3, -0.7, 0.2)
    for shape, seed, taps in (((64, 48, 32), 11, True), ((20, 16, 8), 13, False)):
        nr, nphi, nz = shape
        _say("rhs_tp_noalloc vs rhs_tp", shape)
        plan = B.Plan(nr, nphi, nz, 1.1, 4.0)
        try:
            psi, chi = _spectra(plan, seed)
            (a, b, ta), (c, d, tb) = _both(B, plan, psi, chi, U, taps)
            for x, y in ((a, c), (b, d)):
                assert torch.isfinite(torch.view_as_real(y)).all()
                err = float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(x))
                _say("  rel diff", err)
                assert err <= 1e-12
                assert torch.equal(x, y)
            if taps:
                assert torch.equal(ta, tb)
        finally:
            plan.close()


def test_noalloc_refuses_oversized_plans_and_timing():
    B = _mods()
    big = B.Plan(256, 256, 256, 1.0, 8.6)
    try:
        assert big.layout.workspace_bytes > 192 * 2 ** 20
        e = big.empty_spec()
        with pytest.raises(B.MlgError, match="MLG_E_UNSUPPORTED"):
            B.mlg_rhs_tp_noalloc(big.handle, None, e.data_ptr(), e.data_ptr(), e.data_ptr(), e.data_ptr(), 0, 0)
    finally:
        big.close()
    p = B.Plan(16, 8, 4, 1.0)
    try:
        psi, chi = _spectra(p, 3)
        o1, o2 = p.empty_spec(), p.empty_spec()
        B.mlg_timing_enable(p.handle, True)
        with pytest.raises(B.MlgError, match="MLG_E_ARG"):
            B.mlg_rhs_tp_noalloc(p.handle, None, psi.data_ptr(), chi.data_ptr(), o1.data_ptr(), o2.data_ptr(), 0, 0)
        B.mlg_timing_enable(p.handle, False)
        B.mlg_rhs_tp_noalloc(p.handle, None, psi.data_ptr(), chi.data_ptr(), o1.data_ptr(), o2.data_ptr(), 0,
                             torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(o1)).all()
    finally:
        p.close()
