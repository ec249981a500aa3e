"""The binding checks every tensor it hands to the C ABI (dtype, contiguity, element count, device)
and raises ValueError before any native call; a buffer that passes the checks reaches the library,
which rejects the null plan handle used here with its own error.  CPU only: the plan objects are
built without a device (no native plan exists)."""
import pytest
import torch

from paper_2609_18026_amd import binding as B


def _fake_plan(phys=24, spec=10, nz=2, real_bytes=8):
    p = object.__new__(B.Plan)
    p.handle = 0
    p.device = 0
    p.nr, p.nphi, p.nz = 3, 4, nz
    p.layout = B.mlg_layout(phys, 5, spec, 64, 2, 3, 1, real_bytes, 1, 0)
    p.rdtype = torch.float32 if real_bytes == 4 else torch.float64
    p.cdtype = torch.complex64 if real_bytes == 4 else torch.complex128
    p.ws = torch.empty(64, dtype=torch.uint8)
    return p


@pytest.fixture
def host_buffers(monkeypatch):
    """Treat host tensors as the library's device so that every check after the device check runs."""
    monkeypatch.setattr(B, "_DEVICE_TYPE", "cpu")


def _raises(fn, *args, match):
    with pytest.raises(ValueError, match=match):
        fn(*args)


def test_wrong_dtype_contiguity_and_size_are_rejected(host_buffers):
    p = _fake_plan()
    phys = torch.zeros(24, dtype=torch.float64)
    spec = torch.zeros(10, dtype=torch.complex128)
    _raises(p.forward, phys.float(), spec, match="phys: dtype")
    _raises(p.forward, phys, spec.to(torch.complex64), match="spec: dtype")
    _raises(p.backward, spec[:9], phys, match="spec: 9 elements")
    _raises(p.backward, spec, torch.zeros(48, dtype=torch.float64)[::2], match="phys: tensor must be contiguous")
    _raises(p.rhs_tp, spec, spec, spec, spec[:5], match="chi_n: 5 elements")
    _raises(p.rhs_tp, spec, spec, spec, spec, None, torch.zeros(3, dtype=torch.float64), match="taps: 3 elements")
    _raises(p.synthesize, spec, spec, torch.zeros(6 * 24 - 1, dtype=torch.float64), match="uw:")
    _raises(p.advance, spec, spec, spec, spec, 1, 1, None, None, torch.zeros(59, dtype=torch.complex128),
            match="tmp: 59 elements, need at least 60")
    _raises(p.advance_scalar, 1, 0.25, spec, spec, 1, 0, torch.zeros(29, dtype=torch.complex128),
            match="tmp: 29 elements")
    _raises(p.energy, spec, spec, torch.zeros(1, dtype=torch.float64), match="out: 1 elements")
    _raises(p.step_abcn, spec, spec, spec.real.contiguous(), spec, match="A_prev: dtype")


def test_host_tensors_are_rejected_before_the_library_is_called():
    p = _fake_plan()
    phys = torch.zeros(24, dtype=torch.float64)
    spec = torch.zeros(10, dtype=torch.complex128)
    _raises(p.forward, phys, spec, match="phys: tensor on cpu, expected cuda:0")
    _raises(p.rhs_scalar, 1, 0.25, spec, spec, match="spec_u: tensor on cpu")
    _raises(p.filter_apply, 0, spec, match="spec: tensor on cpu")


def test_fp32_plan_expects_single_precision_buffers(host_buffers):
    p = _fake_plan(real_bytes=4)
    _raises(p.forward, torch.zeros(24, dtype=torch.float64), torch.zeros(10, dtype=torch.complex64),
            match="phys: dtype torch.float64, expected torch.float32")
    _raises(p.forward, torch.zeros(24, dtype=torch.float32), torch.zeros(10, dtype=torch.complex128),
            match="spec: dtype torch.complex128, expected torch.complex64")


def test_batch_and_closure_buffers_are_checked(host_buffers):
    b = object.__new__(B.Batch)
    b.handle, b.device, b.count = 0, 0, 2
    b.offsets = [0, 4, 9]
    b.cdtype = torch.complex128
    b.ws = torch.empty(8, dtype=torch.uint8)
    _raises(b.rhs_kpp, 0.25, torch.zeros(8, dtype=torch.complex128), torch.zeros(9, dtype=torch.complex128),
            match="spec_in: 8 elements, need at least 9")
    _raises(b.rhs_kpp, 0.25, torch.zeros(9, dtype=torch.complex64), torch.zeros(9, dtype=torch.complex128),
            match="spec_in: dtype")
    c = object.__new__(B.Closure)
    c.handle, c.ncols, c.max_batch = 0, 3, 8
    c.plan = _fake_plan()
    _raises(c.features, torch.zeros(10, dtype=torch.complex128), torch.zeros(10, dtype=torch.complex128),
            torch.zeros(3 * B.MLG_CLOSURE_NIN - 1, dtype=torch.float32), match="x_out:")
    _raises(c.forward, torch.zeros(2, B.MLG_CLOSURE_NIN, dtype=torch.float64),
            torch.zeros(2, B.MLG_CLOSURE_NOUT, dtype=torch.float32), match="x: dtype")
    _raises(c.train_step, torch.zeros(4, B.MLG_CLOSURE_NIN), torch.zeros(4, B.MLG_CLOSURE_NOUT),
            torch.zeros(4, dtype=torch.int64), 4, 1e-3, match="idx: dtype")


def test_valid_buffers_reach_the_library(host_buffers, monkeypatch):
    # with every check passed the call goes through to the C ABI, which rejects the null plan itself
    monkeypatch.setattr(B.Plan, "_stream", staticmethod(lambda: 0))
    p = _fake_plan()
    with pytest.raises(B.MlgError, match="MLG_E_ARG"):
        p.forward(torch.zeros(24, dtype=torch.float64), torch.zeros(10, dtype=torch.complex128))


def test_finalizing_guard_skips_native_calls(monkeypatch):
    p = _fake_plan()
    p.handle = 12345          # would be passed to mlg_plan_destroy if __del__ ran the close
    called = []
    monkeypatch.setattr(B, "mlg_plan_destroy", lambda h: called.append(h))
    monkeypatch.setattr(B, "_finalizing", lambda: True)
    p.__del__()
    assert called == []
    monkeypatch.setattr(B, "_finalizing", lambda: False)
    p.__del__()
    assert called == [12345] and p.handle == 0
