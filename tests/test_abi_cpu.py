"""C-ABI checks that need no GPU: the library loads, exports every declared entry point,
and rejects malformed grids before touching a device (Sec. 3.1 chop bounds, ell > 0)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "mlg.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"\b(mlg_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2609_18026_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2609_18026_amd import build
        build.build()
    return binding.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "mlg_forward" in names and "mlg_rhs_tp" in names
    for n in names:
        assert hasattr(L, n), n


def test_binding_names_match_header():
    from paper_2609_18026_amd import binding
    for n in _declared():
        assert n in binding.EXPORTS and callable(getattr(binding, n)), n


@pytest.mark.parametrize("kw,status", [
    (dict(ell=0.0), 1), (dict(ell=-1.0), 1), (dict(ell=math.nan), 5), (dict(lz=math.inf), 5),
    (dict(nr=1), 1), (dict(nrc=40), 1), (dict(nphic=10), 1), (dict(nzc=4), 1), (dict(dealias=2), 1),
    (dict(nphi=14), 4), (dict(nz=7), 4), (dict(nphi=2048), 4),
])
def test_plan_create_rejects_bad_grids(L, kw, status):
    from paper_2609_18026_amd import binding
    args = dict(nr=32, nphi=16, nz=4, nrc=0, nphic=0, nzc=0, ell=1.0, lz=2 * math.pi, dealias=1)
    args.update(kw)
    g = binding.mlg_grid(args["nr"], args["nphi"], args["nz"], args["nrc"], args["nphic"], args["nzc"],
                         args["ell"], args["lz"], args["dealias"])
    h = ctypes.c_void_p(1234)
    st = L.mlg_plan_create(ctypes.byref(g), 0, 0, ctypes.byref(h))
    assert st == status, binding.mlg_last_error()
    assert h.value is None
    assert len(binding.mlg_last_error()) > 0


def test_null_arguments_rejected(L):
    assert L.mlg_plan_create(None, 0, 0, None) == 1
    assert L.mlg_forward(None, None, None, None, None) == 1
    assert L.mlg_rhs_tp(None, None, None, None, None, None, None, None, None) == 1
    assert L.mlg_plan_destroy(None) == 0
    assert L.mlg_filter_setup(None, None) == 1
    assert L.mlg_filter_apply(None, 0, None, None) == 1
    assert L.mlg_filter_state(None, None) == 1
