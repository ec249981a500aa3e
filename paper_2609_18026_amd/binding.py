"""ctypes binding of include/mlg.h.

Functions named like the C entry points take plain integers for device pointers
and streams (e.g. ``tensor.data_ptr()``, ``torch.cuda.current_stream().cuda_stream``)
and raise ``MlgError`` on a non-zero status.  ``Plan`` is a small convenience
wrapper that allocates its workspace as a torch tensor on the plan's device.
"""
from __future__ import annotations

import ctypes
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlg.so")

MLG_FP64, MLG_FP32, MLG_SPLIT_BF16 = 0, 1, 2
MLG_RHS_U2, MLG_RHS_KPP = 0, 1

_STATUS = {0: "MLG_OK", 1: "MLG_E_ARG", 2: "MLG_E_ALLOC", 3: "MLG_E_DEVICE", 4: "MLG_E_UNSUPPORTED",
           5: "MLG_E_NONFINITE"}


class MlgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class mlg_grid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nphi", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nrc", ctypes.c_int32), ("nphic", ctypes.c_int32), ("nzc", ctypes.c_int32),
                ("ell", ctypes.c_double), ("lz", ctypes.c_double), ("dealias", ctypes.c_int32)]


class mlg_layout(ctypes.Structure):
    _fields_ = [("phys_elems", ctypes.c_int64), ("spec_rows", ctypes.c_int64), ("spec_elems", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("M", ctypes.c_int32), ("nrc", ctypes.c_int32),
                ("nzc", ctypes.c_int32), ("real_bytes", ctypes.c_int32), ("dealias_m", ctypes.c_int32),
                ("dealias_k", ctypes.c_int32)]


_lib = None

EXPORTS = ["mlg_plan_create", "mlg_plan_destroy", "mlg_plan_query", "mlg_plan_nodes", "mlg_forward",
           "mlg_backward", "mlg_rhs_scalar", "mlg_rhs_tp", "mlg_rhs_tp_noalloc", "mlg_synthesize", "mlg_tp_energy", "mlg_timing_enable",
           "mlg_timing_read",
           "mlg_batch_create", "mlg_batch_destroy", "mlg_batch_query", "mlg_batch_rhs_scalar", "mlg_batch_set_config",
           "mlg_batch_get_config", "mlg_batch_autotune", "mlg_step_setup", "mlg_step_febe", "mlg_step_abcn",
           "mlg_truncate", "mlg_tp_advance", "mlg_filter_setup", "mlg_filter_apply", "mlg_filter_state",
           "mlg_eval_harmonic", "mlg_scalar_advance", "mlg_set_log_proxy", "mlg_tp_enstrophy",
           "mlg_laplacian_solve", "mlg_remove_far_field",
           "mlg_closure_param_count", "mlg_closure_create", "mlg_closure_destroy",
           "mlg_closure_columns", "mlg_closure_set_params", "mlg_closure_get_params", "mlg_closure_get_grads",
           "mlg_closure_set_scales", "mlg_closure_get_scales", "mlg_closure_features", "mlg_closure_targets",
           "mlg_closure_forward", "mlg_closure_train_step", "mlg_closure_infer", "mlg_closure_stats",
           "mlg_closure_set_reference",
           "mlg_last_error"]

MLG_CLOSURE_NIN, MLG_CLOSURE_NOUT, MLG_CLOSURE_HIDDEN = 258, 256, 256


class mlg_closure_cfg(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("beta", ctypes.c_double)]


class mlg_dissip(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("nu_h", ctypes.c_double), ("p", ctypes.c_int32), ("dt", ctypes.c_double)]


class mlg_filter_cfg(ctypes.Structure):
    _fields_ = [("zeta_c", ctypes.c_double), ("tau", ctypes.c_double), ("eps_max", ctypes.c_double),
                ("relax", ctypes.c_double)]


class mlg_batch_config(ctypes.Structure):
    _fields_ = [("recurrence", ctypes.c_int32), ("threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lines", ctypes.c_int32)]


def lib() -> ctypes.CDLL:
    """Load libmlg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_2609_18026_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.mlg_plan_create.argtypes = [ctypes.POINTER(mlg_grid), i32, i32, ctypes.POINTER(vp)]
    L.mlg_plan_destroy.argtypes = [vp]
    L.mlg_plan_query.argtypes = [vp, ctypes.POINTER(mlg_layout)]
    L.mlg_plan_nodes.argtypes = [vp, vp, vp, vp]
    L.mlg_forward.argtypes = [vp, vp, vp, vp, vp]
    L.mlg_backward.argtypes = [vp, vp, vp, vp, vp]
    L.mlg_rhs_scalar.argtypes = [vp, i32, f64, vp, vp, vp, vp]
    L.mlg_rhs_tp.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mlg_rhs_tp_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.mlg_synthesize.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mlg_tp_energy.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mlg_timing_enable.argtypes = [vp, i32]
    L.mlg_timing_read.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)]
    L.mlg_batch_create.argtypes = [i32, ctypes.POINTER(mlg_grid), i32, i32, ctypes.POINTER(vp)]
    L.mlg_batch_destroy.argtypes = [vp]
    L.mlg_batch_query.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64)]
    L.mlg_batch_rhs_scalar.argtypes = [vp, f64, vp, vp, vp, vp]
    L.mlg_batch_set_config.argtypes = [vp, ctypes.POINTER(mlg_batch_config)]
    L.mlg_batch_get_config.argtypes = [vp, ctypes.POINTER(mlg_batch_config)]
    L.mlg_batch_autotune.argtypes = [vp, f64, vp, vp, vp, vp, ctypes.POINTER(mlg_batch_config),
                                     ctypes.POINTER(f64)]
    L.mlg_step_setup.argtypes = [vp, ctypes.POINTER(mlg_dissip)]
    L.mlg_step_febe.argtypes = [vp, i32, vp, vp, vp, vp]
    L.mlg_step_abcn.argtypes = [vp, vp, vp, vp, vp, vp]
    i64, f32 = ctypes.c_int64, ctypes.c_float
    L.mlg_truncate.argtypes = [vp, vp, vp, vp, vp]
    L.mlg_tp_advance.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp]
    L.mlg_filter_setup.argtypes = [vp, ctypes.POINTER(mlg_filter_cfg)]
    L.mlg_filter_apply.argtypes = [vp, i32, vp, vp]
    L.mlg_filter_state.argtypes = [vp, ctypes.POINTER(f64)]
    L.mlg_eval_harmonic.argtypes = [vp, vp, i32, i32, vp, ctypes.c_int64, vp, vp]
    L.mlg_scalar_advance.argtypes = [vp, i32, f64, vp, vp, i32, i32, vp, vp, vp]
    L.mlg_set_log_proxy.argtypes = [vp, f64, f64]
    L.mlg_laplacian_solve.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.mlg_remove_far_field.argtypes = [vp, vp, vp]
    L.mlg_tp_enstrophy.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mlg_closure_param_count.argtypes = []
    L.mlg_closure_create.argtypes = [ctypes.POINTER(mlg_closure_cfg), vp, ctypes.POINTER(vp)]
    L.mlg_closure_destroy.argtypes = [vp]
    L.mlg_closure_columns.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mlg_closure_set_params.argtypes = [vp, vp]
    L.mlg_closure_get_params.argtypes = [vp, vp]
    L.mlg_closure_get_grads.argtypes = [vp, vp]
    L.mlg_closure_set_scales.argtypes = [vp, vp, vp]
    L.mlg_closure_get_scales.argtypes = [vp, vp, vp]
    L.mlg_closure_features.argtypes = [vp, vp, vp, vp, vp]
    L.mlg_closure_targets.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.mlg_closure_forward.argtypes = [vp, vp, i32, vp, vp]
    L.mlg_closure_train_step.argtypes = [vp, vp, vp, vp, i64, i32, f32, ctypes.POINTER(f32), vp]
    L.mlg_closure_infer.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int32), vp]
    L.mlg_closure_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.mlg_closure_set_reference.argtypes = [vp, vp, vp]
    for name in EXPORTS[:-1]:
        getattr(L, name).restype = ctypes.c_int
    L.mlg_last_error.restype = ctypes.c_char_p
    L.mlg_last_error.argtypes = []
    _lib = L
    return L


def mlg_last_error() -> str:
    return lib().mlg_last_error().decode()


def _check(status: int) -> None:
    if status != 0:
        raise MlgError(status, mlg_last_error())


_DEVICE_TYPE = "cuda"        # where the library's buffers live (the CPU tests of the checks substitute "cpu")


def _ptr(t, name: str, dtypes, numel: int, device: int) -> int:
    """data_ptr() of a tensor the library will read or write, after checking it against what the
    entry point assumes: one of 'dtypes', contiguous, on cuda:'device', at least 'numel' elements.
    A mismatch raises ValueError before any native call (a wrong buffer would make the kernels
    access memory outside it)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {' or '.join(str(d) for d in dtypes)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, need at least {numel}")
    if t.device.type != _DEVICE_TYPE or (t.device.index if t.device.index is not None else 0) != device:
        raise ValueError(f"{name}: tensor on {t.device}, expected {_DEVICE_TYPE}:{device}")
    return t.data_ptr()


def _finalizing() -> bool:
    return sys.is_finalizing()


def mlg_plan_create(grid: mlg_grid, prec: int = MLG_FP64, device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().mlg_plan_create(ctypes.byref(grid), prec, device, ctypes.byref(h)))
    return h.value


def mlg_plan_destroy(plan: int) -> None:
    _check(lib().mlg_plan_destroy(plan))


def mlg_plan_query(plan: int) -> mlg_layout:
    out = mlg_layout()
    _check(lib().mlg_plan_query(plan, ctypes.byref(out)))
    return out


def mlg_plan_nodes(plan: int, nr: int):
    import numpy as np
    x = np.zeros(nr)
    w = np.zeros(nr)
    r = np.zeros(nr)
    _check(lib().mlg_plan_nodes(plan, x.ctypes.data, w.ctypes.data, r.ctypes.data))
    return x, w, r


def mlg_forward(plan: int, phys: int, spec: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_forward(plan, phys, spec, ws, stream))


def mlg_backward(plan: int, spec: int, phys: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_backward(plan, spec, phys, ws, stream))


def mlg_rhs_scalar(plan: int, kind: int, gamma: float, spec_u: int, spec_out: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_rhs_scalar(plan, kind, gamma, spec_u, spec_out, ws, stream))


def mlg_rhs_tp(plan: int, U, psi: int, chi: int, psi_n: int, chi_n: int, taps: int, ws: int,
               stream: int = 0) -> None:
    Uarr = None
    if U is not None:
        Uarr = (ctypes.c_double * 3)(*[float(u) for u in U])
    _check(lib().mlg_rhs_tp(plan, Uarr, psi, chi, psi_n, chi_n, taps, ws, stream))


def mlg_rhs_tp_noalloc(plan: int, U, psi: int, chi: int, psi_n: int, chi_n: int, taps: int, stream: int = 0) -> None:
    Uarr = None
    if U is not None:
        Uarr = (ctypes.c_double * 3)(*[float(u) for u in U])
    _check(lib().mlg_rhs_tp_noalloc(plan, Uarr, psi, chi, psi_n, chi_n, taps, stream))


def mlg_step_setup(plan: int, nu: float, nu_h: float, p: int, dt: float) -> None:
    d = mlg_dissip(nu, nu_h, p, dt)
    _check(lib().mlg_step_setup(plan, ctypes.byref(d)))


def mlg_filter_setup(plan: int, zeta_c: float, tau: float, eps_max: float, relax: float) -> None:
    c = mlg_filter_cfg(zeta_c, tau, eps_max, relax)
    _check(lib().mlg_filter_setup(plan, ctypes.byref(c)))


def mlg_eval_harmonic(plan: int, spec: int, m: int, kk: int, r: int, npts: int, out: int, stream: int = 0) -> None:
    _check(lib().mlg_eval_harmonic(plan, spec, m, kk, r, npts, out, stream))


def mlg_scalar_advance(plan: int, kind: int, gamma: float, state: int, hist: int, nsteps: int, start: int, tmp: int,
                       ws: int, stream: int = 0) -> None:
    _check(lib().mlg_scalar_advance(plan, kind, gamma, state, hist, nsteps, start, tmp, ws, stream))


MLG_LOG_PRESCRIBE, MLG_LOG_SOLVE = 0, 1


def mlg_laplacian_solve(plan: int, variant: int, f: int, s: int, c: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_laplacian_solve(plan, variant, f, s, c, ws, stream))


def mlg_remove_far_field(plan: int, spec: int, stream: int = 0) -> None:
    _check(lib().mlg_remove_far_field(plan, spec, stream))


def mlg_set_log_proxy(plan: int, c_psi: float, c_chi: float) -> None:
    _check(lib().mlg_set_log_proxy(plan, c_psi, c_chi))


def mlg_tp_enstrophy(plan: int, psi: int, chi: int, out: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_tp_enstrophy(plan, psi, chi, out, ws, stream))


def mlg_filter_disable(plan: int) -> None:
    _check(lib().mlg_filter_setup(plan, None))


def mlg_filter_apply(plan: int, slot: int, spec: int, stream: int = 0) -> None:
    _check(lib().mlg_filter_apply(plan, slot, spec, stream))


def mlg_filter_state(plan: int):
    out = (ctypes.c_double * 4)()
    _check(lib().mlg_filter_state(plan, out))
    return tuple(out)


def mlg_step_febe(plan: int, half: int, s: int, A: int, out: int, stream: int = 0) -> None:
    _check(lib().mlg_step_febe(plan, half, s, A, out, stream))


def mlg_step_abcn(plan: int, s: int, A_now: int, A_prev: int, out: int, stream: int = 0) -> None:
    _check(lib().mlg_step_abcn(plan, s, A_now, A_prev, out, stream))


def mlg_synthesize(plan: int, psi: int, chi: int, uw: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_synthesize(plan, psi, chi, uw, ws, stream))


def mlg_tp_energy(plan: int, psi: int, chi: int, energy: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_tp_energy(plan, psi, chi, energy, ws, stream))


def mlg_timing_enable(plan: int, enable: bool) -> None:
    _check(lib().mlg_timing_enable(plan, 1 if enable else 0))


def mlg_timing_read(plan: int, kernel: str):
    """(total milliseconds, launches) recorded for a kernel family since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().mlg_timing_read(plan, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def mlg_truncate(src_plan: int, dst_plan: int, src: int, dst: int, stream: int = 0) -> None:
    _check(lib().mlg_truncate(src_plan, dst_plan, src, dst, stream))


def mlg_tp_advance(plan: int, U, psi: int, chi: int, hist_psi: int, hist_chi: int, nsteps: int, start: int,
                   closure: int, tmp: int, ws: int, stream: int = 0) -> None:
    u = None if U is None else (ctypes.c_double * 3)(*U)
    _check(lib().mlg_tp_advance(plan, u, psi, chi, hist_psi, hist_chi, nsteps, start, closure or None, tmp, ws,
                                stream))


def mlg_closure_param_count() -> int:
    return int(lib().mlg_closure_param_count())


def mlg_closure_create(plan: int, max_batch: int, beta: float) -> int:
    h = ctypes.c_void_p()
    cfg = mlg_closure_cfg(int(max_batch), float(beta))
    _check(lib().mlg_closure_create(ctypes.byref(cfg), plan, ctypes.byref(h)))
    return h.value


def mlg_closure_destroy(closure: int) -> None:
    _check(lib().mlg_closure_destroy(closure))


def mlg_closure_columns(closure: int) -> int:
    n = ctypes.c_int32()
    _check(lib().mlg_closure_columns(closure, ctypes.byref(n)))
    return n.value


def _f32_host(a, n):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def mlg_closure_set_params(closure: int, params) -> None:
    a = _f32_host(params, mlg_closure_param_count())
    _check(lib().mlg_closure_set_params(closure, a.ctypes.data))


def mlg_closure_get_params(closure: int):
    import numpy as np
    a = np.empty(mlg_closure_param_count(), dtype=np.float32)
    _check(lib().mlg_closure_get_params(closure, a.ctypes.data))
    return a


def mlg_closure_get_grads(closure: int):
    import numpy as np
    a = np.empty(mlg_closure_param_count(), dtype=np.float32)
    _check(lib().mlg_closure_get_grads(closure, a.ctypes.data))
    return a


def mlg_closure_set_scales(closure: int, x_scale, y_scale) -> None:
    xs = _f32_host(x_scale, MLG_CLOSURE_NIN)
    ys = _f32_host(y_scale, MLG_CLOSURE_NOUT)
    _check(lib().mlg_closure_set_scales(closure, xs.ctypes.data, ys.ctypes.data))


def mlg_closure_get_scales(closure: int):
    import numpy as np
    xs = np.empty(MLG_CLOSURE_NIN, dtype=np.float32)
    ys = np.empty(MLG_CLOSURE_NOUT, dtype=np.float32)
    _check(lib().mlg_closure_get_scales(closure, xs.ctypes.data, ys.ctypes.data))
    return xs, ys


def mlg_closure_features(closure: int, psi: int, chi: int, x_out: int, stream: int = 0) -> None:
    _check(lib().mlg_closure_features(closure, psi, chi, x_out, stream))


def mlg_closure_targets(closure: int, ref_psi: int, ref_chi: int, psi_n: int, chi_n: int, y_out: int,
                        stream: int = 0) -> None:
    _check(lib().mlg_closure_targets(closure, ref_psi, ref_chi, psi_n, chi_n, y_out, stream))


def mlg_closure_forward(closure: int, x: int, nb: int, y: int, stream: int = 0) -> None:
    _check(lib().mlg_closure_forward(closure, x, nb, y, stream))


def mlg_closure_train_step(closure: int, data_x: int, data_y: int, idx: int, count: int, nb: int, lr: float,
                           want_loss: bool = False, stream: int = 0):
    loss = ctypes.c_float()
    _check(lib().mlg_closure_train_step(closure, data_x, data_y, idx or None, count, nb, lr,
                                        ctypes.byref(loss) if want_loss else None, stream))
    return loss.value if want_loss else None


def mlg_closure_infer(closure: int, psi: int, chi: int, rhs_psi: int, rhs_chi: int, want_flag: bool = False,
                      stream: int = 0):
    f = ctypes.c_int32()
    _check(lib().mlg_closure_infer(closure, psi, chi, rhs_psi, rhs_chi, ctypes.byref(f) if want_flag else None,
                                   stream))
    return f.value if want_flag else None


def mlg_closure_stats(closure: int):
    c, f = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mlg_closure_stats(closure, ctypes.byref(c), ctypes.byref(f)))
    return c.value, f.value


def mlg_closure_set_reference(closure: int, ref: int, U=None) -> None:
    u = None if U is None else (ctypes.c_double * 3)(*[float(x) for x in U])
    _check(lib().mlg_closure_set_reference(closure, ref or None, u))


class Plan:
    """A plan plus its workspace, for torch tensors on the plan's device.

    Tensors: physical fields are real of shape (N_z, N_r, N_phi); spectral fields are complex of
    shape (tau, N_z) (packed triangular rows, see include/mlg.h): float64 / complex128 on MLG_FP64
    plans, float32 / complex64 on MLG_FP32 and MLG_SPLIT_BF16 plans (``rdtype``, ``cdtype``).
    """

    def __init__(self, nr, nphi, nz=1, ell=1.0, lz=6.283185307179586, nrc=0, nphic=0, nzc=0,
                 dealias=1, prec=MLG_FP64, device=0):
        import torch
        self.grid = mlg_grid(nr, nphi, nz, nrc, nphic, nzc, float(ell), float(lz), int(dealias))
        self.device = device
        self.handle = mlg_plan_create(self.grid, prec, device)
        self.layout = mlg_plan_query(self.handle)
        self.nr, self.nphi, self.nz = nr, nphi, nz
        self.rdtype = torch.float32 if self.layout.real_bytes == 4 else torch.float64
        self.cdtype = torch.complex64 if self.layout.real_bytes == 4 else torch.complex128
        self.ws = torch.empty(max(self.layout.workspace_bytes, 8), dtype=torch.uint8, device=f"cuda:{device}")

    # checked device pointers (see _ptr)
    def _phys(self, t, name="phys", count=1):
        return _ptr(t, name, (self.rdtype,), count * self.layout.phys_elems, self.device)

    def _spec(self, t, name="spec", count=1):
        return _ptr(t, name, (self.cdtype,), count * self.layout.spec_elems, self.device)

    def _f64(self, t, name, numel):
        import torch
        return _ptr(t, name, (torch.float64,), numel, self.device)

    def _ws(self):
        import torch
        return _ptr(self.ws, "workspace", (torch.uint8,), self.layout.workspace_bytes, self.device)

    @property
    def tau(self) -> int:
        return self.layout.spec_rows

    def nodes(self):
        return mlg_plan_nodes(self.handle, self.nr)

    def empty_phys(self):
        import torch
        return torch.empty((self.nz, self.nr, self.nphi), dtype=self.rdtype, device=f"cuda:{self.device}")

    def empty_spec(self):
        import torch
        return torch.empty((self.tau, self.nz), dtype=self.cdtype, device=f"cuda:{self.device}")

    @staticmethod
    def _stream():
        import torch
        return torch.cuda.current_stream().cuda_stream

    def forward(self, phys, spec):
        mlg_forward(self.handle, self._phys(phys), self._spec(spec), self._ws(), self._stream())

    def backward(self, spec, phys):
        mlg_backward(self.handle, self._spec(spec), self._phys(phys), self._ws(), self._stream())

    def rhs_scalar(self, kind, gamma, spec_u, spec_out):
        mlg_rhs_scalar(self.handle, kind, gamma, self._spec(spec_u, "spec_u"), self._spec(spec_out, "spec_out"),
                       self._ws(), self._stream())

    def rhs_tp(self, psi, chi, psi_n, chi_n, U=None, taps=None):
        tp = 0 if taps is None else self._f64(taps, "taps", 9 * self.layout.phys_elems + 6 * self.layout.spec_elems)
        mlg_rhs_tp(self.handle, U, self._spec(psi, "psi"), self._spec(chi, "chi"), self._spec(psi_n, "psi_n"),
                   self._spec(chi_n, "chi_n"), tp, self._ws(), self._stream())

    def synthesize(self, psi, chi, uw):
        """uw: float64 tensor of 6 * phys_elems (u_r, u_phi, u_z, w_r, w_phi, w_z)."""
        mlg_synthesize(self.handle, self._spec(psi, "psi"), self._spec(chi, "chi"),
                       self._f64(uw, "uw", 6 * self.layout.phys_elems), self._ws(), self._stream())

    def energy(self, psi, chi, out=None):
        """Axial modal kinetic energy per FFT slot (float64 device tensor of N_z entries)."""
        import torch
        if out is None:
            out = torch.empty(self.nz, dtype=torch.float64, device=f"cuda:{self.device}")
        mlg_tp_energy(self.handle, self._spec(psi, "psi"), self._spec(chi, "chi"), self._f64(out, "out", self.nz),
                      self._ws(), self._stream())
        return out

    def step_setup(self, nu, nu_h=0.0, p=8, dt=1e-2):
        mlg_step_setup(self.handle, nu, nu_h, p, dt)

    def filter_setup(self, zeta_c=2.0 / 3.0, tau=2e-2, eps_max=36.0, relax=0.1):
        """Enable the adaptive modal filter (both states reset); mlg_tp_advance then filters every step."""
        mlg_filter_setup(self.handle, zeta_c, tau, eps_max, relax)

    def filter_disable(self):
        mlg_filter_disable(self.handle)

    def filter_apply(self, slot, spec):
        mlg_filter_apply(self.handle, slot, self._spec(spec), self._stream())

    def advance_scalar(self, kind, gamma, s, hist, nsteps, start=0, tmp=None):
        """nsteps AB-CN steps of one scalar in place (Richardson start when start = 1); returns tmp."""
        import torch
        if tmp is None:
            tmp = torch.empty(3 * self.layout.spec_elems, dtype=torch.complex128, device=f"cuda:{self.device}")
        mlg_scalar_advance(self.handle, kind, gamma, self._spec(s, "state"), self._spec(hist, "hist"), nsteps, start,
                           self._spec(tmp, "tmp", 3), self._ws(), self._stream())
        return tmp

    def laplacian_solve(self, f, s, c=None, variant=MLG_LOG_SOLVE):
        """s = (grad^2)^{-1} f; the m = k = 0 block prescribes c (MLG_LOG_PRESCRIBE, c a float) or
        solves for it (MLG_LOG_SOLVE).  Returns the amplitude as a float64 device tensor of one entry."""
        import torch
        cbuf = torch.tensor([0.0 if c is None else float(c)], dtype=torch.float64, device=f"cuda:{self.device}")
        mlg_laplacian_solve(self.handle, variant, self._spec(f, "f"), self._spec(s, "s"),
                            _ptr(cbuf, "c", (torch.float64,), 1, self.device), self._ws(), self._stream())
        return cbuf

    def remove_far_field(self, spec):
        """Remove the far-field level of every m = 0 harmonic of 'spec' in place."""
        mlg_remove_far_field(self.handle, self._spec(spec), self._stream())

    def set_log_proxy(self, c_psi=0.0, c_chi=0.0):
        """Amplitudes of ln(r^2 + ell^2) carried by psi and chi beyond their regular parts."""
        mlg_set_log_proxy(self.handle, c_psi, c_chi)

    def enstrophy(self, psi, chi, out=None):
        """Enstrophy per axial FFT slot (float64 device tensor of N_z entries; the sum is (1/2) int |w|^2 dV)."""
        import torch
        if out is None:
            out = torch.empty(self.nz, dtype=torch.float64, device=f"cuda:{self.device}")
        mlg_tp_enstrophy(self.handle, self._spec(psi, "psi"), self._spec(chi, "chi"), self._f64(out, "out", self.nz),
                         self._ws(), self._stream())
        return out

    def eval_harmonic(self, spec, m, kk, r):
        """Complex values of the (m, kk) harmonic of 'spec' at the radii r (float64 device tensor)."""
        import torch
        r = r.contiguous()
        out = torch.empty(r.numel(), dtype=torch.complex128, device=r.device)
        mlg_eval_harmonic(self.handle, self._spec(spec), m, kk, self._f64(r, "r", r.numel()), r.numel(),
                          _ptr(out, "out", (torch.complex128,), r.numel(), self.device), self._stream())
        return out

    def filter_state(self):
        """(eps_psi, eps_chi, f_psi, f_chi) after the last application (synchronises)."""
        return mlg_filter_state(self.handle)

    def step_febe(self, half, s, A, out):
        mlg_step_febe(self.handle, half, self._spec(s, "s"), self._spec(A, "A"), self._spec(out, "out"),
                      self._stream())

    def step_abcn(self, s, A_now, A_prev, out):
        mlg_step_abcn(self.handle, self._spec(s, "s"), self._spec(A_now, "A_now"), self._spec(A_prev, "A_prev"),
                      self._spec(out, "out"), self._stream())

    def truncate_to(self, other: "Plan", src, dst):
        """dst (spectral of 'other') = src (spectral of this plan) moved to the other grid."""
        mlg_truncate(self.handle, other.handle, self._spec(src, "src"), other._spec(dst, "dst"), self._stream())

    def advance(self, psi, chi, hist_psi, hist_chi, nsteps, start, U=None, closure=None, tmp=None):
        """nsteps AB-CN steps of (psi, chi) in place; tmp: complex128 tensor of 6 * spec_elems."""
        import torch
        if tmp is None:
            tmp = torch.empty(6 * self.layout.spec_elems, dtype=torch.complex128, device=f"cuda:{self.device}")
        mlg_tp_advance(self.handle, U, self._spec(psi, "psi"), self._spec(chi, "chi"),
                       self._spec(hist_psi, "hist_psi"), self._spec(hist_chi, "hist_chi"),
                       int(nsteps), int(start), closure.handle if closure is not None else 0,
                       self._spec(tmp, "tmp", 6), self._ws(), self._stream())
        return tmp

    def taps_buffer(self):
        import torch
        n = 9 * self.layout.phys_elems + 6 * self.layout.spec_elems
        return torch.zeros(n, dtype=torch.float64, device=f"cuda:{self.device}")

    def close(self):
        if self.handle:
            mlg_plan_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # at interpreter shutdown the HIP runtime may already be torn down: leave the handle to
        # the process exit rather than call into the library
        if not getattr(self, "handle", 0) or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def mlg_batch_create(grids, prec: int = MLG_FP64, device: int = 0) -> int:
    arr = (mlg_grid * len(grids))(*grids)
    h = ctypes.c_void_p()
    _check(lib().mlg_batch_create(len(grids), arr, prec, device, ctypes.byref(h)))
    return h.value


def mlg_batch_destroy(batch: int) -> None:
    _check(lib().mlg_batch_destroy(batch))


def mlg_batch_query(batch: int, count: int):
    import numpy as np
    offs = np.zeros(count + 1, dtype=np.int64)
    ws = ctypes.c_int64()
    _check(lib().mlg_batch_query(batch, offs.ctypes.data, ctypes.byref(ws)))
    return offs, ws.value


def mlg_batch_rhs_scalar(batch: int, gamma: float, spec_in: int, spec_out: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_batch_rhs_scalar(batch, gamma, spec_in, spec_out, ws, stream))


def mlg_batch_set_config(batch: int, cfg: mlg_batch_config) -> None:
    _check(lib().mlg_batch_set_config(batch, ctypes.byref(cfg)))


def mlg_batch_get_config(batch: int) -> mlg_batch_config:
    c = mlg_batch_config()
    _check(lib().mlg_batch_get_config(batch, ctypes.byref(c)))
    return c


def mlg_batch_autotune(batch: int, gamma: float, spec_in: int, spec_out: int, ws: int, stream: int = 0):
    c = mlg_batch_config()
    ms = ctypes.c_double()
    _check(lib().mlg_batch_autotune(batch, gamma, spec_in, spec_out, ws, stream, ctypes.byref(c), ctypes.byref(ms)))
    return c, ms.value


class Batch:
    """Uneven 2D instances advanced together; packed spectra in one torch tensor."""

    def __init__(self, grids, prec=MLG_FP64, device=0):
        import torch
        self.count = len(grids)
        self.prec = prec
        self.device = device
        self.handle = mlg_batch_create(grids, prec, device)
        self.offsets, ws = mlg_batch_query(self.handle, self.count)
        self.ws = torch.empty(max(ws, 8), dtype=torch.uint8, device=f"cuda:{device}")
        self.cdtype = torch.complex64 if prec == MLG_FP32 else torch.complex128

    def empty_spec(self):
        import torch
        return torch.zeros(int(self.offsets[-1]), dtype=self.cdtype, device=f"cuda:{self.device}")

    def _spec(self, t, name):
        return _ptr(t, name, (self.cdtype,), int(self.offsets[-1]), self.device)

    def _ws(self):
        import torch
        return _ptr(self.ws, "workspace", (torch.uint8,), 1, self.device)

    def rhs_kpp(self, gamma, spec_in, spec_out):
        import torch
        mlg_batch_rhs_scalar(self.handle, gamma, self._spec(spec_in, "spec_in"), self._spec(spec_out, "spec_out"),
                             self._ws(), torch.cuda.current_stream().cuda_stream)

    def autotune(self, gamma, spec_in, spec_out):
        import torch
        return mlg_batch_autotune(self.handle, gamma, self._spec(spec_in, "spec_in"), self._spec(spec_out, "spec_out"),
                                  self._ws(), torch.cuda.current_stream().cuda_stream)

    def set_config(self, recurrence, threads, blocks_per_cu, lines):
        mlg_batch_set_config(self.handle, mlg_batch_config(recurrence, threads, blocks_per_cu, lines))

    def get_config(self):
        c = mlg_batch_get_config(self.handle)
        return dict(recurrence=c.recurrence, threads=c.threads, blocks_per_cu=c.blocks_per_cu, lines=c.lines)

    def close(self):
        if self.handle:
            mlg_batch_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if not getattr(self, "handle", 0) or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Closure:
    """A learned closure on a coarse Plan (see include/mlg.h for the network and the judge)."""

    def __init__(self, plan: Plan, max_batch: int = 4096, beta: float = 1.0):
        self.plan = plan  # the closure holds a pointer to the plan; keep it alive
        self.handle = mlg_closure_create(plan.handle, max_batch, beta)
        self.ncols = mlg_closure_columns(self.handle)
        self.max_batch = max_batch

    @staticmethod
    def _stream():
        import torch
        return torch.cuda.current_stream().cuda_stream

    def set_params(self, params):
        mlg_closure_set_params(self.handle, params)

    def get_params(self):
        return mlg_closure_get_params(self.handle)

    def get_grads(self):
        return mlg_closure_get_grads(self.handle)

    def set_scales(self, x_scale, y_scale):
        mlg_closure_set_scales(self.handle, x_scale, y_scale)

    def get_scales(self):
        return mlg_closure_get_scales(self.handle)

    def _f32(self, t, name, numel):
        import torch
        return _ptr(t, name, (torch.float32,), numel, self.plan.device)

    def features(self, psi, chi, x_out):
        p = self.plan
        mlg_closure_features(self.handle, p._spec(psi, "psi"), p._spec(chi, "chi"),
                             self._f32(x_out, "x_out", self.ncols * MLG_CLOSURE_NIN), self._stream())

    def targets(self, ref_psi, ref_chi, psi_n, chi_n, y_out):
        p = self.plan
        mlg_closure_targets(self.handle, p._spec(ref_psi, "ref_psi"), p._spec(ref_chi, "ref_chi"),
                            p._spec(psi_n, "psi_n"), p._spec(chi_n, "chi_n"),
                            self._f32(y_out, "y_out", self.ncols * MLG_CLOSURE_NOUT), self._stream())

    def forward(self, x, y):
        nb = int(x.shape[0])
        mlg_closure_forward(self.handle, self._f32(x, "x", nb * MLG_CLOSURE_NIN), nb,
                            self._f32(y, "y", nb * MLG_CLOSURE_NOUT), self._stream())

    def train_step(self, data_x, data_y, idx, nb, lr, want_loss=False):
        import torch
        count = int(data_x.shape[0])
        ip = 0 if idx is None else _ptr(idx, "idx", (torch.int32,), int(nb), self.plan.device)
        return mlg_closure_train_step(self.handle, self._f32(data_x, "data_x", count * MLG_CLOSURE_NIN),
                                      self._f32(data_y, "data_y", count * MLG_CLOSURE_NOUT),
                                      ip, count, int(nb), float(lr), want_loss, self._stream())

    def infer(self, psi, chi, rhs_psi, rhs_chi, want_flag=False):
        p = self.plan
        return mlg_closure_infer(self.handle, p._spec(psi, "psi"), p._spec(chi, "chi"), p._spec(rhs_psi, "rhs_psi"),
                                 p._spec(rhs_chi, "rhs_chi"), want_flag, self._stream())

    def stats(self):
        return mlg_closure_stats(self.handle)

    def set_reference(self, ref: "Plan | None", U=None):
        """Judge every correction also against the plain term on the finer plan 'ref' (None removes it)."""
        self.ref = ref  # the closure holds a pointer to the plan; keep it alive
        mlg_closure_set_reference(self.handle, ref.handle if ref is not None else 0, U)

    def close(self):
        if self.handle:
            mlg_closure_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if not getattr(self, "handle", 0) or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
