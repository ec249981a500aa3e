"""ctypes binding of include/mlg.h.

Functions named like the C entry points take plain integers for device pointers
and streams (e.g. ``tensor.data_ptr()``, ``torch.cuda.current_stream().cuda_stream``)
and raise ``MlgError`` on a non-zero status.  ``Plan`` is a small convenience
wrapper that allocates its workspace as a torch tensor on the plan's device.
"""
from __future__ import annotations

import ctypes
import os

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
           "mlg_backward", "mlg_rhs_scalar", "mlg_rhs_tp", "mlg_synthesize", "mlg_timing_enable", "mlg_timing_read",
           "mlg_batch_create", "mlg_batch_destroy", "mlg_batch_query", "mlg_batch_rhs_scalar", "mlg_batch_set_config",
           "mlg_batch_get_config", "mlg_batch_autotune", "mlg_step_setup", "mlg_step_febe", "mlg_step_abcn",
           "mlg_last_error"]


class mlg_dissip(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("nu_h", ctypes.c_double), ("p", ctypes.c_int32), ("dt", ctypes.c_double)]


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
    L.mlg_synthesize.argtypes = [vp, vp, vp, vp, vp, vp]
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


def mlg_step_setup(plan: int, nu: float, nu_h: float, p: int, dt: float) -> None:
    d = mlg_dissip(nu, nu_h, p, dt)
    _check(lib().mlg_step_setup(plan, ctypes.byref(d)))


def mlg_step_febe(plan: int, half: int, s: int, A: int, out: int, stream: int = 0) -> None:
    _check(lib().mlg_step_febe(plan, half, s, A, out, stream))


def mlg_step_abcn(plan: int, s: int, A_now: int, A_prev: int, out: int, stream: int = 0) -> None:
    _check(lib().mlg_step_abcn(plan, s, A_now, A_prev, out, stream))


def mlg_synthesize(plan: int, psi: int, chi: int, uw: int, ws: int, stream: int = 0) -> None:
    _check(lib().mlg_synthesize(plan, psi, chi, uw, ws, stream))


def mlg_timing_enable(plan: int, enable: bool) -> None:
    _check(lib().mlg_timing_enable(plan, 1 if enable else 0))


def mlg_timing_read(plan: int, kernel: str):
    """(total milliseconds, launches) recorded for a kernel family since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().mlg_timing_read(plan, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


class Plan:
    """A plan plus its workspace, for torch tensors on the plan's device.

    Tensors: physical fields are float64 of shape (N_z, N_r, N_phi); spectral fields are
    complex128 of shape (tau, N_z) (packed triangular rows, see include/mlg.h).
    """

    def __init__(self, nr, nphi, nz=1, ell=1.0, lz=6.283185307179586, nrc=0, nphic=0, nzc=0,
                 dealias=1, prec=MLG_FP64, device=0):
        import torch
        self.grid = mlg_grid(nr, nphi, nz, nrc, nphic, nzc, float(ell), float(lz), int(dealias))
        self.device = device
        self.handle = mlg_plan_create(self.grid, prec, device)
        self.layout = mlg_plan_query(self.handle)
        self.nr, self.nphi, self.nz = nr, nphi, nz
        self.ws = torch.empty(max(self.layout.workspace_bytes, 8), dtype=torch.uint8, device=f"cuda:{device}")

    @property
    def tau(self) -> int:
        return self.layout.spec_rows

    def nodes(self):
        return mlg_plan_nodes(self.handle, self.nr)

    def empty_phys(self):
        import torch
        return torch.empty((self.nz, self.nr, self.nphi), dtype=torch.float64, device=f"cuda:{self.device}")

    def empty_spec(self):
        import torch
        return torch.empty((self.tau, self.nz), dtype=torch.complex128, device=f"cuda:{self.device}")

    @staticmethod
    def _stream():
        import torch
        return torch.cuda.current_stream().cuda_stream

    def forward(self, phys, spec):
        mlg_forward(self.handle, phys.data_ptr(), spec.data_ptr(), self.ws.data_ptr(), self._stream())

    def backward(self, spec, phys):
        mlg_backward(self.handle, spec.data_ptr(), phys.data_ptr(), self.ws.data_ptr(), self._stream())

    def rhs_scalar(self, kind, gamma, spec_u, spec_out):
        mlg_rhs_scalar(self.handle, kind, gamma, spec_u.data_ptr(), spec_out.data_ptr(), self.ws.data_ptr(),
                       self._stream())

    def rhs_tp(self, psi, chi, psi_n, chi_n, U=None, taps=None):
        mlg_rhs_tp(self.handle, U, psi.data_ptr(), chi.data_ptr(), psi_n.data_ptr(), chi_n.data_ptr(),
                   0 if taps is None else taps.data_ptr(), self.ws.data_ptr(), self._stream())

    def synthesize(self, psi, chi, uw):
        """uw: float64 tensor of 6 * phys_elems (u_r, u_phi, u_z, w_r, w_phi, w_z)."""
        mlg_synthesize(self.handle, psi.data_ptr(), chi.data_ptr(), uw.data_ptr(), self.ws.data_ptr(), self._stream())

    def step_setup(self, nu, nu_h=0.0, p=8, dt=1e-2):
        mlg_step_setup(self.handle, nu, nu_h, p, dt)

    def step_febe(self, half, s, A, out):
        mlg_step_febe(self.handle, half, s.data_ptr(), A.data_ptr(), out.data_ptr(), self._stream())

    def step_abcn(self, s, A_now, A_prev, out):
        mlg_step_abcn(self.handle, s.data_ptr(), A_now.data_ptr(), A_prev.data_ptr(), out.data_ptr(), self._stream())

    def taps_buffer(self):
        import torch
        n = 9 * self.layout.phys_elems + 6 * self.layout.spec_elems
        return torch.zeros(n, dtype=torch.float64, device=f"cuda:{self.device}")

    def close(self):
        if self.handle:
            mlg_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
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

    def rhs_kpp(self, gamma, spec_in, spec_out):
        import torch
        mlg_batch_rhs_scalar(self.handle, gamma, spec_in.data_ptr(), spec_out.data_ptr(), self.ws.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)

    def autotune(self, gamma, spec_in, spec_out):
        import torch
        return mlg_batch_autotune(self.handle, gamma, spec_in.data_ptr(), spec_out.data_ptr(), self.ws.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)

    def set_config(self, recurrence, threads, blocks_per_cu, lines):
        mlg_batch_set_config(self.handle, mlg_batch_config(recurrence, threads, blocks_per_cu, lines))

    def get_config(self):
        c = mlg_batch_get_config(self.handle)
        return dict(recurrence=c.recurrence, threads=c.threads, blocks_per_cu=c.blocks_per_cu, lines=c.lines)

    def close(self):
        if self.handle:
            mlg_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
