"""Python binding of libfnvmc.so (include/fnvmc.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors live on the GPU (torch provides device memory and the
stream); the library must be built (python -m paper_2401_10287_amd.build) and
importing this module fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

from . import inputs as _inputs

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfnvmc.so")

FN_OK, FN_EINVAL, FN_ENOMEM, FN_EUNSUPPORTED, FN_EHIP = 0, 1, 2, 3, 4
FN_FP64, FN_FP32, FN_BF16_MIXED, FN_BF16X3_MIXED, FN_BF16X6_MIXED = 0, 1, 2, 3, 4
FN_BF16W_MIXED, FN_BF16W2_MIXED = 5, 6
FN_OP_LOG_PSI, FN_OP_LOCAL_ENERGY, FN_OP_METROPOLIS, FN_OP_PARAM_GRAD = 0, 1, 2, 3
PRECISIONS = {"fp64": FN_FP64, "fp32": FN_FP32, "bf16": FN_BF16_MIXED, "bf16x3": FN_BF16X3_MIXED,
              "bf16x6": FN_BF16X6_MIXED, "bf16w": FN_BF16W_MIXED, "bf16w2": FN_BF16W2_MIXED}
# modes whose one-electron layer weights are the BF16 roundings of the parameters
BF16_WEIGHT_PRECISIONS = ("bf16w", "bf16w2")


class FnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fnvmc status {status}: {msg}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [("n_nuc", ctypes.c_int32), ("nuc_xyz", ctypes.c_void_p), ("nuc_z", ctypes.c_void_p),
                ("n_up", ctypes.c_int32), ("n_down", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("w1", ctypes.c_int32), ("w2", ctypes.c_int32), ("n_det", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("envelope", ctypes.c_int32)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libfnvmc.so not built at {_LIB_PATH}; run python -m paper_2401_10287_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, u64, u32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32,
                                  ctypes.c_size_t)
    lib.fn_param_count.restype = i64
    lib.fn_param_count.argtypes = [vp]
    lib.fn_workspace_bytes.restype = sz
    lib.fn_workspace_bytes.argtypes = [vp, i64, i32]
    lib.fn_log_psi.restype = i32
    lib.fn_log_psi.argtypes = [vp, vp, vp, i64, vp, vp, vp, sz, vp]
    lib.fn_local_energy.restype = i32
    lib.fn_local_energy.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]
    lib.vmc_metropolis_step.restype = i32
    lib.vmc_metropolis_step.argtypes = [vp, vp, vp, vp, i64, i32, ctypes.c_double, u64, u64, u32, vp, vp, sz, vp]
    lib.vmc_metropolis_step_ext.restype = i32
    lib.vmc_metropolis_step_ext.argtypes = [vp, vp, vp, vp, i64, i32, ctypes.c_double, vp, vp, vp, vp, sz, vp]
    lib.vmc_metropolis_step_noalloc.restype = i32
    lib.vmc_metropolis_step_noalloc.argtypes = [vp, vp, vp, vp, i64, i32, ctypes.c_double, u64, u64, u32, vp, vp]
    lib.vmc_metropolis_step_group.restype = i32
    lib.vmc_metropolis_step_group.argtypes = [vp, vp, vp, i32, vp, vp, vp, i64, i32, ctypes.c_double, vp, sz, vp]
    lib.fn_param_grad.restype = i32
    lib.fn_param_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]
    lib.fn_pretrain_grad.restype = i32
    lib.fn_pretrain_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
    lib.fn_log_psi_vjp.restype = i32
    lib.fn_log_psi_vjp.argtypes = [vp, vp, vp, i64, vp, vp, vp, sz, vp]
    lib.fn_ionic_electron_counts.restype = i32
    lib.fn_ionic_electron_counts.argtypes = [i32, vp, vp, i32, vp]
    lib.fn_init_walkers.restype = i32
    lib.fn_init_walkers.argtypes = [vp, vp, ctypes.c_double, u64, u32, i64, vp, vp]
    lib.fn_energy_stats.restype = i32
    lib.fn_energy_stats.argtypes = [vp, i64, vp, vp, vp]
    lib.fn_last_error.restype = ctypes.c_char_p
    lib.fn_last_error.argtypes = []
    lib.fn_timing_enable.restype = i32
    lib.fn_timing_enable.argtypes = [i32]
    lib.fn_timing_select.restype = i32
    lib.fn_timing_select.argtypes = [ctypes.c_char_p]
    lib.fn_timing_reset.restype = i32
    lib.fn_timing_reset.argtypes = []
    lib.fn_timing_read.restype = i32
    lib.fn_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.fn_tuning_set.restype = i32
    lib.fn_tuning_set.argtypes = [ctypes.c_char_p, i64]
    return lib


LIB = _load()
LIB_PATH = _LIB_PATH

EXPORTED = ["fn_param_count", "fn_workspace_bytes", "fn_log_psi", "fn_local_energy", "vmc_metropolis_step",
            "vmc_metropolis_step_ext", "vmc_metropolis_step_noalloc", "vmc_metropolis_step_group", "fn_param_grad", "fn_pretrain_grad", "fn_log_psi_vjp", "fn_energy_stats", "fn_ionic_electron_counts",
            "fn_init_walkers", "fn_last_error", "fn_timing_enable",
            "fn_timing_select", "fn_timing_reset", "fn_timing_read", "fn_tuning_set", "fn_server_job_bytes", "fn_server_create", "fn_server_submit",
            "fn_server_step", "fn_server_result", "fn_server_cancel", "fn_server_memory", "fn_server_destroy",
            "fn_server_last_error"]
KERNEL_CLASSES = ["stream_gemm", "walker_gemm", "head_gemm", "features", "pair_stream", "spin_mean", "layer_epilogue",
                  "envelope", "det", "combine", "pack", "propose", "accept", "backward"]


def _check(status: int):
    if status != FN_OK:
        raise FnError(status, LIB.fn_last_error().decode())


class Config:
    """A system plus the arithmetic of the network, as the library's fn_config."""

    def __init__(self, system: "_inputs.System", precision: str = "fp32"):
        self.system = system
        self.precision = precision
        self._xyz = np.ascontiguousarray(system.nuc_xyz, dtype=np.float64).reshape(-1)
        self._z = np.ascontiguousarray(system.nuc_z, dtype=np.float64)
        self.c = _Config(system.n_nuc, self._xyz.ctypes.data, self._z.ctypes.data, system.n_up, system.n_dn,
                         system.n_layers, system.w1, system.w2, system.n_det, PRECISIONS[precision],
                         int(system.envelope))
        self.ptr = ctypes.addressof(self.c)
        self.n_elec = system.n_elec
        self.param_dtype = torch.float64 if precision == "fp64" else torch.float32

    def param_count(self) -> int:
        n = LIB.fn_param_count(self.ptr)
        if n < 0:
            _check(FN_EINVAL)
        return int(n)

    def workspace_bytes(self, walkers: int, op: int) -> int:
        n = LIB.fn_workspace_bytes(self.ptr, walkers, op)
        if n == 0:
            raise FnError(FN_EINVAL, LIB.fn_last_error().decode())
        return int(n)


class Workspace:
    """Caller-owned device workspace, grown on demand and 256-byte aligned."""

    def __init__(self, device: Optional[torch.device] = None):
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.buf = None
        self.nbytes = 0

    def get(self, nbytes: int):
        if nbytes > self.nbytes:
            self.buf = None
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.nbytes = nbytes
        base = self.buf.data_ptr()
        return base + (-base) % 256, self.nbytes


_default_ws = {}


def _ws(ws: Optional[Workspace], x: torch.Tensor) -> Workspace:
    if ws is not None:
        return ws
    key = x.device.index
    if key not in _default_ws:
        _default_ws[key] = Workspace(x.device)
    return _default_ws[key]


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _need(t: torch.Tensor, dtype, shape, name):
    if not t.is_cuda or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")


def fn_log_psi(cfg: Config, theta: torch.Tensor, x: torch.Tensor, ws: Optional[Workspace] = None, stream=None,
               out: Optional[torch.Tensor] = None, sign: Optional[torch.Tensor] = None):
    b = x.shape[0]
    _need(theta, cfg.param_dtype, (cfg.param_count(),), "theta")
    _need(x, torch.float64, (b, cfg.n_elec, 3), "x")
    out = torch.empty(b, dtype=torch.float64, device=x.device) if out is None else out
    sign = torch.empty(b, dtype=torch.int8, device=x.device) if sign is None else sign
    w = _ws(ws, x)
    p, n = w.get(cfg.workspace_bytes(b, FN_OP_LOG_PSI))
    _check(LIB.fn_log_psi(cfg.ptr, theta.data_ptr(), x.data_ptr(), b, out.data_ptr(), _ptr(sign), p, n,
                          _stream(stream)))
    return out, sign


def fn_local_energy(cfg: Config, theta: torch.Tensor, x: torch.Tensor, ws: Optional[Workspace] = None, stream=None,
                    want_parts: bool = True):
    b = x.shape[0]
    _need(theta, cfg.param_dtype, (cfg.param_count(),), "theta")
    _need(x, torch.float64, (b, cfg.n_elec, 3), "x")
    e = torch.empty(b, dtype=torch.float64, device=x.device)
    lp = torch.empty(b, dtype=torch.float64, device=x.device)
    parts = torch.empty((b, 4), dtype=torch.float64, device=x.device) if want_parts else None
    w = _ws(ws, x)
    p, n = w.get(cfg.workspace_bytes(b, FN_OP_LOCAL_ENERGY))
    _check(LIB.fn_local_energy(cfg.ptr, theta.data_ptr(), x.data_ptr(), b, e.data_ptr(), lp.data_ptr(), _ptr(parts),
                               p, n, _stream(stream)))
    return e, lp, parts


def vmc_metropolis_step(cfg: Config, theta: torch.Tensor, x: torch.Tensor, log_abs: torch.Tensor, n_steps: int,
                        sigma: float, seed: int, step0: int = 0, stream_id: int = 0,
                        n_accept: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None, stream=None,
                        z: Optional[torch.Tensor] = None, u: Optional[torch.Tensor] = None):
    """In place on x and log_abs; returns n_accept."""
    b = x.shape[0]
    _need(theta, cfg.param_dtype, (cfg.param_count(),), "theta")
    _need(x, torch.float64, (b, cfg.n_elec, 3), "x")
    _need(log_abs, torch.float64, (b,), "log_abs")
    if n_accept is None:
        n_accept = torch.zeros(b, dtype=torch.int32, device=x.device)
    w = _ws(ws, x)
    p, n = w.get(cfg.workspace_bytes(b, FN_OP_METROPOLIS))
    if z is not None or u is not None:
        _need(z, torch.float64, (n_steps, b, 3 * cfg.n_elec), "z")
        _need(u, torch.float64, (n_steps, b), "u")
        _check(LIB.vmc_metropolis_step_ext(cfg.ptr, theta.data_ptr(), x.data_ptr(), log_abs.data_ptr(), b, n_steps,
                                           sigma, z.data_ptr(), u.data_ptr(), n_accept.data_ptr(), p, n,
                                           _stream(stream)))
    else:
        _check(LIB.vmc_metropolis_step(cfg.ptr, theta.data_ptr(), x.data_ptr(), log_abs.data_ptr(), b, n_steps, sigma,
                                       seed, step0, stream_id, n_accept.data_ptr(), p, n, _stream(stream)))
    return n_accept


def vmc_metropolis_step_noalloc(cfg: Config, theta: torch.Tensor, x: torch.Tensor, log_abs: torch.Tensor,
                                n_steps: int, sigma: float, seed: int, step0: int = 0, stream_id: int = 0,
                                n_accept: Optional[torch.Tensor] = None, stream=None):
    """As vmc_metropolis_step with the library's fixed scratch as workspace."""
    b = x.shape[0]
    _need(theta, cfg.param_dtype, (cfg.param_count(),), "theta")
    _need(x, torch.float64, (b, cfg.n_elec, 3), "x")
    _need(log_abs, torch.float64, (b,), "log_abs")
    if n_accept is None:
        n_accept = torch.zeros(b, dtype=torch.int32, device=x.device)
    _check(LIB.vmc_metropolis_step_noalloc(cfg.ptr, theta.data_ptr(), x.data_ptr(), log_abs.data_ptr(), b, n_steps,
                                           sigma, seed, step0, stream_id, n_accept.data_ptr(), _stream(stream)))
    return n_accept


class GroupJob(ctypes.Structure):
    _fields_ = [("walker0", ctypes.c_int64), ("B", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("step0", ctypes.c_uint64), ("stream_id", ctypes.c_uint32)]


def vmc_metropolis_step_group(cfg: Config, theta: torch.Tensor, jobs, x: torch.Tensor, log_abs: torch.Tensor,
                              n_steps: int, sigma: float, n_accept: Optional[torch.Tensor] = None,
                              ws: Optional[Workspace] = None, stream=None):
    """Grouped moves, in place on x and log_abs.  jobs: sequence of (B, seed,
    step0, stream_id) in walker order (job q owns the next B rows)."""
    b = x.shape[0]
    _need(theta, cfg.param_dtype, (cfg.param_count(),), "theta")
    _need(x, torch.float64, (b, cfg.n_elec, 3), "x")
    _need(log_abs, torch.float64, (b,), "log_abs")
    if n_accept is None:
        n_accept = torch.zeros(b, dtype=torch.int32, device=x.device)
    tab = (GroupJob * len(jobs))()
    w0 = 0
    for q, (nb, seed, step0, sid) in enumerate(jobs):
        tab[q] = GroupJob(w0, nb, seed, step0, sid)
        w0 += nb
    w = _ws(ws, x)
    p, n = w.get(cfg.workspace_bytes(b, FN_OP_METROPOLIS))
    _check(LIB.vmc_metropolis_step_group(cfg.ptr, theta.data_ptr(), ctypes.addressof(tab), len(jobs), x.data_ptr(),
                                         log_abs.data_ptr(), n_accept.data_ptr(), b, n_steps, sigma, p, n,
                                         _stream(stream)))
    return n_accept


def fn_param_grad(cfg: Config, theta: torch.Tensor, x: torch.Tensor, e_loc: torch.Tensor,
                  ws: Optional[Workspace] = None, stream=None):
    b = x.shape[0]
    _need(theta, cfg.param_dtype, (cfg.param_count(),), "theta")
    _need(x, torch.float64, (b, cfg.n_elec, 3), "x")
    _need(e_loc, torch.float64, (b,), "e_loc")
    grad = torch.empty_like(theta)
    stats = torch.empty(3, dtype=torch.float64, device=x.device)
    w = _ws(ws, x)
    p, n = w.get(cfg.workspace_bytes(b, FN_OP_PARAM_GRAD))
    _check(LIB.fn_param_grad(cfg.ptr, theta.data_ptr(), x.data_ptr(), b, e_loc.data_ptr(), grad.data_ptr(),
                             stats.data_ptr(), p, n, _stream(stream)))
    return grad, stats


def fn_pretrain_grad(cfg: Config, theta: torch.Tensor, x: torch.Tensor, target_up: Optional[torch.Tensor],
                     target_dn: Optional[torch.Tensor], ws: Optional[Workspace] = None, stream=None):
    """(loss [1] FP64, grad [P]) of the Eq. 5 pretraining loss against target
    orbital values [B][K][n][n] per spin (None for an empty spin)."""
    b = x.shape[0]
    s = cfg.system
    _need(theta, cfg.param_dtype, (cfg.param_count(),), "theta")
    _need(x, torch.float64, (b, cfg.n_elec, 3), "x")
    for t, n, nm in ((target_up, s.n_up, "target_up"), (target_dn, s.n_dn, "target_dn")):
        if n:
            _need(t, torch.float64, (b, s.n_det, n, n), nm)
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    grad = torch.empty_like(theta)
    w = _ws(ws, x)
    p, n = w.get(cfg.workspace_bytes(b, FN_OP_PARAM_GRAD))
    _check(LIB.fn_pretrain_grad(cfg.ptr, theta.data_ptr(), x.data_ptr(), b, _ptr(target_up), _ptr(target_dn),
                                loss.data_ptr(), grad.data_ptr(), p, n, _stream(stream)))
    return loss, grad


def fn_log_psi_vjp(cfg: Config, theta: torch.Tensor, x: torch.Tensor, coeff: torch.Tensor,
                   ws: Optional[Workspace] = None, stream=None):
    b = x.shape[0]
    _need(theta, cfg.param_dtype, (cfg.param_count(),), "theta")
    _need(x, torch.float64, (b, cfg.n_elec, 3), "x")
    _need(coeff, torch.float64, (b,), "coeff")
    grad = torch.empty_like(theta)
    w = _ws(ws, x)
    p, n = w.get(cfg.workspace_bytes(b, FN_OP_PARAM_GRAD))
    _check(LIB.fn_log_psi_vjp(cfg.ptr, theta.data_ptr(), x.data_ptr(), b, coeff.data_ptr(), grad.data_ptr(), p, n,
                              _stream(stream)))
    return grad


def fn_energy_stats(e_loc: torch.Tensor, stream=None):
    """(stats [3] = mean, variance, standard error; coeff [B] = 2 (E_p - mean) / B), FP64 on the device."""
    b = e_loc.shape[0]
    _need(e_loc, torch.float64, (b,), "e_loc")
    stats = torch.empty(3, dtype=torch.float64, device=e_loc.device)
    coeff = torch.empty(b, dtype=torch.float64, device=e_loc.device)
    _check(LIB.fn_energy_stats(e_loc.data_ptr(), b, stats.data_ptr(), coeff.data_ptr(), _stream(stream)))
    return stats, coeff


def fn_ionic_electron_counts(partial_charge, atomic_number, ion_charge: int) -> np.ndarray:
    """Electrons per nucleus of an ion by the charge-initialisation policy (host only)."""
    q = np.ascontiguousarray(partial_charge, dtype=np.float64)
    z = np.ascontiguousarray(atomic_number, dtype=np.int32)
    if q.shape != z.shape or q.ndim != 1:
        raise ValueError("partial_charge and atomic_number must be 1-D of the same length")
    out = np.empty(q.size, dtype=np.int32)
    _check(LIB.fn_ionic_electron_counts(q.size, q.ctypes.data, z.ctypes.data, int(ion_charge), out.ctypes.data))
    return out


def fn_init_walkers(cfg: Config, site, scale: float, seed: int, walkers: int, stream_id: int = 0,
                    device: Optional[torch.device] = None, stream=None) -> torch.Tensor:
    """[B][N][3] FP64 initial walkers on the device: electron i about nucleus site[i]."""
    st = np.ascontiguousarray(site, dtype=np.int32)
    if st.shape != (cfg.n_elec,):
        raise ValueError(f"site: need {cfg.n_elec} nucleus indices")
    dev = device or torch.device("cuda", torch.cuda.current_device())
    x = torch.empty((walkers, cfg.n_elec, 3), dtype=torch.float64, device=dev)
    _check(LIB.fn_init_walkers(cfg.ptr, st.ctypes.data, float(scale), int(seed), int(stream_id), walkers, x.data_ptr(),
                               _stream(stream)))
    return x


def fn_timing_enable(on: bool) -> None:
    _check(LIB.fn_timing_enable(1 if on else 0))


def fn_timing_select(name: Optional[str]) -> None:
    """Record only the kernel class `name` while timing is enabled (None: every class)."""
    _check(LIB.fn_timing_select(None if name is None else name.encode()))


def fn_timing_reset() -> None:
    _check(LIB.fn_timing_reset())


def fn_timing_read(name: str):
    """(summed ms, launches) of one kernel class since the last reset."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(LIB.fn_timing_read(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def fn_tuning_set(name: str, value: int) -> None:
    _check(LIB.fn_tuning_set(name.encode(), int(value)))
