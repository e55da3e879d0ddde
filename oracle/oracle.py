"""ctypes binding of the FP64 CPU oracle (fn_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product path never imports it.
It shares no code with the HIP library; inputs come from the seeded
generators in paper_2401_10287_amd.inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fn_oracle.c")
_LIB = os.path.join(_HERE, "libfn_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no fp contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_sanitizer_driver(out: str) -> str:
    """Compile sanitize_driver.c (the oracle in one translation unit) with
    AddressSanitizer and UndefinedBehaviorSanitizer into the executable
    `out`; raises CalledProcessError with the compiler's output on failure."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", _HERE, "-o", out, os.path.join(_HERE, "sanitize_driver.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


class _Cfg(ctypes.Structure):
    _fields_ = [("n_nuc", ctypes.c_int32), ("nuc_xyz", ctypes.c_void_p), ("nuc_z", ctypes.c_void_p),
                ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("w1", ctypes.c_int32), ("w2", ctypes.c_int32), ("n_det", ctypes.c_int32),
                ("envelope", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        _lib.orc_param_count.restype = i64
        _lib.orc_param_count.argtypes = [vp]
        _lib.orc_log_psi.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp]
        _lib.orc_local_energy.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp]
        _lib.orc_dlogpsi_dtheta_index.argtypes = [vp, vp, vp, i64, vp, i64, vp]
        _lib.orc_metropolis.argtypes = [vp, vp, vp, vp, i64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_uint32, vp, vp, vp]
        _lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
        _lib.orc_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint32, i64, ctypes.c_int32, ctypes.c_uint64, vp, vp]
        _lib.orc_draw_one.argtypes = [ctypes.c_uint64, ctypes.c_uint32, i64, ctypes.c_int32, ctypes.c_uint64, vp, vp]
        _lib.orc_slogdet.argtypes = [ctypes.c_int32, i64, vp, vp, vp]
        _lib.orc_coulomb.argtypes = [vp, vp, i64, vp]
        _lib.orc_orbital_matrices.argtypes = [vp, vp, vp, i64, vp]
        _lib.orc_orbital_matrices_dir.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        _lib.orc_num_threads.restype = ctypes.c_int32
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Oracle bound to one system."""

    def __init__(self, system):
        self.s = system
        self._xyz = _f64(system.nuc_xyz).reshape(-1)
        self._z = _f64(system.nuc_z)
        self.cfg = _Cfg(system.n_nuc, self._xyz.ctypes.data, self._z.ctypes.data, system.n_up, system.n_dn,
                        system.n_layers, system.w1, system.w2, system.n_det, int(system.envelope))
        self._cp = ctypes.byref(self.cfg)
        self.n = system.n_elec

    def param_count(self) -> int:
        return int(lib().orc_param_count(self._cp))

    def log_psi(self, theta, x, theta_dir=None, dets=False, h_last=False):
        x = _f64(x)
        theta = _f64(theta)
        b = x.shape[0]
        la, sg = np.empty(b), np.empty(b)
        dl = np.empty(b) if theta_dir is not None else None
        td = _f64(theta_dir) if theta_dir is not None else None
        dd = np.empty((b, 2, self.s.n_det, 2)) if dets else None
        hl = np.empty((b, self.n, self.s.w1)) if h_last else None
        lib().orc_log_psi(self._cp, _p(theta), _p(td), _p(x), b, _p(la), _p(sg), _p(dl), _p(dd), _p(hl))
        out = {"log_abs": la, "sign": sg}
        if dl is not None:
            out["dlog"] = dl
        if dd is not None:
            out["dets"] = dd
        if hl is not None:
            out["h_last"] = hl
        return out

    def local_energy(self, theta, x):
        x = _f64(x)
        theta = _f64(theta)
        b = x.shape[0]
        e, la, parts = np.empty(b), np.empty(b), np.empty((b, 4))
        grad, lap = np.empty((b, 3 * self.n)), np.empty(b)
        lib().orc_local_energy(self._cp, _p(theta), _p(x), b, _p(e), _p(la), _p(parts), _p(grad), _p(lap))
        return {"e_loc": e, "log_abs": la, "parts": parts, "grad": grad, "lap": lap}

    def dlogpsi_dtheta(self, theta, x, idx):
        x = _f64(x)
        theta = _f64(theta)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.empty((x.shape[0], idx.size))
        lib().orc_dlogpsi_dtheta_index(self._cp, _p(theta), _p(idx), idx.size, _p(x), x.shape[0], _p(out))
        return out

    def orbital_matrices(self, theta, x):
        """[B][2][K][nmax][nmax] values phi_i(r_j) of each spin's orbital matrix."""
        x = _f64(x)
        theta = _f64(theta)
        nmax = max(self.s.n_up, self.s.n_dn)
        out = np.empty((x.shape[0], 2, self.s.n_det, nmax, nmax))
        lib().orc_orbital_matrices(self._cp, _p(theta), _p(x), x.shape[0], _p(out))
        return out

    def orbital_matrices_dir(self, theta, theta_dir, x):
        """(values, derivative along theta_dir) of the orbital matrices, [B][2][K][nmax][nmax] each."""
        x = _f64(x)
        theta = _f64(theta)
        nmax = max(self.s.n_up, self.s.n_dn)
        out = np.empty((x.shape[0], 2, self.s.n_det, nmax, nmax))
        out_d = np.empty_like(out)
        lib().orc_orbital_matrices_dir(self._cp, _p(theta), _p(_f64(theta_dir)), _p(x), x.shape[0], _p(out),
                                       _p(out_d))
        return out, out_d

    def pretrain_loss(self, theta, x, targets, theta_dir=None):
        """Eq. 5: (1/B) sum over walkers, spins, determinants, orbitals and
        electrons of (Phi - target)^2, targets [B][2][K][nmax][nmax] (entries
        outside a spin's n x n block ignored); with theta_dir also the exact
        derivative of the loss along it."""
        B = x.shape[0]
        mask = np.zeros((2, self.s.n_det, max(self.s.n_up, self.s.n_dn), max(self.s.n_up, self.s.n_dn)))
        mask[0, :, :self.s.n_up, :self.s.n_up] = 1.0
        mask[1, :, :self.s.n_dn, :self.s.n_dn] = 1.0
        if theta_dir is None:
            phi = self.orbital_matrices(theta, x)
            return float((((phi - targets) * mask) ** 2).sum() / B)
        phi, dphi = self.orbital_matrices_dir(theta, theta_dir, x)
        r = (phi - targets) * mask
        return float((r ** 2).sum() / B), float(2.0 * (r * dphi).sum() / B)

    def coulomb(self, x):
        x = _f64(x)
        out = np.empty((x.shape[0], 3))
        lib().orc_coulomb(self._cp, _p(x), x.shape[0], _p(out))
        return out

    def metropolis(self, theta, x, log_abs, n_steps, sigma, seed, step0=0, stream_id=0, z=None, u=None):
        """Returns (x, log_abs, n_accept); inputs are copied, not modified."""
        x = _f64(x).copy()
        la = _f64(log_abs).copy()
        theta = _f64(theta)
        acc = np.zeros(x.shape[0], dtype=np.int32)
        zz = _f64(z) if z is not None else None
        uu = _f64(u) if u is not None else None
        lib().orc_metropolis(self._cp, _p(theta), _p(x), _p(la), x.shape[0], n_steps, sigma, seed, step0,
                             stream_id, _p(zz), _p(uu), _p(acc))
        return x, la, acc


def philox4x32_10(counter, key):
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def draws(seed, stream_id, walkers, n3, step):
    z = np.empty((walkers, n3))
    u = np.empty(walkers)
    lib().orc_draws(seed, stream_id, walkers, n3, step, _p(z), _p(u))
    return z, u


def draw_one(seed, stream_id, walker, n3, step):
    """Normal deviates [n3] and the accept uniform of one walker index."""
    z = np.empty(n3)
    u = np.empty(1)
    lib().orc_draw_one(seed, stream_id, walker, n3, step, _p(z), _p(u))
    return z, float(u[0])


def slogdet(a):
    a = _f64(a)
    n = a.shape[-1]
    flat = a.reshape(-1, n, n)
    s, l = np.empty(flat.shape[0]), np.empty(flat.shape[0])
    lib().orc_slogdet(n, flat.shape[0], _p(flat), _p(s), _p(l))
    return s.reshape(a.shape[:-2]), l.reshape(a.shape[:-2])


def num_threads() -> int:
    return int(lib().orc_num_threads())
