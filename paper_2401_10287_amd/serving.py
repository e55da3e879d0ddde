"""Continuous-batching VMC service on one GPU (binding of fn_server_* in
include/fnvmc.h) and a Poisson-arrival load driver.

Each job: one atom or ion (Z in 2..10, net charge -1..+2), a walker batch of
256, 1024 or 4096, 50 Metropolis moves and the energy estimate.  Parameters
of every system type stay resident on the GPU; the server admits jobs by
their HBM footprint in one device arena and overlaps their work on several
streams.  Argument marshalling and the load generator only: the scheduler
and all arithmetic are in the HIP library.

    python -m paper_2401_10287_amd.serving --jobs 500
"""
from __future__ import annotations

import argparse
import ctypes
import json
import time
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from . import fnvmc
from . import inputs as I


class _JobResult(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("mean", ctypes.c_double), ("variance", ctypes.c_double),
                ("std_error", ctypes.c_double), ("acceptance", ctypes.c_double), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double), ("footprint_bytes", ctypes.c_int64),
                ("gang_jobs", ctypes.c_int32)]


_L = fnvmc.LIB
_vp, _i32, _i64, _u64, _u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
_L.fn_server_job_bytes.restype = ctypes.c_size_t
_L.fn_server_job_bytes.argtypes = [_vp, _i64]
_L.fn_server_create.restype = _i32
_L.fn_server_create.argtypes = [_vp, ctypes.c_size_t, _vp, _i32, _i32, _i32, _i64, _vp, ctypes.POINTER(_vp)]
_L.fn_server_cancel.restype = _i32
_L.fn_server_cancel.argtypes = [_vp, _i64]
_L.fn_server_memory.restype = _i32
_L.fn_server_memory.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
_L.fn_server_submit.restype = _i32
_L.fn_server_submit.argtypes = [_vp, _vp, _vp, _vp, _i64, _i32, ctypes.c_double, _u64, _u32, ctypes.POINTER(_i64)]
_L.fn_server_step.restype = _i32
_L.fn_server_step.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_L.fn_server_result.restype = _i32
_L.fn_server_result.argtypes = [_vp, _i64, ctypes.POINTER(_JobResult)]
_L.fn_server_destroy.restype = _i32
_L.fn_server_destroy.argtypes = [_vp]
_L.fn_server_last_error.restype = ctypes.c_char_p
_L.fn_server_last_error.argtypes = []

STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


def _check(st: int):
    if st != 0:
        raise fnvmc.FnError(st, _L.fn_server_last_error().decode())


def job_bytes(cfg: fnvmc.Config, walkers: int) -> int:
    return int(_L.fn_server_job_bytes(cfg.ptr, walkers))


class Server:
    """fn_server over a device arena of `arena_bytes` and `n_streams` streams;
    jobs of one system are admitted in gangs of up to `max_gang` jobs and
    `gang_walkers` walkers (max_gang=1: every job alone)."""

    def __init__(self, arena_bytes: int, n_streams: int = 8, quantum: int = 5, max_gang: int = 16,
                 gang_walkers: int = 4096, device: str = "cuda:0"):
        self.device = torch.device(device)
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        self.base = base + (-base) % 256
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_streams)]
        arr = (_vp * n_streams)(*[s.cuda_stream for s in self.streams])
        # pinned host buffer the per-job results are copied into (caller-owned)
        self.host_results = torch.zeros((n_streams, max_gang, 4), dtype=torch.float64, pin_memory=True)
        h = _vp()
        _check(_L.fn_server_create(self.base, arena_bytes, arr, n_streams, quantum, max_gang, gang_walkers,
                                   self.host_results.data_ptr(), ctypes.byref(h)))
        self.h = h
        self._keep: Dict[int, tuple] = {}

    def submit(self, cfg: fnvmc.Config, theta: torch.Tensor, x0: torch.Tensor, n_steps: int, sigma: float,
               seed: int, stream_id: int) -> int:
        b = x0.shape[0]
        job = _i64()
        # the job reads theta and x0 until it is done; they must be ready on
        # the device before any server stream touches them
        torch.cuda.current_stream(self.device).synchronize()
        _check(_L.fn_server_submit(self.h, cfg.ptr, theta.data_ptr(), x0.data_ptr(), b, n_steps, sigma, seed,
                                   stream_id, ctypes.byref(job)))
        self._keep[job.value] = (cfg, theta, x0)
        return job.value

    def step(self) -> Tuple[int, int]:
        a, q = _i32(), _i32()
        _check(_L.fn_server_step(self.h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def result(self, job: int) -> dict:
        r = _JobResult()
        _check(_L.fn_server_result(self.h, job, ctypes.byref(r)))
        out = {f: getattr(r, f) for f, _ in _JobResult._fields_}
        out["state"] = STATES[r.state]
        if r.state >= 2:
            self._keep.pop(job, None)
        return out

    def cancel(self, job: int) -> None:
        _check(_L.fn_server_cancel(self.h, job))

    def memory(self) -> Tuple[int, int]:
        """(free arena bytes, arena bytes)."""
        f, t = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_L.fn_server_memory(self.h, ctypes.byref(f), ctypes.byref(t)))
        return f.value, t.value

    def drain(self, jobs: List[int], timeout_s: float = 600.0):
        t0 = time.perf_counter()
        pending = set(jobs)
        while pending:
            self.step()
            pending = {j for j in pending if self.result(j)["state"] in ("queued", "running")}
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"{len(pending)} jobs still pending")

    def close(self):
        if self.h:
            _L.fn_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class JobFactory:
    """Seeded job stream of the serving mix with per-type parameters resident
    on the device."""

    def __init__(self, precision: str = "bf16x6", seed: int = 2024, device: str = "cuda:0",
                 sizes=(256, 1024, 4096), n_layers: int = 4, w1: int = 256, w2: int = 32, n_det: int = 16):
        self.types = I.serving_job_types()
        self.rng = np.random.default_rng(seed)
        self.device = torch.device(device)
        self.sizes = sizes
        self.precision = precision
        self.arch = (n_layers, w1, w2, n_det)
        self.cache: Dict[Tuple[int, int], Tuple[fnvmc.Config, torch.Tensor]] = {}

    def system(self, z: int, q: int):
        key = (z, q)
        if key not in self.cache:
            L, w1, w2, K = self.arch
            s = I.atom_ion(z, q, n_layers=L, w1=w1, w2=w2, n_det=K)
            cfg = fnvmc.Config(s, self.precision)
            th = torch.tensor(I.init_params(s, seed=I.THETA_SEED + 100 * z + q + 1), dtype=cfg.param_dtype,
                              device=self.device)
            self.cache[key] = (cfg, th)
        return self.cache[key]

    def job(self, k: int):
        z, q = self.types[int(self.rng.integers(len(self.types)))]
        b = int(self.sizes[int(self.rng.integers(len(self.sizes)))])
        cfg, th = self.system(z, q)
        x0 = torch.tensor(I.init_walkers(cfg.system, b, seed=I.WALKER_SEED + k), device=self.device)
        return cfg, th, x0, (z, q, b)


def run_load(n_jobs: int, rate: Optional[float], precision: str = "bf16x6", arena_gb: float = 64.0,
             n_streams: int = 8, quantum: int = 5, n_steps: int = 50, sigma: float = 0.2, seed: int = 2024,
             sizes=(256, 1024, 4096), max_gang: int = 16, gang_walkers: int = 4096) -> dict:
    """Poisson arrivals at `rate` jobs/s (None: all jobs arrive at t = 0, the
    saturation throughput).  Returns latency percentiles and throughput."""
    fac = JobFactory(precision, seed, sizes=sizes)
    jobs = [fac.job(k) for k in range(n_jobs)]     # parameters and walkers staged before the clock starts
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed + 1)
    arrivals = np.zeros(n_jobs) if rate is None else np.cumsum(rng.exponential(1.0 / rate, n_jobs))
    srv = Server(int(arena_gb * (1 << 30)), n_streams, quantum, max_gang, gang_walkers)
    ids: List[int] = []
    t0 = time.perf_counter()
    nxt = 0
    while True:
        now = time.perf_counter() - t0
        while nxt < n_jobs and arrivals[nxt] <= now:
            cfg, th, x0, _ = jobs[nxt]
            ids.append(srv.submit(cfg, th, x0, n_steps, sigma, seed=I.METROPOLIS_SEED, stream_id=nxt))
            nxt += 1
        active, queued = srv.step()
        if nxt == n_jobs and active == 0 and queued == 0:
            break
        if active == 0 and queued == 0 and nxt < n_jobs:
            time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t0), 0.001)))
    wall = time.perf_counter() - t0
    res = [srv.result(j) for j in ids]
    srv.close()
    lat = np.array([r["done_s"] - r["submit_s"] for r in res])
    failed = sum(r["state"] != "done" for r in res)
    return {"jobs": n_jobs, "rate": rate, "wall_s": wall, "jobs_per_s": n_jobs / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "failed": int(failed), "precision": precision,
            "walker_sizes": list(sizes), "n_streams": n_streams, "quantum": quantum, "arena_gb": arena_gb,
            "max_gang": max_gang, "gang_walkers": gang_walkers,
            "mean_gang_jobs": float(np.mean([r["gang_jobs"] for r in res])), "results": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=500)
    ap.add_argument("--precision", default="bf16x6")
    ap.add_argument("--streams", type=int, default=8)
    ap.add_argument("--quantum", type=int, default=5)
    ap.add_argument("--arena-gb", type=float, default=64.0)
    ap.add_argument("--max-gang", type=int, default=16)
    args = ap.parse_args()
    sat = run_load(args.jobs, None, args.precision, args.arena_gb, args.streams, args.quantum,
                   max_gang=args.max_gang)
    out = {"saturation_jobs_per_s": sat["jobs_per_s"]}
    for frac in (0.5, 0.9):
        r = run_load(args.jobs, frac * sat["jobs_per_s"], args.precision, args.arena_gb, args.streams, args.quantum,
                     max_gang=args.max_gang)
        r.pop("results")
        out[f"load_{frac}"] = r
        print(f"[serving] load {frac}: {r['jobs_per_s']:.2f} jobs/s p50 {r['p50_ms']:.1f} ms p99 {r['p99_ms']:.1f} ms",
              flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
