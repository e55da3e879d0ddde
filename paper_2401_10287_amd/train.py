"""VMC training loop: the steps the paper's Introduction lists (sample the
electrons with Metropolis-Hastings, evaluate the local energy, update the
parameters after a set number of sampling steps; ten moves between updates,
as in the paper's Results) with the gradient of Eq. 6 (FermiNet Training).

The paper names no optimizer; Adam (torch.optim.Adam on the flat parameter
vector) is the reading used here.  Every step of the wavefunction, the
sampler, the energies, the Eq. 6 statistics and the gradient runs in the HIP
library; this module only sequences the calls and applies the optimizer
update to the parameter tensor.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from . import fnvmc


@dataclasses.dataclass
class StepStats:
    energy: float          # batch mean of E_L (Eq. 1)
    variance: float        # 1/B variance of E_L
    std_error: float
    acceptance: float      # accepted moves / proposed moves in this step


class VMCTrainer:
    """Walkers, parameters and Adam state resident on one GPU.

    step(): mc_steps Metropolis moves, the local energies, the Eq. 6
    gradient, one Adam update, and log|psi| of the walkers under the updated
    parameters (the next moves compare against it)."""

    def __init__(self, system, precision: str, theta0, x0, lr: float = 1e-3, betas=(0.9, 0.999),
                 sigma: float = 0.2, mc_steps: int = 10, seed: int = 1, stream_id: int = 0,
                 device: Optional[torch.device] = None):
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.cfg = fnvmc.Config(system, precision)
        self.theta = torch.as_tensor(np.asarray(theta0), dtype=self.cfg.param_dtype).to(self.device).contiguous()
        self.x = torch.as_tensor(np.asarray(x0), dtype=torch.float64).to(self.device).contiguous()
        self.opt = torch.optim.Adam([self.theta], lr=lr, betas=betas)
        self.sigma, self.mc_steps, self.seed, self.stream_id = sigma, mc_steps, seed, stream_id
        self.mc_counter = 0
        self.ws = fnvmc.Workspace(self.device)
        self.n_accept = torch.zeros(self.x.shape[0], dtype=torch.int32, device=self.device)
        self.log_abs, _ = fnvmc.fn_log_psi(self.cfg, self.theta, self.x, ws=self.ws)
        self.history: List[StepStats] = []

    def burn_in(self, n_steps: int) -> float:
        """Metropolis moves without parameter updates; returns the acceptance."""
        self.n_accept.zero_()
        fnvmc.vmc_metropolis_step(self.cfg, self.theta, self.x, self.log_abs, n_steps, self.sigma, self.seed,
                                  self.mc_counter, self.stream_id, n_accept=self.n_accept, ws=self.ws)
        self.mc_counter += n_steps
        return float(self.n_accept.sum().item()) / (n_steps * self.x.shape[0])

    def step(self) -> StepStats:
        self.n_accept.zero_()
        fnvmc.vmc_metropolis_step(self.cfg, self.theta, self.x, self.log_abs, self.mc_steps, self.sigma, self.seed,
                                  self.mc_counter, self.stream_id, n_accept=self.n_accept, ws=self.ws)
        self.mc_counter += self.mc_steps
        e, _, _ = fnvmc.fn_local_energy(self.cfg, self.theta, self.x, ws=self.ws, want_parts=False)
        grad, stats = fnvmc.fn_param_grad(self.cfg, self.theta, self.x, e, ws=self.ws)
        self.theta.grad = grad
        self.opt.step()
        self.theta.grad = None
        fnvmc.fn_log_psi(self.cfg, self.theta, self.x, ws=self.ws, out=self.log_abs)
        st = stats.cpu().numpy()
        out = StepStats(float(st[0]), float(st[1]), float(st[2]),
                        float(self.n_accept.sum().item()) / (self.mc_steps * self.x.shape[0]))
        self.history.append(out)
        return out

    def block_means(self, block: int) -> np.ndarray:
        """Mean energy over consecutive blocks of `block` steps."""
        e = np.array([h.energy for h in self.history])
        n = len(e) // block
        return e[: n * block].reshape(n, block).mean(1)
