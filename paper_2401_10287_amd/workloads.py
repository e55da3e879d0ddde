"""Named workloads for profiling runs (rocprofv3 and the like): a few passes
of one hot-path call on seeded inputs, with the tuning switches set from the
command line, and nothing else on the GPU.

    python -m paper_2401_10287_amd.workloads lih-local-energy --precision bf16 --layer-stack 0 --passes 3

Workloads:
  lih-local-energy   LiH, 4096 walkers (the stored |psi|^2 samples), forward
                     + Laplacian local energy, 4 layers 256/32, 16 determinants
  lih-metropolis     the same system, value-form Metropolis moves (one per pass)
"""
from __future__ import annotations

import argparse
import os
import sys

import torch

from . import fnvmc
from . import inputs as I

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("workload", choices=["lih-local-energy", "lih-metropolis"])
    ap.add_argument("--precision", default="bf16x6", choices=list(fnvmc.PRECISIONS))
    ap.add_argument("--walkers", type=int, default=4096)
    ap.add_argument("--passes", type=int, default=3)
    ap.add_argument("--layer-stack", type=int, default=None, help="tuning switch layer_stack (0, 1, 2)")
    ap.add_argument("--stack-shape", type=int, default=None, help="tuning switch stack_shape (0, 1, 2)")
    ap.add_argument("--stack-regs", type=int, default=None, help="tuning switch stack_regs (0, 1)")
    args = ap.parse_args(argv)
    if args.stack_regs is not None:
        fnvmc.fn_tuning_set("stack_regs", args.stack_regs)
    if args.layer_stack is not None:
        fnvmc.fn_tuning_set("layer_stack", args.layer_stack)
    if args.stack_shape is not None:
        fnvmc.fn_tuning_set("stack_shape", args.stack_shape)
    sys.path.insert(0, os.path.join(_ROOT, "tests"))
    import parity_tools as T          # the stored walker sets

    s = I.lih(args.walkers)
    cfg = fnvmc.Config(s, args.precision)
    dev = torch.device("cuda:0")
    tt = torch.tensor(I.init_params(s), dtype=cfg.param_dtype, device=dev)
    xt = torch.tensor(T.equilibrated("LiH", args.walkers), device=dev)
    ws = fnvmc.Workspace(dev)
    if args.workload == "lih-local-energy":
        for _ in range(args.passes):
            fnvmc.fn_local_energy(cfg, tt, xt, ws=ws, want_parts=False)
    else:
        lp, _ = fnvmc.fn_log_psi(cfg, tt, xt, ws=ws)
        for k in range(args.passes):
            fnvmc.vmc_metropolis_step(cfg, tt, xt, lp, 1, 0.2, seed=I.METROPOLIS_SEED, step0=k, stream_id=0, ws=ws)
    torch.cuda.synchronize()
    print(f"{args.workload}: {args.passes} passes, {args.precision}, {args.walkers} walkers", flush=True)


if __name__ == "__main__":
    main()
