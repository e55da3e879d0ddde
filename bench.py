"""Benchmark: local-energy evaluations per second on one MI355X.

One step = the local energy (forward pass + forward-mode Laplacian + Coulomb
sums, Eq. 2-3 of the paper) of every walker of one batch: LiH (Li Z=3 at the
origin, H Z=1 at 3.015 bohr, 2 up + 2 down electrons), FermiNet with 4
layers, widths 256/32, 16 determinants, 4096 walkers, seeded synthetic
parameters and walker positions resident on the GPU.  The mixed-precision
path (BF16 layer weights, FP32 activations carried exactly as three BF16
parts, FP32 accumulation) is timed, then the plain FP32 path, the six-product
split and the two-part split on the same network and inputs.  In the
BF16-weight modes the network's layer weights are the BF16 roundings of the
seeded parameters, and every leg and the oracle use those parameters.  The walkers are
samples of |psi|^2 (tests/golden/equilibrated_walkers.npz, written by the
oracle's own Metropolis chain), the distribution Eq. 1 averages over; the
mixed result counts only if its batch-mean energy over every walker is within
1 mHa of the FP64 CPU oracle's (the oracle runs on the whole batch by
default) and every walker meets the parity tests' model.  Further legs: the
LiF training step (10 Metropolis moves + local energy + Eq. 6 gradient, 4096
walkers), the H20 local energy (8192 walkers) with the stream layer's
roofline fraction, and Poisson serving runs at 0.5x and 0.9x saturation.

    python bench.py [--steps K] [--warmup W] [--precision bf16w|bf16w2|bf16x6|bf16x3|bf16|fp32]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "local-energy evals/s on 1 GPU (mixed vs plain FP32 at dE<=1 mHa); p50/p99 latency"
PEAK_TFLOPS = {"bf16": 2516.6, "bf16x3": 2516.6, "bf16x6": 2516.6, "bf16w": 2516.6, "bf16w2": 2516.6, "fp32": 157.3,
               "fp64": 78.6}
DTYPE = {"bf16": "bf16", "bf16x3": "bf16", "bf16x6": "bf16", "bf16w": "bf16", "bf16w2": "bf16", "fp32": "f32",
         "fp64": "f64"}
# matrix-core products executed per algorithmic product (operand splits)
PRODUCTS = {"bf16": 1, "bf16x3": 3, "bf16x6": 6, "bf16w": 3, "bf16w2": 2, "fp32": 1, "fp64": 1}
HBM_PEAK_GBPS = 8000.0


def stream_gemm_flops(s, walkers):
    """Algorithmic FLOPs of the per-electron stream-layer products of one
    local-energy pass: 2 B N T (d_h + 2 d_p) w1 per layer, T = 3N + 2 rows
    (value, 3N tangents, Laplacian) per electron, unpadded."""
    from paper_2401_10287_amd import inputs as I
    T = 3 * s.n_elec + 2
    tot = 0
    per_layer = []
    for l in range(s.n_layers):
        d_h, d_p, _ = I.layer_dims(s, l)
        f = 2 * walkers * s.n_elec * T * (d_h + 2 * d_p) * s.w1
        per_layer.append(f)
        tot += f
    return tot, per_layer


def mean_field_flops(s, walkers):
    """Algorithmic FLOPs of the per-walker mean-field products of one
    local-energy pass: 2 B T (2 d_h) w1 per layer ([g_up | g_dn] V_g over the
    T = 3N + 2 rows of each walker)."""
    from paper_2401_10287_amd import inputs as I
    T = 3 * s.n_elec + 2
    return sum(2 * walkers * T * 2 * I.layer_dims(s, l)[0] * s.w1 for l in range(s.n_layers))


def head_flops(s, walkers):
    """Algorithmic FLOPs of the orbital head of one local-energy pass:
    2 B N T w1 (K n_spin) over the T = 3N + 2 rows of every electron."""
    T = 3 * s.n_elec + 2
    return sum(2 * walkers * n * T * s.w1 * s.n_det * n for n in (s.n_up, s.n_dn))


def time_steps(fn, steps, torch):
    """Wall time of `steps` back-to-back calls (no per-step events inside the
    timed region)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def step_latencies(fn, steps, torch):
    """GPU time of each of `steps` more calls, every call bracketed by events
    (a separate pass after the timed one)."""
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for k in range(steps):
        starts[k].record()
        fn()
        ends[k].record()
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])


KERNEL_SOURCE = os.path.join(ROOT, "paper_2401_10287_amd", "csrc", "fn_layer.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stream_layer_hbm_traffic.md")
STACK_SOURCE = os.path.join(ROOT, "paper_2401_10287_amd", "csrc", "fn_stackr.hip")
STACK_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stacked_registers_hbm_traffic.md")


def copy_calibration():
    """A plain device copy of 1 GiB, five times: the counter scale is what
    FETCH_SIZE / WRITE_SIZE report for it divided by 1 GiB."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "copies": 5}))


def kernel_hash(path=KERNEL_SOURCE):
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(summary=TRAFFIC_FILE, source=KERNEL_SOURCE):
    """Bytes per launch of a kernel from its committed counter summary, or
    None when the kernel source changed since the counters were taken."""
    if not os.path.exists(summary):
        return None
    import re
    txt = open(summary).read()
    m = re.search(r"kernel source sha256\[:16\]: `([0-9a-f]+)`", txt)
    t = re.search(r"traffic per launch \(bytes\): `([0-9.e+]+)`", txt)
    if not m or not t or m.group(1) != kernel_hash(source):
        return None
    return float(t.group(1))


def cpu_model():
    try:
        for l in open("/proc/cpuinfo"):
            if l.startswith("model name"):
                return l.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def lif_training_step(prec, steps=10, warmup=2):
    """LiF (4096 walkers) training step: 10 Metropolis moves, the local
    energy and the Eq. 6 gradient with the hand-written backward; ms per step
    (events around each phase) and per phase."""
    import torch
    from paper_2401_10287_amd import fnvmc
    from paper_2401_10287_amd import inputs as I
    import parity_tools as T
    s = I.lif()
    cfg = fnvmc.Config(s, prec)
    tt = torch.tensor(I.init_params(s), dtype=cfg.param_dtype, device="cuda:0")
    xt = torch.tensor(T.equilibrated("LiF", 4096), device="cuda:0")
    ws = fnvmc.Workspace(torch.device("cuda:0"))
    lp, _ = fnvmc.fn_log_psi(cfg, tt, xt, ws=ws)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    tot = np.zeros(3)
    k0 = 0
    for it in range(warmup + steps):
        ev[0].record()
        fnvmc.vmc_metropolis_step(cfg, tt, xt, lp, 10, 0.2, seed=1, step0=k0, ws=ws)
        k0 += 10
        ev[1].record()
        e, _, _ = fnvmc.fn_local_energy(cfg, tt, xt, ws=ws, want_parts=False)
        ev[2].record()
        grad, stats = fnvmc.fn_param_grad(cfg, tt, xt, e, ws=ws)
        ev[3].record()
        torch.cuda.synchronize()
        if it >= warmup:
            tot += [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
    tot /= steps
    print(f"[bench] LiF training step {prec}: {tot.sum():.2f} ms (Metropolis {tot[0]:.2f}, E_L {tot[1]:.2f}, "
          f"gradient {tot[2]:.2f})", file=sys.stderr, flush=True)
    return {"workload": "LiF 4096 walkers, 10 Metropolis moves + local energy + Eq. 6 gradient",
            "precision": prec, "ms_per_step": float(tot.sum()), "metropolis_ms": float(tot[0]),
            "local_energy_ms": float(tot[1]), "gradient_ms": float(tot[2]),
            "energy": float(stats[0].item()), "finite_gradient": bool(torch.isfinite(grad).all().item())}


def h20_local_energy(prec, steps=5, warmup=1, envelope=0):
    """H20 chain (8192 walkers) forward + Laplacian local energy: evals/s,
    the stream layer's algorithmic TFLOP/s over its event-timed launches and
    the time of the envelope + determinant stage.  envelope=1: the isotropic
    envelope (Sigma = sigma I) at sigma = 1, the same wavefunction."""
    import torch
    from paper_2401_10287_amd import fnvmc
    from paper_2401_10287_amd import inputs as I
    import parity_tools as T
    s = I.h_chain() if envelope == 0 else I.isotropic(I.h_chain())
    B = 8192
    cfg = fnvmc.Config(s, prec)
    tt = torch.tensor(I.init_params(s), dtype=cfg.param_dtype, device="cuda:0")
    xt = torch.tensor(T.equilibrated("H20", B), device="cuda:0")
    ws = fnvmc.Workspace(torch.device("cuda:0"))
    for _ in range(warmup):
        fnvmc.fn_local_energy(cfg, tt, xt, ws=ws, want_parts=False)
    torch.cuda.synchronize()
    fnvmc.fn_timing_reset()
    fnvmc.fn_timing_select("stream_gemm")
    fnvmc.fn_timing_enable(True)
    wall = time_steps(lambda: fnvmc.fn_local_energy(cfg, tt, xt, ws=ws, want_parts=False), steps, torch)
    ms_g, n_g = fnvmc.fn_timing_read("stream_gemm")
    fnvmc.fn_timing_reset()
    fnvmc.fn_timing_select("det")
    for _ in range(steps):
        fnvmc.fn_local_energy(cfg, tt, xt, ws=ws, want_parts=False)
    ms_d, _ = fnvmc.fn_timing_read("det")
    fnvmc.fn_timing_enable(False)
    fnvmc.fn_timing_select(None)
    flops, _ = stream_gemm_flops(s, B)
    achieved = flops * steps / (ms_g * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    env = "isotropic" if envelope else "anisotropic"
    print(f"[bench] H20 {prec} {env} envelope: {B * steps / wall:.4g} evals/s, stream layer {achieved:.1f} TFLOP/s "
          f"({achieved / peak:.3f} of peak), envelope + determinants {ms_d / steps:.2f} ms per step",
          file=sys.stderr, flush=True)
    return {"workload": f"H20 chain local energy, 8192 walkers, 4 layers 256/32, 16 determinants, {env} envelope",
            "precision": prec, "evals_per_s": B * steps / wall, "ms_per_step": wall / steps * 1e3,
            "envelope_and_determinants_ms_per_step": ms_d / steps,
            "stream_layer": {"achieved_TFLOPs": achieved, "peak_TFLOPs": peak, "frac": achieved / peak,
                             "launches": n_g}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the clocks take some tens of milliseconds of load to settle: the
    # warm-up covers about 0.2 s of local-energy passes
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="bf16w", choices=["bf16", "bf16x3", "bf16x6", "bf16w", "bf16w2", "fp32"])
    ap.add_argument("--walkers", type=int, default=4096)
    ap.add_argument("--sample", type=int, default=4096,
                    help="walkers checked against / timed on the CPU oracle (default: the whole batch, ~10 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=500, help="jobs of each Poisson serving run (0: skip)")
    ap.add_argument("--no-extra", action="store_true", help="skip the LiF training-step and H20 legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2401_10287_amd import fnvmc
    from paper_2401_10287_amd import inputs as I

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import parity_tools as T

    s = I.lih(args.walkers)
    theta = I.init_params(s).astype(np.float32).astype(np.float64)
    if args.precision in fnvmc.BF16_WEIGHT_PRECISIONS:
        theta = T.bf16_weights(s, theta)       # the BF16-weight network, in every leg
    x = T.equilibrated("LiH", args.walkers)
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, device=dev)
    out = {}
    results = {}
    precs = [args.precision, "fp32"] + [p for p in ("bf16x6", "bf16x3") if p != args.precision]
    for prec in precs:
        cfg = fnvmc.Config(s, prec)
        tt = torch.tensor(theta, dtype=cfg.param_dtype, device=dev)
        ws = fnvmc.Workspace(dev)
        holder = {}

        def step():
            holder["r"] = fnvmc.fn_local_energy(cfg, tt, xt, ws=ws, want_parts=False)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        timing = prec == args.precision
        if timing:
            # inside the timed region only the dominant kernel is bracketed
            # by events (each pair of records costs the stream a few us)
            fnvmc.fn_timing_reset()
            fnvmc.fn_timing_select("stream_gemm")
            fnvmc.fn_timing_enable(True)
        wall = time_steps(step, args.steps, torch)
        if timing:
            fnvmc.fn_timing_enable(False)
            results["stream_gemm"] = fnvmc.fn_timing_read("stream_gemm")
        lat = step_latencies(step, args.steps, torch)
        if timing:
            # per-kernel breakdown from a separate pass with every class bracketed
            fnvmc.fn_timing_reset()
            fnvmc.fn_timing_select(None)
            fnvmc.fn_timing_enable(True)
            nb = min(args.steps, 10)
            for _ in range(nb):
                step()
            torch.cuda.synchronize()
            fnvmc.fn_timing_enable(False)
            results["kernels"] = {k: fnvmc.fn_timing_read(k) for k in fnvmc.KERNEL_CLASSES}
            results["breakdown_steps"] = nb
        e = holder["r"][0].cpu().numpy()
        results[prec] = {"wall": wall, "lat": lat, "e": e, "theta_used": tt.double().cpu().numpy()}
        print(f"[bench] {prec}: {args.steps} steps in {wall:.3f}s, {args.walkers * args.steps / wall:.4g} evals/s",
              file=sys.stderr, flush=True)

    mixed = results[args.precision]
    fp32 = results["fp32"]
    ms_per_step = mixed["wall"] / args.steps * 1e3
    value = args.walkers / (mixed["wall"] / args.steps)
    fp32_value = args.walkers / (fp32["wall"] / args.steps)

    # accuracy gate and CPU baseline: the FP64 oracle on the batch (or its
    # first --sample walkers).  Per walker the parity tests' model: 1e-3 Ha on
    # well-conditioned walkers (kappa <= 10, C <= 50 N); elsewhere the
    # conditioning-scaled bound (FP32) or twice FP32's own error (split
    # modes).  The gate on the reported value is the batch mean over every
    # walker, within 1 mHa, with every walker inside its bound.
    from oracle import oracle as O
    samp = min(args.sample, args.walkers)
    orc = O.Oracle(s)
    t0 = time.perf_counter()
    ref = orc.local_energy(mixed["theta_used"], x[:samp])
    t_orc = time.perf_counter() - t0
    e_ref = ref["e_loc"]
    kappa, cond = T.kappa_and_c(orc, s, mixed["theta_used"], x[:samp])
    d32 = np.abs(fp32["e"][:samp] - e_ref)

    def acc(e, split):
        d = np.abs(e[:samp] - e_ref)
        bound, well = T.energy_bound(kappa, cond, s.n_elec, 1e-3, d32 if split else None)
        return {"batch_mean_err_mHa": float(abs(e[:samp].mean() - e_ref.mean()) * 1e3),
                "max_walker_err_Ha": float(d.max()),
                "max_well_conditioned_err_Ha": float(d[well].max()),
                "well_conditioned_walkers": int(well.sum()),
                "median_abs_err_Ha": float(np.median(d)),
                "worst_err_over_bound": float((d / bound).max())}

    acc_mixed, acc_fp32 = acc(mixed["e"], True), acc(fp32["e"], False)
    d_mixed = acc_mixed["batch_mean_err_mHa"]
    gate_ok = d_mixed <= 1.0 and acc_mixed["worst_err_over_bound"] <= 1.0
    x3 = results.get("bf16x3")
    x6 = results.get("bf16x6") if args.precision != "bf16x6" else None
    print(f"[bench] oracle {samp} walkers in {t_orc:.2f}s; batch-mean |dE| mixed {d_mixed:.5f} mHa, fp32 "
          f"{acc_fp32['batch_mean_err_mHa']:.5f} mHa; worst |dE| / bound mixed "
          f"{acc_mixed['worst_err_over_bound']:.3f}, fp32 {acc_fp32['worst_err_over_bound']:.3f}",
          file=sys.stderr, flush=True)

    # roofline of the dominant kernel: the stacked one-electron stream (every
    # layer's per-electron and mean-field products in one launch per step)
    # or, layer by layer, the fused stream layer (per-electron product)
    kern = results["kernels"]
    ms_g, n_g = results["stream_gemm"]
    flops, _ = stream_gemm_flops(s, args.walkers)
    stacked = n_g == args.steps
    avg_launch_s = ms_g / max(n_g, 1) * 1e-3
    if stacked:
        flops_per_launch = flops + mean_field_flops(s, args.walkers)
        kernel_name = "k_stack_regs (every one-electron layer, per-electron and mean-field products)"
        if kern.get("head_gemm", (0.0, 0))[1] == 0:
            # the orbital head runs in the same launch
            flops_per_launch += head_flops(s, args.walkers)
            kernel_name = "k_stack_regs (every one-electron layer and the orbital head)"
        traffic = measured_traffic(STACK_TRAFFIC_FILE, STACK_SOURCE) if args.walkers == 4096 else None
    else:
        flops_per_launch = flops / s.n_layers
        kernel_name = "k_stream_layer (one layer's per-electron product and epilogue)"
        # the committed counter summary covers the six-product split at 4096 walkers
        traffic = measured_traffic() if (args.precision == "bf16x6" and args.walkers == 4096) else None
    achieved = flops_per_launch / avg_launch_s / 1e12
    peak = PEAK_TFLOPS[args.precision]
    total_kernel_ms = sum(v[0] for v in kern.values())
    nb = results["breakdown_steps"]

    line = {
        "metric": METRIC,
        "value": value if gate_ok else 0.0,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"LiH forward + Laplacian local energy, {args.walkers} walkers, 4 layers 256/32, "
                        f"16 determinants",
            "walkers": args.walkers,
            "precision": args.precision,
            "fp32_evals_per_s": fp32_value,
            "mixed_over_fp32": value / fp32_value,
            "walker_set": "|psi|^2 samples of the seeded network (FP64 oracle chain, 300 moves of 0.2 bohr "
                          "from the seeded start)",
            "accuracy": {"oracle_walkers": samp, "batch_mean_over": "all walkers", "mixed": acc_mixed,
                         "fp32": acc_fp32, "gate_passed": gate_ok},
            "bf16x6": None if x6 is None else {
                "evals_per_s": args.walkers / (x6["wall"] / args.steps),
                "accuracy": acc(x6["e"], True),
                "note": "six-product split of FP32 weights and activations (FP32 operand precision)"},
            "bf16x3": None if x3 is None else {
                "evals_per_s": args.walkers / (x3["wall"] / args.steps),
                "accuracy": acc(x3["e"], True),
                "note": "two-part split (hi + lo, 3 products); not held to the FP32-level bounds"},
            "latency_ms": {"p50": float(np.percentile(mixed["lat"], 50)),
                           "p99": float(np.percentile(mixed["lat"], 99)),
                           "fp32_p50": float(np.percentile(fp32["lat"], 50))},
            "kernel_ms_per_step": {k: v[0] / nb for k, v in kern.items() if v[1]},
        },
        "roofline": {
            "bound": "mfma",
            "kernel": kernel_name,
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "products_per_algorithmic_product": PRODUCTS[args.precision],
            "executed_frac": achieved * PRODUCTS[args.precision] / peak,
            "hbm_GBps": None if traffic is None else traffic / avg_launch_s / 1e9,
            "hbm_frac": None if traffic is None else traffic / avg_launch_s / 1e9 / HBM_PEAK_GBPS,
            "flops_per_launch": flops_per_launch,
            "avg_launch_us": avg_launch_s * 1e6,
            "launches": n_g,
            "kernel_share_of_step": kern["stream_gemm"][0] / max(total_kernel_ms, 1e-9),
        },
    }
    if not args.no_extra:
        line["config"]["lif_training_step"] = lif_training_step(args.precision)
        line["config"]["h20_local_energy"] = h20_local_energy(args.precision)
        line["config"]["h20_local_energy_isotropic"] = h20_local_energy(args.precision, envelope=1)
    if args.serving_jobs > 0:
        from paper_2401_10287_amd import serving
        torch.cuda.synchronize()
        # saturation: the same number of jobs, all queued at t = 0; once with
        # gangs of one system sharing the grouped Metropolis call, once with
        # every job alone
        sat = serving.run_load(args.serving_jobs, None, args.precision)
        solo = serving.run_load(args.serving_jobs, None, args.precision, max_gang=1)
        print(f"[bench] serving saturation: {sat['jobs_per_s']:.1f} jobs/s in gangs (mean "
              f"{sat['mean_gang_jobs']:.2f} jobs), {solo['jobs_per_s']:.1f} jobs/s alone", file=sys.stderr, flush=True)
        runs = {}
        for frac in (0.5, 0.9):
            load = serving.run_load(args.serving_jobs, frac * sat["jobs_per_s"], args.precision,
                                    seed=17 + int(10 * frac))
            print(f"[bench] serving: Poisson at {frac}x: "
                  f"{load['jobs_per_s']:.1f} jobs/s, p50 {load['p50_ms']:.1f} ms p99 {load['p99_ms']:.1f} ms, "
                  f"mean gang {load['mean_gang_jobs']:.2f} jobs", file=sys.stderr, flush=True)
            runs[f"{frac}x"] = {"jobs": load["jobs"], "arrival_rate_jobs_per_s": load["rate"],
                                "jobs_per_s": load["jobs_per_s"], "p50_latency_ms": load["p50_ms"],
                                "p99_latency_ms": load["p99_ms"], "failed": load["failed"],
                                "mean_gang_jobs": load["mean_gang_jobs"]}
        line["config"]["serving"] = {
            "workload": "Poisson stream of VMC jobs, atoms and ions Z 2..10, charge -1..+2, walker batches "
                        "256/1024/4096, 50 Metropolis steps + energy estimate each, 4 layers 256/32, 16 dets",
            "saturation_jobs_per_s": sat["jobs_per_s"], "saturation_mean_gang_jobs": sat["mean_gang_jobs"],
            "saturation_alone_jobs_per_s": solo["jobs_per_s"], "max_gang": sat["max_gang"],
            "gang_walkers": sat["gang_walkers"], "poisson": runs}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = {"value": samp / t_orc, "unit": "evals/s", "cores": O.num_threads(), "kind": "oracle",
                                "cpu_model": cpu_model(),
                                "sample": f"FP64 oracle local energy of the first {samp} of the {args.walkers} "
                                          f"LiH walkers (hyper-dual second derivatives, OpenMP over walkers)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
