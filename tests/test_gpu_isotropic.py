"""The isotropic envelope (Sigma = sigma I, the special case of Eq. 4 with
one scalar per orbital and nucleus) on the GPU: parity with the oracle's
isotropic layout for log|psi|, the local energy, the Metropolis chain and the
parameter gradient, and agreement with the anisotropic kernels at
Sigma = sigma I.  Tolerance model: tests/parity_tools.py."""
import numpy as np
import pytest

import parity_tools as T
from oracle import oracle as O
from paper_2401_10287_amd import inputs as I

pytestmark = pytest.mark.gpu

SYSTEMS = {"He": I.he, "LiH": I.lih, "LiF": I.lif, "H20": I.h_chain}


def _dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_10287_amd import fnvmc
    return torch, fnvmc


def _both_layouts(base, seed, lo=0.5, hi=2.0):
    """theta of the isotropic system with sigma, pi drawn in [lo, hi] and the
    anisotropic theta with Sigma = sigma I and the same everything else."""
    iso = I.isotropic(base)
    rng = np.random.default_rng(seed)
    th_a = I.init_params(base, seed=seed)
    va = I.view_params(base, th_a)
    th_i = np.zeros(I.param_count(iso))
    vi = I.view_params(iso, th_i)
    for name in vi:
        if name.startswith("sig_"):
            sg = rng.uniform(lo, hi, vi[name].shape)
            vi[name][...] = sg
            va[name][...] = sg[..., None, None] * np.eye(3)
        elif name.startswith("pi_"):
            pv = rng.uniform(lo, hi, vi[name].shape)
            vi[name][...] = pv
            va[name][...] = pv
        else:
            vi[name][...] = va[name]
    return iso, th_i, th_a


@pytest.mark.parametrize("name,walkers,energy", [("LiH", 16, True), ("He", 64, True), ("H20", 4, False)])
def test_fp64_parity_random_sigma(name, walkers, energy):
    """FP64, random sigma and pi: log|psi| and E_L equal the oracle's
    isotropic layout (1e-10 relative, 1e-7 Ha); H20 (20 nuclei) log|psi|."""
    torch, fnvmc = _dev()
    base = SYSTEMS[name]()
    iso, th, _ = _both_layouts(base, seed=31)
    x = I.init_walkers(iso, walkers, seed=32)
    cfg = fnvmc.Config(iso, "fp64")
    tt = torch.tensor(th, device="cuda")
    xt = torch.tensor(x, device="cuda")
    o = O.Oracle(iso)
    lps = [fnvmc.fn_log_psi(cfg, tt, xt)[0]]
    if energy:
        e, lp, parts = fnvmc.fn_local_energy(cfg, tt, xt)
        lps.append(lp)
        ref = o.local_energy(th, x)
        T.check_energy(e.cpu().numpy(), ref, f"{name} isotropic fp64", tol=1e-7, parts=parts.cpu().numpy())
    else:
        ref = o.log_psi(th, x)
    torch.cuda.synchronize()
    for l in lps:
        rel = np.abs(l.cpu().numpy() - ref["log_abs"]) / np.maximum(1.0, np.abs(ref["log_abs"]))
        assert rel.max() <= 1e-10, rel.max()


@pytest.mark.parametrize("name,prec,walkers", [("LiH", "fp32", 256), ("LiH", "bf16x6", 256), ("LiF", "fp32", 32),
                                               ("LiF", "bf16x6", 32), ("H20", "bf16x6", 8)])
def test_local_energy_parity(name, prec, walkers):
    """Reduced precision, the seeded parameters (sigma = 1, pi = 1: the same
    wavefunction as the anisotropic layout's Sigma = I, so the stored |psi|^2
    samples apply): E_L against the oracle's isotropic layout under the
    parity model, log|psi| under its bound."""
    torch, fnvmc = _dev()
    iso = I.isotropic(SYSTEMS[name]())
    x = T.equilibrated(name, walkers)
    cfg = fnvmc.Config(iso, prec)
    tt = torch.tensor(I.init_params(iso), dtype=cfg.param_dtype, device="cuda")
    th = tt.double().cpu().numpy()
    xt = torch.tensor(x, device="cuda")
    e, lp, parts = fnvmc.fn_local_energy(cfg, tt, xt)
    torch.cuda.synchronize()
    o = O.Oracle(iso)
    ref = o.local_energy(th, x)
    kap, C = T.kappa_and_c(o, iso, th, x)
    d32 = None
    if prec != "fp32":
        e32, _, _ = fnvmc.fn_local_energy(fnvmc.Config(iso, "fp32"), tt, xt, want_parts=False)
        d32 = np.abs(e32.cpu().numpy() - ref["e_loc"])
    T.check_energy(e.cpu().numpy(), ref, f"{name} isotropic {prec}", kap, C, iso.n_elec, d32=d32,
                   parts=parts.cpu().numpy())
    T.check_logpsi(lp.cpu().numpy(), ref, 1e-5, f"{name} isotropic {prec}", C, False)


@pytest.mark.parametrize("name,prec,walkers", [("LiH", "bf16x6", 128), ("LiF", "fp32", 16), ("H20", "bf16x6", 8)])
def test_isotropic_equals_anisotropic_special_case(name, prec, walkers):
    """Random sigma and pi: the isotropic kernels and the anisotropic ones
    with Sigma = sigma I give the same log|psi| and E_L up to FP64 rounding
    of the envelope (the network products are the same)."""
    torch, fnvmc = _dev()
    base = SYSTEMS[name]()
    iso, th_i, th_a = _both_layouts(base, seed=33, lo=0.8, hi=1.25)
    x = T.equilibrated(name, walkers)
    xt = torch.tensor(x, device="cuda")
    out = []
    for s, th in ((iso, th_i), (base, th_a)):
        cfg = fnvmc.Config(s, prec)
        tt = torch.tensor(th, dtype=cfg.param_dtype, device="cuda")
        e, lp, _ = fnvmc.fn_local_energy(cfg, tt, xt, want_parts=False)
        lv, _ = fnvmc.fn_log_psi(cfg, tt, xt)
        torch.cuda.synchronize()
        out.append((e.cpu().numpy(), lp.cpu().numpy(), lv.cpu().numpy()))
    (ei, li, vi), (ea, la, va) = out
    de = np.abs(ei - ea)
    print(f"{name} {prec}: isotropic vs anisotropic E_L max |d| {de.max():.2e}, log|psi| max |d| "
          f"{np.abs(li - la).max():.2e}")
    assert np.all(np.isfinite(ei)) and np.all(np.isfinite(ea))
    assert de.max() <= 1e-6 * max(1.0, np.abs(ea).max())
    np.testing.assert_allclose(li, la, rtol=0, atol=1e-9 * max(1.0, np.abs(la).max()))
    np.testing.assert_allclose(vi, va, rtol=0, atol=1e-9 * max(1.0, np.abs(va).max()))


def test_gradient_fp64_sigma_and_pi():
    """FP64 backward of the isotropic layout: every sigma and pi, and one
    parameter of every other tensor, against the oracle's exact derivatives
    (reduced LiF network, 16 walkers)."""
    torch, fnvmc = _dev()
    base = I.System("LiF-s", I.lif().nuc_xyz, I.lif().nuc_z, 3, 3, 3, 32, 8, 4, 16, (0, 1, 1, 0, 1, 1), 0.5)
    iso, th, _ = _both_layouts(base, seed=34)
    x = I.init_walkers(iso, 16, seed=35)
    c = np.random.default_rng(36).standard_normal(16)
    cfg = fnvmc.Config(iso, "fp64")
    g = fnvmc.fn_log_psi_vjp(cfg, torch.tensor(th, device="cuda"), torch.tensor(x, device="cuda"),
                             torch.tensor(c, device="cuda")).cpu().numpy()
    idx = []
    for name, (off, shape) in I.param_offsets(iso).items():
        if name == "_total":
            continue
        n = int(np.prod(shape))
        idx += list(range(off, off + n)) if name[:3] in ("sig", "pi_") else [off + (7 * n) // 11]
    idx = np.array(idx, dtype=np.int64)
    ref = c @ O.Oracle(iso).dlogpsi_dtheta(th, x, idx)
    err = np.abs(g[idx] - ref)
    print("isotropic fp64 gradient: max abs err", err.max(), "max |g|", np.abs(ref).max())
    np.testing.assert_allclose(g[idx], ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
def test_gradient_reduced_precision(prec):
    """Reduced precision (reduced LiF network, seeded walkers, some near
    nodes).  Over the well-conditioned walkers (the parity model's kappa and
    C; the others get coefficient 0): one parameter per tensor within 5e-4
    of the summed magnitudes sum_p |c_p d log|psi_p||, as for the
    anisotropic layout.  Over every walker: each sigma and pi equal to the
    anisotropic path's derivative at Sigma = sigma I (the sum of the three
    diagonal entries for sigma) within 1e-5 of the largest, so the
    isotropic backward adds no error to the network's FP32 arithmetic, which
    both layouts share."""
    torch, fnvmc = _dev()
    base = I.System("LiF-m", I.lif().nuc_xyz, I.lif().nuc_z, 6, 6, 4, 64, 16, 4, 32, I.lif().electron_site, 0.5)
    iso, th_i0, th_a0 = _both_layouts(base, seed=37, lo=0.8, hi=1.25)
    x = I.init_walkers(iso, 32, seed=38)
    xt = torch.tensor(x, device="cuda")
    c = np.random.default_rng(39).standard_normal(32) / 32
    cfg_i = fnvmc.Config(iso, prec)
    th = torch.tensor(th_i0, dtype=cfg_i.param_dtype).double().numpy()
    o = O.Oracle(iso)
    kap, C = T.kappa_and_c(o, iso, th, x)
    well = (kap <= T.KAPPA_WELL) & (C <= T.C_WELL_PER_ELECTRON * iso.n_elec)
    cw = np.where(well, c, 0.0)
    grads = {}
    for s, th0 in ((iso, th_i0), (base, th_a0)):
        cfg = fnvmc.Config(s, prec)
        tt = torch.tensor(th0, dtype=cfg.param_dtype, device="cuda")
        grads[s.envelope] = [fnvmc.fn_log_psi_vjp(cfg, tt, xt, torch.tensor(cc, device="cuda")).double().cpu().numpy()
                             for cc in (c, cw)]
    g, gw = grads[1]
    ga, _ = grads[0]
    offi, offa = I.param_offsets(iso), I.param_offsets(base)
    # one index per tensor against the oracle, well-conditioned walkers
    idx = np.array([off + (7 * int(np.prod(shape))) // 11 for name, (off, shape) in offi.items() if name != "_total"])
    d = o.dlogpsi_dtheta(th, x, idx)
    ref = cw @ d
    scale = np.abs(cw) @ np.abs(d)
    err = np.abs(gw[idx] - ref)
    print(f"{prec} isotropic one-per-tensor over {int(well.sum())} of 32 well-conditioned walkers: "
          f"max err / scale {(err / scale).max():.2e}")
    assert np.all(err <= 5e-4 * scale)
    # every sigma and pi against the anisotropic path
    for tag in ("up", "dn"):
        for kind in ("sig", "pi"):
            oi, shp = offi[f"{kind}_{tag}"]
            oa, _ = offa[f"{kind}_{tag}"]
            n = int(np.prod(shp))
            gi = g[oi:oi + n]
            if kind == "sig":
                gref = ga[oa:oa + 9 * n].reshape(n, 9)[:, [0, 4, 8]].sum(1)
            else:
                gref = ga[oa:oa + n]
            sc = np.abs(gref).max()
            dif = np.abs(gi - gref).max()
            print(f"{prec} {kind}_{tag}: isotropic vs anisotropic max |d| {dif:.2e} of max |g| {sc:.2e}")
            assert dif <= 1e-5 * sc


def test_metropolis_chain_fp64():
    """He with the isotropic layout and random sigma, pi, FP64: the in-kernel
    generator's chain takes the oracle's decisions, positions to 1e-13."""
    torch, fnvmc = _dev()
    iso, th, _ = _both_layouts(I.he(), seed=40)
    x = I.init_walkers(iso, 256)
    cfg = fnvmc.Config(iso, "fp64")
    tt = torch.tensor(th, device="cuda")
    xt = torch.tensor(x, device="cuda")
    lp, _ = fnvmc.fn_log_psi(cfg, tt, xt)
    acc = fnvmc.vmc_metropolis_step(cfg, tt, xt, lp, 10, 0.2, seed=5, step0=0, stream_id=3)
    torch.cuda.synchronize()
    o = O.Oracle(iso)
    xo, lo, ao = o.metropolis(th, x, o.log_psi(th, x)["log_abs"], 10, 0.2, seed=5, step0=0, stream_id=3)
    np.testing.assert_array_equal(acc.cpu().numpy(), ao)
    np.testing.assert_allclose(xt.cpu().numpy(), xo, rtol=0, atol=1e-13)
    np.testing.assert_allclose(lp.cpu().numpy(), lo, rtol=0, atol=1e-11)
