"""The pretraining loss of Eq. 5 and its gradient (fn_pretrain_grad) against
the oracle: the loss value and the exact derivative for one parameter of
every tensor group, with synthetic target orbitals (the paper's Hartree-Fock
targets need PySCF: seeded perturbations of the network's own orbitals stand
in for them)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_10287_amd import inputs as I

pytestmark = pytest.mark.gpu


def _group_indices(s):
    idx = []
    for name, (off, shape) in I.param_offsets(s).items():
        if name != "_total":
            idx.append(off + (7 * int(np.prod(shape))) // 11)
    return np.array(idx, dtype=np.int64)


@pytest.mark.parametrize("name,prec,walkers", [("LiH", "fp64", 12), ("LiH", "fp32", 37), ("LiF-m", "bf16x6", 24),
                                               ("Li", "fp32", 16)])
def test_pretrain_loss_and_gradient(name, prec, walkers):
    import torch
    from paper_2401_10287_amd import fnvmc
    assert torch.cuda.is_available()
    if name == "LiH":
        s = I.lih()
    elif name == "Li":
        s = I.atom_ion(3, 0, walkers=walkers)                  # 2 up, 1 down
    else:
        s = I.System("LiF-m", I.lif().nuc_xyz, I.lif().nuc_z, 6, 6, 4, 64, 16, 4, 32, I.lif().electron_site, 0.5)
    cfg = fnvmc.Config(s, prec)
    tt = torch.tensor(I.init_params(s, seed=17), dtype=cfg.param_dtype, device="cuda")
    th = tt.double().cpu().numpy()
    x = I.init_walkers(s, walkers, seed=18)
    o = O.Oracle(s)
    rng = np.random.default_rng(19)
    phi = o.orbital_matrices(th, x)
    T = phi * (1.0 + 0.2 * rng.standard_normal(phi.shape)) + 0.05 * rng.standard_normal(phi.shape)
    tu = torch.tensor(np.ascontiguousarray(T[:, 0, :, :s.n_up, :s.n_up]), device="cuda") if s.n_up else None
    td = torch.tensor(np.ascontiguousarray(T[:, 1, :, :s.n_dn, :s.n_dn]), device="cuda") if s.n_dn else None
    loss, grad = fnvmc.fn_pretrain_grad(cfg, tt, torch.tensor(x, device="cuda"), tu, td)
    torch.cuda.synchronize()
    g = grad.double().cpu().numpy()
    ref_loss = o.pretrain_loss(th, x, T)
    tol = 1e-10 if prec == "fp64" else 1e-5
    print(f"{name} {prec}: loss {loss.item():.8e} oracle {ref_loss:.8e}")
    assert abs(loss.item() - ref_loss) <= tol * abs(ref_loss)
    worst = 0.0
    for i in _group_indices(s):
        d = np.zeros_like(th)
        d[i] = 1.0
        phi_, dphi = o.orbital_matrices_dir(th, d, x)
        r = phi_ - T
        mask = np.zeros_like(r)
        mask[:, 0, :, :s.n_up, :s.n_up] = 1.0
        mask[:, 1, :, :s.n_dn, :s.n_dn] = 1.0
        ref = 2.0 * (r * dphi * mask).sum() / walkers
        scale = 2.0 * np.abs(r * dphi * mask).sum() / walkers
        bound = (1e-9 if prec == "fp64" else 5e-4) * scale + 1e-14
        worst = max(worst, abs(g[i] - ref) / max(scale, 1e-300))
        assert abs(g[i] - ref) <= bound, (i, g[i], ref, scale)
    print(f"{name} {prec}: worst gradient error / scale {worst:.2e}")
