"""Seeded synthetic inputs: molecular systems, network parameters, walkers.

This module is the only code that the HIP path and the CPU oracle share.  It
holds no arithmetic of the method itself: it lists the systems (nuclei,
charges, electron counts, network sizes), draws the initial parameters from a
seed and places the initial walkers around the nuclei (the Electron Sampler
section of the paper: electrons start centred on the nuclei, as many per
nucleus as the nucleus carries in the neutral atom, adjusted for ions).

Parameter layout (flat vector, one entry per scalar parameter):
  for l in 0..L-1 : V_l [d_in][w1], b_l [w1]       d_in rows: h_i, g_up, g_dn, g_i_up, g_i_dn
  for l in 0..L-2 : W2_l [d_p][w2], c2_l [w2]
  for spin in (up, dn) with n_spin > 0:
                    w [w1][K n] (column k n + i), g [K n], pi [K n][M], Sigma [K n][M][3][3]
                    (isotropic envelope: sigma [K n][M] in place of Sigma)
with d_h = 4M, d_p = 4 at layer 0 and d_h = w1, d_p = w2 afterwards, d_in = 3 d_h + 2 d_p.
Every matrix and bias is drawn N(0, 1/fan_in) with fan_in the matrix's input
width; envelope weights pi start at 1 and Sigma at the identity (sigma at 1).
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

THETA_SEED = 2401
WALKER_SEED = 10287
METROPOLIS_SEED = 1


@dataclasses.dataclass
class System:
    name: str
    nuc_xyz: np.ndarray          # [M][3] bohr
    nuc_z: np.ndarray            # [M]
    n_up: int
    n_dn: int
    n_layers: int
    w1: int
    w2: int
    n_det: int
    walkers: int = 256
    # nucleus index of each electron slot, in electron order (up first)
    electron_site: Tuple[int, ...] = ()
    init_scale: float = 1.0
    # 0: anisotropic envelope, a 3x3 Sigma per orbital and nucleus (Eq. 4);
    # 1: its isotropic special case Sigma = sigma I, one scalar per orbital
    # and nucleus
    envelope: int = 0

    @property
    def n_nuc(self) -> int:
        return int(self.nuc_xyz.shape[0])

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn


def _sites_from_counts(counts: Sequence[int], n_up: int, n_dn: int) -> Tuple[int, ...]:
    """Electron -> nucleus assignment: list nucleus slots in atom order with
    their counts, give the even slots to spin up and the odd slots to spin
    down (surplus slots of the majority spin follow in order)."""
    slots: List[int] = []
    for m, cnt in enumerate(counts):
        slots += [m] * int(cnt)
    assert len(slots) == n_up + n_dn, (counts, n_up, n_dn)
    even = slots[0::2]
    odd = slots[1::2]
    if len(even) < n_up:            # more up than even slots: borrow from odd
        extra = n_up - len(even)
        even, odd = even + odd[len(odd) - extra:], odd[: len(odd) - extra]
    elif len(even) > n_up:
        extra = len(even) - n_up
        even, odd = even[: len(even) - extra], odd + even[len(even) - extra:]
    return tuple(even) + tuple(odd)


def isotropic(s: System) -> System:
    """The same system with the isotropic envelope Sigma = sigma I."""
    return dataclasses.replace(s, envelope=1)


def he(walkers: int = 256) -> System:
    """He atom, Z = 2 at the origin, 1 up + 1 down electron; 2 layers, widths
    32/8, 2 determinants; walkers N(0, 1) about the nucleus."""
    return System("He", np.zeros((1, 3)), np.array([2.0]), 1, 1, 2, 32, 8, 2, walkers,
                  (0, 0), 1.0)


def h2(bond: float = 1.4, walkers: int = 256) -> System:
    """H2 molecule: protons at (0, 0, -bond/2) and (0, 0, bond/2) bohr, 1 up
    + 1 down electron, one starting about each proton with N(0, 1) offsets;
    the He network (2 layers, widths 32/8, 2 determinants)."""
    xyz = np.array([[0.0, 0.0, -0.5 * bond], [0.0, 0.0, 0.5 * bond]])
    return System(f"H2-{bond:g}", xyz, np.ones(2), 1, 1, 2, 32, 8, 2, walkers, (0, 1), 1.0)


def lih(walkers: int = 4096) -> System:
    """LiH: Li (Z=3) at the origin, H (Z=1) at (0,0,3.015) bohr; 2 up + 2 down;
    3 electrons start about Li and 1 about H with N(0, 1) offsets; 4 layers,
    widths 256/32, 16 determinants."""
    return System("LiH", np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 3.015]]), np.array([3.0, 1.0]),
                  2, 2, 4, 256, 32, 16, walkers, _sites_from_counts([3, 1], 2, 2), 1.0)


def lif(walkers: int = 4096) -> System:
    """LiF ionic pair: Li (Z=3) at the origin, F (Z=9) at (0,0,2.955) bohr;
    6 up + 6 down; 2 electrons start about Li and 10 about F (Li+ F-) with
    N(0, 0.5) offsets; 4 layers, 256/32, 16 determinants."""
    return System("LiF", np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.955]]), np.array([3.0, 9.0]),
                  6, 6, 4, 256, 32, 16, walkers, _sites_from_counts([2, 10], 6, 6), 0.5)


def h_chain(n: int = 20, spacing: float = 1.8, walkers: int = 8192) -> System:
    """Linear hydrogen chain: n protons on the z axis at `spacing` bohr, one
    electron per atom with N(0, 0.5) offsets, spins alternating along the
    chain; 4 layers, 256/32, 16 determinants."""
    xyz = np.zeros((n, 3))
    xyz[:, 2] = spacing * np.arange(n)
    n_up = (n + 1) // 2
    return System(f"H{n}", xyz, np.ones(n), n_up, n - n_up, 4, 256, 32, 16, walkers,
                  _sites_from_counts([1] * n, n_up, n - n_up), 0.5)


def atom_ion(z: int, charge: int, walkers: int = 256, n_layers: int = 4, w1: int = 256, w2: int = 32,
             n_det: int = 16) -> System:
    """A single atom or ion of nuclear charge z and net charge `charge`
    (N = z - charge electrons, spins split as evenly as possible, the extra
    one up), nucleus at the origin, walkers N(0, 1) about it."""
    n = z - charge
    assert n >= 1
    n_up = (n + 1) // 2
    return System(f"Z{z}q{charge:+d}", np.zeros((1, 3)), np.array([float(z)]), n_up, n - n_up,
                  n_layers, w1, w2, n_det, walkers, tuple([0] * n), 1.0)


def serving_job_types() -> List[Tuple[int, int]]:
    """(Z, charge) pairs of the serving mix: Z in 2..10, charge in -1..+2,
    at least one electron."""
    return [(z, q) for z in range(2, 11) for q in range(-1, 3) if z - q >= 1]


# ---------------------------------------------------------------------------
# parameter layout and seeded initial parameters
# ---------------------------------------------------------------------------
def layer_dims(s: System, l: int) -> Tuple[int, int, int]:
    """(d_h, d_p, d_in) of one-electron layer l."""
    d_h = 4 * s.n_nuc if l == 0 else s.w1
    d_p = 4 if l == 0 else s.w2
    return d_h, d_p, 3 * d_h + 2 * d_p


def param_tensors(s: System) -> List[Tuple[str, Tuple[int, ...], int]]:
    """Tensors of the flat layout in order: (name, shape, fan_in)."""
    out: List[Tuple[str, Tuple[int, ...], int]] = []
    for l in range(s.n_layers):
        _, _, d_in = layer_dims(s, l)
        out.append((f"V{l}", (d_in, s.w1), d_in))
        out.append((f"b{l}", (s.w1,), d_in))
    for l in range(s.n_layers - 1):
        d_p = 4 if l == 0 else s.w2
        out.append((f"W2_{l}", (d_p, s.w2), d_p))
        out.append((f"c2_{l}", (s.w2,), d_p))
    for tag, n in (("up", s.n_up), ("dn", s.n_dn)):
        if n == 0:
            continue
        kn = s.n_det * n
        out.append((f"w_{tag}", (s.w1, kn), s.w1))
        out.append((f"g_{tag}", (kn,), s.w1))
        out.append((f"pi_{tag}", (kn, s.n_nuc), 0))
        out.append((f"sig_{tag}", (kn, s.n_nuc) if s.envelope else (kn, s.n_nuc, 3, 3), 0))
    return out


def param_offsets(s: System) -> dict:
    off = {}
    o = 0
    for name, shape, _ in param_tensors(s):
        off[name] = (o, shape)
        o += int(np.prod(shape))
    off["_total"] = (o, ())
    return off


def param_count(s: System) -> int:
    return param_offsets(s)["_total"][0]


def init_params(s: System, seed: int = THETA_SEED) -> np.ndarray:
    """Flat FP64 parameter vector drawn from `seed`."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape, fan_in in param_tensors(s):
        if name.startswith("pi_"):
            parts.append(np.ones(shape))
        elif name.startswith("sig_"):
            parts.append(np.ones(shape) if s.envelope else np.broadcast_to(np.eye(3), shape).copy())
        else:
            parts.append(rng.standard_normal(shape) / np.sqrt(fan_in))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float64)


def view_params(s: System, theta: np.ndarray) -> dict:
    """Named views into a flat parameter vector (for building test weights)."""
    return {name: theta[o:o + int(np.prod(shape))].reshape(shape)
            for name, (o, shape) in param_offsets(s).items() if name != "_total"}


def init_walkers(s: System, walkers: int | None = None, seed: int = WALKER_SEED) -> np.ndarray:
    """[B][N][3] FP64 walker positions: each electron at its nucleus plus a
    Gaussian offset of the system's scale."""
    b = s.walkers if walkers is None else walkers
    rng = np.random.default_rng(seed)
    centres = s.nuc_xyz[np.array(s.electron_site, dtype=np.int64)]          # [N][3]
    off = rng.standard_normal((b, s.n_elec, 3)) * s.init_scale
    return (centres[None, :, :] + off).astype(np.float64)
