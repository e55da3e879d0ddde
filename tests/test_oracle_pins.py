"""Pins of the FP64 oracle against results fixed by the paper and by the
mathematics, independently of the oracle's own code.

Each test names the part of the method it pins (the paper's Eq. 1-6, the
Electron Sampler and FermiNet Model sections) and a mistake it would catch.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_10287_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small(n_up, n_dn, nuc_xyz, nuc_z, L=2, w1=6, w2=4, K=2, scale=1.0, envelope=0):
    s = I.System("t", np.asarray(nuc_xyz, float).reshape(-1, 3), np.asarray(nuc_z, float), n_up, n_dn, L, w1, w2, K,
                 8, tuple([0] * (n_up + n_dn)), scale, envelope)
    return s


def zero_theta(s):
    th = np.zeros(I.param_count(s))
    v = I.view_params(s, th)
    for name, t in v.items():
        if name.startswith("pi_"):
            t[...] = 1.0
        if name.startswith("sig_"):
            t[...] = 1.0 if s.envelope else np.eye(3)
    return th, v


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
def test_philox_known_answers():
    """Philox4x32-10 against the generator authors' published vectors: any
    wrong multiplier, key increment, round count or word order fails."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = O.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_normal_draws_moments():
    """Box-Muller deviates: mean 0, variance 1, uniforms inside (0, 1]."""
    z, u = O.draws(seed=7, stream_id=3, walkers=20000, n3=12, step=5)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    assert np.all(u > 0) and np.all(u <= 1) and abs(u.mean() - 0.5) < 0.01
    # counters differ per step / stream / seed
    z2, _ = O.draws(seed=7, stream_id=3, walkers=4, n3=12, step=6)
    z3, _ = O.draws(seed=7, stream_id=4, walkers=4, n3=12, step=5)
    assert not np.allclose(z[:4], z2) and not np.allclose(z[:4], z3)


# --------------------------------------------------------------------------
# Coulomb terms of Eq. 2
# --------------------------------------------------------------------------
def test_nuclear_repulsion_closed_forms():
    gold = {}
    for l in open(os.path.join(GOLDEN, "nuclear_repulsion.txt")):
        if l.strip() and l[0] != "#":
            k, v = l.split()
            gold[k] = float(v)
    for s in (I.lih(8), I.lif(8), I.h_chain(walkers=8), I.he(8)):
        name = "H20" if s.name == "H20" else s.name
        parts = O.Oracle(s).coulomb(I.init_walkers(s, 2))
        assert parts[:, 2] == pytest.approx(gold[name], rel=1e-14, abs=1e-14)


def test_coulomb_hand_configuration():
    """Two electrons at (+-1, 0, 0) about a Z=2 nucleus: el-el 1/2 (repulsive),
    nuc-el -2*2/1 (attractive)."""
    s = small(1, 1, [0, 0, 0], [2.0])
    x = np.array([[[1.0, 0, 0], [-1.0, 0, 0]]])
    p = O.Oracle(s).coulomb(x)[0]
    assert p[0] == pytest.approx(0.5) and p[1] == pytest.approx(-4.0) and p[2] == 0.0


# --------------------------------------------------------------------------
# closed-form wavefunctions: kinetic term (Eq. 3), envelope (Eq. 4)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("z,K,L", [(1.0, 1, 1), (2.0, 3, 2), (3.5, 2, 3)])
def test_hydrogenic_exact_local_energy(z, K, L):
    """Orbital weights 0, bias 1, pi = 1, Sigma = Z I gives psi = K exp(-Z r)
    exactly, so E_L = -Z^2/2 at every walker and log|psi| = log K - Z r."""
    s = small(1, 0, [0.3, -0.2, 0.1], [z], L=L, K=K)
    th, v = zero_theta(s)
    rng = np.random.default_rng(0)
    for name in v:       # random network weights must not matter: w = 0
        if name[0] in "VbWc":
            v[name][...] = rng.standard_normal(v[name].shape)
    v["g_up"][...] = 1.0
    v["sig_up"][...] = z * np.eye(3)
    x = rng.standard_normal((16, 1, 3)) + s.nuc_xyz[0]
    o = O.Oracle(s)
    r = o.local_energy(th, x)
    rr = np.linalg.norm(x[:, 0] - s.nuc_xyz[0], axis=1)
    np.testing.assert_allclose(r["e_loc"], -z * z / 2, atol=1e-10)
    np.testing.assert_allclose(r["log_abs"], np.log(K) - z * rr, atol=1e-12)
    # the kinetic part alone is -Z^2/2 + Z/r
    np.testing.assert_allclose(r["parts"][:, 0], -z * z / 2 + z / rr, rtol=1e-10)


def test_helium_product_state():
    """He, 1 up + 1 down, both orbitals exp(-Z r): E_L = -Z^2 + 1/r12."""
    s = I.he(16)
    th = I.init_params(s)
    v = I.view_params(s, th)
    for t in ("up", "dn"):
        v[f"w_{t}"][...] = 0.0
        v[f"g_{t}"][...] = 1.0
        v[f"sig_{t}"][...] = 2.0 * np.eye(3)
    x = I.init_walkers(s)
    r = O.Oracle(s).local_energy(th, x)
    r12 = np.linalg.norm(x[:, 0] - x[:, 1], axis=1)
    np.testing.assert_allclose(r["e_loc"], -4.0 + 1.0 / r12, atol=1e-10)


def _glt(s):
    """g(s) = log tanh(s) and its first two derivatives."""
    return np.log(np.tanh(s)), 2.0 / np.sinh(2 * s), -4.0 * np.cosh(2 * s) / np.sinh(2 * s) ** 2


def test_tanh_radial_closed_form():
    """One layer routing |r - R| through tanh into the orbital: psi =
    tanh(r) exp(-Z r).  Pins the feature order [d, |d|], the h_i block of the
    first layer, the orbital head layout and the tanh forward Laplacian:
    E_kin = -1/2 (u'' + 2u'/r + u'^2) with u = log tanh r - Z r."""
    z = 1.7
    s = small(1, 0, [0, 0, 0], [z], L=1, w1=3, K=1)
    th, v = zero_theta(s)
    v["V0"][3, 1] = 1.0            # |r - R_0| feature -> unit 1
    v["w_up"][1, 0] = 1.0          # unit 1 -> orbital 0 of determinant 0
    v["sig_up"][...] = z * np.eye(3)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((12, 1, 3))
    r = np.linalg.norm(x[:, 0], axis=1)
    g0, g1, g2 = _glt(r)
    u1, u2 = g1 - z, g2
    kin = -0.5 * (u2 + 2 * u1 / r + u1 ** 2)
    out = O.Oracle(s).local_energy(th, x)
    np.testing.assert_allclose(out["log_abs"], g0 - z * r, atol=1e-12)
    np.testing.assert_allclose(out["parts"][:, 0], kin, rtol=1e-9, atol=1e-9)


def _pair_closed_form(x, z, g0, g1, g2):
    """log psi = G(r12) - Z r1 - Z r2 with G, G', G'' given at r12."""
    d = x[:, 0] - x[:, 1]
    r12 = np.linalg.norm(d, axis=1)
    r1, r2 = np.linalg.norm(x[:, 0], axis=1), np.linalg.norm(x[:, 1], axis=1)
    e12 = d / r12[:, None]
    gr1 = g1[:, None] * e12 - z * x[:, 0] / r1[:, None]
    gr2 = -g1[:, None] * e12 - z * x[:, 1] / r2[:, None]
    lap = 2 * (g2 + 2 * g1 / r12) - 2 * z / r1 - 2 * z / r2
    kin = -0.5 * (lap + (gr1 ** 2).sum(1) + (gr2 ** 2).sum(1))
    return g0 - z * (r1 + r2), kin


def test_pair_feature_closed_form():
    """Routing the pair distance through the g_i_dn block of the first layer:
    psi = tanh(r12) exp(-Z r1) exp(-Z r2).  Pins the pair features, the
    down-spin pair mean (self pair zero) and the Laplacian through r12."""
    z = 1.3
    s = small(1, 1, [0, 0, 0], [z], L=1, w1=2, K=1)
    th, v = zero_theta(s)
    v["V0"][19, 0] = 1.0           # rows: h 0-3, g_up 4-7, g_dn 8-11, g_i_up 12-15, g_i_dn 16-19
    v["w_up"][0, 0] = 1.0
    v["g_dn"][0] = 1.0
    v["sig_up"][...] = z * np.eye(3)
    v["sig_dn"][...] = z * np.eye(3)
    x = np.random.default_rng(2).standard_normal((12, 2, 3))
    r12 = np.linalg.norm(x[:, 0] - x[:, 1], axis=1)
    lp, kin = _pair_closed_form(x, z, *_glt(r12))
    out = O.Oracle(s).local_energy(th, x)
    np.testing.assert_allclose(out["log_abs"], lp, atol=1e-12)
    np.testing.assert_allclose(out["parts"][:, 0], kin, rtol=1e-9, atol=1e-9)


def test_two_electron_stream_and_residual_closed_form():
    """Two layers: the first one-electron layer is zero, the pair layer maps
    |r_ij| to tanh(r_ij), the second one-electron layer reads the g_i_dn
    block: psi = tanh(tanh(r12)) exp(-Z (r1 + r2)).  Pins the pair-stream
    weights, the second layer's block order and the residual (adds zero)."""
    z = 0.9
    s = small(1, 1, [0, 0, 0], [z], L=2, w1=3, w2=2, K=1)
    th, v = zero_theta(s)
    v["W2_0"][3, 1] = 1.0
    v["V1"][3 * s.w1 + s.w2 + 1, 2] = 1.0
    v["w_up"][2, 0] = 1.0
    v["g_dn"][0] = 1.0
    v["sig_up"][...] = z * np.eye(3)
    v["sig_dn"][...] = z * np.eye(3)
    x = np.random.default_rng(3).standard_normal((10, 2, 3))
    r12 = np.linalg.norm(x[:, 0] - x[:, 1], axis=1)
    t1 = np.tanh(r12)
    a, da = 1 - t1 ** 2, -2 * t1 * (1 - t1 ** 2)
    g0, g1, g2 = _glt(t1)
    lp, kin = _pair_closed_form(x, z, g0, g1 * a, g2 * a * a + g1 * da)
    out = O.Oracle(s).local_energy(th, x)
    np.testing.assert_allclose(out["log_abs"], lp, atol=1e-12)
    np.testing.assert_allclose(out["parts"][:, 0], kin, rtol=1e-8, atol=1e-8)


def test_mean_field_and_determinant_closed_form():
    """Two up electrons; unit 0 = tanh(mean of |r - R| over up electrons) (the
    g_up block), unit 1 = tanh(x coordinate); orbitals pick units 0 and 1:
    det = e1 e2 tanh(m) (tanh x2 - tanh x1).  Pins the spin mean, the 2x2
    determinant's sign and the row/column convention."""
    z = 1.1
    s = small(2, 0, [0, 0, 0], [z], L=1, w1=2, K=1)
    th, v = zero_theta(s)
    v["V0"][4 + 3, 0] = 1.0        # g_up block, |r| column
    v["V0"][0, 1] = 1.0            # h_i block, x column
    v["w_up"][0, 0] = 1.0          # orbital 0 <- unit 0
    v["w_up"][1, 1] = 1.0          # orbital 1 <- unit 1
    v["sig_up"][...] = z * np.eye(3)
    x = np.random.default_rng(4).standard_normal((20, 2, 3))
    r = np.linalg.norm(x, axis=2)
    m = r.mean(1)
    val = np.exp(-z * r).prod(1) * np.tanh(m) * (np.tanh(x[:, 1, 0]) - np.tanh(x[:, 0, 0]))
    out = O.Oracle(s).log_psi(th, x)
    np.testing.assert_allclose(out["log_abs"], np.log(np.abs(val)), atol=1e-12)
    np.testing.assert_array_equal(out["sign"], np.sign(val))


def test_determinant_sum_with_signs():
    """K = 2 one-electron determinants per spin with constant orbitals:
    psi = (a0 b0 + a1 b1) exp(-Z (r1 + r2)), negative sum -> sign -1."""
    s = small(1, 1, [0, 0, 0], [2.0], L=1, w1=2, K=2)
    th, v = zero_theta(s)
    v["g_up"][:] = [0.5, -3.0]
    v["g_dn"][:] = [2.0, 1.0]
    v["sig_up"][...] = 2 * np.eye(3)
    v["sig_dn"][...] = 2 * np.eye(3)
    x = np.random.default_rng(5).standard_normal((6, 2, 3))
    out = O.Oracle(s).log_psi(th, x)
    r = np.linalg.norm(x, axis=2)
    np.testing.assert_allclose(out["log_abs"], np.log(2.0) - 2 * r.sum(1), atol=1e-12)
    assert np.all(out["sign"] == -1)


def test_identical_determinants_add_log_k():
    s = small(2, 1, [0, 0, 0], [3.0], L=2, K=1)
    s4 = small(2, 1, [0, 0, 0], [3.0], L=2, K=4)
    th1 = I.init_params(s, seed=11)
    v1 = I.view_params(s, th1)
    th4 = np.zeros(I.param_count(s4))
    v4 = I.view_params(s4, th4)
    for name, t in v4.items():
        if name[0] in "VbWc":
            t[...] = v1[name]
        else:     # repeat the one determinant's orbitals K times
            kn1 = v1[name].shape[0] if name[0] != "w" else v1[name].shape[1]
            if name[0] == "w":
                t[...] = np.tile(v1[name], (1, 4))
            else:
                t[...] = np.concatenate([v1[name]] * 4, axis=0)
            assert kn1 * 4 == (t.shape[1] if name[0] == "w" else t.shape[0])
    x = I.init_walkers(s, 8)
    a = O.Oracle(s).log_psi(th1, x)
    b = O.Oracle(s4).log_psi(th4, x)
    np.testing.assert_allclose(b["log_abs"], a["log_abs"] + np.log(4.0), atol=1e-12)
    np.testing.assert_array_equal(a["sign"], b["sign"])


# --------------------------------------------------------------------------
# the slogdet step against LAPACK
# --------------------------------------------------------------------------
def test_slogdet_matches_lapack():
    rng = np.random.default_rng(6)
    for n in range(1, 12):
        a = rng.standard_normal((40, n, n))
        a[0] = a[0] @ np.diag(10.0 ** -np.arange(n))        # ill-conditioned
        s, l = O.slogdet(a)
        s2, l2 = np.linalg.slogdet(a)
        np.testing.assert_array_equal(s, s2)
        np.testing.assert_allclose(l, l2, rtol=1e-12, atol=1e-12)
    s, l = O.slogdet(np.zeros((1, 3, 3)))
    assert s[0] == 0 and l[0] == -np.inf


# --------------------------------------------------------------------------
# derivatives: hyper-dual against finite differences of the value path
# --------------------------------------------------------------------------
def _fd_laplacian(o, th, x, h=1e-3):
    b, n, _ = x.shape
    base = o.log_psi(th, x)["log_abs"]
    lap = np.zeros(b)
    g2 = np.zeros(b)
    for c in range(3 * n):
        xp, xm = x.copy(), x.copy()
        xp.reshape(b, -1)[:, c] += h
        xm.reshape(b, -1)[:, c] -= h
        fp, fm = o.log_psi(th, xp)["log_abs"], o.log_psi(th, xm)["log_abs"]
        lap += (fp - 2 * base + fm) / h ** 2
        g2 += ((fp - fm) / (2 * h)) ** 2
    return lap, g2


@pytest.mark.parametrize("sysname", ["lih_small", "lif_small"])
def test_laplacian_matches_finite_differences(sysname):
    if sysname == "lih_small":
        s = I.System("LiH-s", I.lih().nuc_xyz, I.lih().nuc_z, 2, 2, 3, 12, 6, 3, 4, I.lih().electron_site, 1.0)
    else:
        s = I.System("LiF-s", I.lif().nuc_xyz, I.lif().nuc_z, 3, 2, 3, 10, 5, 2, 4, (0, 1, 1, 0, 1), 0.5)
    th = I.init_params(s, seed=21)
    v = I.view_params(s, th)
    rng = np.random.default_rng(22)
    for t in ("up", "dn"):    # anisotropic envelopes exercise Sigma fully
        v[f"sig_{t}"][...] += 0.3 * rng.standard_normal(v[f"sig_{t}"].shape)
        v[f"pi_{t}"][...] = 0.5 + rng.random(v[f"pi_{t}"].shape)
    x = I.init_walkers(s, 4, seed=23)
    o = O.Oracle(s)
    r = o.local_energy(th, x)
    # Richardson extrapolation of two central-difference steps: O(h^4)
    l1, g1 = _fd_laplacian(o, th, x, 2e-3)
    l2, g2 = _fd_laplacian(o, th, x, 1e-3)
    lap, g2 = (4 * l2 - l1) / 3, (4 * g2 - g1) / 3
    np.testing.assert_allclose(r["lap"], lap, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose((r["grad"] ** 2).sum(1), g2, rtol=2e-6, atol=2e-6)


def test_parameter_derivatives_match_finite_differences():
    s = I.System("LiH-s", I.lih().nuc_xyz, I.lih().nuc_z, 2, 2, 3, 8, 4, 2, 4, I.lih().electron_site, 1.0)
    th = I.init_params(s, seed=31)
    x = I.init_walkers(s, 3, seed=32)
    off = I.param_offsets(s)
    idx = [off[n][0] + 1 for n in ("V0", "b1", "V2", "W2_0", "c2_1", "w_up", "g_dn", "pi_up", "sig_dn")]
    o = O.Oracle(s)
    d = o.dlogpsi_dtheta(th, x, idx)
    for t, i in enumerate(idx):
        h = 1e-6 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (o.log_psi(tp, x)["log_abs"] - o.log_psi(tm, x)["log_abs"]) / (2 * h)
        np.testing.assert_allclose(d[:, t], fd, rtol=1e-6, atol=1e-8)


# --------------------------------------------------------------------------
# symmetries
# --------------------------------------------------------------------------
def test_antisymmetry_same_spin_swap():
    for s in (I.System("LiH-s", I.lih().nuc_xyz, I.lih().nuc_z, 2, 2, 2, 8, 4, 2, 4, I.lih().electron_site, 1.0),
              I.System("LiF-s", I.lif().nuc_xyz, I.lif().nuc_z, 3, 3, 2, 8, 4, 2, 4, (0, 1, 1, 0, 1, 1), 0.5)):
        th = I.init_params(s, seed=41)
        x = I.init_walkers(s, 5, seed=42)
        o = O.Oracle(s)
        a = o.local_energy(th, x)
        sa = o.log_psi(th, x)["sign"]
        for (i, j) in ((0, 1), (s.n_up, s.n_up + 1)):
            y = x.copy()
            y[:, [i, j]] = y[:, [j, i]]
            b = o.local_energy(th, y)
            sb = o.log_psi(th, y)["sign"]
            np.testing.assert_allclose(b["log_abs"], a["log_abs"], atol=1e-12)
            np.testing.assert_array_equal(sb, -sa)
            np.testing.assert_allclose(b["e_loc"], a["e_loc"], rtol=1e-9, atol=1e-9)


def test_translation_invariance():
    s0 = I.System("LiH-s", I.lih().nuc_xyz, I.lih().nuc_z, 2, 2, 2, 8, 4, 2, 4, I.lih().electron_site, 1.0)
    shift = np.array([0.7, -1.3, 2.1])
    s1 = I.System("LiH-t", I.lih().nuc_xyz + shift, I.lih().nuc_z, 2, 2, 2, 8, 4, 2, 4, I.lih().electron_site, 1.0)
    th = I.init_params(s0, seed=51)
    x = I.init_walkers(s0, 5, seed=52)
    a = O.Oracle(s0).local_energy(th, x)
    b = O.Oracle(s1).local_energy(th, x + shift)
    np.testing.assert_allclose(b["log_abs"], a["log_abs"], atol=1e-11)
    np.testing.assert_allclose(b["e_loc"], a["e_loc"], rtol=1e-8, atol=1e-8)


# --------------------------------------------------------------------------
# Metropolis-Hastings (Electron Sampler section)
# --------------------------------------------------------------------------
def _hydrogenic(z, K=1):
    s = small(1, 0, [0, 0, 0], [z], L=1, w1=2, K=K)
    th, v = zero_theta(s)
    v["g_up"][...] = 1.0
    v["sig_up"][...] = z * np.eye(3)
    return s, th


def test_detailed_balance_of_accept_rule():
    """pi(x) a(x->y) = pi(y) a(y->x) with pi = |psi|^2: the acceptance rate
    of a fixed move over a fine grid of u equals min(1, psi(y)^2/psi(x)^2).
    Using |psi| instead of |psi|^2 or a reversed inequality fails."""
    s = I.System("LiH-s", I.lih().nuc_xyz, I.lih().nuc_z, 2, 2, 2, 8, 4, 2, 4, I.lih().electron_site, 1.0)
    th = I.init_params(s, seed=61)
    o = O.Oracle(s)
    rng = np.random.default_rng(62)
    G = 4000
    ugrid = (np.arange(G) + 0.5) / G
    sigma = 0.2
    for _ in range(4):
        x = I.init_walkers(s, 1, seed=int(rng.integers(1 << 30)))
        z = rng.standard_normal((1, 1, 3 * s.n_elec))
        y = x + sigma * z.reshape(x.shape)
        lx = o.log_psi(th, x)["log_abs"]
        ly = o.log_psi(th, y)["log_abs"]
        rates = []
        for (a, la, zz) in ((x, lx, z), (y, ly, -z)):
            xs = np.repeat(a, G, axis=0)
            _, _, acc = o.metropolis(th, xs, np.repeat(la, G), 1, sigma, 0, z=np.repeat(zz, G, axis=1),
                                     u=ugrid[None, :])
            rates.append(acc.mean())
        pxy = np.exp(2 * lx[0]) * rates[0]
        pyx = np.exp(2 * ly[0]) * rates[1]
        assert rates[0] == pytest.approx(min(1.0, np.exp(2 * (ly[0] - lx[0]))), abs=1.0 / G)
        assert pxy == pytest.approx(pyx, rel=2e-3 / min(rates))


def test_chain_samples_hydrogenic_density():
    """Chain on psi = exp(-Z r): samples follow 4 Z^3 r^2 exp(-2 Z r), so
    <r> = 3/(2Z) and the radial histogram matches (chi-square)."""
    z = 2.0
    s, th = _hydrogenic(z)
    o = O.Oracle(s)
    B = 3000
    x = np.random.default_rng(71).standard_normal((B, 1, 3)) * 0.6
    la = o.log_psi(th, x)["log_abs"]
    x, la, acc = o.metropolis(th, x, la, 300, 0.2, seed=9, step0=0)
    rs = []
    for k in range(10):
        x, la, _ = o.metropolis(th, x, la, 20, 0.2, seed=9, step0=300 + 20 * k)
        rs.append(np.linalg.norm(x[:, 0], axis=1))
    r = np.concatenate(rs)
    assert r.mean() == pytest.approx(1.5 / z, abs=0.02)
    # chi-square against the exact radial CDF on equal-probability bins
    from scipy import stats
    cdf = stats.gamma(a=3, scale=1 / (2 * z)).cdf
    edges = stats.gamma(a=3, scale=1 / (2 * z)).ppf(np.linspace(0, 1, 11))
    last = rs[-1]
    counts = np.histogram(last, bins=edges)[0]
    exp_counts = np.diff(cdf(edges)) * last.size
    chi2 = ((counts - exp_counts) ** 2 / exp_counts).sum()
    assert chi2 < 30.0    # 9 dof; p ~ 4e-4


def test_nonfinite_proposal_rejected_and_state_kept():
    s, th = _hydrogenic(1.0)
    o = O.Oracle(s)
    x = np.array([[[0.5, 0.0, 0.0]]])
    la = o.log_psi(th, x)["log_abs"]
    # a proposal onto the nucleus makes the envelope distance zero; make the
    # orbital vanish there instead: psi = 0 at the node x = 0 of tanh(x)
    s2 = small(1, 0, [0, 0, 0], [1.0], L=1, w1=1, K=1)
    th2, v2 = zero_theta(s2)
    v2["V0"][0, 0] = 1.0
    v2["w_up"][0, 0] = 1.0
    o2 = O.Oracle(s2)
    x2 = np.array([[[0.5, 0.3, 0.2]]])
    la2 = o2.log_psi(th2, x2)["log_abs"]
    z = np.array([[[-0.5 / 0.2, 0.0, 0.0]]])
    xn, ln, acc = o2.metropolis(th2, x2, la2, 1, 0.2, 0, z=z, u=np.array([[1e-300]]))
    assert acc[0] == 0 and np.array_equal(xn, x2) and ln[0] == la2[0]
    assert np.isfinite(la[0])


# --------------------------------------------------------------------------
# the training gradient of Eq. 6
# --------------------------------------------------------------------------
def test_vmc_gradient_hydrogenic_scale():
    """psi = exp(-s r) for the 1-electron Z atom: E(s) = s^2/2 - Z s, so
    dE/ds = s - Z.  The estimator 2 < (E_L - E) d log|psi| / ds > over exact
    samples of |psi|^2 (r ~ Gamma(3, 1/(2s))) must reproduce it: pins the
    factor 2, the centring and the sign of Eq. 6, and d log|psi|/d Sigma."""
    z, sc = 2.0, 1.6
    s, th = _hydrogenic(z)
    v = I.view_params(s, th)
    v["sig_up"][...] = sc * np.eye(3)
    rng = np.random.default_rng(81)
    B = 20000
    r = rng.gamma(3.0, 1.0 / (2 * sc), B)
    d = rng.standard_normal((B, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x = (r[:, None] * d)[:, None, :]
    o = O.Oracle(s)
    e = o.local_energy(th, x)["e_loc"]
    np.testing.assert_allclose(e, -sc * sc / 2 + (sc - z) / r, rtol=1e-10)
    off = I.param_offsets(s)["sig_up"][0]
    dl = o.dlogpsi_dtheta(th, x, [off + 0, off + 4, off + 8]).sum(1)    # d/ds along Sigma = s I
    np.testing.assert_allclose(dl, -r, rtol=1e-12)
    grad = 2.0 * np.mean((e - e.mean()) * dl)
    se = 2.0 * np.std((e - e.mean()) * dl) / np.sqrt(B)
    assert abs(grad - (sc - z)) < 5 * se


def test_orbital_matrices_reproduce_log_psi():
    """The exported orbital matrices give back the oracle's log|psi| through a
    library slogdet and the determinant sum."""
    s = I.System("LiF-s", I.lif().nuc_xyz, I.lif().nuc_z, 3, 2, 2, 8, 4, 3, 4, (0, 1, 1, 0, 1), 0.5)
    th = I.init_params(s, seed=91)
    x = I.init_walkers(s, 6, seed=92)
    o = O.Oracle(s)
    A = o.orbital_matrices(th, x)
    su, lu = np.linalg.slogdet(A[:, 0, :, :3, :3])
    sd, ld = np.linalg.slogdet(A[:, 1, :, :2, :2])
    psi = (su * sd * np.exp(lu + ld)).sum(1)
    ref = o.log_psi(th, x)
    np.testing.assert_allclose(np.log(np.abs(psi)), ref["log_abs"], atol=1e-11)
    np.testing.assert_array_equal(np.sign(psi), ref["sign"])


# --------------------------------------------------------------------------
# residual connections of both streams, the envelope's matrix orientation,
# the sum over nuclei and the per-(orbital, nucleus) envelope parameters
# --------------------------------------------------------------------------
def _log_tanh_chain(s, a):
    """G(s) = tanh(tanh(a tanh s) + tanh s) and d^k log G / ds^k, k = 0, 1, 2,
    by the chain rule written out step by step."""
    t = np.tanh(s)
    t1, t2 = 1 - t ** 2, -2 * t * (1 - t ** 2)
    u = np.tanh(a * t)
    u1 = a * (1 - u ** 2) * t1
    u2 = a * (1 - u ** 2) * t2 - 2 * a * a * u * (1 - u ** 2) * t1 ** 2
    v, v1, v2 = u + t, u1 + t1, u2 + t2
    g = np.tanh(v)
    g1 = (1 - g ** 2) * v1
    g2 = (1 - g ** 2) * v2 - 2 * g * (1 - g ** 2) * v1 ** 2
    return np.log(g), g1 / g, g2 / g - (g1 / g) ** 2


def test_residuals_of_both_streams_closed_form():
    """Three layers, one up and one down electron.  Pair stream: layer 0 maps
    |r_ij| to unit 0, layer 1 adds tanh(a h_ij) to its own input (the pair
    residual), so h_ij^2 = tanh(a tanh r_ij) + tanh r_ij.  One-electron
    stream: layer 0 puts tanh|r_i| in unit 1, layers 1 and 2 carry it on by
    their residual only (their own products are zero there), and layer 2 reads
    the down-spin pair mean into unit 0.  Up orbital = unit 0, down orbital =
    unit 1:  psi = G(r12) tanh(r2) exp(-Z (r1 + r2)) with G as in
    _log_tanh_chain.  Dropping the pair residual changes G; dropping the
    one-electron residual zeroes the down orbital."""
    z, a = 0.8, 1.7
    s = small(1, 1, [0, 0, 0], [z], L=3, w1=3, w2=2, K=1)
    th, v = zero_theta(s)
    v["V0"][3, 1] = 1.0                   # layer 0: |r_i - R| -> unit 1
    v["W2_0"][3, 0] = 1.0                 # pair layer 0: |r_ij| -> pair unit 0
    v["W2_1"][0, 0] = a                   # pair layer 1: tanh(a h) (+ h)
    v["V2"][3 * s.w1 + s.w2, 0] = 1.0     # layer 2: g_i_dn, pair unit 0 -> unit 0
    v["w_up"][0, 0] = 1.0
    v["w_dn"][1, 0] = 1.0
    v["sig_up"][...] = z * np.eye(3)
    v["sig_dn"][...] = z * np.eye(3)
    x = np.random.default_rng(7).standard_normal((10, 2, 3))
    d = x[:, 0] - x[:, 1]
    r12 = np.linalg.norm(d, axis=1)
    r1, r2 = np.linalg.norm(x[:, 0], axis=1), np.linalg.norm(x[:, 1], axis=1)
    G0, G1, G2 = _log_tanh_chain(r12, a)
    h0, h1, h2 = _glt(r2)
    e12 = d / r12[:, None]
    gr1 = G1[:, None] * e12 - z * x[:, 0] / r1[:, None]
    gr2 = -G1[:, None] * e12 + (h1 - z)[:, None] * x[:, 1] / r2[:, None]
    lap = 2 * (G2 + 2 * G1 / r12) - 2 * z / r1 + h2 + 2 * (h1 - z) / r2
    kin = -0.5 * (lap + (gr1 ** 2).sum(1) + (gr2 ** 2).sum(1))
    out = O.Oracle(s).local_energy(th, x)
    np.testing.assert_allclose(out["log_abs"], G0 + h0 - z * (r1 + r2), atol=1e-12)
    np.testing.assert_allclose(out["parts"][:, 0], kin, rtol=1e-8, atol=1e-8)


def test_anisotropic_envelope_orientation_closed_form():
    """One electron, orbital weights 0, bias 1, a non-symmetric Sigma S and a
    nucleus off the origin: psi = exp(-|S (r - R)|).  With d = r - R,
    q = |S d| and M = S^T S: grad log psi = -M d / q, lap log psi =
    -(tr M - |M d|^2 / q^2) / q.  S^T d in place of S d changes q (Eq. 4
    reading: Sigma acts on the electron-nucleus vector)."""
    S = np.array([[1.3, 0.4, -0.2], [0.1, 0.9, 0.5], [-0.6, 0.3, 1.1]])
    R = np.array([0.4, -0.3, 0.7])
    s = small(1, 0, R, [2.0], L=1, K=1)
    th, v = zero_theta(s)
    v["g_up"][...] = 1.0
    v["sig_up"][...] = S
    x = np.random.default_rng(8).standard_normal((12, 1, 3))
    dv = x[:, 0] - R
    Sd = dv @ S.T
    q = np.linalg.norm(Sd, axis=1)
    Md = Sd @ S                            # rows of (S^T S d)^T
    trM = np.trace(S.T @ S)
    lapq = (trM - (Md ** 2).sum(1) / q ** 2) / q
    kin = 0.5 * lapq - 0.5 * (Md ** 2).sum(1) / q ** 2
    out = O.Oracle(s).local_energy(th, x)
    np.testing.assert_allclose(out["log_abs"], -q, atol=1e-12)
    np.testing.assert_allclose(out["parts"][:, 0], kin, rtol=1e-10, atol=1e-10)


def test_two_centre_envelope_closed_form():
    """One electron, two nuclei, K = 2 determinants of which only the first
    has a non-zero orbital (bias [1, 0]): psi = p0 exp(-s0 |r - R0|) + p1
    exp(-s1 |r - R1|), the envelope of Eq. 4 summed over nuclei with the
    first orbital's pi and Sigma = s_m I per nucleus (the second orbital's
    entries differ, so a transposed [K n][M] index would pick them up).
    E_kin = -1/2 lap psi / psi with lap exp(-s rho) = (s^2 - 2 s / rho)
    exp(-s rho).  A max over nuclei, or one nucleus only, fails."""
    R = np.array([[0.0, 0.0, -0.6], [0.2, 0.1, 0.9]])
    s = small(1, 0, R, [3.0, 1.0], L=1, K=2)
    th, v = zero_theta(s)
    v["g_up"][:] = [1.0, 0.0]
    p = np.array([[0.7, 1.9], [5.0, 11.0]])
    sg = np.array([[2.1, 0.8], [0.3, 4.0]])
    v["pi_up"][...] = p
    for k in range(2):
        for m in range(2):
            v["sig_up"][k, m] = sg[k, m] * np.eye(3)
    x = np.random.default_rng(9).standard_normal((12, 1, 3))
    rho = np.linalg.norm(x[:, 0][:, None, :] - R[None], axis=2)       # [B][M]
    e = p[0][None] * np.exp(-sg[0][None] * rho)
    psi = e.sum(1)
    lap = (e * (sg[0] ** 2 - 2 * sg[0] / rho)).sum(1)
    out = O.Oracle(s).local_energy(th, x)
    np.testing.assert_allclose(out["log_abs"], np.log(psi), atol=1e-12)
    np.testing.assert_allclose(out["parts"][:, 0], -0.5 * lap / psi, rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------
# the word -> deviate map of the proposal and accept draws
# --------------------------------------------------------------------------
def _u01(a, b):
    """Uniform in (0, 1] from two 32-bit words: ((a << 21 | b >> 11) + 1) 2^-53."""
    return float(((int(a) << 21) | (int(b) >> 11)) + 1) / 2.0 ** 53


def _kat():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    return [[int(t, 16) for t in r] for r in rows]


def test_box_muller_deviates_from_known_answer_words():
    """Deviates computed by hand from the published Philox4x32-10 outputs:
    counter (0, 0, 0, 0) with key (0, 0) is call d = 0 of walker 0, step 0,
    stream 0, seed 0, so z_0 = sqrt(-2 ln u1) cos(2 pi u2) and z_1 the sine,
    u1 from words 0-1 and u2 from words 2-3; counter (ffffffff x 4) with key
    (ffffffff, ffffffff) is the accept call (d = 0xFFFFFFFF) of walker, step
    and stream 0xFFFFFFFF with the all-ones seed, u from words 0-1.  Swapping
    cos and sin, or the two word pairs, fails."""
    k = _kat()
    w = k[0][6:10]
    u1, u2 = _u01(w[0], w[1]), _u01(w[2], w[3])
    z, _ = O.draw_one(seed=0, stream_id=0, walker=0, n3=2, step=0)
    rad = np.sqrt(-2.0 * np.log(u1))
    np.testing.assert_allclose(z, [rad * np.cos(2 * np.pi * u2), rad * np.sin(2 * np.pi * u2)], rtol=1e-15, atol=1e-15)
    w = k[1][6:10]
    _, u = O.draw_one(seed=(1 << 64) - 1, stream_id=0xFFFFFFFF, walker=0xFFFFFFFF, n3=2, step=0xFFFFFFFF)
    assert u == _u01(w[0], w[1])


def test_draw_counter_layout():
    """Each proposal deviate pair q = 2d, 2d + 1 and the accept uniform come
    from the (KAT-pinned) generator at counter (d, walker, step, stream) and
    key (seed low word, seed high word); checked for arbitrary values of each
    field, so swapped counter fields or key words fail."""
    rng = np.random.default_rng(10)
    for _ in range(6):
        seed = int(rng.integers(0, 1 << 63)) * 2 + 1
        stream, walker, step = (int(v) for v in rng.integers(0, 1 << 32, 3))
        n3 = 7
        z, u = O.draw_one(seed=seed, stream_id=stream, walker=walker, n3=n3, step=step)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        for d in range((n3 + 1) // 2):
            o = O.philox4x32_10([d, walker, step, stream], key)
            u1, u2 = _u01(o[0], o[1]), _u01(o[2], o[3])
            rad = np.sqrt(-2.0 * np.log(u1))
            assert z[2 * d] == pytest.approx(rad * np.cos(2 * np.pi * u2), rel=1e-14, abs=1e-15)
            if 2 * d + 1 < n3:
                assert z[2 * d + 1] == pytest.approx(rad * np.sin(2 * np.pi * u2), rel=1e-14, abs=1e-15)
        o = O.philox4x32_10([0xFFFFFFFF, walker, step, stream], key)
        assert u == _u01(o[0], o[1])


# --------------------------------------------------------------------------
# the pretraining loss of Eq. 5
# --------------------------------------------------------------------------
def test_pretrain_loss_closed_form():
    """One electron, one determinant, orbital weights 0: Phi = g exp(-s r),
    so Eq. 5 is (1/B) sum_p (g e_p - T_p)^2 and d/dg = (2/B) sum_p (g e_p -
    T_p) e_p.  Pins the 1/B normalisation (N read as the number of walkers),
    the square and the derivative; targets equal to Phi give 0."""
    z, g = 1.7, 0.8
    s = small(1, 0, [0.1, 0.0, -0.2], [z], L=2, K=1)
    th, v = zero_theta(s)
    v["g_up"][...] = g
    v["sig_up"][...] = z * np.eye(3)
    rng = np.random.default_rng(41)
    x = rng.standard_normal((9, 1, 3))
    e = np.exp(-z * np.linalg.norm(x[:, 0] - s.nuc_xyz[0], axis=1))
    T = np.zeros((9, 2, 1, 1, 1))
    T[:, 0, 0, 0, 0] = rng.standard_normal(9)
    o = O.Oracle(s)
    d = np.zeros_like(th)
    d[I.param_offsets(s)["g_up"][0]] = 1.0
    loss, dloss = o.pretrain_loss(th, x, T, theta_dir=d)
    r = g * e - T[:, 0, 0, 0, 0]
    assert loss == pytest.approx((r ** 2).sum() / 9, rel=1e-13)
    assert dloss == pytest.approx(2 * (r * e).sum() / 9, rel=1e-12)
    assert o.pretrain_loss(th, x, o.orbital_matrices(th, x)) == 0.0


def test_pretrain_loss_derivative_matches_finite_differences():
    s = I.System("LiF-s", I.lif().nuc_xyz, I.lif().nuc_z, 3, 2, 2, 8, 4, 2, 4, (0, 1, 1, 0, 1), 0.5)
    th = I.init_params(s, seed=43)
    x = I.init_walkers(s, 5, seed=44)
    o = O.Oracle(s)
    rng = np.random.default_rng(45)
    T = o.orbital_matrices(th, x) * (1 + 0.3 * rng.standard_normal((5, 2, 2, 3, 3)))
    for _ in range(3):
        d = rng.standard_normal(th.size)
        _, dl = o.pretrain_loss(th, x, T, theta_dir=d)
        h = 1e-6
        fd = (o.pretrain_loss(th + h * d, x, T) - o.pretrain_loss(th - h * d, x, T)) / (2 * h)
        assert dl == pytest.approx(fd, rel=1e-6, abs=1e-9)


# --------------------------------------------------------------------------
# the isotropic envelope Sigma = sigma I (Eq. 4, special case)
# --------------------------------------------------------------------------
def test_isotropic_two_centre_envelope_closed_form():
    """The two-centre closed form with the isotropic layout: one scalar sigma
    per (orbital, nucleus), psi = p0 exp(-|s0| rho0) + p1 exp(-|s1| rho1).
    A negative sigma acts through |sigma| (the norm of sigma I d); the second
    orbital's entries differ, so a transposed [K n][M] index fails, and so
    does reading sigma from the anisotropic layout's stride."""
    R = np.array([[0.0, 0.0, -0.6], [0.2, 0.1, 0.9]])
    s = small(1, 0, R, [3.0, 1.0], L=1, K=2, envelope=1)
    th, v = zero_theta(s)
    assert v["sig_up"].shape == (2, 2)
    v["g_up"][:] = [1.0, 0.0]
    p = np.array([[0.7, 1.9], [5.0, 11.0]])
    sg = np.array([[2.1, -0.8], [0.3, 4.0]])
    v["pi_up"][...] = p
    v["sig_up"][...] = sg
    x = np.random.default_rng(19).standard_normal((12, 1, 3))
    rho = np.linalg.norm(x[:, 0][:, None, :] - R[None], axis=2)
    a = np.abs(sg[0])[None]
    e = p[0][None] * np.exp(-a * rho)
    psi = e.sum(1)
    lap = (e * (a ** 2 - 2 * a / rho)).sum(1)
    out = O.Oracle(s).local_energy(th, x)
    np.testing.assert_allclose(out["log_abs"], np.log(psi), atol=1e-12)
    np.testing.assert_allclose(out["parts"][:, 0], -0.5 * lap / psi, rtol=1e-10, atol=1e-10)


def _iso_pair(seed=71):
    """A LiH-like network with random weights in both layouts, the
    anisotropic one carrying Sigma = sigma I for the isotropic one's sigma."""
    base = I.System("LiH-s", I.lih().nuc_xyz, I.lih().nuc_z, 2, 2, 2, 8, 4, 3, 4, I.lih().electron_site, 1.0)
    iso = I.isotropic(base)
    rng = np.random.default_rng(seed)
    th_a = I.init_params(base, seed=seed)
    va = I.view_params(base, th_a)
    th_i = np.zeros(I.param_count(iso))
    vi = I.view_params(iso, th_i)
    for name in vi:
        if name.startswith("sig_"):
            sg = rng.uniform(0.5, 2.0, vi[name].shape)
            vi[name][...] = sg
            va[name][...] = sg[..., None, None] * np.eye(3)
        elif name.startswith("pi_"):
            pv = rng.uniform(0.5, 1.5, vi[name].shape)
            vi[name][...] = pv
            va[name][...] = pv
        else:
            vi[name][...] = va[name]
    return base, th_a, iso, th_i


def test_isotropic_layout_is_the_anisotropic_special_case():
    """log|psi|, E_L and its parts agree between the isotropic layout and the
    anisotropic one with Sigma = sigma I; the derivative with respect to an
    isotropic sigma equals the sum of the derivatives with respect to the
    three diagonal entries of the corresponding Sigma (chain rule), for
    every sigma of both spins."""
    base, th_a, iso, th_i = _iso_pair()
    x = I.init_walkers(base, 6, seed=72)
    oa, oi = O.Oracle(base), O.Oracle(iso)
    assert oi.param_count() == I.param_count(iso) == I.param_count(base) - 2 * (3 * 2) * 2 * 8
    ra, ri = oa.local_energy(th_a, x), oi.local_energy(th_i, x)
    np.testing.assert_allclose(ri["log_abs"], ra["log_abs"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(ri["e_loc"], ra["e_loc"], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(ri["parts"], ra["parts"], rtol=1e-11, atol=1e-11)
    offa, offi = I.param_offsets(base), I.param_offsets(iso)
    for tag in ("up", "dn"):
        oi0, shp = offi[f"sig_{tag}"]
        oa0, _ = offa[f"sig_{tag}"]
        n = int(np.prod(shp))
        idx_i = oi0 + np.arange(n)
        idx_a = (oa0 + 9 * np.arange(n))[:, None] + np.array([0, 4, 8])[None]
        gi = oi.dlogpsi_dtheta(th_i, x, idx_i)
        ga = oa.dlogpsi_dtheta(th_a, x, idx_a.reshape(-1)).reshape(x.shape[0], n, 3).sum(2)
        np.testing.assert_allclose(gi, ga, rtol=1e-10, atol=1e-12)
        assert np.abs(gi).max() > 1e-3


def test_isotropic_hydrogenic_exact():
    """Isotropic layout, sigma = Z: psi = exp(-Z r), E_L = -Z^2/2 everywhere."""
    s = small(1, 0, [0.3, -0.2, 0.1], [3.0], L=1, K=1, envelope=1)
    th, v = zero_theta(s)
    v["g_up"][...] = 1.0
    v["sig_up"][...] = 3.0
    x = np.random.default_rng(73).standard_normal((16, 1, 3)) + s.nuc_xyz[0]
    r = O.Oracle(s).local_energy(th, x)
    np.testing.assert_allclose(r["e_loc"], -4.5, atol=1e-10)
