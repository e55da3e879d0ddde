"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): a driver that compiles fn_oracle.c into its own translation unit
runs every exported call on small systems (both envelope layouts, an empty
spin channel, several determinants and layers); the run must end without a
sanitizer report, and its results must equal the ordinary build's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_10287_amd import inputs as I



@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("san") / "sanitize_driver")
    try:
        O.build_sanitizer_driver(out)
    except subprocess.CalledProcessError as e:
        if "asan" in (e.stderr or "").lower() or "ubsan" in (e.stderr or "").lower():
            pytest.skip("sanitizer runtime not available: " + e.stderr[-300:])
        raise
    return out


def _cases():
    lih = I.lih()
    small_lih = I.System("LiH-s", lih.nuc_xyz, lih.nuc_z, 2, 2, 3, 8, 4, 3, 4, lih.electron_site, 1.0)
    li_ion = I.atom_ion(3, 1, n_layers=2, w1=8, w2=4, n_det=2)          # 2 up, 0 down
    return [("He", I.he()), ("LiH-s", small_lih), ("LiH-s iso", I.isotropic(small_lih)), ("Li+", li_ion)]


@pytest.mark.parametrize("label,s", _cases(), ids=[c[0] for c in _cases()])
def test_oracle_clean_under_sanitizers(driver, tmp_path, label, s):
    B = 3
    th = I.init_params(s, seed=91)
    rng = np.random.default_rng(92)
    v = I.view_params(s, th)
    for name in v:
        if name.startswith("sig_") or name.startswith("pi_"):
            v[name][...] += 0.1 * rng.standard_normal(v[name].shape)
    d = rng.standard_normal(th.size)
    x = I.init_walkers(s, B, seed=93)
    idx = np.array([0, th.size // 3, th.size - 1], dtype=np.int64)
    N = s.n_elec
    hdr = np.array([s.n_nuc, s.n_up, s.n_dn, s.n_layers, s.w1, s.w2, s.n_det, s.envelope, B, idx.size], np.int32)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        for a in (hdr, np.asarray(s.nuc_xyz, np.float64).reshape(-1), np.asarray(s.nuc_z, np.float64), th, d,
                  np.ascontiguousarray(x).reshape(-1), idx):
            f.write(np.ascontiguousarray(a).tobytes())
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, str(fin), str(fout)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    out = np.fromfile(fout, dtype=np.float64)
    K, nmax = s.n_det, max(s.n_up, s.n_dn)
    sizes = [B, B, B, B, 4 * B, 3 * N * B, B, idx.size * B, B * 2 * K * nmax * nmax, B * 2 * K * nmax * nmax, 3 * B,
             B * K, B * K, B * N * 3, B, B]
    assert out.size == sum(sizes)
    parts = np.split(out, np.cumsum(sizes)[:-1])
    o = O.Oracle(s)
    lp = o.log_psi(th, x, theta_dir=d)
    le = o.local_energy(th, x)
    mats, matd = o.orbital_matrices_dir(th, d, x)
    xm, lm, am = o.metropolis(th, x, lp["log_abs"], 3, 0.2, seed=7, step0=0, stream_id=2)
    ref = [lp["log_abs"], lp["sign"], lp["dlog"], le["e_loc"], le["parts"], le["grad"], le["lap"],
           o.dlogpsi_dtheta(th, x, idx), mats, matd, o.coulomb(x)]
    for got, want in zip(parts[:len(ref)], ref):
        np.testing.assert_allclose(got, np.ravel(want), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(parts[-3], xm.reshape(-1), rtol=0, atol=1e-13)
    np.testing.assert_array_equal(parts[-1], am.astype(np.float64))
