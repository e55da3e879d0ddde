"""Host-side checks of the C ABI: the library loads, exports every symbol
that include/fnvmc.h declares, agrees on the parameter layout and rejects
invalid arguments before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_10287_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fnvmc():
    from paper_2401_10287_amd import fnvmc
    return fnvmc


def test_header_symbols_exported():
    fnvmc = _fnvmc()
    hdr = open(os.path.join(ROOT, "include", "fnvmc.h")).read()
    declared = set(re.findall(r"^\s*(?:fn_status|int64_t|size_t|const char \*)\s*(\w+)\s*\(", hdr, re.M))
    assert declared == set(fnvmc.EXPORTED), declared
    lib = ctypes.CDLL(fnvmc.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("make", [I.he, I.lih, I.lif, I.h_chain, lambda: I.isotropic(I.lih()),
                                  lambda: I.isotropic(I.h_chain())])
def test_param_count_agrees(make):
    fnvmc = _fnvmc()
    s = make()
    n = fnvmc.Config(s, "fp32").param_count()
    assert n == I.param_count(s) == O.Oracle(s).param_count()


def test_serving_types_param_counts():
    fnvmc = _fnvmc()
    for z, q in I.serving_job_types():
        s = I.atom_ion(z, q)
        assert fnvmc.Config(s, "bf16").param_count() == I.param_count(s)


def test_workspace_sizes_positive_and_monotone():
    fnvmc = _fnvmc()
    cfg = fnvmc.Config(I.lih(), "bf16")
    a = cfg.workspace_bytes(64, fnvmc.FN_OP_LOCAL_ENERGY)
    b = cfg.workspace_bytes(4096, fnvmc.FN_OP_LOCAL_ENERGY)
    c = cfg.workspace_bytes(4096, fnvmc.FN_OP_LOG_PSI)
    assert 0 < a < b and 0 < c < b


def test_invalid_config_rejected():
    fnvmc = _fnvmc()
    s = I.lih()
    for field, bad in (("n_layers", 0), ("w1", 0), ("n_det", 0), ("precision", 9), ("n_nuc", 0), ("n_up", -1)):
        cfg = fnvmc.Config(s, "fp32")
        setattr(cfg.c, field, bad)
        assert fnvmc.LIB.fn_param_count(cfg.ptr) == -1
        assert fnvmc.LIB.fn_workspace_bytes(cfg.ptr, 16, 0) == 0
        assert len(fnvmc.LIB.fn_last_error()) > 0


def test_invalid_arguments_return_before_launch():
    fnvmc = _fnvmc()
    cfg = fnvmc.Config(I.he(), "fp64")
    # NULL pointers, negative B, small workspace: all rejected on the host
    assert fnvmc.LIB.fn_log_psi(cfg.ptr, None, None, 4, None, None, None, 0, None) == fnvmc.FN_EINVAL
    assert fnvmc.LIB.fn_local_energy(cfg.ptr, 8, 8, -1, 8, None, None, 8, 0, None) == fnvmc.FN_EINVAL
    st = fnvmc.LIB.fn_local_energy(cfg.ptr, 256, 256, 4, 256, None, None, 256, 16, None)
    assert st == fnvmc.FN_ENOMEM
    assert b"workspace" in fnvmc.LIB.fn_last_error()
    st = fnvmc.LIB.vmc_metropolis_step(cfg.ptr, 256, 256, 256, 4, 1, -1.0, 1, 0, 0, None, 256, 1 << 30, None)
    assert st == fnvmc.FN_EINVAL
    # B == 0 is a no-op
    assert fnvmc.LIB.fn_log_psi(cfg.ptr, None, None, 0, None, None, None, 0, None) == fnvmc.FN_OK


def test_server_job_footprint_host_side():
    from paper_2401_10287_amd import serving
    fnvmc = _fnvmc()
    cfg = fnvmc.Config(I.atom_ion(9, 0), "bf16x6")
    a = serving.job_bytes(cfg, 256)
    b = serving.job_bytes(cfg, 4096)
    assert 0 < a < b
    assert b >= cfg.workspace_bytes(4096, fnvmc.FN_OP_LOCAL_ENERGY)


def test_timing_class_names_checked_on_host():
    fnvmc = _fnvmc()
    assert fnvmc.LIB.fn_timing_select(b"no_such_kernel") == fnvmc.FN_EINVAL
    assert b"no_such_kernel" in fnvmc.LIB.fn_last_error()
    for k in fnvmc.KERNEL_CLASSES:
        assert fnvmc.LIB.fn_timing_select(k.encode()) == fnvmc.FN_OK
    assert fnvmc.LIB.fn_timing_select(None) == fnvmc.FN_OK


def test_tuning_switches_checked_on_host():
    """Every documented tuning switch is accepted (and restored to its
    default), unknown names and out-of-range values are rejected; setting a
    switch touches no device."""
    fnvmc = _fnvmc()
    defaults = {"fused_layer": 1, "layer_dma": 1, "gemm_splitk": 1, "gemm_wide": 1, "pair_mfma": 1, "pair_oc": 0, "pair_items": 0}
    for name, default in defaults.items():
        for v in (0, default):
            assert fnvmc.LIB.fn_tuning_set(name.encode(), v) == fnvmc.FN_OK, name
    assert fnvmc.LIB.fn_tuning_set(b"no_such_switch", 1) == fnvmc.FN_EINVAL
    assert fnvmc.LIB.fn_tuning_set(b"pair_oc", 3) == fnvmc.FN_EINVAL
    assert fnvmc.LIB.fn_tuning_set(b"pair_items", 5000) == fnvmc.FN_EINVAL


def test_group_call_rejects_bad_job_tables():
    """The grouped Metropolis call checks its job table before touching any
    pointer: gaps, overlaps, a wrong total and too many jobs are errors."""
    import ctypes
    from paper_2401_10287_amd import fnvmc
    cfg = fnvmc.Config(I.lih(), "fp32")

    def call(jobs, total):
        tab = (fnvmc.GroupJob * max(1, len(jobs)))(*[fnvmc.GroupJob(*j) for j in jobs])
        return fnvmc.LIB.vmc_metropolis_step_group(cfg.ptr, None, ctypes.addressof(tab), len(jobs), None, None, None,
                                                   total, 1, 0.2, None, 0, None)
    assert call([(0, 10, 1, 0, 0), (12, 5, 1, 0, 0)], 17) == fnvmc.FN_EINVAL        # gap
    assert call([(0, 10, 1, 0, 0), (8, 5, 1, 0, 0)], 15) == fnvmc.FN_EINVAL         # overlap
    assert call([(0, 10, 1, 0, 0)], 11) == fnvmc.FN_EINVAL                          # total
    assert call([(0, 0, 1, 0, 0)], 0) == fnvmc.FN_EINVAL                            # empty job
    assert call([(q, 1, 1, 0, 0) for q in range(65)], 65) == fnvmc.FN_EINVAL        # too many
    assert b"job" in fnvmc.LIB.fn_last_error() or b"B_total" in fnvmc.LIB.fn_last_error()


def test_server_create_checks_gang_limits():
    """fn_server_create validates its gang limits on the host (no device
    work: the arena and stream are never touched without jobs)."""
    import ctypes
    import numpy as np
    from paper_2401_10287_amd import serving  # noqa: F401  (declares the server signatures)
    fnvmc = _fnvmc()
    L = fnvmc.LIB
    res = np.zeros(64 * 4 * 2)
    streams = (ctypes.c_void_p * 2)(None, None)
    h = ctypes.c_void_p()
    for max_gang, walkers in ((0, 4096), (65, 4096), (4, 0)):
        st = L.fn_server_create(1 << 20, 1 << 20, streams, 2, 5, max_gang, walkers, res.ctypes.data, ctypes.byref(h))
        assert st == fnvmc.FN_EINVAL, (max_gang, walkers)
    assert L.fn_server_create(1 << 20, 1 << 20, streams, 2, 5, 64, 4096, res.ctypes.data, ctypes.byref(h)) == 0
    assert L.fn_server_destroy(h) == 0


def test_unknown_envelope_rejected():
    fnvmc = _fnvmc()
    cfg = fnvmc.Config(I.lih(), "fp32")
    cfg.c.envelope = 2
    assert fnvmc.LIB.fn_param_count(cfg.ptr) == -1
    assert b"envelope" in fnvmc.LIB.fn_last_error()
