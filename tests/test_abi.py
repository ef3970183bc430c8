"""CPU checks of the C ABI: the library loads, exports every function that
include/pprt.h declares, its host helpers agree with the oracle, and host-side
validation returns the documented status codes.  No kernel is launched."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from paper_0903_1949_amd import pprt
from oracle.quadrature import gauss_legendre01 as oracle_gauss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = pprt.load_library()
    declared = pprt.declared_symbols()
    assert len(declared) >= 15
    nm = subprocess.run(["nm", "-D", "--defined-only", pprt.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = {line.split()[-1] for line in nm.splitlines() if line.strip()}
    missing = [s for s in declared if s not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for s in declared:
        assert hasattr(lib, s)


def test_version_and_status_strings():
    lib = pprt.load_library()
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    assert lib.pprt_version(C.byref(a), C.byref(b), C.byref(c)) == 0
    assert (a.value, b.value) >= (0, 1)
    for code in range(10):
        assert lib.pprt_status_string(code)
    assert lib.pprt_status_string(99) == b"unknown status"


@pytest.mark.parametrize("n", [1, 2, 3, 4, 8, 16, 32, 64])
def test_host_gauss_rule_matches_oracle(n):
    mu, w = pprt.gauss_legendre01(n)
    mo, wo = oracle_gauss(n)
    assert np.allclose(mu, mo, rtol=0, atol=2e-15)
    # both rules carry the recurrence's rounding, which grows with n
    assert np.max(np.abs(w / wo - 1)) < 1e-15 * n * n + 1e-14
    assert abs(w.sum() - 1) < 1e-14


def test_gauss_rejects_bad_n():
    lib = pprt.load_library()
    mu = (C.c_double * 4)()
    assert lib.pprt_gauss_legendre01(0, mu, mu) == 1
    assert lib.pprt_gauss_legendre01(65, mu, mu) == 1
    assert lib.pprt_gauss_legendre01(4, None, mu) == 1


@pytest.mark.parametrize("kw,status", [
    (dict(nd=[64], na=4, nf=21), "OK"),
    (dict(nd=[48, 256, 100], na=8, nf=1024, precision=pprt.FP64), "OK"),
    (dict(nd=[], na=4, nf=21), "E_SHAPE"),
    (dict(nd=[1], na=4, nf=21), "E_SHAPE"),
    (dict(nd=[5, 0], na=4, nf=21), "E_SHAPE"),
    (dict(nd=[5], na=0, nf=21), "E_SHAPE"),
    (dict(nd=[5], na=33, nf=21), "E_SHAPE"),
    (dict(nd=[5], na=9, nf=21), "E_UNSUPPORTED"),
    (dict(nd=[5], na=4, nf=0), "E_SHAPE"),
    (dict(nd=[5], na=4, nf=8, precision=7), "E_INVALID_ARG"),
    (dict(nd=[5], na=4, nf=8, lower_bc=3), "E_INVALID_ARG"),
    (dict(nd=[5], na=4, nf=8, outputs=0x400), "E_INVALID_ARG"),
    (dict(nd=[5], na=4, nf=8, outputs=0x300), "OK"),
    (dict(nd=[5], na=4, nf=8, waves_per_block=3), "E_INVALID_ARG"),
])
def test_shape_validation(kw, status):
    st, msg = pprt.shape_check(**kw)
    assert st == status, msg
    if status != "OK":
        assert msg


def test_create_without_device_reports_e_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    lib = pprt.load_library()
    h = C.c_void_p()
    assert lib.pprt_create(C.byref(h), 0) == 3
    assert not h.value


def test_null_arguments_rejected_without_device():
    lib = pprt.load_library()
    assert lib.pprt_plan_create(None, None, None, None, None) == 1
    assert lib.pprt_formal_solution(None, None, None) == 1
    assert lib.pprt_two_level_ali_step(None, None, None, None, None, None, None) == 1
    assert lib.pprt_two_level_ali(None, None, None, None, None, None, None, None) == 1
    assert lib.pprt_sync(None, None) == 1
    assert lib.pprt_set_stream(None, None) == 1
    assert lib.pprt_plan_workspace_bytes(None, None) == 1
    assert lib.pprt_plan_set_thick_mode(None, 0) == 1
    assert lib.pprt_thick_counts(None, None, None) == 1
    assert lib.pprt_thick_counts_reset(None) == 1
    assert lib.pprt_plan_scattering_vjp_workspace_bytes(None, None) == 1
    assert lib.pprt_formal_solution_scattering_vjp(None, None, None, None, None, None) == 1
    assert lib.pprt_last_error(None) == b""
    lib.pprt_destroy(None)
    lib.pprt_plan_destroy(None)


def test_binding_refuses_missing_library(tmp_path):
    pprt_mod = pprt
    saved = pprt_mod._lib
    try:
        pprt_mod._lib = None
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            pprt_mod.load_library(str(tmp_path / "libpprt.so"))
    finally:
        pprt_mod._lib = saved
