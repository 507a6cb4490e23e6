"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, and its host-only logic (argument
validation, identifiability verdicts) matches the oracle."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for path in HEADERS:
        txt = open(path).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(octen_[a-z_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def oc():
    from paper_1807_01350_amd import octen
    return octen


def test_library_exports_every_declared_function(oc):
    names = declared_functions()
    assert "octen_init" in names and "octen_fit" in names and "octen_nm_init" in names
    lib = ctypes.CDLL(oc.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) <= set(oc.EXPORTED)


def test_abi_version(oc):
    assert oc.octen_abi_version() == oc.OCTEN_ABI_VERSION == 1


def test_config_struct_layout(oc):
    assert ctypes.sizeof(oc.octen_config) == 56
    assert oc.octen_config.I.offset == 32 and oc.octen_config.flags.offset == 48


@pytest.mark.parametrize("I,J,K,t,R,P,Q,S", [
    (50, 50, 50, 10, 5, 4, 20, 3),
    (1000, 1000, 1000, 50, 10, 12, 60, 3),
    (1000, 1000, 100, 20, 10, 25, 50, 10),
    (50, 50, 50, 10, 1, 4, 20, 3),
    (100000, 100000, 2000, 100, 20, 16, 80, 3),
])
def test_identifiability_matches_oracle(oc, I, J, K, t, R, P, Q, S):
    from oracle import identifiability
    cfg = oc.make_config(I, J, R, P, Q, S)
    st, bits, pmin = oc.octen_check_identifiable(cfg, K, t)
    assert st == oc.OCTEN_OK
    ob, op = identifiability(I, J, K, t, R, P, Q, S)
    assert bits == ob
    assert pmin == pytest.approx(op, rel=1e-15)


@pytest.mark.parametrize("field,value,status", [
    ("R", 0, 1), ("R", 33, 1), ("P", 0, 1), ("S", 0, 1), ("Q", 3, 1), ("Q", 129, 1),
    ("abi_version", 2, 1), ("x_dtype", 7, 1), ("compress_dtype", 3, 6), ("I", 0, 1),
])
def test_invalid_config_rejected_before_any_launch(oc, field, value, status):
    cfg = oc.make_config(50, 50, 5, 4, 20, 3)
    setattr(cfg, field, value)
    st, h = oc.octen_init(cfg, 1, 1, None)
    assert st == status
    assert not h.value
    st, _, _ = oc.octen_check_identifiable(cfg, 10, 10)
    assert st == status


def test_null_arguments_rejected(oc):
    cfg = oc.make_config(50, 50, 5, 4, 20, 3)
    st, h = oc.octen_init(cfg, None, None, None)
    assert st == oc.OCTEN_ERR_ARG and not h.value
    assert oc.octen_update_replicas(None) == oc.OCTEN_ERR_ARG
    assert oc.octen_destroy(None) == oc.OCTEN_ERR_ARG
    assert oc.octen_status_str(oc.OCTEN_ERR_STATE) == "call out of order"


def test_nm_config_struct_layout(oc):
    assert ctypes.sizeof(oc.octen_nm_config) == 64
    assert oc.octen_nm_config.dims.offset == 24


@pytest.mark.parametrize("field,value,status", [
    ("N", 2, 1), ("N", 7, 1), ("R", 0, 1), ("R", 33, 1), ("P", 0, 1), ("S", 0, 1), ("Q", 3, 1),
    ("abi_version", 2, 1), ("Q", 33, 6), ("R", 13, 1),
])
def test_nm_invalid_config_rejected_before_any_launch(oc, field, value, status):
    cfg = oc.make_nm_config((30, 40, 50), 5, 4, 12, 3)
    setattr(cfg, field, value)
    st, h = oc.octen_nm_init(cfg, [1, 1, 1], None)
    assert st == status
    assert not h.value


def test_nm_limits_rejected(oc):
    # Q^N above 2^22 (N = 6, Q = 13) and a zero mode size
    cfg = oc.make_nm_config((30, 30, 30, 30, 30), 5, 4, 13, 3)
    st, h = oc.octen_nm_init(cfg, [1] * 5, None)
    assert st == oc.OCTEN_ERR_UNSUPPORTED and not h.value
    # Q^N above 2^22 at N = 5 (22^5)
    cfg = oc.make_nm_config((30, 30, 30, 30), 5, 4, 22, 3)
    st, h = oc.octen_nm_init(cfg, [1] * 4, None)
    assert st == oc.OCTEN_ERR_UNSUPPORTED and not h.value
    cfg = oc.make_nm_config((30, 0, 30), 5, 4, 12, 3)
    st, h = oc.octen_nm_init(cfg, [1] * 3, None)
    assert st == oc.OCTEN_ERR_ARG and not h.value
    cfg = oc.make_nm_config((30, 40, 50), 5, 4, 12, 3)
    st, h = oc.octen_nm_init(cfg, None, None)
    assert st == oc.OCTEN_ERR_ARG and not h.value
    assert oc.octen_nm_update_replicas(None) == oc.OCTEN_ERR_ARG
    assert oc.octen_nm_destroy(None) == oc.OCTEN_ERR_ARG
