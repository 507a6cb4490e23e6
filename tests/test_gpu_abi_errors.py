"""Call-order and argument errors of the C ABI on a live handle."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture()
def handle():
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth
    U, V = synth.compression_UV(20, 20, 2, 8, 2, 99)
    eng = oc.Octen(20, 20, 3, 2, 8, 2, torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda())
    yield oc, eng, torch
    eng.close()


def test_wrong_call_order(handle):
    oc, eng, torch = handle
    assert oc.octen_update_replicas(eng.h) == oc.OCTEN_ERR_STATE
    assert oc.octen_cp_als_replicas(eng.h, 5, 0.0, oc.OCTEN_INIT_PREV) == oc.OCTEN_ERR_STATE
    A = torch.empty((20, 3), dtype=torch.float64, device="cuda")
    C = torch.empty((10, 3), dtype=torch.float64, device="cuda")
    assert oc.octen_recover_factors(eng.h, A, A, C, 10) == oc.OCTEN_ERR_STATE
    X = torch.randn((4, 20, 20), dtype=torch.float64, device="cuda")
    W = torch.randn((4, eng.M1), dtype=torch.float64, device="cuda")
    eng.compress_batch(X, W)
    eng.update_replicas()
    assert oc.octen_update_replicas(eng.h) == oc.OCTEN_ERR_STATE   # nothing new compressed
    assert oc.octen_recover_factors(eng.h, A, A, C, 10) == oc.OCTEN_ERR_STATE  # no ALS yet
    init = torch.randn((2, 3, 8, 3), dtype=torch.float64, device="cuda")
    eng.cp_als_replicas(5, init=init)
    small = torch.empty((2, 3), dtype=torch.float64, device="cuda")
    assert oc.octen_recover_factors(eng.h, A, A, small, 2) == oc.OCTEN_ERR_ARG  # C too small
    assert eng.recover_factors(A, A.clone(), C) == 4
    assert oc.octen_recover_factors(eng.h, A, A, C, 10) == oc.OCTEN_ERR_STATE  # twice
    assert "recover" in oc.octen_last_error(eng.h)


def test_bad_arguments(handle):
    oc, eng, torch = handle
    W = torch.randn((4, eng.M1), dtype=torch.float64, device="cuda")
    assert oc.octen_compress_batch(eng.h, None, 4, W) == oc.OCTEN_ERR_ARG
    assert oc.octen_compress_batch(eng.h, W, 0, W) == oc.OCTEN_ERR_ARG
    assert oc.octen_cp_als_replicas(eng.h, 0, 0.0, oc.OCTEN_INIT_GIVEN, W) == oc.OCTEN_ERR_ARG
    assert oc.octen_get_state(eng.h, 99, W, 8) == oc.OCTEN_ERR_ARG
    assert oc.octen_get_state(eng.h, oc.OCTEN_STATE_Y, W, 8) == oc.OCTEN_ERR_ARG
