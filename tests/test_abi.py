"""Host-side checks of the C ABI (no GPU needed): the built library loads, exports every
function include/lgsr.h declares, fills documented defaults and rejects bad arguments
before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lgsr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lgsr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2607_04127_amd import lgsr
    if not os.path.exists(lgsr.LIB_PATH):
        pytest.fail("liblgsr.so is not built (python -m paper_2607_04127_amd.build)")
    return lgsr


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 12
    assert set(names) == set(L.EXPORTS)
    cdll = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(cdll, n), n


def test_defaults(L):
    o = L.default_opts()
    assert (o.cutoff_sigma, o.alpha_max, o.near, o.drop_tau, o.flags) == (3.0, pytest.approx(0.99), pytest.approx(0.2),
                                                                          0.5, 0)
    assert o.alpha_thr == pytest.approx(1 / 255) and o.T_min == pytest.approx(1e-4) and o.den_eps == pytest.approx(1e-6)
    w = L.default_loss_weights()
    assert (w.w_depth, w.lambda_n) == (1.0, 1.0) and w.lambda_ng == pytest.approx(0.05)


def test_null_and_bad_arguments_rejected(L):
    lib = L.lib()
    assert lib.lgsr_create(None, 0, None) == L.LGSR_EINVAL
    assert lib.lgsr_forward(None, None, None, 0, None, None, None, None) == L.LGSR_EINVAL
    assert lib.lgsr_loss(None, 0, None, None, None, None, None, None) == L.LGSR_EINVAL
    assert lib.lgsr_backward(None, None, None, None, None) == L.LGSR_EINVAL
    assert lib.lgsr_query(None, None, None) == L.LGSR_EINVAL
    assert lib.lgsr_tile_list(None, None, 0, 0, None, 0, None) == L.LGSR_EINVAL
    assert lib.lgsr_sync(None) == L.LGSR_EINVAL
    lib.lgsr_destroy(None)
    lib.lgsr_state_free(None)
    assert lib.lgsr_last_error(None) == b"null context"


def test_no_device_reports_edevice(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert L.lib().lgsr_create(ctypes.byref(h), 0, None) == L.LGSR_EDEVICE
