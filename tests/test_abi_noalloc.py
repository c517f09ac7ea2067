"""Host-side argument checks of hm_sre_noalloc (no GPU: every call below fails validation before
anything is launched, so the fake device pointers are never dereferenced)."""
import ctypes

import pytest

import paper_2601_07824_amd as hm

HM_OK, HM_E_ARG, HM_E_DTYPE, HM_E_SIZE, HM_E_WORKSPACE, HM_E_UNSUPPORTED, HM_E_HIP, HM_E_ALIGN = range(8)
P = ctypes.c_void_p


@pytest.fixture(scope="module")
def L():
    return hm.lib()


@pytest.fixture(scope="module")
def h(L):
    hh = P()
    assert L.hm_create(ctypes.byref(hh)) == HM_OK
    yield hh
    L.hm_destroy(hh)


def q_arr(*q):
    return (ctypes.c_double * len(q))(*q)


def test_noalloc_argument_errors(L, h):
    q = q_arr(2.0)
    good = P(0x100000)
    f = L.hm_sre_noalloc
    assert f(None, good, 8, 0, q, 1, good, None) == HM_E_ARG
    assert f(h, None, 8, 0, q, 1, good, None) == HM_E_ARG
    assert f(h, good, 8, 0, q, 1, None, None) == HM_E_ARG
    assert f(h, good, 8, 5, q, 1, good, None) == HM_E_DTYPE
    assert f(h, P(0x100004), 8, 0, q, 1, good, None) == HM_E_ALIGN
    assert f(h, good, 8, 0, q, 0, good, None) == HM_E_ARG
    assert f(h, good, 8, 0, q_arr(0.0), 1, good, None) == HM_E_ARG
    # sizes that need the two-pass kernels (and their exchange buffer)
    assert f(h, good, 17, 0, q, 1, good, None) == HM_E_SIZE
    assert f(h, good, 16, 1, q, 1, good, None) == HM_E_SIZE
    assert f(h, good, 27, 0, q, 1, good, None) == HM_E_SIZE
