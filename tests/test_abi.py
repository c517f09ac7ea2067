"""C-ABI checks that need no GPU: the library loads, exports every function include/hmag.h declares,
and rejects invalid arguments synchronously on the host (nothing is launched on error, so fake
device pointers are safe in these cases)."""
import ctypes
import os
import re

import pytest

import paper_2601_07824_amd as hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmag.h")

HM_OK, HM_E_ARG, HM_E_DTYPE, HM_E_SIZE, HM_E_WORKSPACE, HM_E_UNSUPPORTED, HM_E_HIP, HM_E_ALIGN, HM_E_NOT_NORMALIZED = range(9)
P = ctypes.c_void_p


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    return hm.lib()


@pytest.fixture(scope="module")
def h(L):
    hh = P()
    assert L.hm_create(ctypes.byref(hh)) == HM_OK
    yield hh
    L.hm_destroy(hh)


def test_every_declared_symbol_is_exported_and_bound(L):
    decl = declared_functions()
    assert decl, "no declarations parsed"
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(hm.EXPORTED_SYMBOLS) == decl


def test_version_and_status_strings(L):
    assert b"gfx950" in L.hm_version()
    for s in range(9):
        assert L.hm_status_string(s).startswith(b"HM_")


def q_arr(*q):
    return (ctypes.c_double * len(q))(*q)


def test_sre_argument_errors(L, h):
    q = q_arr(2.0)
    good = P(0x100000)  # never dereferenced: every call below fails validation first
    ws = P(0x200000)
    assert L.hm_sre(None, good, 8, 0, q, 1, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre(h, None, 8, 0, q, 1, good, ws, 1 << 30, None) == HM_E_ARG
    assert b"psi" in L.hm_last_error()
    assert L.hm_sre(h, good, 8, 7, q, 1, good, ws, 1 << 30, None) == HM_E_DTYPE
    assert L.hm_sre(h, good, 0, 0, q, 1, good, ws, 1 << 30, None) == HM_E_SIZE
    assert L.hm_sre(h, good, 27, 0, q, 1, good, ws, 1 << 30, None) == HM_E_SIZE
    assert L.hm_sre(h, good, 8, 0, q_arr(-1.0), 1, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre(h, good, 8, 0, q_arr(float("nan")), 1, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre(h, good, 8, 0, q, 0, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre(h, good, 8, 0, q, 9, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre(h, P(0x100004), 8, 0, q, 1, good, ws, 1 << 30, None) == HM_E_ALIGN
    assert L.hm_sre(h, P(0x100008), 8, 1, q, 1, good, ws, 1 << 30, None) == HM_E_ALIGN  # c128 needs 16 B
    assert L.hm_sre(h, good, 8, 0, q, 1, good, P(0x200010), 1 << 30, None) == HM_E_ALIGN
    assert L.hm_sre(h, good, 8, 0, q, 1, good, ws, 16, None) == HM_E_WORKSPACE
    assert b"workspace" in L.hm_last_error()


def test_partial_rows_and_values_errors(L, h):
    q = q_arr(2.0)
    good, ws = P(0x100000), P(0x200000)
    assert L.hm_sre_partial(h, good, 8, 0, q, 1, 5, 3, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_partial(h, good, 8, 0, q, 1, 0, 257, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_rows(h, good, 8, 0, good, -1, q, 1, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_rows(h, good, 8, 0, None, 4, q, 1, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_row_values(h, good, 8, 0, 256, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_row_values(h, good, 8, 0, 3, good, ws, 8, None) == HM_E_WORKSPACE
    assert L.hm_sre_grad(h, good, 8, 0, 1.0, good, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_grad(h, good, 8, 0, 2.0, good, None, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_mana(h, good, 0, 0, good, ws, 1 << 30, None) == HM_E_SIZE
    assert L.hm_mana_partial(h, good, 4, 0, 0, 82, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_finalize(8, q, 1, None, good, None) == HM_E_ARG
    assert L.hm_sre_sampled(h, good, 8, 0, good, 1, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_sampled(h, good, 8, 0, None, 16, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_sampled(h, good, 8, 0, good, 16, good, ws, 64, None) == HM_E_WORKSPACE


def test_batched_errors_and_workspace(L, h):
    q = q_arr(2.0)
    good, ws = P(0x100000), P(0x200000)
    ns = (ctypes.c_int * 4)(3, 8, 8, 20)
    ptrs = (P * 4)(good, good, good, good)
    b, b1 = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.hm_sre_batched_workspace(h, ns, 4, 0, 1, ctypes.byref(b)) == HM_OK
    assert L.hm_workspace_size(h, 0, 20, 0, 1, 0, ctypes.byref(b1)) == HM_OK
    assert b.value >= b1.value and b.value % 256 == 0
    assert L.hm_sre_batched_workspace(h, ns, 0, 0, 1, ctypes.byref(b)) == HM_E_ARG
    bad = (ctypes.c_int * 2)(3, 27)
    assert L.hm_sre_batched_workspace(h, bad, 2, 0, 1, ctypes.byref(b)) == HM_E_SIZE
    assert L.hm_sre_batched(h, None, ns, 4, 0, q, 1, good, ws, 1 << 34, None) == HM_E_ARG
    ptrs[2] = P(0x100004)
    assert L.hm_sre_batched(h, ptrs, ns, 4, 0, q, 1, good, ws, 1 << 34, None) == HM_E_ALIGN
    ptrs[2] = good
    assert L.hm_sre_batched(h, ptrs, ns, 4, 0, q, 1, good, ws, 256, None) == HM_E_WORKSPACE


def test_options_and_forced_paths(L, h):
    hh = P()
    assert L.hm_create(ctypes.byref(hh)) == HM_OK
    try:
        assert L.hm_set_option(hh, 1, 3) == HM_E_ARG
        assert L.hm_set_option(hh, 99, 0) == HM_E_ARG
        b = ctypes.c_size_t()
        assert L.hm_set_option(hh, 1, 2) == HM_OK  # two-pass needs n >= 11 for c64
        assert L.hm_workspace_size(hh, 0, 8, 0, 1, 0, ctypes.byref(b)) == HM_E_UNSUPPORTED
        assert L.hm_workspace_size(hh, 0, 16, 0, 1, 0, ctypes.byref(b)) == HM_OK
        assert L.hm_set_option(hh, 1, 1) == HM_OK  # workgroup-resident holds at most 2^15 folded c64 values
        assert L.hm_workspace_size(hh, 0, 17, 0, 1, 0, ctypes.byref(b)) == HM_E_UNSUPPORTED
        assert L.hm_workspace_size(hh, 0, 16, 0, 1, 0, ctypes.byref(b)) == HM_OK
        assert L.hm_workspace_size(hh, 0, 16, 1, 1, 0, ctypes.byref(b)) == HM_E_UNSUPPORTED  # c128: 2^14
        assert L.hm_set_option(hh, 1, 0) == HM_OK
        assert L.hm_set_option(hh, 3, 3) == HM_E_ARG
        assert L.hm_set_option(hh, 5, 16) == HM_E_ARG
        assert L.hm_set_option(hh, 3, 4) == HM_OK
        assert L.hm_workspace_size(hh, 0, 20, 1, 1, 0, ctypes.byref(b)) == HM_OK
        assert L.hm_set_option(hh, 5, 13) == HM_OK  # row bits 13 leaves 6 for the column pass at n = 20
        assert L.hm_workspace_size(hh, 0, 20, 0, 1, 0, ctypes.byref(b)) == HM_OK
        assert L.hm_set_option(hh, 5, 6) == HM_OK   # 14 column bits: more than a column tile holds
        assert L.hm_workspace_size(hh, 0, 21, 0, 1, 0, ctypes.byref(b)) == HM_E_UNSUPPORTED
    finally:
        L.hm_destroy(hh)


def test_workspace_sizes(L, h):
    b = ctypes.c_size_t()
    prev = 0
    for n in range(1, 23):
        assert L.hm_workspace_size(h, 0, n, 0, 1, 0, ctypes.byref(b)) == HM_OK
        assert b.value >= 16 * (1 << n) and b.value % 256 == 0
        assert b.value >= prev
        prev = b.value
    assert L.hm_workspace_size(h, 0, 8, 5, 1, 0, ctypes.byref(b)) == HM_E_DTYPE
    assert L.hm_workspace_size(h, 1, 20, 0, 1, 4096, ctypes.byref(b)) == HM_OK
    assert L.hm_workspace_size(h, 2, 20, 1, 1, 0, ctypes.byref(b)) == HM_OK and b.value >= 16 << 20


def _ws_ok(ctx_opts, n, dtype):
    hh = P()
    assert hm.lib().hm_create(ctypes.byref(hh)) == HM_OK
    try:
        for k, v in ctx_opts:
            assert hm.lib().hm_set_option(hh, k, v) == HM_OK
        b = ctypes.c_size_t()
        st = hm.lib().hm_workspace_size(hh, 0, n, dtype, 1, 0, ctypes.byref(b))
        return st, hm.lib().hm_last_error()
    finally:
        hm.lib().hm_destroy(hh)


def test_planner_accepts_every_configuration_the_gpu_tests_use():
    """Host-side planning of the forced paths and tile options exercised by the GPU parity tests."""
    FP, BS, RRB, CRB, RB, PIPE, SPLIT = 1, 2, 3, 4, 5, 6, 7
    cases = []
    for rb in (0, 4):
        for dt, n in ((1, 11), (1, 12), (1, 13), (0, 12), (0, 13), (0, 14)):
            cases.append(([(FP, 2), (BS, 5), (RRB, rb), (CRB, rb)], n, dt))
    for split in (1, 2):
        for dt, n in ((1, 12), (1, 13), (1, 14), (0, 12), (0, 13), (0, 15)):
            cases.append(([(FP, 2), (PIPE, 2), (SPLIT, split), (BS, 5)], n, dt))
    for n in (16, 20):
        for dt, rb, rbits, pipe in ((0, 0, 0, 0), (1, 0, 0, 0), (0, 4, 0, 0), (0, 4, 12, 0), (0, 5, 9, 0),
                                    (0, 0, 0, 1), (0, 0, 0, 2), (1, 0, 0, 2)):
            o = [(RRB, rb), (CRB, rb)]
            if rbits and n == 20:
                o.append((RB, rbits))
            if pipe:
                o += [(PIPE, 2), (SPLIT, pipe)]
            cases.append((o, n, dt))
    for dt, n in ((1, 11), (1, 13), (0, 12), (0, 14)):
        cases.append(([(FP, 2), (BS, 7), (SPLIT, 2)], n, dt))
    for n in (13, 15):
        cases.append(([(FP, 2), (BS, 7), (SPLIT, 2), (RRB, 4)], n, 0))
    for dt, n in ((1, 12), (1, 14), (0, 12), (0, 15), (0, 20), (1, 20)):
        cases.append(([(FP, 2), (BS, 5), (8, 2)], n, dt))
    for n in (16, 20):
        cases += [([(PIPE, 1), (RB, 12 if n == 20 else 0), (SPLIT, 2)], n, 0), ([(PIPE, 1), (SPLIT, 2)], n, 1)]
    for dt, n in ((1, 13), (1, 14), (1, 15), (0, 14), (0, 15), (0, 16)):
        cases.append(([(FP, 1)], n, dt))
    cases += [([(FP, 2)], 16, 1), ([(FP, 2), (PIPE, 2)], 16, 1), ([(FP, 2), (PIPE, 2)], 16, 0)]
    for n in range(12, 27):
        for dt in (0, 1):
            if dt == 1 and n > 25:
                continue
            cases.append(([(PIPE, 2)] if n >= 17 else [], n, dt))
    for opts, n, dt in cases:
        st, msg = _ws_ok(opts, n, dt)
        assert st == HM_OK, (opts, n, dt, msg)


def test_autotune_argument_errors(L, h):
    good, ws = P(0x100000), P(0x200000)
    b = ctypes.c_size_t()
    assert L.hm_autotune_workspace(h, 20, 0, 4096, ctypes.byref(b)) == HM_OK and b.value >= 8 << 20
    assert L.hm_autotune_workspace(h, 27, 0, 4096, ctypes.byref(b)) == HM_E_SIZE
    assert L.hm_autotune(h, None, 12, 0, 0, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_autotune(h, good, 12, 0, 0, P(0x200010), 1 << 30, None) == HM_E_ALIGN
    v = (ctypes.c_int64 * 7)()
    assert L.hm_tune_query(h, 12, 0, v, None) == HM_E_ARG  # nothing tuned yet
    assert L.hm_tune_clear(h) == HM_OK


def test_gradient_workspace_all_sizes(L, h):
    b = ctypes.c_size_t()
    for dt in (0, 1):
        for n in range(1, 21):
            assert L.hm_workspace_size(h, 3, n, dt, 1, 0, ctypes.byref(b)) == HM_OK, (n, dt, L.hm_last_error())
            assert b.value >= 256
        assert L.hm_workspace_size(h, 3, 21, dt, 1, 0, ctypes.byref(b)) == HM_E_SIZE
    hh = P()
    assert L.hm_create(ctypes.byref(hh)) == HM_OK
    try:
        assert L.hm_set_option(hh, 1, 2) == HM_OK
        for dt in (0, 1):
            assert L.hm_workspace_size(hh, 3, 12, dt, 1, 0, ctypes.byref(b)) == HM_OK
    finally:
        L.hm_destroy(hh)


def test_batched_gradient_workspace_and_errors(L, h):
    b = ctypes.c_size_t()
    one = ctypes.c_size_t()
    for dt in (0, 1):
        for n in range(1, 21):
            assert L.hm_workspace_size(h, 3, n, dt, 1, 0, ctypes.byref(one)) == HM_OK
            for B in (1, 5, 64, 65, 130):
                assert L.hm_workspace_size(h, 6, n, dt, 1, B, ctypes.byref(b)) == HM_OK, (n, dt, B, L.hm_last_error())
                assert b.value >= 256
                if B == 1:
                    assert b.value == one.value  # a batch of one is the single-state call
        assert L.hm_workspace_size(h, 6, 21, dt, 1, 4, ctypes.byref(b)) == HM_E_SIZE
        assert L.hm_workspace_size(h, 6, 12, dt, 1, 0, ctypes.byref(b)) == HM_E_ARG
    good = P(0x100000)
    ptrs = (P * 2)(good, good)
    ws = P(0x200000)
    out = P(0x300000)
    assert L.hm_sre_grad_batched(None, ptrs, 8, 2, 0, 2.0, out, ptrs, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_grad_batched(h, ptrs, 8, 0, 0, 2.0, out, ptrs, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_grad_batched(h, None, 8, 2, 0, 2.0, out, ptrs, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_grad_batched(h, ptrs, 8, 2, 0, 2.0, out, None, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_grad_batched(h, ptrs, 8, 2, 0, 1.0, out, ptrs, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_grad_batched(h, ptrs, 21, 2, 0, 2.0, out, ptrs, ws, 1 << 30, None) == HM_E_SIZE
    assert L.hm_sre_grad_batched(h, ptrs, 8, 2, 7, 2.0, out, ptrs, ws, 1 << 30, None) == HM_E_DTYPE
    assert L.hm_sre_grad_batched(h, ptrs, 8, 2, 0, 2.0, out, ptrs, ws, 16, None) == HM_E_WORKSPACE
    bad = (P * 2)(good, P(0x100004))  # misaligned second state
    assert L.hm_sre_grad_batched(h, bad, 8, 2, 0, 2.0, out, ptrs, ws, 1 << 30, None) == HM_E_ALIGN


def test_check_norm_option(L, h):
    assert L.hm_set_option(h, 9, 2) == HM_E_ARG
    assert L.hm_set_option(h, 9, -1) == HM_E_ARG
    assert L.hm_set_option(h, 9, 1) == HM_OK
    # argument errors still come first, before any device work
    assert L.hm_sre(h, None, 8, 0, q_arr(2.0), 1, P(0x100000), P(0x200000), 1 << 30, None) == HM_E_ARG
    assert L.hm_set_option(h, 9, 0) == HM_OK


def test_header_is_plain_c_and_links(tmp_path):
    """include/hmag.h compiles as C99 (plain C types only) and a C program links against libhmag.so
    and calls it (no device work: version, status strings, handle, argument errors)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "use_hmag.c"
    src.write_text(r'''
#include "hmag.h"
#include <stdio.h>
#include <string.h>
int main(void) {
  hm_handle h = NULL;
  if (hm_create(&h) != HM_OK) return 1;
  double q = 2.0, out[2];
  hm_status s = hm_sre(h, NULL, 8, HM_C64, &q, 1, out, NULL, 0, NULL);
  printf("%s|%s|%s\n", hm_version(), hm_status_string(s), hm_last_error());
  if (s != HM_E_ARG) return 2;
  if (hm_set_option(h, HM_OPT_CHECK_NORM, 1) != HM_OK) return 3;
  return hm_destroy(h) == HM_OK ? 0 : 4;
}
''')
    exe = tmp_path / "use_hmag"
    libdir = os.path.dirname(hm.lib_path)
    cmd = [gcc, "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", str(src), "-L", libdir, "-lhmag", f"-Wl,-rpath,{libdir}", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "gfx950" in r.stdout and "HM_E_ARG" in r.stdout


def test_mana_workspace_every_size_and_dtype(L, h):
    """hm_workspace_size(HM_OP_MANA) plans every n in [1, 16] for both dtypes (complex128 two-pass
    tiles of 3^8 at n = 15, 16) and returns HM_E_SIZE outside that range."""
    b = ctypes.c_size_t(0)
    for dt in (0, 1):
        for n in range(1, 17):
            assert L.hm_workspace_size(h, 4, n, dt, 1, 0, ctypes.byref(b)) == HM_OK, (n, dt, L.hm_last_error())
            assert b.value >= 256
        for n in (0, 17):
            assert L.hm_workspace_size(h, 4, n, dt, 1, 0, ctypes.byref(b)) == HM_E_SIZE



def test_mc_argument_errors(L, h):
    prm = hm.McParams(5, 2, 100, 10, 0.0, 1)
    b = ctypes.c_size_t(0)
    assert L.hm_sre_mc_workspace(h, 10, 0, ctypes.byref(prm), ctypes.byref(b)) == HM_OK
    assert b.value > 0
    good = P(0x100000)
    args = lambda p: (h, good, 10, 0, ctypes.byref(p), good, good, good, good, good, good, 1 << 40, None)
    for bad in (hm.McParams(4, 2, 100, 10, 0.0, 1), hm.McParams(1, 2, 100, 10, 0.0, 1),
                hm.McParams(5, 0, 100, 10, 0.0, 1), hm.McParams(5, 2, 1, 0, 0.0, 1),
                hm.McParams(5, 2, 100, 99, 0.0, 1), hm.McParams(5, 2, 100, 10, -1.0, 1),
                hm.McParams(5, 2, 100, 10, float("nan"), 1), hm.McParams(5, 2, 100, 10, 0.0, 2)):
        assert L.hm_sre_mc(*args(bad)) == HM_E_ARG, (bad.n_beta, bad.chains_per_beta, bad.n_steps, bad.n_therm)
    assert L.hm_sre_mc(h, good, 10, 0, None, good, good, good, good, good, good, 1 << 40, None) == HM_E_ARG
    assert L.hm_sre_mc(h, good, 10, 0, ctypes.byref(prm), None, good, good, good, good, good, 1 << 40, None) == HM_E_ARG
    assert L.hm_sre_mc(h, good, 27, 0, ctypes.byref(prm), good, good, good, good, good, good, 1 << 40, None) == HM_E_SIZE
    assert L.hm_sre_mc(h, good, 10, 0, ctypes.byref(prm), good, good, good, good, good, good, 16, None) == HM_E_WORKSPACE


def test_autotune_other_plans_argument_errors(L, h):
    good, ws = P(0x100000), P(0x200000)
    b = ctypes.c_size_t(0)
    assert L.hm_autotune_mana_workspace(h, 12, 0, ctypes.byref(b)) == HM_OK and b.value > 256
    assert L.hm_autotune_mana_workspace(h, 17, 0, ctypes.byref(b)) == HM_E_SIZE
    assert L.hm_autotune_mana(h, None, 12, 0, 0, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_autotune_mana(h, good, 0, 0, 0, ws, 1 << 30, None) == HM_E_SIZE
    assert L.hm_autotune_grad_workspace(h, 13, 0, ctypes.byref(b)) == HM_OK and b.value > 256
    assert L.hm_autotune_grad_workspace(h, 21, 0, ctypes.byref(b)) == HM_E_SIZE
    assert L.hm_autotune_grad(h, good, 13, 0, 1.0, good, good, ws, 1 << 30, None) == HM_E_ARG  # q = 1
    assert L.hm_autotune_grad(h, good, 13, 0, 2.0, good, None, ws, 1 << 30, None) == HM_E_ARG
    hh = P()
    assert L.hm_create(ctypes.byref(hh)) == HM_OK
    assert L.hm_set_option(hh, 10, 2) == HM_OK  # HM_OPT_BATCH_LAUNCH fixed: nothing to tune
    ns = (ctypes.c_int * 1)(8)
    ps = (P * 1)(good)
    assert L.hm_autotune_batched(hh, ps, ns, 1, 0, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_set_option(hh, 10, 3) == HM_E_ARG
    L.hm_destroy(hh)


def test_mixed_and_reduced_density_argument_errors(L, h):
    good, ws = P(0x100000), P(0x200000)
    b = ctypes.c_size_t(0)
    assert L.hm_workspace_size(h, 7, 8, 1, 1, 0, ctypes.byref(b)) == HM_OK
    assert b.value >= 9 ** 8 * 16
    assert L.hm_workspace_size(h, 7, 11, 0, 1, 0, ctypes.byref(b)) == HM_E_SIZE
    assert L.hm_mana_mixed(h, good, 0, 0, good, ws, 1 << 40, None) == HM_E_SIZE
    assert L.hm_mana_mixed(h, None, 4, 0, good, ws, 1 << 40, None) == HM_E_ARG
    assert L.hm_mana_mixed(h, good, 4, 0, good, ws, 64, None) == HM_E_WORKSPACE
    assert L.hm_reduced_density(h, good, 8, 9, 0, good, None) == HM_E_SIZE
    assert L.hm_reduced_density(h, good, 12, 11, 0, good, None) == HM_E_SIZE
    assert L.hm_reduced_density(h, good, 8, 4, 0, None, None) == HM_E_ARG


def test_qudit_mana_argument_errors(L, h):
    good, ws = P(0x100000), P(0x200000)
    b = ctypes.c_size_t(0)
    for d, nmax64, nmax128 in ((3, 9, 8), (5, 6, 5), (7, 5, 4)):
        assert L.hm_workspace_size(h, 8, nmax64, 0, 1, d, ctypes.byref(b)) == HM_OK
        assert b.value >= 3 * 8
        assert L.hm_workspace_size(h, 8, nmax64 + 1, 0, 1, d, ctypes.byref(b)) == HM_E_SIZE
        assert L.hm_workspace_size(h, 8, nmax128, 1, 1, d, ctypes.byref(b)) == HM_OK
        assert L.hm_workspace_size(h, 8, nmax128 + 1, 1, 1, d, ctypes.byref(b)) == HM_E_SIZE
        assert L.hm_mana_qudit(h, good, nmax64 + 1, d, 0, good, ws, 1 << 30, None) == HM_E_SIZE
    assert L.hm_workspace_size(h, 8, 3, 0, 1, 4, ctypes.byref(b)) == HM_E_ARG
    assert L.hm_mana_qudit(h, good, 3, 4, 0, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_mana_qudit(h, good, 0, 5, 0, good, ws, 1 << 30, None) == HM_E_SIZE
    assert L.hm_mana_qudit(h, None, 3, 5, 0, good, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_mana_qudit(h, good, 3, 5, 0, None, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_mana_qudit(h, good, 3, 5, 0, good, ws, 8, None) == HM_E_WORKSPACE
    assert L.hm_mana_qudit(h, good, 3, 5, 2, good, ws, 1 << 30, None) == HM_E_DTYPE


def test_long_row_plans(L, h):
    """Rows of 2^14 / 2^15 values exist for complex64 only, 2^15 only with split LDS staging."""
    b = ctypes.c_size_t(0)
    hh = ctypes.c_void_p()
    assert L.hm_create(ctypes.byref(hh)) == HM_OK
    try:
        assert L.hm_set_option(hh, 1, 2) == HM_OK  # two-pass
        for rb, dt, split, want in ((15, 0, 0, HM_OK), (14, 0, 0, HM_OK), (15, 0, 1, HM_E_UNSUPPORTED),
                                    (14, 1, 0, HM_E_UNSUPPORTED), (13, 1, 0, HM_OK)):
            assert L.hm_set_option(hh, 5, rb) == HM_OK
            assert L.hm_set_option(hh, 7, split) == HM_OK
            assert L.hm_workspace_size(hh, 0, 24, dt, 1, 0, ctypes.byref(b)) == want, (rb, dt, split)
    finally:
        L.hm_destroy(hh)


def test_batched_grad_uneven_argument_errors(L, h):
    good, ws = P(0x100000), P(0x200000)
    b = ctypes.c_size_t(0)
    ns = (ctypes.c_int * 4)(8, 8, 13, 9)
    assert L.hm_sre_batched_grad_workspace(h, ns, 4, 0, ctypes.byref(b)) == HM_OK and b.value >= 256
    bad = (ctypes.c_int * 2)(8, 21)
    assert L.hm_sre_batched_grad_workspace(h, bad, 2, 0, ctypes.byref(b)) == HM_E_SIZE
    assert L.hm_sre_batched_grad_workspace(h, ns, 0, 0, ctypes.byref(b)) == HM_E_ARG
    assert L.hm_sre_batched_grad_workspace(h, ns, 4, 2, ctypes.byref(b)) == HM_E_DTYPE
    psis = (ctypes.c_void_p * 4)(good, good, good, good)
    grads = (ctypes.c_void_p * 4)(ws, ws, ws, ws)
    assert L.hm_sre_batched_grad(h, None, ns, 4, 0, 2.0, good, grads, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_batched_grad(h, psis, ns, 4, 0, 1.0, good, grads, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_batched_grad(h, psis, ns, 4, 0, 2.0, None, grads, ws, 1 << 30, None) == HM_E_ARG
    assert L.hm_sre_batched_grad(h, psis, ns, 4, 0, 2.0, good, grads, ws, 64, None) == HM_E_WORKSPACE
