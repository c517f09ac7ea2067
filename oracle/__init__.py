"""FP64 CPU oracle for the exact magic of pure state vectors -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  The GPU library never imports it and shares no code with it.

Wraps ``liboracle.so`` (plain C, OpenMP, built from ``oracle.c`` by :func:`build`) with numpy
arguments.  States are complex128 vectors (little-endian digits, see ``synth.states``).

Family A ("direct") builds every Pauli string / phase-space point operator from its definition
(paper Sec. 2, Eqs. sre, phase-space, mana2).  Family B ("fwht"/"fft") runs Algorithms 2 and 4
plainly.  See ``oracle.c`` for the readings taken where the paper is silent or inconsistent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

c_double_p = ctypes.POINTER(ctypes.c_double)
c_u64_p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2 -fopenmp).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-variable", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i, d, u64 = ctypes.c_int, ctypes.c_double, ctypes.c_uint64
        sig = {
            "oracle_set_threads": (None, [i]),
            "oracle_get_threads": (i, []),
            "oracle_sre_direct_sums": (i, [c_double_p, i, c_double_p, i, c_double_p, c_double_p]),
            "oracle_sre_direct": (i, [c_double_p, i, c_double_p, i, c_double_p]),
            "oracle_sre_row_values_direct": (i, [c_double_p, i, u64, c_double_p]),
            "oracle_sre_grad_direct": (i, [c_double_p, i, d, c_double_p, c_double_p]),
            "oracle_sre_fwht_sums": (i, [c_double_p, i, c_double_p, i, u64, u64, c_double_p]),
            "oracle_sre_fwht": (i, [c_double_p, i, c_double_p, i, c_double_p]),
            "oracle_sre_fwht_rows": (i, [c_double_p, i, c_u64_p, ctypes.c_int64, c_double_p, i, c_double_p]),
            "oracle_sre_row_values_fwht": (i, [c_double_p, i, u64, c_double_p, c_double_p]),
            "oracle_sre_grad_fwht": (i, [c_double_p, i, d, c_double_p, c_double_p]),
            "oracle_sre_finalize": (None, [i, c_double_p, i, c_double_p, c_double_p]),
            "oracle_mana_direct": (i, [c_double_p, i, c_double_p]),
            "oracle_mana_fft_sums": (i, [c_double_p, i, u64, u64, c_double_p]),
            "oracle_mana_fft": (i, [c_double_p, i, c_double_p]),
            "oracle_mana_fft_rows": (i, [c_double_p, i, c_u64_p, ctypes.c_int64, c_double_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _cplx(psi) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    return a


def _dp(a: np.ndarray):
    return a.ctypes.data_as(c_double_p)


def _qarr(q) -> np.ndarray:
    return np.ascontiguousarray(np.atleast_1d(np.asarray(q, dtype=np.float64)))


def _nq(psi: np.ndarray, d: int) -> int:
    D = psi.shape[0]
    n = 0
    while d ** n < D:
        n += 1
    if d ** n != D:
        raise ValueError(f"length {D} is not a power of {d}")
    return n


def _chk(st: int, what: str):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


# ---------------------------------------------------------------------------------------------
# SRE
# ---------------------------------------------------------------------------------------------
def sre_direct(psi, q: Sequence[float] = (2.0,)) -> np.ndarray:
    """[M_q for q in q..., lost_norm] by direct evaluation of all 4^N Pauli strings (O(8^N))."""
    p = _cplx(psi)
    n = _nq(p, 2)
    qa = _qarr(q)
    out = np.zeros(len(qa) + 1)
    _chk(lib().oracle_sre_direct(_dp(p), n, _dp(qa), len(qa), _dp(out)), "sre_direct")
    return out


def sre_direct_sums(psi, q: Sequence[float] = (2.0,)):
    """Raw sums [sum <P>^2, sum <P>^{2q}...] and max |Im <P>| over all Pauli strings."""
    p = _cplx(psi)
    n = _nq(p, 2)
    qa = _qarr(q)
    sums = np.zeros(len(qa) + 1)
    mi = ctypes.c_double(0.0)
    _chk(lib().oracle_sre_direct_sums(_dp(p), n, _dp(qa), len(qa), _dp(sums), ctypes.byref(mi)), "direct_sums")
    return sums, mi.value


def sre_fwht(psi, q: Sequence[float] = (2.0,)) -> np.ndarray:
    """[M_q..., lost_norm] by Algorithm 2 (one FWHT per X-shift), FP64."""
    p = _cplx(psi)
    n = _nq(p, 2)
    qa = _qarr(q)
    out = np.zeros(len(qa) + 1)
    _chk(lib().oracle_sre_fwht(_dp(p), n, _dp(qa), len(qa), _dp(out)), "sre_fwht")
    return out


def sre_fwht_sums(psi, q: Sequence[float] = (2.0,), a0: int = 0, a1: int | None = None) -> np.ndarray:
    """Raw sums over X-shifts [a0, a1): [sum |chi|^2, sum |chi|^{2q} (or chi^2 log2 chi^2 for q=1)...]."""
    p = _cplx(psi)
    n = _nq(p, 2)
    qa = _qarr(q)
    a1 = (1 << n) if a1 is None else a1
    sums = np.zeros(len(qa) + 1)
    _chk(lib().oracle_sre_fwht_sums(_dp(p), n, _dp(qa), len(qa), a0, a1, _dp(sums)), "fwht_sums")
    return sums


def sre_finalize(n: int, q, sums) -> np.ndarray:
    qa = _qarr(q)
    s = np.ascontiguousarray(np.asarray(sums, dtype=np.float64))
    out = np.zeros(len(qa) + 1)
    lib().oracle_sre_finalize(n, _dp(qa), len(qa), _dp(s), _dp(out))
    return out


def sre_rows(psi, rows, q: Sequence[float] = (2.0,)) -> np.ndarray:
    """Per-row sums, shape (n_rows, n_q + 1): [sum_b |chi_b|^2, sum_b |chi_b|^{2q}...] for each a."""
    p = _cplx(psi)
    n = _nq(p, 2)
    qa = _qarr(q)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
    out = np.zeros((len(r), len(qa) + 1))
    _chk(lib().oracle_sre_fwht_rows(_dp(p), n, r.ctypes.data_as(c_u64_p), len(r), _dp(qa), len(qa), _dp(out)),
         "fwht_rows")
    return out


def sre_row_values_direct(psi, a: int) -> np.ndarray:
    p = _cplx(psi)
    n = _nq(p, 2)
    out = np.zeros(1 << n)
    _chk(lib().oracle_sre_row_values_direct(_dp(p), n, int(a), _dp(out)), "row_values_direct")
    return out


def sre_row_values_fwht(psi, a: int):
    """(<P_{a,b}> for all b, max |Im|) from the fast form with the i^{popcount(a&b)} phase."""
    p = _cplx(psi)
    n = _nq(p, 2)
    out = np.zeros(1 << n)
    mi = ctypes.c_double(0.0)
    _chk(lib().oracle_sre_row_values_fwht(_dp(p), n, int(a), _dp(out), ctypes.byref(mi)), "row_values_fwht")
    return out, mi.value


def sre_grad_direct(psi, q: float = 2.0):
    """(array [M_q, lost_norm], g = dM/dRe psi + i dM/dIm psi) by direct Pauli enumeration."""
    p = _cplx(psi)
    n = _nq(p, 2)
    out = np.zeros(2)
    g = np.zeros(1 << n, dtype=np.complex128)
    _chk(lib().oracle_sre_grad_direct(_dp(p), n, float(q), _dp(out), _dp(g)), "grad_direct")
    return out, g


def sre_grad_fwht(psi, q: float = 2.0):
    """Same as :func:`sre_grad_direct`, from the FWHT form (adjoint of Algorithm 2)."""
    p = _cplx(psi)
    n = _nq(p, 2)
    out = np.zeros(2)
    g = np.zeros(1 << n, dtype=np.complex128)
    _chk(lib().oracle_sre_grad_fwht(_dp(p), n, float(q), _dp(out), _dp(g)), "grad_fwht")
    return out, g


# ---------------------------------------------------------------------------------------------
# Mana
# ---------------------------------------------------------------------------------------------
def mana_direct(psi) -> np.ndarray:
    """[mana, sum W, 3^N sum W^2] from every phase-space point operator (O(N 27^N))."""
    p = _cplx(psi)
    n = _nq(p, 3)
    out = np.zeros(3)
    _chk(lib().oracle_mana_direct(_dp(p), n, _dp(out)), "mana_direct")
    return out


def mana_fft(psi) -> np.ndarray:
    """[mana, sum W, 3^N sum W^2] by Algorithm 4 (one Z_3^N Fourier transform per shift)."""
    p = _cplx(psi)
    n = _nq(p, 3)
    out = np.zeros(3)
    _chk(lib().oracle_mana_fft(_dp(p), n, _dp(out)), "mana_fft")
    return out


def mana_fft_sums(psi, a0: int = 0, a1: int | None = None) -> np.ndarray:
    p = _cplx(psi)
    n = _nq(p, 3)
    a1 = 3 ** n if a1 is None else a1
    s = np.zeros(3)
    _chk(lib().oracle_mana_fft_sums(_dp(p), n, a0, a1, _dp(s)), "mana_fft_sums")
    return s


def mana_rows(psi, rows) -> np.ndarray:
    """Per-shift [sum_b |chi_b|, sum_b chi_b, sum_b chi_b^2], shape (n_rows, 3)."""
    p = _cplx(psi)
    n = _nq(p, 3)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
    out = np.zeros((len(r), 3))
    _chk(lib().oracle_mana_fft_rows(_dp(p), n, r.ctypes.data_as(c_u64_p), len(r), _dp(out)), "mana_rows")
    return out
