"""hmag -- numerically exact magic of state vectors on AMD MI355X (gfx950).

Thin Python binding of libhmag.so (C-ABI declared in include/hmag.h).  This module only marshals
arguments: torch supplies device memory and the current HIP stream; every step of the computation
runs in the library's HIP kernels.  There is no CPU fallback -- if libhmag.so is missing or no GPU is
visible the calls raise.

Qubit states (d = 2) are complex64 / complex128 torch tensors of length 2^n on the GPU; qutrit
states (d = 3) have length 3^n.  Digit k of the basis index is qudit k (little-endian).
"""
from __future__ import annotations

import ctypes
import math
import os
import threading
from typing import Sequence

__all__ = [
    "HmError", "lib", "lib_path", "Context", "default_context", "sre", "sre_partial", "sre_finalize",
    "sre_rows", "sre_row_values", "sre_noalloc", "sre_mc", "McParams", "mc_random_inputs", "sre_grad", "sre_grad_batched", "sre_grad_uneven", "SRE", "SREBatched", "sre_batched", "sre_sampled", "autotune", "autotune_mana", "autotune_grad", "autotune_batched", "tuned_plan", "mana", "mana_partial", "mana_mixed", "mana_qudit", "reduced_density_matrix", "workspace_size",
    "HM_C64", "HM_C128", "profile_enable", "profile_reset", "profile_read", "OP_SRE", "OP_SRE_ROWS", "OP_ROW_VALUES", "OP_SRE_GRAD", "OP_MANA",
    "OP_SRE_SAMPLED", "OP_SRE_GRAD_BATCHED", "EXPORTED_SYMBOLS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libhmag.so")

HM_C64, HM_C128 = 0, 1
OP_SRE, OP_SRE_ROWS, OP_ROW_VALUES, OP_SRE_GRAD, OP_MANA, OP_SRE_SAMPLED, OP_SRE_GRAD_BATCHED = 0, 1, 2, 3, 4, 5, 6
OP_MANA_MIXED = 7
OP_MANA_QUDIT = 8
OPT_FORCE_PATH, OPT_BATCH_SHIFTS, OPT_ROW_RB, OPT_COL_RB, OPT_ROW_BITS, OPT_PIPELINE, OPT_LDS_SPLIT, OPT_STREAMS = \
    1, 2, 3, 4, 5, 6, 7, 8
OPT_CHECK_NORM = 9
OPT_BATCH_LAUNCH = 10

_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); this is also the list of symbols the header declares.
_SIGS = {
    "hm_create": (_i, [ctypes.POINTER(_vp)]),
    "hm_destroy": (_i, [_vp]),
    "hm_status_string": (ctypes.c_char_p, [_i]),
    "hm_last_error": (ctypes.c_char_p, []),
    "hm_version": (ctypes.c_char_p, []),
    "hm_set_option": (_i, [_vp, _i, _i64]),
    "hm_workspace_size": (_i, [_vp, _i, _i, _i, _i, _i64, ctypes.POINTER(_sz)]),
    "hm_sre": (_i, [_vp, _vp, _i, _i, _dp, _i, _vp, _vp, _sz, _vp]),
    "hm_sre_partial": (_i, [_vp, _vp, _i, _i, _dp, _i, _u64, _u64, _vp, _vp, _sz, _vp]),
    "hm_sre_finalize": (_i, [_i, _dp, _i, _vp, _vp, _vp]),
    "hm_sre_rows": (_i, [_vp, _vp, _i, _i, _vp, _i64, _dp, _i, _vp, _vp, _sz, _vp]),
    "hm_sre_row_values": (_i, [_vp, _vp, _i, _i, _u64, _vp, _vp, _sz, _vp]),
    "hm_sre_grad": (_i, [_vp, _vp, _i, _i, ctypes.c_double, _vp, _vp, _vp, _sz, _vp]),
    "hm_sre_grad_batched": (_i, [_vp, ctypes.POINTER(_vp), _i, _i, _i, ctypes.c_double, _vp, ctypes.POINTER(_vp),
                                 _vp, _sz, _vp]),
    "hm_mana": (_i, [_vp, _vp, _i, _i, _vp, _vp, _sz, _vp]),
    "hm_mana_partial": (_i, [_vp, _vp, _i, _i, _u64, _u64, _vp, _vp, _sz, _vp]),
    "hm_mana_mixed": (_i, [_vp, _vp, _i, _i, _vp, _vp, _sz, _vp]),
    "hm_mana_qudit": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp, _sz, _vp]),
    "hm_reduced_density": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp]),
    "hm_sre_batched_grad_workspace": (_i, [_vp, ctypes.POINTER(_i), _i, _i, ctypes.POINTER(_sz)]),
    "hm_sre_batched_grad": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_i), _i, _i, ctypes.c_double, _vp,
                                 ctypes.POINTER(_vp), _vp, _sz, _vp]),
    "hm_sre_batched_workspace": (_i, [_vp, ctypes.POINTER(_i), _i, _i, _i, ctypes.POINTER(_sz)]),
    "hm_sre_batched": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_i), _i, _i, _dp, _i, _vp, _vp, _sz, _vp]),
    "hm_sre_sampled": (_i, [_vp, _vp, _i, _i, _vp, _i64, _vp, _vp, _sz, _vp]),
    "hm_sre_noalloc": (_i, [_vp, _vp, _i, _i, _dp, _i, _vp, _vp]),
    "hm_sre_mc_workspace": (_i, [_vp, _i, _i, _vp, ctypes.POINTER(_sz)]),
    "hm_sre_mc": (_i, [_vp, _vp, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "hm_autotune_workspace": (_i, [_vp, _i, _i, _i64, ctypes.POINTER(_sz)]),
    "hm_autotune": (_i, [_vp, _vp, _i, _i, _i64, _vp, _sz, _vp]),
    "hm_tune_query": (_i, [_vp, _i, _i, ctypes.POINTER(_i64), _dp]),
    "hm_autotune_mana_workspace": (_i, [_vp, _i, _i, ctypes.POINTER(_sz)]),
    "hm_autotune_mana": (_i, [_vp, _vp, _i, _i, _i64, _vp, _sz, _vp]),
    "hm_autotune_grad_workspace": (_i, [_vp, _i, _i, ctypes.POINTER(_sz)]),
    "hm_autotune_grad": (_i, [_vp, _vp, _i, _i, ctypes.c_double, _vp, _vp, _vp, _sz, _vp]),
    "hm_autotune_batched": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_i), _i, _i, _vp, _vp, _sz, _vp]),
    "hm_tune_clear": (_i, [_vp]),
    "hm_profile_enable": (_i, [_i]),
    "hm_profile_reset": (_i, []),
    "hm_profile_query": (_i, [_i, ctypes.c_char_p, _sz, ctypes.POINTER(_i64), ctypes.POINTER(_i64), _dp]),
}
EXPORTED_SYMBOLS = tuple(_SIGS)

_lib = None
_lock = threading.Lock()


class HmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


def lib():
    """Load libhmag.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(lib_path):
                    raise RuntimeError(f"{lib_path} is missing: build it with paper_2601_07824_amd.build.build()")
                L = ctypes.CDLL(lib_path)
                for name, (res, args) in _SIGS.items():
                    f = getattr(L, name)
                    f.restype = res
                    f.argtypes = args
                _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        L = lib()
        raise HmError(st, f"{L.hm_status_string(st).decode()}: {L.hm_last_error().decode()}")


class Context:
    """Owns one hm_handle (plans and options; no device memory)."""

    def __init__(self):
        h = _vp()
        _check(lib().hm_create(ctypes.byref(h)))
        self.h = h

    def set_option(self, opt: int, value: int):
        _check(lib().hm_set_option(self.h, opt, value))

    def force_path(self, path: int):
        self.set_option(OPT_FORCE_PATH, path)

    def batch_shifts(self, b: int):
        self.set_option(OPT_BATCH_SHIFTS, b)

    def close(self):
        if self.h:
            lib().hm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = None


def default_context() -> Context:
    global _default
    if _default is None:
        _default = Context()
    return _default


# ------------------------------------------------------------------------------------------------
# marshalling helpers (torch is used only for memory and streams)
# ------------------------------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex64:
        return HM_C64
    if t.dtype == torch.complex128:
        return HM_C128
    raise TypeError(f"state must be complex64 or complex128, got {t.dtype}")


def _state(psi, d: int):
    torch = _torch()
    if not isinstance(psi, torch.Tensor) or not psi.is_cuda:
        raise TypeError("state must be a torch tensor on the GPU")
    if psi.dim() != 1:
        raise ValueError("state must be one-dimensional")
    psi = psi.contiguous()
    D = psi.numel()
    n = round(math.log(D, d)) if D > 0 else -1
    if n < 1 or d ** n != D:
        raise ValueError(f"state length {D} is not {d}^n with n >= 1")
    return psi, n


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _q(q) -> tuple:
    qs = [float(x) for x in (q if isinstance(q, (list, tuple)) else [q])]
    arr = (ctypes.c_double * len(qs))(*qs)
    return arr, len(qs)


def _ptr(t) -> _vp:
    return _vp(t.data_ptr())


def workspace_size(op: int, n: int, dtype_code: int, n_q: int = 1, count: int = 0, ctx: Context | None = None) -> int:
    ctx = ctx or default_context()
    b = _sz(0)
    _check(lib().hm_workspace_size(ctx.h, op, n, dtype_code, n_q, count, ctypes.byref(b)))
    return b.value


def _workspace(nbytes: int, device, stream=None):
    """Scratch for one call.  Allocated through torch's caching allocator on the current stream; when
    the call runs on another stream the block is marked as used there, so the allocator does not hand
    it out again before that stream is done with it."""
    torch = _torch()
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if stream is not None and stream != torch.cuda.current_stream(device):
        ws.record_stream(stream)
    return ws


def profile_enable(on: bool | int = True):
    """Bracket library kernel launches with hipEvents on their stream (see hm_profile_enable):
    True = every launch, an int k > 1 = every k-th launch of each kernel family, False = off."""
    every = int(on) if not isinstance(on, bool) else (1 if on else 0)
    _check(lib().hm_profile_enable(every))


def profile_reset():
    _check(lib().hm_profile_reset())


def profile_read() -> dict:
    """{kernel family: (launches, timed launches, total device ms of the timed ones)} since the
    last reset."""
    out = {}
    i = 0
    buf = ctypes.create_string_buffer(128)
    while True:
        n, c, ms = _i64(0), _i64(0), ctypes.c_double(0.0)
        st = lib().hm_profile_query(i, buf, 128, ctypes.byref(n), ctypes.byref(c), ctypes.byref(ms))
        if st != 0:
            break
        out[buf.value.decode()] = (n.value, c.value, ms.value)
        i += 1
    return out


# ------------------------------------------------------------------------------------------------
# qubits
# ------------------------------------------------------------------------------------------------
def sre(psi, q: Sequence[float] | float = (2.0,), *, ctx: Context | None = None, stream=None):
    """[M_q for each q..., lost_norm] as a float64 tensor on the state's device."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    qa, nq = _q(q)
    dt = _dtype_code(psi)
    ws = _workspace(workspace_size(OP_SRE, n, dt, nq, 0, ctx), psi.device, stream)
    out = torch.empty(nq + 1, dtype=torch.float64, device=psi.device)
    _check(lib().hm_sre(ctx.h, _ptr(psi), n, dt, qa, nq, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def sre_noalloc(psi, q: Sequence[float] | float = (2.0,), *, out=None, ctx: Context | None = None, stream=None):
    """hm_sre_noalloc: [M_q..., lost_norm] with no device allocation inside the library (its scratch
    array is used instead of a workspace).  `out` (float64, n_q + 1 values, on the state's device) may
    be given so that the call allocates nothing on the Python side either."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    qa, nq = _q(q)
    dt = _dtype_code(psi)
    if out is None:
        out = torch.empty(nq + 1, dtype=torch.float64, device=psi.device)
    elif out.dtype != torch.float64 or out.numel() < nq + 1 or not out.is_contiguous() or out.device != psi.device:
        raise ValueError("out must be a contiguous float64 tensor of n_q + 1 values on the state's device")
    _check(lib().hm_sre_noalloc(ctx.h, _ptr(psi), n, dt, qa, nq, _ptr(out), _stream(stream)))
    return out


def sre_partial(psi, q=(2.0,), a0: int = 0, a1: int | None = None, *, ctx: Context | None = None, stream=None):
    """Raw sums over X-shifts [a0, a1): [sum |chi|^2, sum |chi|^{2q}...] (float64 tensor)."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    a1 = (1 << n) if a1 is None else a1
    qa, nq = _q(q)
    dt = _dtype_code(psi)
    ws = _workspace(workspace_size(OP_SRE, n, dt, nq, 0, ctx), psi.device, stream)
    out = torch.empty(nq + 1, dtype=torch.float64, device=psi.device)
    _check(lib().hm_sre_partial(ctx.h, _ptr(psi), n, dt, qa, nq, a0, a1, _ptr(out), _ptr(ws), ws.numel(),
                                _stream(stream)))
    return out


def sre_finalize(n: int, q, sums, *, stream=None):
    torch = _torch()
    qa, nq = _q(q)
    out = torch.empty(nq + 1, dtype=torch.float64, device=sums.device)
    sums = sums.contiguous()
    _check(lib().hm_sre_finalize(n, qa, nq, _ptr(sums), _ptr(out), _stream(stream)))
    return out


def sre_rows(psi, rows, q=(2.0,), *, ctx: Context | None = None, stream=None):
    """Per-row sums (n_rows, n_q + 1): [sum_b |chi_b(a)|^2, sum_b |chi_b(a)|^{2q}...] for a in rows."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    qa, nq = _q(q)
    dt = _dtype_code(psi)
    if not isinstance(rows, torch.Tensor):
        rows = torch.as_tensor(rows, dtype=torch.int64)
    rows = rows.to(device=psi.device, dtype=torch.int64).contiguous()
    nr = rows.numel()
    out = torch.empty((nr, nq + 1), dtype=torch.float64, device=psi.device)
    ws = _workspace(workspace_size(OP_SRE_ROWS, n, dt, nq, nr, ctx), psi.device, stream)
    _check(lib().hm_sre_rows(ctx.h, _ptr(psi), n, dt, _ptr(rows), nr, qa, nq, _ptr(out), _ptr(ws), ws.numel(),
                             _stream(stream)))
    return out


TUNE_KEYS = ("force_path", "batch_shifts", "row_rb", "col_rb", "row_bits", "pipeline", "lds_split", "streams")


def autotune(psi, sample_shifts: int = 16384, *, ctx: Context | None = None, stream=None) -> dict:
    """Time the candidate SRE plans for this state's size and dtype on the device, keep the fastest
    in the context (used from then on for options left automatic) and return it."""
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    dt = _dtype_code(psi)
    b = _sz(0)
    _check(lib().hm_autotune_workspace(ctx.h, n, dt, sample_shifts, ctypes.byref(b)))
    ws = _workspace(b.value, psi.device, stream)
    _check(lib().hm_autotune(ctx.h, _ptr(psi), n, dt, sample_shifts, _ptr(ws), ws.numel(), _stream(stream)))
    return tuned_plan(n, dt, ctx=ctx)


def autotune_mana(psi, sample_shifts: int = 4096, *, ctx: Context | None = None, stream=None):
    """Time the mana launch plans for this qutrit state's size and dtype and keep the fastest in ctx."""
    ctx = ctx or default_context()
    psi, n = _state(psi, 3)
    dt = _dtype_code(psi)
    b = _sz(0)
    _check(lib().hm_autotune_mana_workspace(ctx.h, n, dt, ctypes.byref(b)))
    ws = _workspace(b.value, psi.device, stream)
    _check(lib().hm_autotune_mana(ctx.h, _ptr(psi), n, dt, sample_shifts, _ptr(ws), ws.numel(), _stream(stream)))


def autotune_grad(psi, q: float = 2.0, *, ctx: Context | None = None, stream=None):
    """Time the gradient paths for this state's size and dtype and keep the fastest in ctx."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    dt = _dtype_code(psi)
    b = _sz(0)
    _check(lib().hm_autotune_grad_workspace(ctx.h, n, dt, ctypes.byref(b)))
    ws = _workspace(b.value, psi.device, stream)
    out = torch.empty(2, dtype=torch.float64, device=psi.device)
    grad = torch.empty_like(psi)
    _check(lib().hm_autotune_grad(ctx.h, _ptr(psi), n, dt, float(q), _ptr(out), _ptr(grad), _ptr(ws), ws.numel(),
                                  _stream(stream)))


def autotune_batched(states, *, ctx: Context | None = None, stream=None):
    """Time hm_sre_batched's launch forms on these states and keep the faster in ctx."""
    torch = _torch()
    ctx = ctx or default_context()
    sts, ns = [], []
    for s in states:
        s, n = _state(s, 2)
        sts.append(s)
        ns.append(n)
    dt = _dtype_code(sts[0])
    B = len(sts)
    ns_c = (_i * B)(*ns)
    ptrs = (_vp * B)(*[s.data_ptr() for s in sts])
    need = 0
    for mode in (1, 2):
        c2 = Context()
        c2.set_option(OPT_BATCH_LAUNCH, mode)
        b = _sz(0)
        _check(lib().hm_sre_batched_workspace(c2.h, ns_c, B, dt, 1, ctypes.byref(b)))
        need = max(need, b.value)
    ws = _workspace(need, sts[0].device, stream)
    out = torch.empty((B, 2), dtype=torch.float64, device=sts[0].device)
    _check(lib().hm_autotune_batched(ctx.h, ptrs, ns_c, B, dt, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))


def tuned_plan(n: int, dtype_code: int, *, ctx: Context | None = None) -> dict:
    """The plan the autotuner stored for (n, dtype code), with its milliseconds per X-shift."""
    ctx = ctx or default_context()
    v = (_i64 * 8)()
    ms = ctypes.c_double(0.0)
    _check(lib().hm_tune_query(ctx.h, n, dtype_code, v, ctypes.byref(ms)))
    d = dict(zip(TUNE_KEYS, [int(x) for x in v]))
    d["ms_per_shift"] = ms.value
    return d


def sre_batched(states, q=(2.0,), *, ctx: Context | None = None, stream=None):
    """[M_q..., lost_norm] for each of several qubit states (list of GPU tensors of one dtype,
    any lengths 2^n).  Returns a float64 tensor of shape (len(states), n_q + 1)."""
    torch = _torch()
    ctx = ctx or default_context()
    sts, ns = [], []
    for s in states:
        s, n = _state(s, 2)
        sts.append(s)
        ns.append(n)
    if not sts:
        raise ValueError("no states")
    dt = _dtype_code(sts[0])
    if any(_dtype_code(s) != dt for s in sts):
        raise TypeError("all states must share one dtype")
    qa, nq = _q(q)
    B = len(sts)
    ns_c = (_i * B)(*ns)
    ptrs = (_vp * B)(*[s.data_ptr() for s in sts])
    b = _sz(0)
    _check(lib().hm_sre_batched_workspace(ctx.h, ns_c, B, dt, nq, ctypes.byref(b)))
    ws = _workspace(b.value, sts[0].device, stream)
    out = torch.empty((B, nq + 1), dtype=torch.float64, device=sts[0].device)
    _check(lib().hm_sre_batched(ctx.h, ptrs, ns_c, B, dt, qa, nq, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    out._hm_keepalive = (sts, ws)
    return out


def sre_sampled(psi, n_rows: int = 4096, seed: int = 0, rows=None, *, ctx: Context | None = None, stream=None):
    """Monte Carlo M_2: tensor [M2_hat, standard error, S_hat, std S].  The a = 0 row is exact; the
    other rows are drawn i.i.d. uniformly in [1, 2^n) with numpy's PCG64 (seed) unless given."""
    import numpy as np
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    dt = _dtype_code(psi)
    if rows is None:
        rows = np.random.default_rng(seed).integers(1, 2 ** n, size=n_rows, dtype=np.uint64)
    rows = torch.as_tensor(np.asarray(rows, dtype=np.int64)).to(psi.device)
    out = torch.empty(4, dtype=torch.float64, device=psi.device)
    ws = _workspace(workspace_size(OP_SRE_SAMPLED, n, dt, 1, rows.numel(), ctx), psi.device, stream)
    _check(lib().hm_sre_sampled(ctx.h, _ptr(psi), n, dt, _ptr(rows), rows.numel(), _ptr(out), _ptr(ws), ws.numel(),
                                _stream(stream)))
    return out


class McParams(ctypes.Structure):
    """hm_mc_params (include/hmag.h)."""
    _fields_ = [("n_beta", _i), ("chains_per_beta", _i), ("n_steps", _i64), ("n_therm", _i64),
                ("epsilon", ctypes.c_double), ("exclude_identity", _i)]


def mc_random_inputs(n: int, n_beta: int, chains_per_beta: int, n_steps: int, seed: int):
    """The chains' randomness drawn with numpy's PCG64 (seed): initial X-strings uniform in [1, 2^n),
    single-bit-flip XOR masks and acceptance uniforms, each (n_steps, C) with C = n_beta chains_per_beta."""
    import numpy as np
    C = n_beta * chains_per_beta
    g = np.random.default_rng(seed)
    a_init = g.integers(1, 2 ** n, size=C, dtype=np.uint64)
    moves = np.uint64(1) << g.integers(0, n, size=(n_steps, C)).astype(np.uint64)
    uniforms = g.random((n_steps, C))
    return a_init, moves, uniforms


def sre_mc(psi, n_beta: int = 17, chains_per_beta: int = 1, n_steps: int = 1000, n_therm: int = 100,
           epsilon: float = 0.0, exclude_identity: bool = True, seed: int = 0, inputs=None, *,
           ctx: Context | None = None, stream=None):
    """Monte Carlo M_2 by thermodynamic integration (hm_sre_mc).  inputs = (a_init, moves, uniforms)
    as numpy arrays, else drawn by mc_random_inputs(seed).  Returns (out, trace): out = [M2_hat, dM2,
    I, S2_hat, then per beta point <f>, var, sigma^2, tau_int, acceptance] (float64 tensor), trace =
    (n_steps, C) energies."""
    import numpy as np
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    dt = _dtype_code(psi)
    C = n_beta * chains_per_beta
    if inputs is None:
        inputs = mc_random_inputs(n, n_beta, chains_per_beta, n_steps, seed)
    a_init, moves, uniforms = (np.ascontiguousarray(v) for v in inputs)
    if a_init.shape != (C,) or moves.shape != (n_steps, C) or uniforms.shape != (n_steps, C):
        raise ValueError("inputs must have shapes (C,), (n_steps, C), (n_steps, C)")
    dev = psi.device
    a_t = torch.from_numpy(a_init.astype(np.uint64).view(np.int64)).to(dev)
    m_t = torch.from_numpy(moves.astype(np.uint64).view(np.int64)).to(dev)
    u_t = torch.from_numpy(uniforms.astype(np.float64)).to(dev)
    prm = McParams(n_beta, chains_per_beta, n_steps, n_therm, float(epsilon), int(bool(exclude_identity)))
    b = _sz(0)
    _check(lib().hm_sre_mc_workspace(ctx.h, n, dt, ctypes.byref(prm), ctypes.byref(b)))
    ws = _workspace(b.value, dev, stream)
    out = torch.empty(4 + 5 * n_beta, dtype=torch.float64, device=dev)
    trace = torch.empty((n_steps, C), dtype=torch.float64, device=dev)
    _check(lib().hm_sre_mc(ctx.h, _ptr(psi), n, dt, ctypes.byref(prm), _ptr(a_t), _ptr(m_t), _ptr(u_t), _ptr(out),
                           _ptr(trace), _ptr(ws), ws.numel(), _stream(stream)))
    out._hm_keepalive = (a_t, m_t, u_t, ws)
    return out, trace


def sre_row_values(psi, a: int, *, ctx: Context | None = None, stream=None):
    """<P_{a,b}> for b in [0, 2^n) (float64 tensor)."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    dt = _dtype_code(psi)
    out = torch.empty(1 << n, dtype=torch.float64, device=psi.device)
    ws = _workspace(workspace_size(OP_ROW_VALUES, n, dt, 1, 0, ctx), psi.device, stream)
    _check(lib().hm_sre_row_values(ctx.h, _ptr(psi), n, dt, int(a), _ptr(out), _ptr(ws), ws.numel(),
                                   _stream(stream)))
    return out


def sre_grad(psi, q: float = 2.0, *, ctx: Context | None = None, stream=None):
    """(tensor [M_q, lost_norm], grad = dM_q/dRe psi + i dM_q/dIm psi) in one fused call."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 2)
    dt = _dtype_code(psi)
    out = torch.empty(2, dtype=torch.float64, device=psi.device)
    grad = torch.empty_like(psi)
    ws = _workspace(workspace_size(OP_SRE_GRAD, n, dt, 1, 0, ctx), psi.device, stream)
    _check(lib().hm_sre_grad(ctx.h, _ptr(psi), n, dt, float(q), _ptr(out), _ptr(grad), _ptr(ws), ws.numel(),
                             _stream(stream)))
    return out, grad


def sre_grad_batched(states, q: float = 2.0, *, ctx: Context | None = None, stream=None):
    """hm_sre_grad for several states of one size: states is a GPU tensor of shape (B, 2^n) or a list
    of B one-dimensional ones.  Returns (float64 tensor (B, 2) of [M_q, lost_norm], gradients in the
    same form as states: a (B, 2^n) tensor, or a list)."""
    torch = _torch()
    ctx = ctx or default_context()
    as_rows = isinstance(states, torch.Tensor)
    if as_rows:
        if states.dim() != 2 or states.shape[0] < 1:
            raise ValueError("states must have shape (B, 2^n) with B >= 1")
        states = states.contiguous()
        sts = list(states.unbind(0))
    else:
        sts = list(states)
    if not sts:
        raise ValueError("no states")
    sts = [_state(s, 2) for s in sts]
    n = sts[0][1]
    if any(m != n for _, m in sts):
        raise ValueError("all states must have the same qubit count")
    sts = [s for s, _ in sts]
    dt = _dtype_code(sts[0])
    if any(_dtype_code(s) != dt for s in sts):
        raise TypeError("all states must share one dtype")
    B = len(sts)
    grads = torch.empty((B, 1 << n), dtype=sts[0].dtype, device=sts[0].device)
    out = torch.empty((B, 2), dtype=torch.float64, device=sts[0].device)
    ptrs = (_vp * B)(*[s.data_ptr() for s in sts])
    gptrs = (_vp * B)(*[grads[i].data_ptr() for i in range(B)])
    ws = _workspace(workspace_size(OP_SRE_GRAD_BATCHED, n, dt, 1, B, ctx), sts[0].device, stream)
    _check(lib().hm_sre_grad_batched(ctx.h, ptrs, n, B, dt, float(q), _ptr(out), gptrs, _ptr(ws), ws.numel(),
                                     _stream(stream)))
    return out, (grads if as_rows else list(grads.unbind(0)))


def sre_grad_uneven(states, q: float = 2.0, *, ctx: Context | None = None, stream=None):
    """hm_sre_batched_grad: fused forward + adjoint of M_q for a list of states of uneven n (one
    dtype).  Returns (out, grads): out is a (B, 2) float64 tensor of [M_q, lost_norm], grads a list of
    tensors shaped like the states.  Consecutive states of equal n share one batched launch."""
    torch = _torch()
    ctx = ctx or default_context()
    states = [s for s in states]
    if not states:
        raise ValueError("empty batch")
    checked = [_state(s, 2) for s in states]
    psis = [c[0] for c in checked]
    ns = [c[1] for c in checked]
    dt = _dtype_code(psis[0])
    if any(_dtype_code(p) != dt for p in psis) or any(p.device != psis[0].device for p in psis):
        raise TypeError("all states must share one dtype and device")
    B = len(psis)
    grads = [torch.empty_like(p) for p in psis]
    out = torch.empty((B, 2), dtype=torch.float64, device=psis[0].device)
    ns_a = (_i * B)(*ns)
    pp = (_vp * B)(*[p.data_ptr() for p in psis])
    gp = (_vp * B)(*[g.data_ptr() for g in grads])
    nb = _sz(0)
    _check(lib().hm_sre_batched_grad_workspace(ctx.h, ns_a, B, dt, ctypes.byref(nb)))
    ws = _workspace(nb.value, psis[0].device, stream)
    _check(lib().hm_sre_batched_grad(ctx.h, pp, ns_a, B, dt, float(q), _ptr(out), gp, _ptr(ws), ws.numel(),
                                     _stream(stream)))
    return out, grads


def _make_autograd():
    torch = _torch()

    def _needs_grad(ctx_, q):
        need = bool(ctx_.needs_input_grad[0])
        if need and float(q) == 1.0:
            raise ValueError("the gradient of M_q is built for q != 1 (q = 1 is the Shannon limit); "
                             "call with a state that does not require grad, or another q")
        return need

    class SRE(torch.autograd.Function):
        """M_q(psi) as a differentiable scalar.  When psi requires grad, forward runs the fused
        forward + adjoint kernel once and keeps dM/dpsi for backward (one library call per step);
        otherwise it runs the plain forward."""

        @staticmethod
        def forward(ctx_, psi, q=2.0):
            if _needs_grad(ctx_, q):
                out, grad = sre_grad(psi, float(q))
                ctx_.save_for_backward(grad)
                return out[0]
            return sre(psi, (float(q),))[0]

        @staticmethod
        def backward(ctx_, g):
            (grad,) = ctx_.saved_tensors
            return grad * g.to(grad.real.dtype), None

    class SREBatched(torch.autograd.Function):
        """M_q of each row of a (B, 2^n) batch as a differentiable vector; with grad required, forward
        runs the batched fused forward + adjoint once and keeps the gradients for backward."""

        @staticmethod
        def forward(ctx_, psis, q=2.0):
            if _needs_grad(ctx_, q):
                out, grads = sre_grad_batched(psis, float(q))
                ctx_.save_for_backward(grads)
                return out[:, 0]
            return sre_batched(list(psis.contiguous().unbind(0)), (float(q),))[:, 0]

        @staticmethod
        def backward(ctx_, g):
            (grads,) = ctx_.saved_tensors
            return grads * g.to(grads.real.dtype)[:, None], None

    return SRE, SREBatched


class _LazyFn:
    _cls = None

    def __init__(self, index: int):
        self._index = index

    def __getattr__(self, item):
        if _LazyFn._cls is None:
            _LazyFn._cls = _make_autograd()
        return getattr(_LazyFn._cls[self._index], item)


SRE = _LazyFn(0)
SREBatched = _LazyFn(1)


# ------------------------------------------------------------------------------------------------
# qutrits
# ------------------------------------------------------------------------------------------------
def mana(psi, *, ctx: Context | None = None, stream=None):
    """[mana, sum W, 3^n sum W^2] as a float64 tensor."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 3)
    dt = _dtype_code(psi)
    out = torch.empty(3, dtype=torch.float64, device=psi.device)
    ws = _workspace(workspace_size(OP_MANA, n, dt, 1, 0, ctx), psi.device, stream)
    _check(lib().hm_mana(ctx.h, _ptr(psi), n, dt, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def mana_partial(psi, a0: int = 0, a1: int | None = None, *, ctx: Context | None = None, stream=None):
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 3)
    a1 = 3 ** n if a1 is None else a1
    dt = _dtype_code(psi)
    out = torch.empty(3, dtype=torch.float64, device=psi.device)
    ws = _workspace(workspace_size(OP_MANA, n, dt, 1, 0, ctx), psi.device, stream)
    _check(lib().hm_mana_partial(ctx.h, _ptr(psi), n, dt, a0, a1, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def mana_mixed(rho, *, ctx: Context | None = None, stream=None):
    """[mana, Tr rho, Tr rho^2] of a mixed qutrit state given as a 3^n x 3^n GPU tensor (row-major,
    complex64 or complex128)."""
    torch = _torch()
    ctx = ctx or default_context()
    if not isinstance(rho, torch.Tensor) or not rho.is_cuda or rho.dim() != 2 or rho.shape[0] != rho.shape[1]:
        raise TypeError("rho must be a square GPU tensor")
    rho = rho.contiguous()
    D = rho.shape[0]
    n = round(math.log(D, 3)) if D > 0 else -1
    if n < 1 or 3 ** n != D:
        raise ValueError(f"dimension {D} is not 3^n with n >= 1")
    dt = _dtype_code(rho)
    out = torch.empty(3, dtype=torch.float64, device=rho.device)
    ws = _workspace(workspace_size(OP_MANA_MIXED, n, dt, 1, 0, ctx), rho.device, stream)
    _check(lib().hm_mana_mixed(ctx.h, _ptr(rho), n, dt, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def mana_qudit(psi, d: int, *, ctx: Context | None = None, stream=None):
    """[mana, sum W, d^n sum W^2] of a pure state of n qudits of odd prime dimension d in {3, 5, 7}
    (GPU tensor of d^n amplitudes, complex64 or complex128)."""
    torch = _torch()
    ctx = ctx or default_context()
    if d not in (3, 5, 7):
        raise ValueError(f"d = {d} is not 3, 5 or 7")
    psi, n = _state(psi, d)
    dt = _dtype_code(psi)
    out = torch.empty(3, dtype=torch.float64, device=psi.device)
    ws = _workspace(workspace_size(OP_MANA_QUDIT, n, dt, 1, d, ctx), psi.device, stream)
    _check(lib().hm_mana_qudit(ctx.h, _ptr(psi), n, int(d), dt, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def reduced_density_matrix(psi, n_a: int, *, ctx: Context | None = None, stream=None):
    """Reduced density matrix (3^n_a x 3^n_a GPU tensor, the state's dtype) of a qutrit state on its
    first n_a qutrits."""
    torch = _torch()
    ctx = ctx or default_context()
    psi, n = _state(psi, 3)
    dt = _dtype_code(psi)
    if not 1 <= n_a <= min(n, 10):
        raise ValueError(f"n_a = {n_a} outside [1, min(n, 10)]")
    D = 3 ** n_a
    rho = torch.empty((D, D), dtype=psi.dtype, device=psi.device)
    _check(lib().hm_reduced_density(ctx.h, _ptr(psi), n, int(n_a), dt, _ptr(rho), _stream(stream)))
    return rho
