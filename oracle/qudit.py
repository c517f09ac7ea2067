"""FP64 CPU oracle of the pure-state mana of N qudits of odd prime dimension d -- TEST
INFRASTRUCTURE ONLY (only tests/ and the CPU-baseline leg of bench.py use it).

Sec. "Mana for qutrits" notes that its construction holds for any odd prime d: clock and shift
operators (Eq. clock_and_shift) with omega_d = exp(2 pi i / d), Heisenberg-Weyl operators
T_ab = omega_d^{-2^{-1} a b} Z^a X^b with 2^{-1} = (d + 1)/2 the inverse of 2 in Z_d (Eq.
pauli_qudit), phase-space point operators A_0 = d^{-N} sum_u T_u and A_u = T_u A_0 T_u^dagger (Eq.
phase-space), W(u) = tr(A_u rho)/d^N and mana = log2 sum_u |W(u)| (Eqs. mana, mana2 with 3 -> d).

Three computations that share nothing but the single-qudit Heisenberg-Weyl matrices:
  * ``wigner_dense``: every N-qudit T_u as a dense d^N x d^N Kronecker product and
    <psi|A_u|psi> = (T_u^dagger psi)^dagger A_0 (T_u^dagger psi) (N <= 2 at d = 5, 7);
  * ``mana_tensor``: A_u is the tensor product of single-qudit A_{u_k}; tr(A_u |psi><psi|) is the
    contraction of |psi><psi| with one d^2 x (d x d) matrix per qudit, leg by leg (no d^N x d^N
    operator is formed);
  * ``mana_fft``: Algorithm 4 with 3 -> d (Sec. "Calculation of mana for pure qutrit states"): for
    every shift a in Z_d^N, alpha = X_a psi (alpha_x = psi_{x - a}, digit-wise mod d),
    v_x = conj(alpha_x) alpha_{-x}, chi = F_d^{(x)N} v with (F_d)_{jk} = omega_d^{2jk}
    (Eqs. mana_FT, F3_unnorm_def with 3 -> d), accumulating sum_{a,b} |chi_b(a)|.

Every function returns [mana, sum_u W(u), d^N sum_u W(u)^2] (the last two are 1 for a normalised
pure state).  Qudit k is base-d digit k of the basis index (little-endian).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

ODD_PRIMES = (3, 5, 7, 11, 13)


def _n_of(D: int, d: int) -> int:
    if d not in ODD_PRIMES:
        raise ValueError(f"d = {d} is not an odd prime of {ODD_PRIMES}")
    n = int(round(math.log(D, d)))
    if d ** n != D:
        raise ValueError(f"length {D} is not a power of {d}")
    return n


def _omega(d: int) -> complex:
    return np.exp(2j * math.pi / d)


def clock_shift(d: int):
    """(X, Z) of Eq. clock_and_shift: X|k> = |k+1 mod d>, Z|k> = omega^k |k>."""
    X = np.zeros((d, d), dtype=np.complex128)
    for k in range(d):
        X[(k + 1) % d, k] = 1.0
    Z = np.diag([_omega(d) ** k for k in range(d)])
    return X, Z


def heisenberg_weyl_1site(d: int) -> dict:
    """{(a, b): T_ab} for a, b in Z_d (Eq. pauli_qudit)."""
    X, Z = clock_shift(d)
    inv2 = (d + 1) // 2
    w = _omega(d)
    return {(a, b): w ** ((-inv2 * a * b) % d) * np.linalg.matrix_power(Z, a) @ np.linalg.matrix_power(X, b)
            for a in range(d) for b in range(d)}


def phase_space_1site(d: int) -> dict:
    """{(a, b): A_ab} for one qudit: A_0 = (1/d) sum_u T_u, A_u = T_u A_0 T_u^dagger."""
    T = heisenberg_weyl_1site(d)
    A0 = sum(T.values()) / d
    return {u: Tu @ A0 @ Tu.conj().T for u, Tu in T.items()}


def _kron_sites(mats):
    """mats[k] acts on qudit k (digit k); the most significant qudit is the left Kronecker factor."""
    out = np.ones((1, 1), dtype=np.complex128)
    for m in mats:
        out = np.kron(m, out)
    return out


def _diagnostics(sum_abs: float, s: float, s2: float, n: int, d: int) -> np.ndarray:
    D = float(d) ** n
    return np.array([math.log2(sum_abs / D), s / D, s2 / D])


def wigner_dense(psi, d: int) -> np.ndarray:
    """<psi|A_u|psi> for every u in Z_d^{2N} (real), from N-qudit dense T_u and A_0."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = _n_of(len(psi), d)
    T1 = heisenberg_weyl_1site(d)
    keys = sorted(T1)
    Tn = [_kron_sites([T1[u] for u in us]) for us in itertools.product(keys, repeat=n)]
    A0 = sum(Tn) / d ** n
    vals = []
    for Tu in Tn:
        phi = Tu.conj().T @ psi
        vals.append(np.vdot(phi, A0 @ phi))
    vals = np.array(vals)
    assert np.max(np.abs(vals.imag)) < 1e-10, "phase-space point operators are Hermitian"
    return vals.real


def mana_dense(psi, d: int) -> np.ndarray:
    n = _n_of(len(psi), d)
    w = wigner_dense(psi, d)
    return _diagnostics(np.sum(np.abs(w)), np.sum(w), np.sum(w * w), n, d)


def mana_tensor(psi, d: int) -> np.ndarray:
    """Contracts |psi><psi| with M[u, x, y] = A_u[y, x] on every qudit (u = d a + b)."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = _n_of(len(psi), d)
    A = phase_space_1site(d)
    M = np.stack([A[u].T for u in sorted(A)])  # [u][x][y] = A_u[y, x]
    # rho[x, y] with x, y split into digits; numpy's C order puts digit n-1 first, so axis j of the
    # x block (and n + j of the y block) is digit n-1-j of x (of y)
    R = np.multiply.outer(psi, psi.conj()).reshape((d,) * (2 * n))
    for j in range(n):
        # contract x-axis j and y-axis n + j (the same qudit); the new u axis is put back at j, and the
        # y block shrinks by one axis each step, so its axis for this qudit is always n
        R = np.tensordot(M, R, axes=([1, 2], [j, n]))
        R = np.moveaxis(R, 0, j)
    w = R.reshape(-1)
    assert np.max(np.abs(w.imag)) < 1e-10 * max(1.0, np.max(np.abs(w)))
    w = w.real
    return _diagnostics(np.sum(np.abs(w)), np.sum(w), np.sum(w * w), n, d)


def _digits(n: int, d: int) -> np.ndarray:
    """dig[k, x] = base-d digit k of x, for x in [0, d^n)."""
    x = np.arange(d ** n)
    return np.array([(x // d ** k) % d for k in range(n)], dtype=np.int64)


def _from_digits(dig: np.ndarray, d: int) -> np.ndarray:
    w = d ** np.arange(dig.shape[0], dtype=np.int64)
    return np.tensordot(w, dig, axes=(0, 0))


def mana_fft_sums(psi, d: int, a0: int = 0, a1: int | None = None, chunk: int = 256) -> np.ndarray:
    """[sum |chi|, sum chi, sum chi^2] over shifts a in [a0, a1) by Algorithm 4 with 3 -> d."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = _n_of(len(psi), d)
    D = d ** n
    a1 = D if a1 is None else a1
    dig = _digits(n, d)
    neg = _from_digits((-dig) % d, d)  # index of -x
    w = _omega(d)
    F = np.array([[w ** ((2 * j * k) % d) for k in range(d)] for j in range(d)])  # (F_d)_{jk}
    tot = np.zeros(3)
    for c0 in range(a0, a1, chunk):
        a = np.arange(c0, min(a1, c0 + chunk))
        adig = np.array([(a // d ** k) % d for k in range(n)], dtype=np.int64)  # [k][shift]
        # alpha_x = psi_{x - a}
        src = _from_digits((dig[:, None, :] - adig[:, :, None]) % d, d)  # [shift][x]
        alpha = psi[src]
        v = np.conj(alpha) * alpha[:, neg]
        t = v.reshape((len(a),) + (d,) * n)
        for ax in range(1, n + 1):
            t = np.moveaxis(np.tensordot(F, t, axes=([1], [ax])), 0, ax)
        chi = t.reshape(len(a), -1)
        assert np.max(np.abs(chi.imag)) < 1e-9 * max(1.0, np.max(np.abs(chi)))
        chi = chi.real
        tot += [np.sum(np.abs(chi)), np.sum(chi), np.sum(chi * chi)]
    return tot


def mana_fft(psi, d: int) -> np.ndarray:
    n = _n_of(len(psi), d)
    s = mana_fft_sums(psi, d)
    return _diagnostics(s[0], s[1], s[2], n, d)
