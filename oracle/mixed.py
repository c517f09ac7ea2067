"""FP64 CPU oracle of the mana of mixed qutrit states -- TEST INFRASTRUCTURE ONLY (only tests/ and
the CPU-baseline leg of bench.py use it).

Two independent computations of W(u) = Tr(rho A_u) / 3^N over all u in Z_3^{2N} and of
mana(rho) = log2 sum_u |W(u)| (Eq. mana):

  * ``wigner_mixed_dense``: the definition, with every N-qutrit phase-space point operator built from
    the Heisenberg-Weyl strings (Eqs. clock_and_shift, pauli_qudit, phase-space) as a dense matrix
    (N <= 4);
  * ``mana_mixed_alg6``: the paper's fast tensor-product transform (Sec. "Mana of mixed states via a
    fast tensor-product transform", Eq. MN_factor_mana and its Algorithm): the single-qutrit 9 x 9
    matrix M with rows vec(A_u^T) (column-stacking vec), the vectorisation Vec_N with local labels
    mu_k = 3 i_k + j_k and base-9 position sum_k mu_k 9^(N-1-k), and M applied along every leg.

Reading (the paper's vec conventions disagree): M is built from the column-stacking vec while Vec_N
uses mu = 3 i + j (row-major within a qutrit), so the transform as printed yields the Wigner function of
rho^T = conj(rho), a permutation of the phase-space points of W(rho); sum |W| and the diagnostics are
unchanged, and the oracle follows the printed steps.  The final sum is divided by 3^N (W = Tr(A rho)/3^N,
as for pure states).  ``reduced_density`` traces out qutrits n_a..N-1 (the high base-3 digits).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from oracle.dense import kron_all, qutrit_phase_space_ops_1site


def _n3(D: int) -> int:
    n = int(round(math.log(D, 3)))
    if 3 ** n != D:
        raise ValueError(f"dimension {D} is not a power of 3")
    return n


def _diagnostics(w_sum_abs, w_sum, w_sum_sq, n):
    """[mana, sum W, 3^N sum W^2] from sums of w = Tr(rho A_u) = 3^N W."""
    D = 3.0 ** n
    return np.array([math.log2(w_sum_abs / D), w_sum / D, w_sum_sq / D])


def wigner_mixed_dense(rho: np.ndarray) -> np.ndarray:
    """W(u) = Tr(A_u rho) / 3^N for every u (real parts), from the definitions (N <= 4)."""
    rho = np.asarray(rho, dtype=np.complex128)
    n = _n3(rho.shape[0])
    T1 = qutrit_phase_space_ops_1site()
    keys = list(T1)
    Tn = {us: kron_all([T1[u] for u in us]) for us in itertools.product(keys, repeat=n)}
    A0 = sum(Tn.values()) / 3 ** n
    W = []
    for Tu in Tn.values():
        Au = Tu @ A0 @ Tu.conj().T
        W.append(np.trace(Au @ rho) / 3 ** n)
    W = np.array(W)
    assert np.max(np.abs(W.imag)) < 1e-10, "Wigner function of a Hermitian operator is real"
    return W.real


def mana_mixed_dense(rho) -> np.ndarray:
    n = _n3(np.asarray(rho).shape[0])
    W = wigner_mixed_dense(rho)
    D = 3.0 ** n
    return _diagnostics(np.sum(np.abs(W)) * D, np.sum(W) * D, np.sum(W ** 2) * D * D, n)


def single_qutrit_M() -> np.ndarray:
    """M[u, alpha] = vec(A_u^T)[alpha] (column-stacking vec), u = 3a + b as in the dense oracle."""
    T1 = qutrit_phase_space_ops_1site()
    A0 = sum(T1.values()) / 3
    M = np.zeros((9, 9), dtype=np.complex128)
    for u, (key, T) in enumerate(sorted(T1.items())):
        Au = T @ A0 @ T.conj().T
        M[u] = Au.T.reshape(-1, order="F")  # column-stacking vec of A_u^T
    return M


def vec_n(rho: np.ndarray) -> np.ndarray:
    """Vec_N: v[sum_k mu_k 9^(N-1-k)] = rho[i, j], mu_k = 3 i_k + j_k (i_k, j_k: digit k of i, j)."""
    rho = np.asarray(rho, dtype=np.complex128)
    n = _n3(rho.shape[0])
    D = 3 ** n
    i = np.arange(D)
    dig = np.array([(i // 3 ** k) % 3 for k in range(n)])  # dig[k, x] = digit k of x
    p = np.zeros((D, D), dtype=np.int64)
    for k in range(n):
        mu = 3 * dig[k][:, None] + dig[k][None, :]
        p += mu * 9 ** (n - 1 - k)
    v = np.empty(D * D, dtype=np.complex128)
    v[p.reshape(-1)] = rho.reshape(-1)
    return v


def mana_mixed_alg6(rho) -> np.ndarray:
    """[mana, sum W, 3^N sum W^2] by applying M along every leg of Vec_N(rho) (the fast transform)."""
    rho = np.asarray(rho, dtype=np.complex128)
    n = _n3(rho.shape[0])
    M = single_qutrit_M()
    v = vec_n(rho)
    for leg in range(n):
        ns = 9 ** (n - 1 - leg)  # entries differing only in digit leg are ns apart
        t = v.reshape(-1, 9, ns)  # [blocks][fiber element][offset]
        v = np.einsum("ua,bam->bum", M, t).reshape(-1)
    w = v
    assert np.max(np.abs(w.imag)) < 1e-8 * max(1.0, np.max(np.abs(w)))
    w = w.real
    return _diagnostics(np.sum(np.abs(w)), np.sum(w), np.sum(w ** 2), n)


def reduced_density(psi, n_a: int) -> np.ndarray:
    """rho_A = Tr_B |psi><psi| for A = qutrits 0..n_a-1 (low base-3 digits), as a 3^n_a x 3^n_a matrix."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = _n3(len(psi))
    m = psi.reshape(3 ** (n - n_a), 3 ** n_a)  # [b][a]: index = a + 3^n_a b
    return m.T @ m.conj()
