"""Pins of the odd-prime qudit mana oracle (oracle/qudit.py) -- CPU only.

* d = 3 reduces to the qutrit oracle, which is pinned on its own (test_oracle_mana.py): the C oracle's
  direct phase-space sum and Algorithm 4, and the dense qutrit construction.
* Single-qudit operator identities that the definitions fix (Eqs. clock_and_shift, pauli_qudit,
  phase-space): A_0|x> = |-x>, tr(A_u A_u') = d delta, A_u Hermitian, sum_u A_u = d I, and the
  Heisenberg-Weyl operators closing up to phases.
* The three computations agree (dense operators, leg-by-leg tensor contraction, Algorithm 4 with
  3 -> d) at d = 5, 7.
* Discrete Hudson theorem: stabilizer states (random Clifford circuits) have mana 0; Clifford
  invariance and additivity of a magic state's mana; sum W = 1 and d^N sum W^2 = 1 for pure states.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import dense, qudit
from synth import states as S



@pytest.mark.parametrize("n", [1, 2, 3])
def test_d3_reduces_to_qutrit_oracle(n):
    psi = S.gaussian_state(n, 3, seed=30 + n)
    want = oracle.mana_direct(psi)
    for got in (qudit.mana_fft(psi, 3), qudit.mana_tensor(psi, 3)):
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    if n <= 2:
        np.testing.assert_allclose(qudit.mana_dense(psi, 3), dense.mana_dense(psi), rtol=1e-12, atol=1e-12)
        # the same Wigner values, point by point (both enumerate u in the same (a, b) order per site)
        np.testing.assert_allclose(qudit.wigner_dense(psi, 3) / 3 ** n, dense.wigner_dense(psi), atol=1e-13)


@pytest.mark.parametrize("d", [3, 5, 7])
def test_single_qudit_operator_identities(d):
    X, Z = qudit.clock_shift(d)
    w = np.exp(2j * math.pi / d)
    np.testing.assert_allclose(Z @ X, w * X @ Z, atol=1e-13)  # ZX = omega XZ
    A = qudit.phase_space_1site(d)
    keys = sorted(A)
    for x in range(d):
        e = np.zeros(d)
        e[x] = 1
        np.testing.assert_allclose(A[(0, 0)] @ e, np.eye(d)[(-x) % d], atol=1e-13)  # A_0|x> = |-x>
    G = np.array([[np.trace(A[u] @ A[v]) for v in keys] for u in keys])
    np.testing.assert_allclose(G, d * np.eye(d * d), atol=1e-12)
    for u in keys:
        np.testing.assert_allclose(A[u], A[u].conj().T, atol=1e-13)
    np.testing.assert_allclose(sum(A.values()), d * np.eye(d), atol=1e-12)


@pytest.mark.parametrize("d,n", [(5, 1), (5, 2), (7, 1), (7, 2), (5, 3)])
def test_three_computations_agree(d, n):
    psi = S.gaussian_state(n, d, seed=100 * d + n)
    a = qudit.mana_fft(psi, d)
    b = qudit.mana_tensor(psi, d)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)
    if d ** n <= 49:  # dense d^N x d^N operators for every u (d^{2N} of them)
        c = qudit.mana_dense(psi, d)
        np.testing.assert_allclose(a, c, rtol=1e-12, atol=1e-12)
    assert a[0] > 0.1  # a Haar-like state has magic
    np.testing.assert_allclose(a[1:], [1.0, 1.0], atol=1e-12)


@pytest.mark.parametrize("d,n", [(5, 1), (5, 2), (5, 3), (7, 1), (7, 2), (7, 3)])
def test_stabilizer_states_have_zero_mana(d, n):
    for seed in range(3):
        psi = S.random_qudit_clifford_state(n, d, seed=seed)
        got = qudit.mana_fft(psi, d)
        assert abs(got[0]) < 1e-12, (d, n, seed, got)
        np.testing.assert_allclose(got[1:], [1.0, 1.0], atol=1e-12)


@pytest.mark.parametrize("d", [5, 7])
def test_clifford_invariance_and_additivity(d):
    n = 2
    g = S.qudit_clifford_gates(d)
    # a magic product state: the cubic phase gate on F|0>
    one = S.qudit_cubic_phase(d) @ g["F"] @ np.eye(d)[0]
    m1 = qudit.mana_fft(one, d)[0]
    assert m1 > 0.05
    prod = S.product_state([one, one])
    np.testing.assert_allclose(qudit.mana_fft(prod, d)[0], 2 * m1, rtol=1e-12)
    psi = S.apply_ops(S.gaussian_state(n, d, seed=7), n, S.random_qudit_clifford_ops(n, d, 6, seed=8), d=d)
    base = S.gaussian_state(n, d, seed=7)
    np.testing.assert_allclose(qudit.mana_fft(psi, d), qudit.mana_fft(base, d), rtol=1e-11, atol=1e-12)


def test_shift_ranges_add_up():
    d, n = 5, 3
    psi = S.gaussian_state(n, d, seed=55)
    whole = qudit.mana_fft_sums(psi, d)
    parts = qudit.mana_fft_sums(psi, d, 0, 40) + qudit.mana_fft_sums(psi, d, 40, 125)
    np.testing.assert_allclose(parts, whole, rtol=1e-13)


def test_rejects_bad_dimension():
    with pytest.raises(ValueError):
        qudit.mana_fft(np.ones(4) / 2, 4)
    with pytest.raises(ValueError):
        qudit.mana_fft(np.ones(6), 5)
