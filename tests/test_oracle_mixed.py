"""Pins of the mixed-state mana oracle (oracle/mixed.py): the fast transform of the paper against the
definition (dense phase-space operators), against the pure-state Algorithm 4 on |psi><psi|, closed
forms (maximally mixed state, Tr rho, purity Tr rho^2), additivity on products, Clifford invariance,
zero mana of stabilizer mixtures, and the partial trace."""
import math

import numpy as np
import pytest

from oracle import mixed
from synth import states as S


@pytest.mark.parametrize("n", [1, 2, 3])
def test_fast_transform_equals_definition(n):
    for seed, rank in ((9601, None), (9602, 1), (9603, 2)):
        rho = S.random_density(n, rank=rank, seed=seed + n)
        np.testing.assert_allclose(mixed.mana_mixed_alg6(rho), mixed.mana_mixed_dense(rho), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_pure_states_match_algorithm_4(orc, n):
    psi = S.gaussian_state(n, d=3, seed=9610 + n)
    np.testing.assert_allclose(mixed.mana_mixed_alg6(S.pure_density(psi)), orc.mana_fft(psi), rtol=1e-11, atol=1e-11)


def test_closed_forms():
    n = 4
    D = 3 ** n
    got = mixed.mana_mixed_alg6(np.eye(D, dtype=np.complex128) / D)
    np.testing.assert_allclose(got, [0.0, 1.0, 1.0 / D], atol=1e-13)  # W = 1/9^N, purity 1/3^N
    rho = S.random_density(n, seed=9620)
    got = mixed.mana_mixed_alg6(2.5 * rho)
    assert abs(got[1] - 2.5) < 1e-12  # sum W = Tr rho
    assert abs(got[2] - 2.5 ** 2 * np.trace(rho @ rho).real) < 1e-12  # 3^N sum W^2 = Tr rho^2
    assert got[0] > 0  # a generic mixed state has mana; sum |W| >= sum W


def test_additivity_and_clifford_invariance():
    r1, r2 = S.random_density(2, seed=9631), S.random_density(2, seed=9632)
    prod = np.kron(r2, r1)  # qutrits 0, 1 carry r1 (low digits), qutrits 2, 3 carry r2
    got = mixed.mana_mixed_alg6(prod)[0]
    assert abs(got - (mixed.mana_mixed_alg6(r1)[0] + mixed.mana_mixed_alg6(r2)[0])) < 1e-11
    n = 3
    rho = S.random_density(n, rank=2, seed=9633)
    U = S.ops_unitary(n, S.random_qutrit_clifford_ops(n, 6, seed=9634))
    assert abs(mixed.mana_mixed_alg6(U @ rho @ U.conj().T)[0] - mixed.mana_mixed_alg6(rho)[0]) < 1e-11


def test_stabilizer_mixture_has_zero_mana():
    n = 3
    w = np.random.default_rng(9640).dirichlet(np.ones(4))
    rho = sum(wk * S.pure_density(S.random_qutrit_clifford_state(n, seed=9641 + k)) for k, wk in enumerate(w))
    got = mixed.mana_mixed_alg6(rho)
    assert abs(got[0]) < 1e-12 and abs(got[1] - 1) < 1e-12


def test_reduced_density():
    singles = [S.gaussian_state(1, d=3, seed=9650 + k) for k in range(5)]
    psi = S.product_state(singles)
    rho = mixed.reduced_density(psi, 2)
    want = np.kron(np.outer(singles[1], singles[1].conj()), np.outer(singles[0], singles[0].conj()))
    np.testing.assert_allclose(rho, want, atol=1e-14)
    psi = S.gaussian_state(6, d=3, seed=9660)
    rho = mixed.reduced_density(psi, 4)
    assert abs(np.trace(rho) - 1) < 1e-13 and np.allclose(rho, rho.conj().T)
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-13
    # mana of a reduced product state = sum of the kept single-qutrit manas
    psi = S.product_state(singles)
    got = mixed.mana_mixed_alg6(mixed.reduced_density(psi, 3))[0]
    want = sum(mixed.mana_mixed_alg6(S.pure_density(s))[0] for s in singles[:3])
    assert abs(got - want) < 1e-11
