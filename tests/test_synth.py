"""Checks of the seeded state generators (CPU only): unitarity, Clifford-ness, determinism."""
import itertools
import math

import numpy as np

from oracle import dense
from synth import states as S


def _is_pauli_up_to_phase(M, n):
    for letters in itertools.product("IXYZ", repeat=n):
        P = dense.kron_all([dense.PAULI[c] for c in letters])
        ph = np.vdot(P.reshape(-1), M.reshape(-1)) / 2 ** n
        if abs(abs(ph) - 1) < 1e-12 and np.allclose(M, ph * P, atol=1e-12):
            return True
    return False


def test_haar_gates_unitary():
    g = np.random.default_rng(0)
    for m in (4, 9):
        U = S.haar_unitary(m, g)
        np.testing.assert_allclose(U.conj().T @ U, np.eye(m), atol=1e-12)


def test_qubit_clifford_generators_map_paulis_to_paulis():
    for name, U in S._ONEQ_CLIFF.items():
        for c in "XYZ":
            assert _is_pauli_up_to_phase(U @ dense.PAULI[c] @ U.conj().T, 1), name
    for a, b in itertools.product("IXYZ", repeat=2):
        P = dense.kron_all([dense.PAULI[a], dense.PAULI[b]])
        assert _is_pauli_up_to_phase(S.CZ @ P @ S.CZ.conj().T, 2)


def test_qutrit_clifford_generators_map_weyl_to_weyl():
    T = dense.qutrit_phase_space_ops_1site()
    ops1 = list(T.values())
    ops2 = [np.kron(a, b) for a in ops1 for b in ops1]

    def in_group(M, group):
        for G in group:
            ph = np.vdot(G.reshape(-1), M.reshape(-1)) / G.shape[0]
            if abs(abs(ph) - 1) < 1e-12 and np.allclose(M, ph * G, atol=1e-12):
                return True
        return False

    for U in (S.F3, S.D3):
        for W in ops1:
            assert in_group(U @ W @ U.conj().T, ops1)
    for W in ops2:
        assert in_group(S.SUM3 @ W @ S.SUM3.conj().T, ops2)


def test_circuits_preserve_norm_and_are_seeded():
    a = S.brickwall_haar(8, 8, seed=3)
    b = S.brickwall_haar(8, 8, seed=3)
    assert np.array_equal(a, b) and abs(np.linalg.norm(a) - 1) < 1e-12
    c = S.brickwall_haar(5, 5, seed=1, d=3)
    assert abs(np.linalg.norm(c) - 1) < 1e-12
    assert abs(np.linalg.norm(S.clifford_t_state(6, 4, seed=2)) - 1) < 1e-12


def test_brickwall_layers():
    assert S.brickwall_pairs(6, 1) == [(0, 1), (2, 3), (4, 5)]
    assert S.brickwall_pairs(6, 2) == [(1, 2), (3, 4)]
    assert S.brickwall_pairs(5, 1) == [(0, 1), (2, 3)]


def test_product_state_little_endian():
    s0 = np.array([1, 0], dtype=complex)
    s1 = np.array([0, 1], dtype=complex)
    v = S.product_state([s1, s0, s0])  # qubit 0 in |1> -> index 1
    assert v[1] == 1 and np.count_nonzero(v) == 1


def test_torch_circuit_matches_numpy():
    import torch
    n = 5
    ang = np.random.default_rng(4).uniform(0, 2 * math.pi, (2, 2, n))
    a = S.ry_rz_cz_state(n, ang)
    b = S.ry_rz_cz_state_torch(n, torch.tensor(ang)).numpy()
    np.testing.assert_allclose(a, b, atol=1e-12)
