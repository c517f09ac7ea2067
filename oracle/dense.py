"""Dense-matrix oracle for tiny systems -- TEST INFRASTRUCTURE ONLY.

Builds every operator as an explicit d^N x d^N matrix with Kronecker products and evaluates
<psi|O|psi> by matrix-vector products.  Independent of the C oracle (no shared code); used to pin
it at N <= 5 qubits and N <= 3 qutrits.

Qudit k is digit k of the basis index (little-endian), so the Kronecker product lists the most
significant qudit first.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def kron_all(mats_by_site):
    """mats_by_site[k] acts on qudit k; returns the full matrix."""
    out = np.ones((1, 1), dtype=np.complex128)
    for m in mats_by_site:
        out = np.kron(m, out)
    return out


def pauli_expectations(psi: np.ndarray) -> np.ndarray:
    """<psi|P|psi> for all 4^N Pauli strings (Eq. sre), as a real array."""
    n = int(round(math.log2(len(psi))))
    vals = []
    for letters in itertools.product("IXYZ", repeat=n):
        P = kron_all([PAULI[c] for c in letters])
        e = np.vdot(psi, P @ psi)
        assert abs(e.imag) < 1e-12
        vals.append(e.real)
    return np.array(vals)


def sre_dense(psi: np.ndarray, q=(2.0,)) -> np.ndarray:
    """[M_q..., lost_norm] from Eq. (sre); M_1 as the Shannon limit."""
    n = int(round(math.log2(len(psi))))
    e2 = pauli_expectations(psi) ** 2
    out = []
    for qq in q:
        if qq == 1.0:
            nz = e2[e2 > 0]
            out.append(-np.sum(nz * np.log2(nz)) / 2 ** n)
        else:
            out.append(math.log2(np.sum(e2 ** qq) / 2 ** n) / (1 - qq))
    out.append(1 - np.sum(e2) / 2 ** n)
    return np.array(out)


def qutrit_phase_space_ops_1site():
    """Single-qutrit A_u from Eqs. (clock_and_shift), (pauli_qudit), (phase-space); u = 3a + b."""
    w = np.exp(2j * math.pi / 3)
    X = np.roll(np.eye(3), 1, axis=0).astype(np.complex128)  # X|k> = |k+1>
    Z = np.diag([w ** k for k in range(3)])
    T = {}
    for a in range(3):
        for b in range(3):
            T[(a, b)] = w ** ((-2 * a * b) % 3) * np.linalg.matrix_power(Z, a) @ np.linalg.matrix_power(X, b)
    return T


def wigner_dense(psi: np.ndarray) -> np.ndarray:
    """W(u) = tr(A_u rho)/3^N for every u in Z_3^{2N}, built from N-qutrit T_u and A_0 directly."""
    n = int(round(math.log(len(psi), 3)))
    T1 = qutrit_phase_space_ops_1site()
    keys = list(T1)
    # N-qutrit Heisenberg-Weyl strings T_u = (x)_k T_{u_k}
    Tn = {}
    for us in itertools.product(keys, repeat=n):
        Tn[us] = kron_all([T1[u] for u in us])
    A0 = sum(Tn.values()) / 3 ** n
    W = []
    for us, Tu in Tn.items():
        Au = Tu @ A0 @ Tu.conj().T
        W.append(np.vdot(psi, Au @ psi).real / 3 ** n)
    return np.array(W)


def mana_dense(psi: np.ndarray) -> np.ndarray:
    """[mana, sum W, 3^N sum W^2] from Eq. (mana2)."""
    n = int(round(math.log(len(psi), 3)))
    W = wigner_dense(psi)
    return np.array([math.log2(np.sum(np.abs(W))), np.sum(W), 3 ** n * np.sum(W ** 2)])
