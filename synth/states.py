"""Seeded synthetic state vectors of N qudits (d = 2 qubits, d = 3 qutrits, odd primes d = 5, 7).

Conventions used everywhere in this repository:

* A state of N qudits is a complex128 numpy vector of length d**N.
* Little-endian digits: basis index i = sum_k x_k * d**k, so qudit k is digit k of the index.
* All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64); the same seed gives the
  same state on every machine.

The generators mirror the workloads of the paper's benchmarks (Sec. "Examples and benchmarks":
brick-wall circuits of Haar-random two-qudit gates, Eq. randC) plus states whose magic is known in
closed form (stabilizer states from random Clifford circuits, Clifford images of T-states, product
states).  Nothing here computes a magic measure.
"""
from __future__ import annotations

import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np

__all__ = [
    "rng", "gaussian_state", "zero_state", "ghz_state", "product_state", "qubit_product_state",
    "random_product_state", "haar_unitary", "apply_1q", "apply_2q", "brickwall_pairs",
    "brickwall_haar", "H", "S", "T", "CZ", "random_clifford_ops", "apply_ops",
    "random_clifford_state", "clifford_t_state", "t_plus_clifford_state", "F3", "D3", "SUM3",
    "random_qutrit_clifford_ops", "random_qutrit_clifford_state", "ry_rz_cz_state",
    "ry_rz_cz_state_torch", "uniform_rows", "parity_conserving_state", "to_c64_exact",
    "random_density", "pure_density", "ops_unitary", "qudit_clifford_gates", "random_qudit_clifford_ops",
    "random_qudit_clifford_state", "qudit_cubic_phase",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _normalise(v: np.ndarray) -> np.ndarray:
    return (v / np.linalg.norm(v)).astype(np.complex128)


def gaussian_state(n: int, d: int = 2, seed: int = 0) -> np.ndarray:
    """i.i.d. complex Gaussian CN(0,1) amplitudes, L2-normalised (a Haar-random state)."""
    g = rng(seed)
    D = d ** n
    v = g.standard_normal(D) + 1j * g.standard_normal(D)
    return _normalise(v)


def zero_state(n: int, d: int = 2) -> np.ndarray:
    v = np.zeros(d ** n, dtype=np.complex128)
    v[0] = 1.0
    return v


def ghz_state(n: int) -> np.ndarray:
    v = np.zeros(2 ** n, dtype=np.complex128)
    v[0] = v[-1] = 1.0 / math.sqrt(2.0)
    return v


def product_state(singles: Sequence[np.ndarray]) -> np.ndarray:
    """Tensor product; ``singles[k]`` is the state of qudit k (digit k of the index)."""
    out = np.ones(1, dtype=np.complex128)
    for s in singles:  # kron(s_k, rest) puts qudit k above the ones already present
        out = np.kron(np.asarray(s, dtype=np.complex128), out)
    return out


def qubit_product_state(thetas: Iterable[float], phis: Iterable[float]) -> np.ndarray:
    """prod_k [cos(theta_k/2)|0> + e^{i phi_k} sin(theta_k/2)|1>]."""
    singles = [np.array([math.cos(t / 2), complex(math.cos(p), math.sin(p)) * math.sin(t / 2)])
               for t, p in zip(thetas, phis)]
    return product_state(singles)


def random_product_state(n: int, d: int = 2, seed: int = 0) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Product of n seeded single-qudit CN(0,1) states; returns (state, list of single-site states)."""
    g = rng(seed)
    singles = []
    for _ in range(n):
        s = g.standard_normal(d) + 1j * g.standard_normal(d)
        singles.append(_normalise(s))
    return product_state(singles), singles


def haar_unitary(m: int, g: np.random.Generator) -> np.ndarray:
    """Haar-random U(m): QR of a complex Ginibre matrix with the phases of diag(R) divided out."""
    z = (g.standard_normal((m, m)) + 1j * g.standard_normal((m, m))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def _axis(n: int, k: int) -> int:
    # numpy C-order reshape to (d,)*n puts the most significant digit (qudit n-1) on axis 0
    return n - 1 - k


def apply_1q(psi: np.ndarray, n: int, k: int, U: np.ndarray, d: int = 2) -> np.ndarray:
    t = psi.reshape((d,) * n)
    t = np.moveaxis(np.tensordot(U, t, axes=([1], [_axis(n, k)])), 0, _axis(n, k))
    return np.ascontiguousarray(t).reshape(-1)


def apply_2q(psi: np.ndarray, n: int, k1: int, k2: int, U: np.ndarray, d: int = 2) -> np.ndarray:
    """Apply a d^2 x d^2 gate; its row/column index is d*x_{k1} + x_{k2}."""
    t = psi.reshape((d,) * n)
    a1, a2 = _axis(n, k1), _axis(n, k2)
    U4 = U.reshape(d, d, d, d)
    t = np.tensordot(U4, t, axes=([2, 3], [a1, a2]))
    t = np.moveaxis(t, [0, 1], [a1, a2])
    return np.ascontiguousarray(t).reshape(-1)


def brickwall_pairs(n: int, layer: int) -> List[Tuple[int, int]]:
    """Pairs acted on by layer ``layer`` (1-based) of the open-chain brick-wall circuit.

    Odd layers couple (0,1), (2,3), ...; even layers couple (1,2), (3,4), ... (0-based sites).
    """
    start = 0 if layer % 2 == 1 else 1
    return [(i, i + 1) for i in range(start, n - 1, 2)]


def brickwall_haar(n: int, depth: int, seed: int = 0, d: int = 2) -> np.ndarray:
    """|0...0> evolved by ``depth`` brick-wall layers of Haar-random U(d^2) gates."""
    g = rng(seed)
    psi = zero_state(n, d)
    for layer in range(1, depth + 1):
        for (i, j) in brickwall_pairs(n, layer):
            psi = apply_2q(psi, n, i, j, haar_unitary(d * d, g), d)
    return psi


# ----------------------------------------------------------------------------------------------
# Qubit Clifford circuits
# ----------------------------------------------------------------------------------------------
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
T = np.array([[1, 0], [0, np.exp(1j * math.pi / 4)]], dtype=np.complex128)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
_ONEQ_CLIFF = {
    "I": np.eye(2, dtype=np.complex128), "H": H, "S": S, "HS": H @ S, "SH": S @ H,
    "HSH": H @ S @ H, "SHS": S @ H @ S, "Z": S @ S,
}
_ONEQ_NAMES = sorted(_ONEQ_CLIFF)


def random_clifford_ops(n: int, layers: int, seed: int) -> list:
    """``layers`` layers of random single-qubit Cliffords followed by CZ on random disjoint pairs."""
    g = rng(seed)
    ops = []
    for _ in range(layers):
        for k in range(n):
            ops.append(("1q", k, _ONEQ_CLIFF[_ONEQ_NAMES[g.integers(len(_ONEQ_NAMES))]]))
        perm = g.permutation(n)
        for p in range(0, n - 1, 2):
            if g.random() < 0.75:
                ops.append(("2q", int(perm[p]), int(perm[p + 1]), CZ))
    return ops


def apply_ops(psi: np.ndarray, n: int, ops: list, d: int = 2) -> np.ndarray:
    for op in ops:
        if op[0] == "1q":
            psi = apply_1q(psi, n, op[1], op[2], d)
        else:
            psi = apply_2q(psi, n, op[1], op[2], op[3], d)
    return psi


def random_clifford_state(n: int, seed: int, layers: int | None = None) -> np.ndarray:
    """Stabilizer state: random Clifford circuit (4N layers by default) applied to |0...0>."""
    return apply_ops(zero_state(n), n, random_clifford_ops(n, layers or 4 * n, seed))


def clifford_t_state(n: int, k: int, seed: int, layers: int | None = None) -> np.ndarray:
    """Random Clifford circuit with ``k`` T gates inserted at seeded random (layer, qubit) slots."""
    layers = layers or 4 * n
    g = rng(seed + 7919)
    ops = random_clifford_ops(n, layers, seed)
    one_q = [i for i, op in enumerate(ops) if op[0] == "1q"]
    slots = set(int(s) for s in g.choice(len(one_q), size=min(k, len(one_q)), replace=False))
    out = []
    for i, op in enumerate(ops):
        out.append(op)
        if op[0] == "1q" and one_q.index(i) in slots:
            out.append(("1q", op[1], T))
    return apply_ops(zero_state(n), n, out)


def t_plus_clifford_state(n: int, k: int, seed: int, layers: int | None = None) -> np.ndarray:
    """Random Clifford circuit applied to (T|+>)^{(x)k} (x) |0>^{(x)(n-k)} (first k qubits)."""
    plus_t = np.array([1.0, np.exp(1j * math.pi / 4)], dtype=np.complex128) / math.sqrt(2.0)
    zero = np.array([1.0, 0.0], dtype=np.complex128)
    psi = product_state([plus_t] * k + [zero] * (n - k))
    return apply_ops(psi, n, random_clifford_ops(n, layers or 4 * n, seed))


def parity_conserving_state(n: int, seed: int) -> np.ndarray:
    """Random state supported only on even-Hamming-weight basis states (Z2 parity symmetry)."""
    g = rng(seed)
    D = 2 ** n
    v = g.standard_normal(D) + 1j * g.standard_normal(D)
    w = np.array([bin(i).count("1") & 1 for i in range(D)])
    v[w == 1] = 0
    return _normalise(v)


# ----------------------------------------------------------------------------------------------
# Qutrit Clifford circuits
# ----------------------------------------------------------------------------------------------
_W3 = np.exp(2j * math.pi / 3)
F3 = np.array([[_W3 ** (j * k) for k in range(3)] for j in range(3)], dtype=np.complex128) / math.sqrt(3)
D3 = np.diag([_W3 ** (j * j) for j in range(3)]).astype(np.complex128)
SUM3 = np.zeros((9, 9), dtype=np.complex128)
for _i in range(3):
    for _j in range(3):
        SUM3[3 * _i + (_i + _j) % 3, 3 * _i + _j] = 1.0
_ONEQ3 = {"I": np.eye(3, dtype=np.complex128), "F": F3, "D": D3, "FD": F3 @ D3, "DF": D3 @ F3,
          "FDF": F3 @ D3 @ F3, "DD": D3 @ D3}
_ONEQ3_NAMES = sorted(_ONEQ3)


def random_qutrit_clifford_ops(n: int, layers: int, seed: int) -> list:
    g = rng(seed)
    ops = []
    for _ in range(layers):
        for k in range(n):
            ops.append(("1q", k, _ONEQ3[_ONEQ3_NAMES[g.integers(len(_ONEQ3_NAMES))]]))
        perm = g.permutation(n)
        for p in range(0, n - 1, 2):
            if g.random() < 0.75:
                ops.append(("2q", int(perm[p]), int(perm[p + 1]), SUM3))
    return ops


def random_qutrit_clifford_state(n: int, seed: int, layers: int | None = None) -> np.ndarray:
    return apply_ops(zero_state(n, 3), n, random_qutrit_clifford_ops(n, layers or 4 * n, seed), d=3)


# ----------------------------------------------------------------------------------------------
# Clifford circuits of qudits of odd prime dimension d
# ----------------------------------------------------------------------------------------------
def qudit_clifford_gates(d: int) -> dict:
    """Generators of the single-qudit Clifford group for odd prime d and the two-qudit SUM gate:
    F|j> = d^{-1/2} sum_k omega^{jk}|k>, P = diag(omega^{j^2}), X, Z; SUM|i, j> = |i, i + j>
    (row/column index d*x_{k1} + x_{k2}, the layout of apply_2q)."""
    w = np.exp(2j * math.pi / d)
    j = np.arange(d)
    F = w ** np.outer(j, j) / math.sqrt(d)
    P = np.diag(w ** ((j * j) % d))
    X = np.roll(np.eye(d), 1, axis=0).astype(np.complex128)
    Z = np.diag(w ** j)
    SUM = np.zeros((d * d, d * d), dtype=np.complex128)
    for a in range(d):
        for b in range(d):
            SUM[d * a + (a + b) % d, d * a + b] = 1.0
    return {"F": F.astype(np.complex128), "P": P.astype(np.complex128), "X": X, "Z": Z.astype(np.complex128),
            "FP": (F @ P).astype(np.complex128), "PF": (P @ F).astype(np.complex128), "SUM": SUM}


def qudit_cubic_phase(d: int, c: int = 1) -> np.ndarray:
    """diag(omega^{c j^3}): a non-Clifford single-qudit gate for d >= 5 (a source of magic)."""
    w = np.exp(2j * math.pi / d)
    j = np.arange(d)
    return np.diag(w ** ((c * j ** 3) % d)).astype(np.complex128)


def random_qudit_clifford_ops(n: int, d: int, layers: int, seed: int) -> list:
    """``layers`` layers of random single-qudit Clifford generators, then SUM on random disjoint pairs."""
    gates = qudit_clifford_gates(d)
    names = ["F", "P", "X", "Z", "FP", "PF"]
    g = rng(seed)
    ops = []
    for _ in range(layers):
        for k in range(n):
            ops.append(("1q", k, gates[names[g.integers(len(names))]]))
        perm = g.permutation(n)
        for p in range(0, n - 1, 2):
            if g.random() < 0.75:
                ops.append(("2q", int(perm[p]), int(perm[p + 1]), gates["SUM"]))
    return ops


def random_qudit_clifford_state(n: int, d: int, seed: int, layers: int | None = None) -> np.ndarray:
    """Stabilizer state of N qudits: a random Clifford circuit (4N layers by default) on |0...0>."""
    return apply_ops(zero_state(n, d), n, random_qudit_clifford_ops(n, d, layers or 4 * n, seed), d=d)


# ----------------------------------------------------------------------------------------------
# Parameterised circuit for gradients: two layers of RY, RZ on every qubit followed by a CZ chain
# ----------------------------------------------------------------------------------------------
def _ry(t):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def _rz(p):
    return np.diag([np.exp(-0.5j * p), np.exp(0.5j * p)]).astype(np.complex128)


def ry_rz_cz_state(n: int, angles: np.ndarray) -> np.ndarray:
    """angles: shape (2, 2, n) = [layer][theta/phi][qubit]; RZ(phi) RY(theta) per qubit, then CZ(i,i+1)."""
    psi = zero_state(n)
    for layer in range(2):
        for k in range(n):
            psi = apply_1q(psi, n, k, _rz(angles[layer, 1, k]) @ _ry(angles[layer, 0, k]))
        for k in range(n - 1):
            psi = apply_2q(psi, n, k, k + 1, CZ)
    return psi


def ry_rz_cz_state_torch(n: int, angles, dtype=None):
    """Differentiable torch version of :func:`ry_rz_cz_state` (angles: real tensor (2, 2, n))."""
    import torch
    dtype = dtype or torch.complex128
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    psi = torch.zeros((2,) * n, dtype=dtype, device=angles.device)
    psi.view(-1)[0] = 1.0
    idx = torch.arange(2 ** n, device=angles.device)
    for layer in range(2):
        for k in range(n):
            th = angles[layer, 0, k].to(rdt)
            ph = angles[layer, 1, k].to(rdt)
            c, s = torch.cos(th / 2), torch.sin(th / 2)
            ry = torch.stack([torch.stack([c, -s]), torch.stack([s, c])]).to(dtype)
            e = torch.exp(torch.complex(torch.zeros_like(ph), -0.5 * ph))
            rz = torch.diag(torch.stack([e, torch.conj(e)]))
            U = rz @ ry
            ax = n - 1 - k
            psi = torch.movedim(torch.tensordot(U, psi, dims=([1], [ax])), 0, ax)
        flat = psi.reshape(-1)
        sign = torch.ones(2 ** n, dtype=rdt, device=angles.device)
        for k in range(n - 1):
            both = ((idx >> k) & 1) & ((idx >> (k + 1)) & 1)
            sign = sign * (1 - 2 * both).to(rdt)
        psi = (flat * sign.to(dtype)).reshape((2,) * n)
    return psi.reshape(-1)


def uniform_rows(n: int, n_rows: int, seed: int) -> np.ndarray:
    """i.i.d. uniform X-strings a in [0, 2^n), with replacement (uint64)."""
    return rng(seed).integers(0, 2 ** n, size=n_rows, dtype=np.uint64)


def to_c64_exact(psi: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Cast to complex64 and return (c64 vector, the same values widened back to complex128)."""
    c64 = psi.astype(np.complex64)
    return c64, c64.astype(np.complex128)


# ----------------------------------------------------------------------------------------------
# Density matrices of qutrits (mixed-state mana)
# ----------------------------------------------------------------------------------------------
def random_density(n: int, d: int = 3, rank: int | None = None, seed: int = 0) -> np.ndarray:
    """G G^dagger / tr with G a d^n x rank complex Ginibre matrix (rank d^n by default): a seeded
    random mixed state, as a d^n x d^n complex128 matrix (row index = ket, little-endian digits)."""
    g = rng(seed)
    D = d ** n
    r = D if rank is None else rank
    G = g.standard_normal((D, r)) + 1j * g.standard_normal((D, r))
    rho = G @ G.conj().T
    return (rho / np.trace(rho).real).astype(np.complex128)


def pure_density(psi: np.ndarray) -> np.ndarray:
    return np.outer(psi, psi.conj())


def ops_unitary(n: int, ops: list, d: int = 3) -> np.ndarray:
    """The d^n x d^n unitary of a gate list (columns = images of the basis states)."""
    D = d ** n
    U = np.empty((D, D), dtype=np.complex128)
    for c in range(D):
        e = np.zeros(D, dtype=np.complex128)
        e[c] = 1.0
        U[:, c] = apply_ops(e, n, ops, d)
    return U
