"""Pins of the FP64 qubit oracle against what the paper and the mathematics fix (CPU only).

Every check here is independent of the oracle's own formulas: a dense Kronecker-product
construction, textbook closed forms, invariants stated in Sec. 2 of the paper, and the printed
stabilizer example of Sec. "Exact calculation of stabilizer Renyi entropy".
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import dense
from synth import states as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
QS = (1.0, 2.0, 3.0, 0.5)


def bloch(theta, phi):
    return math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)


def single_qubit_sre(theta, phi, q):
    """Closed form: the four Paulis I, X, Y, Z have expectations 1, x, y, z (Bloch vector)."""
    r = bloch(theta, phi)
    if q == 1.0:
        return -0.5 * sum(c * c * math.log2(c * c) for c in r if c != 0.0)
    return math.log2((1 + sum(abs(c) ** (2 * q) for c in r)) / 2) / (1 - q)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_direct_and_fwht_match_dense_kronecker(orc, n):
    for seed in range(3):
        psi = S.gaussian_state(n, seed=100 * n + seed)
        ref = dense.sre_dense(psi, QS)
        np.testing.assert_allclose(orc.sre_direct(psi, QS), ref, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(orc.sre_fwht(psi, QS), ref, rtol=1e-12, atol=1e-13)


def test_direct_pauli_expectations_are_real(orc):
    psi = S.gaussian_state(6, seed=7)
    _, max_im = orc.sre_direct_sums(psi, (2.0,))
    assert max_im < 1e-14


@pytest.mark.parametrize("n", [6, 8])
def test_fwht_matches_direct(orc, n):
    for seed in range(2):
        psi = S.gaussian_state(n, seed=200 + seed)
        np.testing.assert_allclose(orc.sre_fwht(psi, QS), orc.sre_direct(psi, QS), rtol=1e-12, atol=1e-13)


def test_single_qubit_bloch_closed_form(orc):
    g = np.random.default_rng(5)
    for _ in range(20):
        th, ph = g.uniform(0, math.pi), g.uniform(0, 2 * math.pi)
        psi = S.qubit_product_state([th], [ph])
        got = orc.sre_fwht(psi, QS)
        want = [single_qubit_sre(th, ph, q) for q in QS]
        np.testing.assert_allclose(got[:-1], want, rtol=1e-12, atol=1e-13)


def test_t_state_values(orc):
    """T|+> has Bloch vector (1/sqrt2, 1/sqrt2, 0): M_1 = 1/2, M_2 = log2(4/3), M_3 = log2(8/5)/2."""
    psi = S.qubit_product_state([math.pi / 2], [math.pi / 4])
    got = orc.sre_direct(psi, (1.0, 2.0, 3.0))
    np.testing.assert_allclose(got[:3], [0.5, math.log2(4 / 3), 0.5 * math.log2(8 / 5)], rtol=1e-13)


def test_additivity_on_products(orc):
    """M_q(phi (x) psi) = M_q(phi) + M_q(psi) (Sec. 2, additivity)."""
    g = np.random.default_rng(11)
    th, ph = g.uniform(0, math.pi, 7), g.uniform(0, 2 * math.pi, 7)
    psi = S.qubit_product_state(th, ph)
    got = orc.sre_fwht(psi, QS)
    want = [sum(single_qubit_sre(t, p, q) for t, p in zip(th, ph)) for q in QS]
    np.testing.assert_allclose(got[:-1], want, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("n", [3, 6, 8])
def test_stabilizer_states_have_zero_sre(orc, n):
    """Faithfulness (Sec. 2): M_q = 0 on stabilizer states."""
    cases = [S.zero_state(n), S.ghz_state(n)] + [S.random_clifford_state(n, seed=s) for s in range(3)]
    for psi in cases:
        got = orc.sre_fwht(psi, QS)
        np.testing.assert_allclose(got, 0.0, atol=1e-12)


def test_clifford_invariance(orc):
    """M_q(C psi) = M_q(psi) for Clifford C (Sec. 2)."""
    n = 7
    psi = S.gaussian_state(n, seed=3)
    ref = orc.sre_fwht(psi, QS)
    for s in range(3):
        cpsi = S.apply_ops(psi, n, S.random_clifford_ops(n, 3 * n, seed=40 + s))
        np.testing.assert_allclose(orc.sre_fwht(cpsi, QS), ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("k", [0, 1, 3, 5])
def test_clifford_image_of_t_states(orc, k):
    """Clifford invariance + additivity: C (T|+>)^{(x)k} |0...0> has M_2 = k log2(4/3)."""
    psi = S.t_plus_clifford_state(8, k, seed=90 + k)
    got = orc.sre_fwht(psi, (2.0,))
    assert abs(got[0] - k * math.log2(4 / 3)) < 1e-11
    assert abs(got[1]) < 1e-13


def test_lost_norm_vanishes(orc):
    """sum_P <P>^2 / 2^N = 1 for a normalised state (Eq. distNAT)."""
    for n in (5, 9):
        psi = S.gaussian_state(n, seed=n)
        assert abs(orc.sre_fwht(psi, (2.0,))[1]) < 1e-13


def test_haar_average_matches_closed_form(orc):
    """Mean M_2 of Haar-random states approaches log2(2^N + 3) - 2 (paper, after the first example)."""
    n = 9
    vals = [orc.sre_fwht(S.gaussian_state(n, seed=5000 + s), (2.0,))[0] for s in range(12)]
    want = math.log2(2 ** n + 3) - 2
    # M_2 = -log2(S_2/2^N) is concave in S_2, so the sample mean sits slightly below; allow 4 sigma.
    sem = np.std(vals, ddof=1) / math.sqrt(len(vals))
    assert abs(np.mean(vals) - want) < 4 * sem + 2e-3


def test_row_values_direct_vs_fast_phase(orc):
    """<P_{a,b}> = i^{popcount(a&b)} chi_b(a) (Pauli parametrisation, Sec. 2) and Im = 0."""
    psi = S.gaussian_state(7, seed=8)
    for a in (0, 1, 5, 77, 127):
        d = orc.sre_row_values_direct(psi, a)
        f, mi = orc.sre_row_values_fwht(psi, a)
        np.testing.assert_allclose(f, d, atol=1e-14)
        assert mi < 1e-14


def test_row_parseval_and_identity_column(orc):
    """sum_b |chi_b(a)|^2 = 2^N sum_x |psi_{x^a}|^2 |psi_x|^2 and chi_0(a) = <psi|X_a|psi>."""
    n = 8
    psi = S.gaussian_state(n, seed=9)
    rows = np.array([0, 3, 100, 255], dtype=np.uint64)
    rs = orc.sre_rows(psi, rows, (2.0,))
    x = np.arange(2 ** n)
    for r, a in enumerate(rows):
        want = 2 ** n * np.sum(np.abs(psi[x ^ int(a)]) ** 2 * np.abs(psi) ** 2)
        assert abs(rs[r, 0] - want) < 1e-12 * max(1.0, want)
        vals, _ = orc.sre_row_values_fwht(psi, int(a))
        assert abs(vals[0] - np.vdot(psi[x ^ int(a)], psi).real) < 1e-13


def test_rows_sum_to_total(orc):
    n = 7
    psi = S.gaussian_state(n, seed=10)
    rows = np.arange(2 ** n, dtype=np.uint64)
    rs = orc.sre_rows(psi, rows, (2.0, 3.0))
    np.testing.assert_allclose(rs.sum(axis=0), orc.sre_fwht_sums(psi, (2.0, 3.0)), rtol=1e-13)
    half = orc.sre_fwht_sums(psi, (2.0, 3.0), 0, 50) + orc.sre_fwht_sums(psi, (2.0, 3.0), 50, 128)
    np.testing.assert_allclose(half, orc.sre_fwht_sums(psi, (2.0, 3.0)), rtol=1e-13)


def test_parity_symmetry_zeroes_odd_rows(orc):
    """Z2-parity-conserving states have S(a) = 0 exactly for odd |a| (Sec. on sampling, vanishing sectors)."""
    n = 8
    psi = S.parity_conserving_state(n, seed=12)
    rows = np.arange(2 ** n, dtype=np.uint64)
    rs = orc.sre_rows(psi, rows, (2.0,))
    odd = np.array([bin(a).count("1") & 1 for a in range(2 ** n)], dtype=bool)
    assert np.all(rs[odd] == 0.0)
    assert np.all(rs[~odd][:, 1] > 0)


def test_paper_printed_stabilizer_example(orc):
    """Printed example: rand_haar(16; depth=0) = |0>^{(x)16} gives SRE = -0.0, lost_norm = 0.0.

    Only the identity row a = 0 carries weight for |0...0>; rows a != 0 vanish.  Checked on the
    identity row and a seeded sample of other rows (the full 4^16 enumeration is left to the
    GPU tests)."""
    with open(os.path.join(GOLDEN, "paper_examples.json")) as f:
        ex = json.load(f)["sre_depth0_n16"]
    n = ex["n"]
    psi = S.zero_state(n)
    rows = np.concatenate([[0], S.uniform_rows(n, 31, seed=1)]).astype(np.uint64)
    rs = orc.sre_rows(psi, rows, (2.0,))
    total = rs[rows == 0][0]
    assert np.all(rs[rows != 0] == 0.0)
    m2 = -math.log2(total[1] / 2 ** n)
    lost = 1 - total[0] / 2 ** n
    assert abs(m2 - ex["M2"]) <= ex["tol"] and abs(lost - ex["lost_norm"]) <= ex["tol"]


def test_shannon_limit_is_limit_of_renyi(orc):
    """M_1 is the q -> 1 limit of Eq. (sre)."""
    psi = S.gaussian_state(5, seed=13)
    m = orc.sre_fwht(psi, (1.0, 1.0 - 1e-5, 1.0 + 1e-5))
    assert abs(m[0] - 0.5 * (m[1] + m[2])) < 1e-6
