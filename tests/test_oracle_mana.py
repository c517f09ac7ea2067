"""Pins of the FP64 qutrit (mana) oracle (CPU only): dense construction of every phase-space point
operator, the discrete Hudson theorem on stabilizer states, the strange state, additivity, the
Wigner normalisation and purity identities, and the printed stabilizer example."""
import json
import math
import os

import numpy as np
import pytest

from oracle import dense
from synth import states as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [1, 2, 3])
def test_direct_and_fft_match_dense(orc, n):
    for seed in range(3):
        psi = S.gaussian_state(n, d=3, seed=300 + 10 * n + seed)
        ref = dense.mana_dense(psi)
        np.testing.assert_allclose(orc.mana_direct(psi), ref, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(orc.mana_fft(psi), ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("n", [4, 5])
def test_fft_matches_direct(orc, n):
    psi = S.gaussian_state(n, d=3, seed=400 + n)
    np.testing.assert_allclose(orc.mana_fft(psi), orc.mana_direct(psi), rtol=1e-12, atol=1e-13)


def test_dense_phase_space_operators_are_orthogonal_and_reflect():
    """tr(A_u A_u') = 3 delta_uu' (Eq. phase-space) and A_0 |x> = |-x> (Eq. A0_reflection), one qutrit."""
    T = dense.qutrit_phase_space_ops_1site()
    A0 = sum(T.values()) / 3
    A = {k: t @ A0 @ t.conj().T for k, t in T.items()}
    for k1 in A:
        for k2 in A:
            want = 3.0 if k1 == k2 else 0.0
            assert abs(np.trace(A[k1] @ A[k2]) - want) < 1e-12
    refl = np.zeros((3, 3))
    for x in range(3):
        refl[(-x) % 3, x] = 1
    np.testing.assert_allclose(A0, refl, atol=1e-12)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_stabilizer_states_have_zero_mana(orc, n):
    """Discrete Hudson theorem: stabilizer states have W >= 0, hence mana 0."""
    for psi in [S.zero_state(n, 3)] + [S.random_qutrit_clifford_state(n, seed=s) for s in range(3)]:
        out = orc.mana_fft(psi)
        assert abs(out[0]) < 1e-12
        np.testing.assert_allclose(out[1:], 1.0, atol=1e-12)


def test_strange_state():
    """(|1> - |2>)/sqrt(2): W = 1/3 on 8 points except -1/3 at the origin -> sum |W| = 5/3."""
    import oracle
    psi = np.array([0, 1, -1], dtype=np.complex128) / math.sqrt(2)
    want = math.log2(5 / 3)
    assert abs(oracle.mana_direct(psi)[0] - want) < 1e-13
    assert abs(oracle.mana_fft(psi)[0] - want) < 1e-13
    W = np.sort(dense.wigner_dense(psi))
    np.testing.assert_allclose(W, [-1 / 3] + [1 / 6] * 8, atol=1e-13)


def test_additivity_on_products(orc):
    psi, singles = S.random_product_state(5, d=3, seed=21)
    want = sum(float(orc.mana_direct(s)[0]) for s in singles)
    assert abs(orc.mana_fft(psi)[0] - want) < 1e-11


def test_clifford_invariance(orc):
    n = 4
    psi = S.gaussian_state(n, d=3, seed=22)
    ref = orc.mana_fft(psi)
    cpsi = S.apply_ops(psi, n, S.random_qutrit_clifford_ops(n, 3 * n, seed=23), d=3)
    np.testing.assert_allclose(orc.mana_fft(cpsi), ref, rtol=1e-11, atol=1e-12)


def test_wigner_normalisation_and_purity(orc):
    """sum_u W = 1 (Sec. 2) and 3^N sum_u W^2 = tr(rho^2) = 1 (orthogonality + purity)."""
    for n in (3, 6):
        out = orc.mana_fft(S.gaussian_state(n, d=3, seed=n))
        np.testing.assert_allclose(out[1:], 1.0, atol=1e-12)


def test_rows_sum_to_total(orc):
    n = 4
    psi = S.gaussian_state(n, d=3, seed=24)
    rows = np.arange(3 ** n, dtype=np.uint64)
    np.testing.assert_allclose(orc.mana_rows(psi, rows).sum(axis=0), orc.mana_fft_sums(psi), rtol=1e-13)


def test_transform_output_is_real(orc):
    """chi_b(a) is real for every a, b (v_{-x} = conj(v_x)): sum chi^2 equals sum |chi|^2."""
    n = 3
    psi = S.gaussian_state(n, d=3, seed=25)
    s = orc.mana_fft_sums(psi)
    # sum_b chi_b^2 (real part squared) is recovered by the purity identity only if Im chi = 0
    assert abs(s[2] / 3 ** n - 1.0) < 1e-12


def test_paper_printed_stabilizer_example(orc):
    """Printed example: rand_haar(10; depth=0, q=3) = |0>^{(x)10}, Mana = -1.97e-14 (zero to rounding).

    For |0...0> only the shift a = 0 carries weight, so it is checked on a = 0 and a seeded sample
    of other shifts."""
    with open(os.path.join(GOLDEN, "paper_examples.json")) as f:
        ex = json.load(f)["mana_depth0_n10"]
    n = ex["n"]
    psi = S.zero_state(n, 3)
    rows = np.concatenate([[0], np.random.default_rng(3).integers(1, 3 ** n, 15)]).astype(np.uint64)
    rs = orc.mana_rows(psi, rows)
    assert np.all(rs[1:] == 0.0)
    mana = math.log2(rs[0, 0] / 3 ** n)
    assert abs(mana - ex["mana"]) <= ex["tol"]
