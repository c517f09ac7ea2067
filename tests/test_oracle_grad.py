"""Pins of the oracle gradient g = dM_q/dRe(psi) + i dM_q/dIm(psi) (CPU only): central finite
differences of Eq. (sre) evaluated by the direct oracle, the homogeneity and phase-invariance
identities, and agreement of the direct and transform-based gradients."""
import math

import numpy as np
import pytest

from synth import states as S


@pytest.mark.parametrize("n,q", [(3, 2.0), (4, 2.0), (5, 3.0), (4, 1.5)])
def test_direct_vs_fwht_gradient(orc, n, q):
    psi = S.gaussian_state(n, seed=600 + n)
    o1, g1 = orc.sre_grad_direct(psi, q)
    o2, g2 = orc.sre_grad_fwht(psi, q)
    np.testing.assert_allclose(o1, o2, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g2, g1, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("q", [2.0, 3.0])
def test_central_finite_differences(orc, q):
    """h = 1e-6 central differences of M_q on raw (unnormalised) coordinates, FP64."""
    n = 4
    psi = S.gaussian_state(n, seed=610)
    _, g = orc.sre_grad_fwht(psi, q)
    h = 1e-6
    fd = np.zeros_like(g)
    for y in range(2 ** n):
        for unit, part in ((1.0, "re"), (1j, "im")):
            e = np.zeros_like(psi)
            e[y] = unit * h
            d = (orc.sre_direct(psi + e, (q,))[0] - orc.sre_direct(psi - e, (q,))[0]) / (2 * h)
            fd[y] += d if part == "re" else 1j * d
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("q", [2.0, 3.0])
def test_homogeneity_and_phase_invariance(orc, q):
    """S_q has degree 4q in |psi|: Re <psi, g> = 4q / ((1-q) ln 2); M_q is phase-invariant: Im <psi, g> = 0."""
    psi = S.gaussian_state(7, seed=620)
    _, g = orc.sre_grad_fwht(psi, q)
    ip = np.vdot(g, psi)
    assert abs(ip.real - 4 * q / ((1 - q) * math.log(2))) < 1e-10
    assert abs(ip.imag) < 1e-10
