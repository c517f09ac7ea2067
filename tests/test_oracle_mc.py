"""Pins of the Monte Carlo / thermodynamic-integration oracle (oracle/mc.py) against what the
mathematics fixes: Simpson's rule is exact on cubics, the autocorrelation time of an AR(1) process,
the integration identity ln Z_1 - ln Z_0 with the identity string re-added (exactly M_2), the
stationary distribution of the Metropolis chain, acceptance of every move at beta = 0, and the
estimate agreeing with the exact M_2 within its error bar, whose size falls like n^-1/2."""
import math

import numpy as np
import pytest

from oracle import mc
from synth import states as S


def test_simpson_weights_exact_on_cubics():
    for L in (3, 5, 9, 17, 33):
        b, w = mc.betas(L), mc.simpson_weights(L)
        for k in range(4):
            assert abs(float(np.dot(w, b ** k)) - 1.0 / (k + 1)) < 1e-14, (L, k)
        assert abs(float(np.dot(w, b ** 4)) - 0.2) > 1e-6 if L == 3 else True
    for L in (2, 4, 1):
        with pytest.raises(ValueError):
            mc.simpson_weights(L)


def test_tau_int_of_ar1_and_iid():
    g = np.random.default_rng(77)
    phi, n = 0.6, 200000
    e = g.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    for i in range(1, n):
        x[i] = phi * x[i - 1] + e[i]
    want = (1 + phi) / (2 * (1 - phi))  # sum over all lags of phi^|t|, halved
    assert abs(mc.tau_int(x) - want) < 0.1 * want
    assert abs(mc.tau_int(g.standard_normal(n)) - 0.5) < 0.05
    assert mc.tau_int(np.ones(100)) == 0.5


@pytest.mark.parametrize("excl", [True, False])
def test_integration_identity_gives_m2(orc, excl):
    """int_0^1 <f>_beta = ln 2^N - ln Z_1, and with the identity re-added -log2(e^-I + 2^-N) is exactly
    M_2 (without exclusion: I / ln 2); Simpson on 33 points reproduces the integral."""
    n = 5
    psi = S.gaussian_state(n, seed=9105)
    ex = mc.exact_ti(psi, 33, exclude_identity=excl)
    m2 = orc.sre_fwht(psi, (2.0,))[0]
    got = -math.log2(math.exp(-ex["I_exact"]) + (2.0 ** -n if excl else 0.0))
    assert abs(got - m2) < 1e-12, (got, m2)
    assert abs(ex["I_quad"] - ex["I_exact"]) < 1e-4, ex
    assert np.all(np.diff(ex["mean"]) <= 1e-12)  # <f>_beta decreases with beta (d/dbeta = -Var f)


def test_metropolis_stationary_distribution(orc):
    """N = 3, single-bit flips: the chain's visit frequencies at beta = 1/2 and 1 match
    Pi_beta(a) ~ exp(-beta f(a)) within 4.5 standard errors per string (autocorrelation allowed for by
    a factor 2 tau)."""
    n, L, R, steps = 3, 3, 1, 40000
    psi = S.gaussian_state(n, seed=9103)
    g = np.random.default_rng(9203)
    moves = (np.uint64(1) << g.integers(0, n, size=(steps, L * R)).astype(np.uint64))
    uni = g.random((steps, L * R))
    a0 = g.integers(1, 2 ** n, size=L * R).astype(np.uint64)
    trace, acc, st = mc.run_chains(psi, L, R, a0, moves, uni, return_states=True)
    f = mc.exact_ti(psi, 3)["f"]
    for c, beta in ((1, 0.5), (2, 1.0)):
        p = np.exp(-beta * (f - f.min()))
        p /= p.sum()
        counts = np.bincount(st[1000:, c].astype(np.int64), minlength=2 ** n) / (steps - 1000)
        tau = mc.tau_int(trace[1000:, c])
        se = np.sqrt(p * (1 - p) * 2 * tau / (steps - 1000))
        assert np.all(np.abs(counts - p) <= 4.5 * se + 1e-12), (beta, counts, p)
    assert acc[0] == steps  # beta = 0 accepts every move


def test_estimate_matches_exact_within_error_bar(orc):
    n, L, R, steps, therm = 8, 9, 4, 1500, 100
    psi = S.brickwall_haar(n, 2 * n, seed=9108)
    g = np.random.default_rng(9208)
    C = L * R
    moves = (np.uint64(1) << g.integers(0, n, size=(steps, C)).astype(np.uint64))
    uni = g.random((steps, C))
    a0 = g.integers(1, 2 ** n, size=C).astype(np.uint64)
    trace, _ = mc.run_chains(psi, L, R, a0, moves, uni)
    est = mc.estimate(trace, L, R, therm, n)
    m2 = orc.sre_fwht(psi, (2.0,))[0]
    assert 0 < est["dM2"] < 0.1, est["dM2"]
    assert abs(est["M2"] - m2) <= 4 * est["dM2"], (est["M2"], m2, est["dM2"])


def test_error_bar_falls_like_inverse_sqrt_n(orc):
    n, L, R = 7, 5, 2
    psi = S.brickwall_haar(n, 2 * n, seed=9107)
    g = np.random.default_rng(9207)
    C = L * R
    out = []
    for steps in (400, 1600):
        moves = (np.uint64(1) << g.integers(0, n, size=(steps, C)).astype(np.uint64))
        uni = g.random((steps, C))
        a0 = g.integers(1, 2 ** n, size=C).astype(np.uint64)
        trace, _ = mc.run_chains(psi, L, R, a0, moves, uni)
        out.append(mc.estimate(trace, L, R, 50, n)["dM2"] * math.sqrt(steps - 50))
    assert 0.6 < out[1] / out[0] < 1.6, out
