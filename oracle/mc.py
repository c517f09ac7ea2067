"""FP64 CPU oracle of the Monte Carlo estimate of M_2 by thermodynamic integration -- TEST
INFRASTRUCTURE ONLY (only tests/, the smoke check and the CPU-baseline leg of bench.py use it).

Follows the paper's sampling algorithm for the SRE (Sec. "Monte Carlo sampling algorithm for SRE",
the thermodynamic-integration scheme and its Algorithm), in its notation:

  * energy of an X-string a:  f(a) = -ln( S(a) + eps ),  S(a) = sum_b <psi|X_a Z_b|psi>^4   (Eq. feP),
    computed with one fast Walsh-Hadamard transform per row (``oracle.sre_rows``, Algorithm 2);
  * Boltzmann weights Pi_beta(a) ~ exp(-beta f(a)) (Eq. Boltz), sampled by Metropolis-Hastings
    with a symmetric proposal a' = a XOR m and acceptance min(1, exp(-beta (f(a') - f(a))));
  * I = int_0^1 <f>_beta d beta (Eq. Ie) on the grid beta_l = l / (L - 1) with Simpson weights w_l;
    since <f>_beta = -d ln Z_beta / d beta (Eq. f_expect_beta_reg), I = ln Z_0 - ln Z_1 with
    Z_0 = 2^N and Z_1 = S_2 + 2^N eps;
  * M_2 = -log2(S_2 / 2^N) = -log2(e^-I - eps);
  * error bar  dM_2 = (1/ln 2) sqrt( sum_l w_l^2 2 tau_l sigma_l^2 / n_l ) (Eqs. Var_I_eps, m2error),
    tau_l the integrated autocorrelation time of the chain at beta_l.

Readings taken where the paper is silent or inconsistent:
  * sign of the integration identity: Eq. TI_logZ_reg states ln Z_1 - ln Z_0, the negative of what
    Eq. f_expect_beta_reg integrates to, and the algorithm's return value -I / ln 2 is then negative
    for every state with S(a) < 1; the reading I = ln Z_0 - ln Z_1, M_2 = -log2(e^-I - eps) (= I / ln 2
    for eps = 0) is the one the definitions fix;
  * the energy uses the natural log: the Boltzmann and integration identities and M_2 = -I / ln 2
    hold only for it (Eq. feP prints log2);
  * L is odd (composite Simpson needs an even number of panels; the algorithm asks for an even L);
  * the identity string (a = 0, b = 0, <I> = 1) can be left out of the sampled energy and added back
    exactly, as the paper does for its figure: S'(0) = S(0) - <I>^4 = sum_{b != 0} <Z_b>^4, and
    then Z_1 = S_2 - 1 + 2^N eps, so M_2 = -log2(e^-I - eps + 2^-N);
  * several independent chains may run at each beta (chains_per_beta = R): the estimate of <f>_beta
    is the mean of their means, with variance sum_r 2 tau_r sigma_r^2 / (n R^2);
  * tau_int = 1/2 + sum_{t=1}^{W} rho(t), with rho(t) = C(t)/C(0), C(t) = (1/n) sum_i dx_i dx_{i+t},
    and W the smallest window with W >= 5 tau(W) (automatic windowing), W <= n/2;
  * the random numbers of the chain (initial strings, XOR masks of the proposals, the uniforms of the
    acceptance test) are inputs, so the oracle and the GPU chains can be compared step by step.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as _orc

WINDOW_C = 5.0


def simpson_weights(L: int) -> np.ndarray:
    """Composite Simpson weights on beta_l = l/(L-1), l = 0..L-1 (L odd, >= 3)."""
    if L < 3 or L % 2 == 0:
        raise ValueError("Simpson's rule needs an odd number of grid points >= 3")
    h = 1.0 / (L - 1)
    w = np.ones(L)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    return w * h / 3.0


def betas(L: int) -> np.ndarray:
    return np.arange(L, dtype=np.float64) / (L - 1)


def tau_int(x) -> float:
    """Integrated autocorrelation time with automatic windowing (see module docstring)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 2:
        return 0.5
    d = x - x.mean()
    c0 = float(np.dot(d, d)) / n
    if c0 == 0.0:
        return 0.5
    tau = 0.5
    for t in range(1, n // 2 + 1):
        tau += float(np.dot(d[:-t], d[t:])) / n / c0
        if t >= WINDOW_C * tau:
            break
    return tau


def identity_free_s0(psi) -> float:
    """S'(0) = sum_{b != 0} <Z_b>^4 (the a = 0 row without the identity string), from the row values."""
    vals, _ = _orc.sre_row_values_fwht(psi, 0)
    return float(np.sum(vals[1:] ** 4))


def row_s(psi, rows, s0_excl: float | None) -> np.ndarray:
    """S(a) for each a in rows (S'(0) in place of S(0) when s0_excl is given)."""
    rows = np.asarray(rows, dtype=np.uint64)
    s = _orc.sre_rows(psi, rows, (2.0,))[:, 1].copy()
    if s0_excl is not None:
        s[rows == 0] = s0_excl
    return s


def energy(s, eps: float) -> np.ndarray:
    """f = -ln(S + eps); +inf where S + eps is zero."""
    v = np.asarray(s, dtype=np.float64) + eps
    with np.errstate(divide="ignore"):
        return np.where(v > 0.0, -np.log(np.where(v > 0.0, v, 1.0)), np.inf)


def run_chains(psi, L: int, R: int, a_init, moves, uniforms, eps: float = 0.0, exclude_identity: bool = True,
               return_states: bool = False):
    """See _run_chains; small states run the row transforms on one host thread (the per-step calls
    are too short to share out)."""
    small = len(psi) <= 4096
    keep = _orc.get_threads()
    if small:
        _orc.set_threads(1)
    try:
        return _run_chains(psi, L, R, a_init, moves, uniforms, eps, exclude_identity, return_states)
    finally:
        if small:
            _orc.set_threads(keep)


def _run_chains(psi, L: int, R: int, a_init, moves, uniforms, eps: float, exclude_identity: bool,
                return_states: bool):
    """Runs the L * R Metropolis chains (chain c = l * R + r at beta_l) for moves.shape[0] steps.

    a_init: (C,) uint64; moves: (n_steps, C) uint64 XOR masks; uniforms: (n_steps, C) in [0, 1).
    Returns (trace (n_steps, C) of the current energy after each step, accepted moves per chain) and,
    with return_states, the (n_steps, C) current X-strings."""
    C = L * R
    a_init = np.asarray(a_init, dtype=np.uint64)
    moves = np.asarray(moves, dtype=np.uint64)
    uniforms = np.asarray(uniforms, dtype=np.float64)
    n_steps = moves.shape[0]
    assert a_init.shape == (C,) and moves.shape == (n_steps, C) and uniforms.shape == (n_steps, C)
    beta = np.repeat(betas(L), R)
    s0 = identity_free_s0(psi) if exclude_identity else None
    cur = a_init.copy()
    f_cur = energy(row_s(psi, cur, s0), eps)
    trace = np.empty((n_steps, C))
    states = np.empty((n_steps, C), dtype=np.uint64) if return_states else None
    accepted = np.zeros(C, dtype=np.int64)
    for t in range(n_steps):
        prop = cur ^ moves[t]
        f_new = energy(row_s(psi, prop, s0), eps)
        # accept at beta = 0, on a lower energy, or with probability exp(-beta (f' - f))
        with np.errstate(invalid="ignore", over="ignore"):
            d = f_new - f_cur
            acc = (beta == 0.0) | (d <= 0.0) | (uniforms[t] < np.exp(-beta * d))
        cur = np.where(acc, prop, cur)
        f_cur = np.where(acc, f_new, f_cur)
        accepted += acc
        trace[t] = f_cur
        if return_states:
            states[t] = cur
    if return_states:
        return trace, accepted, states
    return trace, accepted


def estimate(trace, L: int, R: int, n_therm: int, n: int, eps: float = 0.0, exclude_identity: bool = True) -> dict:
    """M_2 estimate and error bar from the chains' energy traces (samples n_therm.. of each chain)."""
    x = np.asarray(trace, dtype=np.float64)[n_therm:]
    m = x.shape[0]
    w = simpson_weights(L)
    mean_l = np.empty(L)
    var_l = np.empty(L)  # variance of the beta-point estimate
    sig2_l = np.empty(L)
    tau_l = np.empty(L)
    for l in range(L):
        means, vs, s2s, taus = [], [], [], []
        for r in range(R):
            col = x[:, l * R + r]
            mu = float(col.mean())
            s2 = float(np.mean((col - mu) ** 2))
            tau = tau_int(col)
            means.append(mu)
            s2s.append(s2)
            taus.append(tau)
            vs.append(2.0 * tau * s2 / m)
        mean_l[l] = float(np.mean(means))
        var_l[l] = float(np.sum(vs)) / R ** 2
        sig2_l[l] = float(np.mean(s2s))
        tau_l[l] = float(np.mean(taus))
    I = float(np.dot(w, mean_l))
    var_I = float(np.dot(w ** 2, var_l))
    extra = 2.0 ** -n if exclude_identity else 0.0
    s_over_D = math.exp(-I) - eps + extra
    M2 = -math.log2(s_over_D)
    dM2 = math.exp(-I) / s_over_D * math.sqrt(var_I) / math.log(2.0)
    return {"M2": M2, "dM2": dM2, "I": I, "S2": s_over_D * 2.0 ** n, "mean": mean_l, "var": var_l,
            "sigma2": sig2_l, "tau": tau_l}


def exact_ti(psi, L: int, eps: float = 0.0, exclude_identity: bool = True) -> dict:
    """<f>_beta_l by enumeration of all 2^N rows (small N) and the Simpson integral, against the closed
    form ln Z_0 - ln Z_1."""
    n = int(round(math.log2(len(psi))))
    rows = np.arange(2 ** n, dtype=np.uint64)
    s0 = identity_free_s0(psi) if exclude_identity else None
    f = energy(row_s(psi, rows, s0), eps)
    mean_l = np.empty(L)
    for l, b in enumerate(betas(L)):
        lw = -b * f
        lw -= lw.max()
        p = np.exp(lw)
        p /= p.sum()
        mean_l[l] = float(np.dot(p, f))
    I_quad = float(np.dot(simpson_weights(L), mean_l))
    Z1 = float(np.sum(np.exp(-f)))
    I_exact = n * math.log(2.0) - math.log(Z1)
    return {"mean": mean_l, "I_quad": I_quad, "I_exact": I_exact, "f": f}
