"""GPU parity of the batched-states entry point (many states of uneven qubit count in one call) and
of the uniform-row Monte Carlo estimator of M_2, through the C-ABI.

Batched results are checked per state against the FP64 oracle (complex128 <= 1e-10 relative,
complex64 <= 1e-5) and against the single-state entry point.  The Monte Carlo estimate is checked
against the oracle applied to the same rows (the estimator is a deterministic function of the rows)
and, statistically, against the exact M_2 within five standard errors.
"""
import math

import numpy as np
import pytest

from synth import states as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def hm():
    import paper_2601_07824_amd as m
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)


def gpu_state(psi, c64):
    if c64:
        v, w = S.to_c64_exact(psi)
        return torch.from_numpy(v).to(_dev()), w
    return torch.from_numpy(psi).to(_dev()), psi


TOL = {False: 1e-10, True: 1e-5}


@pytest.mark.parametrize("c64", [False, True])
def test_batched_uneven_sizes_vs_oracle(orc, hm, c64):
    # resident sizes, repeats of one size out of order, and one two-pass size per dtype
    ns = [3, 8, 1, 8, 12, 5, 8, 14, 2, (17 if c64 else 16), 12]
    psis = [S.brickwall_haar(n, 2 * n, seed=7000 + i) if n > 1 else S.gaussian_state(1, seed=7000 + i)
            for i, n in enumerate(ns)]
    xs, ws = zip(*[gpu_state(p, c64) for p in psis])
    q = (1.0, 2.0, 3.0)
    say(f"[batched] ns={ns} c64={c64}")
    got = hm.sre_batched(list(xs), q).cpu().numpy()
    assert got.shape == (len(ns), len(q) + 1)
    for i, (n, w) in enumerate(zip(ns, ws)):
        want = orc.sre_direct(w, q) if n <= 6 else orc.sre_fwht(w, q)
        err = np.max(np.abs(got[i, :-1] - want[:-1]) / np.maximum(1.0, np.abs(want[:-1])))
        assert err < TOL[c64], (i, n, got[i], want)
        assert abs(got[i, -1] - want[-1]) < (1e-5 if c64 else 1e-12), (i, n, got[i], want)
        single = hm.sre(xs[i], q).cpu().numpy()
        np.testing.assert_allclose(got[i], single, rtol=TOL[c64], atol=(1e-6 if c64 else 1e-13))


def test_batched_more_than_one_launch(orc, hm):
    """70 states of n = 6 (two launches of at most 64) plus 3 of n = 10, c64."""
    ns = [6] * 70 + [10] * 3
    psis = [S.gaussian_state(n, seed=7100 + i) for i, n in enumerate(ns)]
    xs, ws = zip(*[gpu_state(p, True) for p in psis])
    say("[batched] 73 states")
    got = hm.sre_batched(list(xs), (2.0,)).cpu().numpy()
    for i, w in enumerate(ws):
        want = orc.sre_fwht(w, (2.0,))
        assert abs(got[i, 0] - want[0]) < 1e-5 * max(1.0, abs(want[0])), (i, got[i], want)
    # stabilizer and product members keep their exact values inside a batch
    stab = S.random_clifford_state(9, seed=7150)
    tpl, k = S.t_plus_clifford_state(9, 3, seed=7151), 3
    got = hm.sre_batched([gpu_state(stab, False)[0], gpu_state(tpl, False)[0]], (2.0,)).cpu().numpy()
    assert abs(got[0, 0]) < 1e-10 and abs(got[1, 0] - k * math.log2(4 / 3)) < 1e-9, got


def test_batched_1024_states_n10_to_16(orc, hm):
    """The batched benchmark workload: 1024 complex64 states with N uniform in [10, 16] (seed 5005),
    one persistent launch.  Every state against its own single call, 24 sampled states against the
    FP64 oracle."""
    rng = np.random.default_rng(5005)
    ns = rng.integers(10, 17, size=1024)
    psis = [S.gaussian_state(int(n), seed=5000 + i) for i, n in enumerate(ns)]
    xs, ws = zip(*[gpu_state(p, True) for p in psis])
    say("[batched 1024] one call")
    got = hm.sre_batched(list(xs), (2.0,)).cpu().numpy()
    single = np.stack([hm.sre(x, (2.0,)).cpu().numpy() for x in xs])
    np.testing.assert_allclose(got[:, 0], single[:, 0], rtol=2e-6, atol=0)
    for i in np.random.default_rng(5006).choice(1024, 24, replace=False):
        want = orc.sre_fwht(ws[i], (2.0,))
        assert abs(got[i, 0] - want[0]) <= 1e-5 * abs(want[0]), (i, ns[i], got[i], want)


@pytest.mark.parametrize("c64", [False, True])
def test_persistent_launch_equals_per_size_launches(hm, c64):
    """HM_OPT_BATCH_LAUNCH: the one persistent launch (default) and one launch per size class give
    the same M_2 up to FP64 summation order and the FP32 tile shape."""
    ns = [15, 6, 11, 9, 13, 6, 15, 7, 12, 10] if c64 else [14, 5, 11, 9, 12, 5, 14, 7, 10]
    xs = [gpu_state(S.gaussian_state(n, seed=7300 + i), c64)[0] for i, n in enumerate(ns)]
    per = hm.Context()
    per.set_option(hm.OPT_BATCH_LAUNCH, 2)
    say(f"[batched launch forms] c64={c64}")
    a = hm.sre_batched(xs, (1.0, 2.0)).cpu().numpy()
    b = hm.sre_batched(xs, (1.0, 2.0), ctx=per).cpu().numpy()
    np.testing.assert_allclose(a[:, :2], b[:, :2], rtol=(2e-6 if c64 else 1e-12), atol=0)


def test_per_size_launch_beyond_one_grid(hm):
    """A size class whose row tiles outnumber one launch's grid (64 states at n = 16: 4.2e6
    one-shift tiles > 2^21 workgroups) runs in several chunked launches; the per-class form equals
    the persistent launch and single calls."""
    xs = [gpu_state(S.gaussian_state(16, seed=7400 + i), True)[0] for i in range(64)]
    per = hm.Context()
    per.set_option(hm.OPT_BATCH_LAUNCH, 2)
    say("[batched chunked launches] 64 x n=16 c64")
    a = hm.sre_batched(xs, (2.0,)).cpu().numpy()
    b = hm.sre_batched(xs, (2.0,), ctx=per).cpu().numpy()
    np.testing.assert_allclose(a[:, 0], b[:, 0], rtol=2e-6, atol=0)
    for i in (0, 17, 63):
        c = hm.sre(xs[i], (2.0,)).cpu().numpy()
        np.testing.assert_allclose(b[i, :2], c, rtol=2e-6, atol=1e-9)


def test_batched_deterministic(hm):
    xs = [gpu_state(S.gaussian_state(n, seed=7200 + n), True)[0] for n in (7, 11, 11, 15)]
    say("[batched determinism]")
    a = hm.sre_batched(xs, (2.0,)).cpu().numpy()
    b = hm.sre_batched(xs, (2.0,)).cpu().numpy()
    assert np.array_equal(a, b)


def test_batched_rejects_mixed_dtypes(hm):
    a = gpu_state(S.gaussian_state(4, seed=1), True)[0]
    b = gpu_state(S.gaussian_state(4, seed=2), False)[0]
    with pytest.raises(TypeError):
        hm.sre_batched([a, b])


def sampled_reference(orc, w, n, rows):
    """The estimator written out from oracle row sums: exact a = 0 row plus the mean over the
    sampled rows a != 0."""
    rows = np.asarray(rows, dtype=np.uint64)
    s0 = orc.sre_rows(w, np.array([0], dtype=np.uint64), (2.0,))[0, 1]
    s = orc.sre_rows(w, rows, (2.0,))[:, 1][rows != 0]
    D = 2.0 ** n
    mean, std = s.mean(), s.std(ddof=1)
    shat = (s0 + (D - 1) * mean) / D
    return np.array([-math.log2(shat), (D - 1) / D * std / (math.sqrt(len(s)) * shat * math.log(2)), shat, std])


@pytest.mark.parametrize("c64,n", [(False, 10), (True, 16), (True, 20)])
def test_sampled_matches_oracle_on_same_rows(orc, hm, c64, n):
    psi = S.brickwall_haar(n, 2 * n, seed=7300 + n)
    x, w = gpu_state(psi, c64)
    rows = S.uniform_rows(n, 64 if n == 20 else 256, seed=7301)
    rows[3] = 0  # skipped by the estimator
    say(f"[sampled] n={n} c64={c64} rows={len(rows)}")
    got = hm.sre_sampled(x, rows=rows).cpu().numpy()
    want = sampled_reference(orc, w, n, rows)
    tol = 1e-5 if c64 else 1e-10
    np.testing.assert_allclose(got, want, rtol=tol * 10, atol=0)


def test_sampled_all_rows_is_exact(orc, hm):
    """Every nonzero row once: the estimate equals the exact M_2."""
    n = 9
    psi = S.gaussian_state(n, seed=7350)
    x, w = gpu_state(psi, False)
    got = hm.sre_sampled(x, rows=np.arange(1, 2 ** n)).cpu().numpy()
    assert abs(got[0] - orc.sre_fwht(w, (2.0,))[0]) < 1e-10, got


def test_sampled_estimate_within_error_bars(hm):
    """M_2 of random circuit states at N = 16, 18, 20 vs the exact value: |M_hat - M| < 5 sigma."""
    for n in (16, 18, 20):
        x, _ = gpu_state(S.brickwall_haar(n, 2 * n, seed=7400 + n), True)
        exact = hm.sre(x, (2.0,)).cpu().numpy()[0]
        for seed in (1, 2):
            est = hm.sre_sampled(x, n_rows=1024, seed=seed).cpu().numpy()
            say(f"[sampled stats] n={n} seed={seed} est={est[0]:.6f} +- {est[1]:.2e} exact={exact:.6f}")
            assert 0 < est[1] < 0.05
            assert abs(est[0] - exact) < 5 * est[1], (est, exact)


def test_sampled_large_n_runs(hm):
    """N = 24 complex64 Gaussian state (128 MB), 4096 rows: finite and close to the Haar value."""
    n = 24
    g = torch.Generator(device="cpu").manual_seed(7500)
    v = torch.randn(2 ** n, 2, generator=g, dtype=torch.float32)
    x = torch.view_as_complex(v).to(_dev())
    x /= torch.linalg.vector_norm(x)
    say("[sampled] n=24 rows=4096")
    est = hm.sre_sampled(x, n_rows=4096, seed=3).cpu().numpy()
    want = math.log2(2 ** n + 3) - 2   # Haar average, approached by Gaussian states
    assert np.all(np.isfinite(est)) and abs(est[0] - want) < max(10 * est[1], 0.01), (est, want)
