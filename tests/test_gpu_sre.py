"""GPU parity of the qubit SRE kernels against the FP64 oracle, through the C-ABI.

Tolerances: FP64 transforms (complex128 input) <= 1e-10 relative (absolute when the reference is 0);
FP32 transforms (complex64 input) <= 1e-5 relative on M_q (absolute 1e-5 when the reference is 0).
Complex64 runs are compared with the oracle evaluated on the same complex64 values widened to
complex128, so both sides see identical inputs.
"""
import json
import math
import os

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


def rel_err(got, want, floor=1.0):
    got, want = np.asarray(got, dtype=float), np.asarray(want, dtype=float)
    return np.max(np.abs(got - want) / np.maximum(np.abs(want), floor))


def gpu_state(psi, c64: bool):
    if c64:
        v, w = S.to_c64_exact(psi)
        return torch.from_numpy(v).to(_dev()), w
    return torch.from_numpy(psi).to(_dev()), psi


TOL = {False: 1e-10, True: 1e-5}


# ---------------------------------------------------------------------------------------------
# Qubit SRE, N = 8: the small configuration (M_1, M_2, M_3, all 256 shifts)
# ---------------------------------------------------------------------------------------------
def n8_states():
    g = np.random.default_rng(1008)
    th, ph = g.uniform(0, math.pi, 8), g.uniform(0, 2 * math.pi, 8)
    out = [("gauss%d" % s, S.gaussian_state(8, seed=1000 + s)) for s in range(4)]
    out += [("zero", S.zero_state(8)), ("ghz", S.ghz_state(8)), ("product", S.qubit_product_state(th, ph))]
    return out


@pytest.mark.parametrize("c64", [False, True])
def test_n8_vs_direct_oracle(orc, hm, c64):
    q = (1.0, 2.0, 3.0)
    for name, psi in n8_states():
        say(f"[sre n8] state={name} c64={c64}")
        x, w = gpu_state(psi, c64)
        got = hm.sre(x, q).cpu().numpy()
        want = orc.sre_direct(w, q)
        assert rel_err(got[:3], want[:3]) < TOL[c64], (name, got, want)
        assert abs(got[3] - want[3]) < (1e-12 if not c64 else 1e-6), (name, got, want)


# ---------------------------------------------------------------------------------------------
# All sizes and both kernel families vs Algorithm 2 on the CPU
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("c64", [False, True])
@pytest.mark.parametrize("n", list(range(1, 14)))
def test_sizes_auto_path(orc, hm, n, c64):
    q = (2.0,) if n % 2 else (1.0, 2.0, 3.0, 0.5)
    psi = S.gaussian_state(n, seed=2000 + n)
    say(f"[sre sizes] n={n} c64={c64} q={q}")
    x, w = gpu_state(psi, c64)
    got = hm.sre(x, q).cpu().numpy()
    want = orc.sre_fwht(w, q)
    assert rel_err(got[:-1], want[:-1]) < TOL[c64], (got, want)
    assert abs(got[-1] - want[-1]) < (1e-12 if not c64 else 2e-6)


@pytest.mark.parametrize("rb", [0, 4])
@pytest.mark.parametrize("c64,n", [(False, 11), (False, 12), (False, 13), (True, 12), (True, 13), (True, 14)])
def test_forced_two_pass(orc, hm, n, c64, rb):
    """Two-pass kernels at sizes the oracle finishes quickly; batch of 5 shifts -> ragged last batch;
    default and 2^4-value register tiles in both passes."""
    ctx = hm.Context()
    ctx.force_path(2)
    ctx.batch_shifts(5)
    if rb:
        ctx.set_option(hm.OPT_ROW_RB, rb)
        ctx.set_option(hm.OPT_COL_RB, rb)
    psi = S.brickwall_haar(n, 2 * n, seed=3000 + n)
    for q in ((2.0,), (1.0, 2.0, 3.0)):
        say(f"[sre two-pass] n={n} c64={c64} q={q}")
        x, w = gpu_state(psi, c64)
        got = hm.sre(x, q, ctx=ctx).cpu().numpy()
        want = orc.sre_fwht(w, q)
        assert rel_err(got[:-1], want[:-1]) < TOL[c64], (got, want)


@pytest.mark.parametrize("c64,n,row_rb", [(False, 11, 0), (False, 13, 0), (True, 12, 0), (True, 14, 0), (True, 13, 4),
                                          (True, 15, 4)])
def test_two_pass_split_lds(orc, hm, n, c64, row_rb):
    """Sequential two-pass kernels with split LDS staging (real and imaginary parts in turn), also
    with 2^4-value row tiles."""
    ctx = hm.Context()
    ctx.force_path(2)
    ctx.batch_shifts(7)
    ctx.set_option(hm.OPT_LDS_SPLIT, 2)
    if row_rb:
        ctx.set_option(hm.OPT_ROW_RB, row_rb)
    psi = S.brickwall_haar(n, 2 * n, seed=3040 + n)
    x, w = gpu_state(psi, c64)
    for q in ((2.0,), (1.0, 3.0)):
        say(f"[sre two-pass split] n={n} c64={c64} q={q}")
        got = hm.sre(x, q, ctx=ctx).cpu().numpy()
        want = orc.sre_fwht(w, q)
        assert rel_err(got[:-1], want[:-1]) < TOL[c64], (got, want)


@pytest.mark.parametrize("c64,n", [(False, 12), (False, 14), (True, 12), (True, 15)])
def test_two_pass_two_streams(orc, hm, n, c64):
    """Sequential two-pass batches alternating between the caller's stream and the internal one:
    full sums (ragged batches), a partial range and explicit rows, against the oracle."""
    psi = S.brickwall_haar(n, 2 * n, seed=3060 + n)
    x, w = gpu_state(psi, c64)
    ctx = hm.Context()
    ctx.force_path(2)
    ctx.batch_shifts(5)
    ctx.set_option(hm.OPT_STREAMS, 2)
    say(f"[sre two streams] n={n} c64={c64}")
    got = hm.sre(x, (1.0, 2.0), ctx=ctx).cpu().numpy()
    want = orc.sre_fwht(w, (1.0, 2.0))
    assert rel_err(got[:-1], want[:-1]) < TOL[c64], (got, want)
    got = hm.sre_partial(x, (2.0,), 7, 40, ctx=ctx).cpu().numpy()
    np.testing.assert_allclose(got, orc.sre_fwht_sums(w, (2.0,), 7, 40), rtol=(1e-11 if not c64 else 2e-6))
    rows = S.uniform_rows(n, 23, seed=3061).astype(np.int64)
    got = hm.sre_rows(x, rows, (2.0,), ctx=ctx).cpu().numpy()
    want = orc.sre_rows(w, rows.astype(np.uint64), (2.0,))
    assert rel_err(got, want, floor=1e-15) < (1e-10 if not c64 else 1e-5)


@pytest.mark.parametrize("split", [1, 2])
@pytest.mark.parametrize("c64,n", [(False, 12), (False, 13), (False, 14), (True, 12), (True, 13), (True, 15)])
def test_pipelined_two_pass(orc, hm, n, c64, split):
    """Pipelined launches (row pass of batch k beside the column pass of batch k - 1): many ragged
    batches, a single batch (one row-only and one column-only launch), and a partial range of two
    batches; complex and split LDS staging."""
    psi = S.brickwall_haar(n, 2 * n, seed=3050 + n)
    x, w = gpu_state(psi, c64)
    for batch, q in ((5, (2.0,)), (5, (1.0, 2.0, 3.0)), (2 ** n, (2.0,))):
        ctx = hm.Context()
        ctx.force_path(2)
        ctx.set_option(hm.OPT_PIPELINE, 2)
        ctx.set_option(hm.OPT_LDS_SPLIT, split)
        ctx.batch_shifts(batch)
        say(f"[sre pipelined] n={n} c64={c64} split={split} batch={batch} q={q}")
        got = hm.sre(x, q, ctx=ctx).cpu().numpy()
        want = orc.sre_fwht(w, q)
        assert rel_err(got[:-1], want[:-1]) < TOL[c64], (got, want)
        assert abs(got[-1] - want[-1]) < (1e-12 if not c64 else 2e-6)
    ctx = hm.Context()
    ctx.force_path(2)
    ctx.set_option(hm.OPT_PIPELINE, 2)
    ctx.set_option(hm.OPT_LDS_SPLIT, split)
    ctx.batch_shifts(4)
    got = hm.sre_partial(x, (2.0,), 3, 10, ctx=ctx).cpu().numpy()
    want = orc.sre_fwht_sums(w, (2.0,), 3, 10)
    np.testing.assert_allclose(got, want, rtol=(1e-11 if not c64 else 2e-6))


@pytest.mark.parametrize("c64,n", [(False, 13), (False, 14), (False, 15), (True, 14), (True, 15), (True, 16)])
def test_vgpr_resident_large_tiles(orc, hm, c64, n):
    """Workgroup-resident tiles of 2^13..2^15 folded values (relayouts one component at a time),
    checked on sampled rows of the same launch configuration and on a T-state property."""
    ctx = hm.Context()
    ctx.force_path(1)
    psi = S.gaussian_state(n, seed=3150 + n)
    x, w = gpu_state(psi, c64)
    rows = np.concatenate([[0, 1, 2 ** n - 1, 2 ** (n - 1)], S.uniform_rows(n, 12, seed=3151)]).astype(np.int64)
    say(f"[sre resident large] n={n} c64={c64}")
    got = hm.sre_rows(x, rows, (2.0,), ctx=ctx).cpu().numpy()
    want = orc.sre_rows(w, rows.astype(np.uint64), (2.0,))
    assert rel_err(got, want, floor=1e-15) < (1e-10 if not c64 else 1e-5)
    k = 3
    tp = S.t_plus_clifford_state(n, k, seed=3152 + n, layers=n)
    xt, _ = gpu_state(tp, c64)
    m = hm.sre(xt, (2.0,), ctx=ctx).cpu().numpy()
    assert abs(m[0] - k * math.log2(4 / 3)) < (1e-9 if not c64 else 1e-5)


@pytest.mark.parametrize("c64,n", [(True, 11), (True, 13), (True, 14), (True, 15), (False, 11), (False, 12), (False, 14)])
def test_resident_split_staging(orc, hm, c64, n):
    """Workgroup-resident tiles of 2^10..2^14 values with split LDS staging and the raised
    occupancy register budget, against the oracle (single state and a batch of three)."""
    ctx = hm.Context()
    ctx.force_path(1)
    ctx.set_option(hm.OPT_LDS_SPLIT, 2)
    psi = S.gaussian_state(n, seed=3170 + n)
    x, w = gpu_state(psi, c64)
    say(f"[sre resident split] n={n} c64={c64}")
    got = hm.sre(x, (1.0, 2.0, 3.0), ctx=ctx).cpu().numpy()
    want = orc.sre_fwht(w, (1.0, 2.0, 3.0))
    assert rel_err(got[:-1], want[:-1]) < TOL[c64], (got, want)
    got = hm.sre_batched([x, x, x], (2.0,), ctx=ctx).cpu().numpy()
    assert rel_err(got[:, 0], np.full(3, want[1])) < TOL[c64], (got, want)


@pytest.mark.parametrize("c64", [False, True])
def test_workgroup_resident_largest(orc, hm, c64):
    n = 13 if c64 else 12
    ctx = hm.Context()
    ctx.force_path(1)
    psi = S.gaussian_state(n, seed=3100)
    say(f"[sre resident max] n={n} c64={c64}")
    x, w = gpu_state(psi, c64)
    got = hm.sre(x, (2.0,), ctx=ctx).cpu().numpy()
    want = orc.sre_fwht(w, (2.0,))
    assert rel_err(got[:1], want[:1]) < TOL[c64]


@pytest.mark.parametrize("c64", [False, True])
def test_partial_ranges_add_up(orc, hm, c64):
    """hm_sre_partial on ragged ranges equals the oracle's sums over the same ranges."""
    n = 10
    psi = S.gaussian_state(n, seed=3200)
    x, w = gpu_state(psi, c64)
    q = (2.0, 3.0)
    cuts = [0, 1, 2, 37, 511, 512, 513, 1000, 1024]
    for a0, a1 in zip(cuts[:-1], cuts[1:]):
        say(f"[sre partial] range=[{a0},{a1}) c64={c64}")
        got = hm.sre_partial(x, q, a0, a1).cpu().numpy()
        want = orc.sre_fwht_sums(w, q, a0, a1)
        assert rel_err(got, want, floor=1e-300) < (1e-11 if not c64 else 2e-6), (a0, a1, got, want)
    say("[sre partial] empty range")
    assert np.all(hm.sre_partial(x, q, 7, 7).cpu().numpy() == 0)


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("c64", [False, True])
def test_rows_vs_oracle(orc, hm, path, c64):
    n = 12
    ctx = hm.Context()
    ctx.force_path(path)
    ctx.batch_shifts(7)
    psi = S.gaussian_state(n, seed=3300)
    rows = np.concatenate([[0, 1, 2 ** n - 1, 2 ** (n - 1), 5, 5], S.uniform_rows(n, 40, seed=3301)]).astype(np.int64)
    x, w = gpu_state(psi, c64)
    say(f"[sre rows] n={n} path={path} c64={c64} rows={len(rows)}")
    got = hm.sre_rows(x, rows, (2.0,), ctx=ctx).cpu().numpy()
    want = orc.sre_rows(w, rows.astype(np.uint64), (2.0,))
    assert rel_err(got, want, floor=1e-12) < (1e-11 if not c64 else 2e-6)


def test_rows_out_of_range_give_nan(hm):
    n = 9
    x = torch.from_numpy(S.gaussian_state(n, seed=1)).to(_dev())
    say("[sre rows] out-of-range row")
    got = hm.sre_rows(x, [3, 2 ** n, 4], (2.0,)).cpu().numpy()
    assert np.all(np.isnan(got[1])) and np.all(np.isfinite(got[[0, 2]]))


@pytest.mark.parametrize("c64", [False, True])
def test_row_values_vs_oracle(orc, hm, c64):
    n = 9
    psi = S.gaussian_state(n, seed=3400)
    x, w = gpu_state(psi, c64)
    for a in (0, 1, 300, 511):
        say(f"[sre row values] a={a} c64={c64}")
        got = hm.sre_row_values(x, a).cpu().numpy()
        want, _ = orc.sre_row_values_fwht(w, a)
        assert np.max(np.abs(got - want)) < (1e-13 if not c64 else 1e-6)


def test_determinism_bitwise(hm):
    for n, c64 in ((12, True), (15, True), (11, False)):
        x, _ = gpu_state(S.gaussian_state(n, seed=3500), c64)
        say(f"[sre determinism] n={n} c64={c64}")
        a = hm.sre(x, (2.0, 3.0)).cpu().numpy()
        b = hm.sre(x, (2.0, 3.0)).cpu().numpy()
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------------------------
# Full sizes: properties that hold at any N, and sampled rows against the oracle
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [16, 20])
def test_full_size_stabilizer_and_t_states(hm, n):
    """Random Clifford circuits give M_2 = 0; Clifford images of (T|+>)^k give k log2(4/3) exactly."""
    for c64 in (True, False):
        for k in (0, 1, 4):
            psi = S.t_plus_clifford_state(n, k, seed=4000 + n + k, layers=2 * n)
            x, _ = gpu_state(psi, c64)
            say(f"[sre full] n={n} k={k} c64={c64}")
            got = hm.sre(x, (2.0,)).cpu().numpy()
            want = k * math.log2(4 / 3)
            tol = 1e-5 * max(want, 1.0) if c64 else 1e-9
            assert abs(got[0] - want) < tol, (got, want)
            assert abs(got[1]) < (1e-5 if c64 else 1e-10)


@pytest.mark.parametrize("n", [16, 20])
def test_full_size_sampled_rows(orc, hm, n):
    """Per-row sums of the launch configuration used for the full N vs the oracle (also with the
    tile variants the planner can pick)."""
    psi = S.brickwall_haar(n, 2 * n, seed=4100 + n)
    rows = np.concatenate([[0, 1, 2 ** n - 1], S.uniform_rows(n, 13, seed=4101)]).astype(np.int64)
    for c64, rb, rbits, pipe in ((True, 0, 0, 0), (False, 0, 0, 0), (True, 4, 0, 0), (True, 4, 12, 0), (True, 5, 9, 0),
                                 (True, 0, 0, 1), (True, 0, 0, 2), (False, 0, 0, 2), (True, 0, 12, -2),
                                 (False, 0, 0, -2)):
        ctx = hm.Context()
        if pipe > 0:
            ctx.set_option(hm.OPT_PIPELINE, 2)
            ctx.set_option(hm.OPT_LDS_SPLIT, pipe)
        elif pipe < 0:  # sequential launches, split LDS staging
            ctx.set_option(hm.OPT_PIPELINE, 1)
            ctx.set_option(hm.OPT_LDS_SPLIT, -pipe)
        if rb:
            ctx.set_option(hm.OPT_ROW_RB, rb)
            ctx.set_option(hm.OPT_COL_RB, rb)
        if rbits and n == 20:
            ctx.set_option(hm.OPT_ROW_BITS, rbits)
        x, w = gpu_state(psi, c64)
        say(f"[sre full rows] n={n} c64={c64} rb={rb} row_bits={rbits} pipe={pipe}")
        got = hm.sre_rows(x, rows, (2.0,), ctx=ctx).cpu().numpy()
        want = orc.sre_rows(w, rows.astype(np.uint64), (2.0,))
        assert rel_err(got, want, floor=1e-15) < (1e-10 if not c64 else 1e-5)


def test_full_size_n16_vs_golden(hm):
    """N = 16 against FP64 oracle values stored by tests/golden/make_golden.py (both paths)."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_golden.json")))
    cases = (("sre_brickwall_n16_d32_seed4200_c64", S.brickwall_haar(16, 32, seed=4200), True, (2.0,)),
             ("sre_gauss_n16_seed4201_c128", S.gaussian_state(16, seed=4201), False, (1.0, 2.0, 3.0)))
    for key, psi, c64, q in cases:
        want = np.array(gold[key]["values"])
        # c128 holds at most 2^14 folded values per workgroup, so n = 16 is two-pass only
        for path, pipe in (((1, 0), (2, 0), (2, 2)) if c64 else ((2, 0), (2, 2))):
            ctx = hm.Context()
            ctx.force_path(path)
            if pipe:
                ctx.set_option(hm.OPT_PIPELINE, pipe)
            x, _ = gpu_state(psi, c64)
            say(f"[sre n16 golden] {key} path={path} pipe={pipe}")
            got = hm.sre(x, q, ctx=ctx).cpu().numpy()
            assert rel_err(got[:-1], want[:-1]) < (1e-5 if c64 else 1e-10), (got, want)
            assert abs(got[-1] - want[-1]) < (1e-5 if c64 else 1e-12)


@pytest.mark.parametrize("c64,n", [(True, 16), (False, 14), (True, 18)])
def test_autotuned_plan_matches(orc, hm, c64, n):
    """The autotuner's choice is a valid plan and gives the same values as the default plan
    (and as the oracle where it is quick)."""
    psi = S.brickwall_haar(n, 2 * n, seed=3700 + n)
    x, w = gpu_state(psi, c64)
    ctx = hm.Context()
    say(f"[autotune] n={n} c64={c64}")
    plan = hm.autotune(x, 4096, ctx=ctx)
    say(f"[autotune] plan {plan}")
    assert plan["force_path"] in (1, 2) and plan["ms_per_shift"] > 0
    got = hm.sre(x, (2.0,), ctx=ctx).cpu().numpy()
    ref = hm.sre(x, (2.0,)).cpu().numpy()
    assert rel_err(got[:-1], ref[:-1]) < (2e-6 if c64 else 1e-11), (got, ref)
    assert abs(got[-1] - ref[-1]) < (1e-6 if c64 else 1e-12), (got, ref)
    if n <= 14:
        want = orc.sre_fwht(w, (2.0,))
        assert rel_err(got[:-1], want[:-1]) < TOL[c64]


@pytest.mark.parametrize("c64,n", [(True, 26), (False, 25)])
def test_maximum_sizes_sampled_rows(orc, hm, c64, n):
    """Largest supported states (complex64 n = 26: 512 MB; complex128 n = 25: 512 MB): per-row sums
    of a few X-rows (both fold cases and the a = 0 row) against the oracle, in the launch
    configuration the planner picks at that size."""
    g = np.random.default_rng(4300 + n)
    psi = (g.standard_normal(2 ** n) + 1j * g.standard_normal(2 ** n)).astype(np.complex128)
    psi /= np.linalg.norm(psi)
    x, w = gpu_state(psi, c64)
    del psi
    rows = np.array([0, 5, 2 ** (n - 1) + 3], dtype=np.int64)
    say(f"[sre max size rows] n={n} c64={c64}")
    got = hm.sre_rows(x, rows, (2.0,)).cpu().numpy()
    want = orc.sre_rows(w, rows.astype(np.uint64), (2.0,))
    assert rel_err(got, want, floor=1e-15) < (1e-5 if c64 else 1e-10), (got, want)


@pytest.mark.parametrize("n", [22, 24])
def test_long_rows_at_large_n(orc, hm, n):
    """From n = 22 the planner gives the complex64 two-pass row pass rows of up to 2^15 values, so
    that the column tiles stay 2^5 columns wide.  Raw sums over two shift ranges (the a = 0 row and
    both fold cases) against the oracle, on the default plan and with the row bits forced to 12..15
    (the split of the previous default and every long-row kernel)."""
    g = np.random.default_rng(4400 + n)
    psi = (g.standard_normal(2 ** n) + 1j * g.standard_normal(2 ** n)).astype(np.complex128)
    psi /= np.linalg.norm(psi)
    x, w = gpu_state(psi, True)
    del psi
    half = 2 ** (n - 1)
    for a0, a1 in ((0, 24), (half - 5, half + 19)):
        want = orc.sre_fwht_sums(w, (2.0,), a0, a1)
        for rb in (0, 12, 13, 14, 15):
            ctx = hm.Context()
            ctx.force_path(2)
            if rb:
                ctx.set_option(hm.OPT_ROW_BITS, rb)
            say(f"[sre long rows] n={n} shifts [{a0}, {a1}) row_bits={rb or 'default'}")
            got = hm.sre_partial(x, (2.0,), a0, a1, ctx=ctx).cpu().numpy()
            assert rel_err(got, want, floor=1e-12) < 2e-6, (rb, got, want)


@pytest.mark.parametrize("k", [1, 4, 16])
def test_clifford_t_n16_vs_golden(hm, k):
    """Random Clifford circuits with k T gates at seeded positions (n = 16), complex64 values and
    the same values widened to complex128, against FP64 oracle values stored by
    tests/golden/make_golden.py."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_golden.json")))
    want = np.array(gold[f"sre_clifford_t_n16_k{k}_seed42{k:02d}_c64"]["values"])
    v, w = S.to_c64_exact(S.clifford_t_state(16, k, seed=4200 + k))
    for t, tol in ((torch.from_numpy(v), 1e-5), (torch.from_numpy(w), 1e-10)):
        say(f"[sre clifford+T golden] k={k} dtype={t.dtype}")
        got = hm.sre(t.to(_dev()), (2.0,)).cpu().numpy()
        assert abs(got[0] - want[0]) < tol * max(1.0, abs(want[0])), (got, want)
        assert abs(got[1] - want[1]) < (1e-6 if tol > 1e-9 else 1e-12), (got, want)


def test_sharded_evaluation_n20(hm):
    """The multi-GPU plan on one GPU: the X-shifts of the N = 20 bench state split into 8 equal
    shards (one per prospective GPU), hm_sre_partial on each, the partial sums added in shard order
    (what one all-reduce would do) and finalised with hm_sre_finalize, against the single call.
    The sums differ only in FP64 grouping."""
    n, G = 20, 8
    v, _ = S.to_c64_exact(S.brickwall_haar(n, 2 * n, seed=2020))
    x = torch.from_numpy(v).to(_dev())
    q = (2.0,)
    say("[sre sharded] n=20, 8 shards")
    parts = [hm.sre_partial(x, q, r * (2 ** n // G), (r + 1) * (2 ** n // G)) for r in range(G)]
    total = parts[0].clone()
    for p in parts[1:]:
        total += p
    got = hm.sre_finalize(n, q, total).cpu().numpy()
    want = hm.sre(x, q).cpu().numpy()
    assert abs(got[0] - want[0]) < 1e-12 * abs(want[0]), (got, want)
    assert abs(got[1] - want[1]) < 1e-12, (got, want)


@pytest.mark.parametrize("c64", [False, True])
def test_two_pass_eight_renyi_indices(orc, hm, c64):
    """The largest q list (8 indices, fractional, q = 1 and large q) through the two-pass kernels'
    general-q accumulation, ragged batches, against Algorithm 2 on the CPU."""
    n = 12
    q = (0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0, 8.0)
    ctx = hm.Context()
    ctx.force_path(2)
    ctx.batch_shifts(37)
    psi = S.brickwall_haar(n, 2 * n, seed=3900)
    x, w = gpu_state(psi, c64)
    say(f"[sre two-pass 8 q] c64={c64}")
    got = hm.sre(x, q, ctx=ctx).cpu().numpy()
    want = orc.sre_fwht(w, q)
    assert rel_err(got[:-1], want[:-1]) < TOL[c64], (got, want)
    assert abs(got[-1] - want[-1]) < (1e-12 if not c64 else 2e-6)
