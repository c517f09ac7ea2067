"""GPU parity of the qutrit mana kernels (Algorithm 4) against the FP64 oracle, through the C-ABI.

Tolerances: complex128 <= 1e-10 relative on mana (absolute when 0) and on the two normalisation
diagnostics; complex64 <= 1e-5.  Large N use properties that hold at any size: stabilizer states
have mana 0 (discrete Hudson theorem), mana is additive on products, sum W = 1, 3^N sum W^2 = 1.
"""
import json
import math
import os

import numpy as np
import pytest

from synth import states as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_golden.json")


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
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_small_sizes_vs_oracle(orc, hm, n, c64):
    psi = S.gaussian_state(n, d=3, seed=5000 + n)
    x, w = gpu_state(psi, c64)
    say(f"[mana] n={n} c64={c64}")
    got = hm.mana(x).cpu().numpy()
    want = orc.mana_direct(w) if n <= 5 else orc.mana_fft(w)
    assert abs(got[0] - want[0]) <= TOL[c64] * max(1.0, abs(want[0])), (got, want)
    np.testing.assert_allclose(got[1:], want[1:], atol=TOL[c64] * 10)


@pytest.mark.parametrize("c64", [False, True])
def test_two_pass_n9_vs_oracle(orc, hm, c64):
    n = 9
    psi = S.brickwall_haar(n, 4, seed=5009, d=3)
    x, w = gpu_state(psi, c64)
    say(f"[mana two-pass] n={n} c64={c64}")
    got = hm.mana(x).cpu().numpy()
    want = orc.mana_fft(w)
    assert abs(got[0] - want[0]) <= TOL[c64] * max(1.0, abs(want[0])), (got, want)


@pytest.mark.parametrize("streams", [1, 2])
@pytest.mark.parametrize("batch", [7, 64])
def test_two_pass_batches(orc, hm, batch, streams):
    """Launch batches of 7 shifts (rounded up to 4 shift pairs; ragged last launch) and of 64 at
    n = 10, complex128, on one stream or alternating over two."""
    n = 10
    psi = S.gaussian_state(n, d=3, seed=5020)
    x, w = gpu_state(psi, False)
    ctx = hm.Context()
    ctx.batch_shifts(batch)
    ctx.set_option(hm.OPT_STREAMS, streams)
    say(f"[mana batch] n={n} batch={batch} streams={streams}")
    got = hm.mana(x, ctx=ctx).cpu().numpy()
    want = orc.mana_fft(w)
    assert abs(got[0] - want[0]) <= 1e-10 * max(1.0, abs(want[0])), (got, want)


@pytest.mark.parametrize("c64", [False, True])
def test_one_and_two_streams_agree_at_n12(hm, c64):
    """Full size: the two-stream plan and the one-stream plan (default) differ only in how the FP64
    partial sums are grouped."""
    x, _ = gpu_state(S.gaussian_state(12, d=3, seed=5012), c64)
    two = hm.Context()
    two.set_option(hm.OPT_STREAMS, 2)
    say(f"[mana streams] n=12 c64={c64}")
    a = hm.mana(x).cpu().numpy()
    b = hm.mana(x, ctx=two).cpu().numpy()
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=0)
    assert np.array_equal(b, hm.mana(x, ctx=two).cpu().numpy())  # deterministic


def test_golden_values(hm):
    gold = json.load(open(GOLDEN))
    for key, n, c64, seed in (("mana_gauss_n8_seed5008_c128", 8, False, 5008), ("mana_gauss_n10_seed5010_c64", 10, True, 5010)):
        want = gold[key]["values"]
        x, _ = gpu_state(S.gaussian_state(n, d=3, seed=seed), c64)
        say(f"[mana golden] {key}")
        got = hm.mana(x).cpu().numpy()
        assert abs(got[0] - want[0]) <= TOL[c64] * max(1.0, abs(want[0])), (key, got, want)


@pytest.mark.parametrize("c64", [False, True])
def test_partial_ranges(orc, hm, c64):
    n = 5
    psi = S.gaussian_state(n, d=3, seed=5100)
    x, w = gpu_state(psi, c64)
    D = 3 ** n
    cuts = [0, 1, 2, 3, 40, 121, 122, D]
    for a0, a1 in zip(cuts[:-1], cuts[1:]):
        say(f"[mana partial] [{a0},{a1}) c64={c64}")
        got = hm.mana_partial(x, a0, a1).cpu().numpy()
        want = orc.mana_fft_sums(w, a0, a1)
        np.testing.assert_allclose(got, want, rtol=(1e-11 if not c64 else 2e-6), atol=1e-9)
    assert np.all(hm.mana_partial(x, 7, 7).cpu().numpy() == 0)


@pytest.mark.parametrize("n", [6, 10, 12])
def test_stabilizer_states_zero(hm, n):
    """Hudson: stabilizer states have W >= 0, so mana = 0.  With FP32 transforms the 9^N - 3^N
    Wigner values that are exactly zero come out as rounding noise, and sum |W| turns that noise into
    a one-sided excess (about 1.5e-5 at N = 10 and 4.5e-5 at N = 12, growing like sqrt(9^N)); the
    complex64 bound is therefore an absolute 1e-4 for N <= 12.  Complex128 stays at 1e-9."""
    for c64 in (False, True):
        psi = S.random_qutrit_clifford_state(n, seed=5200 + n, layers=2 * n)
        x, _ = gpu_state(psi, c64)
        say(f"[mana stabilizer] n={n} c64={c64}")
        got = hm.mana(x).cpu().numpy()
        tol = 1e-9 if not c64 else 1e-4
        assert 0 <= got[0] < tol or abs(got[0]) < 1e-12, got
        tol_n = 1e-9 if not c64 else 1e-5
        assert abs(got[1] - 1) < tol_n and abs(got[2] - 1) < tol_n, got


@pytest.mark.parametrize("n", [9, 12])
def test_additivity_at_full_size(orc, hm, n):
    """Mana of a product equals the sum of single-qutrit manas (computed by the direct oracle)."""
    psi, singles = S.random_product_state(n, d=3, seed=5300 + n)
    want = sum(float(orc.mana_direct(s)[0]) for s in singles)
    for c64 in (False, True):
        x, _ = gpu_state(psi, c64)
        say(f"[mana product] n={n} c64={c64}")
        got = hm.mana(x).cpu().numpy()
        assert abs(got[0] - want) <= (1e-9 if not c64 else 1e-5) * max(1.0, want), (got, want)


def test_strange_state_products(hm):
    """(|1> - |2>)/sqrt2 has mana log2(5/3); k copies next to |0>s give k log2(5/3)."""
    strange = np.array([0, 1, -1], dtype=np.complex128) / math.sqrt(2)
    zero = np.array([1, 0, 0], dtype=np.complex128)
    for n, k in ((4, 2), (11, 3)):
        psi = S.product_state([strange] * k + [zero] * (n - k))
        x, _ = gpu_state(psi, False)
        say(f"[mana strange] n={n} k={k}")
        got = hm.mana(x).cpu().numpy()
        assert abs(got[0] - k * math.log2(5 / 3)) < 1e-10


def test_normalisation_diagnostics_full_size(hm):
    n = 12
    x, _ = gpu_state(S.gaussian_state(n, d=3, seed=5400), True)
    say("[mana diag] n=12 c64")
    got = hm.mana(x).cpu().numpy()
    assert abs(got[1] - 1) < 1e-5 and abs(got[2] - 1) < 1e-5, got
    assert 0 < got[0] < n * math.log2(3)


def test_determinism(hm):
    x, _ = gpu_state(S.gaussian_state(10, d=3, seed=5500), True)
    say("[mana determinism] n=10")
    a = hm.mana(x).cpu().numpy()
    b = hm.mana(x).cpu().numpy()
    assert np.array_equal(a, b)


def test_maximum_size_partial(orc, hm):
    """n = 16 qutrits (3^16 complex64 values, 344 MB): sums over a few shift pairs (a0 = 0 and an
    interior range, both ragged) against the oracle."""
    n = 16
    g = np.random.default_rng(5600)
    psi = (g.standard_normal(3 ** n) + 1j * g.standard_normal(3 ** n)).astype(np.complex128)
    psi /= np.linalg.norm(psi)
    x, w = gpu_state(psi, True)
    del psi
    for a0, a1 in ((0, 3), (3 ** 15 + 1, 3 ** 15 + 4)):
        say(f"[mana max size] n={n} [{a0},{a1})")
        got = hm.mana_partial(x, a0, a1).cpu().numpy()
        want = orc.mana_fft_sums(w, a0, a1)
        np.testing.assert_allclose(got, want, rtol=2e-5, atol=1e-6)


@pytest.mark.parametrize("n", [13, 14, 15, 16])
def test_c128_large_sizes_partial(orc, hm, n):
    """complex128 two-pass tiles up to n = 16 (rows and columns of 3^8 at n = 15, 16): sums over two
    ragged shift ranges against the oracle (full evaluations there take minutes to hours)."""
    g = np.random.default_rng(5700 + n)
    psi = (g.standard_normal(3 ** n) + 1j * g.standard_normal(3 ** n)).astype(np.complex128)
    psi /= np.linalg.norm(psi)
    x = torch.from_numpy(psi).to(_dev())
    for a0, a1 in ((0, 3), (3 ** (n - 1) + 1, 3 ** (n - 1) + 4)):
        say(f"[mana c128 large] n={n} [{a0},{a1})")
        got = hm.mana_partial(x, a0, a1).cpu().numpy()
        want = orc.mana_fft_sums(psi, a0, a1)
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("c64", [False, True])
@pytest.mark.parametrize("n", [9, 10, 11, 12, 13])
def test_row_tiles_ragged_batches(orc, hm, n, c64):
    """Every two-pass row-tile shape (rows of 3^4..3^7 values, 1 to 27 rows per tile) with launch
    batches of 5 shifts (3 pairs, the last launch ragged) over an odd shift range, against the
    oracle's sums over the same range."""
    psi = S.gaussian_state(n, d=3, seed=5800 + n)
    x, w = gpu_state(psi, c64)
    ctx = hm.Context()
    ctx.batch_shifts(5)
    a0, a1 = 3 ** n // 2 - 7, 3 ** n // 2 + 6
    say(f"[mana row tiles] n={n} c64={c64} [{a0},{a1})")
    got = hm.mana_partial(x, a0, a1, ctx=ctx).cpu().numpy()
    want = orc.mana_fft_sums(w, a0, a1)
    np.testing.assert_allclose(got, want, rtol=(1e-10 if not c64 else 2e-6), atol=1e-9)
