"""hm_sre_noalloc (the SRE entry point that allocates nothing) against hm_sre through the C-ABI.

Both run the same kernels and the same fixed-order FP64 reduction, so the results must agree bit for
bit; each call is also checked against the FP64 oracle (1e-5 relative on complex64 inputs, 1e-10 on
complex128).  Two calls in a row share the library's scratch array; the second is smaller, so stale
per-shift sums from the first would show up in its totals.
"""
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


def _state(psi, c64):
    if c64:
        v, w = S.to_c64_exact(psi)
        return torch.from_numpy(v).to(_dev()), w
    return torch.from_numpy(psi).to(_dev()), psi


def _rel(got, want):
    got, want = np.asarray(got, dtype=float), np.asarray(want, dtype=float)
    return float(np.max(np.abs(got - want) / np.maximum(np.abs(want), 1.0)))


def test_noalloc_equals_sre_two_calls_second_smaller(orc, hm):
    qs = (1.0, 2.0, 3.0)
    cases = [(14, True, 7014), (10, False, 7010)]  # second call: fewer shifts, other dtype
    for n, c64, seed in cases:
        print(f"noalloc: n={n} c64={c64} seed={seed} q={qs}", flush=True)
        x, w = _state(S.gaussian_state(n, seed=seed), c64)
        got = hm.sre_noalloc(x, qs).cpu().numpy()
        ref = hm.sre(x, qs).cpu().numpy()
        want = orc.sre_fwht(w, qs)
        print(f"  noalloc={got} sre={ref} oracle={want}", flush=True)
        assert np.array_equal(got, ref), (got, ref)
        assert _rel(got, want) <= (1e-5 if c64 else 1e-10)


def test_noalloc_largest_scratch_use_and_preallocated_out(orc, hm):
    """n = 16 complex64 with eight Renyi indices fills the whole scratch array (2^16 x 9 doubles);
    then n = 8 into a caller-provided output."""
    qs = (0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0, 8.0)
    print("noalloc: n=16 c64 seed=7016 eight q", flush=True)
    x, _ = _state(S.brickwall_haar(16, 32, seed=7016), True)
    got = hm.sre_noalloc(x, qs).cpu().numpy()
    ref = hm.sre(x, qs).cpu().numpy()
    assert np.array_equal(got, ref), (got, ref)
    print("noalloc: n=8 c128 seed=7008 into a preallocated out", flush=True)
    y, w = _state(S.gaussian_state(8, seed=7008), False)
    out = torch.full((9,), float("nan"), dtype=torch.float64, device=_dev())
    r = hm.sre_noalloc(y, qs, out=out)
    assert r.data_ptr() == out.data_ptr()
    got = out.cpu().numpy()
    assert np.array_equal(got, hm.sre(y, qs).cpu().numpy())
    assert _rel(got, orc.sre_direct(w, qs)) <= 1e-10


def test_noalloc_rejects_two_pass_sizes(hm):
    x = torch.zeros(1 << 17, dtype=torch.complex64, device=_dev())
    with pytest.raises(hm.HmError) as e:
        hm.sre_noalloc(x, (2.0,))
    assert e.value.status == 3  # HM_E_SIZE
    ctx = hm.Context()
    ctx.force_path(2)
    x = torch.zeros(1 << 14, dtype=torch.complex64, device=_dev())
    with pytest.raises(hm.HmError) as e:
        hm.sre_noalloc(x, (2.0,), ctx=ctx)
    assert e.value.status == 3
