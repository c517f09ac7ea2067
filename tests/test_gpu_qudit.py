"""hm_mana_qudit (pure-state mana of qudits of odd prime dimension d = 3, 5, 7) against the FP64
oracle (oracle/qudit.py, pinned in test_oracle_qudit.py) on the same seeded complex64-exact or
complex128 inputs, at every size the kernel holds (n = 1 .. 9/6/5 for d = 3/5/7 complex64,
8/5/4 complex128; odd d^n gives a ragged last shift pair), stabilizer states (mana 0 within the
FP32 bound), the d = 3 path against hm_mana, determinism, and the host-side errors.

Bounds: complex128 1e-10 absolute on mana and the diagnostics; complex64 (FP32 transforms, FP64
sums) 2e-5 absolute on mana (the one-sided |.| noise on exact zeros grows with d^n) and 1e-5 on the
diagnostics."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import qudit as Q  # noqa: E402
from synth import states as S  # noqa: E402

@pytest.fixture(scope="module")
def hm():
    import paper_2601_07824_amd as m
    m.lib()
    return m


NMAX = {(3, False): 9, (5, False): 6, (7, False): 5, (3, True): 8, (5, True): 5, (7, True): 4}


def _dev(psi, c128):
    if c128:
        return torch.from_numpy(psi).cuda(), psi
    x = psi.astype(np.complex64)
    return torch.from_numpy(x).cuda(), x.astype(np.complex128)


def _oracle(psi, d):
    # the sums of Algorithm 4 with 3 -> d; large sizes only where it finishes in seconds
    return Q.mana_fft(psi, d)


def _cases():
    out = []
    for (d, c128), nmax in NMAX.items():
        for n in range(1, nmax + 1):
            if d ** (2 * n) <= 10 ** 7:  # oracle in seconds
                out.append((d, n, c128))
    return out


@pytest.mark.parametrize("d,n,c128", _cases())
def test_against_oracle(hm, d, n, c128):
    psi = S.gaussian_state(n, d, seed=1000 * d + n)
    x, xo = _dev(psi, c128)
    got = hm.mana_qudit(x, d).cpu().numpy()
    want = _oracle(xo, d)
    tol = 1e-10 if c128 else 2e-5
    print(f"[qudit] d={d} n={n} {'c128' if c128 else 'c64'} gpu={got} oracle={want}", flush=True)
    assert abs(got[0] - want[0]) <= tol * max(1.0, abs(want[0])), (got, want)
    np.testing.assert_allclose(got[1:], want[1:], atol=(1e-10 if c128 else 1e-5))


@pytest.mark.parametrize("d,c128", [(3, False), (5, False), (7, False), (3, True), (5, True), (7, True)])
def test_largest_size_properties(hm, d, c128):
    """The largest n of each kernel: sum W = 1 and d^n sum W^2 = 1 for a normalised pure state,
    mana of a product of single-qudit magic states is additive, stabilizer states have mana 0."""
    n = NMAX[(d, c128)]
    dt = torch.complex128 if c128 else torch.complex64
    psi = torch.from_numpy(S.gaussian_state(n, d, seed=77)).to(dt).cuda()
    psi = psi / torch.linalg.vector_norm(psi)
    got = hm.mana_qudit(psi, d).cpu().numpy()
    tol = 1e-10 if c128 else 1e-5
    assert abs(got[1] - 1) < tol and abs(got[2] - 1) < tol, got
    g = S.qudit_clifford_gates(d)
    one = (S.qudit_cubic_phase(d) if d > 3 else np.diag(np.exp(2j * np.pi * np.arange(3) ** 3 / 9))) @ g["F"][:, 0]
    m1 = Q.mana_fft(one, d)[0]
    prod = torch.from_numpy(S.product_state([one] * n)).to(dt).cuda()
    mp = hm.mana_qudit(prod, d).cpu().numpy()[0]
    assert abs(mp - n * m1) <= (1e-10 if c128 else 5e-5) * max(1.0, n * m1), (mp, n * m1)
    st = torch.from_numpy(S.random_qudit_clifford_state(n, d, seed=5)).to(dt).cuda()
    ms = hm.mana_qudit(st, d).cpu().numpy()
    print(f"[qudit max] d={d} n={n} stabilizer mana={ms[0]:.3e} product={mp:.8f} ({n * m1:.8f})", flush=True)
    assert 0 <= ms[0] < (1e-10 if c128 else 2e-4) or abs(ms[0]) < 1e-12, ms


@pytest.mark.parametrize("n,c128", [(4, True), (7, True), (9, False)])
def test_d3_equals_hm_mana(hm, n, c128):
    psi = torch.from_numpy(S.gaussian_state(n, 3, seed=9 + n)).to(torch.complex128 if c128 else torch.complex64).cuda()
    a = hm.mana_qudit(psi, 3).cpu().numpy()
    b = hm.mana(psi).cpu().numpy()
    np.testing.assert_allclose(a, b, rtol=(1e-12 if c128 else 0), atol=(1e-12 if c128 else 2e-5))


def test_deterministic(hm):
    psi = torch.from_numpy(S.gaussian_state(5, 5, seed=3).astype(np.complex64)).cuda()
    a = hm.mana_qudit(psi, 5).cpu().numpy()
    b = hm.mana_qudit(psi, 5).cpu().numpy()
    assert np.array_equal(a, b)


def test_errors(hm):
    psi = torch.zeros(5 ** 7, dtype=torch.complex64, device="cuda")
    with pytest.raises(hm.HmError):
        hm.mana_qudit(psi, 5)  # n = 7 > 6
    with pytest.raises(ValueError):
        hm.mana_qudit(torch.zeros(4 ** 3, dtype=torch.complex64, device="cuda"), 4)
    with pytest.raises(ValueError):
        hm.mana_qudit(torch.zeros(26, dtype=torch.complex64, device="cuda"), 5)
