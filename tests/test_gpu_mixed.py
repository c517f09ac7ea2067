"""GPU mana of mixed qutrit states (hm_mana_mixed) and reduced density matrices (hm_reduced_density)
against the FP64 oracle (oracle/mixed.py: the paper's fast transform, itself pinned to the
definition).  Bounds: complex128 1e-10 relative on mana (absolute when 0) and on Tr rho, Tr rho^2;
complex64 1e-5."""
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


TOL = {False: 1e-10, True: 1e-5}


def on_gpu(a, c64):
    a64 = a.astype(np.complex64) if c64 else a
    return torch.from_numpy(np.ascontiguousarray(a64)).to(_dev()), a64.astype(np.complex128)


@pytest.mark.parametrize("c64", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_random_mixed_states_vs_oracle(hm, n, c64):
    from oracle import mixed
    for rank, seed in ((None, 9700 + n), (2, 9720 + n)):
        rho, w = on_gpu(S.random_density(n, rank=rank, seed=seed), c64)
        print(f"[mixed] n={n} rank={rank} c64={c64}", flush=True)
        got = hm.mana_mixed(rho).cpu().numpy()
        want = mixed.mana_mixed_alg6(w)
        assert abs(got[0] - want[0]) <= TOL[c64] * max(1.0, abs(want[0])), (got, want)
        np.testing.assert_allclose(got[1:], want[1:], rtol=TOL[c64], atol=TOL[c64])


@pytest.mark.parametrize("n", [6, 8])
def test_pure_density_equals_pure_state_mana(hm, n):
    psi = S.gaussian_state(n, d=3, seed=9740 + n)
    x = torch.from_numpy(psi).to(_dev())
    rho = torch.outer(x, x.conj()).contiguous()
    print(f"[mixed pure] n={n}", flush=True)
    got = hm.mana_mixed(rho).cpu().numpy()
    want = hm.mana(x).cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)


def test_maximally_mixed(hm):
    n = 6
    D = 3 ** n
    rho = (torch.eye(D, dtype=torch.complex128, device=_dev()) / D).contiguous()
    got = hm.mana_mixed(rho).cpu().numpy()
    np.testing.assert_allclose(got, [0.0, 1.0, 1.0 / D], atol=1e-13)


@pytest.mark.parametrize("c64", [False, True])
def test_reduced_density_and_subsystem_mana(hm, c64):
    """Brick-wall qutrit state (N = 10, depth 3); rho_A on 1, 4 and 7 qutrits against the partial
    trace of the oracle, and the mana of rho_A (7 qutrits) against the oracle's fast transform."""
    from oracle import mixed
    n = 10
    psi = S.brickwall_haar(n, 3, seed=9750, d=3)
    x, w = on_gpu(psi, c64)
    for n_a in (1, 4, 7):
        print(f"[reduced density] n={n} n_a={n_a} c64={c64}", flush=True)
        rho = hm.reduced_density_matrix(x, n_a)
        want = mixed.reduced_density(w, n_a)
        np.testing.assert_allclose(rho.cpu().numpy(), want, atol=(1e-14 if not c64 else 1e-7))
    got = hm.mana_mixed(rho).cpu().numpy()
    want = mixed.mana_mixed_alg6(rho.cpu().numpy().astype(np.complex128))
    assert abs(got[0] - want[0]) <= TOL[c64] * max(1.0, abs(want[0])), (got, want)


def test_largest_subsystem_n_a_10(hm):
    """N_A = 10 (9^10 complex64 values, 28 GB), the paper's largest subsystem: Tr rho = 1 and the
    purity against sum |rho_ij|^2, mana between 0 and the bound log2(3^N_A) / 2."""
    n, n_a = 11, 10
    psi = S.brickwall_haar(n, 3, seed=9760, d=3)
    x = torch.from_numpy(psi.astype(np.complex64)).to(_dev())
    print("[mixed max] n_a=10 c64", flush=True)
    rho = hm.reduced_density_matrix(x, n_a)
    got = hm.mana_mixed(rho).cpu().numpy()
    purity = float(torch.sum(torch.abs(rho.to(torch.complex64)) ** 2, dtype=torch.float64).item())
    del rho
    print(f"[mixed max] mana={got[0]:.6f} tr={got[1]:.8f} purity={got[2]:.6e} (direct {purity:.6e})", flush=True)
    assert abs(got[1] - 1.0) < 1e-5
    assert abs(got[2] - purity) < 1e-5 * purity
    assert 0.0 < got[0] < n_a * math.log2(3) / 2 + 1e-6
