"""The headline configurations against FP64 oracle values stored by tests/golden/make_golden.py
(which calls only oracle/): M_2 of the N = 20 brick-wall state (depth 40, seed 2020) -- the
benchmark's state -- with complex64 transforms and M_1, M_2, M_3 with complex128; the mana of the
N = 12 Gaussian qutrit state (seed 1212) with complex64 and complex128; and the gradient of M_2 at
N = 16 and 18 (two-layer RY/RZ + CZ circuit states) on 4096 seeded entries.

Bounds: complex64 (FP32 transforms, FP64 sums) 1e-5 relative on M and mana; complex128 1e-10.
Gradients (FP32 transforms): every sampled entry within 1e-4 of the largest gradient entry, and
relative L2 error over the sample <= 1e-4; with complex128 (FP64 transforms, N = 18) 1e-9.  A case whose golden value has not been generated yet
is skipped with that reason.
"""
import json
import math
import os

import numpy as np
import pytest

from synth import states as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.join(os.path.dirname(__file__), "golden")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def hm():
    import paper_2601_07824_amd as m
    m.lib()
    return m


def gold(key, fname="oracle_golden.json"):
    path = os.path.join(HERE, fname)
    data = json.load(open(path)) if os.path.exists(path) else {}
    if key not in data:
        pytest.skip(f"golden value {key} not generated (tests/golden/make_golden.py)")
    return data[key]


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("c64", [True, False])
def test_sre_n20_bench_state(hm, c64):
    key = "sre_brickwall_n20_d40_seed2020_" + ("c64" if c64 else "c128")
    g = gold(key)
    psi = S.brickwall_haar(20, 40, seed=2020)
    x = torch.from_numpy(S.to_c64_exact(psi)[0] if c64 else psi).to(_dev())
    got = hm.sre(x, tuple(g["q"])).cpu().numpy()
    want = np.asarray(g["values"])
    err = np.abs(got[:-1] - want[:-1]) / np.abs(want[:-1])
    say(f"[headline sre n20] {key} gpu={got} oracle={want} rel_err={err}")
    assert np.all(err <= (1e-5 if c64 else 1e-10)), (got, want)
    assert abs(got[-1] - want[-1]) <= (1e-5 if c64 else 1e-12)


@pytest.mark.parametrize("c64", [True, False])
def test_mana_n12_bench_state(hm, c64):
    key = "mana_gauss_n12_seed1212_" + ("c64" if c64 else "c128")
    g = gold(key)
    psi = S.gaussian_state(12, d=3, seed=1212)
    x = torch.from_numpy(S.to_c64_exact(psi)[0] if c64 else psi).to(_dev())
    got = hm.mana(x).cpu().numpy()
    want = np.asarray(g["values"])
    err = abs(got[0] - want[0]) / abs(want[0])
    say(f"[headline mana n12] {key} gpu={got} oracle={want} rel_err={err:.3e}")
    assert err <= (1e-5 if c64 else 1e-10), (got, want)
    np.testing.assert_allclose(got[1:], want[1:], atol=(1e-5 if c64 else 1e-10))


@pytest.mark.parametrize("n,c128", [(16, False), (18, False), (18, True)])
def test_grad_circuit_states(hm, n, c128):
    """The stored FP64 oracle gradient of the complex64-exact circuit state, against the complex64
    kernels (FP32 transforms) and, at N = 18, the complex128 kernels on the same values widened."""
    key = f"grad_ryrzcz_n{n}_seed{4000 + n}_c64"
    g = gold(key, "grad_golden.json")
    ang = np.random.default_rng(4000 + n).uniform(0, 2 * math.pi, (2, 2, n))
    v64, w = S.to_c64_exact(S.ry_rz_cz_state(n, ang))
    x = torch.from_numpy(w if c128 else v64).to(_dev())
    out, grad = hm.sre_grad(x, g["q"])
    out = out.cpu().numpy()
    idx = np.asarray(g["idx"], dtype=np.int64)
    got = grad.cpu().numpy()[idx].astype(np.complex128)
    want = np.asarray(g["g_re"]) + 1j * np.asarray(g["g_im"])
    d = np.abs(got - want)
    rel_l2 = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    say(f"[headline grad n{n}] M={out[0]:.9f} oracle={g['values'][0]:.9f} max|dg|/|g|inf={d.max() / g['norm_inf']:.2e} "
        f"rel_l2={rel_l2:.2e} |g|_2 gpu={float(torch.linalg.vector_norm(grad).item()):.9f} oracle={g['norm2']:.9f}")
    tol = 1e-9 if c128 else 1e-4
    assert abs(out[0] - g["values"][0]) <= (1e-11 if c128 else 1e-5) * abs(g["values"][0])
    assert np.all(d <= tol * g["norm_inf"]), d.max()
    assert rel_l2 <= tol
    assert abs(float(torch.linalg.vector_norm(grad).item()) - g["norm2"]) <= tol * g["norm2"]
