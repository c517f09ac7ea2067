"""Autotuners of the mana, gradient and batched plans: after tuning, the calls on the tuned handle
give the results of the untuned calls (up to the grouping of the FP64 sums), and hm_tune_clear
forgets the choices."""
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


@pytest.mark.parametrize("n,c64", [(10, True), (11, False)])
def test_autotune_mana(hm, n, c64):
    psi = S.gaussian_state(n, d=3, seed=9900 + n)
    x = torch.from_numpy(S.to_c64_exact(psi)[0] if c64 else psi).to(_dev())
    print(f"[autotune mana] n={n} c64={c64}", flush=True)
    ref = hm.mana(x).cpu().numpy()
    ctx = hm.Context()
    hm.autotune_mana(x, 2048, ctx=ctx)
    got = hm.mana(x, ctx=ctx).cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)
    hm.lib().hm_tune_clear(ctx.h)
    np.testing.assert_allclose(hm.mana(x, ctx=ctx).cpu().numpy(), ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("n", [12, 13])
def test_autotune_grad(hm, n):
    x = torch.from_numpy(S.to_c64_exact(S.gaussian_state(n, seed=9920 + n))[0]).to(_dev())
    print(f"[autotune grad] n={n}", flush=True)
    o_ref, g_ref = hm.sre_grad(x, 2.0)
    ctx = hm.Context()
    hm.autotune_grad(x, 2.0, ctx=ctx)
    o, g = hm.sre_grad(x, 2.0, ctx=ctx)
    assert abs(o[0].item() - o_ref[0].item()) <= 1e-5 * abs(o_ref[0].item())
    rel = (torch.linalg.vector_norm(g - g_ref) / torch.linalg.vector_norm(g_ref)).item()
    assert rel <= 1e-4, rel


def test_autotune_batched(hm):
    ns = [12, 8, 15, 10, 13, 9]
    xs = [torch.from_numpy(S.to_c64_exact(S.gaussian_state(n, seed=9940 + i))[0]).to(_dev()) for i, n in enumerate(ns)]
    print("[autotune batched]", flush=True)
    ref = hm.sre_batched(xs, (2.0,)).cpu().numpy()
    ctx = hm.Context()
    hm.autotune_batched(xs, ctx=ctx)
    got = hm.sre_batched(xs, (2.0,), ctx=ctx).cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=1e-7)
