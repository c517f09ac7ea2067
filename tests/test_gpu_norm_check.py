"""GPU checks of the optional normalisation check (HM_OPT_CHECK_NORM): unit states pass through
every entry point that takes a state, states whose squared norm is off 1 by more than the tolerance
(1e-5 complex64, 1e-12 complex128) are rejected with HM_E_NOT_NORMALIZED and leave the outputs
untouched, and deviations inside the tolerance are accepted."""
import numpy as np
import pytest

from synth import states as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HM_E_NOT_NORMALIZED = 8


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def hm():
    import paper_2601_07824_amd as m
    m.lib()
    return m


@pytest.fixture()
def ctx(hm):
    c = hm.Context()
    c.set_option(hm.OPT_CHECK_NORM, 1)
    return c


def state(n, d, c64, scale=1.0, seed=8000):
    psi = S.gaussian_state(n, d=d, seed=seed + n) * scale
    v = S.to_c64_exact(psi)[0] if c64 else psi
    return torch.from_numpy(v).to(_dev())


@pytest.mark.parametrize("c64", [False, True])
def test_unit_states_pass_every_entry(hm, ctx, c64):
    x = state(10, 2, c64)
    print(f"[norm check] unit states c64={c64}", flush=True)
    want = hm.sre(x, (2.0,)).cpu().numpy()
    np.testing.assert_array_equal(hm.sre(x, (2.0,), ctx=ctx).cpu().numpy(), want)
    hm.sre_partial(x, (2.0,), 0, 64, ctx=ctx)
    hm.sre_rows(x, [0, 3, 700], (2.0,), ctx=ctx)
    hm.sre_row_values(x, 5, ctx=ctx)
    hm.sre_grad(x, 2.0, ctx=ctx)
    hm.sre_grad_batched(torch.stack([x, x]), 2.0, ctx=ctx)
    hm.sre_batched([x, state(7, 2, c64)], (2.0,), ctx=ctx)
    hm.sre_sampled(x, n_rows=16, ctx=ctx)
    m = state(6, 3, c64)
    hm.mana(m, ctx=ctx)
    hm.mana_partial(m, 0, 9, ctx=ctx)
    torch.cuda.synchronize()


@pytest.mark.parametrize("c64", [False, True])
def test_off_norm_states_are_rejected(hm, ctx, c64):
    # squared norm off by 2e-4 (complex64 bound 1e-5) and by 2e-10 (complex128 bound 1e-12)
    scale = np.sqrt(1 + (2e-4 if c64 else 2e-10))
    x = state(9, 2, c64, scale)
    out = torch.full((2,), -7.0, dtype=torch.float64, device=_dev())
    print(f"[norm check] rejected c64={c64}", flush=True)
    for call in (lambda: hm.sre(x, (2.0,), ctx=ctx), lambda: hm.sre_grad(x, 2.0, ctx=ctx),
                 lambda: hm.sre_grad_batched(torch.stack([state(9, 2, c64), x]), 2.0, ctx=ctx),
                 lambda: hm.sre_batched([state(9, 2, c64), x], (2.0,), ctx=ctx),
                 lambda: hm.mana(state(6, 3, c64, scale), ctx=ctx)):
        with pytest.raises(hm.HmError) as e:
            call()
        assert e.value.status == HM_E_NOT_NORMALIZED, e.value
    # nothing was enqueued for the rejected calls: an output buffer passed through the C-ABI keeps
    # its contents
    L = hm.lib()
    import ctypes
    qa = (ctypes.c_double * 1)(2.0)
    ws = torch.empty(hm.workspace_size(hm.OP_SRE, 9, 1 if not c64 else 0, 1, 0, ctx), dtype=torch.uint8, device=_dev())
    st = L.hm_sre(ctx.h, ctypes.c_void_p(x.data_ptr()), 9, 0 if c64 else 1, qa, 1, ctypes.c_void_p(out.data_ptr()),
                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == HM_E_NOT_NORMALIZED
    assert torch.all(out == -7.0)


@pytest.mark.parametrize("c64", [False, True])
def test_deviation_inside_tolerance_is_accepted(hm, ctx, c64):
    scale = np.sqrt(1 + (2e-6 if c64 else 2e-13))
    x = state(9, 2, c64, scale)
    print(f"[norm check] inside tolerance c64={c64}", flush=True)
    hm.sre(x, (2.0,), ctx=ctx)
    torch.cuda.synchronize()
