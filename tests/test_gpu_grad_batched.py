"""GPU parity of the batched fused forward + adjoint (hm_sre_grad_batched): each state of a batch
against the single-state entry point and the FP64 oracle gradient, through the C-ABI and through
torch.autograd over a batch of 64 parameterised RY/RZ + CZ circuits.

Tolerances: against the single-state call (the same arithmetic, other workgroup partition of the
shift sums) relative L2 <= 1e-5 for complex64 and 1e-12 for complex128; against the oracle the
single-state bounds (1e-4 / 1e-9).
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


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def batch_states(n, B, c64, seed):
    """B Gaussian states of n qubits as a (B, 2^n) GPU tensor, and the exact complex128 values."""
    rows, exact = [], []
    for i in range(B):
        psi = S.gaussian_state(n, seed=seed + i)
        if c64:
            v, w = S.to_c64_exact(psi)
        else:
            v, w = psi, psi
        rows.append(v)
        exact.append(w)
    return torch.from_numpy(np.stack(rows)).to(_dev()), exact


# (n, complex64, batch): resident sizes (one launch per 64 states, 70 = 64 + 6), and complex64
# n = 14 / complex128 n = 13, which run the two-pass kernels state after state on one workspace.
CASES = [(3, False, 2), (6, True, 5), (9, False, 7), (12, True, 64), (12, False, 9), (13, True, 70), (14, True, 3), (15, True, 3),
         (13, False, 3)]


@pytest.mark.parametrize("n,c64,B", CASES)
def test_grad_batched_vs_single_and_oracle(orc, hm, n, c64, B):
    X, exact = batch_states(n, B, c64, seed=7000 + 100 * n + B)
    for q in ((2.0, 3.0) if n <= 9 else (2.0,)):
        say(f"[grad batched] n={n} c64={c64} B={B} q={q}")
        out, G = hm.sre_grad_batched(X, q)
        torch.cuda.synchronize()
        out = out.cpu().numpy()
        G = G.cpu().numpy().astype(np.complex128)
        tol_s = 1e-5 if c64 else 1e-12
        for i in range(B):
            o1, g1 = hm.sre_grad(X[i], q)
            g1 = g1.cpu().numpy().astype(np.complex128)
            assert rel_l2(G[i], g1) < tol_s, (i, rel_l2(G[i], g1))
            np.testing.assert_allclose(out[i], o1.cpu().numpy(), rtol=tol_s, atol=tol_s)
        for i in sorted({0, B - 1}):
            want_out, want_g = orc.sre_grad_fwht(exact[i], q)
            assert rel_l2(G[i], want_g) < (1e-4 if c64 else 1e-9), (i, rel_l2(G[i], want_g))
            np.testing.assert_allclose(out[i], want_out, rtol=(1e-5 if c64 else 1e-11),
                                       atol=(1e-6 if c64 else 1e-12))


def test_grad_batched_list_input_and_identities(hm):
    """List form of the call; homogeneity Re <psi, g> = 4q / ((1 - q) ln 2) and phase invariance."""
    n, B = 10, 4
    X, _ = batch_states(n, B, True, seed=7400)
    say("[grad batched] list input n=10")
    out, gs = hm.sre_grad_batched(list(X.unbind(0)), 2.0)
    assert isinstance(gs, list) and len(gs) == B
    want = 4 * 2.0 / ((1 - 2.0) * math.log(2))
    for i in range(B):
        ip = torch.vdot(gs[i].to(torch.complex128), X[i].to(torch.complex128)).item()
        assert abs(ip.real - want) < 1e-4 * abs(want) and abs(ip.imag) < 1e-4 * abs(want), (i, ip)


def test_grad_batched_rejects_mixed_sizes(hm):
    dev = _dev()
    a = torch.zeros(1 << 4, dtype=torch.complex64, device=dev)
    b = torch.zeros(1 << 5, dtype=torch.complex64, device=dev)
    with pytest.raises(ValueError):
        hm.sre_grad_batched([a, b], 2.0)


def test_autograd_batched_circuits(orc, hm):
    """64 seeded 2-layer RY/RZ + CZ circuits at n = 12, complex64 states, one batched backward:
    angle gradients against central differences (h = 1e-6) of the FP64 oracle on sampled angles,
    and the batched M_2 against the oracle."""
    n, B = 12, 64
    dev = _dev()
    rng = np.random.default_rng(7500)
    ang0 = rng.uniform(0, 2 * math.pi, (B, 2, 2, n))
    ang = torch.tensor(ang0, dtype=torch.float64, device=dev, requires_grad=True)
    psis = torch.stack([S.ry_rz_cz_state_torch(n, ang[i]) for i in range(B)]).to(torch.complex64)
    say("[grad autograd batched] 64 circuits n=12")
    m2 = hm.SREBatched.apply(psis, 2.0)
    assert m2.shape == (B,)
    m2.sum().backward()
    got = ang.grad.cpu().numpy()
    for i in (0, B - 1):
        want = orc.sre_fwht(S.ry_rz_cz_state(n, ang0[i]), (2.0,))[0]
        assert abs(m2[i].item() - want) < 1e-5 * abs(want), (i, m2[i].item(), want)
    h = 1e-6
    for i, idx in ((0, (0, 0, 3)), (0, (1, 1, 7)), (B - 1, (1, 0, 0)), (B - 1, (0, 1, 11))):
        ap, am = ang0[i].copy(), ang0[i].copy()
        ap[idx] += h
        am[idx] -= h
        fd = (orc.sre_fwht(S.ry_rz_cz_state(n, ap), (2.0,))[0] - orc.sre_fwht(S.ry_rz_cz_state(n, am), (2.0,))[0]) / (2 * h)
        an = got[(i,) + idx]
        say(f"[grad autograd batched] state {i} angle {idx}: fd={fd:.8e} an={an:.8e}")
        # complex64 states: the FP32 forward limits the agreement to about 1e-5 relative
        assert abs(an - fd) < 1e-4 * max(1.0, abs(fd)), (i, idx, an, fd)


@pytest.mark.parametrize("n,c64", [(8, True), (13, True), (12, False), (15, True)])
def test_batch_of_one_is_the_single_call(hm, n, c64):
    """A batch of one state runs exactly the single-state launch: bitwise equal results."""
    X, _ = batch_states(n, 1, c64, seed=7600 + n)
    say(f"[grad batched] batch of one n={n} c64={c64}")
    out, G = hm.sre_grad_batched(X, 2.0)
    o1, g1 = hm.sre_grad(X[0], 2.0)
    assert np.array_equal(out[0].cpu().numpy(), o1.cpu().numpy())
    assert np.array_equal(G[0].cpu().numpy(), g1.cpu().numpy())


@pytest.mark.parametrize("c64", [True, False])
def test_grad_uneven_sizes_vs_single_calls(hm, c64):
    """hm_sre_batched_grad on a batch of uneven n (runs of equal n share a batched launch; resident and
    two-pass sizes, a two-lane run at n = 15) against one hm_sre_grad call per state."""
    ns = [8, 8, 12, 13, 13, 9, 15, 15, 6] if c64 else [8, 8, 11, 12, 13, 9, 6]
    X = [torch.from_numpy(S.gaussian_state(n, seed=7600 + i)).to(torch.complex64 if c64 else torch.complex128).cuda()
         for i, n in enumerate(ns)]
    say(f"[grad uneven] c64={c64} ns={ns}")
    out, G = hm.sre_grad_uneven(X, 2.0)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    tol = 1e-5 if c64 else 1e-12
    for i, x in enumerate(X):
        o1, g1 = hm.sre_grad(x, 2.0)
        assert rel_l2(G[i].cpu().numpy().astype(np.complex128), g1.cpu().numpy().astype(np.complex128)) < tol, i
        np.testing.assert_allclose(out[i], o1.cpu().numpy(), rtol=tol, atol=tol)
