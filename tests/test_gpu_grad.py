"""GPU parity of the fused forward + adjoint SRE kernel (dM_q/dpsi) against the FP64 oracle gradients,
central finite differences and the homogeneity / phase-invariance identities, through the C-ABI and
through torch.autograd (including a parameterised RY/RZ + CZ circuit).

Tolerances: complex128 relative L2 <= 1e-9; complex64 (FP32 transforms, FP32 accumulation of the
per-workgroup gradient partials, FP64 across workgroups) relative L2 <= 1e-4.
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


def gpu_state(psi, c64):
    if c64:
        v, w = S.to_c64_exact(psi)
        return torch.from_numpy(v).to(_dev()), w
    return torch.from_numpy(psi).to(_dev()), psi


@pytest.mark.parametrize("c64", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 10])
def test_grad_vs_direct_oracle(orc, hm, n, c64):
    psi = S.gaussian_state(n, seed=6000 + n)
    x, w = gpu_state(psi, c64)
    for q in (2.0, 3.0):
        say(f"[grad] n={n} c64={c64} q={q}")
        out, g = hm.sre_grad(x, q)
        want_out, want_g = (orc.sre_grad_direct(w, q) if n <= 7 else orc.sre_grad_fwht(w, q))
        got_g = g.cpu().numpy().astype(np.complex128)
        tol = 1e-4 if c64 else 1e-9
        assert rel_l2(got_g, want_g) < tol, (n, q, rel_l2(got_g, want_g))
        np.testing.assert_allclose(out.cpu().numpy(), want_out, rtol=(1e-5 if c64 else 1e-11), atol=1e-6 if c64 else 1e-12)


@pytest.mark.parametrize("c64,n", [(False, 11), (False, 12), (True, 12), (True, 13)])
def test_grad_largest_resident_vs_fwht_oracle(orc, hm, n, c64):
    psi = S.ry_rz_cz_state(n, np.random.default_rng(6100 + n).uniform(0, 2 * math.pi, (2, 2, n)))
    x, w = gpu_state(psi, c64)
    say(f"[grad resident max] n={n} c64={c64}")
    out, g = hm.sre_grad(x, 2.0)
    want_out, want_g = orc.sre_grad_fwht(w, 2.0)
    assert rel_l2(g.cpu().numpy().astype(np.complex128), want_g) < (1e-4 if c64 else 1e-9)


def test_grad_central_differences(hm):
    """h = 1e-6 central differences of the FP64 GPU forward on sampled coordinates (Re and Im)."""
    n = 9
    psi = S.gaussian_state(n, seed=6200)
    x = torch.from_numpy(psi).to(_dev())
    _, g = hm.sre_grad(x, 2.0)
    g = g.cpu().numpy()
    h = 1e-6
    for y in np.random.default_rng(6201).choice(2 ** n, 16, replace=False):
        for unit in (1.0, 1j):
            e = np.zeros_like(psi)
            e[y] = unit * h
            say(f"[grad fd] y={y} unit={unit}")
            mp = hm.sre(torch.from_numpy(psi + e).to(_dev()), (2.0,))[0].item()
            mm = hm.sre(torch.from_numpy(psi - e).to(_dev()), (2.0,))[0].item()
            fd = (mp - mm) / (2 * h)
            an = g[y].real if unit == 1.0 else g[y].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (y, unit, fd, an)


@pytest.mark.parametrize("c64", [False, True])
def test_homogeneity_and_phase_invariance(hm, c64):
    n = 12
    x, _ = gpu_state(S.gaussian_state(n, seed=6300), c64)
    say(f"[grad identities] n={n} c64={c64}")
    _, g = hm.sre_grad(x, 2.0)
    ip = torch.vdot(g.to(torch.complex128), x.to(torch.complex128)).item()
    want = 4 * 2.0 / ((1 - 2.0) * math.log(2))  # -8 / ln 2
    tol = 1e-4 if c64 else 1e-9
    assert abs(ip.real - want) < tol * abs(want) and abs(ip.imag) < tol * abs(want), ip


def test_autograd_through_circuit(orc, hm):
    """d M_2(psi(theta)) / d theta via torch.autograd + the library adjoint, vs FD on the angles."""
    n = 8
    dev = _dev()
    ang0 = np.random.default_rng(6400).uniform(0, 2 * math.pi, (2, 2, n))
    ang = torch.tensor(ang0, dtype=torch.float64, device=dev, requires_grad=True)
    psi = S.ry_rz_cz_state_torch(n, ang)
    say("[grad autograd] circuit n=8")
    m2 = hm.SRE.apply(psi, 2.0)
    m2.backward()
    got = ang.grad.cpu().numpy()
    h = 1e-6
    fd = np.zeros_like(ang0)
    for idx in np.ndindex(ang0.shape):
        ap, am = ang0.copy(), ang0.copy()
        ap[idx] += h
        am[idx] -= h
        fp = orc.sre_fwht(S.ry_rz_cz_state(n, ap), (2.0,))[0]
        fm = orc.sre_fwht(S.ry_rz_cz_state(n, am), (2.0,))[0]
        fd[idx] = (fp - fm) / (2 * h)
    assert np.max(np.abs(got - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd))), np.max(np.abs(got - fd))
    assert abs(m2.item() - orc.sre_fwht(S.ry_rz_cz_state(n, ang0), (2.0,))[0]) < 1e-10


def test_grad_determinism(hm):
    x, _ = gpu_state(S.gaussian_state(11, seed=6500), True)
    say("[grad determinism]")
    a = hm.sre_grad(x, 2.0)[1].cpu().numpy()
    b = hm.sre_grad(x, 2.0)[1].cpu().numpy()
    assert np.array_equal(a, b)


# ---- two-pass gradient (row pass, adjoint column pass, backward row pass, accumulation) ----------
@pytest.mark.parametrize("batch", [96, 0, 64])
@pytest.mark.parametrize("c64,n,forced", [(False, 12, True), (True, 12, True), (True, 13, True), (False, 13, False),
                                          (True, 14, False), (False, 14, False)])
def test_grad_two_pass_vs_fwht_oracle(orc, hm, c64, n, forced, batch):
    """batch 96: unaligned batches (backward row pass and accumulation as separate kernels, last batch
    ragged); default batches (up to n = 15 large batches through the separate kernels); batch 64
    (aligned, at most 2^nl shifts: the fused backward-row + accumulation kernel for every batch after
    the first, the default from n = 16 on)."""
    psi = S.ry_rz_cz_state(n, np.random.default_rng(6600 + n).uniform(0, 2 * math.pi, (2, 2, n)))
    x, w = gpu_state(psi, c64)
    ctx = hm.Context()
    if forced:
        ctx.force_path(2)
    if batch:
        ctx.batch_shifts(batch)
    for q in ((2.0, 3.0) if n <= 13 else (2.0,)):
        say(f"[grad two-pass] n={n} c64={c64} forced={forced} batch={batch} q={q}")
        out, g = hm.sre_grad(x, q, ctx=ctx)
        want_out, want_g = orc.sre_grad_fwht(w, q)
        err = rel_l2(g.cpu().numpy().astype(np.complex128), want_g)
        assert err < (1e-4 if c64 else 1e-9), (n, q, err)
        np.testing.assert_allclose(out.cpu().numpy(), want_out, rtol=(1e-5 if c64 else 1e-11),
                                   atol=1e-6 if c64 else 1e-12)


@pytest.mark.parametrize("n", [16, 18])
def test_grad_two_pass_identities_and_dtypes(hm, n):
    """Homogeneity Re<g, psi> = 4q / ((1-q) ln 2) and Im<g, psi> = 0 at full size, complex64 against
    complex128 gradients, and M_q against the forward entry point."""
    psi = S.ry_rz_cz_state(n, np.random.default_rng(6700 + n).uniform(0, 2 * math.pi, (2, 2, n)))
    gs = {}
    for c64 in (False, True):
        x, _ = gpu_state(psi, c64)
        say(f"[grad two-pass full] n={n} c64={c64}")
        out, g = hm.sre_grad(x, 2.0)
        gs[c64] = g.cpu().numpy().astype(np.complex128)
        ip = np.vdot(gs[c64], x.cpu().numpy().astype(np.complex128))
        want = 4 * 2.0 / ((1 - 2.0) * math.log(2))
        tol = 1e-4 if c64 else 1e-9
        assert abs(ip.real - want) < tol * abs(want) and abs(ip.imag) < tol * abs(want), ip
        m = hm.sre(x, (2.0,)).cpu().numpy()
        assert abs(out.cpu().numpy()[0] - m[0]) < (1e-5 if c64 else 1e-10) * max(1.0, abs(m[0]))
    assert rel_l2(gs[True], gs[False]) < 1e-4


def test_grad_two_pass_central_differences(hm):
    """N = 16 (two-pass): h = 1e-6 central differences of the FP64 forward on sampled coordinates."""
    n = 16
    psi = S.gaussian_state(n, seed=6800)
    x = torch.from_numpy(psi).to(_dev())
    _, g = hm.sre_grad(x, 2.0)
    g = g.cpu().numpy()
    h = 1e-6
    for y in np.random.default_rng(6801).choice(2 ** n, 8, replace=False):
        for unit in (1.0, 1j):
            e = np.zeros_like(psi)
            e[y] = unit * h
            mp = hm.sre(torch.from_numpy(psi + e).to(_dev()), (2.0,))[0].item()
            mm = hm.sre(torch.from_numpy(psi - e).to(_dev()), (2.0,))[0].item()
            fd = (mp - mm) / (2 * h)
            an = g[y].real if unit == 1.0 else g[y].imag
            say(f"[grad two-pass fd] y={y} unit={unit} fd={fd:.9e} an={an:.9e}")
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)) + 1e-5 * abs(an), (y, unit, fd, an)


def test_autograd_circuit_two_pass(hm):
    """d M_2(psi(theta)) / d theta at N = 14 through torch.autograd and the two-pass adjoint, against
    central differences of the complex128 forward on the angles."""
    n = 14
    dev = _dev()
    ang0 = np.random.default_rng(6900).uniform(0, 2 * math.pi, (2, 2, n))
    ang = torch.tensor(ang0, dtype=torch.float64, device=dev, requires_grad=True)
    psi = S.ry_rz_cz_state_torch(n, ang)
    say("[grad autograd] circuit n=14 two-pass")
    m2 = hm.SRE.apply(psi, 2.0)
    m2.backward()
    got = ang.grad.cpu().numpy()
    h = 1e-6
    fd = np.zeros_like(ang0)
    for idx in np.ndindex(ang0.shape):
        ap, am = ang0.copy(), ang0.copy()
        ap[idx] += h
        am[idx] -= h
        fp = hm.sre(torch.from_numpy(S.ry_rz_cz_state(n, ap)).to(dev), (2.0,))[0].item()
        fm = hm.sre(torch.from_numpy(S.ry_rz_cz_state(n, am)).to(dev), (2.0,))[0].item()
        fd[idx] = (fp - fm) / (2 * h)
    assert np.max(np.abs(got - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd))), np.max(np.abs(got - fd))


def test_grad_two_pass_deterministic(hm):
    x, _ = gpu_state(S.gaussian_state(15, seed=6950), True)
    a = hm.sre_grad(x, 2.0)[1].cpu().numpy()
    b = hm.sre_grad(x, 2.0)[1].cpu().numpy()
    assert np.array_equal(a, b)


def test_grad_maximum_size_identities(hm):
    """n = 20 (largest gradient size), complex64: homogeneity and phase invariance of the gradient
    and M_2 against the forward entry point."""
    n = 20
    psi = S.ry_rz_cz_state(n, np.random.default_rng(6990).uniform(0, 2 * math.pi, (2, 2, n)))
    x, _ = gpu_state(psi, True)
    say("[grad max size] n=20 c64")
    out, g = hm.sre_grad(x, 2.0)
    ip = torch.vdot(g.to(torch.complex128), x.to(torch.complex128)).item()
    want = 4 * 2.0 / ((1 - 2.0) * math.log(2))
    assert abs(ip.real - want) < 1e-4 * abs(want) and abs(ip.imag) < 1e-4 * abs(want), ip
    m = hm.sre(x, (2.0,)).cpu().numpy()
    assert abs(out.cpu().numpy()[0] - m[0]) < 1e-5 * abs(m[0])


def test_grad_maximum_size_c64_vs_c128(hm):
    """n = 20, the largest gradient size (rows of 2^10 values in the fused backward kernel, the
    software-pipelined FP32 form): the complex64 gradient against the complex128 gradient (FP64
    transforms, the one-value-at-a-time form) of the same complex64-exact state, element by element
    in relative L2, and the complex128 gradient against the homogeneity identity."""
    n = 20
    psi = S.ry_rz_cz_state(n, np.random.default_rng(6991).uniform(0, 2 * math.pi, (2, 2, n)))
    v64, w = S.to_c64_exact(psi)
    say("[grad max size] n=20 c64 vs c128")
    o64, g64 = hm.sre_grad(torch.from_numpy(v64).to(_dev()), 2.0)
    x128 = torch.from_numpy(w).to(_dev())
    o128, g128 = hm.sre_grad(x128, 2.0)
    ip = torch.vdot(g128, x128).item()
    want = 4 * 2.0 / ((1 - 2.0) * math.log(2))
    assert abs(ip.real - want) < 1e-9 * abs(want) and abs(ip.imag) < 1e-9 * abs(want), ip
    err = rel_l2(g64.cpu().numpy().astype(np.complex128), g128.cpu().numpy())
    assert err < 1e-4, err
    assert abs(o64.cpu().numpy()[0] - o128.cpu().numpy()[0]) < 1e-5 * abs(o128.cpu().numpy()[0])


@pytest.mark.parametrize("c64,n,forced", [(False, 5, False), (True, 9, False), (False, 13, True), (True, 14, False)])
def test_grad_fractional_q(orc, hm, c64, n, forced):
    """q = 1.5 (the general |chi|^{2q-2} chi seed, no integer shortcut) on the resident and two-pass
    kernels against the FP64 oracle gradient."""
    psi = S.gaussian_state(n, seed=6800 + n)
    x, w = gpu_state(psi, c64)
    ctx = hm.Context()
    if forced:
        ctx.force_path(2)
    say(f"[grad q=1.5] n={n} c64={c64} forced={forced}")
    out, g = hm.sre_grad(x, 1.5, ctx=ctx)
    want_out, want_g = orc.sre_grad_direct(w, 1.5) if n <= 7 else orc.sre_grad_fwht(w, 1.5)
    assert rel_l2(g.cpu().numpy().astype(np.complex128), want_g) < (1e-4 if c64 else 1e-9)
    np.testing.assert_allclose(out.cpu().numpy(), want_out, rtol=(1e-5 if c64 else 1e-11), atol=1e-6 if c64 else 1e-12)


def test_autograd_step_is_one_fused_call(hm, monkeypatch):
    """With psi requiring grad, SRE.apply runs hm_sre_grad once in forward and nothing in backward;
    the value equals the fused call's M_q and the gradient its dM/dpsi (bitwise)."""
    import paper_2601_07824_amd as mod
    calls = {"sre": 0, "sre_grad": 0}
    real_sre, real_grad = mod.sre, mod.sre_grad

    def c_sre(*a, **k):
        calls["sre"] += 1
        return real_sre(*a, **k)

    def c_grad(*a, **k):
        calls["sre_grad"] += 1
        return real_grad(*a, **k)

    monkeypatch.setattr(mod, "sre", c_sre)
    monkeypatch.setattr(mod, "sre_grad", c_grad)
    x, _ = gpu_state(S.gaussian_state(12, seed=6600), True)
    say("[grad autograd] one fused call per step, n=12 c64")
    xg = x.clone().requires_grad_(True)
    m = hm.SRE.apply(xg, 2.0)
    m.backward()
    assert calls == {"sre": 0, "sre_grad": 1}, calls
    out, g = real_grad(x, 2.0)
    assert m.item() == out[0].item()
    assert torch.equal(xg.grad, g)
    calls.update(sre=0, sre_grad=0)
    with torch.no_grad():
        m0 = hm.SRE.apply(x, 2.0)
    assert calls == {"sre": 1, "sre_grad": 0}, calls
    assert abs(m0.item() - out[0].item()) < 1e-5 * abs(out[0].item())
