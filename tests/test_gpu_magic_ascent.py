"""Gradient ascent of M_2 through the fused forward + adjoint kernel and torch autograd over a
parameterised circuit (examples/magic_ascent.py).  For small steps every step must raise M_2, and
the gain of a step must match the first-order prediction lr * |dM_2/dangles|^2, which checks the
kernel's dM_2/dpsi along the circuit's tangent directions on both gradient paths (workgroup-resident
at n = 10, two-pass at n = 15)."""
import importlib.util
import math
import os
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _example():
    spec = importlib.util.spec_from_file_location("magic_ascent", os.path.join(ROOT, "examples", "magic_ascent.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("n,dtype,steps,lr", [(10, "c64", 12, 0.02), (10, "c128", 6, 0.02), (15, "c64", 3, 0.01)])
def test_ascent_raises_m2(n, dtype, steps, lr):
    ex = _example()
    dt = torch.complex64 if dtype == "c64" else torch.complex128
    hist, _ = ex.ascend(n, steps, lr, seed=7, dtype=dt)
    m = [h["M2"] for h in hist]
    print(f"[magic ascent] n={n} {dtype} M2 {m[0]:.6f} -> {m[-1]:.6f}", flush=True)
    assert m[-1] <= math.log2((2 ** n + 1) / 3) + 1e-6
    for k in range(1, len(hist)):
        gain = m[k] - m[k - 1]
        pred = lr * hist[k - 1]["grad_norm2"]
        assert gain > 0, (k, m)
        # second-order remainder: |gain - pred| small against pred for these step sizes
        assert abs(gain - pred) <= 0.25 * pred + (2e-6 if dtype == "c64" else 1e-12), (k, gain, pred)
