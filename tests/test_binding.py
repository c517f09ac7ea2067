"""Host-side checks of the Python binding (no GPU): argument errors raised before any library call."""
import pytest

torch = pytest.importorskip("torch")

import paper_2601_07824_amd as hm  # noqa: E402


def test_autograd_rejects_q1_when_grad_is_needed():
    """The adjoint is built for q != 1; SRE.apply says so in forward, before anything runs."""
    x = torch.zeros(16, dtype=torch.complex64, requires_grad=True)
    with pytest.raises(ValueError, match="q != 1"):
        hm.SRE.apply(x, 1.0)
    xb = torch.zeros((2, 16), dtype=torch.complex64, requires_grad=True)
    with pytest.raises(ValueError, match="q != 1"):
        hm.SREBatched.apply(xb, 1.0)


def test_states_must_live_on_the_gpu():
    with pytest.raises(TypeError, match="GPU"):
        hm.sre(torch.zeros(16, dtype=torch.complex64))
    with pytest.raises(TypeError, match="GPU"):
        hm.sre_noalloc(torch.zeros(16, dtype=torch.complex64))
