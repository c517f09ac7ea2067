"""Gradient ascent of the stabilizer Renyi entropy M_2 over the angles of a parameterised circuit.

The circuit is two layers of RZ(phi) RY(theta) on every qubit, each followed by a chain of CZ gates
(``synth.states.ry_rz_cz_state_torch``, differentiable in torch).  M_2 of the circuit's output state
(Eq. sre with q = 2) and dM_2/dpsi come from one call of the fused forward + adjoint kernel through
``paper_2601_07824_amd.SRE``; torch's autograd carries dM_2/dpsi back through the circuit to the
angles, which take plain gradient-ascent steps.  The magic of an N-qubit pure state is bounded by
M_2 <= log2((2^N + 1) / 3) (the Haar-typical value sits just below it), so the run shows how far a
shallow circuit can be pushed.

    python examples/magic_ascent.py --n 12 --steps 60 --lr 0.1
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import torch  # noqa: E402

import paper_2601_07824_amd as hm  # noqa: E402
from synth.states import ry_rz_cz_state_torch  # noqa: E402


def ascend(n: int, steps: int, lr: float, seed: int = 0, device: str = "cuda",
           dtype=torch.complex64, init_scale: float = 0.3):
    """Runs `steps` ascent steps from seeded random angles (normal, std `init_scale`).

    Returns (history, angles): history[k] = {"M2": M_2 before step k, "grad_norm2": |dM_2/dangles|^2
    at that point}; the first-order gain of step k is lr * grad_norm2."""
    g = torch.Generator().manual_seed(seed)
    angles = (init_scale * torch.randn((2, 2, n), generator=g, dtype=torch.float64)).to(device)
    angles.requires_grad_(True)
    history = []
    for _ in range(steps):
        psi = ry_rz_cz_state_torch(n, angles, dtype=dtype)
        m2 = hm.SRE.apply(psi, 2.0)
        angles.grad = None
        m2.backward()
        history.append({"M2": float(m2.detach()), "grad_norm2": float((angles.grad ** 2).sum())})
        with torch.no_grad():
            angles += lr * angles.grad
    return history, angles.detach()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=12)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--lr", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--c128", action="store_true", help="complex128 state (FP64 transforms)")
    args = ap.parse_args()
    hist, _ = ascend(args.n, args.steps, args.lr, args.seed,
                     dtype=torch.complex128 if args.c128 else torch.complex64)
    bound = math.log2((2 ** args.n + 1) / 3)
    for k, h in enumerate(hist):
        print(json.dumps({"step": k, **h}))
    print(json.dumps({"n": args.n, "M2_first": hist[0]["M2"], "M2_last": hist[-1]["M2"], "M2_bound": bound}))


if __name__ == "__main__":
    main()
