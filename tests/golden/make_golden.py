"""Writes tests/golden/oracle_golden.json: FP64 oracle values for seeded states too large to
recompute inside the test run.  Calls only the oracle and the seeded generators.

The headline cases (M_2 of the N = 20 brick-wall state of depth 40, seed 2020; mana of the N = 12
Gaussian qutrit state, seed 1212; gradients of M_2 at N = 16 and 18 for the two-layer RY/RZ + CZ
circuit states) take about an hour each on an 8-core host; cases already in the file are skipped,
so the script can be stopped and restarted.

Usage: python tests/golden/make_golden.py [key-substring ...]
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import states as S  # noqa: E402

OUT = os.path.join(HERE, "oracle_golden.json")
OUT_GRAD = os.path.join(HERE, "grad_golden.json")  # gradient samples (compact JSON, one line per case)


def cases():
    # (key, builder, kind, q)
    yield ("sre_brickwall_n16_d32_seed4200_c64", lambda: S.to_c64_exact(S.brickwall_haar(16, 32, seed=4200))[1], "sre", [2.0])
    yield ("sre_gauss_n16_seed4201_c128", lambda: S.gaussian_state(16, seed=4201), "sre", [1.0, 2.0, 3.0])
    for k in (1, 4, 16):
        yield (f"sre_clifford_t_n16_k{k}_seed42{k:02d}_c64",
               (lambda k=k: S.to_c64_exact(S.clifford_t_state(16, k, seed=4200 + k))[1]), "sre", [2.0])
    yield ("mana_gauss_n8_seed5008_c128", lambda: S.gaussian_state(8, d=3, seed=5008), "mana", None)
    yield ("mana_gauss_n10_seed5010_c64", lambda: S.to_c64_exact(S.gaussian_state(10, d=3, seed=5010))[1], "mana", None)
    # headline configurations (the benchmark's states)
    yield ("sre_brickwall_n20_d40_seed2020_c64", lambda: S.to_c64_exact(S.brickwall_haar(20, 40, seed=2020))[1],
           "sre", [2.0])
    yield ("mana_gauss_n12_seed1212_c64", lambda: S.to_c64_exact(S.gaussian_state(12, d=3, seed=1212))[1], "mana", None)
    for n in (16, 18):
        yield (f"grad_ryrzcz_n{n}_seed{4000 + n}_c64",
               (lambda n=n: S.to_c64_exact(S.ry_rz_cz_state(
                   n, np.random.default_rng(4000 + n).uniform(0, 2 * math.pi, (2, 2, n))))[1]), "grad", 2.0)
    yield ("sre_brickwall_n20_d40_seed2020_c128", lambda: S.brickwall_haar(20, 40, seed=2020), "sre", [1.0, 2.0, 3.0])
    yield ("mana_gauss_n12_seed1212_c128", lambda: S.gaussian_state(12, d=3, seed=1212), "mana", None)


GRAD_SAMPLE = 4096


def grad_record(psi, q):
    """M_q, lost_norm, the 2-norm and max-norm of the gradient and its values at 4096 seeded indices
    (seed = length of the state), all from the FP64 adjoint of Algorithm 2."""
    out, g = oracle.sre_grad_fwht(psi, q)
    idx = np.sort(np.random.default_rng(len(psi)).choice(len(psi), GRAD_SAMPLE, replace=False))
    return {"values": [float(v) for v in out], "norm2": float(np.linalg.norm(g)),
            "norm_inf": float(np.max(np.abs(g))), "idx": [int(i) for i in idx],
            "g_re": [float(v) for v in g[idx].real], "g_im": [float(v) for v in g[idx].imag]}


def main():
    data = {"_generator": "tests/golden/make_golden.py (oracle.sre_fwht / oracle.mana_fft, FP64)"}
    if os.path.exists(OUT):
        data.update(json.load(open(OUT)))
    grads = json.load(open(OUT_GRAD)) if os.path.exists(OUT_GRAD) else {}
    only = sys.argv[1:]
    for key, build, kind, q in cases():
        if key in data or key in grads or (only and not any(o in key for o in only)):
            continue
        t = time.time()
        psi = build()
        if kind == "grad":
            rec = {"kind": kind, "q": q, **grad_record(psi, q)}
        else:
            vals = oracle.sre_fwht(psi, q) if kind == "sre" else oracle.mana_fft(psi)
            rec = {"kind": kind, "q": q, "values": [float(v) for v in vals]}
        rec["seconds"] = round(time.time() - t, 1)
        rec["oracle_threads"] = oracle.get_threads()
        print(key, {k: v for k, v in rec.items() if k not in ("idx", "g_re", "g_im")}, flush=True)
        if kind == "grad":
            grads[key] = rec
            with open(OUT_GRAD, "w") as f:
                f.write("{\n" + ",\n".join(json.dumps(k) + ": " + json.dumps(v) for k, v in grads.items()) + "\n}\n")
            continue
        data[key] = rec
        json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
