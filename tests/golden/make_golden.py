"""Writes tests/golden/oracle_golden.json: FP64 oracle values for seeded states too large to
recompute inside the test run.  Calls only the oracle and the seeded generators.

Usage: python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import states as S  # noqa: E402

OUT = os.path.join(HERE, "oracle_golden.json")


def cases():
    # (key, builder, kind, q)
    yield ("sre_brickwall_n16_d32_seed4200_c64", lambda: S.to_c64_exact(S.brickwall_haar(16, 32, seed=4200))[1], "sre", [2.0])
    yield ("sre_gauss_n16_seed4201_c128", lambda: S.gaussian_state(16, seed=4201), "sre", [1.0, 2.0, 3.0])
    for k in (1, 4, 16):
        yield (f"sre_clifford_t_n16_k{k}_seed42{k:02d}_c64",
               (lambda k=k: S.to_c64_exact(S.clifford_t_state(16, k, seed=4200 + k))[1]), "sre", [2.0])
    yield ("mana_gauss_n8_seed5008_c128", lambda: S.gaussian_state(8, d=3, seed=5008), "mana", None)
    yield ("mana_gauss_n10_seed5010_c64", lambda: S.to_c64_exact(S.gaussian_state(10, d=3, seed=5010))[1], "mana", None)


def main():
    data = {"_generator": "tests/golden/make_golden.py (oracle.sre_fwht / oracle.mana_fft, FP64)"}
    if os.path.exists(OUT):
        data.update(json.load(open(OUT)))
    for key, build, kind, q in cases():
        if key in data:
            continue
        t = time.time()
        psi = build()
        vals = oracle.sre_fwht(psi, q) if kind == "sre" else oracle.mana_fft(psi)
        data[key] = {"kind": kind, "q": q, "values": [float(v) for v in vals], "seconds": round(time.time() - t, 1)}
        print(key, data[key], flush=True)
        json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
