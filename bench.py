#!/usr/bin/env python3
"""Throughput of exact stabilizer Renyi entropy M_2 on one MI355X.

Workload (one "step"): M_2 of one N = 20 qubit state (complex64 amplitudes, FP32 transforms, FP64
sums), i.e. all 4^20 Pauli expectation values, through hm_sre.  The state is a seeded brick-wall
circuit of Haar-random two-qubit gates of depth 2N applied to |0...0> (the paper's benchmark
workload); it is resident in HBM before the timed region starts.

Prints one JSON line.  `value` is Pauli expectations per second (4^N / seconds per step).
`roofline` describes the dominant kernel, timed with hipEvents on its launch stream during the timed
steps.  `cpu_baseline` times the FP64 oracle (plain Algorithm 2 in C, OpenMP over X-shifts) on a
bounded prefix of the same workload's X-shifts.  `secondary` holds the other rows of the metric
(complex128 transforms, mana, fwd+grad) when available.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LANE_OPS_PER_S = 256 * 64 * 2.4e9  # VALU lane operations per second (no packed FP32): 39.3e12


def sre_kernel_mix(N: int, family: str, nl: int, nh: int):
    """(FP32 flops, VALU lane-ops) per folded complex value for one kernel family."""
    if family == "sre_rowpass_write":      # product + nl butterfly stages
        return 6 + 2 * nl, 4 + 2 * nl
    if family == "sre_colpass":            # nh butterfly stages + reduction of Re, Im
        return 2 * nh + 8, 2 * nh + 6
    if family == "sre_rowpass_resident":   # product + all stages + reduction
        return 6 + 2 * (N - 1) + 8, 4 + 2 * (N - 1) + 6
    return None


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if the kernel source is
    unchanged since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{workload}/{kernel}")
        src = open(os.path.join(ROOT, "paper_2601_07824_amd", "csrc", rec["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha"]:
            return None
        return rec["bytes_per_launch"]
    except Exception:
        return None


def cpu_baseline(psi_w, N: int, target_s: float = 12.0):
    import oracle
    cores = oracle.get_threads()
    k = 64
    t = time.perf_counter()
    oracle.sre_fwht_sums(psi_w, (2.0,), 0, k)
    dt = time.perf_counter() - t
    k2 = max(k, min(1 << N, int(k * target_s / max(dt, 1e-3))))
    k2 = (k2 // cores) * cores or cores
    t = time.perf_counter()
    oracle.sre_fwht_sums(psi_w, (2.0,), 0, k2)
    dt = time.perf_counter() - t
    return {"value": k2 * float(2 ** N) / dt, "unit": "Pauli expectations/s", "cores": cores, "kind": "oracle",
            "sample": f"X-shifts a in [0, {k2}) of the N={N} workload ({k2} of {2 ** N} rows, "
                      f"{k2 * 2 ** N:.3e} expectations, {dt:.1f} s, FP64 C + OpenMP)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=20, help="qubits (default 20)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the X-shift loop "
              "would be sharded over GPUs with one all-reduce of the partial sums, see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2601_07824_amd as hm
    from synth import states as S

    dev = torch.device("cuda:0")
    N = args.n
    seed = 2020
    psi = S.brickwall_haar(N, 2 * N, seed=seed)
    c64, c64w = S.to_c64_exact(psi)
    x = torch.from_numpy(c64).to(dev)
    ctx = hm.default_context()

    for _ in range(args.warmup):
        hm.sre(x, (2.0,))
    torch.cuda.synchronize()

    hm.profile_reset()
    hm.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = hm.sre(x, (2.0,))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hm.profile_enable(False)
    prof = hm.profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    res = out.cpu().numpy()
    value = float(4 ** N) / (ms * 1e-3)

    # dominant kernel and its roofline
    nf = N - 1
    nl = (nf + 1) // 2
    nh = nf - nl
    fam = max(prof, key=lambda k: prof[k][1])
    cnt, tot_ms = prof[fam]
    mix = sre_kernel_mix(N, fam, nl, nh)
    roof = None
    if mix:
        flops_per_val, ops_per_val = mix
        vals_per_launch = float(2 ** N) * float(2 ** nf) / cnt / args.steps * args.steps  # per launch
        vals_per_launch = float(2 ** N) * float(2 ** nf) * args.steps / cnt
        t_launch = tot_ms * 1e-3 / cnt
        achieved = vals_per_launch * flops_per_val / t_launch / 1e12
        peak = LANE_OPS_PER_S * flops_per_val / ops_per_val / 1e12
        roof = {"bound": "alu", "kernel": fam, "achieved": round(achieved, 2), "peak": round(peak, 2),
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": traffic_for(fam, f"sre_n{N}_c64"),
                "launches": cnt, "avg_launch_ms": round(tot_ms / cnt, 4),
                "flops_per_launch": vals_per_launch * flops_per_val,
                "note": "FP32 VALU, no packed FP32: 39.3e12 lane-ops/s x (flops/op of this kernel's mix)"}

    line = {
        "metric": "Pauli expectations/s for M_2 (N=20 qubits) & mana (N=12); fwd vs fwd+grad",
        "value": value, "unit": "Pauli expectations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 (fp32 transforms, fp64 sums)", "data": "synthetic",
        "config": {"workload": f"SRE M_2, N={N} qubits, complex64, brick-wall Haar circuit depth {2 * N}, seed {seed}, "
                               f"all 4^{N} Pauli strings", "parallelism": "none (1 GPU)"},
        "result": {"M2": float(res[0]), "lost_norm": float(res[1])},
        "kernel_ms": {k: round(v[1] / args.steps, 3) for k, v in prof.items()},
        "roofline": roof,
    }

    if not args.no_secondary:
        sec = {}
        # complex128 (FP64 transforms) forward on the same state
        x128 = torch.from_numpy(psi).to(dev)
        hm.sre(x128, (2.0,))
        torch.cuda.synchronize()
        t = time.perf_counter()
        o = hm.sre(x128, (2.0,))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        sec["sre_fwd_c128"] = {"value": float(4 ** N) / dt, "ms": dt * 1e3, "M2": float(o[0].item())}
        for key, fn in (("mana_n12_c64", lambda: hm.mana(torch.from_numpy(
                S.to_c64_exact(S.gaussian_state(12, d=3, seed=1212))[0]).to(dev))),
                        ("sre_fwd_grad_c64", lambda: hm.sre_grad(x, 2.0))):
            try:
                fn()
                torch.cuda.synchronize()
                t = time.perf_counter()
                o = fn()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                work = 9.0 ** 12 if key.startswith("mana") else 4.0 ** N
                sec[key] = {"value": work / dt, "ms": dt * 1e3,
                            "unit": "phase-space points/s" if key.startswith("mana") else "Pauli expectations/s"}
            except hm.HmError as e:
                sec[key] = {"value": None, "error": str(e)[:160]}
        line["secondary"] = sec

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c64w, N)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
