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

# FP32 VALU lane operations per second without packed FP32: the vector peak of 157.3 TFLOP/s counts
# an FMA as 2 FLOP, i.e. 78.6e12 lane-FMAs/s = 2 wave64 instructions per CU per cycle at 2.4 GHz
# (a plain loop of FP32 adds measured 57e12 adds/s on MI355X, above one instruction per CU-cycle).
LANE_OPS_PER_S = 2 * 256 * 64 * 2.4e9


def sre_kernel_mix(N: int, family: str, nl: int, nh: int):
    """(FP32 flops, VALU lane-ops) per folded complex value for one kernel family."""
    if family == "sre_rowpass_write":      # product + nl butterfly stages
        return 6 + 2 * nl, 4 + 2 * nl
    if family == "sre_colpass":            # nh butterfly stages + reduction of Re, Im
        return 2 * nh + 8, 2 * nh + 6
    if family == "sre_rowpass_resident":   # product + all stages + reduction
        return 6 + 2 * (N - 1) + 8, 4 + 2 * (N - 1) + 6
    return None


def PROFILE_EVERY(N: int, shifts: int) -> int:
    """Sampling interval of the kernel timing: about 256 timed launches per family and step."""
    per_launch = max(1, (128 << 20) // (8 << max(N - 1, 0)))  # shifts per two-pass launch, roughly
    return max(1, shifts // per_launch // 256)


HBM_PEAK_GBS = 8000.0


def roofline(fam: str, N: int, vals_per_launch: float, t_launch: float, launches_per_step: int, plan: dict | None):
    """Roofline of one kernel family (complex64).  Two-pass kernels move the half-transformed vector
    through device memory (8 B per folded value written by the row pass and read by the column
    pass; the pipelined kernel does both): that compulsory exchange is their bound.  The
    workgroup-resident kernel touches device memory only for the state and is bound by FP32 VALU
    arithmetic."""
    nf = N - 1
    nl = (plan or {}).get("row_bits") or (nf + 1) // 2  # index bits of the row pass in the timed plan
    nh = nf - nl
    xbytes = {"sre_rowpass_write": 8.0, "sre_colpass": 8.0, "sre_pair": 16.0}.get(fam)
    mix = sre_kernel_mix(N, fam if fam != "sre_pair" else "sre_rowpass_write", nl, nh)
    r = {"kernel": fam, "launches_per_step": launches_per_step, "avg_launch_ms": round(t_launch * 1e3, 5)}
    valu = None
    if mix:
        flops_per_val, ops_per_val = mix
        achieved = vals_per_launch * flops_per_val / t_launch / 1e12
        peak = LANE_OPS_PER_S * flops_per_val / ops_per_val / 1e12
        valu = {"achieved": round(achieved, 2), "peak": round(peak, 2), "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4)}
    if xbytes:
        bpl = vals_per_launch * xbytes
        achieved = bpl / t_launch / 1e9
        r.update({"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_launch": bpl,
                  "traffic": traffic_for(fam, f"sre_n{N}_c64", plan), "valu": valu,
                  "note": "achieved = exchange bytes (8 B per folded value per pass) / average launch time"})
    elif valu:
        r.update({"bound": "alu", **valu, "traffic": traffic_for(fam, f"sre_n{N}_c64", plan),
                  "note": "FP32 VALU without packed FP32: 78.6e12 lane-ops/s x flops per op of this kernel"})
    return r


def traffic_for(kernel: str, workload: str, plan: dict | None):
    """HBM/MALL bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE of the committed counter runs,
    each scaled by what the same counter reads for a plain 256 MiB device copy), if the kernel
    sources are unchanged since the counters were taken and the launch configuration is the same;
    else None.  A kernel may have one record per measured plan."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or not plan:
        return None
    try:
        recs = json.load(open(path)).get(f"{workload}/{kernel}")
        if recs is None:
            return None
        for rec in (recs if isinstance(recs, list) else [recs]):  # one record per measured plan
            h = hashlib.sha256()
            for src in rec["sources"]:
                h.update(open(os.path.join(ROOT, src), "rb").read())
            if h.hexdigest()[:16] == rec["source_sha"] and all(plan.get(k) == v for k, v in rec["plan"].items()):
                return rec["bytes_per_launch"]
        return None
    except Exception:
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
            "cpu_model": cpu_model(),
            "sample": f"X-shifts a in [0, {k2}) of the N={N} workload ({k2} of {2 ** N} rows, "
                      f"{k2 * 2 ** N:.3e} expectations, {dt:.1f} s, FP64 C + OpenMP)"}


def _timed(torch, fn, reps=1):
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        o = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps, o


GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_golden.json")


def golden(key):
    """FP64 oracle values stored by tests/golden/make_golden.py (None if not generated)."""
    try:
        return json.load(open(GOLDEN)).get(key)
    except (OSError, ValueError):
        return None


def error_vs_oracle(got: float, key: str, index: int = 0):
    g = golden(key)
    if not g:
        return None
    want = g["values"][index]
    return {"oracle": want, "abs": abs(got - want), "rel": abs(got - want) / abs(want), "golden": key}


def profiled(hm, torch, fn, every=1):
    """Runs fn() once with every-th launch of each kernel family timed on its stream; returns
    (wall seconds, fn's result, {family: (launches, timed, ms)})."""
    fn()
    torch.cuda.synchronize()
    hm.profile_reset()
    hm.profile_enable(every)
    torch.cuda.synchronize()
    t = time.perf_counter()
    o = fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    hm.profile_enable(False)
    return dt, o, hm.profile_read()


def exchange_roofline(prof, fam_bytes: dict, work_values: float):
    """Roofline of the dominant exchange kernel of a two-pass run: bytes per launch = the values it
    moves (work_values / launches) x the bytes each value moves through device memory."""
    est = {k: v[2] / max(v[1], 1) * v[0] for k, v in prof.items() if v[1] > 0 and k in fam_bytes}
    if not est:
        return None
    fam = max(est, key=est.get)
    launches, timed, tot_ms = prof[fam]
    t_launch = tot_ms * 1e-3 / timed
    bpl = work_values / launches * fam_bytes[fam]
    return {"kernel": fam, "bound": "hbm", "launches": launches, "avg_launch_ms": round(t_launch * 1e3, 5),
            "bytes_per_launch": bpl, "achieved": round(bpl / t_launch / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(bpl / t_launch / 1e9 / HBM_PEAK_GBS, 4)}


def mixed_pass_bytes(na: int, value_bytes: int = 16) -> float:
    """Bytes the mixed-state mana streams through HBM: the first pass reads rho and writes the
    reordered copy (qutrits 0..2), each further pass but the last reads and writes it (two qutrits),
    the last reads it; 9^na values each time."""
    m = min(na, 3)
    rest = na - m
    passes = (rest + 1) // 2
    units = (1 if passes == 0 else 2) + 2 * max(passes - 1, 0) + (1 if passes else 0)
    return units * 9.0 ** na * value_bytes


def secondary(hm, S, torch, dev, psi, N):
    """The other rows of the metric, each timed once after a warm-up call (wall clock around the
    call, state resident; plans autotuned where noted): complex128 forward at the headline N
    (tuned, with the roofline of its dominant kernel), mana at N = 12 (tuned, roofline), fused
    forward + adjoint against the plain forwards at N = 13 (workgroup-resident gradient) and N = 18
    (two-pass gradient), batches of 64 circuit states at N = 12 and 16 (batched fused forward +
    adjoint, 64 single calls, FP64 forward), the batched form on 1024 states of uneven size (one
    persistent launch, and the autotuned launch form), the uniform-row Monte Carlo estimator at
    N = 24, the thermodynamic-integration estimator at N = 16, 18, 20 against the exact value and at
    N = 24, 26, and each result's error against the stored FP64 oracle values where they exist."""
    import numpy as np
    sec = {}
    try:
        x128 = torch.from_numpy(psi).to(dev)
        c128 = hm.Context()
        # one stream, as the headline: with two, a kernel's event-bracketed time overlaps the other
        # stream's kernels and no longer measures that kernel
        c128.set_option(hm.OPT_STREAMS, 1)
        hm.autotune(x128, 16384, ctx=c128)
        dt, o, prof = profiled(hm, torch, lambda: hm.sre(x128, (2.0,), ctx=c128), every=64)
        m2 = float(o[0].item())
        sec["sre_fwd_c128_n%d" % N] = {
            "value": 4.0 ** N / dt, "unit": "Pauli expectations/s", "ms": dt * 1e3, "M2": m2,
            "error_vs_oracle": error_vs_oracle(m2, "sre_brickwall_n%d_d%d_seed2020_c128" % (N, 2 * N), 1),
            # 4^N / 2 folded FP64 complex values per evaluation, 16 B each written by the row pass and
            # read by the column pass (both by the pipelined kernel)
            "roofline": exchange_roofline(prof, {"sre_rowpass_write": 16.0, "sre_colpass": 16.0, "sre_pair": 32.0},
                                          4.0 ** N / 2.0),
            "plan": hm.tuned_plan(N, hm.HM_C128, ctx=c128)}
        del x128
        m = torch.from_numpy(S.to_c64_exact(S.gaussian_state(12, d=3, seed=1212))[0]).to(dev)
        cm = hm.Context()
        hm.autotune_mana(m, 4096, ctx=cm)
        dt, o, prof = profiled(hm, torch, lambda: hm.mana(m, ctx=cm), every=16)
        mana = float(o[0].item())
        sec["mana_n12_c64"] = {
            "value": 9.0 ** 12 / dt, "unit": "phase-space points/s", "ms": dt * 1e3, "mana": mana,
            "error_vs_oracle": error_vs_oracle(mana, "mana_gauss_n12_seed1212_c64"),
            # packed values: 9^12 / 2 per evaluation, 8 B each written by the row pass and read by the column pass
            "roofline": exchange_roofline(prof, {"mana_rowpass_write": 8.0, "mana_colpass": 8.0}, 9.0 ** 12 / 2.0),
            "roofline_whole": {"bytes": 9.0 ** 12 / 2.0 * 16.0, "achieved_GBs": 9.0 ** 12 / 2.0 * 16.0 / dt / 1e9,
                               "frac": 9.0 ** 12 / 2.0 * 16.0 / dt / 1e9 / HBM_PEAK_GBS}}
        del m
        ng = 13
        pg = S.ry_rz_cz_state(ng, np.random.default_rng(4013).uniform(0, 2 * math.pi, (2, 2, ng)))
        g64 = torch.from_numpy(S.to_c64_exact(pg)[0]).to(dev)
        g128 = torch.from_numpy(pg).to(dev)
        for key, fn in (("sre_fwd_grad_c64_n13", lambda: hm.sre_grad(g64, 2.0)),
                        ("sre_fwd_c64_n13", lambda: hm.sre(g64, (2.0,))),
                        ("sre_fwd_c128_n13", lambda: hm.sre(g128, (2.0,)))):
            dt, _ = _timed(torch, fn, reps=20)
            sec[key] = {"value": 4.0 ** ng / dt, "unit": "Pauli expectations/s", "ms": dt * 1e3}
        ng = 18
        pg = S.ry_rz_cz_state(ng, np.random.default_rng(4018).uniform(0, 2 * math.pi, (2, 2, ng)))
        g64 = torch.from_numpy(S.to_c64_exact(pg)[0]).to(dev)
        g128 = torch.from_numpy(pg).to(dev)
        for key, fn in (("sre_fwd_grad_c64_n18", lambda: hm.sre_grad(g64, 2.0)),
                        ("sre_fwd_c64_n18", lambda: hm.sre(g64, (2.0,))),
                        ("sre_fwd_c128_n18", lambda: hm.sre(g128, (2.0,)))):
            dt, o = _timed(torch, fn)
            sec[key] = {"value": 4.0 ** ng / dt, "unit": "Pauli expectations/s", "ms": dt * 1e3}
        for ng in (12, 16):
            # a batch of 64 seeded 2-layer RY/RZ + CZ circuit states: batched fused forward + adjoint,
            # the same states one call at a time, and the plain FP64 forward of the batch
            angs = np.random.default_rng(4100 + ng).uniform(0, 2 * math.pi, (64, 2, 2, ng))
            pgs = np.stack([S.ry_rz_cz_state(ng, a) for a in angs])
            b64 = torch.from_numpy(np.stack([S.to_c64_exact(p)[0] for p in pgs])).to(dev)
            b128 = [t for t in torch.from_numpy(pgs).to(dev).unbind(0)]
            for key, fn in (("sre_fwd_grad_c64_n%d_batch64" % ng, lambda: hm.sre_grad_batched(b64, 2.0)),
                            ("sre_fwd_grad_c64_n%d_64calls" % ng, lambda: [hm.sre_grad(b64[i], 2.0) for i in range(64)]),
                            ("sre_fwd_c128_n%d_batch64" % ng, lambda: hm.sre_batched(b128, (2.0,)))):
                dt, _ = _timed(torch, fn, reps=5 if ng <= 12 else 1)
                sec[key] = {"value": 64 * 4.0 ** ng / dt, "unit": "Pauli expectations/s", "ms": dt * 1e3,
                            "states": 64}
            del b64, b128
        rng = np.random.default_rng(5005)
        ns = rng.integers(10, 17, size=1024)
        states = [torch.from_numpy(S.to_c64_exact(S.gaussian_state(int(n), seed=5000 + i))[0]).to(dev)
                  for i, n in enumerate(ns)]
        dt, _ = _timed(torch, lambda: hm.sre_batched(states, (2.0,)))
        sec["sre_batched_1024_n10to16_c64"] = {"value": float(np.sum(4.0 ** ns)) / dt, "unit": "Pauli expectations/s",
                                               "ms": dt * 1e3, "states": 1024, "launch": "one persistent launch"}
        cb = hm.Context()
        hm.autotune_batched(states, ctx=cb)
        dt, _ = _timed(torch, lambda: hm.sre_batched(states, (2.0,), ctx=cb))
        sec["sre_batched_1024_n10to16_c64_tuned"] = {"value": float(np.sum(4.0 ** ns)) / dt,
                                                     "unit": "Pauli expectations/s", "ms": dt * 1e3, "states": 1024}
        del states
        g = torch.Generator(device="cpu").manual_seed(2424)
        v = torch.view_as_complex(torch.randn(2 ** 24, 2, generator=g, dtype=torch.float32)).to(dev)
        v /= torch.linalg.vector_norm(v)
        c24 = hm.Context()
        hm.autotune(v, 256, ctx=c24)
        dt, o = _timed(torch, lambda: hm.sre_sampled(v, n_rows=4096, seed=24, ctx=c24))
        sec["sre_mc_n24_4096rows_c64"] = {"value": 4097 * 2.0 ** 24 / dt, "unit": "Pauli expectations/s",
                                          "ms": dt * 1e3, "M2_hat": float(o[0].item()),
                                          "stderr": float(o[1].item())}
        # thermodynamic integration (L = 9 beta points x 32 chains, 600 Metropolis steps, 100 left out)
        for nm in (16, 18, 20):
            x = torch.from_numpy(S.to_c64_exact(S.brickwall_haar(nm, 2 * nm, seed=9500 + nm))[0]).to(dev)
            exact = float(hm.sre(x, (2.0,))[0].item())
            t = time.perf_counter()
            out, _ = hm.sre_mc(x, 9, 32, 600, 100, seed=9600 + nm)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            sec["sre_mc_ti_n%d_c64" % nm] = {"M2_hat": float(out[0].item()), "dM2": float(out[1].item()),
                                             "M2_exact": exact, "error": float(out[0].item()) - exact,
                                             "rows": 9 * 32 * 601, "ms": dt * 1e3,
                                             "value": 9 * 32 * 601 * 2.0 ** nm / dt, "unit": "Pauli expectations/s"}
        for nm, steps in ((24, 400), (26, 200)):
            g = torch.Generator(device="cpu").manual_seed(2400 + nm)
            v = torch.view_as_complex(torch.randn(2 ** nm, 2, generator=g, dtype=torch.float32)).to(dev)
            v /= torch.linalg.vector_norm(v)
            t = time.perf_counter()
            out, _ = hm.sre_mc(v, 17, 4, steps, steps // 8, seed=9700 + nm)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            sec["sre_mc_ti_n%d_c64" % nm] = {"M2_hat": float(out[0].item()), "dM2": float(out[1].item()),
                                             "haar_mean": math.log2(2.0 ** nm + 3) - 2, "rows": 17 * 4 * (steps + 1),
                                             "ms": dt * 1e3, "value": 17 * 4 * (steps + 1) * 2.0 ** nm / dt,
                                             "unit": "Pauli expectations/s"}
            del v
        # mixed-state mana of subsystems of a qutrit brick-wall state (depth 3), complex128 as in the
        # paper's table: N_A = 8 of N = 10 and N_A = 10 of N = 11 (reduced density matrix included)
        for nq, na in ((10, 8), (11, 10)):
            x = torch.from_numpy(S.brickwall_haar(nq, 3, seed=9800 + nq, d=3)).to(dev)
            rho = hm.reduced_density_matrix(x, na)
            torch.cuda.synchronize()
            dt, o = _timed(torch, lambda: hm.mana_mixed(rho))
            sec["mana_mixed_na%d_c128" % na] = {"ms": dt * 1e3, "mana": float(o[0].item()), "trace": float(o[1].item()),
                                                "purity": float(o[2].item()), "value": 9.0 ** na / dt,
                                                "unit": "phase-space points/s",
                                                "hbm_bytes": mixed_pass_bytes(na),
                                                "hbm_frac": mixed_pass_bytes(na) / dt / 1e9 / HBM_PEAK_GBS}
            del rho
        # pure-state mana of qudits of odd prime dimension at the largest sizes of the LDS-resident
        # kernel (Gaussian states): d^(2n) phase-space points per evaluation
        for d, nd, dt_ in ((5, 6, torch.complex64), (7, 5, torch.complex64), (5, 5, torch.complex128),
                           (7, 4, torch.complex128)):
            x = torch.from_numpy(S.gaussian_state(nd, d, seed=9900 + 10 * d + nd)).to(dt_).to(dev)
            dt, o = _timed(torch, lambda: hm.mana_qudit(x, d))
            sec["mana_qudit_d%d_n%d_%s" % (d, nd, "c64" if dt_ == torch.complex64 else "c128")] = {
                "ms": dt * 1e3, "mana": float(o[0].item()), "value": float(d) ** (2 * nd) / dt,
                "unit": "phase-space points/s"}
            del x
    except hm.HmError as e:
        sec["error"] = str(e)[:200]
    return sec


def oracle_table(hm, S, torch, dev, target_s: float = 2.0):
    """GPU (complex64 and complex128, full evaluation, tuned plan) and FP64 oracle (the plain
    Algorithms 2 and 4 in C with OpenMP, on a prefix of the shifts sized to about target_s) rates at
    the sizes the method is usually run at.  Rates are per Pauli string / phase-space point."""
    import oracle
    rows = []
    for d, n in ((2, 8), (2, 12), (2, 16), (2, 20), (3, 6), (3, 8), (3, 10), (3, 12)):
        psi = S.brickwall_haar(n, 2 * n, seed=3000 + n, d=d)
        v64, w64 = S.to_c64_exact(psi)
        work = float(d ** n) ** 2
        rec = {"d": d, "n": n}
        for name, arr in (("gpu_c64", v64), ("gpu_c128", psi)):
            x = torch.from_numpy(arr).to(dev)
            ctx = hm.Context()
            if d == 2 and n >= 12:
                hm.autotune(x, 4096, ctx=ctx)
            fn = (lambda: hm.sre(x, (2.0,), ctx=ctx)) if d == 2 else (lambda: hm.mana(x, ctx=ctx))
            reps = 1 if work > 1e11 else 20
            dt, _ = _timed(torch, fn, reps)
            rec[name] = work / dt
        shifts = d ** n
        k = min(shifts, 8)
        f = (lambda a1: oracle.sre_fwht_sums(w64, (2.0,), 0, a1)) if d == 2 else (lambda a1: oracle.mana_fft_sums(w64, 0, a1))
        t = time.perf_counter()
        f(k)
        dt = time.perf_counter() - t
        k = max(k, min(shifts, int(k * target_s / max(dt, 1e-4))))
        t = time.perf_counter()
        f(k)
        dt = time.perf_counter() - t
        rec["oracle"] = k * float(d ** n) / dt
        rec["oracle_sample"] = f"{k} of {shifts} shifts, {dt:.2f} s"
        rows.append(rec)
    return {"unit": "Pauli strings or phase-space points per second", "oracle_threads": oracle.get_threads(),
            "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=20, help="qubits (default 20)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--shifts", type=int, default=0,
                    help="profiling runs: evaluate only X-shifts [0, SHIFTS) per step (0 = all 2^N)")
    ap.add_argument("--batch", type=int, default=0, help="X-shifts per two-pass launch (0 = planner default)")
    ap.add_argument("--pipeline", type=int, default=0, choices=(0, 1, 2), help="HM_OPT_PIPELINE")
    ap.add_argument("--lds-split", type=int, default=0, choices=(0, 1, 2), help="HM_OPT_LDS_SPLIT")
    ap.add_argument("--row-bits", type=int, default=0, help="HM_OPT_ROW_BITS (0 = planner default)")
    ap.add_argument("--no-autotune", action="store_true", help="skip the plan autotuner (untimed, before warm-up)")
    ap.add_argument("--grad-only", type=int, default=0, metavar="N",
                    help="time only the fused forward + adjoint of M_2 at N qubits (profiling runs)")
    ap.add_argument("--mana-only", type=int, default=0, metavar="N",
                    help="profiling runs: time only the qutrit mana of an N-qutrit complex64 state per step")
    ap.add_argument("--batched-only", action="store_true",
                    help="profiling runs: time only hm_sre_batched on the 1024 states with n in [10, 16] per step")
    ap.add_argument("--mixed-only", type=int, default=0, metavar="NA",
                    help="profiling runs: time only the mixed-state mana of an N_A-qutrit reduced density matrix")
    ap.add_argument("--mc-only", type=int, default=0, metavar="N",
                    help="profiling runs: time only the thermodynamic-integration Monte Carlo M_2 at N qubits")
    ap.add_argument("--oracle-table", action="store_true",
                    help="print GPU and oracle rates side by side for SRE n = 8, 12, 16, 20 and mana n = 6, 8, 10, 12"
                         " (oracle on a bounded prefix of the shifts) and exit")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="counter calibration: time a plain device copy of this many MiB five times and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the X-shift loop "
              "would be sharded over GPUs, each evaluating hm_sre_partial on its share, with one all-reduce of "
              "the partial sums)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2601_07824_amd as hm
    from synth import states as S

    dev = torch.device("cuda:0")
    if args.oracle_table:
        print(json.dumps(oracle_table(hm, S, torch, dev)), flush=True)
        return
    if args.mana_only:
        n = args.mana_only
        m = torch.from_numpy(S.to_c64_exact(S.gaussian_state(n, d=3, seed=1212))[0]).to(dev)
        for _ in range(args.warmup):
            hm.mana(m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            o = hm.mana(m)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        print(json.dumps({"metric": "phase-space points/s (mana)", "value": 9.0 ** n / (ms * 1e-3),
                          "unit": "phase-space points/s", "ms_per_step": ms, "steps": args.steps,
                          "config": {"workload": f"mana, N={n} qutrits, complex64 Gaussian state, seed 1212"},
                          "mana": float(o[0].item())}), flush=True)
        return
    def only_loop(fn, name, unit, work, workload, extra=None):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            o = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        rec = {"metric": name, "value": work / (ms * 1e-3), "unit": unit, "ms_per_step": ms, "steps": args.steps,
               "config": {"workload": workload}}
        rec.update(extra(o) if extra else {})
        print(json.dumps(rec), flush=True)

    if args.batched_only:
        rng = np.random.default_rng(5005)
        ns = rng.integers(10, 17, size=1024)
        states = [torch.from_numpy(S.to_c64_exact(S.gaussian_state(int(n), seed=5000 + i))[0]).to(dev)
                  for i, n in enumerate(ns)]
        only_loop(lambda: hm.sre_batched(states, (2.0,)), "Pauli expectations/s (batched M_2)", "Pauli expectations/s",
                  float(np.sum(4.0 ** ns)), "1024 complex64 Gaussian states, n uniform in [10, 16] (seed 5005), one call")
        return
    if args.mixed_only:
        na = args.mixed_only
        x = torch.from_numpy(S.brickwall_haar(na + 2, 3, seed=9800 + na + 2, d=3)).to(dev)
        rho = hm.reduced_density_matrix(x, na)
        only_loop(lambda: hm.mana_mixed(rho), "phase-space points/s (mixed-state mana)", "phase-space points/s",
                  9.0 ** na, f"mixed-state mana, N_A={na} of a {na + 2}-qutrit brick-wall state (depth 3), complex128",
                  lambda o: {"mana": float(o[0].item())})
        return
    if args.mc_only:
        nm = args.mc_only
        g = torch.Generator(device="cpu").manual_seed(2400 + nm)
        v = torch.view_as_complex(torch.randn(2 ** nm, 2, generator=g, dtype=torch.float32)).to(dev)
        v /= torch.linalg.vector_norm(v)
        only_loop(lambda: hm.sre_mc(v, 17, 4, 200, 25, seed=9700 + nm)[0],
                  "Pauli expectations/s (thermodynamic-integration M_2)", "Pauli expectations/s",
                  17 * 4 * 201 * 2.0 ** nm, f"MC-TI M_2, N={nm}, complex64 Gaussian state, 17 beta x 4 chains x 200 steps",
                  lambda o: {"M2_hat": float(o[0].item()), "dM2": float(o[1].item())})
        return
    if args.grad_only:
        n = args.grad_only
        import numpy as np
        pg = S.ry_rz_cz_state(n, np.random.default_rng(4000 + n).uniform(0, 2 * math.pi, (2, 2, n)))
        g = torch.from_numpy(S.to_c64_exact(pg)[0]).to(dev)
        for _ in range(args.warmup):
            hm.sre_grad(g, 2.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            o, _ = hm.sre_grad(g, 2.0)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        print(json.dumps({"metric": "Pauli expectations/s (fwd+grad M_2)", "value": 4.0 ** n / (ms * 1e-3),
                          "unit": "Pauli expectations/s", "ms_per_step": ms, "steps": args.steps,
                          "config": {"workload": f"fwd+grad M_2, N={n} qubits, complex64 2-layer RY/RZ + CZ "
                                                 f"circuit state, seed {4000 + n}"},
                          "M2": float(o[0].item())}), flush=True)
        return
    if args.copy_mib:
        n = args.copy_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_mib, "launches": 5}), flush=True)
        return
    N = args.n
    seed = 2020
    psi = S.brickwall_haar(N, 2 * N, seed=seed)
    c64, c64w = S.to_c64_exact(psi)
    x = torch.from_numpy(c64).to(dev)
    ctx = hm.Context()
    if args.batch:
        ctx.batch_shifts(args.batch)
    if args.pipeline:
        ctx.set_option(hm.OPT_PIPELINE, args.pipeline)
    if args.lds_split:
        ctx.set_option(hm.OPT_LDS_SPLIT, args.lds_split)
    if args.row_bits:
        ctx.set_option(hm.OPT_ROW_BITS, args.row_bits)
    shifts = args.shifts if args.shifts else 2 ** N
    plan = None
    if not args.no_autotune and not (args.batch or args.pipeline or args.lds_split or args.row_bits):
        # One stream: with two, the row and column passes of different batches overlap and each
        # kernel's event-bracketed duration no longer measures that kernel (the two-stream plan is
        # reported among the secondary rows).
        ctx.set_option(hm.OPT_STREAMS, 1)
        t = time.perf_counter()
        plan = hm.autotune(x, 16384, ctx=ctx)
        plan["tune_s"] = round(time.perf_counter() - t, 3)

    def step():
        if args.shifts:
            return hm.sre_partial(x, (2.0,), 0, shifts, ctx=ctx)
        return hm.sre(x, (2.0,), ctx=ctx)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Kernel timing inside the timed region: hipEvents on the launch stream around every k-th launch
    # of each kernel family (k chosen so that a few hundred launches per family are timed).
    hm.profile_reset()
    hm.profile_enable(PROFILE_EVERY(N, shifts))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hm.profile_enable(False)
    prof = hm.profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    res = out.cpu().numpy()
    work = float(shifts) * float(2 ** N)  # Pauli expectations per step
    value = work / (ms * 1e-3)

    # dominant kernel (largest estimated device time per step) and its roofline
    est = {k: v[2] / max(v[1], 1) * v[0] for k, v in prof.items() if v[1] > 0}
    fam = max(est, key=est.get)
    launches, timed, tot_ms = prof[fam]
    t_launch = tot_ms * 1e-3 / timed
    vals_per_launch = work / 2.0 * args.steps / launches  # folded values per launch
    eff_plan = plan or {"batch_shifts": args.batch, "row_bits": args.row_bits, "lds_split": args.lds_split,
                        "pipeline": args.pipeline}
    roof = roofline(fam, N, vals_per_launch, t_launch, launches // args.steps, eff_plan)

    line = {
        "metric": "Pauli expectations/s for M_2 (N=20 qubits) & mana (N=12); fwd vs fwd+grad",
        "value": value, "unit": "Pauli expectations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "precision": "complex64 state, FP32 transforms, FP64 sums over Pauli strings and shifts",
        "config": {"workload": f"SRE M_2, N={N} qubits, complex64, brick-wall Haar circuit depth {2 * N}, seed {seed}, "
                               + (f"all 4^{N} Pauli strings" if not args.shifts else
                                  f"X-shifts [0, {shifts}) x 2^{N} Z-strings (profiling subset)"),
                   "parallelism": "none (1 GPU)"},
        "result": ({"M2": float(res[0]), "lost_norm": float(res[1]),
                    "error_vs_oracle": error_vs_oracle(float(res[0]), "sre_brickwall_n%d_d%d_seed%d_c64" % (N, 2 * N, seed))}
                   if not args.shifts else {"partial_sums": [float(v) for v in res]}),
        "kernel_ms_per_step": {k: round(est[k] / args.steps, 3) for k in est},
        "roofline": roof,
        "plan": plan,
    }

    if not args.no_secondary and not args.shifts:
        line["secondary"] = secondary(hm, S, torch, dev, psi, N)
        # the same workload with every plan option open to the autotuner (two streams included)
        c2 = hm.Context()
        p2 = hm.autotune(x, 16384, ctx=c2)
        dt, o = _timed(torch, lambda: hm.sre(x, (2.0,), ctx=c2))
        line["secondary"]["sre_fwd_c64_n%d_any_plan" % N] = {"value": 4.0 ** N / dt, "unit": "Pauli expectations/s",
                                                            "ms": dt * 1e3, "plan": p2}

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c64w, N)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
