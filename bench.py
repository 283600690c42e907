#!/usr/bin/env python3
"""Throughput of batched TFHE gate bootstrapping on one MI355X.

One step = one full pass of the hot path over one query: the 16-bit
two-dimensional interval validation of 1,024 records (4 comparators and 3
ANDs per record: 199,680 blind rotations, 134,144 key switches, 19 circuit
levels), every level a batched blind-rotation launch plus a batched
key-switching launch.  Inputs are resident in device memory before timing.

Prints one JSON line: blind rotations per second (value), the plain
one-gate-per-launch rate on the same GPU, per-query latency percentiles,
the live roofline of the blind-rotation kernel (HIP events around each of
its launches) and the CPU oracle timed on a bounded sample of host work.

Inputs are seeded and synthetic: evaluation keys and ciphertexts are uniform
32-bit words, which is how real LWE/RLWE samples are distributed; the work
per bootstrap does not depend on the values beyond that distribution.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one blind rotation (n = 630 external products, each
# 6 forward + 2 inverse 1024-point transforms of 5,120 butterflies and
# 12 x 1,024 pointwise products): 630 * (8 * 5120 + 12 * 1024).
MODMUL_PER_BR = 630 * (8 * 5120 + 12 * 1024)  # 33,546,240
# Integer VALU peak of MI355X: 256 CUs x 64 lanes/clock x 2.4 GHz, and the
# VALU operations of one Goldilocks multiply-and-reduce on gfx950 (4 32x32->64
# multiply-adds + 12 adds/selects for the 2^64 = 2^32 - 1 fold).
VALU_LANE_OPS = 256 * 64 * 2.4e9
OPS_PER_MODMUL = 16
PEAK_MODMUL = VALU_LANE_OPS / OPS_PER_MODMUL  # 2.4576e12 modmul/s

WORKLOADS = {
    "intv-1024": dict(mode="intv", M=1024, l=16, lS=0, d=2,
                      label="interval validation, 1024 records, 16-bit 2-D boxes"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * p / 100.0
    f = int(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def cpu_baseline(seconds: float, threads: int):
    """The oracle, as it stands, on host cores: AND gates on uniform inputs."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    from oracle import oracle as O
    from paper_2506_12761_amd import synth
    bk, ksk = synth.uniform_keys(0xB0B)
    keys = O.Keys(np.zeros(630, np.uint32), np.zeros(1024, np.uint32), bk, ksk)
    cts = synth.uniform_ciphertexts(0xB0B, "cpu", (2 * threads, 2))
    deadline = time.perf_counter() + seconds

    def worker(t):
        done = 0
        while time.perf_counter() < deadline:
            O.gate(keys, O.AND, cts[t % len(cts), 0], cts[t % len(cts), 1])
            done += 1
        return done

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        counts = list(ex.map(worker, range(threads)))
    el = time.perf_counter() - t0
    total = sum(counts)
    return {"value": total / el, "unit": "bootstraps/s", "cores": threads, "kind": "oracle",
            "sample": "%d AND gates (1 blind rotation + 1 key switch each) on uniform ciphertexts, "
                      "%d threads, %.1f s wall" % (total, threads, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="intv-1024", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-gates", type=int, default=32)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true", help="replay the level sequence as a HIP graph "
                    "(disables per-launch timing)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(records would shard across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2506_12761_amd import synth, vlp
    assert torch.cuda.is_available(), "no HIP device"
    wl = WORKLOADS[args.workload]
    mode, M, l, lS, d = wl["mode"], wl["M"], wl["l"], wl["lS"], wl["d"]

    log("generating synthetic keys and ciphertexts ...")
    bk, ksk = synth.uniform_keys(0x5EED0002)
    q_shape = (d, l) if mode != "idm" else (l,)
    loc_shape = {"intv": (M, d, 2, l), "cov": (M, d, l), "idm": (M, l)}[mode]
    query = synth.uniform_ciphertexts(0x5EED0002, "query", q_shape)
    db_loc = synth.uniform_ciphertexts(0x5EED0002, "db_loc", loc_shape)
    db_pay = synth.uniform_ciphertexts(0x5EED0002, "db_pay", (M, lS)) if lS else None

    ctx = vlp.Context(0)
    ks = ctx.load_keys(bk, ksk)
    d_q, d_loc = ctx.tensor(query), ctx.tensor(db_loc)
    d_pay = ctx.tensor(db_pay) if lS else None
    d_R = ctx.empty(lS, 631) if lS else None
    d_v = ctx.empty(M, 631)
    shape = vlp.make_shape(mode, M, l, lS, d)
    prog = vlp.vlp_program_create(ctx.ctx, ks, shape, d_q, d_loc, d_pay, d_R, d_v)
    counts = vlp.vlp_program_counts(ctx.ctx, prog)
    br_step, ks_step = counts["blind_rotations"], counts["key_switches"]
    log("program: %s" % counts)

    def step():
        vlp.vlp_program_reset(ctx.ctx, prog)
        vlp.vlp_program_run(ctx.ctx, prog, use_graph=args.graph)

    for _ in range(args.warmup):
        step()
    ctx.sync()
    log("warmup done")

    stream = ctx.stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    if not args.graph:
        vlp.vlp_profile_enable(ctx.ctx, True)
        vlp.vlp_profile_read(ctx.ctx)  # clear
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    prof = vlp.vlp_profile_read(ctx.ctx) if not args.graph else None
    vlp.vlp_profile_enable(ctx.ctx, False)
    value = br_step * args.steps / elapsed
    log("timed %d steps in %.3f s: %.1f blind rotations/s" % (args.steps, elapsed, value))

    # Plain form: one AND gate per launch, launched back to back.
    P = args.plain_gates
    a = ctx.tensor(synth.uniform_ciphertexts(7, "plain_a", (P,)))
    b = ctx.tensor(synth.uniform_ciphertexts(7, "plain_b", (P,)))
    o = ctx.empty(P, 631)
    vlp.vlp_gate(ctx.ctx, ks, "AND", a[0:1], b[0:1], None, o[0:1], 1)
    ctx.sync()
    tp0 = time.perf_counter()
    for g in range(P):
        vlp.vlp_gate(ctx.ctx, ks, "AND", a[g:g + 1], b[g:g + 1], None, o[g:g + 1], 1)
    ctx.sync()
    plain_rate = P / (time.perf_counter() - tp0)
    log("plain: %.1f blind rotations/s" % plain_rate)

    roofline = None
    if prof and prof["br"]["launches"]:
        br = prof["br"]
        avg_ms = br["ms"] / br["launches"]
        per_launch = MODMUL_PER_BR * br["items"] / br["launches"]
        achieved = per_launch / (avg_ms * 1e-3)
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_MODMUL / 1e12,
                    "unit": "Tmodmul/s", "frac": achieved / PEAK_MODMUL, "traffic": None,
                    "kernel": "br_kernel", "launches": br["launches"], "avg_launch_ms": avg_ms,
                    "ks_kernel_ms_share": prof["ks"]["ms"] / max(1e-9, prof["ks"]["ms"] + br["ms"])}

    cpu = None
    if not args.no_cpu_baseline:
        threads = max(1, min(16, os.cpu_count() or 1))
        log("cpu baseline: %d threads, %.0f s ..." % (threads, args.cpu_seconds))
        cpu = cpu_baseline(args.cpu_seconds, threads)

    out = {
        "metric": "bootstrapped gates/s (batched vs plain) at 1 GPU; PIR query p50/p99 latency",
        "value": value,
        "unit": "bootstraps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded uniform keys and ciphertexts)",
        "config": {"workload": wl["label"], "records": M, "l_I": l, "d": d, "l_S": lS,
                   "blind_rotations_per_step": br_step, "key_switches_per_step": ks_step,
                   "levels": counts["levels"], "graph": bool(args.graph)},
        "gates_per_s": counts["gates"] * args.steps / elapsed,
        "key_switches_per_s": ks_step * args.steps / elapsed,
        "plain_bootstraps_per_s": plain_rate,
        "speedup_batched_vs_plain": value / plain_rate,
        "query_latency_ms": {"p50": percentile(step_ms, 50), "p99": percentile(step_ms, 99)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    vlp.vlp_program_destroy(ctx.ctx, prog)
    ctx.close()


if __name__ == "__main__":
    main()
