#!/usr/bin/env python3
"""Throughput of batched TFHE gate bootstrapping on one MI355X.

One step = one full pass of the hot path over one query: the 16-bit
two-dimensional interval validation of 1,024 records (4 comparators and 3
ANDs per record: 199,680 blind rotations, 134,144 key switches, 19 circuit
levels), every level launched as rounds of 1,024 blind rotations (two
wavefronts each, one per prime) plus one batched key-switching launch.
Inputs are resident in device memory before timing.

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
# Integer VALU peak of MI355X for that unit of work: 256 CUs x 64 lanes x
# 2.4 GHz = 39.3 T VALU lane-instructions/s, divided by the instructions of
# one exact modular multiplication.  The products need a modulus above
# 2^51.6; the cheapest exact form on the 32-bit VALU is one residue
# butterfly per prime of a two-prime RNS (26-bit primes), each a signed
# Shoup product (v_mul_hi_i32, v_mul_lo_u32, v_mad_u64_u32) plus one add and
# one subtract: 2 x 5 = 10 instructions.  (A 64-bit Goldilocks multiply
# takes about 16.)
VALU_LANE_OPS = 256 * 64 * 2.4e9
OPS_PER_RESIDUE_BUTTERFLY = 5
RESIDUES_PER_MODMUL = 2
PEAK_MODMUL = VALU_LANE_OPS / (OPS_PER_RESIDUE_BUTTERFLY * RESIDUES_PER_MODMUL)  # 3.932e12 modmul/s

# A workload is one or more programs run together (their levels merged).
# HBM-side traffic of the blind-rotation kernel per launch on the default
# workload, from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE;
# copy-calibrated), valid only for the kernel sources it was measured on
# (their sha256 prefix) and the launch shape it was measured with.
TRAFFIC_MEASURED = {"kernel_sha": "749f0fca55ff871c", "bytes_per_launch": 5.16355e+08,
                    "launch": {"br_waves_per_rotation": 0, "br_rotations_per_block": 4, "br_blocks_per_cu": 1,
                               "ks_gates_per_block": 512}}
KERNEL_SOURCES = ("kernels.hip", "wave_ntt.h", "rns.h", "vlp_api.cpp")


def kernel_sha() -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_2506_12761_amd", "csrc")
    return hashlib.sha256(b"".join(open(os.path.join(d, n), "rb").read() for n in KERNEL_SOURCES)).hexdigest()[:16]


WORKLOADS = {
    "intv-1024": dict(label="interval validation, 1024 records, 16-bit 2-D boxes",
                      programs=[dict(mode="intv", M=1024, l=16, lS=0, d=2)]),
    # 4,096 cells, each an equality cell (CoV, depth 7) or a range cell (IntV,
    # depth 23) by a seeded fair coin; both kinds share every launch.
    "mixed-4096": dict(label="4096 20-bit cells, equality or range per cell (seeded coin)",
                       programs="mixed"),
    "idm-65536": dict(label="identifier match, 65536 records, 32-bit ids, 64-bit payload selection + XOR tree",
                      programs=[dict(mode="idm", M=65536, l=32, lS=64, d=1)]),
    "interval-8bit": dict(label="one 8-bit value against one interval (49 bootstraps)",
                          programs=[dict(mode="intv", M=1, l=8, lS=0, d=1)]),
}


# The identifier-match workload reported beside the main line: one full query
# over 65,536 records (32-bit identifiers, 64 payload bits, pairwise XOR tree).
CONFIG4 = dict(mode="idm", M=65536, l=32, lS=64, d=1)


def device_inputs(ctx, spec, seed):
    """Query, database and output buffers of one program, the ciphertexts as
    uniform 32-bit words drawn on the device from a seeded generator."""
    from paper_2506_12761_amd.autotune import uniform_words
    mode, M, l, lS, d = spec["mode"], spec["M"], spec["l"], spec["lS"], spec["d"]
    q_shape = (d, l) if mode != "idm" else (l,)
    loc_shape = {"intv": (M, d, 2, l), "cov": (M, d, l), "idm": (M, l)}[mode]
    d_q = uniform_words(ctx, q_shape + (631,), seed)
    d_loc = uniform_words(ctx, loc_shape + (631,), seed + 1)
    d_pay = uniform_words(ctx, (M, lS, 631), seed + 2) if lS else None
    d_R = ctx.empty(lS, 631) if lS else None
    return d_q, d_loc, d_pay, d_R, ctx.empty(M, 631)


def br_roofline(prof):
    """Blind-rotation kernel rate against the derived integer peak, from the
    library's per-launch HIP-event timing, and the key-switching share."""
    br, ks = prof["br"], prof["ks"]
    avg_ms = br["ms"] / br["launches"]
    achieved = MODMUL_PER_BR * br["items"] / br["launches"] / (avg_ms * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_MODMUL / 1e12, "unit": "Tmodmul/s",
            "frac": achieved / PEAK_MODMUL, "launches": br["launches"], "avg_launch_ms": avg_ms,
            "ks_kernel_ms_share": ks["ms"] / max(1e-9, ks["ms"] + br["ms"]),
            "ks_launches": ks["launches"], "ks_ms": ks["ms"]}


def config4_query(ctx, ks, seed=0x5EED0004):
    """One full identifier-match query (Alg. 3: equality of 32-bit
    identifiers, Alg. 9 selection of 64 payload bits, pairwise XOR
    aggregation) over 65,536 records, inputs resident on the device; timed
    with HIP events on the library's stream, level by level."""
    import torch

    from paper_2506_12761_amd import vlp
    spec = dict(CONFIG4)
    bufs = device_inputs(ctx, spec, seed)
    shape = vlp.make_shape(spec["mode"], spec["M"], spec["l"], spec["lS"], spec["d"])
    t0 = time.perf_counter()
    prog = vlp.vlp_program_create(ctx.ctx, ks, shape, *bufs)
    build_s = time.perf_counter() - t0
    counts = vlp.vlp_program_counts(ctx.ctx, prog)
    log("config 4: %s, program built in %.1f s" % (counts, build_s))
    vlp.vlp_profile_enable(ctx.ctx, True)
    vlp.vlp_profile_read(ctx.ctx)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.sync()
    t0 = time.perf_counter()
    e0.record(ctx.stream)
    level = 0
    while True:
        rem = vlp.vlp_step(ctx.ctx, [prog])
        level += 1
        ctx.sync()
        log("config 4: level %d of %d done, %.1f s" % (level, counts["levels"], time.perf_counter() - t0))
        if not rem:
            break
    e1.record(ctx.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    prof = vlp.vlp_profile_read(ctx.ctx)
    vlp.vlp_profile_enable(ctx.ctx, False)
    vlp.vlp_program_destroy(ctx.ctx, prog)
    del bufs
    torch.cuda.empty_cache()
    return {"workload": "identifier match, 65536 records, 32-bit ids, 64-bit payload selection + pairwise XOR tree",
            "programs": [spec], "value": counts["blind_rotations"] / (ms * 1e-3), "unit": "bootstraps/s",
            "s_per_query": ms * 1e-3, "gates_per_s": counts["gates"] / (ms * 1e-3),
            "blind_rotations": counts["blind_rotations"], "key_switches": counts["key_switches"],
            "levels": counts["levels"], "program_build_s": build_s, "roofline": br_roofline(prof)}


def mixed_programs(cells=4096, seed=0x5EED0003):
    import synth
    coin = synth.bits(synth.stream(seed, "cell_kind"), (cells,))
    n_eq = int(coin.sum())
    return [dict(mode="cov", M=n_eq, l=20, lS=0, d=2), dict(mode="intv", M=cells - n_eq, l=20, lS=0, d=2)]


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
    import synth
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
    # One thread, gates one after another: the mean time of one gate.
    single, t1 = 0, time.perf_counter()
    while single < 2 or (single < 20 and time.perf_counter() - t1 < 3.0):
        O.gate(keys, O.AND, cts[single % len(cts), 0], cts[single % len(cts), 1])
        single += 1
    single_ms = (time.perf_counter() - t1) * 1e3 / single
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": total / el, "unit": "bootstraps/s", "cores": threads, "kind": "oracle",
            "sample": "%d AND gates (1 blind rotation + 1 key switch each) on uniform ciphertexts, "
                      "%d threads, %.1f s wall" % (total, threads, el),
            "single_thread_ms_per_gate": single_ms, "single_thread_gates": single,
            "host": {"cpu_model": model, "cpus_available": avail, "cpu_count": os.cpu_count()}}


# Query shapes of the paper's four datasets (Table 3: records M, interval or
# identifier bits l_I, payload bits l_S), with the modes Table 4 runs on them.
TABLE3 = [("covid-kor", "intv", 9, 16, 9), ("covid-kor", "idm", 9, 16, 9), ("covid-usa", "intv", 58, 16, 22),
          ("covid-usa", "idm", 58, 16, 22), ("gdacs", "cov", 9, 16, 16), ("weather-usa", "idm", 304, 16, 128)]


def table3_bench(args):
    """One full query (Algorithm 3) per Table-3 shape, baseline circuits
    (Alg. 7 AND chain, Alg. 10 XOR chain), optimized circuits (Alg. 11/12,
    XOR tree) and optimized circuits with 16-input XOR aggregation; synthetic
    uniform data of those shapes; latency per query."""
    import synth
    from paper_2506_12761_amd import vlp
    ctx = vlp.Context(0)
    bk, ksk = synth.uniform_keys(0x5EED0006)
    ks = ctx.load_keys(bk, ksk)
    rows = []
    for k, (name, mode, M, l, lS) in enumerate(TABLE3):
        d = 1 if mode == "idm" else 2
        qs = (d, l) if mode != "idm" else (l,)
        ls = {"intv": (M, d, 2, l), "cov": (M, d, l), "idm": (M, l)}[mode]
        q = ctx.tensor(synth.uniform_ciphertexts(k, "q", qs))
        loc = ctx.tensor(synth.uniform_ciphertexts(k, "l", ls))
        pay = ctx.tensor(synth.uniform_ciphertexts(k, "p", (M, lS)))
        R, v = ctx.empty(lS, 631), ctx.empty(M, 631)
        rec = {"dataset": name, "mode": mode, "M": M, "l_I": l, "l_S": lS}
        for opt, agg_k in ((False, 0), (True, 0), (True, 16)):
            sh = vlp.make_shape(mode, M, l, lS, d, opt, agg_k)
            plan = vlp.vlp_plan_counts(sh)
            vlp.vlp_evaluate(ctx.ctx, ks, sh, q, loc, pay, R, v)  # build + warm
            ctx.sync()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                vlp.vlp_evaluate(ctx.ctx, ks, sh, q, loc, pay, R, v)
            ctx.sync()
            dt = (time.perf_counter() - t0) / args.steps
            key = "base" if not opt else ("opt" if not agg_k else "opt_xor16")
            rec[key] = {"s": dt, "blind_rotations": plan["blind_rotations"], "levels": plan["levels"]}
        rec["speedup_opt_vs_base"] = rec["base"]["s"] / rec["opt"]["s"]
        rec["speedup_opt_xor16_vs_base"] = rec["base"]["s"] / rec["opt_xor16"]["s"]
        log(json.dumps(rec))
        rows.append(rec)
    print(json.dumps({"metric": "PIR query latency per Table-3 shape, baseline vs optimized circuits, 1 GPU",
                      "unit": "s", "higher_is_better": False, "data": "synthetic (uniform words of the dataset shapes)",
                      "steps": args.steps, "rows": rows}), flush=True)
    ctx.close()


def server_enc_bench(args):
    """ServerEnc (Alg. 2) of the identifier-match database of 65,536 records
    (32-bit identifiers, 64 payload bits: 6,291,456 ciphertexts, 15.9 GB of
    public key) from a device-resident public key, out of place (the HBM
    roofline case: every word read once and written once) and in place (only
    the body words change).  Public key and data are seeded synthetic words."""
    import torch

    from paper_2506_12761_amd import vlp
    M, l, lS = 65536, 32, 64
    ctx = vlp.Context(0)
    dev = ctx.device
    g = torch.Generator(device=dev)
    g.manual_seed(0x5EED0007)
    with torch.cuda.stream(ctx.stream):
        pk_loc = torch.empty((M, l, 631), dtype=torch.int32, device=dev).random_(generator=g)
        pk_pay = torch.empty((M, lS, 631), dtype=torch.int32, device=dev).random_(generator=g)
        loc = torch.randint(0, 2**31 - 1, (M,), dtype=torch.int64, device=dev, generator=g)
        pay = torch.randint(0, 2, (M, lS), dtype=torch.uint8, device=dev, generator=g)
        out_loc, out_pay = torch.empty_like(pk_loc), torch.empty_like(pk_pay)
    ctx.sync()
    sh = vlp.make_shape("idm", M, l, lS, 1)
    count = M * (l + lS)
    res = {}
    for form, (o_loc, o_pay) in (("copy", (out_loc, out_pay)), ("inplace", (pk_loc, pk_pay))):
        for _ in range(max(1, args.warmup)):
            vlp.vlp_server_encrypt(ctx.ctx, sh, pk_loc, pk_pay, loc, pay, o_loc, o_pay)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(args.steps):
            vlp.vlp_server_encrypt(ctx.ctx, sh, pk_loc, pk_pay, loc, pay, o_loc, o_pay)
        e1.record(ctx.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res[form] = {"ms_per_call": ms, "ciphertexts_per_s": count / (ms * 1e-3)}
    # A plain device-to-device copy of the same public key, the practical ceiling.
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(ctx.stream):
        out_loc.copy_(pk_loc)
        out_pay.copy_(pk_pay)
        e0.record(ctx.stream)
        for _ in range(args.steps):
            out_loc.copy_(pk_loc)
            out_pay.copy_(pk_pay)
        e1.record(ctx.stream)
    e1.synchronize()
    copy_ms = e0.elapsed_time(e1) / args.steps
    res["device_copy"] = {"ms_per_call": copy_ms, "GB_per_s": count * 631 * 4 * 2 / (copy_ms * 1e-3) / 1e9}
    alg = count * 631 * 4 * 2 + M * 8 + M * lS  # words read + written, values, payload bytes
    gbs = alg / (res["copy"]["ms_per_call"] * 1e-3) / 1e9
    print(json.dumps({
        "metric": "ServerEnc (Alg. 2) ciphertexts/s at 1 GPU, device-resident public key",
        "value": res["copy"]["ciphertexts_per_s"], "unit": "ciphertexts/s", "higher_is_better": True,
        "steps": args.steps, "warmup": args.warmup, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "identifier-match database, 65536 records, 32-bit ids, 64 payload bits",
                   "ciphertexts": count, "public_key_bytes": count * 631 * 4},
        "forms": res,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                     "traffic": None, "algorithmic_bytes_per_call": alg}}), flush=True)
    ctx.close()


# Key switching on the matrix cores: per gate, a product of the one-hot digit
# matrix (1,024 coefficients x 8 levels x 4 digit values = 32,768 columns)
# with the key's 4 byte planes of 640 (631 padded) words, 2 ops per
# multiply-add; dense int8 peak of MI355X 5.0 POP/s.  The method's own work is
# at most 8,192 row subtractions of 631 words (5,169,152 adds; 3/4 of that on
# average for uniform digits).
KS_MFMA_OPS = 2 * 1024 * 8 * 4 * 640 * 4  # 167,772,160
PEAK_INT8_OPS = 5.0e15
KS_ADDS_MAX = 1024 * 8 * 631


def keyswitch_bench(args):
    """vlp_keyswitch over `--ks-gates` uniform LWE_N ciphertexts (one launch
    of up to 16,384 gates per chunk), timed with HIP events on the library's
    stream; rate against the int8 matrix-core peak."""
    import torch

    from paper_2506_12761_amd import vlp
    from paper_2506_12761_amd.autotune import uniform_words
    ctx = vlp.Context(0)
    ks = ctx.load_keys(uniform_words(ctx, (630, 6, 2, 1024), 21), uniform_words(ctx, (1024, 8, 4, 631), 22))
    if args.ks_gates_per_block:
        t = vlp.vlp_get_tuning(ctx.ctx)
        vlp.vlp_set_tuning(ctx.ctx, t.br_rotations_per_block, t.br_blocks_per_cu, args.ks_gates_per_block,
                           t.br_waves_per_rotation)
    B = args.ks_gates
    d_in = uniform_words(ctx, (B, 1025), 23)
    d_out = ctx.empty(B, 631)
    for _ in range(max(1, args.warmup)):
        vlp.vlp_keyswitch(ctx.ctx, ks, d_in, d_out, B)
    ctx.sync()
    vlp.vlp_profile_enable(ctx.ctx, True)
    vlp.vlp_profile_read(ctx.ctx)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    for _ in range(args.steps):
        vlp.vlp_keyswitch(ctx.ctx, ks, d_in, d_out, B)
    e1.record(ctx.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    prof = vlp.vlp_profile_read(ctx.ctx)
    rate = B / (ms * 1e-3)
    ops = KS_MFMA_OPS * rate
    t = vlp.vlp_get_tuning(ctx.ctx)
    print(json.dumps({
        "metric": "key switches/s at 1 GPU (LWE_1024 -> LWE_630, base 2^2, 8 levels)", "value": rate,
        "unit": "key switches/s", "higher_is_better": True, "steps": args.steps, "warmup": args.warmup,
        "dtype": "u32 (int8 matrix-core planes)", "data": "synthetic (seeded uniform key and ciphertexts)",
        "config": {"workload": "%d key switches per call" % B, "ks_gates_per_block": t.ks_gates_per_block},
        "ms_per_call": ms, "timed_calls_ms_per_call": prof["ks"]["ms"] / max(1, args.steps),
        "roofline": {"bound": "mfma", "achieved": ops / 1e12, "peak": PEAK_INT8_OPS / 1e12, "unit": "TOP/s (int8)",
                     "frac": ops / PEAK_INT8_OPS, "traffic": None, "mfma_ops_per_key_switch": KS_MFMA_OPS},
        "algorithmic": {"adds_per_s_max": KS_ADDS_MAX * rate, "adds_per_s_mean": 0.75 * KS_ADDS_MAX * rate,
                        "key_bytes_per_call": 83886080 * -(-B // 16384)},
    }), flush=True)
    ctx.close()


class SkipIdleClock:
    """Wall clock that skips the device's idle gaps: when no request is active
    the server's wait for the next arrival advances this clock instead of
    sleeping.  Nothing runs during such a gap, so no latency changes."""

    def __init__(self):
        self.offset = 0.0

    def __call__(self):
        return time.perf_counter() + self.offset

    def sleep(self, dt):
        self.offset += max(0.0, dt)


def serve_bench(args):
    """Poisson stream of PIR queries (config 5): modes uniform over {IntV
    16-bit, CoV 20-bit, IdM 32-bit}, records log-uniform in [min, max], 64
    payload bits, full Alg. 3 with the pairwise XOR aggregation, one client
    (own seeded keys) per request.  Keys and the request's encrypted database
    are drawn on the device when the request is admitted (they count against
    the HBM budget while it runs); latency runs from arrival to the result R
    copied to the host.  Arrival rate = load x the calibrated saturated rate
    of the stream's mean query."""
    import numpy as np
    import torch

    import synth
    from paper_2506_12761_amd import vlp
    from paper_2506_12761_amd.autotune import uniform_words
    from paper_2506_12761_amd.serve import GpuExecutor, Request, poisson_arrivals, serve
    ctx = vlp.Context(0)
    g = synth.stream(0x5EED0005, "serve")
    kinds = [("intv", 16, 2), ("cov", 20, 2), ("idm", 32, 1)]
    reqs = []
    for rid in range(args.requests):
        mode, l, d = kinds[int(g.integers(0, 3))]
        M = int(2 ** g.uniform(np.log2(args.min_records), np.log2(args.max_records)))
        reqs.append(Request(rid, rid, mode, M, l, 64, d, arrival=0.0))

    def plan_br(r):
        return vlp.vlp_plan_counts(vlp.make_shape(r.mode, r.M, r.l_I, r.l_S, r.d))["blind_rotations"]

    def keys_of(client):
        return (uniform_words(ctx, (630, 6, 2, 1024), 0x5EED0500 + 2 * client),
                uniform_words(ctx, (1024, 8, 4, 631), 0x5EED0501 + 2 * client))

    def inputs_of(r):
        shp = (r.d, r.l_I) if r.mode != "idm" else (r.l_I,)
        lshape = {"intv": (r.M, r.d, 2, r.l_I), "cov": (r.M, r.d, r.l_I), "idm": (r.M, r.l_I)}[r.mode]
        return {"query": uniform_words(ctx, shp + (631,), 0x5EED1000 + 4 * r.rid),
                "db_loc": uniform_words(ctx, lshape + (631,), 0x5EED1001 + 4 * r.rid),
                "db_pay": uniform_words(ctx, (r.M, r.l_S, 631), 0x5EED1002 + 4 * r.rid),
                "R": ctx.empty(r.l_S, 631), "v": ctx.empty(r.M, 631)}

    # Saturated rate: blind rotations per second of one merged 1,024-record query.
    cal = device_inputs(ctx, dict(mode="intv", M=1024, l=16, lS=0, d=2), 0x5EED0600)
    bk, ksk = keys_of(10**6)
    ks = ctx.load_keys(bk, ksk)
    del bk, ksk
    sh = vlp.make_shape("intv", 1024, 16, 0, 2)
    vlp.vlp_evaluate(ctx.ctx, ks, sh, *cal)
    ctx.sync()
    t0 = time.perf_counter()
    vlp.vlp_evaluate(ctx.ctx, ks, sh, *cal)
    ctx.sync()
    br_rate = vlp.vlp_plan_counts(sh)["blind_rotations"] / (time.perf_counter() - t0)
    ctx.drop_keys(ks)
    del cal
    torch.cuda.empty_cache()
    mean_br = sum(plan_br(r) for r in reqs) / len(reqs)
    rate = args.arrival_rate or args.load * br_rate / mean_br
    for r, t in zip(reqs, poisson_arrivals(rate, len(reqs), g)):
        r.arrival = t
    budget = int(args.hbm_budget_gb * 2**30)
    log("serving %d requests, rate %.5f/s (load %.2f of %.0f bootstraps/s, mean query %.0f bootstraps), "
        "policy %s, step cap %s, budget %.0f GiB" % (len(reqs), rate, args.load, br_rate, mean_br, args.policy,
                                                      args.step_cap, args.hbm_budget_gb))
    ex = GpuExecutor(ctx, key_factory=keys_of, input_factory=inputs_of, budget=budget)
    clk = SkipIdleClock()
    st = serve(reqs, ex, clock=clk, sleep=clk.sleep, log=log, policy=args.policy,
               step_cap=args.step_cap or None)
    total_br = sum(plan_br(r) for r in st["requests"])
    busy_s = st["wall_s"]
    out = {
        "metric": "PIR query latency under Poisson load (continuous batching), 1 GPU",
        "value": st["p50_ms"], "unit": "ms (p50)", "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
        "max_ms": max(r.latency for r in st["requests"]) * 1e3,
        "higher_is_better": False, "queries_per_s": st["queries_per_s"],
        "bootstraps_per_s_during_serving": total_br / busy_s, "n_gpus": 1,
        "queries": st["queries"], "steps": st["steps"], "max_active": st["max_active"],
        "budget_rejections": st["budget_rejections"], "arrival_rate_per_s": rate, "load": args.load,
        "calibrated_bootstraps_per_s": br_rate, "mean_query_bootstraps": mean_br,
        "policy": args.policy, "step_cap": args.step_cap or None, "hbm_budget_bytes": budget,
        "clock": "idle gaps between arrivals skipped (device idle; latencies unchanged)",
        "dtype": "u32", "data": "synthetic (seeded uniform keys and ciphertexts, drawn on the device at admission)",
        "config": {"workload": "serving: modes uniform over IntV-16/CoV-20/IdM-32, records log-uniform "
                               "%d..%d, 64 payload bits, one client per request" % (args.min_records,
                                                                                     args.max_records),
                   "per_request": [(r.mode, r.M, plan_br(r), round(r.arrival, 2), round(r.latency * 1e3, 1))
                                   for r in st["requests"]]},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


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
    ap.add_argument("--records", type=int, default=0, help="override the record count of every program")
    ap.add_argument("--agg-k", type=int, default=0, help="aggregate with k-input XORs (2..16) where l_S > 0")
    ap.add_argument("--tuned", action="store_true", help="apply the cached autotuner result")
    ap.add_argument("--br-rotations-per-block", type=int, default=0,
                    help="blind rotations per workgroup (1, 2, 4; 8 with one wavefront per rotation)")
    ap.add_argument("--br-blocks", type=int, default=0, help="blind-rotation workgroups per CU the grid is sized for")
    ap.add_argument("--ks-gates-per-block", type=int, default=0, choices=(0, 128, 256, 512),
                    help="most gates a key-switching workgroup takes (0: library default)")
    ap.add_argument("--br-waves-per-rotation", type=int, default=-1, choices=(-1, 0, 1, 2, 4),
                    help="wavefronts per blind rotation (0: automatic by launch size)")
    ap.add_argument("--serve", action="store_true", help="run the serving experiment instead")
    ap.add_argument("--table3", action="store_true", help="replay the paper's dataset shapes instead")
    ap.add_argument("--server-enc", action="store_true", help="time ServerEnc of a 65,536-record database instead")
    ap.add_argument("--progress", action="store_true", help="wait for and report every circuit level")
    ap.add_argument("--requests", type=int, default=50)
    ap.add_argument("--min-records", type=int, default=256)
    ap.add_argument("--max-records", type=int, default=16384)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate as a fraction of the saturated rate")
    ap.add_argument("--arrival-rate", type=float, default=0.0, help="queries/s (overrides --load)")
    ap.add_argument("--policy", default="srpt", choices=("all", "srpt"),
                    help="which admitted queries a step advances (serve.py)")
    ap.add_argument("--step-cap", type=int, default=65536, help="most blind rotations per step under srpt")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0, help="device memory the server may hold")
    ap.add_argument("--keyswitch", action="store_true", help="time key switching alone instead")
    ap.add_argument("--ks-gates", type=int, default=16384, help="key switches per call with --keyswitch")
    ap.add_argument("--graph-steps", type=int, default=3,
                    help="after the timed steps, time this many HIP-graph replays of the same program (0: none)")
    ap.add_argument("--no-config4", action="store_true",
                    help="skip the 65,536-record identifier-match query reported beside the main line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device with a plain copy kernel (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(records would shard across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        return serve_bench(args)
    if args.table3:
        return table3_bench(args)
    if args.server_enc:
        return server_enc_bench(args)
    if args.keyswitch:
        return keyswitch_bench(args)
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.arange(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return

    import torch

    from paper_2506_12761_amd import vlp
    assert torch.cuda.is_available(), "no HIP device"
    wl = WORKLOADS[args.workload]
    specs = mixed_programs() if wl["programs"] == "mixed" else [dict(p) for p in wl["programs"]]
    if args.records:
        for p in specs:
            p["M"] = args.records

    from paper_2506_12761_amd.autotune import uniform_words
    log("generating synthetic keys and ciphertexts on the device ...")
    ctx = vlp.Context(0)
    ks = ctx.load_keys(uniform_words(ctx, (630, 6, 2, 1024), 0x5EED0002),
                       uniform_words(ctx, (1024, 8, 4, 631), 0x5EED0012))
    if args.tuned:
        from paper_2506_12761_amd import autotune
        log("cached tuning applied: %s" % autotune.load_cached(ctx, args.workload))
    if args.br_rotations_per_block or args.br_blocks or args.br_waves_per_rotation >= 0 or args.ks_gates_per_block:
        t = vlp.vlp_get_tuning(ctx.ctx)
        vlp.vlp_set_tuning(ctx.ctx, args.br_rotations_per_block or t.br_rotations_per_block,
                           args.br_blocks or t.br_blocks_per_cu,
                           args.ks_gates_per_block or t.ks_gates_per_block,
                           args.br_waves_per_rotation if args.br_waves_per_rotation >= 0 else t.br_waves_per_rotation)
    t = vlp.vlp_get_tuning(ctx.ctx)
    launch = {"br_waves_per_rotation": t.br_waves_per_rotation, "br_rotations_per_block": t.br_rotations_per_block,
              "br_blocks_per_cu": t.br_blocks_per_cu, "ks_gates_per_block": t.ks_gates_per_block}
    progs, keep = [], []
    for k, p in enumerate(specs):
        bufs = device_inputs(ctx, p, 0x5EED0100 + 16 * k)
        keep.append(bufs)
        shape = vlp.make_shape(p["mode"], p["M"], p["l"], p["lS"], p["d"], True, args.agg_k if p["lS"] else 0)
        progs.append(vlp.vlp_program_create(ctx.ctx, ks, shape, *bufs))
    counts = [vlp.vlp_program_counts(ctx.ctx, pr) for pr in progs]
    br_step = sum(c["blind_rotations"] for c in counts)
    ks_step = sum(c["key_switches"] for c in counts)
    gates_step = sum(c["gates"] for c in counts)
    levels = max(c["levels"] for c in counts)
    log("programs: %s" % counts)

    def step():
        for pr in progs:
            vlp.vlp_program_reset(ctx.ctx, pr)
        if args.progress:  # level by level, waiting for each (long workloads report as they go)
            lvl = 0
            while True:
                rem = vlp.vlp_step(ctx.ctx, progs)
                ctx.sync()
                lvl += 1
                log("level %d done" % lvl)
                if not rem:
                    break
        elif len(progs) == 1:
            vlp.vlp_program_run(ctx.ctx, progs[0], use_graph=args.graph)
        else:
            while vlp.vlp_step(ctx.ctx, progs):
                pass

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

    # The same step replayed as a HIP graph (the program's whole level sequence
    # captured once; a reset and one graph launch per step), timed beside it.
    graph_replay = None
    if len(progs) == 1 and not args.graph and not args.progress and args.graph_steps > 0:
        vlp.vlp_program_reset(ctx.ctx, progs[0])
        vlp.vlp_program_run(ctx.ctx, progs[0], use_graph=True)  # captures the graph
        ctx.sync()
        evg = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.graph_steps)]
        tg0 = time.perf_counter()
        for k in range(args.graph_steps):
            evg[k][0].record(stream)
            vlp.vlp_program_reset(ctx.ctx, progs[0])
            vlp.vlp_program_run(ctx.ctx, progs[0], use_graph=True)
            evg[k][1].record(stream)
        ctx.sync()
        g_elapsed = time.perf_counter() - tg0
        graph_replay = {"steps": args.graph_steps, "ms_per_step": g_elapsed * 1e3 / args.graph_steps,
                        "value": br_step * args.graph_steps / g_elapsed,
                        "device_ms_per_step": [a.elapsed_time(b) for a, b in evg],
                        "vs_launches": elapsed / args.steps / (g_elapsed / args.graph_steps)}
        log("graph replay: %.1f ms per step (launches: %.1f)" % (graph_replay["ms_per_step"], elapsed * 1e3 / args.steps))

    # Plain form: one AND gate per launch, launched back to back.
    P = args.plain_gates
    a = uniform_words(ctx, (P, 631), 7)
    b = uniform_words(ctx, (P, 631), 8)
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
        # Algorithmic bytes per launch: the transformed key once (61,931,520 B), the two
        # input ciphertexts (2 x 2,524 B) and the extracted output (4,100 B) per rotation.
        alg_bytes = 61931520 + (2 * 2524 + 4100) * br["items"] / br["launches"]
        traffic = None
        if (args.workload == "intv-1024" and TRAFFIC_MEASURED["kernel_sha"] == kernel_sha()
                and TRAFFIC_MEASURED["launch"] == launch):
            traffic = TRAFFIC_MEASURED["bytes_per_launch"]
        roofline = br_roofline(prof)
        achieved = roofline["achieved"] * 1e12
        roofline.update({"traffic": traffic, "traffic_unit": "B per launch", "algorithmic_bytes_per_launch": alg_bytes,
                         "kernel": {0: "br2_kernel (br4_kernel for short rounds)", 1: "br_kernel", 2: "br2_kernel",
                                    4: "br4_kernel"}[launch["br_waves_per_rotation"]]})
        # Beside the derived peak: the measured rate of the transforms' own residue
        # butterflies (register-resident, every CU busy, the 6:2 forward:inverse mix of
        # a CMux), two of which make one modular multiplication.
        mp = vlp.vlp_measure_modmul_peak(0)
        roofline["peak_measured"] = mp["mixed"] / RESIDUES_PER_MODMUL / 1e12
        roofline["frac_of_peak_measured"] = achieved / (mp["mixed"] / RESIDUES_PER_MODMUL)
        log("measured residue-butterfly peak: %.3f T/s forward, %.3f T/s inverse, %.3f T/s mixed"
            % (mp["fwd"] / 1e12, mp["inv"] / 1e12, mp["mixed"] / 1e12))

    config4 = None
    if not args.no_config4 and args.workload != "idm-65536":
        for pr in progs:
            vlp.vlp_program_destroy(ctx.ctx, pr)
        progs = []
        del keep
        torch.cuda.empty_cache()
        config4 = config4_query(ctx, ks)
        log("config 4: %.1f s per query, %.0f bootstraps/s, blind rotation %.1f%% of the derived peak, "
            "key switching %.1f%% of kernel time" % (config4["s_per_query"], config4["value"],
                                                     100 * config4["roofline"]["frac"],
                                                     100 * config4["roofline"]["ks_kernel_ms_share"]))

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
        "dtype": "u32",
        "data": "synthetic (seeded uniform keys and ciphertexts)",
        "config": {"workload": wl["label"], "programs": specs, "agg_k": args.agg_k,
                   "blind_rotations_per_step": br_step, "key_switches_per_step": ks_step,
                   "levels": levels, "graph": bool(args.graph), "launch": launch},
        "gates_per_s": gates_step * args.steps / elapsed,
        "key_switches_per_s": ks_step * args.steps / elapsed,
        "plain_bootstraps_per_s": plain_rate,
        "speedup_batched_vs_plain": value / plain_rate,
        "query_latency_ms": {"p50": percentile(step_ms, 50), "p99": percentile(step_ms, 99)},
        "roofline": roofline,
        "graph_replay": graph_replay,
        "cpu_baseline": cpu,
        "config4": config4,
    }
    print(json.dumps(out), flush=True)
    for pr in progs:
        vlp.vlp_program_destroy(ctx.ctx, pr)
    ctx.close()


if __name__ == "__main__":
    main()
