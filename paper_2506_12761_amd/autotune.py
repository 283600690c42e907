"""Autotuner for the batched kernels' launch shape, with a JSON cache.

Two sweeps:
  * launch shape -- wavefronts per blind rotation (1, 2, 4 or automatic),
    rotations per workgroup, workgroups per CU a launch is sized for, gates
    per key-switching workgroup -- timed
    on a caller-supplied program (one full pass each), the fastest is set on
    the context and cached per device and workload;
  * batch size -- blind rotations per launch from 256 to 16,384, timed with
    the elementwise bootstrap call, giving the throughput curve that tells how
    many independent gates a launch needs to fill the device.
"""
from __future__ import annotations

import json
import os
import time

from . import vlp

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")

# (wavefronts per rotation, rotations per workgroup, workgroups per CU, gates
# per key-switching workgroup); 0 wavefronts per rotation = automatic by launch size
SHAPES = ([(1, w, b, k) for w in (1, 2, 4, 8) for b in (1, 2, 4) for k in (4, 8) if w * b <= 8]
          + [(r, q, b, k) for r in (0, 2) for (q, b) in ((1, 4), (2, 2), (4, 1)) for k in (4, 8, 16)]
          + [(4, 1, b, k) for b in (1, 2) for k in (4, 8)])


def _apply(ctx, best: dict) -> None:
    vlp.vlp_set_tuning(ctx.ctx, best["br_rotations_per_block"], best["br_blocks_per_cu"], best["ks_gates_per_block"],
                       best.get("br_waves_per_rotation", 0))


def _time_program(ctx, prog) -> float:
    vlp.vlp_sync(ctx.ctx)
    t0 = time.perf_counter()
    vlp.vlp_program_reset(ctx.ctx, prog)
    vlp.vlp_program_run(ctx.ctx, prog, use_graph=False)
    vlp.vlp_sync(ctx.ctx)
    return time.perf_counter() - t0


def tune_launch(ctx, prog, shapes=SHAPES, log=None) -> dict:
    """Times `prog` under each launch shape; sets and returns the best."""
    results = []
    for (r, w, b, k) in shapes:
        vlp.vlp_set_tuning(ctx.ctx, w, b, k, r)
        dt = _time_program(ctx, prog)
        results.append({"br_waves_per_rotation": r, "br_rotations_per_block": w, "br_blocks_per_cu": b,
                        "ks_gates_per_block": k, "s": dt})
        if log:
            log("tune waves/rotation=%d rotations/block=%d blocks/CU=%d ks gates/block=%d: %.3f s" % (r, w, b, k, dt))
    best = min(results, key=lambda r: r["s"])
    _apply(ctx, best)
    return {"best": best, "all": results}


def sweep_batch(ctx, ks, sizes=(256, 512, 1024, 2048, 4096, 8192, 16384), seed=11, log=None) -> list:
    """Blind rotations per second against the number of rotations per launch."""
    from . import synth
    out = []
    big = max(sizes)
    d_in = ctx.tensor(synth.uniform_ciphertexts(seed, "batch", (big,)))
    d_out = ctx.empty(big, vlp.CT_N)
    for B in sizes:
        vlp.vlp_bootstrap(ctx.ctx, ks, d_in, d_out, vlp.MU, B)  # warm
        vlp.vlp_sync(ctx.ctx)
        t0 = time.perf_counter()
        vlp.vlp_bootstrap(ctx.ctx, ks, d_in, d_out, vlp.MU, B)
        vlp.vlp_sync(ctx.ctx)
        dt = time.perf_counter() - t0
        out.append({"batch": B, "s": dt, "bootstraps_per_s": B / dt})
        if log:
            log("batch %6d: %.3f s, %.0f bootstraps/s" % (B, dt, B / dt))
    return out


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return "%s/%dcu" % (getattr(p, "gcnArchName", p.name), p.multi_processor_count)


def load_cached(ctx, workload: str) -> bool:
    """Applies a cached launch shape for (device, workload), if any."""
    if not os.path.exists(CACHE):
        return False
    try:
        data = json.load(open(CACHE))
        best = data[device_key()][workload]["best"]
    except (KeyError, ValueError, OSError):
        return False
    _apply(ctx, best)
    return True


def save(workload: str, result: dict) -> None:
    data = {}
    if os.path.exists(CACHE):
        try:
            data = json.load(open(CACHE))
        except ValueError:
            data = {}
    data.setdefault(device_key(), {})[workload] = result
    with open(CACHE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def main():
    """Tune the launch shape on the interval-validation program (records
    configurable), sweep the batch size, and cache the result."""
    import argparse
    import sys

    from . import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--records", type=int, default=256)
    ap.add_argument("--workload", default="intv-1024")
    args = ap.parse_args()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    ctx = vlp.Context(0)
    bk, ksk = synth.uniform_keys(0x5EED0002)
    ks = ctx.load_keys(bk, ksk)
    M = args.records
    q = ctx.tensor(synth.uniform_ciphertexts(3, "q", (2, 16)))
    loc = ctx.tensor(synth.uniform_ciphertexts(3, "l", (M, 2, 2, 16)))
    v = ctx.empty(M, vlp.CT_n)
    prog = vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape("intv", M, 16, 0, 2), q, loc, None, None, v)
    _time_program(ctx, prog)  # warm
    res = tune_launch(ctx, prog, log=log)
    res["batch_sweep"] = sweep_batch(ctx, ks, log=log)
    res["records_tuned_on"] = M
    save(args.workload, res)
    print(json.dumps({"best": res["best"], "batch_sweep": res["batch_sweep"]}))
    vlp.vlp_program_destroy(ctx.ctx, prog)
    ctx.close()


if __name__ == "__main__":
    main()
