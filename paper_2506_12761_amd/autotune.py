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
SHAPES = ([(1, w, b, 512) for w in (1, 2, 4, 8) for b in (1, 2, 4) if w * b <= 8]
          + [(r, q, b, k) for r in (0, 2) for (q, b) in ((1, 4), (2, 2), (4, 1)) for k in (128, 256, 512)]
          + [(4, 1, b, 512) for b in (1, 2)])


def _apply(ctx, best: dict) -> None:
    vlp.vlp_set_tuning(ctx.ctx, best["br_rotations_per_block"], best["br_blocks_per_cu"], best["ks_gates_per_block"],
                       best.get("br_waves_per_rotation", 0))


def uniform_words(ctx, shape, seed: int):
    """Uniform 32-bit words drawn on the device (timing inputs only: the
    kernels' work does not depend on the values)."""
    torch = ctx.torch
    g = torch.Generator(device=ctx.device)
    g.manual_seed(seed)
    with torch.cuda.stream(ctx.stream):
        t = torch.randint(-2**31, 2**31, tuple(shape), dtype=torch.int32, device=ctx.device, generator=g)
    ctx.stream.synchronize()
    return t


def _time_program(ctx, prog) -> float:
    vlp.vlp_sync(ctx.ctx)
    t0 = time.perf_counter()
    vlp.vlp_program_reset(ctx.ctx, prog)
    vlp.vlp_program_run(ctx.ctx, prog, use_graph=False)
    vlp.vlp_sync(ctx.ctx)
    return time.perf_counter() - t0


def tune_launch(ctx, prog, shapes=SHAPES, repeats: int = 3, log=None) -> dict:
    """Times `prog` under each launch shape (median of `repeats` passes after
    one warm pass); sets and returns the best."""
    results = []
    for (r, w, b, k) in shapes:
        vlp.vlp_set_tuning(ctx.ctx, w, b, k, r)
        _time_program(ctx, prog)
        dt = sorted(_time_program(ctx, prog) for _ in range(max(1, repeats)))[max(1, repeats) // 2]
        results.append({"br_waves_per_rotation": r, "br_rotations_per_block": w, "br_blocks_per_cu": b,
                        "ks_gates_per_block": k, "s": dt})
        if log:
            log("tune waves/rotation=%d rotations/block=%d blocks/CU=%d ks gates/block=%d: %.3f s" % (r, w, b, k, dt))
    best = min(results, key=lambda r: r["s"])
    _apply(ctx, best)
    return {"best": best, "all": results}


def sweep_batch(ctx, ks, sizes=(256, 512, 1024, 2048, 4096, 8192, 16384), seed=11, log=None) -> list:
    """Blind rotations per second against the number of rotations per launch."""
    out = []
    big = max(sizes)
    d_in = uniform_words(ctx, (big, vlp.CT_n), seed)
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


def workload_key(mode: str, records: int) -> str:
    """Cache key of a workload: its mode and the records it was tuned on."""
    return "%s-%d" % (mode, records)


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

    ap = argparse.ArgumentParser()
    ap.add_argument("--records", type=int, default=1024)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    ctx = vlp.Context(0)
    ks = ctx.load_keys(uniform_words(ctx, (630, 6, 2, 1024), 1), uniform_words(ctx, (1024, 8, 4, vlp.CT_n), 2))
    M = args.records
    q = uniform_words(ctx, (2, 16, vlp.CT_n), 3)
    loc = uniform_words(ctx, (M, 2, 2, 16, vlp.CT_n), 4)
    v = ctx.empty(M, vlp.CT_n)
    prog = vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape("intv", M, 16, 0, 2), q, loc, None, None, v)
    _time_program(ctx, prog)  # warm
    res = tune_launch(ctx, prog, repeats=args.repeats, log=log)
    res["batch_sweep"] = sweep_batch(ctx, ks, log=log)
    res["records_tuned_on"] = M
    save(workload_key("intv", M), res)
    print(json.dumps({"best": res["best"], "batch_sweep": res["batch_sweep"]}))
    vlp.vlp_program_destroy(ctx.ctx, prog)
    ctx.close()


if __name__ == "__main__":
    main()
