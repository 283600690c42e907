"""The autotuner on the GPU: it times a small program under several launch
shapes, applies the fastest, caches it by device and workload, and the
program's words under the chosen (and every tried) shape equal the oracle's."""
import json

import numpy as np
import pytest

from oracle import oracle as O
from oracle import workloads as W

pytestmark = pytest.mark.gpu


def test_autotuner_applies_a_valid_shape_and_stays_exact(oracle_keys, tmp_path, monkeypatch):
    from paper_2506_12761_amd import autotune, vlp
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tuning.json"))
    P = W.plain_workload("intv", 3, 5, 2, 2, seed=91)
    enc = W.encrypt_workload(oracle_keys, P, seed=91)
    v_want, R_want = W.oracle_outputs(oracle_keys, P, enc)
    with vlp.Context(0) as ctx:
        ks = ctx.load_keys(oracle_keys.bk, oracle_keys.ksk)
        bufs = (ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"]), ctx.tensor(enc["db_pay"]),
                ctx.empty(2, O.n + 1), ctx.empty(3, O.n + 1))
        prog = vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape("intv", 3, 5, 2, 2), *bufs)
        shapes = [(0, 4, 1, 512), (2, 1, 4, 256), (4, 1, 2, 128), (1, 2, 2, 512)]
        res = autotune.tune_launch(ctx, prog, shapes=shapes, repeats=1)
        best = res["best"]
        assert len(res["all"]) == len(shapes) and best["s"] == min(r["s"] for r in res["all"])
        t = vlp.vlp_get_tuning(ctx.ctx)
        assert (t.br_waves_per_rotation, t.br_rotations_per_block, t.br_blocks_per_cu, t.ks_gates_per_block) == \
            (best["br_waves_per_rotation"], best["br_rotations_per_block"], best["br_blocks_per_cu"],
             best["ks_gates_per_block"])
        # The tuned program, run again, gives the oracle's words.
        ctx.zero(bufs[3])
        ctx.zero(bufs[4])
        vlp.vlp_program_reset(ctx.ctx, prog)
        vlp.vlp_program_run(ctx.ctx, prog, use_graph=False)
        ctx.sync()
        assert np.array_equal(ctx.to_host(bufs[4]), v_want) and np.array_equal(ctx.to_host(bufs[3]), R_want)
        # Cache round trip under the workload key, applied to a fresh context.
        key = autotune.workload_key("intv", 3)
        autotune.save(key, res)
        assert key in json.load(open(autotune.CACHE))[autotune.device_key()]
        vlp.vlp_program_destroy(ctx.ctx, prog)
    with vlp.Context(0) as ctx2:
        vlp.vlp_set_tuning(ctx2.ctx, 2, 2, 256, 2)
        assert autotune.load_cached(ctx2, key)
        t = vlp.vlp_get_tuning(ctx2.ctx)
        assert (t.br_waves_per_rotation, t.br_rotations_per_block, t.br_blocks_per_cu, t.ks_gates_per_block) == \
            (best["br_waves_per_rotation"], best["br_rotations_per_block"], best["br_blocks_per_cu"],
             best["ks_gates_per_block"])
        assert not autotune.load_cached(ctx2, "no-such-workload")
