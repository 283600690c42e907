"""Serving on the GPU: every query's result words are identical when it runs
alone and when it runs merged with others (different clients, keys, modes
and depths), and they decrypt to the plaintext answer."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import workloads as W
import synth
from paper_2506_12761_amd.serve import GpuExecutor, Request, serve

pytestmark = pytest.mark.gpu


def test_alone_equals_mixed():
    from paper_2506_12761_amd import vlp
    keys = {0: O.keygen(synth.key_randomness(0x5EED0101)), 1: O.keygen(synth.key_randomness(0x5EED0102))}
    # The first two arrive together, so they are admitted before the first
    # step and run merged whatever the kernels' speed; the later two join
    # while others may still run.
    specs = [(0, "intv", 2, 6, 3, 2, 0.00), (1, "cov", 3, 5, 2, 2, 0.00), (0, "idm", 4, 6, 4, 1, 0.02),
             (1, "intv", 1, 5, 2, 1, 0.20)]
    with vlp.Context(0) as ctx:
        ks = {c: ctx.load_keys(k.bk, k.ksk) for c, k in keys.items()}
        reqs, plain = [], []
        for rid, (client, mode, M, l, lS, d, t) in enumerate(specs):
            P = W.plain_workload(mode, M, l, lS, d, seed=1000 + rid)
            enc = W.encrypt_workload(keys[client], P, seed=1000 + rid)
            pay = {"query": ctx.tensor(enc["query"]), "db_loc": ctx.tensor(enc["db_loc"]),
                   "db_pay": ctx.tensor(enc["db_pay"]), "R": ctx.empty(lS, O.n + 1), "v": ctx.empty(M, O.n + 1)}
            reqs.append(Request(rid, client, mode, M, l, lS, d, arrival=t, payload=pay))
            plain.append(P)
        # alone
        alone = []
        for r in reqs:
            p = r.payload
            vlp.vlp_evaluate(ctx.ctx, ks[r.client], vlp.make_shape(r.mode, r.M, r.l_I, r.l_S, r.d),
                             p["query"], p["db_loc"], p["db_pay"], p["R"], p["v"])
            ctx.sync()
            alone.append((ctx.to_host(p["R"]).copy(), ctx.to_host(p["v"]).copy()))
            ctx.zero(p["R"])
            ctx.zero(p["v"])
        ctx.sync()
        st = serve(reqs, GpuExecutor(ctx, ks))
        assert st["queries"] == len(reqs) and st["max_active"] >= 2
        for r, (R_a, v_a), P in zip(reqs, alone, plain):
            R_m, v_m = ctx.to_host(r.payload["R"]), ctx.to_host(r.payload["v"])
            assert np.array_equal(R_m, R_a) and np.array_equal(v_m, v_a), r.rid
            assert np.array_equal(O.decrypt(keys[r.client], v_m), P["v"])
            assert np.array_equal(O.decrypt(keys[r.client], R_m), P["R"])
