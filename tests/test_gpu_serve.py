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


def _setup(ctx, keys, specs):
    ks = {c: ctx.load_keys(k.bk, k.ksk) for c, k in keys.items()}
    reqs, plain = [], []
    for rid, (client, mode, M, l, lS, d, t) in enumerate(specs):
        P = W.plain_workload(mode, M, l, lS, d, seed=1000 + rid)
        enc = W.encrypt_workload(keys[client], P, seed=1000 + rid)
        pay = {"query": ctx.tensor(enc["query"]), "db_loc": ctx.tensor(enc["db_loc"]),
               "db_pay": ctx.tensor(enc["db_pay"]), "R": ctx.empty(lS, O.n + 1), "v": ctx.empty(M, O.n + 1)}
        reqs.append(Request(rid, client, mode, M, l, lS, d, arrival=t, payload=pay))
        plain.append(P)
    return ks, reqs, plain


def _alone(ctx, ks, reqs):
    from paper_2506_12761_amd import vlp
    out = []
    for r in reqs:
        p = r.payload
        vlp.vlp_evaluate(ctx.ctx, ks[r.client], vlp.make_shape(r.mode, r.M, r.l_I, r.l_S, r.d),
                         p["query"], p["db_loc"], p["db_pay"], p["R"], p["v"])
        ctx.sync()
        out.append((ctx.to_host(p["R"]).copy(), ctx.to_host(p["v"]).copy()))
        ctx.zero(p["R"])
        ctx.zero(p["v"])
    ctx.sync()
    return out


def test_srpt_policy_under_a_tight_budget_equals_alone():
    """The shortest-remaining-work policy with a small rotation cap per step
    and a device budget that holds one query's program at a time: queries
    wait for memory, the steps advance subsets of the active queries, and
    every result is still word for word the query run alone."""
    from paper_2506_12761_amd import vlp
    keys = {0: O.keygen(synth.key_randomness(0x5EED0101)), 1: O.keygen(synth.key_randomness(0x5EED0102))}
    specs = [(0, "idm", 6, 5, 3, 1, 0.0), (1, "cov", 2, 4, 2, 2, 0.0), (0, "intv", 2, 4, 2, 2, 0.0),
             (1, "idm", 3, 3, 2, 1, 0.01)]
    with vlp.Context(0) as ctx:
        ks, reqs, plain = _setup(ctx, keys, specs)
        alone = _alone(ctx, ks, reqs)
        need = [vlp.vlp_plan_bytes(vlp.make_shape(r.mode, r.M, r.l_I, r.l_S, r.d), True) for r in reqs]
        ex = GpuExecutor(ctx, ks)
        ex.budget = ex.held() + max(need) + min(need) // 2
        st = serve(reqs, ex, policy="srpt", step_cap=40)
        assert st["queries"] == len(reqs) and st["budget_rejections"] > 0 and st["policy"] == "srpt"
        for r, (R_a, v_a), P in zip(reqs, alone, plain):
            R_m, v_m = ctx.to_host(r.payload["R"]), ctx.to_host(r.payload["v"])
            assert np.array_equal(R_m, R_a) and np.array_equal(v_m, v_a), r.rid
            assert np.array_equal(O.decrypt(keys[r.client], R_m), P["R"])


def test_plan_bytes_is_what_a_program_reserves():
    """vlp_plan_bytes bounds what vlp_program_create takes from the budget
    (its step-scratch share may already be covered by the context's scratch)."""
    from paper_2506_12761_amd import vlp
    keys = O.keygen(synth.key_randomness(0x5EED0101))
    with vlp.Context(0) as ctx:
        ks = ctx.load_keys(keys.bk, keys.ksk)
        for (mode, M, l, lS, d) in (("idm", 40, 8, 5, 1), ("intv", 3, 6, 0, 2)):
            sh = vlp.make_shape(mode, M, l, lS, d)
            plan = vlp.vlp_plan_bytes(sh, True)
            q, loc = ctx.empty(d * l, O.n + 1), ctx.empty(M * d * (2 if mode == "intv" else 1) * l, O.n + 1)
            pay, R, v = (ctx.empty(M * lS, O.n + 1), ctx.empty(lS, O.n + 1), ctx.empty(M, O.n + 1)) if lS else \
                (None, None, ctx.empty(M, O.n + 1))
            u0 = vlp.vlp_mem_info(ctx.ctx)[0]
            pr = vlp.vlp_program_create(ctx.ctx, ks, sh, q, loc, pay, R, v)
            delta = vlp.vlp_mem_info(ctx.ctx)[0] - u0
            assert delta <= plan + (1 << 20) and delta > 0, (mode, delta, plan)
            vlp.vlp_program_destroy(ctx.ctx, pr)
            # The program's memory is returned; only the grown step scratch stays with the context.
            assert vlp.vlp_mem_info(ctx.ctx)[0] - u0 <= max(1 << 20, plan)


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


def test_alone_equals_mixed_at_larger_sizes():
    """Three queries of 64-200 records (all three modes, two clients) through
    the serving loop with the shortest-remaining-work policy and a small
    per-step cap: every result word equals the query run alone, and v and R
    decrypt to the plaintext answers."""
    from paper_2506_12761_amd import vlp
    keys = {0: O.keygen(synth.key_randomness(0x5EED0103)), 1: O.keygen(synth.key_randomness(0x5EED0104))}
    specs = [(0, "idm", 200, 8, 4, 1, 0.0), (1, "cov", 100, 6, 3, 2, 0.0), (0, "intv", 64, 8, 2, 2, 0.0)]
    with vlp.Context(0) as ctx:
        ks, reqs, plain = _setup(ctx, keys, specs)
        alone = _alone(ctx, ks, reqs)
        st = serve(reqs, GpuExecutor(ctx, ks), policy="srpt", step_cap=2048)
        assert st["queries"] == len(reqs) and st["max_active"] >= 2
        for r, (R_a, v_a), P in zip(reqs, alone, plain):
            R_m, v_m = ctx.to_host(r.payload["R"]), ctx.to_host(r.payload["v"])
            assert np.array_equal(R_m, R_a) and np.array_equal(v_m, v_a), r.rid
            assert np.array_equal(O.decrypt(keys[r.client], v_m), P["v"])
            assert np.array_equal(O.decrypt(keys[r.client], R_m), P["R"])
