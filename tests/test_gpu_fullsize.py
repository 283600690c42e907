"""Parity at the benchmark's full sizes and launch configurations.

The 1,024-record 16-bit two-dimensional interval query runs exactly as
bench.py runs it (one program, level by level, default launch shape); every
one of the 1,024 validation bits decrypts to the plaintext predicate, and a
seeded sample of records is recomputed word for word by the oracle (each
record's circuit depends only on the query and that record's bounds).  The
mixed-depth cells (20-bit coordinate and range cells, Alg. 8 and Alg. 4)
run as two programs advanced together, as bench.py runs them; the
identifier match with payload selection and XOR aggregation (Alg. 9 and 10)
is compared word for word on its aggregate R, both at a size the oracle
covers whole and as a record slice merged into the full-size launches."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import workloads as W
import synth

pytestmark = pytest.mark.gpu


def _run(keys, mode, M, l, lS, d, seed, sample):
    from paper_2506_12761_amd import vlp
    P = W.plain_workload(mode, M, l, lS, d, seed)
    enc = W.encrypt_workload(keys, P, seed)
    with vlp.Context(0) as ctx:
        ks = ctx.load_keys(keys.bk, keys.ksk)
        q, loc = ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"])
        pay = ctx.tensor(enc["db_pay"]) if lS else None
        R = ctx.empty(lS, O.n + 1) if lS else None
        v = ctx.empty(M, O.n + 1)
        prog = vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape(mode, M, l, lS, d), q, loc, pay, R, v)
        vlp.vlp_program_run(ctx.ctx, prog, use_graph=False)
        ctx.sync()
        v_got = ctx.to_host(v).copy()
        R_got = ctx.to_host(R).copy() if lS else None
        vlp.vlp_program_destroy(ctx.ctx, prog)
    assert np.array_equal(O.decrypt(keys, v_got), P["v"])
    if lS:
        assert np.array_equal(O.decrypt(keys, R_got), P["R"])
    idx = synth.stream(seed, "sample").choice(M, size=sample, replace=False)
    if P["v"].any():  # include a matching record when there is one
        idx[0] = int(np.flatnonzero(P["v"])[0])
    Q, e = W.record_slice(P, enc, np.sort(idx))
    Q["lS"] = 0
    v_want, _ = W.oracle_outputs(keys, Q, e)
    assert np.array_equal(v_got[np.sort(idx)], v_want)
    return P


def test_interval_1024_records_full_size(oracle_keys):
    P = _run(oracle_keys, "intv", 1024, 16, 0, 2, seed=0x5EED0002, sample=3)
    assert P["v"].sum() >= 1


def test_identifier_4096_records_with_payload(oracle_keys):
    P = _run(oracle_keys, "idm", 4096, 32, 64, 1, seed=0x5EED0004, sample=2)
    assert P["v"].sum() >= 1


def _stepped(ctx, progs):
    """Advance programs together (vlp_step) to the end; returns the step count."""
    from paper_2506_12761_amd import vlp
    steps, rem = 0, 1
    while rem:
        rem = vlp.vlp_step(ctx.ctx, progs)
        steps += 1
    ctx.sync()
    return steps


def test_identifier_aggregation_word_exact(oracle_keys):
    """100 records with 5-bit identifiers (several records match the query)
    and 4 payload bits: the selection and the ragged 7-level XOR tree over 100
    records give the oracle's R word for word, and every v."""
    from paper_2506_12761_amd import vlp
    M, l, lS, seed = 100, 5, 4, 0x5EED0104
    P = W.plain_workload("idm", M, l, lS, 1, seed)
    assert P["v"].sum() >= 2
    enc = W.encrypt_workload(oracle_keys, P, seed)
    with vlp.Context(0) as ctx:
        ks = ctx.load_keys(oracle_keys.bk, oracle_keys.ksk)
        q, loc, pay = ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"]), ctx.tensor(enc["db_pay"])
        R, v = ctx.empty(lS, O.n + 1), ctx.empty(M, O.n + 1)
        prog = vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape("idm", M, l, lS, 1), q, loc, pay, R, v)
        assert vlp.vlp_program_counts(ctx.ctx, prog)["levels"] == 1 + 3 + 1 + 7
        vlp.vlp_program_run(ctx.ctx, prog, use_graph=False)
        ctx.sync()
        v_got, R_got = ctx.to_host(v).copy(), ctx.to_host(R).copy()
        vlp.vlp_program_destroy(ctx.ctx, prog)
    v_want, R_want = W.oracle_outputs(oracle_keys, P, enc)
    assert np.array_equal(v_got, v_want)
    assert np.array_equal(R_got, R_want)
    assert np.array_equal(O.decrypt(oracle_keys, R_got), P["R"])


def test_mixed_depth_cells_merged_launch(oracle_keys):
    """The 4,096 mixed cells: 20-bit coordinate cells (CoV, depth 7) and
    20-bit range cells (IntV, depth 23) by a seeded coin, as two programs
    whose levels share every launch.  Every v decrypts to its predicate; two
    cells of each kind (a matching one among them) equal the oracle word for
    word."""
    import bench
    from paper_2506_12761_amd import vlp
    specs = bench.mixed_programs()
    assert [s["mode"] for s in specs] == ["cov", "intv"] and sum(s["M"] for s in specs) == 4096
    runs = []
    with vlp.Context(0) as ctx:
        ks = ctx.load_keys(oracle_keys.bk, oracle_keys.ksk)
        progs, bufs = [], []
        for k, sp in enumerate(specs):
            seed = 0x5EED0003 + 16 * k
            P = W.plain_workload(sp["mode"], sp["M"], sp["l"], 0, sp["d"], seed)
            enc = W.encrypt_workload(oracle_keys, P, seed)
            q, loc = ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"])
            v = ctx.empty(sp["M"], O.n + 1)
            progs.append(vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape(sp["mode"], sp["M"], 20, 0, 2), q, loc,
                                                None, None, v))
            bufs.append((q, loc, v))
            runs.append((P, enc, seed))
        levels = [vlp.vlp_program_counts(ctx.ctx, pr)["levels"] for pr in progs]
        assert levels == [7, 23]
        print("mixed cells: stepping", flush=True)
        assert _stepped(ctx, progs) == 23
        got = [ctx.to_host(b[2]).copy() for b in bufs]
        for pr in progs:
            vlp.vlp_program_destroy(ctx.ctx, pr)
    for (P, enc, seed), v_got in zip(runs, got):
        assert np.array_equal(O.decrypt(oracle_keys, v_got), P["v"]), P["mode"]
        assert P["v"].sum() >= 1
        idx = synth.stream(seed, "sample").choice(P["M"], size=2, replace=False)
        idx[0] = int(np.flatnonzero(P["v"])[0])
        idx = np.sort(idx)
        Q, e = W.record_slice(P, enc, idx)
        v_want, _ = W.oracle_outputs(oracle_keys, Q, e)
        assert np.array_equal(v_got[idx], v_want), P["mode"]


def test_identifier_full_size_with_payload_slice_merged(oracle_keys):
    """4,096 records with 32-bit identifiers and 64 payload bits, advanced
    together with an 8-record slice of the same database (the matching record
    among them) whose payload is kept: the slice's R (selection plus a 3-level
    XOR tree) equals the oracle's word for word, while the full query's v and
    R decrypt to the plaintext result and sampled v equal the oracle's."""
    from paper_2506_12761_amd import vlp
    M, l, lS, seed = 4096, 32, 64, 0x5EED0004
    P = W.plain_workload("idm", M, l, lS, 1, seed)
    enc = W.encrypt_workload(oracle_keys, P, seed)
    hit = int(np.flatnonzero(P["v"])[0])
    sl = np.sort(np.unique(np.concatenate([[hit], synth.stream(seed, "slice").choice(M, size=7, replace=False)])))[:8]
    Q, e = W.record_slice(P, enc, sl)
    with vlp.Context(0) as ctx:
        ks = ctx.load_keys(oracle_keys.bk, oracle_keys.ksk)
        full = [ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"]), ctx.tensor(enc["db_pay"]),
                ctx.empty(lS, O.n + 1), ctx.empty(M, O.n + 1)]
        part = [full[0], ctx.tensor(e["db_loc"]), ctx.tensor(e["db_pay"]), ctx.empty(lS, O.n + 1),
                ctx.empty(len(sl), O.n + 1)]
        progs = [vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape("idm", M, l, lS, 1), *full),
                 vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape("idm", len(sl), l, lS, 1), *part)]
        print("identifier 4096 + slice: stepping", flush=True)
        _stepped(ctx, progs)
        v_full, R_full = ctx.to_host(full[4]).copy(), ctx.to_host(full[3]).copy()
        v_part, R_part = ctx.to_host(part[4]).copy(), ctx.to_host(part[3]).copy()
        for pr in progs:
            vlp.vlp_program_destroy(ctx.ctx, pr)
    assert np.array_equal(O.decrypt(oracle_keys, v_full), P["v"])
    assert np.array_equal(O.decrypt(oracle_keys, R_full), P["R"])
    assert np.array_equal(v_part, v_full[sl])       # a record's v does not depend on the other records
    v_want, R_want = W.oracle_outputs(oracle_keys, Q, e)
    assert np.array_equal(v_part, v_want)
    assert np.array_equal(R_part, R_want)
    assert np.array_equal(O.decrypt(oracle_keys, R_part), Q["v"] @ Q["pay"] % 2)
