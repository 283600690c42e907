"""Parity at the benchmark's full size and launch configuration.

The 1,024-record 16-bit two-dimensional interval query runs exactly as
bench.py runs it (one program, level by level, default launch shape); every
one of the 1,024 validation bits decrypts to the plaintext predicate, and a
seeded sample of records is recomputed word for word by the oracle (each
record's circuit depends only on the query and that record's bounds)."""
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
