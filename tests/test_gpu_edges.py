"""Edge cases through the C ABI: empty batches, argument errors, the memory
budget, tuning validation, and the extreme shapes of the evaluation
(64-bit identifiers, 2-bit intervals, one record, one payload bit)."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import workloads as W
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu(oracle_keys):
    from paper_2506_12761_amd import vlp
    ctx = vlp.Context(0)
    ks = ctx.load_keys(oracle_keys.bk, oracle_keys.ksk)
    yield vlp, ctx, ks
    ctx.close()


def _words(seed, shape):
    return synth.uniform_u32(synth.stream(seed, "edge"), shape)


def test_empty_batches_are_noops(gpu):
    vlp, ctx, ks = gpu
    a = ctx.tensor(_words(1, (2, O.n + 1)))
    big = ctx.tensor(_words(2, (2, O.N + 1)))
    before_a, before_big = ctx.to_host(a).copy(), ctx.to_host(big).copy()
    vlp.vlp_bootstrap(ctx.ctx, ks, a, big, O.MU, 0)
    vlp.vlp_keyswitch(ctx.ctx, ks, big, a, 0)
    vlp.vlp_gate(ctx.ctx, ks, "AND", a, a, None, big, 0)
    ctx.sync()
    assert np.array_equal(ctx.to_host(a), before_a) and np.array_equal(ctx.to_host(big), before_big)


def test_argument_errors(gpu):
    vlp, ctx, ks = gpu
    x = ctx.tensor(_words(3, (4, O.n + 1)))
    y = ctx.tensor(_words(4, (4, O.n + 1)))

    def einval(fn, *args):
        with pytest.raises(vlp.VlpError) as e:
            fn(*args)
        assert e.value.status == vlp.VLP_EINVAL, e.value

    einval(vlp.vlp_gate, ctx.ctx, ks, "AND", x, y, None, x[1:], 3)          # output overlaps an input
    einval(vlp.vlp_gate, ctx.ctx, ks, "AND", x, None, None, y, 4)           # AND needs b
    einval(vlp.vlp_gate, ctx.ctx, ks, "XOR", x, y, x, y[2:], 2)            # c only for MUX
    einval(vlp.vlp_gate, ctx.ctx, ks, "MUX", x, y, None, y[2:], 2)         # MUX needs c
    einval(vlp.vlp_gate, ctx.ctx, ks, 42, x, y, None, y, 1)                # unknown op
    einval(vlp.vlp_keyswitch, ctx.ctx, ks, x, x, 1)                         # in and out overlap
    einval(vlp.vlp_bootstrap, ctx.ctx, None, x, y, O.MU, 1)                 # no keyset
    einval(vlp.vlp_evaluate, ctx.ctx, ks, vlp.make_shape("idm", 2, 4, 0, 1, True, 17), x, y, None, None, None)
    einval(vlp.vlp_evaluate, ctx.ctx, ks, vlp.make_shape("intv", 2, 1, 0, 1), x, y, None, None, None)
    # The failed calls left the context usable.
    vlp.vlp_gate(ctx.ctx, ks, "NOT", x, None, None, y, 4)
    ctx.sync()
    assert np.array_equal(ctx.to_host(y), (0 - ctx.to_host(x).astype(np.uint64)).astype(np.uint32))


def test_keyset_of_another_context_is_rejected(gpu, oracle_keys):
    vlp, ctx, ks = gpu
    other = vlp.Context(0)
    try:
        x = ctx.tensor(_words(5, (1, O.n + 1)))
        y = ctx.empty(1, O.N + 1)
        with pytest.raises(vlp.VlpError) as e:
            vlp.vlp_bootstrap(other.ctx, ks, x, y, O.MU, 1)
        assert e.value.status == vlp.VLP_EINVAL
    finally:
        other.close()


def test_budget_too_small_for_a_keyset(oracle_keys):
    from paper_2506_12761_amd import vlp
    small = vlp.Context(0, hbm_budget=64 << 20)  # below the 145.8 MB a keyset needs
    try:
        used0, budget = vlp.vlp_mem_info(small.ctx)
        assert budget == 64 << 20
        with pytest.raises(vlp.VlpError) as e:
            small.load_keys(oracle_keys.bk, oracle_keys.ksk)
        assert e.value.status == vlp.VLP_EBUDGET
        assert vlp.vlp_mem_info(small.ctx)[0] == used0
    finally:
        small.close()


@pytest.mark.parametrize("bad", [(1, 1, 512, 3), (8, 1, 512, 2), (2, 1, 512, 4), (4, 0, 512, 0), (4, 65, 512, 0),
                                 (4, 1, 8, 0), (4, 1, 64, 0), (4, 1, 1024, 0)])
def test_tuning_validation(gpu, bad):
    vlp, ctx, ks = gpu
    old = vlp.vlp_get_tuning(ctx.ctx)
    with pytest.raises(vlp.VlpError) as e:
        vlp.vlp_set_tuning(ctx.ctx, *bad)
    assert e.value.status == vlp.VLP_EINVAL
    now = vlp.vlp_get_tuning(ctx.ctx)
    assert (now.br_rotations_per_block, now.br_blocks_per_cu, now.ks_gates_per_block, now.br_waves_per_rotation) == \
        (old.br_rotations_per_block, old.br_blocks_per_cu, old.ks_gates_per_block, old.br_waves_per_rotation)


@pytest.mark.parametrize("mode,M,l,lS,d", [
    ("idm", 2, 64, 1, 1),    # widest identifiers, one payload bit
    ("intv", 3, 2, 2, 1),    # narrowest signed intervals
    ("idm", 1, 5, 5, 1),     # one record: the result is the selection itself
    ("cov", 1, 3, 0, 1),     # one record, one coordinate, no payload
])
def test_evaluate_extreme_shapes(gpu, oracle_keys, mode, M, l, lS, d):
    vlp, ctx, ks = gpu
    P = W.plain_workload(mode, M, l, lS, d, seed=500 + M * l)
    enc = W.encrypt_workload(oracle_keys, P, seed=501 + l)
    q, loc = ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"])
    pay = ctx.tensor(enc["db_pay"]) if lS else None
    R = ctx.empty(lS, O.n + 1) if lS else None
    v = ctx.empty(M, O.n + 1)
    vlp.vlp_evaluate(ctx.ctx, ks, vlp.make_shape(mode, M, l, lS, d), q, loc, pay, R, v)
    ctx.sync()
    v_want, R_want = W.oracle_outputs(oracle_keys, P, enc)
    assert np.array_equal(ctx.to_host(v), v_want)
    assert np.array_equal(O.decrypt(oracle_keys, ctx.to_host(v)), P["v"])
    if lS:
        assert np.array_equal(ctx.to_host(R), R_want)
        assert np.array_equal(O.decrypt(oracle_keys, ctx.to_host(R)), P["R"])


def test_circuit_argument_of_the_ex_calls(gpu, oracle_keys):
    """The plain calls, given only the five-field shape, evaluate the
    optimized circuits, as the _ex calls do with a NULL circuit or {1, 0};
    {0, 0} gives the baseline chains' words; a bad agg_k is an argument error."""
    vlp, ctx, ks = gpu
    mode, M, l, lS, d = "idm", 3, 5, 2, 1
    P = W.plain_workload(mode, M, l, lS, d, seed=77)
    enc = W.encrypt_workload(oracle_keys, P, seed=78)
    q, loc, pay = ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"]), ctx.tensor(enc["db_pay"])
    shape = vlp.vlp_shape(vlp.MODES[mode], M, l, lS, d)
    want = {True: W.oracle_outputs(oracle_keys, P, enc, optimized=True),
            False: W.oracle_outputs(oracle_keys, P, enc, optimized=False)}
    runs = [(lambda R, v: vlp.vlp_evaluate(ctx.ctx, ks, shape, q, loc, pay, R, v), True),
            (lambda R, v: vlp.vlp_evaluate_ex(ctx.ctx, ks, shape, None, q, loc, pay, R, v), True),
            (lambda R, v: vlp.vlp_evaluate_ex(ctx.ctx, ks, shape, vlp.vlp_circuit(1, 0), q, loc, pay, R, v), True),
            (lambda R, v: vlp.vlp_evaluate_ex(ctx.ctx, ks, shape, vlp.vlp_circuit(0, 0), q, loc, pay, R, v), False)]
    for run, opt in runs:
        R, v = ctx.empty(lS, O.n + 1), ctx.empty(M, O.n + 1)
        run(R, v)
        ctx.sync()
        v_want, R_want = want[opt]
        assert np.array_equal(ctx.to_host(v), v_want) and np.array_equal(ctx.to_host(R), R_want), opt
    R, v = ctx.empty(lS, O.n + 1), ctx.empty(M, O.n + 1)
    with pytest.raises(vlp.VlpError) as e:
        vlp.vlp_evaluate_ex(ctx.ctx, ks, shape, vlp.vlp_circuit(1, 1), q, loc, pay, R, v)
    assert e.value.status == vlp.VLP_EINVAL
    pr = vlp.vlp_program_create(ctx.ctx, ks, shape, q, loc, pay, R, v)
    assert vlp.vlp_program_counts(ctx.ctx, pr)["blind_rotations"] == vlp.vlp_plan_counts(shape)["blind_rotations"]
    vlp.vlp_program_destroy(ctx.ctx, pr)


def test_step_rejects_a_program_listed_twice(gpu, oracle_keys):
    """A duplicated handle is an argument error that enqueues nothing; the
    programs then step to the oracle's words, and a program part-way through
    finishes under vlp_program_run with the graph flag."""
    vlp, ctx, ks = gpu
    runs = []
    for (mode, M, l, lS, d, seed) in (("idm", 3, 4, 2, 1, 31), ("cov", 2, 3, 2, 1, 32)):
        P = W.plain_workload(mode, M, l, lS, d, seed)
        enc = W.encrypt_workload(oracle_keys, P, seed)
        bufs = (ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"]), ctx.tensor(enc["db_pay"]),
                ctx.empty(lS, O.n + 1), ctx.empty(M, O.n + 1))
        pr = vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape(mode, M, l, lS, d), *bufs)
        runs.append((P, enc, bufs, pr))
    a, b = runs[0][3], runs[1][3]
    with pytest.raises(vlp.VlpError) as e:
        vlp.vlp_step(ctx.ctx, [a, b, a])
    assert e.value.status == vlp.VLP_EINVAL
    assert vlp.vlp_step(ctx.ctx, [a, b]) == 2              # one level of each
    vlp.vlp_program_run(ctx.ctx, a, use_graph=True)        # the rest of a, without the graph
    while vlp.vlp_step(ctx.ctx, [a, b]):
        pass
    ctx.sync()
    for P, enc, bufs, pr in runs:
        v_want, R_want = W.oracle_outputs(oracle_keys, P, enc)
        assert np.array_equal(ctx.to_host(bufs[4]), v_want) and np.array_equal(ctx.to_host(bufs[3]), R_want)
        vlp.vlp_program_destroy(ctx.ctx, pr)


def test_graph_follows_a_tuning_change(gpu, oracle_keys):
    """A program replayed from its HIP graph, then run again after the launch
    shape changed (captured again with the new shape), gives the oracle's
    words both times."""
    vlp, ctx, ks = gpu
    P = W.plain_workload("intv", 2, 4, 2, 2, 41)
    enc = W.encrypt_workload(oracle_keys, P, 41)
    bufs = (ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"]), ctx.tensor(enc["db_pay"]),
            ctx.empty(2, O.n + 1), ctx.empty(2, O.n + 1))
    pr = vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape("intv", 2, 4, 2, 2), *bufs)
    v_want, R_want = W.oracle_outputs(oracle_keys, P, enc)
    old = vlp.vlp_get_tuning(ctx.ctx)
    try:
        for tune in (None, (1, 2, 128, 4), (2, 1, 256, 2)):
            if tune:
                vlp.vlp_set_tuning(ctx.ctx, *tune)
            for _ in range(2):
                ctx.zero(bufs[3])
                ctx.zero(bufs[4])
                vlp.vlp_program_reset(ctx.ctx, pr)
                vlp.vlp_program_run(ctx.ctx, pr, use_graph=True)
                ctx.sync()
                assert np.array_equal(ctx.to_host(bufs[4]), v_want), tune
                assert np.array_equal(ctx.to_host(bufs[3]), R_want), tune
    finally:
        vlp.vlp_set_tuning(ctx.ctx, old.br_rotations_per_block, old.br_blocks_per_cu, old.ks_gates_per_block,
                           old.br_waves_per_rotation)
        vlp.vlp_program_destroy(ctx.ctx, pr)
