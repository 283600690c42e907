"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import workloads as W
import synth

pytestmark = pytest.mark.gpu
MU = O.MU


@pytest.fixture(scope="module")
def gpu(oracle_keys):
    from paper_2506_12761_amd import vlp
    ctx = vlp.Context(0)
    ks = ctx.load_keys(oracle_keys.bk, oracle_keys.ksk)
    yield vlp, ctx, ks
    ctx.close()


def _rand_words(seed, shape):
    return synth.uniform_u32(synth.stream(seed, "words"), shape)


def _pool(fn, items):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(O.default_threads()) as ex:
        return list(ex.map(fn, items))


def test_bootstrap_parity(gpu, oracle_keys):
    vlp, ctx, ks = gpu
    B = 37  # several waves and a ragged tail
    ins = _rand_words(1, (B, O.n + 1))
    ins[1, :O.n] = 0                                   # trivial input: no rotation at all
    ins[2, : O.n // 2] = np.uint32(0x000FFFFF)          # many masks that switch to zero
    masks, noise = synth.lwe_randomness(2, "bs", 4)
    ins[3:7] = O.encrypt_bits(oracle_keys, np.array([1, 0, 1, 1]), masks, noise)
    d_in = ctx.tensor(ins)
    d_out = ctx.empty(B, O.N + 1)
    for mu in (MU, 1 << 30):
        vlp.vlp_bootstrap(ctx.ctx, ks, d_in, d_out, mu, B)
        ctx.sync()
        got = ctx.to_host(d_out)
        want = _pool(lambda c: O.bootstrap_wo_ks(oracle_keys, c, mu), list(ins))
        for b in range(B):
            assert np.array_equal(got[b], want[b]), (mu, b)


@pytest.mark.parametrize("gates_per_block,B", [(128, 21), (512, 21), (128, 8197), (256, 8197), (512, 8197),
                                               (512, 16384 + 8197), (512, 40000)])
def test_keyswitch_parity(gpu, oracle_keys, gates_per_block, B):
    """Every key-switching tile shape on the matrix cores equals the oracle:
    at most 128, 256 or 512 gates per workgroup, with the coefficients split
    over up to 32 workgroups whose partial sums are added atomically into
    outputs that start dirty (small launches), or not split; launches above
    16,384 gates run as several launches sharing one digit buffer; the last
    gate tile is partial.  Large launches are checked on 48 sampled gates."""
    vlp, ctx, ks = gpu
    ins = _rand_words(3 + B, (B, O.N + 1))
    ins[0] = 0
    d_in = ctx.tensor(ins)
    d_out = ctx.tensor(_rand_words(4, (B, O.n + 1)))
    old = vlp.vlp_get_tuning(ctx.ctx)
    try:
        vlp.vlp_set_tuning(ctx.ctx, old.br_rotations_per_block, old.br_blocks_per_cu, gates_per_block,
                           old.br_waves_per_rotation)
        vlp.vlp_keyswitch(ctx.ctx, ks, d_in, d_out, B)
        ctx.sync()
    finally:
        vlp.vlp_set_tuning(ctx.ctx, old.br_rotations_per_block, old.br_blocks_per_cu, old.ks_gates_per_block,
                           old.br_waves_per_rotation)
    got = ctx.to_host(d_out)
    idx = range(B) if B <= 64 else sorted(set(synth.stream(B, "ks-sample").choice(B, 46, replace=False)) | {0, B - 1})
    for b in idx:
        assert np.array_equal(got[b], O.keyswitch(oracle_keys, ins[b])), (gates_per_block, b)


@pytest.mark.parametrize("op", ["AND", "OR", "NAND", "XOR", "XNOR", "NOT", "MUX"])
def test_gate_parity(gpu, oracle_keys, op):
    vlp, ctx, ks = gpu
    B = 11
    g = synth.stream(4, "gate:" + op)
    bits = synth.bits(g, (3, B))
    bits[:, :8] = np.array([[0, 0, 0, 0, 1, 1, 1, 1], [0, 0, 1, 1, 0, 0, 1, 1], [0, 1, 0, 1, 0, 1, 0, 1]])
    masks, noise = synth.lwe_randomness(5, "gate:" + op, 3 * B)
    cts = O.encrypt_bits(oracle_keys, bits, masks.reshape(3, B, O.n), noise.reshape(3, B))
    a, b, c = (ctx.tensor(cts[i]) for i in range(3))
    out = ctx.empty(B, O.n + 1)
    vlp.vlp_gate(ctx.ctx, ks, op, a, None if op == "NOT" else b, c if op == "MUX" else None, out, B)
    ctx.sync()
    got = ctx.to_host(out)
    want = _pool(lambda k: O.gate(oracle_keys, op, cts[0][k], cts[1][k], cts[2][k]), range(B))
    truth = {"AND": lambda x, y, z: x & y, "OR": lambda x, y, z: x | y, "NAND": lambda x, y, z: 1 - (x & y),
             "XOR": lambda x, y, z: x ^ y, "XNOR": lambda x, y, z: 1 - (x ^ y), "NOT": lambda x, y, z: 1 - x,
             "MUX": lambda x, y, z: y if x else z}[op]
    for k in range(B):
        assert np.array_equal(got[k], want[k]), k
        assert int(O.decrypt(oracle_keys, got[k])) == truth(*[int(bits[i, k]) for i in range(3)])


def _run_eval(gpu, keys, mode, M, l, lS, d, seed, optimized=True, use_graph_twice=False, agg_k=0):
    vlp, ctx, ks = gpu
    P = W.plain_workload(mode, M, l, lS, d, seed)
    enc = W.encrypt_workload(keys, P, seed)
    q, loc = ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"])
    pay = ctx.tensor(enc["db_pay"]) if lS else None
    R = ctx.empty(lS, O.n + 1) if lS else None
    v = ctx.empty(M, O.n + 1)
    shape = vlp.make_shape(mode, M, l, lS, d, optimized, agg_k)
    vlp.vlp_evaluate(ctx.ctx, ks, shape, q, loc, pay, R, v)
    ctx.sync()
    res = [(ctx.to_host(v).copy(), ctx.to_host(R).copy() if lS else None)]
    if use_graph_twice:
        ctx.zero(v)
        if lS:
            ctx.zero(R)
        vlp.vlp_evaluate(ctx.ctx, ks, shape, q, loc, pay, R, v)  # replays the captured graph
        ctx.sync()
        res.append((ctx.to_host(v).copy(), ctx.to_host(R).copy() if lS else None))
    return P, enc, res


@pytest.mark.parametrize("case", [
    ("intv", 1, 8, 0, 1),      # the 49-bootstrap one-dimensional interval test
    ("intv", 2, 6, 3, 2),
    ("cov", 3, 5, 2, 2),
    ("idm", 5, 6, 4, 1),
])
def test_evaluate_parity(gpu, oracle_keys, case):
    mode, M, l, lS, d = case
    P, enc, res = _run_eval(gpu, oracle_keys, mode, M, l, lS, d, seed=hash(case) & 0xFFFF, use_graph_twice=True)
    v_want, R_want = W.oracle_outputs(oracle_keys, P, enc)
    for v_got, R_got in res:
        assert np.array_equal(v_got, v_want)
        assert np.array_equal(O.decrypt(oracle_keys, v_got), P["v"])
        if lS:
            assert np.array_equal(R_got, R_want)
            assert np.array_equal(O.decrypt(oracle_keys, R_got), P["R"])


def test_evaluate_unoptimized_parity(gpu, oracle_keys):
    P, enc, res = _run_eval(gpu, oracle_keys, "cov", 3, 4, 2, 2, seed=77, optimized=False)
    v_want, R_want = W.oracle_outputs(oracle_keys, P, enc, optimized=False)
    assert np.array_equal(res[0][0], v_want) and np.array_equal(res[0][1], R_want)


@pytest.mark.parametrize("mode,M,l,lS,d,k", [("idm", 7, 4, 3, 1, 3), ("idm", 18, 3, 2, 1, 16),
                                              ("intv", 5, 5, 2, 2, 4), ("cov", 3, 4, 2, 1, 2)])
def test_evaluate_k_ary_aggregation_parity(gpu, oracle_keys, mode, M, l, lS, d, k):
    """Aggregation by k-input XORs (operand lists of up to 16 ciphertexts in
    the blind rotation's pre-combination) equals the oracle word for word,
    also on the replayed graph; 18 records at k = 16 leave a group of two."""
    P, enc, res = _run_eval(gpu, oracle_keys, mode, M, l, lS, d, seed=1000 + M * k, use_graph_twice=True,
                            agg_k=k)
    v_want, R_want = W.oracle_outputs(oracle_keys, P, enc, agg_k=k)
    for v_got, R_got in res:
        assert np.array_equal(v_got, v_want)
        assert np.array_equal(R_got, R_want)
        assert np.array_equal(O.decrypt(oracle_keys, R_got), P["R"])


def test_step_merges_programs(gpu, oracle_keys):
    """Two programs of different modes and depths advanced together give the
    same words as each run alone."""
    vlp, ctx, ks = gpu
    progs, bufs, wants = [], [], []
    for (mode, M, l, lS, d, seed) in (("intv", 2, 5, 2, 2, 11), ("idm", 3, 4, 3, 1, 12)):
        P = W.plain_workload(mode, M, l, lS, d, seed)
        enc = W.encrypt_workload(oracle_keys, P, seed)
        q, loc, pay = ctx.tensor(enc["query"]), ctx.tensor(enc["db_loc"]), ctx.tensor(enc["db_pay"])
        R, v = ctx.empty(lS, O.n + 1), ctx.empty(M, O.n + 1)
        pr = vlp.vlp_program_create(ctx.ctx, ks, vlp.make_shape(mode, M, l, lS, d), q, loc, pay, R, v)
        progs.append(pr)
        bufs.append((q, loc, pay, R, v))
        wants.append(W.oracle_outputs(oracle_keys, P, enc))
    rem = 1
    steps = 0
    while rem:
        rem = vlp.vlp_step(ctx.ctx, progs)
        steps += 1
    ctx.sync()
    assert steps == max(vlp.vlp_program_counts(ctx.ctx, p)["levels"] for p in progs)
    for (q, loc, pay, R, v), (vw, Rw) in zip(bufs, wants):
        assert np.array_equal(ctx.to_host(v), vw) and np.array_equal(ctx.to_host(R), Rw)
    for p in progs:
        vlp.vlp_program_destroy(ctx.ctx, p)


@pytest.mark.parametrize("per_rot,rpb,blocks", [(1, 1, 4), (1, 2, 2), (1, 4, 1), (1, 8, 1), (2, 1, 4), (2, 1, 1),
                                                (2, 2, 2), (2, 4, 1), (4, 1, 2), (4, 1, 1), (0, 4, 1), (0, 1, 4)])
def test_bootstrap_parity_every_launch_shape(gpu, oracle_keys, per_rot, rpb, blocks):
    """Each blind-rotation kernel and workgroup shape matches the oracle word
    for word: one wavefront per rotation (the 8-wave form has its own register
    plan: key read at use, 32-bit accumulators), two (one per prime; 1, 2 or 4
    rotations per workgroup in lockstep) and four (prime x accumulator half),
    and the automatic choice.  41 items leave the last workgroup partly idle
    (a lockstep workgroup then repeats an item without writing it)."""
    vlp, ctx, ks = gpu
    B = 41
    ins = _rand_words(11, (B, O.n + 1))
    masks, noise = synth.lwe_randomness(12, "shape", 3)
    ins[:3] = O.encrypt_bits(oracle_keys, np.array([1, 0, 1]), masks, noise)
    d_in = ctx.tensor(ins)
    d_out = ctx.empty(B, O.N + 1)
    old = vlp.vlp_get_tuning(ctx.ctx)
    try:
        vlp.vlp_set_tuning(ctx.ctx, rpb, blocks, old.ks_gates_per_block, per_rot)
        vlp.vlp_bootstrap(ctx.ctx, ks, d_in, d_out, MU, B)
        ctx.sync()
    finally:
        vlp.vlp_set_tuning(ctx.ctx, old.br_rotations_per_block, old.br_blocks_per_cu, old.ks_gates_per_block,
                           old.br_waves_per_rotation)
    got = ctx.to_host(d_out)
    want = _pool(lambda c: O.bootstrap_wo_ks(oracle_keys, c, MU), list(ins))
    for b in range(B):
        assert np.array_equal(got[b], want[b]), (per_rot, rpb, blocks, b)
