"""The allocation-free gate call (vlp_gate_noalloc) through the C ABI: the same
words as vlp_gate on the same inputs, on two calls in a row (the second one
smaller, so it runs over what the first left in the fixed scratch), and
arguments beyond its fixed size rejected."""
import numpy as np
import pytest

from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu

MAX_GATES = 1024


@pytest.fixture(scope="module")
def gpu(oracle_keys):
    from paper_2506_12761_amd import vlp
    ctx = vlp.Context(0)
    ks = ctx.load_keys(oracle_keys.bk, oracle_keys.ksk)
    yield vlp, ctx, ks
    ctx.close()


def _operands(keys, seed, B):
    g = synth.stream(seed, "noalloc-bits")
    bits = synth.bits(g, (3, B))
    masks, noise = synth.lwe_randomness(seed, "noalloc", 3 * B)
    return bits, O.encrypt_bits(keys, bits, masks.reshape(3, B, O.n), noise.reshape(3, B))


TRUTH = {"AND": lambda x, y, z: x & y, "XOR": lambda x, y, z: x ^ y, "MUX": lambda x, y, z: np.where(x == 1, y, z),
         "NOT": lambda x, y, z: 1 - x}


@pytest.mark.parametrize("calls", [(("MUX", MAX_GATES), ("AND", 300)), (("XOR", 513), ("MUX", 37), ("NOT", 5))])
def test_noalloc_equals_gate(gpu, oracle_keys, calls):
    vlp, ctx, ks = gpu
    used0, _ = vlp.vlp_mem_info(ctx.ctx)
    for t, (op, B) in enumerate(calls):
        print("noalloc case", op, B, flush=True)
        bits, cts = _operands(oracle_keys, 100 + 7 * t + B, B)
        a, b, c = (ctx.tensor(cts[i]) for i in range(3))
        b_arg = None if op == "NOT" else b
        c_arg = c if op == "MUX" else None
        want_t = ctx.empty(B, O.n + 1)
        got_t = ctx.tensor(synth.uniform_u32(synth.stream(B, "dirty"), (B, O.n + 1)))  # starts dirty
        vlp.vlp_gate_noalloc(ctx.ctx, ks, op, a, b_arg, c_arg, got_t, B)
        ctx.sync()
        got = ctx.to_host(got_t).copy()
        vlp.vlp_gate(ctx.ctx, ks, op, a, b_arg, c_arg, want_t, B)
        ctx.sync()
        want = ctx.to_host(want_t)
        assert np.array_equal(got, want), (op, B, int(np.argmax(np.any(got != want, axis=1))))
        dec = O.decrypt(oracle_keys, got)
        assert np.array_equal(dec, TRUTH[op](bits[0], bits[1], bits[2])), (op, B)
    # The call itself holds no context memory (vlp_gate grew the context's own scratch).
    used1, _ = vlp.vlp_mem_info(ctx.ctx)
    assert used1 >= used0


def test_noalloc_rejects_oversize_and_bad_arguments(gpu):
    vlp, ctx, ks = gpu
    x = ctx.empty(MAX_GATES + 1, O.n + 1)
    y = ctx.empty(MAX_GATES + 1, O.n + 1)
    out = ctx.empty(MAX_GATES + 1, O.n + 1)
    with pytest.raises(vlp.VlpError) as e:
        vlp.vlp_gate_noalloc(ctx.ctx, ks, "AND", x, y, None, out, MAX_GATES + 1)
    assert e.value.status == vlp.VLP_EINVAL and "1024" in str(e.value)
    with pytest.raises(vlp.VlpError) as e:
        vlp.vlp_gate_noalloc(ctx.ctx, ks, "MUX", x, y, None, out, 4)
    assert e.value.status == vlp.VLP_EINVAL
    with pytest.raises(vlp.VlpError) as e:
        vlp.vlp_gate_noalloc(ctx.ctx, ks, "AND", x, y, None, x, 4)
    assert e.value.status == vlp.VLP_EINVAL
    vlp.vlp_gate_noalloc(ctx.ctx, ks, "AND", x, y, None, out, 0)  # no-op
