"""Pins for the oracle's bootstrapping and gates.

Closed forms: (1) a trivial input (mask 0) never rotates, so the output is
exactly the trivial (0, +-mu); (2) with noise-free degenerate keys (ring key
S = 0, BK_i = s_i times the gadget, KSK = 0) every CMux is exact and the
output is exactly (0, +mu) iff (b~ - sum a~_i s_i) mod 2048 < 1024.
Semantics: every gate's truth table by decryption under real seeded keys,
with the output phase inside a noise band around +-1/8.
A schoolbook-product bootstrap must equal the transform-product bootstrap.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O
import synth

MU = O.MU
n, N = O.n, O.N


def _rand_ct(rng):
    return rng.integers(0, 2**32, size=n + 1, dtype=np.uint64).astype(np.uint32)


def test_trivial_input_closed_form(oracle_keys):
    for b in (0, 1, 2**20 - 1, 2**20, 2**31 - 2**20 - 1, 2**31 - 2**20, 2**31, 2**32 - 1, 0x12345678, 0xDEADBEEF):
        ct = np.zeros(n + 1, np.uint32)
        ct[n] = b
        out = O.bootstrap(oracle_keys, ct)
        bbar = ((b + 2**20) % 2**32) >> 21
        want = np.zeros(n + 1, np.uint32)
        want[n] = MU if bbar < 1024 else 2**32 - MU
        assert np.array_equal(out, want), hex(b)


def test_degenerate_keys_closed_form():
    rng = np.random.default_rng(5)
    s = rng.integers(0, 2, size=n).astype(np.uint32)
    K = O.degenerate_keys(s)
    cts = [_rand_ct(rng) for _ in range(6)]
    # force a few zero modswitched masks and the phase boundary cases
    cts[0][:100] = 0
    cts[1][n] = 0
    with ThreadPoolExecutor(4) as ex:
        outs = list(ex.map(lambda c: O.bootstrap(K, c), cts))
        accs = list(ex.map(lambda c: O.blind_rotate(K, c), cts))
    for ct, out, acc in zip(cts, outs, accs):
        ab = (((ct.astype(np.int64) + 2**20) % 2**32) >> 21)
        ph = int((ab[n] - int((ab[:n] * s).sum())) % 2048)
        want = np.zeros(n + 1, np.uint32)
        want[n] = MU if ph < 1024 else 2**32 - MU
        assert np.array_equal(out, want)
        # the accumulator itself: (0, X^(-ph) * mu * (1 + ... + X^(N-1)))
        assert not acc[0].any()
        k = (-ph) % 2048
        v = np.full(N, MU, np.int64)
        rot = np.roll(v, k % N)
        rot[: k % N] *= -1
        if k >= N:
            rot = -rot
        assert np.array_equal(acc[1], (rot % 2**32).astype(np.uint32))


def test_sample_extract_definition():
    rng = np.random.default_rng(9)
    acc = rng.integers(0, 2**32, size=(2, N), dtype=np.uint64).astype(np.uint32)
    out = O.sample_extract(acc)
    assert out[0] == acc[0, 0] and out[N] == acc[1, 0]
    for j in (1, 2, 500, 1023):
        assert out[j] == (2**32 - int(acc[0, N - j])) % 2**32


def test_sample_extract_phase_is_constant_coefficient(oracle_keys):
    """phase of the extracted LWE under S = constant coefficient of B - A*S."""
    rng = np.random.default_rng(10)
    A = rng.integers(0, 2**32, size=N, dtype=np.uint64).astype(np.uint32)
    B = rng.integers(0, 2**32, size=N, dtype=np.uint64).astype(np.uint32)
    ext = O.sample_extract(np.stack([A, B]))
    prod = np.zeros(N, np.uint32)
    O.lib().orc_negamul_schoolbook(N, np.ascontiguousarray(oracle_keys.S, np.int32), A, prod)
    assert int(O.phase(oracle_keys, ext)) == (int(B[0]) - int(prod[0])) % 2**32


def test_keyswitch_preserves_phase(oracle_keys):
    rng = np.random.default_rng(12)
    for _ in range(3):
        a = rng.integers(0, 2**32, size=N, dtype=np.uint64).astype(np.uint32)
        mu = int(rng.integers(0, 2**32))
        ct = np.zeros(N + 1, np.uint32)
        ct[:N] = a
        ct[N] = (int((a.astype(np.uint64) * oracle_keys.S).sum()) + mu) % 2**32
        out = O.keyswitch(oracle_keys, ct)
        err = (int(O.phase(oracle_keys, out)) - mu) % 2**32
        err = err - 2**32 if err >= 2**31 else err
        # rounding (std ~2^18.7) plus key-switching-key noise (std ~2^23.3)
        assert abs(err) < 2**27


def _truth(op, a, b, c):
    return {O.AND: a & b, O.OR: a | b, O.NAND: 1 - (a & b), O.XOR: a ^ b,
            O.XNOR: 1 - (a ^ b), O.NOT: 1 - a, O.MUX: b if a else c}[op]


def test_gate_truth_tables(oracle_keys):
    K = oracle_keys
    masks, noise = synth.lwe_randomness(0x5EED0002, "truth", 3 * 8)
    jobs, want = [], []
    i = 0
    for op in (O.AND, O.OR, O.NAND, O.XOR, O.XNOR, O.NOT, O.MUX):
        combos = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in ((0, 1) if op == O.MUX else (0,))]
        for (a, b, c) in combos:
            cts = O.encrypt_bits(K, np.array([a, b, c]), masks[(3 * i) % 24:(3 * i) % 24 + 3], noise[(3 * i) % 24:(3 * i) % 24 + 3])
            i += 1
            jobs.append((op, cts[0], cts[1], cts[2]))
            want.append(_truth(op, a, b, c))
    outs = O.gates_parallel(K, jobs)
    for (op, *_), out, w in zip(jobs, outs, want):
        assert int(O.decrypt(K, out)) == w, op
        ph = int(O.phase(K, out))
        target = MU if w else 2**32 - MU
        err = (ph - target) % 2**32
        err = err - 2**32 if err >= 2**31 else err
        assert abs(err) < 2**27, (op, err)  # within 1/32 of +-1/8


def test_fresh_encryption_decrypts(oracle_keys):
    masks, noise = synth.lwe_randomness(0x5EED0003, "fresh", 64)
    bitsv = np.random.default_rng(1).integers(0, 2, 64)
    cts = O.encrypt_bits(oracle_keys, bitsv, masks, noise)
    assert np.array_equal(O.decrypt(oracle_keys, cts), bitsv.astype(np.uint8))


@pytest.mark.slow
def test_schoolbook_bootstrap_equals_transform_bootstrap(oracle_keys):
    """One full bootstrap with every product taken by the schoolbook sum."""
    rng = np.random.default_rng(13)
    ct = _rand_ct(rng)
    ref = O.bootstrap_wo_ks(oracle_keys, ct)
    O.lib().orc_set_schoolbook(1)
    try:
        sb = O.bootstrap_wo_ks(oracle_keys, ct)
    finally:
        O.lib().orc_set_schoolbook(0)
    assert np.array_equal(ref, sb)


def test_vectorised_encryption_matches_scalar(oracle_keys):
    masks, noise = synth.lwe_randomness(0x5EED0004, "vec", 40)
    bitsv = np.random.default_rng(2).integers(0, 2, 40)
    a = O.encrypt_bits(oracle_keys, bitsv, masks, noise)
    b = O.encrypt_bits_np(oracle_keys, bitsv, masks, noise)
    assert np.array_equal(a, b)
