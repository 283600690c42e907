"""Encrypted circuits through the oracle: decryption equals the plaintext predicate."""
import numpy as np
import pytest

from oracle import circuits as C
from oracle import oracle as O
import synth


def _enc_int(K, val, l, name, seed):
    masks, noise = synth.lwe_randomness(seed, name, l)
    return O.encrypt_bits(K, synth.to_bits(np.array([val]), l)[0], masks, noise)


def test_interval_8bit_encrypted(oracle_keys):
    """The 49-bootstrap one-dimensional interval test, for x inside, at the
    left edge and outside a seeded interval."""
    K = oracle_keys
    g = synth.stream(0x5EED0001, "cfg1")
    a, b = (int(v) for v in synth.signed_ints(g, 2, 8))
    lo, hi = min(a, b), max(a, b)
    if lo == hi:
        hi = lo + 1
    G = C.GraphBuilder()
    x = [G.input(("x", i)) for i in range(8)]
    blo = [G.input(("lo", i)) for i in range(8)]
    bhi = [G.input(("hi", i)) for i in range(8)]
    v = C.intv(G, [x], [(blo, bhi)], 8)
    assert G.counts()[1] == 49
    ilo = _enc_int(K, lo, 8, "lo", 11)
    ihi = _enc_int(K, hi, 8, "hi", 12)
    for xv in (lo, hi, (lo + hi) // 2, lo - 1 if lo > -128 else hi + 1):
        if not -128 <= xv < 128:
            continue
        ix = _enc_int(K, xv, 8, "x%d" % xv, 13)
        inputs = {}
        for i in range(8):
            inputs[("x", i)] = ix[i]
            inputs[("lo", i)] = ilo[i]
            inputs[("hi", i)] = ihi[i]
        vals = G.evaluate(K, inputs)
        assert int(O.decrypt(K, vals[v])) == int(lo <= xv < hi), (lo, hi, xv)


@pytest.mark.slow
def test_interval_8bit_encrypted_all_256_values(oracle_keys):
    """Every 8-bit x (all 256) through the encrypted 49-bootstrap interval
    circuit against one seeded interval: 256 independent copies of the
    circuit in one graph (12,544 bootstraps), each decrypting to
    lo <= x < hi (Theorem 2) and passing the noise check."""
    K = oracle_keys
    g = synth.stream(0x5EED0001, "cfg1")
    a, b = (int(v) for v in synth.signed_ints(g, 2, 8))
    lo, hi = min(a, b), max(a, b)
    if lo == hi:
        hi = lo + 1
    G = C.GraphBuilder()
    blo = [G.input(("lo", i)) for i in range(8)]
    bhi = [G.input(("hi", i)) for i in range(8)]
    outs = []
    for xv in range(-128, 128):
        x = [G.input(("x", xv, i)) for i in range(8)]
        outs.append(C.intv(G, [x], [(blo, bhi)], 8))
    assert G.counts()[1] == 49 * 256
    ilo = _enc_int(K, lo, 8, "lo", 11)
    ihi = _enc_int(K, hi, 8, "hi", 12)
    masks, noise = synth.lwe_randomness(13, "x-all", 256 * 8)
    xb = synth.to_bits(np.arange(-128, 128), 8)                     # [256][8]
    ix = O.encrypt_bits_np(K, xb, masks, noise)                      # [256][8][631]
    inputs = {("lo", i): ilo[i] for i in range(8)}
    inputs.update({("hi", i): ihi[i] for i in range(8)})
    for k, xv in enumerate(range(-128, 128)):
        for i in range(8):
            inputs[("x", xv, i)] = ix[k, i]
    vals = G.evaluate(K, inputs)
    got, ok = O.decrypt_checked(K, np.stack([vals[v] for v in outs]))
    want = np.array([int(lo <= xv < hi) for xv in range(-128, 128)], np.uint8)
    assert np.array_equal(got, want) and ok.all()
    assert 0 < want.sum() < 256
