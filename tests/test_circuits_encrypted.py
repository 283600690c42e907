"""Encrypted circuits through the oracle: decryption equals the plaintext predicate."""
import numpy as np

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
