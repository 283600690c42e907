"""Decrypt-failure detection (client side, on the oracle): a ciphertext whose
noise reaches the 1/16 budget of Section 2.2 is flagged, and every wrong
decryption produced by injected oversize noise is among the flagged ones.
Bootstrapping resets the noise, so a gate fed an over-noisy input can return
a clean-looking ciphertext of the wrong bit: the check belongs on the inputs."""
import numpy as np

from oracle import oracle as O
import synth


def _enc(keys, bits, noise, seed):
    masks, _ = synth.lwe_randomness(seed, "noise-test", len(bits))
    return O.encrypt_bits_np(keys, np.asarray(bits), masks, np.asarray(noise, np.int64).astype(np.int32))


def test_fresh_ciphertexts_pass(oracle_keys):
    """Table 5's noise (sigma = 2^-15, budget 1/16 = 2^12 sigma) never trips the detector."""
    g = synth.stream(71, "bits")
    bits = synth.bits(g, (2000,))
    masks, noise = synth.lwe_randomness(72, "fresh", 2000)
    ct = O.encrypt_bits_np(oracle_keys, bits, masks, noise)
    dec, ok = O.decrypt_checked(oracle_keys, ct)
    assert ok.all() and np.array_equal(dec, bits)
    assert np.array_equal(O.noise_of(oracle_keys, ct), noise.astype(np.int64))


def test_injected_oversize_noise_is_flagged(oracle_keys):
    """Noise drawn uniformly with magnitude in [1/16, 3/16): every ciphertext
    is flagged; those whose noise crossed past the boundary (|e| > 1/8 towards
    it) decrypt wrongly, and each of those is flagged."""
    g = synth.stream(73, "oversize")
    bits = synth.bits(g, (3000,)).astype(np.int64)
    mag = g.integers(O.NOISE_BUDGET, 3 * O.NOISE_BUDGET, size=3000, dtype=np.int64)
    sign = np.where(synth.bits(g, (3000,)) == 1, 1, -1)
    ct = _enc(oracle_keys, bits, sign * mag, 74)
    dec, ok = O.decrypt_checked(oracle_keys, ct)
    wrong = dec != bits
    # towards the boundary = towards 0 for both encodings (+1/8 minus, -1/8 plus)
    crossed = (mag > O.MU) & (sign == np.where(bits == 1, -1, 1))
    assert np.array_equal(wrong, crossed) and wrong.sum() > 300
    assert not ok.any()
    assert not (wrong & ok).any()


def test_budget_edge(oracle_keys):
    """The detector's threshold sits exactly at 1/16: noise 2^28 - 1 passes, 2^28 is flagged."""
    e = np.array([O.NOISE_BUDGET - 1, -(O.NOISE_BUDGET - 1), O.NOISE_BUDGET, -O.NOISE_BUDGET], np.int64)
    ct = _enc(oracle_keys, [1, 0, 1, 0], e, 75)
    _, ok = O.decrypt_checked(oracle_keys, ct)
    assert ok.tolist() == [True, True, False, False]


def test_gate_hides_input_noise_so_inputs_are_checked(oracle_keys):
    """An AND gate whose input carries noise past 1/8 computes on the wrong
    bit and outputs a freshly bootstrapped, clean-looking ciphertext of the
    wrong result; the detector fires on that input, not on the output."""
    K = oracle_keys
    a = _enc(K, [1], [-(O.MU + (O.MU >> 1))], 76)[0]   # bit 1 with noise -3/16: reads as 0
    b = _enc(K, [1], [0], 77)[0]
    out = O.gate(K, "AND", a, b)
    out_bit, out_ok = O.decrypt_checked(K, out)
    assert int(out_bit) == 0 and bool(out_ok)          # wrong (1 AND 1 = 1), yet clean
    _, in_ok = O.decrypt_checked(K, np.stack([a, b]))
    assert in_ok.tolist() == [False, True]
