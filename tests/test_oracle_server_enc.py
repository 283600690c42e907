"""Pins of the preprocessing oracle (PubKeyGen, Alg. 1; ServerEnc, Alg. 2).

What fixes the expected values here is the definition of LWE decryption and
of Ecd (Section 2.2), and two's-complement bit strings produced by Python's
string formatting (a route that shares nothing with the oracle's shifts)."""
import numpy as np
import pytest

from oracle import circuits as C
from oracle import oracle as O
from oracle import server_enc as SE
from oracle import workloads as W
import synth


def bits_by_format(x: int, l: int) -> list:
    """LSB-first bits of the l-bit two's-complement form, via a binary string."""
    return [int(ch) for ch in reversed(format(x % (1 << l), "0%db" % l))]


@pytest.mark.parametrize("x,l,want", [(-1, 8, [1] * 8), (-8, 4, [0, 0, 0, 1]), (5, 4, [1, 0, 1, 0]),
                                      (-3, 4, [1, 0, 1, 1]), (0, 3, [0, 0, 0]), (2**15 - 1, 16, [1] * 15 + [0])])
def test_bit_of_twos_complement(x, l, want):
    assert [SE.bit_of(x, j) for j in range(l)] == want == bits_by_format(x, l)


def _pk(keys, slots, seed, name):
    count = int(np.prod(slots))
    masks, noise = synth.lwe_randomness(seed, name, count)
    return SE.pub_key_gen(keys, slots, masks, noise), masks, noise


def test_pub_key_is_encryption_of_zero(oracle_keys):
    """Every public-key ciphertext has phase equal to its noise: an encryption of 0."""
    pk, masks, noise = _pk(oracle_keys, (3, 5), 41, "pk")
    ph = O.phase(oracle_keys, pk).astype(np.int64).reshape(-1)
    ph = np.where(ph >= 2**31, ph - 2**32, ph)
    assert np.array_equal(ph, noise.astype(np.int64))
    assert np.array_equal(pk[..., :O.n].reshape(-1, O.n), masks)


@pytest.mark.parametrize("mode,M,l,d", [("intv", 3, 5, 2), ("cov", 4, 6, 1), ("idm", 5, 7, 1)])
def test_server_enc_loc(oracle_keys, mode, M, l, d):
    g = synth.stream(7, "se:" + mode)
    if mode == "intv":
        loc = synth.signed_ints(g, (M, d, 2), l)
    elif mode == "cov":
        loc = synth.signed_ints(g, (M, d), l)
    else:
        loc = synth.unsigned_ints(g, (M,), l).astype(np.int64)
    slots = SE.loc_slots(mode, M, l, d)
    pk, masks, noise = _pk(oracle_keys, slots, 42, "pk:" + mode)
    ct = SE.server_enc_loc(mode, l, pk, loc)
    want = np.array([bits_by_format(int(x), l) for x in np.asarray(loc).reshape(-1)], np.uint8).reshape(slots)
    assert np.array_equal(O.decrypt(oracle_keys, ct), want)
    # The masks are the public key's; the phase is Ecd(bit) plus exactly the key's noise.
    assert np.array_equal(ct[..., :O.n], pk[..., :O.n])
    ph = O.phase(oracle_keys, ct).astype(np.int64).reshape(-1)
    ecd = np.where(want.reshape(-1) == 1, 2**29, -(2**29))
    err = (ph - ecd) % 2**32
    err = np.where(err >= 2**31, err - 2**32, err)
    assert np.array_equal(err, noise.astype(np.int64))


def test_server_enc_pay(oracle_keys):
    pay = np.array([[0, 1, 2, 255], [1, 0, 0, 7]], np.uint8)  # nonzero bytes are 1
    pk, _, noise = _pk(oracle_keys, (2, 4), 43, "pk:pay")
    ct = SE.server_enc_pay(pk, pay)
    assert np.array_equal(O.decrypt(oracle_keys, ct), (pay != 0).astype(np.uint8))
    assert np.array_equal(ct[..., :O.n], pk[..., :O.n])


def test_server_encrypted_db_answers_query(oracle_keys):
    """A database encrypted by ServerEnc under the public key answers an IdM
    query (Alg. 3) with the plaintext result."""
    P = W.plain_workload("idm", 3, 2, 2, 1, seed=5)
    pk_loc, _, _ = _pk(oracle_keys, SE.loc_slots("idm", 3, 2, 1), 44, "pk:l")
    pk_pay, _, _ = _pk(oracle_keys, (3, 2), 44, "pk:p")
    enc = W.encrypt_workload(oracle_keys, P, seed=6)
    enc["db_loc"] = SE.server_enc_loc("idm", 2, pk_loc, P["loc"])
    enc["db_pay"] = SE.server_enc_pay(pk_pay, P["pay"])
    v, R = W.oracle_outputs(oracle_keys, P, enc)
    assert np.array_equal(O.decrypt(oracle_keys, v), P["v"])
    assert np.array_equal(O.decrypt(oracle_keys, R), P["R"])
