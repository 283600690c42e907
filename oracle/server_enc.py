"""Oracle for the preprocessing phase: PubKeyGen (Alg. 1) and ServerEnc (Alg. 2).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the product
library.

PubKeyGen (client side) draws one LWE encryption of zero per ciphertext slot
of the encrypted database; ServerEnc (server side) adds the trivial
ciphertext (0, Ecd(bit)) of each database bit to its slot, so the server
encrypts without the secret key.  The slot layouts are the evaluation call's
database layouts:
  IntV [M][d][2][l_I]  (left bound, right bound)
  CoV  [M][d][l_I]
  IdM  [M][l_I]
  payload [M][l_S]
Reading: for IntV each record holds two integers per coordinate (the bounds
of its interval), so the interval public key holds two ciphertexts per
(record, bit, coordinate) where Alg. 1 writes one.

Bits are LSB first; bit j of an integer is bit j of its two's-complement
form (signed for IntV and CoV, unsigned identifiers for IdM: both are the
same low l_I bits).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def loc_slots(mode: str, M: int, l: int, d: int) -> tuple:
    """Shape of the location-slot array (without the ciphertext axis)."""
    if mode == "intv":
        return (M, d, 2, l)
    if mode == "cov":
        return (M, d, l)
    if mode == "idm":
        return (M, l)
    raise ValueError(mode)


def pub_key_gen(keys: O.Keys, slots: tuple, masks, noise) -> np.ndarray:
    """Alg. 1: for every slot, a uniform mask a and noise e give the
    encryption of zero (a, <a, s> + e).  masks [..][n], noise [..] (ints)."""
    masks = np.asarray(masks, np.uint32).reshape(-1, O.n)
    noise = np.asarray(noise, np.int64).reshape(-1)
    count = int(np.prod(slots))
    assert masks.shape[0] == count and noise.shape[0] == count
    s = keys.s.astype(np.int64)
    out = np.empty((count, O.n + 1), np.uint32)
    for t in range(count):
        a = masks[t].astype(np.int64)
        b = (int(np.dot(a, s)) + int(noise[t])) % (1 << 32)
        out[t, :O.n] = masks[t]
        out[t, O.n] = b
    return out.reshape(slots + (O.n + 1,))


def bit_of(value: int, j: int) -> int:
    """Bit j (LSB = 0) of the two's-complement form of an integer."""
    return (int(value) >> j) & 1


def server_enc_loc(mode: str, l: int, pk_loc, loc) -> np.ndarray:
    """Alg. 2, location part: slot (record i, bit j, coordinate k [, bound])
    becomes pk + (0, Ecd(x_{i,k}[j])).  loc: IntV [M][d][2], CoV [M][d],
    IdM [M] integers."""
    pk = np.asarray(pk_loc, np.uint32)
    out = pk.copy()
    loc = np.asarray(loc)
    M = loc.shape[0]
    for i in range(M):
        for j in range(l):
            if mode == "idm":
                x = int(loc[i])
                out[i, j, O.n] = (int(pk[i, j, O.n]) + O.encode(bit_of(x, j))) % (1 << 32)
                continue
            for k in range(loc.shape[1]):
                if mode == "intv":
                    for side in range(2):
                        x = int(loc[i, k, side])
                        out[i, k, side, j, O.n] = (int(pk[i, k, side, j, O.n]) + O.encode(bit_of(x, j))) % (1 << 32)
                else:
                    x = int(loc[i, k])
                    out[i, k, j, O.n] = (int(pk[i, k, j, O.n]) + O.encode(bit_of(x, j))) % (1 << 32)
    return out


def server_enc_pay(pk_pay, pay) -> np.ndarray:
    """Alg. 2, payload part: slot (record i, bit j) becomes pk + (0, Ecd(S_i[j]));
    a payload byte that is not zero is the bit 1."""
    pk = np.asarray(pk_pay, np.uint32)
    out = pk.copy()
    pay = np.asarray(pay)
    M, lS = pay.shape
    for i in range(M):
        for j in range(lS):
            bit = 1 if int(pay[i, j]) != 0 else 0
            out[i, j, O.n] = (int(pk[i, j, O.n]) + O.encode(bit)) % (1 << 32)
    return out
