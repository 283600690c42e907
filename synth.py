"""Seeded synthetic input generation.

This module only draws random numbers: uniform torus words, uniform bits and
rounded Gaussian noise words.  It performs none of the scheme's arithmetic
(no encryption, no key construction, no circuit logic), so that both the
CPU oracle and the GPU path can take their inputs from it without sharing
any of the method's computation.

Every draw comes from a named sub-stream of one 64-bit seed.  A sub-stream is
a Philox-4x64 counter generator whose 128-bit key is the first 16 bytes of
SHA-256(b"vlp-synth" || seed || name), so streams are independent of the
order in which they are requested.

Noise convention (paper, Section 2.2 and Table 5): a Gaussian of standard
deviation sigma on the torus becomes the int32 word round(sigma * 2^32 * g)
with g ~ N(0, 1).
"""
from __future__ import annotations

import hashlib
import struct

import numpy as np

# Table 5 standard deviations, as powers of two on the torus.
SIGMA_LWE_LOG2 = -15   # key-switching / LWE-level encryptions
SIGMA_BK_LOG2 = -25    # bootstrapping-key rows (TRLWE level)


def stream(seed: int, name: str) -> np.random.Generator:
    """Independent generator for sub-stream `name` of `seed`."""
    h = hashlib.sha256(b"vlp-synth" + struct.pack("<Q", seed & (2**64 - 1)) + name.encode()).digest()
    key = np.frombuffer(h[:16], dtype=np.uint64).copy()
    return np.random.Generator(np.random.Philox(key=key))


def uniform_u32(g: np.random.Generator, shape) -> np.ndarray:
    """Uniform 32-bit torus words."""
    return g.integers(0, 2**32, size=shape, dtype=np.uint64).astype(np.uint32)


def bits(g: np.random.Generator, shape) -> np.ndarray:
    """Uniform bits as uint32 0/1."""
    return g.integers(0, 2, size=shape, dtype=np.uint32)


def noise_i32(g: np.random.Generator, shape, sigma_log2: int) -> np.ndarray:
    """Rounded Gaussian noise words: round(2^(32+sigma_log2) * N(0,1)) as int32."""
    scale = float(2.0 ** (32 + sigma_log2))
    x = np.rint(g.standard_normal(size=shape) * scale)
    return x.astype(np.int64).astype(np.int32)


def signed_ints(g: np.random.Generator, shape, l: int) -> np.ndarray:
    """Uniform signed l-bit integers in [-2^(l-1), 2^(l-1)) as int64."""
    return g.integers(-(2 ** (l - 1)), 2 ** (l - 1), size=shape, dtype=np.int64)


def unsigned_ints(g: np.random.Generator, shape, l: int) -> np.ndarray:
    """Uniform unsigned l-bit integers as uint64 (l <= 64)."""
    if l == 64:
        return g.integers(0, 2**64 - 1, size=shape, dtype=np.uint64, endpoint=True)
    return g.integers(0, 2**l, size=shape, dtype=np.uint64)


def to_bits(values: np.ndarray, l: int) -> np.ndarray:
    """Two's-complement bit vectors, LSB first: shape values.shape + (l,), uint32 0/1."""
    v = np.asarray(values).astype(np.int64).astype(np.uint64)
    sh = np.arange(l, dtype=np.uint64)
    return ((v[..., None] >> sh) & np.uint64(1)).astype(np.uint32)


# ---------------------------------------------------------------------------
# Randomness bundles.  Each returns only raw random numbers.
# ---------------------------------------------------------------------------

def key_randomness(seed: int, n: int = 630, N: int = 1024, ell: int = 3, ks_t: int = 8,
                   ks_base: int = 4) -> dict:
    """Random numbers a client key generation consumes (secret bits, masks, noise)."""
    return {
        "s": bits(stream(seed, "lwe_key"), (n,)),
        "S": bits(stream(seed, "trlwe_key"), (N,)),
        "bk_mask": uniform_u32(stream(seed, "bk_mask"), (n, 2 * ell, N)),
        "bk_noise": noise_i32(stream(seed, "bk_noise"), (n, 2 * ell, N), SIGMA_BK_LOG2),
        "ksk_mask": uniform_u32(stream(seed, "ksk_mask"), (N, ks_t, ks_base - 1, n)),
        "ksk_noise": noise_i32(stream(seed, "ksk_noise"), (N, ks_t, ks_base - 1), SIGMA_LWE_LOG2),
    }


def lwe_randomness(seed: int, name: str, count: int, n: int = 630) -> tuple[np.ndarray, np.ndarray]:
    """Masks [count][n] and noise [count] for `count` fresh LWE encryptions."""
    masks = uniform_u32(stream(seed, name + ":mask"), (count, n))
    noise = noise_i32(stream(seed, name + ":noise"), (count,), SIGMA_LWE_LOG2)
    return masks, noise


def uniform_keys(seed: int, n: int = 630, N: int = 1024, ell: int = 3, ks_t: int = 8,
                 ks_base: int = 4) -> tuple[np.ndarray, np.ndarray]:
    """Evaluation-key-shaped uniform words.

    Real keys are LWE/RLWE samples, which are indistinguishable from uniform;
    the GPU path's cost does not depend on key values beyond the distribution
    of decomposition digits, so these serve throughput measurement.  The
    ks entries for digit 0 are zero, as in a real key switching key.
    """
    bk = uniform_u32(stream(seed, "uniform_bk"), (n, 2 * ell, 2, N))
    ksk = uniform_u32(stream(seed, "uniform_ksk"), (N, ks_t, ks_base, n + 1))
    ksk[:, :, 0, :] = 0
    return bk, ksk


def uniform_ciphertexts(seed: int, name: str, shape, n: int = 630) -> np.ndarray:
    """Uniform LWE-shaped words [..., n+1] (distributed like fresh ciphertexts)."""
    return uniform_u32(stream(seed, "uniform_ct:" + name), tuple(shape) + (n + 1,))
