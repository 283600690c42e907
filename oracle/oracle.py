"""Python face of the CPU oracle (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product library.

It wraps the C oracle (keys, encryption, BlindRotate / SampleExtract /
KeySwitch, gates) and runs independent gates on a thread pool; ctypes
releases the GIL during each foreign call, so threads give real parallelism.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "tfhe_oracle.c")

n, N, ELL, KS_T, KS_BASE = 630, 1024, 3, 8, 4
MU = 1 << 29  # 1/8 on the torus
AND, OR, NAND, XOR, XNOR, NOT, MUX = range(7)
GATE_NAMES = {"AND": AND, "OR": OR, "NAND": NAND, "XOR": XOR, "XNOR": XNOR, "NOT": NOT, "MUX": MUX}


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler."""
    if force or not os.path.exists(LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wno-maybe-uninitialized",
                               "-shared", "-fPIC", "-o", LIB_PATH, SRC_PATH])
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        vp = ctypes.c_void_p
        sig = {
            "orc_init": (None, []),
            "orc_prime": (ctypes.c_uint64, []),
            "orc_psi": (ctypes.c_uint64, [ctypes.c_int]),
            "orc_ntt_forward": (None, [ctypes.c_int, u64p, u64p]),
            "orc_ntt_inverse": (None, [ctypes.c_int, u64p, u64p]),
            "orc_set_schoolbook": (None, [ctypes.c_int]),
            "orc_negamul_schoolbook": (None, [ctypes.c_int, i32p, u32p, u32p]),
            "orc_negamul_ntt": (None, [ctypes.c_int, i32p, u32p, u32p]),
            "orc_mul_by_xk": (None, [ctypes.c_int, u32p, ctypes.c_int, u32p]),
            "orc_modswitch": (ctypes.c_uint32, [ctypes.c_uint32]),
            "orc_decompose": (None, [ctypes.c_uint32, i32p]),
            "orc_ks_digits": (None, [ctypes.c_uint32, u32p]),
            "orc_lwe_encrypt": (None, [ctypes.c_int, u32p, u32p, ctypes.c_int32, ctypes.c_uint32, u32p]),
            "orc_lwe_phase": (ctypes.c_uint32, [ctypes.c_int, u32p, u32p]),
            "orc_lwe_decrypt": (ctypes.c_int, [ctypes.c_int, u32p, u32p]),
            "orc_keygen_bk": (None, [u32p, u32p, u32p, i32p, u32p]),
            "orc_keygen_ksk": (None, [u32p, u32p, u32p, i32p, u32p]),
            "orc_keys_load": (vp, [u32p, u32p]),
            "orc_keys_free": (None, [vp]),
            "orc_blind_rotate": (None, [vp, u32p, ctypes.c_uint32, u32p]),
            "orc_sample_extract": (None, [u32p, u32p]),
            "orc_keyswitch": (None, [vp, u32p, u32p]),
            "orc_bootstrap_wo_ks": (None, [vp, u32p, ctypes.c_uint32, u32p]),
            "orc_bootstrap": (None, [vp, u32p, ctypes.c_uint32, u32p]),
            "orc_gate": (ctypes.c_int, [vp, ctypes.c_int, u32p, u32p, u32p, u32p]),
            "orc_modswitch_arr": (None, [ctypes.c_size_t, u32p, u32p]),
            "orc_decompose_arr": (None, [ctypes.c_size_t, u32p, i32p]),
            "orc_ks_digits_arr": (None, [ctypes.c_size_t, u32p, u32p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        L.orc_init()
        _lib = L
    return _lib


def _u32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x).astype(np.uint32))


# ----------------------------------------------------------------------------
# Keys
# ----------------------------------------------------------------------------
class Keys:
    """A client key set as the oracle holds it: secret keys plus evaluation keys.

    bk: u32 [630][6][2][1024] (coefficient domain), ksk: u32 [1024][8][4][631].
    """

    def __init__(self, s, S, bk, ksk):
        self.s = _u32(s)
        self.S = _u32(S)
        self.bk = _u32(bk)
        self.ksk = _u32(ksk)
        self._h = lib().orc_keys_load(self.bk, self.ksk)
        if not self._h:
            raise MemoryError("oracle key load failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_keys_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h


def keygen(rand: dict) -> Keys:
    """Build a key set from the random numbers of synth.key_randomness()."""
    L = lib()
    s, S = _u32(rand["s"]), _u32(rand["S"])
    bk = np.zeros((n, 2 * ELL, 2, N), np.uint32)
    L.orc_keygen_bk(s, S, _u32(rand["bk_mask"]), np.ascontiguousarray(rand["bk_noise"], np.int32), bk)
    ksk = np.zeros((N, KS_T, KS_BASE, n + 1), np.uint32)
    L.orc_keygen_ksk(s, S, _u32(rand["ksk_mask"]), np.ascontiguousarray(rand["ksk_noise"], np.int32), ksk)
    return Keys(s, S, bk, ksk)


def degenerate_keys(s) -> Keys:
    """Noise-free keys with an all-zero ring key S: BK_i = s_i * gadget, KSK = 0.

    With these keys every bootstrap is a closed form (see test-suite)."""
    s = _u32(s)
    bk = np.zeros((n, 2 * ELL, 2, N), np.uint32)
    for r in range(2 * ELL):
        c, j = divmod(r, ELL)
        bk[:, r, c, 0] = (s.astype(np.uint64) << np.uint64(32 - 7 * (j + 1))).astype(np.uint32)
    ksk = np.zeros((N, KS_T, KS_BASE, n + 1), np.uint32)
    return Keys(s, np.zeros(N, np.uint32), bk, ksk)


# ----------------------------------------------------------------------------
# LWE helpers
# ----------------------------------------------------------------------------
def encode(bit: int) -> int:
    """Ecd(m) = m/4 - 1/8 as a torus32 word (Section 2.2)."""
    return MU if bit else (2**32 - MU)


def encrypt_bits(keys: Keys, bits_arr, masks, noise) -> np.ndarray:
    """Encrypt an array of bits; masks [..., 630], noise [...]; returns [..., 631]."""
    L = lib()
    b = np.asarray(bits_arr).astype(np.uint32)
    shape = b.shape
    bf = b.reshape(-1)
    mf = _u32(masks).reshape(-1, n)
    nf = np.asarray(noise, np.int32).reshape(-1)
    out = np.zeros((bf.size, n + 1), np.uint32)
    for i in range(bf.size):
        L.orc_lwe_encrypt(n, keys.s, np.ascontiguousarray(mf[i]), int(nf[i]), encode(int(bf[i])), out[i])
    return out.reshape(shape + (n + 1,))


def encrypt_bits_np(keys: Keys, bits_arr, masks, noise) -> np.ndarray:
    """Same as encrypt_bits, vectorised with numpy (b = <a, s> + Ecd(bit) + e mod 2^32)."""
    b = np.asarray(bits_arr).astype(np.uint64)
    shape = b.shape
    m = _u32(masks).reshape(-1, n)
    dot = (m.astype(np.uint64) * keys.s.astype(np.uint64)[None, :]).sum(axis=1)
    mu = np.where(b.reshape(-1) == 1, MU, 2**32 - MU).astype(np.uint64)
    e = np.asarray(noise, np.int64).reshape(-1).astype(np.uint64)
    body = (dot + mu + e) & np.uint64(0xFFFFFFFF)
    out = np.empty((m.shape[0], n + 1), np.uint32)
    out[:, :n] = m
    out[:, n] = body.astype(np.uint32)
    return out.reshape(shape + (n + 1,))


def trivial(bit: int) -> np.ndarray:
    """Noiseless ciphertext (0, Ecd(bit))."""
    ct = np.zeros(n + 1, np.uint32)
    ct[n] = encode(bit)
    return ct


def phase(keys: Keys, ct) -> np.ndarray:
    ct = _u32(ct)
    flat = ct.reshape(-1, ct.shape[-1])
    d = flat.shape[1] - 1
    key = keys.s if d == n else keys.S
    # b - <a, s> (mod 2^32), with int64 accumulation then wrap.
    acc = (flat[:, :d].astype(np.uint64) * key.astype(np.uint64)).sum(axis=1) & 0xFFFFFFFF
    ph = (flat[:, d].astype(np.uint64) - acc) & 0xFFFFFFFF
    return ph.astype(np.uint32).reshape(ct.shape[:-1])


def decrypt(keys: Keys, ct) -> np.ndarray:
    """Bit = 1 iff the phase, as a signed word, is >= 0 (nearest of +-1/8)."""
    return (phase(keys, ct).astype(np.int64) < 2**31).astype(np.uint8)


# Decryption is correct while a ciphertext's noise stays below 1/16 of the
# torus (Section 2.2; a gate's input is the sum of two ciphertexts, whose
# noise must stay below the 1/8 distance between the encodings and 0).
NOISE_BUDGET = 1 << 28  # 1/16 as a torus32 word


def noise_of(keys: Keys, ct) -> np.ndarray:
    """Signed noise of ciphertexts (int64 words): the phase, centred, minus the
    nearer of the two encodings +-1/8."""
    ph = phase(keys, ct).astype(np.int64)
    ph = np.where(ph >= 2**31, ph - 2**32, ph)
    return np.where(ph >= 0, ph - MU, ph + MU)


def decrypt_checked(keys: Keys, ct) -> tuple[np.ndarray, np.ndarray]:
    """(bits, ok): the decrypted bits, and ok = False wherever the noise has
    reached the 1/16 budget -- there the phase lies within 1/16 of a decision
    boundary (0 or 1/2) and the bit may be wrong."""
    return decrypt(keys, ct), np.abs(noise_of(keys, ct)) < NOISE_BUDGET


# ----------------------------------------------------------------------------
# Bootstrapping and gates
# ----------------------------------------------------------------------------
def blind_rotate(keys: Keys, ct, mu: int = MU) -> np.ndarray:
    out = np.zeros((2, N), np.uint32)
    lib().orc_blind_rotate(keys.handle, _u32(ct), mu, out)
    return out


def sample_extract(trlwe) -> np.ndarray:
    out = np.zeros(N + 1, np.uint32)
    lib().orc_sample_extract(_u32(trlwe), out)
    return out


def keyswitch(keys: Keys, ct_N) -> np.ndarray:
    out = np.zeros(n + 1, np.uint32)
    lib().orc_keyswitch(keys.handle, _u32(ct_N), out)
    return out


def bootstrap_wo_ks(keys: Keys, ct, mu: int = MU) -> np.ndarray:
    out = np.zeros(N + 1, np.uint32)
    lib().orc_bootstrap_wo_ks(keys.handle, _u32(ct), mu, out)
    return out


def bootstrap(keys: Keys, ct, mu: int = MU) -> np.ndarray:
    out = np.zeros(n + 1, np.uint32)
    lib().orc_bootstrap(keys.handle, _u32(ct), mu, out)
    return out


def gate(keys: Keys, op, a, b=None, c=None) -> np.ndarray:
    if isinstance(op, str):
        op = GATE_NAMES[op]
    z = np.zeros(n + 1, np.uint32)
    a = _u32(a)
    b = _u32(b) if b is not None else z
    c = _u32(c) if c is not None else z
    out = np.zeros(n + 1, np.uint32)
    rc = lib().orc_gate(keys.handle, int(op), a, b, c, out)
    if rc != 0:
        raise ValueError("bad gate op %r" % op)
    return out


def xor_k(keys: Keys, cts) -> np.ndarray:
    """XOR of k >= 2 ciphertexts with one bootstrap: the k-input form of the
    XOR gate's pre-combination, (0, (k-1)/4) + 2 * (c_1 + ... + c_k), whose
    phase is -1/4 for an even number of ones and +1/4 for an odd number; then
    BlindRotate with test value 1/8, SampleExtract and KeySwitch.  k = 2 is
    the XOR gate (0, 1/4) + 2(a + b).  Noise: 4k times an input's variance."""
    cts = [_u32(c) for c in cts]
    k = len(cts)
    if k < 2:
        raise ValueError("xor_k needs at least two inputs")
    acc = np.zeros(n + 1, np.uint64)
    for c in cts:
        acc += 2 * c.astype(np.uint64)
    acc[n] += (k - 1) * (1 << 30)
    return bootstrap(keys, (acc & np.uint64(0xFFFFFFFF)).astype(np.uint32), MU)


def modswitch_arr(x) -> np.ndarray:
    x = _u32(x)
    out = np.zeros_like(x)
    lib().orc_modswitch_arr(x.size, x, out)
    return out


def decompose_arr(x) -> np.ndarray:
    x = _u32(x)
    out = np.zeros(x.shape + (ELL,), np.int32)
    lib().orc_decompose_arr(x.size, x, out)
    return out


def ks_digits_arr(x) -> np.ndarray:
    x = _u32(x)
    out = np.zeros(x.shape + (KS_T,), np.uint32)
    lib().orc_ks_digits_arr(x.size, x, out)
    return out


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def gates_parallel(keys: Keys, jobs, threads: int | None = None) -> list:
    """Run independent gates [(op, a, b, c), ...] on a thread pool."""
    threads = threads or default_threads()
    if threads == 1 or len(jobs) <= 1:
        return [gate(keys, *j) for j in jobs]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda j: gate(keys, *j), jobs))
