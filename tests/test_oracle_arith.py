"""Pins for the oracle's arithmetic: the transform, products and digit conventions.

Each check compares the oracle with something other than itself: the
transform's defining sum evaluated with Python integers, a brute-force
polynomial product written in Python, closed forms (monomial products are
signed rotations), and the defining properties of the rounding and digit
conventions, swept over every rounding bucket.
"""
import numpy as np
import pytest

from oracle import oracle as O

P = (1 << 62) - (1 << 16) + 1


def _is_prime(n):
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:  # deterministic for n < 3.3e24
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_oracle_prime_and_root():
    L = O.lib()
    assert L.orc_prime() == P
    assert _is_prime(P) and (P - 1) % 2048 == 0
    assert P > 2 ** 52  # |exact product coefficient| <= 1024 * 64 * 2^32 = 2^48 < P/2
    for N in (2, 4, 8, 1024):
        psi = L.orc_psi(N)
        assert pow(psi, N, P) == P - 1 and pow(psi, 2 * N, P) == 1


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_ntt_matches_defining_sum(N):
    """Forward transform = sum_j a_j psi^((2k+1)j), evaluated with Python ints."""
    rng = np.random.default_rng(N)
    psi = O.lib().orc_psi(N)
    for _ in range(5):
        a = rng.integers(0, P, size=N, dtype=np.uint64)
        out = np.zeros(N, np.uint64)
        O.lib().orc_ntt_forward(N, a, out)
        want = [sum(int(a[j]) * pow(psi, (2 * k + 1) * j, P) for j in range(N)) % P for k in range(N)]
        assert [int(x) for x in out] == want


@pytest.mark.parametrize("N", [2, 16, 1024])
def test_ntt_roundtrip(N):
    rng = np.random.default_rng(100 + N)
    a = rng.integers(0, P, size=N, dtype=np.uint64)
    f = np.zeros(N, np.uint64)
    g = np.zeros(N, np.uint64)
    O.lib().orc_ntt_forward(N, a, f)
    O.lib().orc_ntt_inverse(N, f, g)
    assert np.array_equal(a, g)


def _negamul_python(d, t):
    """Brute-force product in Z[X]/(X^N+1), reduced mod 2^32 (Python ints)."""
    N = len(d)
    c = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                c[k] += int(d[i]) * int(t[j])
            else:
                c[k - N] -= int(d[i]) * int(t[j])
    return [x % (1 << 32) for x in c]


def _both(N, d, t):
    d = np.ascontiguousarray(d, np.int32)
    t = np.ascontiguousarray(t, np.uint32)
    a = np.zeros(N, np.uint32)
    b = np.zeros(N, np.uint32)
    O.lib().orc_negamul_schoolbook(N, d, t, a)
    O.lib().orc_negamul_ntt(N, d, t, b)
    return a, b


def test_negamul_exhaustive_tiny_rings():
    """Every digit pair in [-64, 63]-edge values x torus edge values, N = 2 and 4."""
    dvals = [-64, -63, -1, 0, 1, 62, 63]
    tvals = [0, 1, 2**31 - 1, 2**31, 2**32 - 1]
    for N in (2, 4):
        import itertools
        dsets = list(itertools.product(dvals, repeat=N)) if N == 2 else \
            [tuple(np.random.default_rng(i).choice(dvals, N)) for i in range(300)]
        tsets = list(itertools.product(tvals, repeat=N)) if N == 2 else \
            [tuple(np.random.default_rng(1000 + i).choice(tvals, N)) for i in range(60)]
        for d in dsets:
            for t in tsets:
                a, b = _both(N, d, t)
                want = _negamul_python(d, t)
                assert list(a) == want and list(b) == want


def test_negamul_random_medium_vs_python():
    rng = np.random.default_rng(7)
    for N in (8, 32):
        for _ in range(10):
            d = rng.integers(-64, 64, size=N)
            t = rng.integers(0, 2**32, size=N, dtype=np.uint64)
            a, b = _both(N, d, t)
            want = _negamul_python(d, t)
            assert list(a) == want and list(b) == want


def test_negamul_n1024_ntt_equals_schoolbook():
    rng = np.random.default_rng(11)
    for dlo, dhi in ((-64, 64), (0, 2)):
        d = rng.integers(dlo, dhi, size=1024)
        t = rng.integers(0, 2**32, size=1024, dtype=np.uint64)
        a, b = _both(1024, d, t)
        assert np.array_equal(a, b)


def test_monomial_product_is_signed_rotation():
    """X^k * p: coefficient j of p moves to j+k, negated when it wraps past N."""
    rng = np.random.default_rng(3)
    N = 1024
    p = rng.integers(0, 2**32, size=N, dtype=np.uint64).astype(np.uint32)
    for k in (0, 1, 5, 511, 1023, 1024, 1025, 2047):
        out = np.zeros(N, np.uint32)
        O.lib().orc_mul_by_xk(N, p, k, out)
        # closed form with numpy: rotate by k mod N, negate the wrapped part, negate all if k >= N
        kk = k % N
        want = np.roll(p, kk).astype(np.int64)
        want[:kk] = -want[:kk]
        if k >= N:
            want = -want
        assert np.array_equal(out, (want % 2**32).astype(np.uint32))
        # and the same via the schoolbook product with the digit monomial +-X^kk
        d = np.zeros(N, np.int32)
        d[kk] = -1 if k >= N else 1
        a, b = _both(N, d, p)
        assert np.array_equal(a, out) and np.array_equal(b, out)


def _bucket_sweep(shift):
    """Every value k*2^shift + r for r at the bucket's edges and middle."""
    k = np.arange(0, 2 ** (32 - shift), dtype=np.uint64)
    half = 1 << (shift - 1)
    offs = [0, 1, half - 1, half, half + 1, (1 << shift) - 1]
    return np.concatenate([((k << np.uint64(shift)) + np.uint64(o)) & np.uint64(0xFFFFFFFF)
                           for o in offs]).astype(np.uint32)


def _signed(x):
    x = np.asarray(x, np.int64) % 2**32
    return np.where(x >= 2**31, x - 2**32, x)


def test_modswitch_rounds_half_up():
    """abar = x * 2048 / 2^32 rounded half up, mod 2048: x - abar*2^21 in [-2^20, 2^20)."""
    x = np.concatenate([_bucket_sweep(21), np.random.default_rng(1).integers(0, 2**32, 2**20, dtype=np.uint64).astype(np.uint32)])
    a = O.modswitch_arr(x)
    assert a.max() < 2048
    err = _signed(x.astype(np.int64) - a.astype(np.int64) * 2**21)
    assert err.min() >= -(2**20) and err.max() < 2**20


def test_decompose_balanced_digits():
    """Digits in [-64, 63]; recomposition sum d_j 2^(32-7(j+1)) is x rounded to
    2^11 (half up): x - recomposition in [-2^10, 2^10)."""
    x = np.concatenate([_bucket_sweep(11), np.random.default_rng(2).integers(0, 2**32, 2**21, dtype=np.uint64).astype(np.uint32)])
    d = O.decompose_arr(x).astype(np.int64)
    assert d.min() >= -64 and d.max() <= 63
    rec = d[:, 0] * 2**25 + d[:, 1] * 2**18 + d[:, 2] * 2**11
    err = _signed(x.astype(np.int64) - rec)
    assert err.min() >= -(2**10) and err.max() < 2**10
    # edge values by hand: 0, the half-up tie, and the top of the torus
    assert O.decompose_arr(np.array([0], np.uint32)).tolist() == [[0, 0, 0]]
    assert O.decompose_arr(np.array([1 << 10], np.uint32)).tolist() == [[0, 0, 1]]
    assert O.decompose_arr(np.array([(1 << 10) - 1], np.uint32)).tolist() == [[0, 0, 0]]
    assert O.decompose_arr(np.array([0x80000000], np.uint32)).tolist() == [[-64, 0, 0]]
    assert O.decompose_arr(np.array([0xFFFFFFFF], np.uint32)).tolist() == [[0, 0, 0]]


def test_ks_digits():
    """Unsigned base-4 digits of x rounded to 16 bits: x - recomposition in [-2^15, 2^15)."""
    x = np.concatenate([_bucket_sweep(16), np.random.default_rng(4).integers(0, 2**32, 2**20, dtype=np.uint64).astype(np.uint32)])
    d = O.ks_digits_arr(x).astype(np.int64)
    assert d.min() >= 0 and d.max() <= 3
    rec = sum(d[:, j] * 2 ** (32 - 2 * (j + 1)) for j in range(8))
    err = _signed(x.astype(np.int64) - rec)
    assert err.min() >= -(2**15) and err.max() < 2**15
