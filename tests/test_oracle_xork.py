"""Pins of the k-input XOR and the k-ary aggregation (oracle).

Fixed by: the XOR gate's own definition (k = 2), parity by decryption under
real keys, the measured noise of bootstrapped gate outputs against the
decision threshold of the k-input form, and plaintext parity of the
aggregation tree (PlainBuilder) against numpy's XOR reduction."""
import numpy as np
import pytest

from oracle import circuits as C
from oracle import oracle as O
from oracle import workloads as W
import synth

K_MAX = 16  # the largest k the library accepts


def _enc(keys, bits, seed, name):
    masks, noise = synth.lwe_randomness(seed, name, len(bits))
    return O.encrypt_bits_np(keys, np.asarray(bits), masks, noise)


def test_xor_k_with_two_inputs_is_the_xor_gate(oracle_keys):
    bits = np.array([0, 0, 1, 1, 0, 1])
    a = _enc(oracle_keys, bits, 31, "xk-a")
    b = _enc(oracle_keys, bits[::-1].copy(), 31, "xk-b")
    for i in range(len(bits)):
        assert np.array_equal(O.xor_k(oracle_keys, [a[i], b[i]]), O.gate(oracle_keys, O.XOR, a[i], b[i]))


@pytest.mark.parametrize("k", [3, 4, 5])
def test_xor_k_truth_table(oracle_keys, k):
    pats = [[(p >> t) & 1 for t in range(k)] for p in range(1 << k)]
    cts = _enc(oracle_keys, np.array(pats).reshape(-1), 32 + k, "xk-tt").reshape(len(pats), k, O.n + 1)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(O.default_threads()) as ex:
        outs = list(ex.map(lambda c: O.xor_k(oracle_keys, list(c)), cts))
    got = O.decrypt(oracle_keys, np.stack(outs))
    assert list(got) == [sum(p) % 2 for p in pats]


def test_xor_k_on_gate_outputs_at_the_largest_k(oracle_keys):
    """Inputs that are themselves bootstrapped gate outputs (the aggregation's
    case), k = K_MAX, several random patterns."""
    g = synth.stream(40, "xk-big")
    n_pat = 6
    bits = synth.bits(g, (n_pat * K_MAX,))
    ones = _enc(oracle_keys, np.ones(n_pat * K_MAX, np.uint32), 41, "xk-one")
    x = _enc(oracle_keys, bits, 41, "xk-x")
    gated = O.gates_parallel(oracle_keys, [(O.AND, x[i], ones[i], None) for i in range(n_pat * K_MAX)])
    for p in range(n_pat):
        out = O.xor_k(oracle_keys, gated[p * K_MAX:(p + 1) * K_MAX])
        assert O.decrypt(oracle_keys, out) == int(bits[p * K_MAX:(p + 1) * K_MAX].sum() % 2)


def test_noise_budget_of_the_largest_k(oracle_keys):
    """The phase error of a bootstrapped gate output (measured), summed over
    K_MAX inputs with weight 2, stays far inside the 1/4 decision distance of
    the k-input form: at least 8 standard deviations (Gaussian tail < 1e-15),
    with the modulus-switch rounding of the next bootstrap included."""
    g = synth.stream(42, "xk-noise")
    N = 96
    a, b = synth.bits(g, (N,)), synth.bits(g, (N,))
    A, B = _enc(oracle_keys, a, 43, "xn-a"), _enc(oracle_keys, b, 43, "xn-b")
    outs = np.stack(O.gates_parallel(oracle_keys, [(O.AND, A[i], B[i], None) for i in range(N)]))
    ph = O.phase(oracle_keys, outs).astype(np.int64)
    e = (ph - np.where((a & b) == 1, 2**29, -(2**29))) % 2**32
    e = np.where(e >= 2**31, e - 2**32, e) / 2.0**32
    sigma_u = e.std()
    assert sigma_u < 2.0**-7.5  # a gate output's noise (measured about 2^-8.4)
    sigma_ms = np.sqrt((O.n + 1) / 2 / 12) / 2048  # rounding of ~n/2 key-selected terms to 1/2048
    sigma = np.sqrt(4 * K_MAX * sigma_u**2 + sigma_ms**2)
    assert 0.25 / sigma >= 8.0, (sigma_u, sigma)


def test_ktree_parity_plaintext():
    """The k-ary aggregation computes the XOR over records (all k, ragged M)."""
    g = synth.stream(44, "kt-plain")
    for k in (2, 3, 4, 7, 16):
        for M in (1, 2, 5, 16, 17, 40):
            S = synth.bits(g, (M, 3)).astype(bool)
            got = np.array(C.homsum_ktree(C.PlainBuilder(), list(S), k))
            assert np.array_equal(got, np.logical_xor.reduce(S, axis=0)), (k, M)


def test_ktree_structure():
    """Gate count (M - 1) / (k - 1) per bit rounded up per round, depth ceil(log_k M)."""
    for k in (2, 4, 16):
        for M in (1, 5, 16, 17, 300):
            G = C.GraphBuilder()
            S = [[G.input((i, 0))] for i in range(M)]
            C.homsum_ktree(G, S, k)
            gates, br = G.counts()
            n, rounds, want = M, 0, 0
            while n > 1:
                want += n // k + (1 if n % k > 1 else 0)
                n = (n + k - 1) // k
                rounds += 1
            assert (gates, br, G.depth()) == (want, want, rounds), (k, M)


def test_ktree_query_end_to_end(oracle_keys):
    """An IdM query whose aggregation uses 3-input XORs decrypts to the plaintext R."""
    P = W.plain_workload("idm", 5, 2, 2, 1, seed=8)
    enc = W.encrypt_workload(oracle_keys, P, seed=9)
    v, R = W.oracle_outputs(oracle_keys, P, enc, agg_k=3)
    assert np.array_equal(O.decrypt(oracle_keys, v), P["v"])
    assert np.array_equal(O.decrypt(oracle_keys, R), P["R"])
