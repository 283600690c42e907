"""Plaintext pins for the circuits (theorems of Section 4; proofs in Appendix A).

The circuit code runs on numpy booleans over every input of a small width and
is compared with the predicates the paper proves: signed <= and < (Theorem 1,
Corollary 1), the half-open box of IntV (Theorem 2), equality (Lemma 1) and
CoV (Theorem 3), zero-out (Lemma 2) and aggregation (Lemma 3).  Gate counts
and depths of the recorded gate graphs are checked against counts derived by
hand from the algorithms.
"""
import numpy as np
import pytest

from oracle import circuits as C
import synth

PB = C.PlainBuilder()


def _bits(vals, l):
    """list of l boolean arrays, LSB first (two's complement)."""
    b = synth.to_bits(vals, l).astype(bool)
    return [b[..., i] for i in range(l)]


def test_comparators_all_8bit_pairs():
    l = 8
    v = np.arange(-128, 128)
    x, y = np.meshgrid(v, v, indexing="ij")
    x, y = x.ravel(), y.ravel()
    bx, by = _bits(x, l), _bits(y, l)
    assert np.array_equal(C.comp(PB, bx, by, l, strict=False), x <= y)
    assert np.array_equal(C.comp(PB, bx, by, l, strict=True), x < y)


def test_interval_1d_all_8bit_triples():
    """AND(CompLE(lo, x), CompL(x, hi)) == [lo <= x < hi] over all 2^24 triples."""
    l = 8
    v = np.arange(-128, 128, dtype=np.int64)
    lo, hi = np.meshgrid(v, v, indexing="ij")
    lo, hi = lo.ravel(), hi.ravel()
    blo, bhi = _bits(lo, l), _bits(hi, l)
    for xv in range(-128, 128):
        bx = _bits(np.full(1, xv), l)
        got = C.intv(PB, [bx], [(blo, bhi)], l)
        assert np.array_equal(got, (lo <= xv) & (xv < hi)), xv


def test_interval_2d_random_16bit():
    l = 16
    g = synth.stream(1, "intv2d")
    M = 200000
    x, y, a, b, c, d = (synth.signed_ints(g, M, l) for _ in range(6))
    xl, xr = np.minimum(a, b), np.maximum(a, b)
    yl, yr = np.minimum(c, d), np.maximum(c, d)
    got = C.intv(PB, [_bits(x, l), _bits(y, l)], [(_bits(xl, l), _bits(xr, l)), (_bits(yl, l), _bits(yr, l))], l)
    assert np.array_equal(got, (xl <= x) & (x < xr) & (yl <= y) & (y < yr))


def test_equality_all_8bit_pairs_both_forms():
    l = 8
    v = np.arange(-128, 128)
    x, y = np.meshgrid(v, v, indexing="ij")
    x, y = x.ravel(), y.ravel()
    bx, by = _bits(x, l), _bits(y, l)
    assert np.array_equal(C.eq_opt(PB, bx, by, l), x == y)
    assert np.array_equal(C.eq_chain(PB, bx, by, l), x == y)
    for ll in (1, 3, 5, 7):  # trees with odd widths
        m = (1 << ll) - 1
        assert np.array_equal(C.eq_opt(PB, bx[:ll], by[:ll], ll), (x & m) == (y & m))


def test_cov_and_idm():
    l = 20
    g = synth.stream(2, "cov")
    M = 100000
    x, y = synth.signed_ints(g, M, l), synth.signed_ints(g, M, l)
    lx = np.where(synth.bits(g, M) == 1, x, synth.signed_ints(g, M, l))
    ly = np.where(synth.bits(g, M) == 1, y, synth.signed_ints(g, M, l))
    got = C.cov(PB, [_bits(x, l), _bits(y, l)], [_bits(lx, l), _bits(ly, l)], l)
    assert np.array_equal(got, (x == lx) & (y == ly))
    ids = synth.unsigned_ints(g, M, 32)
    rid = np.where(synth.bits(g, M) == 1, ids, synth.unsigned_ints(g, M, 32))
    got = C.idm(PB, _bits(ids.astype(np.int64), 32), _bits(rid.astype(np.int64), 32), 32)
    assert np.array_equal(got, ids == rid)


def test_select_and_aggregate():
    g = synth.stream(3, "sel")
    M, lS = 13, 9
    S = synth.bits(g, (M, lS)).astype(bool)
    for hit in (None, 0, 5, 12):
        v = np.zeros(M, bool)
        if hit is not None:
            v[hit] = True
        sel = [C.select(PB, v[i], list(S[i])) for i in range(M)]
        for i in range(M):
            assert np.array_equal(np.array(sel[i]), S[i] & v[i])
        want = S[hit] if hit is not None else np.zeros(lS, bool)
        assert np.array_equal(np.array(C.homsum_tree(PB, sel)), want)
        assert np.array_equal(np.array(C.homsum_chain(PB, sel)), want)
    # with several hits the result is the XOR of the selected records
    v = synth.bits(g, M).astype(bool)
    sel = [C.select(PB, v[i], list(S[i])) for i in range(M)]
    want = np.bitwise_xor.reduce(S & v[:, None], axis=0)
    assert np.array_equal(np.array(C.homsum_tree(PB, sel)), want)


def _graph_counts(fn):
    G = C.GraphBuilder()
    fn(G)
    g, br = G.counts()
    return g, br, G.depth()


def _inp(G, name, l):
    return [G.input((name, i)) for i in range(l)]


@pytest.mark.parametrize("l", [8, 16, 20])
def test_gate_counts(l):
    # comparator: 1 XOR + (l-1) XNOR + l MUX -> 3l blind rotations, depth l+1
    g, br, dep = _graph_counts(lambda G: C.comp(G, _inp(G, "a", l), _inp(G, "b", l), l, False))
    assert (br, dep) == (3 * l, l + 1)
    # IntV 2-D: 12l + 3 blind rotations, depth l + 3
    g, br, dep = _graph_counts(lambda G: C.intv(G, [_inp(G, "x", l), _inp(G, "y", l)],
                                                [(_inp(G, "xl", l), _inp(G, "xr", l)), (_inp(G, "yl", l), _inp(G, "yr", l))], l))
    assert (br, dep) == (12 * l + 3, l + 3)
    # equality tree: 2l - 1, depth 1 + ceil(log2 l); CoV: 4l - 1, depth 2 + ceil(log2 l)
    lg = int(np.ceil(np.log2(l)))
    g, br, dep = _graph_counts(lambda G: C.eq_opt(G, _inp(G, "a", l), _inp(G, "b", l), l))
    assert (br, dep) == (2 * l - 1, 1 + lg)
    g, br, dep = _graph_counts(lambda G: C.cov(G, [_inp(G, "x", l), _inp(G, "y", l)], [_inp(G, "lx", l), _inp(G, "ly", l)], l))
    assert (br, dep) == (4 * l - 1, 2 + lg)


def test_config_counts():
    # one-dimensional 8-bit interval: 49 blind rotations, depth 10
    g, br, dep = _graph_counts(lambda G: C.intv(G, [_inp(G, "x", 8)], [(_inp(G, "lo", 8), _inp(G, "hi", 8))], 8))
    assert (br, dep) == (49, 10)

    # identifier match 32 bits + 64-bit payload selection: 63 + 64 per record, 7 levels
    def idm_sel(G):
        v = C.idm(G, _inp(G, "q", 32), _inp(G, "id", 32), 32)
        return C.select(G, v, _inp(G, "S", 64))
    g, br, dep = _graph_counts(idm_sel)
    assert (br, dep) == (127, 7)
