"""Pins against the tables the paper prints (fixtures under tests/golden/,
each citing its table):

  Table 5  TFHE parameters: the oracle's constants and key shapes, the
           library's parameter set, the input generator's noise widths, and
           the algorithmic count per blind rotation that the roofline uses;
  Table 3  dataset shapes and the modes run on them: the query shapes the
           benchmark evaluates, and the library's host plan of each equal to
           the oracle's circuit graph;
  Table 2  maximum parallel units per component: the widest level of every
           circuit of the oracle (comparators and equality tests l_I gates
           wide, IntV 2d and CoV d of them, selection l_S, the pairwise
           aggregation floor(M/2) l_S, which is M l_S / 2 for even M, a
           query M records wide).
"""
import math
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

from oracle import circuits as C
from oracle import oracle as O
import synth
from paper_2506_12761_amd import vlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].split()
        if line:
            out.append(line)
    return out


def _params():
    return {k: int(v) for k, v in _rows("table5_tfhe_params.txt")}


def _datasets():
    return [(r[0], int(r[1]), int(r[2]), int(r[3]), r[4].split(",")) for r in _rows("table3_datasets.txt")]


def _units():
    return {r[0]: (r[1], r[2]) for r in _rows("table2_parallel_units.txt")}


def _eval_units(expr, **env):
    """A product of integers and variable names, optionally over an integer."""
    num, _, den = expr.partition("/")
    v = Fraction(1)
    for tok in num.split("*"):
        v *= int(tok) if tok.isdigit() else env[tok]
    return v / (int(den) if den else 1)


# ---------------------------------------------------------------- Table 5

def test_fixture_parameters_complete():
    assert set(_params()) == {"n", "k", "N", "ks_base_log2", "ks_levels", "ks_sigma_log2", "bk_base_log2",
                              "bk_levels", "bk_sigma_log2"}


def test_oracle_constants_and_key_shapes():
    p = _params()
    assert (O.n, O.N, O.ELL, O.KS_T, O.KS_BASE) == (p["n"], p["N"], p["bk_levels"], p["ks_levels"],
                                                    2 ** p["ks_base_log2"])
    keys = O.keygen(synth.key_randomness(0x7AB1E5))
    k1 = p["k"] + 1
    assert keys.bk.shape == (p["n"], k1 * p["bk_levels"], k1, p["N"])
    assert keys.ksk.shape == (p["N"], p["ks_levels"], 2 ** p["ks_base_log2"], p["n"] + 1)


def test_library_parameter_set():
    p = _params()
    q = vlp.vlp_default_params()
    assert (q.n, q.N, q.k, q.bg_bit, q.ell, q.ks_basebit, q.ks_t) == (
        p["n"], p["N"], p["k"], p["bk_base_log2"], p["bk_levels"], p["ks_base_log2"], p["ks_levels"])


def test_generator_noise_widths():
    """Key noise words are round(sigma 2^32 g): their sample standard
    deviation matches the table's sigma (3.9M bootstrapping-key samples, 1%;
    24,576 key-switching-key samples, 3%)."""
    p = _params()
    assert (synth.SIGMA_BK_LOG2, synth.SIGMA_LWE_LOG2) == (p["bk_sigma_log2"], p["ks_sigma_log2"])
    r = synth.key_randomness(0x7AB1E6)
    for name, lg, tol in (("bk_noise", p["bk_sigma_log2"], 0.01), ("ksk_noise", p["ks_sigma_log2"], 0.03)):
        x = r[name].astype(np.float64).ravel()
        want = 2.0 ** (32 + lg)
        assert abs(x.mean()) < 5 * want / math.sqrt(x.size), name
        assert abs(x.std() / want - 1) < tol, (name, x.std(), want)


def test_roofline_count_from_the_parameters():
    """Per CMux: (k+1) l_BK forward and k+1 inverse transforms of N/2 log2 N
    butterflies, and (k+1) x (k+1) l_BK pointwise rows of N products; n CMux
    steps per blind rotation."""
    p = _params()
    sys.path.insert(0, ROOT)
    import bench
    k1, N = p["k"] + 1, p["N"]
    transforms = k1 * p["bk_levels"] + k1
    per_cmux = transforms * (N // 2) * int(math.log2(N)) + k1 * k1 * p["bk_levels"] * N
    assert bench.MODMUL_PER_BR == p["n"] * per_cmux


# ---------------------------------------------------------------- Table 3

def test_benchmark_shapes_are_the_datasets():
    want = {(name, mode, M, lI, lS) for name, M, lI, lS, modes in _datasets() for mode in modes}
    sys.path.insert(0, ROOT)
    import bench
    assert set(bench.TABLE3) == want and len(bench.TABLE3) == len(want)


def _query_graph(mode, M, l, lS, d, opt=True, agg_k=0):
    G = C.GraphBuilder()
    if mode == "intv":
        q = [[G.input(("q", k, i)) for i in range(l)] for k in range(d)]
        db = [[([G.input(("lo", r, k, i)) for i in range(l)], [G.input(("hi", r, k, i)) for i in range(l)])
               for k in range(d)] for r in range(M)]
    elif mode == "cov":
        q = [[G.input(("q", k, i)) for i in range(l)] for k in range(d)]
        db = [[[G.input(("c", r, k, i)) for i in range(l)] for k in range(d)] for r in range(M)]
    else:
        q = [G.input(("q", i)) for i in range(l)]
        db = [[G.input(("id", r, i)) for i in range(l)] for r in range(M)]
    pay = [[G.input(("S", r, j)) for j in range(lS)] for r in range(M)] if lS else None
    C.query(G, mode, q, db, pay, l, optimized=opt, agg_k=agg_k)
    return G


@pytest.mark.parametrize("row", _datasets(), ids=lambda r: r[0])
def test_library_plan_of_each_dataset_shape(row):
    name, M, l, lS, modes = row
    for mode in modes:
        d = 1 if mode == "idm" else 2
        for opt, agg_k in ((False, 0), (True, 0), (True, 16)):
            c = vlp.vlp_plan_counts(vlp.make_shape(mode, M, l, lS, d, opt, agg_k))
            G = _query_graph(mode, M, l, lS, d, opt, agg_k)
            g, br = G.counts()
            assert (c["gates"], c["blind_rotations"], c["levels"]) == (g, br, G.depth()), (name, mode, opt, agg_k)


# ---------------------------------------------------------------- Table 2

def _widest(G):
    """Most gates on one level of the graph (inputs and constants excluded)."""
    per = {}
    for nd, lvl in zip(G.nodes, G.level):
        if nd[0] not in ("in", "const"):
            per[lvl] = per.get(lvl, 0) + 1
    return max(per.values(), default=0)


def _bits(G, name, l):
    return [G.input((name, i)) for i in range(l)]


SHAPES = [(M, 16, lS) for _, M, _, lS, _ in _datasets()] + [(1, 1, 1), (2, 3, 5), (5, 8, 7), (6, 2, 3), (7, 20, 4)]


def test_fixture_components():
    assert set(_units()) == {"large-scale", "homsum", "bitwise-and", "intv", "cov", "idm", "comp", "eq"}


@pytest.mark.parametrize("shape", SHAPES)
def test_innermost_components_are_l_bits_wide(shape):
    M, l, lS = shape
    U = _units()
    assert U["comp"][1] == U["eq"][1] == "innermost"
    for strict in (False, True):
        G = C.GraphBuilder()
        C.comp(G, _bits(G, "a", l), _bits(G, "b", l), l, strict)
        assert _widest(G) == _eval_units(U["comp"][0], l_I=l)
    for eq in (C.eq_opt, C.eq_chain):
        G = C.GraphBuilder()
        eq(G, _bits(G, "a", l), _bits(G, "b", l), l)
        assert _widest(G) == _eval_units(U["eq"][0], l_I=l)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("d", [1, 2])
def test_mid_level_components(shape, d):
    M, l, lS = shape
    U = _units()
    for comp in ("intv", "cov", "idm", "bitwise-and"):
        assert U[comp][1] == "mid"
    G = C.GraphBuilder()
    C.intv(G, [_bits(G, ("x", k), l) for k in range(d)],
           [(_bits(G, ("lo", k), l), _bits(G, ("hi", k), l)) for k in range(d)], l)
    assert _widest(G) == _eval_units(U["intv"][0], d=d) * l
    G = C.GraphBuilder()
    C.cov(G, [_bits(G, ("x", k), l) for k in range(d)], [_bits(G, ("c", k), l) for k in range(d)], l)
    assert _widest(G) == _eval_units(U["cov"][0], d=d) * l
    G = C.GraphBuilder()
    C.idm(G, _bits(G, "q", l), _bits(G, "id", l), l)
    assert _widest(G) == _eval_units(U["idm"][0]) * l
    G = C.GraphBuilder()
    C.select(G, G.input("v"), _bits(G, "S", lS))
    assert _widest(G) == _eval_units(U["bitwise-and"][0], l_S=lS)


@pytest.mark.parametrize("shape", SHAPES)
def test_outermost_components(shape):
    """The pairwise aggregation's first level XORs floor(M/2) record pairs
    (M l_S / 2 for even M); a query validates its M records side by side."""
    M, l, lS = shape
    U = _units()
    assert U["homsum"][1] == U["large-scale"][1] == "outermost"
    G = C.GraphBuilder()
    C.homsum_tree(G, [_bits(G, ("S", r), lS) for r in range(M)])
    bound = _eval_units(U["homsum"][0], M=M, l_S=lS)
    assert _widest(G) == (M // 2) * lS <= bound and (M % 2 or _widest(G) == bound)
    for mode, d, per_record in (("intv", 2, 2 * 2 * l), ("cov", 2, 2 * l), ("idm", 1, l)):
        G = _query_graph(mode, M, l, 0, d)
        assert _widest(G) == _eval_units(U["large-scale"][0], M=M) * per_record, mode
