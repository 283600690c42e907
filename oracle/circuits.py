"""VeLoPIR gate circuits, written once over an abstract gate builder.

TEST INFRASTRUCTURE ONLY (part of the oracle).

The circuits follow the paper's algorithms in their order of gates:
  comparators  Alg. 5 (HomCompLE) / Alg. 6 (HomCompL), with the XNORs hoisted
               as in Alg. 11 (HomCompLeOPT) -- the same gate graph;
  equality     Alg. 12 (HomEqOPT): XNOR per bit, then a pairwise AND tree
               with strides 1, 2, 4, ...; and Alg. 7 (HomEQ), the AND chain
               from a trivial 1;
  IntV         Alg. 4; CoV Alg. 8; IdM = HomEqOPT on identifier bits (Sec. 4.2);
  selection    Alg. 9 (HomBitwiseAND);
  aggregation  Alg. 10 (HomSum, XOR chain from a trivial 0) and its pairwise
               XOR-tree form of Section 6.1, part (5); and, beyond the paper,
               a k-ary tree of k-input XORs (one bootstrap per k inputs);
  query        Alg. 3 (validate, zero out, aggregate).
Bits are least-significant first; bit l-1 is the two's-complement sign
(Appendix A, proof of Theorem 1).

Two builders run them:
  PlainBuilder  -- numpy booleans, vectorised over many plaintext inputs
                   (brute force against the theorems' predicates);
  GraphBuilder  -- records the gate graph, which `evaluate` then runs on
                   ciphertexts with the oracle, level by level on a thread pool
                   (order of independent gates does not change any result).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import oracle as O

XORK = "xork"  # graph node kind of the k-input XOR


# ----------------------------------------------------------------------------
# Circuits
# ----------------------------------------------------------------------------
def comp(B, c1, c2, l: int, strict: bool):
    """HomCompLE (strict=False) / HomCompL (strict=True): Enc(c1 <= c2) / Enc(c1 < c2)."""
    t0 = B.xor(c1[l - 1], c2[l - 1])
    t1 = [B.xnor(c1[i], c2[i]) for i in range(l - 1)]
    t = B.trivial(0 if strict else 1)
    for i in range(l - 1):
        t = B.mux(t1[i], t, c2[i])
    return B.mux(t0, c1[l - 1], t)


def eq_opt(B, c1, c2, l: int):
    """HomEqOPT: XNOR per bit, then t[i] = AND(t[i], t[i+k]) for k = 1, 2, 4, ..."""
    t = [B.xnor(c1[i], c2[i]) for i in range(l)]
    k = 1
    while k < l:
        for i in range(0, l, 2 * k):
            if i + k < l:
                t[i] = B.and_(t[i], t[i + k])
        k *= 2
    return t[0]


def eq_chain(B, c1, c2, l: int):
    """HomEQ (Alg. 7): r = trivial 1; r = AND(r, XNOR(c1[i], c2[i])) for each bit."""
    r = B.trivial(1)
    for i in range(l):
        r = B.and_(r, B.xnor(c1[i], c2[i]))
    return r


def intv(B, q, loc, l: int):
    """IntV (Alg. 4) for d = len(q) coordinates.

    q[k] = bits of the query coordinate k; loc[k] = (left bits, right bits).
    Per coordinate: AND(CompLE(left, q), CompL(q, right)); then AND over the
    coordinates in order (for d = 2 this is the paper's v = AND(v_x, v_y))."""
    per_dim = []
    lefts = [comp(B, loc[k][0], q[k], l, strict=False) for k in range(len(q))]
    rights = [comp(B, q[k], loc[k][1], l, strict=True) for k in range(len(q))]
    for k in range(len(q)):
        per_dim.append(B.and_(lefts[k], rights[k]))
    v = per_dim[0]
    for k in range(1, len(q)):
        v = B.and_(v, per_dim[k])
    return v


def cov(B, q, loc, l: int, eq=eq_opt):
    """CoV (Alg. 8): AND over coordinates of HomEQ(q[k], loc[k])."""
    vs = [eq(B, q[k], loc[k], l) for k in range(len(q))]
    v = vs[0]
    for k in range(1, len(q)):
        v = B.and_(v, vs[k])
    return v


def idm(B, qid, rid, l: int, eq=eq_opt):
    """IdM: HomEQ directly on the identifier bits, no final AND."""
    return eq(B, qid, rid, l)


def select(B, v, S):
    """HomBitwiseAND (Alg. 9): S[j] = AND(v, S[j])."""
    return [B.and_(v, s) for s in S]


def homsum_tree(B, S):
    """Pairwise XOR reduction over records (Section 6.1 part (5)); R = S[0]."""
    S = [list(x) for x in S]
    M = len(S)
    k = 1
    while k < M:
        for i in range(0, M, 2 * k):
            if i + k < M:
                S[i] = [B.xor(a, b) for a, b in zip(S[i], S[i + k])]
        k *= 2
    return S[0]


def homsum_ktree(B, S, k: int):
    """Aggregation by k-input XORs: the records' selected bits are taken in
    consecutive groups of k, each group XORed with one bootstrap (a group of
    one passes through), and the group results reduced the same way until one
    remains.  k = 2 is a pairwise tree (grouping 0-1, 2-3, ... per round)."""
    cur = [list(x) for x in S]
    while len(cur) > 1:
        nxt = []
        for g in range(0, len(cur), k):
            grp = cur[g:g + k]
            if len(grp) == 1:
                nxt.append(grp[0])
            else:
                nxt.append([B.xork([row[j] for row in grp]) for j in range(len(grp[0]))])
        cur = nxt
    return cur[0]


def homsum_chain(B, S):
    """HomSum (Alg. 10): R = trivial zeros; R[j] = XOR(R[j], S_i[j]) for every record."""
    R = [B.trivial(0) for _ in S[0]]
    for Si in S:
        R = [B.xor(r, s) for r, s in zip(R, Si)]
    return R


def query(B, mode: str, q, db_loc, db_pay, l: int, optimized: bool = True, agg_k: int = 0):
    """VeLoPIR (Alg. 3): returns (v per record, R or None).

    mode: "intv" (db_loc[i] = [(left, right)] per coordinate), "cov"
    (db_loc[i] = [bits] per coordinate) or "idm" (db_loc[i] = id bits, q = id bits).
    agg_k >= 2 aggregates with k-input XORs instead of Alg. 10 / the pairwise tree."""
    eq = eq_opt if optimized else eq_chain
    vs = []
    for loc in db_loc:
        if mode == "intv":
            vs.append(intv(B, q, loc, l))
        elif mode == "cov":
            vs.append(cov(B, q, loc, l, eq))
        elif mode == "idm":
            vs.append(idm(B, q, loc, l, eq))
        else:
            raise ValueError(mode)
    if db_pay is None:
        return vs, None
    sel = [select(B, v, S) for v, S in zip(vs, db_pay)]
    if agg_k >= 2:
        R = homsum_ktree(B, sel, agg_k)
    else:
        R = homsum_tree(B, sel) if optimized else homsum_chain(B, sel)
    return vs, R


# ----------------------------------------------------------------------------
# Builders
# ----------------------------------------------------------------------------
class PlainBuilder:
    """Plaintext gates on numpy boolean arrays."""

    def trivial(self, bit):
        return np.bool_(bool(bit))

    def xor(self, a, b):
        return np.logical_xor(a, b)

    def xnor(self, a, b):
        return np.logical_not(np.logical_xor(a, b))

    def and_(self, a, b):
        return np.logical_and(a, b)

    def mux(self, s, x, y):
        return np.where(s, x, y)

    def xork(self, args):
        r = args[0]
        for a in args[1:]:
            r = np.logical_xor(r, a)
        return r


class GraphBuilder:
    """Records a gate graph; node ids index `self.nodes`.

    Node kinds: ("in", key) -- an input ciphertext supplied at evaluation;
    ("const", bit) -- a trivial ciphertext; (op, a, b, c) -- a gate."""

    def __init__(self):
        self.nodes = []
        self.level = []
        self._inputs = {}

    def _add(self, node, lvl):
        self.nodes.append(node)
        self.level.append(lvl)
        return len(self.nodes) - 1

    def input(self, key):
        if key not in self._inputs:
            self._inputs[key] = self._add(("in", key), 0)
        return self._inputs[key]

    def trivial(self, bit):
        return self._add(("const", int(bit)), 0)

    def _gate(self, op, *args):
        lvl = 1 + max(self.level[a] for a in args)
        return self._add((op,) + tuple(args), lvl)

    def xor(self, a, b):
        return self._gate(O.XOR, a, b)

    def xnor(self, a, b):
        return self._gate(O.XNOR, a, b)

    def and_(self, a, b):
        return self._gate(O.AND, a, b)

    def mux(self, s, x, y):
        return self._gate(O.MUX, s, x, y)

    def xork(self, args):
        return self._gate(XORK, *args)

    def counts(self):
        """(gates, blind rotations) of the recorded graph."""
        g = br = 0
        for nd in self.nodes:
            if nd[0] in ("in", "const"):
                continue
            g += 1
            br += 2 if nd[0] == O.MUX else 1
        return g, br

    def depth(self):
        return max(self.level) if self.level else 0

    def evaluate(self, keys, inputs: dict, threads: int | None = None) -> list:
        """Run every gate with the oracle; inputs maps input key -> ciphertext."""
        vals = [None] * len(self.nodes)
        by_level = {}
        for i, nd in enumerate(self.nodes):
            if nd[0] == "in":
                vals[i] = np.asarray(inputs[nd[1]], np.uint32)
            elif nd[0] == "const":
                vals[i] = O.trivial(nd[1])
            else:
                by_level.setdefault(self.level[i], []).append(i)
        threads = threads or O.default_threads()

        def run(i):
            nd = self.nodes[i]
            args = [vals[a] for a in nd[1:]]
            if nd[0] == XORK:
                return O.xor_k(keys, args)
            while len(args) < 3:
                args.append(None)
            return O.gate(keys, nd[0], *args)

        with ThreadPoolExecutor(max_workers=threads) as ex:
            for lvl in sorted(by_level):
                ids = by_level[lvl]
                for i, out in zip(ids, ex.map(run, ids)):
                    vals[i] = out
        return vals
