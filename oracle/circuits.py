"""VeLoPIR gate circuits, written once over an abstract gate builder.

TEST INFRASTRUCTURE ONLY (part of the oracle).

The circuits, from their definitions:
  comparators  HomCompLE / HomCompL (Alg. 5 / 6; Alg. 11 is the same gate
               graph): Theorem 1's bitwise recurrence -- the comparison of the
               low bits is kept where two bits agree and replaced by c2's bit
               where they differ; different sign bits decide alone;
  equality     the AND of per-bit XNORs, as a pairwise reduction (Alg. 12,
               HomEqOPT) or as a chain from a trivial 1 (Alg. 7, HomEQ);
  IntV         Alg. 4; CoV Alg. 8; IdM = HomEqOPT on identifier bits (Sec. 4.2);
  selection    Alg. 9 (HomBitwiseAND);
  aggregation  Alg. 10 (HomSum, XOR chain from a trivial 0) and its pairwise
               form of Section 6.1, part (5); and, beyond the paper, a
               reduction by k-input XORs (one bootstrap per k inputs);
  query        Alg. 3 (validate, zero out, aggregate).
A pairwise reduction combines neighbours (0, 1), (2, 3), ... and passes an
unpaired last element through, round after round, until one element remains.
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
def pairwise(xs, combine):
    """Pairwise reduction of the non-empty list xs by combine(left, right)."""
    xs = list(xs)
    while len(xs) > 1:
        xs = [combine(xs[i], xs[i + 1]) if i + 1 < len(xs) else xs[i] for i in range(0, len(xs), 2)]
    return xs[0]


def comp(B, c1, c2, l: int, strict: bool):
    """HomCompLE (strict=False) / HomCompL (strict=True): Enc(c1 <= c2) / Enc(c1 < c2).

    `low` compares bits 0..i-1: on equal low parts it is true for <= and false
    for <; a higher bit where c1 and c2 agree keeps it, one where they differ
    sets it to c2's bit (c2 has the 1 exactly when c1 is the smaller).  With
    different sign bits the negative one (sign 1) is the smaller."""
    signs_differ = B.xor(c1[l - 1], c2[l - 1])
    agree = [B.xnor(c1[i], c2[i]) for i in range(l - 1)]
    low = B.trivial(0 if strict else 1)
    for i in range(l - 1):
        low = B.mux(agree[i], low, c2[i])
    return B.mux(signs_differ, c1[l - 1], low)


def eq_opt(B, c1, c2, l: int):
    """HomEqOPT: the pairwise AND reduction of the per-bit XNORs."""
    return pairwise([B.xnor(c1[i], c2[i]) for i in range(l)], B.and_)


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
    """Pairwise XOR reduction over the records' selected bits (Section 6.1 part (5))."""
    return pairwise([list(x) for x in S], lambda x, y: [B.xor(a, b) for a, b in zip(x, y)])


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
