"""Seeded encrypted workloads and their oracle results.

TEST INFRASTRUCTURE ONLY (part of the oracle): plaintext values come from
the seeded generator (synth), ciphertexts from the oracle's encryption, and
expected outputs from the oracle's gates run over the circuit graphs.

Array layouts match the library's evaluate call:
  query  IntV/CoV [d][l][631], IdM [l][631]
  db_loc IntV [M][d][2][l][631] (left, right), CoV [M][d][l][631], IdM [M][l][631]
  db_pay [M][l_S][631]
"""
from __future__ import annotations

import numpy as np

import synth

from . import circuits as C
from . import oracle as O


def plain_workload(mode: str, M: int, l: int, lS: int, d: int, seed: int, hit: bool = True) -> dict:
    """Plaintext query and database, with the predicate per record and R."""
    g = synth.stream(seed, "plain:%s" % mode)
    P = {"mode": mode, "M": M, "l": l, "lS": lS, "d": d}
    if mode == "intv":
        a = synth.signed_ints(g, (M, d), l)
        b = synth.signed_ints(g, (M, d), l)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        q = synth.signed_ints(g, (d,), l)
        if hit:  # put the query inside one record's box
            r = int(g.integers(0, M))
            for k in range(d):
                if lo[r, k] == hi[r, k]:
                    hi[r, k] = min(hi[r, k] + 1, 2 ** (l - 1) - 1)
                    lo[r, k] = hi[r, k] - 1
                q[k] = int(g.integers(lo[r, k], hi[r, k]))
        P["loc"] = np.stack([lo, hi], axis=2)  # [M][d][2]
        v = np.all((lo <= q[None, :]) & (q[None, :] < hi), axis=1)
    elif mode == "cov":
        loc = synth.signed_ints(g, (M, d), l)
        q = synth.signed_ints(g, (d,), l)
        if hit:
            q = loc[int(g.integers(0, M))].copy()
        P["loc"] = loc
        v = np.all(loc == q[None, :], axis=1)
    elif mode == "idm":
        loc = synth.unsigned_ints(g, (M,), l).astype(np.int64)
        q = synth.unsigned_ints(g, (), l).astype(np.int64)
        if hit:
            q = loc[int(g.integers(0, M))]
        P["loc"] = loc
        v = loc == q
    else:
        raise ValueError(mode)
    P["q"] = q
    P["v"] = v.astype(np.uint8)
    P["pay"] = synth.bits(g, (M, lS)).astype(np.uint8)
    R = np.zeros(lS, np.uint8)
    for i in range(M):
        if v[i]:
            R ^= P["pay"][i]
    P["R"] = R
    return P


def encrypt_workload(keys: O.Keys, P: dict, seed: int) -> dict:
    mode, M, l, lS, d = P["mode"], P["M"], P["l"], P["lS"], P["d"]
    if mode == "idm":
        qb = synth.to_bits(np.asarray(P["q"]), l)                 # [l]
        lb = synth.to_bits(P["loc"], l)                           # [M][l]
    elif mode == "intv":
        qb = synth.to_bits(P["q"], l)                             # [d][l]
        lb = synth.to_bits(P["loc"], l)                           # [M][d][2][l]
    else:
        qb = synth.to_bits(P["q"], l)                             # [d][l]
        lb = synth.to_bits(P["loc"], l)                           # [M][d][l]
    out = {}
    for name, b in (("query", qb), ("db_loc", lb), ("db_pay", P["pay"])):
        if b.size == 0:
            out[name] = np.zeros(b.shape + (O.n + 1,), np.uint32)
            continue
        masks, noise = synth.lwe_randomness(seed, "enc:" + name, b.size)
        out[name] = O.encrypt_bits_np(keys, b, masks, noise)
    return out


def record_slice(P: dict, enc: dict, idx) -> tuple[dict, dict]:
    """The sub-workload made of records `idx` (same query), for sampled checks."""
    idx = np.asarray(idx)
    Q = dict(P)
    Q["M"] = len(idx)
    Q["loc"] = P["loc"][idx]
    Q["pay"] = P["pay"][idx]
    Q["v"] = P["v"][idx]
    e = {"query": enc["query"], "db_loc": enc["db_loc"][idx], "db_pay": enc["db_pay"][idx]}
    return Q, e


def graph_for(mode: str, M: int, l: int, lS: int, d: int, optimized: bool = True, agg_k: int = 0):
    """Circuit graph of the whole query with input keys naming array positions."""
    G = C.GraphBuilder()
    if mode == "idm":
        q = [G.input(("query", (i,))) for i in range(l)]
        db = [[G.input(("db_loc", (r, i))) for i in range(l)] for r in range(M)]
    elif mode == "intv":
        q = [[G.input(("query", (k, i))) for i in range(l)] for k in range(d)]
        db = [[([G.input(("db_loc", (r, k, 0, i))) for i in range(l)],
                [G.input(("db_loc", (r, k, 1, i))) for i in range(l)]) for k in range(d)] for r in range(M)]
    else:
        q = [[G.input(("query", (k, i))) for i in range(l)] for k in range(d)]
        db = [[[G.input(("db_loc", (r, k, i))) for i in range(l)] for k in range(d)] for r in range(M)]
    pay = [[G.input(("db_pay", (r, j))) for j in range(lS)] for r in range(M)] if lS else None
    vs, R = C.query(G, mode, q, db, pay, l, optimized=optimized, agg_k=agg_k)
    return G, vs, R


def oracle_outputs(keys: O.Keys, P: dict, enc: dict, optimized: bool = True, threads=None, agg_k: int = 0):
    """(v [M][631], R [lS][631]) computed by the oracle."""
    G, vs, R = graph_for(P["mode"], P["M"], P["l"], P["lS"], P["d"], optimized, agg_k)
    inputs = {}
    for nd in G.nodes:
        if nd[0] == "in":
            name, idx = nd[1]
            inputs[nd[1]] = enc[name][idx]
    vals = G.evaluate(keys, inputs, threads)
    v = np.stack([vals[x] for x in vs])
    Rv = np.stack([vals[x] for x in R]) if R else np.zeros((0, O.n + 1), np.uint32)
    return v, Rv
