// Gate netlists of the VeLoPIR circuits (host C++).
//
// The circuits, from their definitions:
//   comparator   Theorems 1-2 (Alg. 5 / 6, same graph as Alg. 11): the
//                comparison of the low bits, carried up bit by bit, kept
//                where the bits agree and replaced by c2's bit where they
//                differ; the sign bits decide when they differ
//   equality     the AND of per-bit XNORs, as a balanced pairwise reduction
//                (Alg. 12) or as a chain from a trivial 1 (Alg. 7)
//   IntV Alg. 4, CoV Alg. 8, IdM (equality of identifier bits, Section 4.2)
//   zero-out     Alg. 9;  aggregation: pairwise XOR reduction over records
//                (Section 6.1 (5)) or Alg. 10's XOR chain from a trivial 0, or
//                (agg_k, beyond the paper) a reduction by k-input XORs.
// A pairwise reduction combines neighbours (0,1), (2,3), ... and passes an
// unpaired last element through, round after round, until one remains.
// Bits are least-significant first; bit l-1 is the sign bit.
#include "netlist.h"

#include <algorithm>
#include <cstring>

namespace vlp {

uint64_t Netlist::blind_rotations() const {
  uint64_t n = 0;
  for (const Gate& g : gates) n += g.op == VLP_MUX ? 2 : (g.op == VLP_NOT ? 0 : 1);
  return n;
}

uint64_t Netlist::key_switches() const {
  uint64_t n = 0;
  for (const Gate& g : gates) n += g.op == VLP_NOT ? 0 : 1;
  return n;
}

namespace {

int plain(uint8_t op, int a, int b, int c) {
  switch (op) {
    case VLP_AND: return a & b;
    case VLP_OR: return a | b;
    case VLP_NAND: return 1 - (a & b);
    case VLP_XOR: return a ^ b;
    case VLP_XNOR: return 1 - (a ^ b);
    case VLP_NOT: return 1 - a;
    default: return a ? b : c;
  }
}

struct Builder {
  Netlist& nl;

  uint32_t level_of(const Operand& o) const { return o.src == Src::Gate ? nl.gates[o.index].level : 0; }

  Operand gate(uint8_t op, Operand a, Operand b, Operand c = Operand()) {
    // A gate whose operands are all trivial ciphertexts is itself the trivial
    // ciphertext of its value: bootstrapping a trivial input gives exactly
    // (0, +-1/8), and key switching a trivial input leaves it unchanged.  A
    // gate with some trivial operands is bootstrapped like any other (a MUX
    // with a trivial select too: its two rotations still run on the other
    // operands, so its words are not those of the selected operand).
    const bool ac = a.is_const(), bc = op == VLP_NOT || b.is_const(), cc = op != VLP_MUX || c.is_const();
    if (ac && bc && cc) return Operand::cst(plain(op, (int)a.index, (int)b.index, (int)c.index));
    Gate g;
    g.op = op;
    g.a = a;
    g.b = b;
    g.c = c;
    g.level = 1 + std::max(level_of(a), std::max(level_of(b), level_of(c)));
    g.out_slot = -1;
    nl.gates.push_back(g);
    nl.levels = std::max(nl.levels, g.level);
    return Operand::gate((uint32_t)nl.gates.size() - 1);
  }
  // XOR of ops (size >= 1) with one bootstrap: (0, (k-1)/4) + 2 * sum.
  Operand XORK(const std::vector<Operand>& ops) {
    if (ops.size() == 1) return ops[0];
    bool all_const = true;
    int parity = 0;
    uint32_t lvl = 0;
    for (const Operand& o : ops) {
      all_const = all_const && o.is_const();
      parity ^= o.is_const() ? (int)o.index : 0;
      lvl = std::max(lvl, level_of(o));
    }
    if (all_const) return Operand::cst(parity);
    Gate g;
    g.op = OP_XORK;
    g.a = ops[0];
    g.b = ops[1];
    g.c = Operand();
    g.level = 1 + lvl;
    g.out_slot = -1;
    g.xk_first = (uint32_t)nl.xk_ops.size();
    g.xk_count = (uint32_t)ops.size() - 2;
    for (size_t t = 2; t < ops.size(); ++t) nl.xk_ops.push_back(ops[t]);
    nl.gates.push_back(g);
    nl.levels = std::max(nl.levels, g.level);
    return Operand::gate((uint32_t)nl.gates.size() - 1);
  }
  Operand AND(Operand a, Operand b) { return gate(VLP_AND, a, b); }
  Operand XOR(Operand a, Operand b) { return gate(VLP_XOR, a, b); }
  Operand XNOR(Operand a, Operand b) { return gate(VLP_XNOR, a, b); }
  Operand MUX(Operand s, Operand x, Operand y) { return gate(VLP_MUX, s, x, y); }

  // Enc(c1 <= c2) (strict = false) or Enc(c1 < c2) (strict = true), signed.
  // `low` is the comparison of the bits below i: where c1[i] == c2[i] it
  // carries on, where they differ c1 < c2 on bits 0..i exactly when c2[i] is
  // 1; on equal low parts it is true for <= and false for <.  Different sign
  // bits decide alone: then c1 is the smaller one exactly when it is negative.
  Operand comp(const std::vector<Operand>& c1, const std::vector<Operand>& c2, uint32_t l, bool strict) {
    const Operand signs_differ = XOR(c1[l - 1], c2[l - 1]);
    std::vector<Operand> agree(l - 1);
    for (uint32_t i = 0; i + 1 < l; ++i) agree[i] = XNOR(c1[i], c2[i]);
    Operand low = Operand::cst(strict ? 0 : 1);
    for (uint32_t i = 0; i + 1 < l; ++i) low = MUX(agree[i], low, c2[i]);
    return MUX(signs_differ, c1[l - 1], low);
  }

  // Enc(c1 == c2): the AND of the per-bit XNORs.
  Operand eq(const std::vector<Operand>& c1, const std::vector<Operand>& c2, uint32_t l, bool tree) {
    std::vector<Operand> same(l);
    for (uint32_t i = 0; i < l; ++i) same[i] = XNOR(c1[i], c2[i]);
    if (!tree) {
      Operand r = Operand::cst(1);
      for (const Operand& x : same) r = AND(r, x);
      return r;
    }
    return pairwise(std::move(same), [this](Operand x, Operand y) { return AND(x, y); });
  }

  // Pairwise reduction of xs (non-empty) by `combine`.
  template <class T, class F>
  static T pairwise(std::vector<T> xs, F combine) {
    while (xs.size() > 1) {
      std::vector<T> next;
      for (size_t i = 0; i < xs.size(); i += 2) next.push_back(i + 1 < xs.size() ? combine(xs[i], xs[i + 1]) : xs[i]);
      xs.swap(next);
    }
    return xs[0];
  }
};

std::vector<Operand> bits(Operand (*mk)(uint32_t), uint32_t base, uint32_t l) {
  std::vector<Operand> v(l);
  for (uint32_t i = 0; i < l; ++i) v[i] = mk(base + i);
  return v;
}

}  // namespace

Operand add_gate(Netlist& nl, uint8_t op, Operand a, Operand b, Operand c) {
  Builder B{nl};
  return B.gate(op, a, b, c);
}

static_assert(sizeof(vlp_mode) == sizeof(int), "the mode field is read as an int");

bool shape_valid(const vlp_shape& sh, const char** why) {
  const uint32_t M = sh.M, l = sh.l_I, lS = sh.l_S, d = sh.d;
  // A C caller may store any integer in the mode field: read its bytes as an
  // int (loading an enum outside its enumerators is undefined in C++).
  int mode;
  std::memcpy(&mode, &sh.mode, sizeof mode);
  if (mode != VLP_INTV && mode != VLP_COV && mode != VLP_IDM) { *why = "unknown mode"; return false; }
  if (M == 0 || M > (1u << 24)) { *why = "M must be in [1, 2^24]"; return false; }
  if (l < 1 || l > 64) { *why = "l_I must be in [1, 64]"; return false; }
  if (sh.mode == VLP_INTV && l < 2) { *why = "IntV needs l_I >= 2"; return false; }
  if (lS > 1024) { *why = "l_S must be <= 1024"; return false; }
  if (sh.mode != VLP_IDM && (d < 1 || d > 2)) { *why = "d must be 1 or 2"; return false; }
  return true;
}

bool circuit_valid(const vlp_circuit& c, const char** why) {
  if (c.agg_k == 1 || c.agg_k > AGG_K_MAX) { *why = "agg_k must be 0 or in [2, 16]"; return false; }
  return true;
}

bool build_netlist(const vlp_shape& sh, const vlp_circuit& circ, Netlist& nl, const char** why) {
  nl = Netlist();
  if (!shape_valid(sh, why) || !circuit_valid(circ, why)) return false;
  const uint32_t M = sh.M, l = sh.l_I, lS = sh.l_S;
  const uint32_t d = sh.mode == VLP_IDM ? 1 : sh.d;
  nl.M = M;
  nl.l_S = lS;
  Builder B{nl};
  const bool opt = circ.optimized != 0;

  // Validation (Alg. 4 / Alg. 8 / IdM), record by record.
  nl.v_of_record.resize(M);
  for (uint32_t i = 0; i < M; ++i) {
    Operand v;
    if (sh.mode == VLP_INTV) {
      std::vector<Operand> lefts(d), rights(d);
      for (uint32_t k = 0; k < d; ++k) {
        const auto q = bits(Operand::q, k * l, l);
        const auto lo = bits(Operand::loc, ((i * d + k) * 2 + 0) * l, l);
        const auto hi = bits(Operand::loc, ((i * d + k) * 2 + 1) * l, l);
        lefts[k] = B.comp(lo, q, l, false);   // left <= x
        rights[k] = B.comp(q, hi, l, true);   // x < right
      }
      std::vector<Operand> per(d);
      for (uint32_t k = 0; k < d; ++k) per[k] = B.AND(lefts[k], rights[k]);
      v = per[0];
      for (uint32_t k = 1; k < d; ++k) v = B.AND(v, per[k]);
    } else if (sh.mode == VLP_COV) {
      std::vector<Operand> per(d);
      for (uint32_t k = 0; k < d; ++k)
        per[k] = B.eq(bits(Operand::q, k * l, l), bits(Operand::loc, (i * d + k) * l, l), l, opt);
      v = per[0];
      for (uint32_t k = 1; k < d; ++k) v = B.AND(v, per[k]);
    } else {
      v = B.eq(bits(Operand::q, 0, l), bits(Operand::loc, i * l, l), l, opt);
    }
    nl.v_of_record[i] = v;
  }
  if (lS == 0) return true;

  // Zero-out (Alg. 9) and aggregation.
  std::vector<std::vector<Operand>> S(M, std::vector<Operand>(lS));
  for (uint32_t i = 0; i < M; ++i)
    for (uint32_t j = 0; j < lS; ++j) S[i][j] = B.AND(nl.v_of_record[i], Operand::pay(i * lS + j));
  if (circ.agg_k >= 2) {
    // Consecutive groups of k (a group of one passes through), repeated on the group results.
    const uint32_t K = circ.agg_k;
    std::vector<std::vector<Operand>> cur = S;
    while (cur.size() > 1) {
      std::vector<std::vector<Operand>> nxt;
      for (size_t g0 = 0; g0 < cur.size(); g0 += K) {
        const size_t gn = std::min<size_t>(K, cur.size() - g0);
        if (gn == 1) {
          nxt.push_back(cur[g0]);
          continue;
        }
        std::vector<Operand> row(lS);
        for (uint32_t j = 0; j < lS; ++j) {
          std::vector<Operand> ops(gn);
          for (size_t t = 0; t < gn; ++t) ops[t] = cur[g0 + t][j];
          row[j] = B.XORK(ops);
        }
        nxt.push_back(row);
      }
      cur.swap(nxt);
    }
    nl.result = cur[0];
  } else if (opt) {
    nl.result = Builder::pairwise(std::move(S), [&B, lS](const std::vector<Operand>& x, const std::vector<Operand>& y) {
      std::vector<Operand> r(lS);
      for (uint32_t j = 0; j < lS; ++j) r[j] = B.XOR(x[j], y[j]);
      return r;
    });
  } else {
    std::vector<Operand> R(lS, Operand::cst(0));
    for (uint32_t i = 0; i < M; ++i)
      for (uint32_t j = 0; j < lS; ++j) R[j] = B.XOR(R[j], S[i][j]);
    nl.result = R;
  }
  return true;
}

}  // namespace vlp
