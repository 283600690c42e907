// Gate netlists of the VeLoPIR circuits (host C++).
//
// Each builder follows one of the paper's algorithms in its order of gates:
//   comparator   Alg. 5 / 6 with the XNORs hoisted as in Alg. 11 (same graph)
//   equality     Alg. 12 (XNOR per bit, pairwise AND tree, strides 1, 2, 4, ...)
//                or Alg. 7 (AND chain from a trivial 1)
//   IntV Alg. 4, CoV Alg. 8, IdM (HomEQ on identifier bits, Section 4.2)
//   zero-out     Alg. 9;  aggregation: pairwise XOR tree (Section 6.1 (5)) or
//                Alg. 10's XOR chain from a trivial 0.
// Bits are least-significant first; bit l-1 is the sign bit.
#include "netlist.h"

#include <algorithm>

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
    // Gates whose operands are all trivial ciphertexts are themselves trivial.
    const bool ac = a.is_const(), bc = op == VLP_NOT || b.is_const(), cc = op != VLP_MUX || c.is_const();
    if (ac && bc && cc) return Operand::cst(plain(op, (int)a.index, (int)b.index, (int)c.index));
    if (op == VLP_MUX && ac) return a.index ? b : c;  // known select
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
  Operand AND(Operand a, Operand b) { return gate(VLP_AND, a, b); }
  Operand XOR(Operand a, Operand b) { return gate(VLP_XOR, a, b); }
  Operand XNOR(Operand a, Operand b) { return gate(VLP_XNOR, a, b); }
  Operand MUX(Operand s, Operand x, Operand y) { return gate(VLP_MUX, s, x, y); }

  // Enc(c1 <= c2) (strict = false) or Enc(c1 < c2) (strict = true), signed.
  Operand comp(const std::vector<Operand>& c1, const std::vector<Operand>& c2, uint32_t l, bool strict) {
    const Operand t0 = XOR(c1[l - 1], c2[l - 1]);
    std::vector<Operand> t1(l - 1);
    for (uint32_t i = 0; i + 1 < l; ++i) t1[i] = XNOR(c1[i], c2[i]);
    Operand t = Operand::cst(strict ? 0 : 1);
    for (uint32_t i = 0; i + 1 < l; ++i) t = MUX(t1[i], t, c2[i]);
    return MUX(t0, c1[l - 1], t);
  }

  Operand eq(const std::vector<Operand>& c1, const std::vector<Operand>& c2, uint32_t l, bool tree) {
    if (!tree) {
      Operand r = Operand::cst(1);
      for (uint32_t i = 0; i < l; ++i) r = AND(r, XNOR(c1[i], c2[i]));
      return r;
    }
    std::vector<Operand> t(l);
    for (uint32_t i = 0; i < l; ++i) t[i] = XNOR(c1[i], c2[i]);
    for (uint32_t k = 1; k < l; k *= 2)
      for (uint32_t i = 0; i < l; i += 2 * k)
        if (i + k < l) t[i] = AND(t[i], t[i + k]);
    return t[0];
  }
};

std::vector<Operand> bits(Operand (*mk)(uint32_t), uint32_t base, uint32_t l) {
  std::vector<Operand> v(l);
  for (uint32_t i = 0; i < l; ++i) v[i] = mk(base + i);
  return v;
}

}  // namespace

bool shape_valid(const vlp_shape& sh, const char** why) {
  const uint32_t M = sh.M, l = sh.l_I, lS = sh.l_S, d = sh.d;
  if (sh.mode != VLP_INTV && sh.mode != VLP_COV && sh.mode != VLP_IDM) { *why = "unknown mode"; return false; }
  if (M == 0 || M > (1u << 24)) { *why = "M must be in [1, 2^24]"; return false; }
  if (l < 1 || l > 64) { *why = "l_I must be in [1, 64]"; return false; }
  if (sh.mode == VLP_INTV && l < 2) { *why = "IntV needs l_I >= 2"; return false; }
  if (lS > 1024) { *why = "l_S must be <= 1024"; return false; }
  if (sh.mode != VLP_IDM && (d < 1 || d > 2)) { *why = "d must be 1 or 2"; return false; }
  return true;
}

bool build_netlist(const vlp_shape& sh, Netlist& nl, const char** why) {
  nl = Netlist();
  const uint32_t M = sh.M, l = sh.l_I, lS = sh.l_S;
  const uint32_t d = sh.mode == VLP_IDM ? 1 : sh.d;
  if (!shape_valid(sh, why)) return false;
  nl.M = M;
  nl.l_S = lS;
  Builder B{nl};
  const bool opt = sh.optimized != 0;

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
  if (opt) {
    for (uint32_t k = 1; k < M; k *= 2)
      for (uint32_t i = 0; i < M; i += 2 * k)
        if (i + k < M)
          for (uint32_t j = 0; j < lS; ++j) S[i][j] = B.XOR(S[i][j], S[i + k][j]);
    nl.result = S[0];
  } else {
    std::vector<Operand> R(lS, Operand::cst(0));
    for (uint32_t i = 0; i < M; ++i)
      for (uint32_t j = 0; j < lS; ++j) R[j] = B.XOR(R[j], S[i][j]);
    nl.result = R;
  }
  return true;
}

}  // namespace vlp
