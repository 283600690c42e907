// Builds the gate netlists of many shapes under AddressSanitizer and
// UndefinedBehaviorSanitizer and checks their structure: operands refer to
// inputs in range or to earlier gates, levels are 1 + the deepest operand,
// results are distinct gates, invalid shapes are rejected.
#include <cstdio>
#include <set>
#include <vector>

#include "netlist.h"

using namespace vlp;

static bool check(const vlp_shape& sh, const vlp_circuit& circ) {
  Netlist nl;
  const char* why = "";
  if (!build_netlist(sh, circ, nl, &why)) {
    std::printf("rejected a valid shape: %s\n", why);
    return false;
  }
  const uint32_t d = sh.mode == VLP_IDM ? 1 : sh.d;
  const size_t nq = (size_t)d * sh.l_I;
  const size_t nloc = sh.mode == VLP_INTV ? (size_t)sh.M * d * 2 * sh.l_I : (size_t)sh.M * d * sh.l_I;
  const size_t npay = (size_t)sh.M * sh.l_S;
  auto level = [&](const Operand& o, size_t g) -> long {
    switch (o.src) {
      case Src::Query: return o.index < nq ? 0 : -1;
      case Src::DbLoc: return o.index < nloc ? 0 : -1;
      case Src::DbPay: return o.index < npay ? 0 : -1;
      case Src::Const: return o.index <= 1 ? 0 : -1;
      case Src::Gate: return o.index < g ? (long)nl.gates[o.index].level : -1;
      default: return -2;  // unused operand
    }
  };
  for (size_t g = 0; g < nl.gates.size(); ++g) {
    const Gate& G = nl.gates[g];
    std::vector<Operand> ops{G.a};
    if (G.op != VLP_NOT) ops.push_back(G.b);
    if (G.op == VLP_MUX) ops.push_back(G.c);
    if (G.op == OP_XORK)
      for (uint32_t t = 0; t < G.xk_count; ++t) ops.push_back(nl.xk_ops.at(G.xk_first + t));
    long mx = 0;
    for (const Operand& o : ops) {
      const long l = level(o, g);
      if (l < 0) {
        std::printf("gate %zu has a bad operand\n", g);
        return false;
      }
      mx = l > mx ? l : mx;
    }
    if ((long)G.level != mx + 1) {
      std::printf("gate %zu level %u, operands at %ld\n", g, G.level, mx);
      return false;
    }
  }
  std::set<uint32_t> seen;
  for (const Operand& r : nl.result)
    if (r.src != Src::Gate || !seen.insert(r.index).second) {
      std::printf("result bits are not distinct gates\n");
      return false;
    }
  return nl.result.size() == sh.l_S && nl.v_of_record.size() == sh.M;
}

int main() {
  int n = 0;
  for (int mode = 0; mode < 3; ++mode)
    for (uint32_t M : {1u, 2u, 5u, 17u, 33u})
      for (uint32_t l : {2u, 3u, 8u, 16u, 64u})
        for (uint32_t lS : {0u, 1u, 4u})
          for (uint32_t opt = 0; opt < 2; ++opt)
            for (uint32_t k : {0u, 2u, 3u, 16u}) {
              const vlp_shape sh{(vlp_mode)mode, M, l, lS, 2};
              if (!check(sh, vlp_circuit{opt, k})) return 1;
              ++n;
            }
  const vlp_shape big{VLP_IDM, 4, 8, 1024, 1};
  if (!check(big, vlp_circuit{1, 16})) return 1;
  const char* why = "";
  Netlist nl;
  for (const vlp_shape& bad : {vlp_shape{VLP_INTV, 3, 1, 0, 1}, vlp_shape{VLP_IDM, 0, 8, 0, 1},
                               vlp_shape{VLP_COV, 3, 65, 0, 1}, vlp_shape{VLP_COV, 3, 8, 0, 3},
                               vlp_shape{VLP_IDM, 3, 8, 1025, 1}, vlp_shape{(vlp_mode)7, 3, 8, 2, 1}})
    if (build_netlist(bad, vlp_circuit{1, 0}, nl, &why)) {
      std::printf("accepted an invalid shape\n");
      return 1;
    }
  for (const vlp_circuit& bad : {vlp_circuit{1, 1}, vlp_circuit{1, 17}, vlp_circuit{0, 1u << 31}})
    if (build_netlist(vlp_shape{VLP_IDM, 3, 8, 2, 1}, bad, nl, &why)) {
      std::printf("accepted an invalid circuit\n");
      return 1;
    }
  // A MUX with a trivial select is bootstrapped like any other gate (its two
  // rotations run on the other operands); a gate of trivial operands only is
  // the trivial operand of its value; a trivial operand beside a real one
  // still leaves a gate.
  {
    Netlist t;
    const Operand m = add_gate(t, VLP_MUX, Operand::cst(1), Operand::q(0), Operand::q(1));
    if (m.src != Src::Gate || t.gates.size() != 1 || t.gates[0].level != 1 || t.blind_rotations() != 2 ||
        t.key_switches() != 1) {
      std::printf("a MUX with a trivial select was not kept as a bootstrapped gate\n");
      return 1;
    }
    const Operand m2 = add_gate(t, VLP_MUX, Operand::cst(0), Operand::cst(1), m);
    if (m2.src != Src::Gate || t.gates.back().level != 2) {
      std::printf("a MUX of a trivial select and a trivial operand was not kept\n");
      return 1;
    }
    const Operand k = add_gate(t, VLP_MUX, Operand::cst(1), Operand::cst(0), Operand::cst(1));
    const Operand x = add_gate(t, VLP_XNOR, Operand::cst(1), Operand::cst(1));
    if (!k.is_const() || k.index != 0 || !x.is_const() || x.index != 1 || t.gates.size() != 2) {
      std::printf("gates of trivial operands were not folded to their value\n");
      return 1;
    }
    const Operand a = add_gate(t, VLP_AND, Operand::cst(1), Operand::loc(3));
    if (a.src != Src::Gate || t.gates.size() != 3) {
      std::printf("a gate with one real operand was folded\n");
      return 1;
    }
  }
  std::printf("netlist OK (%d shapes)\n", n + 1);
  return 0;
}
