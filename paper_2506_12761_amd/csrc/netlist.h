// Gate netlists of the VeLoPIR circuits and their level schedule (host C++).
#pragma once
#include <stdint.h>

#include <vector>

#include "../../include/vlp.h"

namespace vlp {

// Where a ciphertext operand lives.
enum class Src : uint8_t { None = 0, Query, DbLoc, DbPay, Gate, Const };

struct Operand {
  Src src = Src::None;
  uint32_t index = 0;  // ciphertext index within the region (gate id for Src::Gate, bit for Src::Const)
  static Operand q(uint32_t i) { return {Src::Query, i}; }
  static Operand loc(uint32_t i) { return {Src::DbLoc, i}; }
  static Operand pay(uint32_t i) { return {Src::DbPay, i}; }
  static Operand gate(uint32_t g) { return {Src::Gate, g}; }
  static Operand cst(int bit) { return {Src::Const, (uint32_t)(bit ? 1 : 0)}; }
  bool is_const() const { return src == Src::Const; }
};

// Internal op of the k-input XOR (aggregation with agg_k): operands a, b and
// Netlist::xk_ops[xk_first .. xk_first + xk_count).
constexpr uint8_t OP_XORK = 7;
constexpr uint32_t AGG_K_MAX = 16;

struct Gate {
  uint8_t op;        // vlp_gate_op (AND, XOR, XNOR, MUX, ...) or OP_XORK
  Operand a, b, c;   // MUX(a = select, b = if 1, c = if 0)
  uint32_t level;    // 1 + max level of the gate operands (inputs are level 0)
  int32_t out_slot;  // >= 0: written to user output slot (v_out / R), else internal
  uint32_t xk_first = 0, xk_count = 0;  // OP_XORK: operands beyond a and b
};

// Output slots: validation bit of record i -> slot i; aggregated bit j -> slot M + j.
struct Netlist {
  std::vector<Gate> gates;
  uint32_t levels = 0;
  uint32_t M = 0, l_S = 0;
  std::vector<Operand> v_of_record;  // M entries
  std::vector<Operand> result;       // l_S entries (R), may be gates or inputs
  std::vector<Operand> xk_ops;       // extra operands of OP_XORK gates
  uint64_t blind_rotations() const;
  uint64_t key_switches() const;
};

// Builds the gate netlist of Algorithm 3 for `shape` with the circuits
// `circuit` (validation by IntV, CoV or IdM, zero-out, aggregation).  Returns
// false for shapes or circuits out of range.
// Limits every call taking a shape enforces (mode, M, l_I, l_S, d).
bool shape_valid(const vlp_shape& shape, const char** why);
// agg_k is 0 or in [2, 16].
bool circuit_valid(const vlp_circuit& circuit, const char** why);
// Appends one gate as the circuit builders do (a gate of trivial operands
// only becomes the trivial operand of its value) and returns its operand.
Operand add_gate(Netlist& nl, uint8_t op, Operand a, Operand b, Operand c = Operand());
bool build_netlist(const vlp_shape& shape, const vlp_circuit& circuit, Netlist& out, const char** why);

}  // namespace vlp
