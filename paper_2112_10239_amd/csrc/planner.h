// Host-side planning: gate lists -> passes -> stages -> device ops, light
// cones, and per-row gate coefficients.  Integer work plus fp64 trigonometry;
// no device calls.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "qsim_types.h"

namespace qsim {

enum GateKind { G_RX = 0, G_RY = 1, G_RZ = 2, G_CZ = 3, G_CNOT = 4, G_U1 = 5 };

// A gate of the user's circuit (validated copy).
struct Gate {
  int kind, q0, q1, param;
  double angle;
  double mat[8];  // U1 only
};

struct Term {
  double c = 0;
  std::vector<std::pair<int, char>> ops;  // (qubit, 'X'|'Y'|'Z'); empty = identity
};

struct CircuitDesc {
  int n = 0, n_params = 0;
  std::vector<Gate> gates;
};

// Planner-level operation ("pgate"): a fused gate, a gradient probe, or a
// measurement / H-apply term.
enum PGKind { PG_U, PG_RY, PG_X, PG_PHASE, PG_CZ, PG_GRAD, PG_MEAS_Z, PG_MEAS_F, PG_H_Z, PG_H_F, PG_TAB, PG_INITF };

// PG_INITF coefficient slots: init_slots(n) consecutive slots hold, per physical
// qubit q, (U_q|0>)_0 and (U_q|0>)_1 as 4 scalars (re, im, re, im), U_q being
// the slot in srcs[q] (-1: identity); gen is the chunk a slot holds.
inline int init_slots(int n) { return (4 * n + 7) / 8; }

// PG_TAB coefficient slots: kTabSlots consecutive slots hold the block of one
// OP_UTAB op: uncontrolled rotations on the register bits of a stage (identity
// on bits without one), each written as U_j = X^{f_j} P_j T_j E_j with
// T_j = [[1, -k_j], [k_j, 1]], |k_j| <= 1, diagonal P_j and E_j = diag(1, e_j),
// and X^{f_j} a swap of the bit's two values (needed when |u01| > |u00|).  The
// swaps of all bits commute past everything else and leave the registers
// permuted: register i holds the amplitude of register index i ^ F, which the
// stage's exit (LDS write or store) absorbs into its addresses.  A PG_TAB
// slot's srcs list, per register bit, the coefficient slot of the rotation on
// it (-1: none); its gen field is the chunk it holds.
// Block layout in scalars (T = float or double):
//   [0, 32)  post table: 16 complex products of the P_j over the register bits
//   [32, 64) pre table: 16 complex products of the E_j
//   [64, 68) k per register bit
//   [68]     F (swap mask) as raw 32-bit bits
//   [69]     nonzero raw bits when the pre table is not all ones
constexpr int kTabSlots = 9;

struct PGate {
  int kind = PG_U;
  int q = -1;    // target / diagonal qubit / first CZ qubit
  int q2 = -1;   // control / second CZ qubit
  int slot = -1; // coefficient slot, or gradient slot for PG_GRAD
  int gen = 0;   // PG_GRAD generator: 'X', 'Y' or 'Z'
  bool inverse = false;   // coefficient = adjoint of the product
  bool real_pre = false;  // product is RY's followed by RZ's: U = diag(..) K with real K
  std::vector<int> srcs;  // source gates, in application order
  uint64_t fmask = 0, zmask = 0;  // terms: flip (X|Y) and sign (Y|Z) masks, physical
  int ph = 0;                     // terms: i^ph
  double c = 0;                   // terms: coefficient
};

struct Plan {
  int n = 0, m = 0, r = 0;
  std::vector<PassDesc> passes;
  std::vector<StageDesc> stages;
  std::vector<DevOp> ops;
  std::vector<PGate> slots;       // coefficient slot specs (index = slot)
  int n_meas = 0;                 // measurement partial columns
  int n_gslots = 0;               // gradient slots
  std::vector<int> gslot_param;   // gradient slot -> parameter index
  double const_term = 0;          // identity terms, added on the host
  std::vector<int32_t> order;     // (pass, stage, op, source gate) quadruples
  int meas_passes = 0;
  std::vector<int> qmap;          // qubit -> index bit after the last gate pass (empty: identity)
  bool want_trace = false;        // host checks: record every stage's items, then its permutation,
  std::vector<PGate> trace;       // in index-bit coordinates (kind -1: a stage ends)
};

enum PlanMode { PM_FWD = 0, PM_ADJ = 1 };

struct PlanOptions {
  int m_max = 14;       // tile qubits
  int r = 4;            // register bits per stage
  int c_low = 6;        // always-local low bits for coalesced HBM access
  bool init = true;     // first pass generates |0...0>
  bool store_final = true;  // keep the final state in HBM
  bool fuse = true;     // fuse runs of single-qubit gates on one qubit
  int max_grad = kMaxGradPerPass;  // gradient probes per pass
  bool absorb = true;   // allow CNOT runs as stage exit permutations
  int io_lo = -1;       // lowest local bit a register bit may use in a stage that loads or
                        // stores (HBM coalescing); -1: c_low
  bool entry_perm = true;  // with factored: a permute-only first stage folded into the loads
  bool exit_perm = true;   // with factored: the last stage's CNOT run folded into the stores
  bool init_factors = true;  // with factored and init: leading single-qubit gates folded into the start state
  bool batch_probes = false;  // adjoint plans: diagonals as tables and probes in groups (OP_PTAB,
                              // OP_GZS, OP_GXYS)
  bool factored = false;  // runs of uncontrolled rotations on register bits as one OP_UTAB
                          // (single-state float kernels with r <= 4; needs plan.slots)
  bool relabel = false;   // without store_final: the qubits held in the low index bits change
                          // between passes (plan.qmap: the final map)
  bool relabel_kept = false;  // also relabel plans that keep the final state (their last pass
                              // puts the qubits back in order)
  int c_low_relabel = 5;  // c_low of plans that relabel
  bool early_terms = true;  // terms with X/Y factors measured in the gate passes once ready
};

// Validation; returns "" when fine.
std::string validate_circuit(const CircuitDesc& c);
std::string validate_terms(const std::vector<Term>& t, int n);

// Preprocess the circuit into forward pgates (fused) with coefficient slots.
void forward_pgates(const CircuitDesc& c, bool fuse, std::vector<PGate>& out, std::vector<PGate>& slots);
// Reverse sweep for the adjoint method: for every gate from last to first a
// gradient probe (parameterised rotations) followed by the inverse gate.
void adjoint_pgates(const CircuitDesc& c, std::vector<PGate>& out, std::vector<PGate>& slots,
                    std::vector<int>& gslot_param);
// Measurement (PG_MEAS_*) or H-apply (PG_H_*) pgates for the non-identity terms.
// 'relabel' (optional) maps circuit qubits to the plan's qubits.
void term_pgates(const std::vector<Term>& terms, bool happly, std::vector<PGate>& out, double& const_term,
                 const std::vector<int>* relabel = nullptr);

// Forward plan with measurement of 'meas' at the end (meas may be empty).
int plan_forward(int n, const std::vector<PGate>& gates, const std::vector<PGate>& meas, const PlanOptions& o,
                 Plan& plan, std::string& err);
// Dual-state plans: lambda = H psi, then the adjoint sweep with gradient probes.
int plan_happly(int n, const std::vector<PGate>& hterms, const PlanOptions& o, Plan& plan, std::string& err);
int plan_adjoint(int n, const std::vector<PGate>& gates, const PlanOptions& o, Plan& plan, std::string& err);

// Add diagonal measurement terms (PG_MEAS_Z) to the last stage of a plan that
// ends with all gates applied; marks the last pass PF_MEASURE.  Lets a plan of
// the gates alone be shared by requests that differ only in a diagonal H.
void append_diag_measure(Plan& plan, const std::vector<PGate>& meas);

// Canonical light cone of one term: ascending qubits and in-cone gate indices.
// Gates with skip[g] != 0 (optional) are treated as absent.
void light_cone(const CircuitDesc& c, const std::vector<int>& support, std::vector<int>& set,
                std::vector<int>& gates, const std::vector<char>* skip = nullptr);

// Gates that can be dropped for any diagonal (Z-string) observable: diagonal
// gates (RZ, CZ) all of whose later gates on the same qubits are droppable too.
// They commute with the observable and with each other, so they cancel in <P>.
std::vector<char> trailing_diagonal(const CircuitDesc& c);

// Per-row coefficient table for the slots, T = float or double; 8 values per slot.
template <class T>
void build_coefficients(const CircuitDesc& c, const std::vector<PGate>& slots, const double* params, int batch,
                        int64_t row_stride, T* out);

// Flat slot and gate tables for building coefficient rows on the device.
void coef_slot_table(const std::vector<PGate>& slots, std::vector<CoefSlot>& out, std::vector<int32_t>& srcs);
void coef_gate_table(const CircuitDesc& c, std::vector<CoefGate>& out);

// Cache key of a plan: the circuit's structure (gate kinds, qubits, parameter
// indices), the terms and the plan variant, serialised; keys compare by value.
std::string structure_key(const CircuitDesc& c, const std::vector<Term>& terms, int extra);

}  // namespace qsim
