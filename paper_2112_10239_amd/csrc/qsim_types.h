// Device-visible plan descriptors shared by the host planner and the HIP kernels.
//
// A state of n qubits is processed in *passes*.  A pass splits the 2^n
// amplitudes into tiles of 2^m amplitudes that share the values of the n-m
// "non-local" index bits; every tile is read from HBM once, transformed on
// chip and written back once.  Inside a tile, a local index l in [0, 2^m)
// has bit k at physical position lpos[k].
//
// A pass is a sequence of *stages*.  In a stage every thread holds 2^r
// amplitudes in registers that differ in the r "register bits" rb[] (local
// indices); the thread's own local index bits are tb[] (the other m-r local
// indices, ascending).  Ops of a stage act on register bits (non-diagonal
// gates, flips) or on any bit (diagonal gates, measurement signs).  Between
// stages the tile is exchanged through LDS; the first stage reads from HBM
// (or generates |0...0>) and the last stage writes to HBM.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace qsim {

enum OpType : uint8_t {
  OP_NONE = 0,
  OP_U = 1,       // general 2x2 on register bit j (coef: u00,u01,u10,u11 complex), optional control
  OP_RY = 2,      // real rotation [[c,-s],[s,c]] on register bit j (coef: c, s), optional control
  OP_X = 3,       // Pauli X on register bit j, optional control (CNOT)
  OP_PHASE = 4,   // diag(d0, d1) on bit (ck,cb) (coef: d0, d1 complex)
  OP_CZ = 5,      // multiply by -1 when bits (ck,cb) and (ck2,cb2) are both 1
  OP_MEAS_Z = 6,  // acc += c * sum_i (-1)^{z(i)} |a_i|^2
  OP_MEAS_F = 7,  // acc += c * Re( i^ph * sum_i (-1)^{z(i)} conj(a_{i^f}) a_i )
  OP_GRAD_X = 8,  // g[slot] += Im sum_i conj(b_i) a_{i^J}
  OP_GRAD_Y = 9,  // g[slot] += Im sum_i conj(b_i) (-i)(-1)^{bit_J(i)} a_{i^J}
  OP_GRAD_Z = 10, // g[slot] += Im sum_i conj(b_i) (-1)^{bit(i)} a_i   (bit = (ck,cb))
  OP_H_Z = 11,    // b_i += c (-1)^{z(i)} a_i
  OP_H_F = 12,    // b_i += c i^ph (-1)^{z(i^f)} a_{i^f}
  OP_MEAS_ZS = 13,// group of diagonal terms: the next 'slot' ops are term records (rz, tz, pz, c);
                  // acc += sum_t c_t (-1)^{thread/tile parity} W[rz_t], W = Walsh transform of |a_i|^2
  OP_UALL = 14,   // one uncontrolled op per register bit: the next r ops are OP_U (or, with j = 1 in the
  OP_RYALL = 15,  // header, OP_RY) records for register bits 0..r-1 in order (gates on distinct qubits)
  OP_UTAB = 16,   // uncontrolled rotations on every register bit, factored (see the PG_TAB block layout
                  // in planner.h); slot = first of the block's coefficient slots; no records follow;
                  // always the last op of its stage (its register swaps go to the stage's exit)
  OP_DTAB = 17,   // the pre table of the OP_UTAB that follows (same slot)
  OP_PTAB = 18,   // diagonal phases on both states: a_i *= d_i f (and b_i in dual kernels) with d the post
                  // table of a PG_TAB block whose members are diagonal gates on register bits (slot = the
                  // block's first slot; -1: none) and f the per-thread product of the phases of the next
                  // 'j' ops, records of diagonal gates on thread or tile bits (ck, cb; slot: d0, d1)
  OP_GZS = 19,    // Z-generator probes on the same states: the next 'slot' ops (at most 4) are records
                  // (ck, cb: the qubit's bit; slot: gradient slot); g += Im sum_i conj(b_i) (-1)^{bit(i)} a_i
  OP_GXYS = 20,   // X/Y-generator probes on register bits: the next 'slot' ops (at most 4) are records
                  // (j: register bit; ph: 0 for X, 1 for Y; slot: gradient slot), as OP_GRAD_X / OP_GRAD_Y
  OP_CZS = 21,    // a run of CZs as one sign pattern over the register index: rz holds the pairs on two
                  // register bits (bit i set: register index i changes sign); the next j ops are OP_CZ
                  // records of the other pairs (one register bit: a linear term; none: a constant)
};

// Bit reference kinds for controls, diagonal bits and z-masks.
enum BitKind : uint8_t { BK_NONE = 0, BK_REG = 1, BK_THREAD = 2, BK_TILE = 3 };

struct DevOp {
  uint8_t type;
  uint8_t j;          // register bit (0..r-1) for non-diagonal ops
  uint8_t ck, cb;     // control bit / diagonal bit: kind and index (register bit, local index, or physical pos)
  uint8_t ck2, cb2;   // second diagonal bit (CZ)
  uint8_t ph;         // phase exponent: multiply by i^ph (measurement / H-apply)
  uint8_t pad;
  int32_t slot;       // coefficient slot (gates) or gradient slot (OP_GRAD_*)
  uint32_t rz;        // z-mask over register bits
  uint32_t tz;        // z-mask over the thread's local-index bits
  uint32_t fr;        // flip mask over register bits (OP_MEAS_F, OP_H_F)
  uint64_t pz;        // z-mask over physical (tile) bits
  double c;           // term coefficient (measurement / H-apply)
};
static_assert(sizeof(DevOp) == 40, "DevOp layout");

constexpr int kMaxLocal = 16;
constexpr int kMaxQubits = 40;
constexpr int kMaxGradPerPass = 128;

constexpr int kMaxRegBits = 5;
constexpr int kMaxAffine = 8;

// A stage may end with a permutation of the tile: a run of CNOTs whose
// qubits are local (controls may also be non-local index bits) is a GF(2)
// affine map l -> M l + b(tile) on the local index, applied by writing each
// amplitude to its image in LDS at the exchange that ends the stage.
struct StageDesc {
  // Header: everything the pass kernel needs at the start of a stage, read as
  // one 64-byte block.  LDS addressing is precomputed on the host in swizzled
  // slots (the swizzle is linear over XOR, so a slot is the XOR of the parts
  // of its index bits).  Reading the stage's registers: slot of register i of
  // thread t = XOR_{k<6} t_k rd_lane[k] ^ rd_wave[t >> 6] ^ XOR_{j in i} rd_reg[j];
  // writing them at the exchange that ends the stage (through its exit
  // permutation when it has one, else the same slots):
  //   XOR_{k<6} t_k wr_lane[k] ^ wr_wave[t >> 6] ^ XOR_{tile bits} wr_aff ^ XOR_{j in i} wr_reg[j].
  // Entries for thread bits at or above m - r, and for register bits at or
  // above r, are zero.
  int32_t op_begin, op_end;
  uint16_t has_perm, n_aff; // exit permutation present; affine terms used
  uint32_t flags;           // SF_* below
  uint16_t rd_lane[6];
  uint16_t wr_lane[6];
  uint16_t rd_reg[6];
  uint16_t wr_reg[6];
  // the rest
  uint8_t rb[8];            // register bits as local indices
  uint8_t tb[kMaxLocal];    // thread bits as local indices: lane bits, then wave bits (m - r used)
  uint16_t tcol[kMaxLocal]; // M applied to thread bit k
  uint16_t preg[1 << kMaxRegBits];  // M applied to register offset i
  uint8_t aff_pos[kMaxAffine];      // physical non-local bit of affine term j
  uint16_t aff_mask[kMaxAffine];    // xor into the image when that bit is 1
  uint8_t tpos[kMaxLocal];  // physical bit of thread bit k (the pass's lpos[tb[k]])
  uint8_t rpos[8];          // physical bit of register bit j (lpos[rb[j]])
  uint8_t rbs[8];           // register bits as local indices, ascending (r used)
  uint16_t rd_wave[16];
  uint16_t wr_wave[16];
  uint16_t wr_aff[kMaxAffine];
};
// StageDesc flags: the stage has ops that read index bits (controls,
// diagonals, measurement signs: the thread's local index is needed); its last
// op is a factored rotation group (run after the op loop), whose first
// coefficient slot is flags >> 8; the exchange that ends the stage keeps every
// amplitude in its wave (each wave writes and reads its own block of slots, no
// workgroup barrier); the trailing factored group's tables are real (every
// member a real rotation: one real product per amplitude in two-state kernels).
enum StageFlags : uint32_t { SF_INDEX_OPS = 1, SF_LAST_UTAB = 2, SF_WAVE_LOCAL = 4, SF_REAL_TAB = 8 };
static_assert(sizeof(StageDesc) == 320, "StageDesc layout");
static_assert(offsetof(StageDesc, rb) == 64, "StageDesc header");

enum PassFlags : int32_t {
  PF_INIT = 1,      // first stage generates |0...0> instead of loading a
  PF_LOAD_A = 2,    // load a (psi) from HBM in the first stage
  PF_STORE_A = 4,   // store a in the last stage
  PF_LOAD_B = 8,    // load b (lambda) in the first stage (dual kernels)
  PF_STORE_B = 16,  // store b in the last stage (dual kernels)
  PF_ZERO_B = 32,   // b starts at zero (H-apply)
  PF_MEASURE = 64,  // write the block's measurement partial
  PF_GRAD = 128,    // write the block's gradient partials
};

struct PassDesc {
  int32_t n, m, r, flags;
  int32_t stage_begin, stage_end;
  int32_t meas_index;     // measurement partial column (PF_MEASURE)
  int32_t grad_begin;     // first gradient slot of this pass (PF_GRAD)
  int32_t grad_count;     // number of gradient slots used by this pass
  int32_t store_stage;    // absolute stage index after whose ops a (and b) are stored
  uint8_t lpos[kMaxLocal];   // physical bit of local index k
  uint8_t npos[kMaxQubits];  // physical bits of the non-local index, ascending (n - m used)
  // Entry permutation: a CNOT run that the planner applies while loading (the
  // first stage's registers are read from their sources under its inverse).
  // Source offsets are in physical index bits and XOR together.
  int32_t entry_perm;          // 1 when the loads go through the entry permutation
  int32_t n_eaff;              // affine terms used
  uint64_t ecol[kMaxLocal];    // source offset of the first stage's thread bit k
  uint64_t ereg[8];            // source offset of its register bit j
  uint64_t eaff[kMaxAffine];   // xor into the source offset when the tile's bit eaff_pos[j] is 1
  uint8_t eaff_pos[kMaxAffine];
  // Exit permutation: the last stage's CNOT run applied in the store addresses
  // (destination offsets under l -> M l ^ b, in physical index bits).
  int32_t exit_perm;           // 1 when the stores go through the exit permutation
  int32_t n_xaff;
  uint64_t xcol[kMaxLocal];    // destination offset of the last stage's thread bit k
  uint64_t xreg[8];            // destination offset of its register bit j
  uint64_t xaff[kMaxAffine];   // xor into the destination when the tile's bit xaff_pos[j] is 1
  uint8_t xaff_pos[kMaxAffine];
  // Product-state start (first pass only): the circuit's leading single-qubit
  // gates on every qubit are folded into the generated state prod_q U_q|0>; the
  // coefficient block at init_slot holds (U_q|0>)_0 and (U_q|0>)_1 per physical
  // qubit q (4 scalars each; 1 and 0 for qubits without such gates).
  int32_t init_fac;            // 1 when the first pass generates the product state
  int32_t init_slot;
};
static_assert(sizeof(PassDesc) == 648, "PassDesc layout");

// One light cone (or one small whole circuit) run by a single workgroup.
struct ConeDesc {
  int32_t pass_begin, pass_end;  // into the pass array
  int32_t coef_begin;            // first coefficient slot of this cone
  int32_t out_index;             // partial column written by this cone's measurement
  int64_t scratch_off;           // amplitude offset of the cone's state in scratch (s > m only)
  int32_t n;                     // cone qubits
  int32_t pad;
};

// One request's pass inside a multi-request launch (serving): blocks
// [tile_begin, tile_begin + 2^(n-m)) of the launch run this pass.
struct PassItem {
  const PassDesc* pass;
  const StageDesc* stages;
  const DevOp* ops;
  void* A;
  void* B;
  const void* coef;
  double* meas;        // [n_meas][tiles] of this request
  double* grad;        // [n_gslots][tiles] of this request
  int64_t tile_begin;
};

// Coefficient rows built on the device (parameters resident in device memory):
// one record per coefficient slot of a plan, and one per gate of the circuit.
enum CoefKind : int32_t {
  CK_U = 0,      // general 2x2: u00, u01, u10, u11 (complex)
  CK_RY = 1,     // real rotation: c, s
  CK_PHASE = 2,  // diagonal: d0, d1 (complex)
  CK_TAB = 3,    // factored group block over kTabSlots slots (written by its gen 0 slot)
  CK_INITF = 4,  // product-start block: (U_q|0>)_0, (U_q|0>)_1 per qubit (written by gen 0)
};

struct CoefSlot {
  int32_t kind;     // CoefKind
  int32_t inverse;  // the adjoint of the product of the source gates
  int32_t gen;      // chunk of a block (CK_TAB, CK_INITF)
  int32_t q;        // CK_TAB: register bits; CK_INITF: qubits
  int32_t src_off;  // sources: gate indices (CK_U/RY/PHASE, application order) or
  int32_t src_cnt;  // member slots (CK_TAB per register bit, CK_INITF per qubit; -1 = none)
};
static_assert(sizeof(CoefSlot) == 24, "CoefSlot layout");

struct CoefGate {
  int32_t kind;   // gate kind of the C-ABI (RX 0, RY 1, RZ 2, U1 5)
  int32_t param;  // parameter index, -1 = fixed angle
  double angle;
  double mat[8];  // U1: row-major (re, im)
};
static_assert(sizeof(CoefGate) == 80, "CoefGate layout");

}  // namespace qsim
