// Host planner: turns an ordered gate list into tiled passes, register
// stages and device ops; builds light cones and per-row coefficients.
//
// Pass selection.  A gate whose target is not among a pass's local qubits
// cannot be applied in that pass (its amplitude pairs straddle tiles), while
// diagonal gates (RZ phases, CZ) and the control of a CNOT need no locality.
// Gates are applied in a per-qubit order: a gate is ready once every earlier
// gate sharing a qubit with it has been applied.  Each pass picks its local
// set greedily among a few candidates (grown from the earliest ready gates,
// or a contiguous window of qubits) and applies every ready gate it can; one
// forward scan with "blocked" qubits computes that closure exactly.  This
// plays the role that contraction-path search plays in the paper's stack
// (Sec. 1, Sec. 3), for a memory layout where every pass streams the whole
// state through HBM once.
//
// Stage selection does the same at the register level inside a tile.
#include "planner.h"

#include "coefmath.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <thread>

namespace qsim {

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------

std::string validate_circuit(const CircuitDesc& c) {
  if (c.n < 1 || c.n > (1 << 24)) return "n_qubits out of range";
  if (c.n_params < 0) return "n_params < 0";
  for (size_t g = 0; g < c.gates.size(); ++g) {
    const Gate& x = c.gates[g];
    auto at = [g](const char* what) { return "gate " + std::to_string(g) + ": " + what; };
    if (x.q0 < 0 || x.q0 >= c.n) return at("qubit out of range");
    switch (x.kind) {
      case G_CZ:
      case G_CNOT:
        if (x.q1 < 0 || x.q1 >= c.n) return at("second qubit out of range");
        if (x.q1 == x.q0) return at("duplicate qubit");
        break;
      case G_RX:
      case G_RY:
      case G_RZ:
        if (x.param >= c.n_params) return at("parameter index out of range");
        break;
      case G_U1: {  // the factored rotation form relies on unitarity
        double err = 0;
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            double re = (i == j) ? -1.0 : 0.0, im = 0.0;  // (U^dagger U - I)_ij
            for (int k = 0; k < 2; ++k) {
              const double ar = x.mat[(k * 2 + i) * 2], ai = -x.mat[(k * 2 + i) * 2 + 1];
              const double br = x.mat[(k * 2 + j) * 2], bi = x.mat[(k * 2 + j) * 2 + 1];
              re += ar * br - ai * bi;
              im += ar * bi + ai * br;
            }
            err = std::max(err, std::max(std::fabs(re), std::fabs(im)));
          }
        if (!(err <= 1e-8)) return at("U1 matrix is not unitary");
        break;
      }
      default:
        return at("unknown gate kind");
    }
  }
  return "";
}

std::string validate_terms(const std::vector<Term>& terms, int n) {
  for (size_t t = 0; t < terms.size(); ++t) {
    const auto& ops = terms[t].ops;
    for (size_t k = 0; k < ops.size(); ++k) {
      const int q = ops[k].first;
      const char p = ops[k].second;
      if (q < 0 || q >= n) return "term " + std::to_string(t) + ": qubit out of range";
      if (p != 'X' && p != 'Y' && p != 'Z') return "term " + std::to_string(t) + ": bad Pauli letter";
      for (size_t k2 = 0; k2 < k; ++k2)
        if (ops[k2].first == q) return "term " + std::to_string(t) + ": duplicate qubit";
    }
  }
  return "";
}

// ---------------------------------------------------------------------------
// pgates
// ---------------------------------------------------------------------------

static int kind_of_1q(int k) { return k == G_RY ? PG_RY : k == G_RZ ? PG_PHASE : PG_U; }

void forward_pgates(const CircuitDesc& c, bool fuse, std::vector<PGate>& out, std::vector<PGate>& slots) {
  out.clear();
  slots.clear();
  std::vector<int> open(c.n, -1);  // pgate holding the current run of 1-qubit gates on a qubit
  for (int g = 0; g < (int)c.gates.size(); ++g) {
    const Gate& x = c.gates[g];
    if (x.kind == G_CZ || x.kind == G_CNOT) {
      open[x.q0] = open[x.q1] = -1;
      PGate p;
      if (x.kind == G_CZ) {
        p.kind = PG_CZ;
        p.q = x.q0;
        p.q2 = x.q1;
      } else {
        p.kind = PG_X;
        p.q = x.q1;   // target
        p.q2 = x.q0;  // control
      }
      p.srcs = {g};
      out.push_back(p);
      continue;
    }
    const int pk = kind_of_1q(x.kind);
    if (fuse && open[x.q0] >= 0) {
      PGate& p = out[open[x.q0]];
      p.srcs.push_back(g);
      if (p.kind != pk) p.kind = PG_U;  // RY after RY stays real, RZ after RZ stays diagonal
      continue;
    }
    PGate p;
    p.kind = pk;
    p.q = x.q0;
    p.srcs = {g};
    open[x.q0] = (int)out.size();
    out.push_back(p);
  }
  for (auto& p : out) {
    if (p.kind == PG_U || p.kind == PG_RY || p.kind == PG_PHASE) {
      // RY's then RZ's: the factored form needs no pre-diagonal
      bool seen_diag = false, seen_ry = false, ok = true;
      for (int g : p.srcs) {
        const int k = c.gates[g].kind;
        if (k == G_RY) {
          ok = ok && !seen_diag;
          seen_ry = true;
        } else if (k == G_RZ) {
          seen_diag = true;
        } else {
          ok = false;
        }
      }
      p.real_pre = ok && seen_ry;
      p.slot = (int)slots.size();
      slots.push_back(p);
    }
  }
}

void adjoint_pgates(const CircuitDesc& c, std::vector<PGate>& out, std::vector<PGate>& slots,
                    std::vector<int>& gslot_param) {
  out.clear();
  slots.clear();
  gslot_param.clear();
  for (int g = (int)c.gates.size() - 1; g >= 0; --g) {
    const Gate& x = c.gates[g];
    if (x.kind == G_CZ || x.kind == G_CNOT) {  // self-inverse
      PGate p;
      p.kind = x.kind == G_CZ ? PG_CZ : PG_X;
      p.q = x.kind == G_CZ ? x.q0 : x.q1;
      p.q2 = x.kind == G_CZ ? x.q1 : x.q0;
      p.srcs = {g};
      out.push_back(p);
      continue;
    }
    if ((x.kind == G_RX || x.kind == G_RY || x.kind == G_RZ) && x.param >= 0) {
      PGate gp;
      gp.kind = PG_GRAD;
      gp.q = x.q0;
      gp.gen = x.kind == G_RX ? 'X' : x.kind == G_RY ? 'Y' : 'Z';
      gp.slot = x.param;  // parameter index; the plan numbers gradient slots in execution order
      gp.srcs = {g};
      gslot_param.push_back(x.param);
      out.push_back(gp);
    }
    PGate p;
    p.kind = kind_of_1q(x.kind);
    p.q = x.q0;
    p.srcs = {g};
    p.inverse = true;
    p.real_pre = x.kind == G_RY;  // RY^-1 is real: a factored group needs no pre-diagonal for it
    p.slot = (int)slots.size();
    slots.push_back(p);
    out.push_back(p);
  }
}

void term_pgates(const std::vector<Term>& terms, bool happly, std::vector<PGate>& out, double& const_term,
                 const std::vector<int>* relabel) {
  out.clear();
  const_term = 0;
  for (const Term& t : terms) {
    if (t.ops.empty()) {
      const_term += t.c;
      continue;
    }
    PGate p;
    int ny = 0;
    for (auto [q0, L] : t.ops) {
      const int q = relabel ? (*relabel)[q0] : q0;
      const uint64_t b = 1ull << q;
      if (L == 'X' || L == 'Y') p.fmask |= b;
      if (L == 'Y' || L == 'Z') p.zmask |= b;
      if (L == 'Y') ++ny;
    }
    p.ph = ny & 3;
    p.c = t.c;
    p.kind = p.fmask ? (happly ? PG_H_F : PG_MEAS_F) : (happly ? PG_H_Z : PG_MEAS_Z);
    out.push_back(p);
  }
}

// ---------------------------------------------------------------------------
// pass and stage planning
// ---------------------------------------------------------------------------

namespace {

bool is_term(const PGate& g) { return g.kind >= PG_MEAS_Z && g.kind <= PG_H_F; }

// Qubits that must be local (register-resident) for g to be applied.
uint64_t need_mask(const PGate& g) {
  switch (g.kind) {
    case PG_U:
    case PG_RY:
    case PG_X:
      return 1ull << g.q;
    case PG_GRAD:
      return g.gen == 'Z' ? 0 : 1ull << g.q;
    case PG_MEAS_F:
    case PG_H_F:
      return g.fmask;
    default:
      return 0;
  }
}

// Whether gate g commutes with the Pauli term t (fmask: X/Y factors, zmask:
// Y/Z factors): a CNOT fixes X on its target and Z on its control, a diagonal
// gate fixes Z on its qubits; other single-qubit gates are taken not to commute
// with any factor on their qubit.
bool commutes_with_term(const PGate& g, const PGate& t) {
  auto f = [&](int q) { return q >= 0 && ((t.fmask >> q) & 1); };
  auto z = [&](int q) { return q >= 0 && ((t.zmask >> q) & 1); };
  switch (g.kind) {
    case PG_X:
      return !z(g.q) && !f(g.q2);
    case PG_CZ:
      return !f(g.q) && !f(g.q2);
    case PG_PHASE:
      return !f(g.q) && g.q2 < 0;
    default:
      return !f(g.q) && !z(g.q) && !f(g.q2) && !z(g.q2);
  }
}

// Qubits that order g against other gates.
int order_qubits(const PGate& g, int out[2]) {
  if (is_term(g)) return 0;
  int k = 0;
  if (g.q >= 0) out[k++] = g.q;
  if (g.q2 >= 0) out[k++] = g.q2;
  return k;
}

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// One forward scan: which pending gates a pass with local mask L applies.
double scan_pass(const std::vector<PGate>& G, const std::vector<int>& pending, uint64_t L, int n, int max_grad,
                 std::vector<int>* applied) {
  std::vector<char> blocked(n, 0);
  double score = 0;
  int ngrad = 0;
  for (int idx : pending) {
    const PGate& g = G[idx];
    if (is_term(g)) {
      // a term placed after the last gate it does not commute with: measured
      // once no earlier gate on its qubits waits; later gates commute with it,
      // so it blocks nothing
      const uint64_t supp = g.fmask | g.zmask;
      bool b = false;
      for (int q = 0; q < n; ++q) b |= ((supp >> q) & 1) && blocked[q];
      if (!b && (g.fmask & ~L) == 0) {
        score += 0.01;
        if (applied) applied->push_back(idx);
      }
      continue;
    }
    int qs[2];
    const int k = order_qubits(g, qs);
    bool b = false;
    for (int t = 0; t < k; ++t) b |= blocked[qs[t]] != 0;
    const uint64_t need = need_mask(g);
    bool ok = !b && (need & ~L) == 0;
    if (ok && g.kind == PG_GRAD && ngrad >= max_grad) ok = false;
    if (ok) {
      score += need ? 1.0 : 0.01;
      if (g.kind == PG_GRAD) ++ngrad;
      if (applied) applied->push_back(idx);
    } else {
      for (int t = 0; t < k; ++t) blocked[qs[t]] = 1;
    }
  }
  return score;
}

// Candidate grown from the earliest ready gates.
uint64_t grow_candidate(const std::vector<PGate>& G, const std::vector<int>& pending, uint64_t base, int n, int m) {
  std::vector<char> blocked(n, 0);
  uint64_t L = base;
  for (int idx : pending) {
    const PGate& g = G[idx];
    if (is_term(g)) continue;
    int qs[2];
    const int k = order_qubits(g, qs);
    bool b = false;
    for (int t = 0; t < k; ++t) b |= blocked[qs[t]] != 0;
    const uint64_t need = need_mask(g);
    if (!b && (need & ~L) != 0 && popcount64(L | need) <= m) L |= need;
    if (b || (need & ~L) != 0)
      for (int t = 0; t < k; ++t) blocked[qs[t]] = 1;
  }
  for (int q = 0; q < n && popcount64(L) < m; ++q) L |= 1ull << q;
  return L;
}

struct StageBuild {
  std::vector<int> rb;  // local indices
  std::vector<const PGate*> items;
  std::vector<const PGate*> perm;  // CNOTs applied as the stage's exit permutation, in order
  std::vector<int> tord;           // thread bits as local indices: lane bits first, then wave bits
};

// Relative costs used to choose between stage layouts (one LDS exchange of the
// tile versus register ops), in units of one general 2x2 op.
constexpr double kCostExchange = 2.0;
constexpr double kCostExchangeFactored = 1.35;
constexpr double kCostFactored = 1.2;
double op_cost(const PGate& g) {
  switch (g.kind) {
    case PG_U: return 1.0;
    case PG_RY: return 0.6;
    case PG_X: return 0.5;
    case PG_PHASE: return 0.6;
    case PG_CZ: return 0.3;
    case PG_GRAD: return 0.6;
    default: return 0.3;
  }
}

bool rb_has(const std::vector<int>& rb, int k) { return std::find(rb.begin(), rb.end(), k) != rb.end(); }

void fill_rb(std::vector<int>& rb, int r, int m, int lo) {
  for (int k = m - 1; k >= lo && (int)rb.size() < r; --k)
    if (!rb_has(rb, k)) rb.push_back(k);
  for (int k = m - 1; k >= 0 && (int)rb.size() < r; --k)
    if (!rb_has(rb, k)) rb.push_back(k);
}

// Local indices of a physical mask (all bits must be local).
std::vector<int> local_bits(uint64_t mask, const std::vector<int>& lidx) {
  std::vector<int> out;
  while (mask) {
    const int q = __builtin_ctzll(mask);
    mask &= mask - 1;
    out.push_back(lidx[q]);
  }
  return out;
}

// Try to place item g into a stage with register bits rb (extending rb within r and 'lo').
bool try_place(const PGate& g, std::vector<int>& rb, int r, int lo, const std::vector<int>& lidx) {
  const std::vector<int> need = local_bits(need_mask(g), lidx);
  std::vector<int> add;
  for (int k : need)
    if (!rb_has(rb, k)) {
      if (k < lo) return false;
      add.push_back(k);
    }
  if ((int)(rb.size() + add.size()) > r) return false;
  for (int k : add) rb.push_back(k);
  return true;
}

struct BitRef {
  uint8_t kind, idx;
};

struct PassEmitter {
  Plan& plan;
  int n, m, r;
  std::vector<int> L;     // physical qubits, ascending
  std::vector<int> lidx;  // physical -> local index (-1 = non-local)

  bool allow_absorb = true;
  bool allow_fused_bits = false;  // OP_UALL / OP_RYALL (single-state kernels with r <= 4 only)
  bool allow_factored = false;    // OP_UTAB (single-state float kernels with r <= 4 only)
  int io_lo = -1;                 // see PlanOptions::io_lo
  bool batch_probes = false;      // adjoint sweeps: diagonals and probes regrouped (see emit)
  bool allow_entry = false;       // fold a permute-only first stage into the loads
  bool allow_exit = false;        // apply the last stage's CNOT run in the store addresses
  bool sink_rotations = true;     // see sink()
  bool lanes_by_image = false;    // store stage with an exit permutation: lane bits are the thread
                                  // bits whose images are lowest (the permutation may move index bits)

  PassEmitter(Plan& p, int n_, int m_, int r_, uint64_t Lmask) : plan(p), n(n_), m(m_), r(r_), lidx(n_, -1) {
    for (int q = 0; q < n; ++q)
      if ((Lmask >> q) & 1) {
        lidx[q] = (int)L.size();
        L.push_back(q);
      }
  }

  BitRef bitref(int q, const std::vector<int>& rb) const {
    const int k = lidx[q];
    if (k < 0) return {BK_TILE, (uint8_t)q};
    for (int j = 0; j < (int)rb.size(); ++j)
      if (rb[j] == k) return {BK_REG, (uint8_t)j};
    return {BK_THREAD, (uint8_t)k};
  }

  void zmasks(uint64_t z, const std::vector<int>& rb, DevOp& op) const {
    op.rz = op.tz = 0;
    op.pz = 0;
    while (z) {
      const int q = __builtin_ctzll(z);
      z &= z - 1;
      const BitRef b = bitref(q, rb);
      if (b.kind == BK_REG) op.rz |= 1u << b.idx;
      else if (b.kind == BK_THREAD) op.tz |= 1u << b.idx;
      else op.pz |= 1ull << b.idx;
    }
  }

  DevOp to_devop(const PGate& g, const std::vector<int>& rb) const {
    DevOp op;
    std::memset(&op, 0, sizeof(op));
    op.slot = g.slot;
    auto regpos = [&](int q) { return bitref(q, rb).idx; };
    switch (g.kind) {
      case PG_U:
      case PG_RY:
      case PG_X: {
        op.type = g.kind == PG_U ? OP_U : g.kind == PG_RY ? OP_RY : OP_X;
        op.j = regpos(g.q);
        if (g.q2 >= 0) {
          const BitRef b = bitref(g.q2, rb);
          op.ck = b.kind;
          op.cb = b.idx;
        }
        break;
      }
      case PG_PHASE: {
        op.type = OP_PHASE;
        const BitRef b = bitref(g.q, rb);
        op.ck = b.kind;
        op.cb = b.idx;
        break;
      }
      case PG_CZ: {
        op.type = OP_CZ;
        const BitRef a = bitref(g.q, rb), b = bitref(g.q2, rb);
        op.ck = a.kind;
        op.cb = a.idx;
        op.ck2 = b.kind;
        op.cb2 = b.idx;
        break;
      }
      case PG_GRAD: {
        if (g.gen == 'Z') {
          op.type = OP_GRAD_Z;
          const BitRef b = bitref(g.q, rb);
          op.ck = b.kind;
          op.cb = b.idx;
        } else {
          op.type = g.gen == 'X' ? OP_GRAD_X : OP_GRAD_Y;
          op.j = regpos(g.q);
        }
        break;
      }
      case PG_MEAS_Z:
      case PG_H_Z:
      case PG_MEAS_F:
      case PG_H_F: {
        op.type = g.kind == PG_MEAS_Z ? OP_MEAS_Z : g.kind == PG_H_Z ? OP_H_Z : g.kind == PG_MEAS_F ? OP_MEAS_F : OP_H_F;
        zmasks(g.zmask, rb, op);
        uint64_t f = g.fmask;
        while (f) {
          const int q = __builtin_ctzll(f);
          f &= f - 1;
          op.fr |= 1u << bitref(q, rb).idx;
        }
        op.ph = (uint8_t)g.ph;
        op.c = g.c;
        break;
      }
    }
    return op;
  }

  // Splits the pass's items into stages.  With 'absorb', a CNOT whose qubits
  // no earlier item of the stage still needs is taken out of the op stream
  // and applied as part of the stage's exit permutation; later items on its
  // qubits move to the next stage.
  std::vector<StageBuild> build_stages(const std::vector<const PGate*>& mod, const std::vector<const PGate*>& ro,
                                       bool loads, bool stores, int c_low, bool absorb, int& store_rel) const {
    const int lo_io = io_lo >= 0 ? std::min(io_lo, c_low) : c_low;
    const int lo_load = loads ? lo_io : 0;
    const int lo_store = stores ? lo_io : 0;
    std::vector<StageBuild> sb;
    std::vector<const PGate*> pending = mod;
    bool first = true, stalled = false;
    while (!pending.empty()) {
      StageBuild s;
      std::vector<char> blocked(n, 0), permuted(n, 0);
      std::vector<const PGate*> rest;
      // gates that will want register bits (CNOTs go to the permutation)
      bool gates_left = false;
      for (const PGate* g : pending)
        gates_left |= !is_term(*g) && need_mask(*g) != 0 && !(absorb && g->kind == PG_X);
      gates_left &= !stalled;
      std::vector<const PGate*> held;  // terms left to a later stage
      for (const PGate* g : pending) {
        if (is_term(*g)) {
          // a term among the gates (after the last one it does not commute
          // with): in the first stage where no earlier gate on its qubits waits
          // or is left to the stage's permutation, on register bits the gates
          // already use while gates remain; blocks nothing
          const uint64_t supp = g->fmask | g->zmask;
          bool b = false;
          for (int q = 0; q < n; ++q) b |= ((supp >> q) & 1) && (blocked[q] || permuted[q]);
          for (const PGate* it : s.items) {
            if (is_term(*it)) continue;
            int iq[2];
            const int ik = order_qubits(*it, iq);
            for (int t = 0; t < ik; ++t) b |= ((supp >> iq[t]) & 1) != 0;
          }
          if (gates_left)
            for (int k : local_bits(g->fmask, lidx)) b |= !rb_has(s.rb, k);
          // it commutes with every item of the stage, so it is measured first
          if (!b && try_place(*g, s.rb, r, first ? lo_load : 0, lidx)) {
            s.items.insert(s.items.begin(), g);
          } else {
            rest.push_back(g);
            held.push_back(g);
          }
          continue;
        }
        int qs[2];
        const int k = order_qubits(*g, qs);
        bool b = false, pt = false;
        for (int t = 0; t < k; ++t) {
          b |= blocked[qs[t]] != 0;
          pt |= permuted[qs[t]] != 0;
        }
        // the gates after a term commute with it, except the index-bit swaps a
        // relabelling pass ends with: those wait for the terms they move
        for (const PGate* t : held) b |= !commutes_with_term(*g, *t);
        if (!b && absorb && g->kind == PG_X) {
          s.perm.push_back(g);
          for (int t = 0; t < k; ++t) permuted[qs[t]] = 1;
          continue;
        }
        if (!b && !pt && try_place(*g, s.rb, r, first ? lo_load : 0, lidx)) {
          s.items.push_back(g);
        } else {
          for (int t = 0; t < k; ++t) blocked[qs[t]] = 1;
          rest.push_back(g);
        }
      }
      // a stage that placed nothing: the terms take free register bits next
      stalled = s.items.empty() && s.perm.empty();
      fill_rb(s.rb, r, m, first ? lo_load : 0);
      sb.push_back(std::move(s));
      pending.swap(rest);
      first = false;
    }
    if (sb.empty()) {
      StageBuild s;
      fill_rb(s.rb, r, m, lo_load);
      sb.push_back(std::move(s));
    }
    // a permutation is realised at an exchange: give the last one a stage to land
    // in, unless it can go into the store addresses (stored pass, nothing read after)
    if (!sb.back().perm.empty()) {
      bool fold = allow_exit && stores && ro.empty() && sb.size() >= 2;
      for (int k : sb.back().rb) fold &= k >= lo_store;
      if (!fold) {
        StageBuild s;
        fill_rb(s.rb, r, m, lo_store);
        sb.push_back(std::move(s));
      }
    }
    store_rel = -1;
    if (stores) {
      bool ok = true;
      for (int k : sb.back().rb) ok &= k >= lo_store;
      if (!ok) {
        StageBuild s;
        fill_rb(s.rb, r, m, lo_store);
        sb.push_back(std::move(s));
      }
      store_rel = (int)sb.size() - 1;
    }
    // read-only terms: the last stage first, then new stages
    std::vector<const PGate*> left;
    for (const PGate* g : ro) {
      std::vector<int> rb = sb.back().rb;
      if (try_place(*g, rb, r, 0, lidx) && rb.size() == sb.back().rb.size()) sb.back().items.push_back(g);
      else left.push_back(g);
    }
    while (!left.empty()) {
      StageBuild s;
      std::vector<const PGate*> rest;
      for (const PGate* g : left) {
        if (try_place(*g, s.rb, r, 0, lidx)) s.items.push_back(g);
        else rest.push_back(g);
      }
      fill_rb(s.rb, r, m, 0);
      sb.push_back(std::move(s));
      left.swap(rest);
    }
    if (sink_rotations)
      for (StageBuild& st : sb) sink(st.items);
    return sb;
  }

  // Uncontrolled rotations move to the end of their stage past every later item
  // that leaves their qubit alone (probes, terms and diagonals on other qubits
  // commute with them), so that they can form the stage's trailing factored group.
  void sink(std::vector<const PGate*>& items) const {
    std::vector<char> ht(n, 0);  // qubits of the items that stay ahead, after the current one
    std::vector<const PGate*> head, tail;
    for (size_t i = items.size(); i-- > 0;) {
      const PGate* g = items[i];
      const bool rot = (g->kind == PG_U || g->kind == PG_RY) && g->q2 < 0;
      if (rot && !ht[g->q]) {
        tail.push_back(g);
        continue;
      }
      head.push_back(g);
      if (is_term(*g)) {
        for (int q = 0; q < n; ++q)
          if (((g->fmask | g->zmask) >> q) & 1) ht[q] = 1;
      } else {
        if (g->q >= 0) ht[g->q] = 1;
        if (g->q2 >= 0) ht[g->q2] = 1;
      }
    }
    items.assign(head.rbegin(), head.rend());
    items.insert(items.end(), tail.rbegin(), tail.rend());
  }

  // One OP_MEAS_ZS followed by a record per diagonal term items[i0, i1).
  void emit_zgroup(const std::vector<const PGate*>& items, size_t i0, size_t i1, const std::vector<int>& rb) {
    DevOp head;
    std::memset(&head, 0, sizeof(head));
    head.type = OP_MEAS_ZS;
    head.slot = (int)(i1 - i0);
    plan.ops.push_back(head);
    for (size_t k = i0; k < i1; ++k) {
      DevOp rec = to_devop(*items[k], rb);
      rec.type = OP_NONE;
      plan.ops.push_back(rec);
    }
  }

  double stages_cost(const std::vector<StageBuild>& sb) const {
    if (!allow_factored || r > 4) {
      double c = kCostExchange * (double)(sb.size() - 1);
      for (const StageBuild& s : sb)
        for (const PGate* g : s.items) c += op_cost(*g);
      return c;
    }
    // With factored rotations (in units of one general rotation applied alone,
    // from timings of the single-state pass kernel): an exchange costs about
    // 1.35, the trailing run of uncontrolled rotations on distinct register bits
    // about 1.2 when it becomes one factored op.
    double c = kCostExchangeFactored * (double)(sb.size() - 1);
    for (const StageBuild& s : sb) {
      size_t tail = s.items.size();  // start of the longest suffix of such rotations
      std::vector<char> used(r, 0);
      int direct = 0;  // instructions per pair, one by one (16 per general rotation, 8 per RY)
      while (tail > 0) {
        const PGate* h = s.items[tail - 1];
        if ((h->kind != PG_U && h->kind != PG_RY) || h->q2 >= 0) break;
        const BitRef b = bitref(h->q, s.rb);
        if (b.kind != BK_REG || used[b.idx]) break;
        used[b.idx] = 1;
        direct += h->kind == PG_U ? 16 : 8;
        --tail;
      }
      const bool fac = tail < s.items.size() && direct > 4 * r + 8;
      for (size_t i = 0; i < (fac ? tail : s.items.size()); ++i) c += op_cost(*s.items[i]);
      if (fac) c += kCostFactored;
    }
    return c;
  }

  // Fill the exit permutation of a stage from its CNOT run.
  // Images of a stage's CNOT run on the local index: l -> M l ^ b(tile), with
  // col[k] = M e_k and b = XOR of the masks of the affine terms whose
  // (physical, non-local) control bit is set in the tile.
  void perm_images(const StageBuild& s, std::vector<uint32_t>& col,
                   std::vector<std::pair<int, uint32_t>>& aff) const {
    col.assign(m, 0);
    for (int k = 0; k < m; ++k) col[k] = 1u << k;
    aff.clear();
    auto lbit = [&](uint32_t v, int c) { return (v >> c) & 1u; };
    for (const PGate* g : s.perm) {
      const int t = lidx[g->q];     // target is local
      const int cq = g->q2;         // control: local or non-local
      const int c = lidx[cq];
      for (int k = 0; k < m; ++k)
        if (c >= 0 && lbit(col[k], c)) col[k] ^= 1u << t;
      for (auto& a : aff)
        if (c >= 0 && lbit(a.second, c)) a.second ^= 1u << t;
      if (c < 0) {
        bool found = false;
        for (auto& a : aff)
          if (a.first == cq) {
            a.second ^= 1u << t;
            found = true;
          }
        if (!found) aff.push_back({cq, 1u << t});
      }
    }
  }

  // Physical index bits of a local index value.
  uint64_t phys(uint32_t l) const {
    uint64_t v = 0;
    for (int k = 0; k < m; ++k)
      if ((l >> k) & 1u) v |= 1ull << L[k];
    return v;
  }

  // Thread orders of stages first.. of a pass.  Lane bits are the lowest
  // non-register local indices except for the wave bits (the top m - r - 6
  // thread bits); the wave bits are chosen per stage so that as many exchanges
  // as possible keep every amplitude in its wave: the same wave bits on both
  // sides and no CNOT of the writer's exit permutation targeting one of them.
  // Such an exchange needs no workgroup barrier (each wave writes and reads its
  // own block of LDS).  Stages that load or store keep the lowest bits as lane
  // bits (whole segments per access; the lane bits above the always-local ones
  // are often the next index bits, which makes the segments longer).
  void choose_thread_orders(std::vector<StageBuild>& sb, int first, bool load_first, int store_idx) const {
    const int ns = (int)sb.size(), nt = m - r, nw = nt - 6;
    for (int s = first; s < ns; ++s) {
      sb[s].tord.clear();
      for (int k = 0; k < m; ++k)
        if (!rb_has(sb[s].rb, k)) sb[s].tord.push_back(k);
    }
    if (lanes_by_image && store_idx == ns - 1 && store_idx >= first && !sb[store_idx].perm.empty()) {
      // the store addresses apply the stage's permutation: order the thread bits
      // by the highest index bit of their image, so that the lane bits write
      // the lowest index bits
      std::vector<uint32_t> col;
      std::vector<std::pair<int, uint32_t>> aff;
      perm_images(sb[store_idx], col, aff);
      std::vector<int>& T = sb[store_idx].tord;
      std::stable_sort(T.begin(), T.end(), [&](int a, int b) {
        return 31 - __builtin_clz(col[a]) < 31 - __builtin_clz(col[b]);
      });
    }
    if (nw <= 0 || ns - first < 2) return;
    std::vector<std::vector<uint32_t>> cand(ns);
    std::vector<uint32_t> tgt(ns, 0);
    size_t width = 1;
    for (int s = first; s < ns; ++s) {
      const std::vector<int>& T = sb[s].tord;
      for (const PGate* g : sb[s].perm) tgt[s] |= 1u << lidx[g->q];
      uint32_t top = 0;
      for (int k = nt - nw; k < nt; ++k) top |= 1u << T[k];
      if ((s == first && load_first) || s == store_idx) {
        cand[s] = {top};  // the lowest thread bits stay lane bits: whole segments per access
        continue;
      }
      // every nw-subset of the thread bits (the default, the top ones, first)
      cand[s].push_back(top);
      std::vector<int> idx(nw);
      for (int i = 0; i < nw; ++i) idx[i] = i;
      while (true) {
        uint32_t w = 0;
        for (int i = 0; i < nw; ++i) w |= 1u << T[idx[i]];
        if (w != top) cand[s].push_back(w);
        int i = nw - 1;
        while (i >= 0 && idx[i] == nt - nw + i) --i;
        if (i < 0) break;
        ++idx[i];
        for (int j = i + 1; j < nw; ++j) idx[j] = idx[j - 1] + 1;
      }
      width = std::max(width, cand[s].size());
    }
    // longest chain of barrier-free exchanges: dynamic programme over the
    // stages (greedy beyond a size bound: keep the previous wave bits when allowed)
    std::vector<uint32_t> pick(ns);
    if ((double)ns * (double)width * (double)width <= 4e6) {
      std::vector<std::vector<int>> score(ns), from(ns);
      score[first].assign(cand[first].size(), 0);
      from[first].assign(cand[first].size(), -1);
      for (int s = first + 1; s < ns; ++s) {
        score[s].assign(cand[s].size(), -1);
        from[s].assign(cand[s].size(), 0);
        for (size_t c = 0; c < cand[s].size(); ++c)
          for (size_t p = 0; p < cand[s - 1].size(); ++p) {
            const int v = score[s - 1][p] + ((cand[s - 1][p] == cand[s][c] && !(tgt[s - 1] & cand[s][c])) ? 1 : 0);
            if (v > score[s][c]) {
              score[s][c] = v;
              from[s][c] = (int)p;
            }
          }
      }
      int c = 0;
      for (size_t k = 1; k < cand[ns - 1].size(); ++k)
        if (score[ns - 1][k] > score[ns - 1][c]) c = (int)k;
      for (int s = ns - 1; s >= first; --s) {
        pick[s] = cand[s][c];
        c = from[s][c];
      }
    } else {
      pick[first] = cand[first][0];
      for (int s = first + 1; s < ns; ++s) {
        pick[s] = cand[s][0];
        if (!(tgt[s - 1] & pick[s - 1]))
          for (uint32_t w : cand[s])
            if (w == pick[s - 1]) pick[s] = w;
      }
    }
    for (int s = first; s < ns; ++s) {
      std::vector<int> lanes, waves;
      for (int k : sb[s].tord) ((pick[s] >> k) & 1u ? waves : lanes).push_back(k);
      sb[s].tord = lanes;
      sb[s].tord.insert(sb[s].tord.end(), waves.begin(), waves.end());
    }
  }

  // The first stage of a loading pass only permutes: fold its CNOT run into the
  // loads of the next stage (registers read from M^-1 (l ^ b)) and drop it.
  bool fold_entry(std::vector<StageBuild>& sb, PassDesc& pd) const {
    if (sb.size() < 2 || !sb[0].items.empty() || sb[0].perm.empty()) return false;
    std::vector<uint32_t> col;
    std::vector<std::pair<int, uint32_t>> aff;
    perm_images(sb[0], col, aff);
    int na = 0;
    for (auto& a : aff) na += a.second != 0;
    if (na > kMaxAffine) return false;
    // inverse of M over GF(2): rows of [M | I] reduced
    std::vector<uint64_t> row(m, 0);  // low 32 bits: M's row, high: the identity's
    for (int t = 0; t < m; ++t) {
      uint32_t rv = 0;
      for (int k = 0; k < m; ++k) rv |= ((col[k] >> t) & 1u) << k;
      row[t] = rv | (1ull << (32 + t));
    }
    for (int c = 0; c < m; ++c) {
      int piv = -1;
      for (int t = c; t < m; ++t)
        if ((row[t] >> c) & 1ull) {
          piv = t;
          break;
        }
      if (piv < 0) return false;
      std::swap(row[c], row[piv]);
      for (int t = 0; t < m; ++t)
        if (t != c && ((row[t] >> c) & 1ull)) row[t] ^= row[c];
    }
    auto minv = [&](uint32_t v) {  // M^-1 v
      uint32_t out = 0;
      for (int t = 0; t < m; ++t) {
        const uint32_t rinv = (uint32_t)(row[t] >> 32);
        out |= (uint32_t)(__builtin_popcount(rinv & v) & 1) << t;
      }
      return out;
    };
    const StageBuild& s1 = sb[1];
    pd.entry_perm = 1;
    int t = 0;
    for (int k : s1.tord) pd.ecol[t++] = phys(minv(1u << k));
    for (int j = 0; j < r; ++j) pd.ereg[j] = phys(minv(1u << s1.rb[j]));
    pd.n_eaff = 0;
    for (auto& a : aff)
      if (a.second) {
        pd.eaff_pos[pd.n_eaff] = (uint8_t)a.first;
        pd.eaff[pd.n_eaff] = phys(minv(a.second));
        ++pd.n_eaff;
      }
    return true;
  }

  void fill_perm(const StageBuild& s, StageDesc& st) const {
    st.has_perm = 0;
    st.n_aff = 0;
    // identity images by default (used when has_perm == 0 only for clarity)
    std::vector<uint32_t> col(m);
    for (int k = 0; k < m; ++k) col[k] = 1u << k;
    std::vector<std::pair<int, uint32_t>> aff;  // (physical non-local bit, image mask)
    auto lbit = [&](uint32_t v, int c) { return (v >> c) & 1u; };
    for (const PGate* g : s.perm) {
      const int t = lidx[g->q];     // target is local
      const int cq = g->q2;         // control: local or non-local
      const int c = lidx[cq];
      for (int k = 0; k < m; ++k)
        if (c >= 0 && lbit(col[k], c)) col[k] ^= 1u << t;
      for (auto& a : aff)
        if (c >= 0 && lbit(a.second, c)) a.second ^= 1u << t;
      if (c < 0) {
        bool found = false;
        for (auto& a : aff)
          if (a.first == cq) {
            a.second ^= 1u << t;
            found = true;
          }
        if (!found) aff.push_back({cq, 1u << t});
      }
    }
    if (s.perm.empty()) return;
    st.has_perm = 1;
    int t = 0;
    for (int k : s.tord) st.tcol[t++] = (uint16_t)col[k];
    for (int i = 0; i < (1 << r); ++i) {
      uint32_t v = 0;
      for (int j = 0; j < r; ++j)
        if ((i >> j) & 1) v ^= col[s.rb[j]];
      st.preg[i] = (uint16_t)v;
    }
    for (auto& a : aff)
      if (a.second) {
        st.aff_pos[st.n_aff] = (uint8_t)a.first;
        st.aff_mask[st.n_aff] = (uint16_t)a.second;
        ++st.n_aff;
      }
  }

  // Emits one pass.  'mod' items modify the state(s) and keep their order;
  // 'ro' items are read-only terms measured after all of 'mod'.
  void emit(const std::vector<const PGate*>& mod, const std::vector<const PGate*>& ro, int flags,
            int c_low, int src_pass_index) {
    const bool loads = flags & (PF_LOAD_A | PF_LOAD_B);
    const bool stores = flags & (PF_STORE_A | PF_STORE_B);
    int store_rel = -1, store_rel2 = -1;
    std::vector<StageBuild> sb = build_stages(mod, ro, loads, stores, c_low, false, store_rel);
    bool can_absorb = allow_absorb && m <= 16;
    for (const PGate* g : mod)
      if (g->kind == PG_X && lidx[g->q2] < 0) {
        int na = 0;  // count distinct non-local controls (affine terms)
        std::vector<int> seen;
        for (const PGate* h : mod)
          if (h->kind == PG_X && lidx[h->q2] < 0 && std::find(seen.begin(), seen.end(), h->q2) == seen.end()) {
            seen.push_back(h->q2);
            ++na;
          }
        can_absorb &= na <= kMaxAffine;
        break;
      }
    if (can_absorb) {
      std::vector<StageBuild> sb2 = build_stages(mod, ro, loads, stores, c_low, true, store_rel2);
      if (stages_cost(sb2) < stages_cost(sb)) {
        sb.swap(sb2);
        store_rel = store_rel2;
      }
    }

    PassDesc pd;
    std::memset(&pd, 0, sizeof(pd));
    pd.n = n;
    pd.m = m;
    pd.r = r;
    pd.flags = flags;
    const int pass_no0 = (int)plan.passes.size();
    bool folded = false;
    if (allow_entry && (flags & PF_LOAD_A) && !(flags & PF_INIT) && store_rel != 0 && sb.size() >= 2) {
      choose_thread_orders(sb, 1, true, store_rel);  // the second stage loads once the first is folded
      folded = fold_entry(sb, pd);
    }
    if (!folded) choose_thread_orders(sb, 0, loads, store_rel);
    if (folded && plan.want_trace) {
      for (const PGate* g : sb[0].perm) plan.trace.push_back(*g);
      plan.trace.push_back(PGate{-1});
    }
    if (folded) {
      for (const PGate* g : sb[0].perm)
        for (int src : g->srcs) {  // applied while loading: ahead of the first stage's ops
          plan.order.push_back(pass_no0);
          plan.order.push_back(0);
          plan.order.push_back(-1);
          plan.order.push_back(src);
        }
      sb.erase(sb.begin());
      if (store_rel > 0) --store_rel;
    }
    pd.stage_begin = (int)plan.stages.size();
    pd.meas_index = -1;
    pd.store_stage = store_rel >= 0 ? pd.stage_begin + store_rel : -1;
    for (int k = 0; k < m; ++k) pd.lpos[k] = (uint8_t)L[k];
    {
      int j = 0;
      for (int q = 0; q < n; ++q)
        if (lidx[q] < 0) pd.npos[j++] = (uint8_t)q;
    }
    bool any_meas = false;
    int gmin = 1 << 30, gcount = 0;
    const int pass_no = (int)plan.passes.size();
    for (int si = 0; si < (int)sb.size(); ++si) {
      StageDesc st;
      std::memset(&st, 0, sizeof(st));
      const auto& rb = sb[si].rb;
      for (int j = 0; j < r; ++j) {
        st.rb[j] = (uint8_t)rb[j];
        st.rpos[j] = (uint8_t)L[rb[j]];
      }
      {
        std::vector<int> srt(rb.begin(), rb.begin() + r);
        std::sort(srt.begin(), srt.end());
        for (int j = 0; j < r; ++j) st.rbs[j] = (uint8_t)srt[j];
      }
      {
        int t = 0;
        for (int k : sb[si].tord) {
          st.tpos[t] = (uint8_t)L[k];
          st.tb[t++] = (uint8_t)k;
        }
      }
      st.op_begin = (int)plan.ops.size();
      const auto& its = sb[si].items;
      if (plan.want_trace) {
        for (const PGate* g : its) plan.trace.push_back(*g);
        for (const PGate* g : sb[si].perm) plan.trace.push_back(*g);
        plan.trace.push_back(PGate{-1});
      }
      auto record_order = [&](const PGate* h, int at) {
        for (int src : h->srcs) {
          plan.order.push_back(pass_no);
          plan.order.push_back(si);
          plan.order.push_back(at);
          plan.order.push_back(src);
        }
      };
      // Uncontrolled rotations on distinct register bits that end the stage's ops
      // (they commute) as one factored op, U_j = X^f P_j T_j E_j with diagonal P_j,
      // E_j, a real T_j of two multiply-adds per amplitude and a swap X^f left to
      // the stage's exit addressing; the P's (and E's) form one table over the
      // register index.  Taken (returns true) when cheaper than the rotations one
      // by one (instructions per amplitude pair: 16 per general rotation, 8 per
      // RY; factored 4 per register bit, 8 per table).
      auto emit_factored = [&](const std::vector<const PGate*>& run) {
        std::vector<const PGate*> member(r, nullptr);
        int cost = 0;
        bool pre = false;
        for (const PGate* h : run) {
          member[bitref(h->q, rb).idx] = h;
          cost += h->kind == PG_U ? 16 : 8;
          pre = pre || !h->real_pre;
        }
        if (!(cost > 4 * r + 8 + (pre ? 8 : 0))) return false;
        DevOp head;
        std::memset(&head, 0, sizeof(head));
        head.type = OP_UTAB;
        head.j = pre ? 1 : 0;
        head.slot = (int)plan.slots.size();
        PGate tab;
        tab.kind = PG_TAB;
        tab.q = r;
        for (int j = 0; j < r; ++j) {
          tab.srcs.push_back(member[j] ? member[j]->slot : -1);
          if (member[j]) head.fr |= 1u << j;
        }
        for (int chunk = 0; chunk < kTabSlots; ++chunk) {
          tab.gen = chunk;
          tab.slot = (int)plan.slots.size();
          plan.slots.push_back(tab);
        }
        if (pre) {
          DevOp d = head;
          d.type = OP_DTAB;
          plan.ops.push_back(d);
        }
        const int at = (int)plan.ops.size() - st.op_begin;
        plan.ops.push_back(head);
        for (int j = 0; j < r; ++j)
          if (member[j]) record_order(member[j], at);
        return true;
      };
      // gradient probes in groups of up to four (OP_GZS / OP_GXYS + records)
      auto emit_probes = [&](const std::vector<const PGate*>& probes, bool zgen) {
        for (size_t k0 = 0; k0 < probes.size(); k0 += 4) {
          const size_t k1 = std::min(probes.size(), k0 + 4);
          DevOp head;
          std::memset(&head, 0, sizeof(head));
          head.type = zgen ? OP_GZS : OP_GXYS;
          head.slot = (int)(k1 - k0);
          const int at = (int)plan.ops.size() - st.op_begin;
          plan.ops.push_back(head);
          for (size_t k = k0; k < k1; ++k) {
            const PGate* h = probes[k];
            DevOp rec = to_devop(*h, rb);
            rec.type = OP_NONE;
            rec.ph = h->gen == 'Y' ? 1 : 0;
            rec.slot = plan.n_gslots++;
            gmin = std::min(gmin, rec.slot);
            ++gcount;
            plan.gslot_param.push_back(h->slot);  // a probe's slot field holds its parameter index
            plan.ops.push_back(rec);
            record_order(h, at);
          }
        }
      };
      for (size_t ii = 0; ii < its.size(); ++ii) {
        const PGate* g = its[ii];
        // Adjoint sweep on two states.  A run of diagonal items (inverse phases,
        // CZ) and Z-generator probes: the diagonals first, register-bit phases on
        // distinct bits as one table over the register index, then the probes.
        // Both states receive the same diagonal unitary D, and D commutes with Z,
        // so <D lambda|Z|D psi> = <lambda|Z|psi> wherever a probe is taken.
        auto zrun = [&](const PGate* h) {
          return (h->kind == PG_GRAD && h->gen == 'Z') || (h->kind == PG_PHASE && h->q2 < 0) || h->kind == PG_CZ;
        };
        if (batch_probes && r <= 4 && zrun(g)) {
          size_t jj = ii;
          while (jj < its.size() && zrun(its[jj])) ++jj;
          std::vector<const PGate*> reg_ph(r, nullptr), lane_ph, others, probes;
          for (size_t k = ii; k < jj; ++k) {
            const PGate* h = its[k];
            if (h->kind == PG_GRAD) {
              probes.push_back(h);
            } else if (h->kind == PG_PHASE) {
              const BitRef b = bitref(h->q, rb);
              if (b.kind == BK_REG && !reg_ph[b.idx]) reg_ph[b.idx] = h;
              else if (b.kind != BK_REG && lane_ph.size() < 255) lane_ph.push_back(h);
              else others.push_back(h);
            } else {
              others.push_back(h);
            }
          }
          bool any_reg = false;
          for (const PGate* h : reg_ph) any_reg |= h != nullptr;
          if (any_reg || !lane_ph.empty()) {
            DevOp head;
            std::memset(&head, 0, sizeof(head));
            head.type = OP_PTAB;
            head.slot = -1;
            head.j = (uint8_t)lane_ph.size();
            if (any_reg) {
              head.slot = (int)plan.slots.size();
              PGate tab;
              tab.kind = PG_TAB;
              tab.q = r;
              for (int j = 0; j < r; ++j) tab.srcs.push_back(reg_ph[j] ? reg_ph[j]->slot : -1);
              for (int chunk = 0; chunk < kTabSlots; ++chunk) {
                tab.gen = chunk;
                tab.slot = (int)plan.slots.size();
                plan.slots.push_back(tab);
              }
            }
            const int at = (int)plan.ops.size() - st.op_begin;
            plan.ops.push_back(head);
            for (const PGate* h : reg_ph)
              if (h) record_order(h, at);
            for (const PGate* h : lane_ph) {  // records: the phase's bit and coefficient slot
              DevOp rec = to_devop(*h, rb);
              rec.type = OP_NONE;
              plan.ops.push_back(rec);
              record_order(h, at);
            }
          }
          for (const PGate* h : others) {
            record_order(h, (int)plan.ops.size() - st.op_begin);
            plan.ops.push_back(to_devop(*h, rb));
          }
          emit_probes(probes, true);
          ii = jj - 1;
          continue;
        }
        // A run of X/Y-generator probes and uncontrolled rotations on register
        // bits, where no probe follows a rotation on its own qubit: the probes
        // first, then the rotations in their order.  A rotation on another qubit
        // commutes with the probe's Pauli.
        auto xyrun = [&](const PGate* h) {
          if (h->q < 0 || h->q2 >= 0 || bitref(h->q, rb).kind != BK_REG) return false;
          return (h->kind == PG_GRAD && h->gen != 'Z') || h->kind == PG_RY || h->kind == PG_U;
        };
        if (batch_probes && xyrun(g) && g->kind == PG_GRAD) {
          size_t jj = ii;
          std::vector<int> rotated;  // qubits rotated so far in the run
          while (jj < its.size() && xyrun(its[jj])) {
            const PGate* h = its[jj];
            if (h->kind == PG_GRAD) {
              if (std::find(rotated.begin(), rotated.end(), h->q) != rotated.end()) break;
            } else {
              rotated.push_back(h->q);
            }
            ++jj;
          }
          std::vector<const PGate*> probes, rots;
          for (size_t k = ii; k < jj; ++k) (its[k]->kind == PG_GRAD ? probes : rots).push_back(its[k]);
          emit_probes(probes, false);
          // rotations that end the stage, one per register bit at most: a factored group
          bool distinct = !rots.empty();
          uint32_t used = 0;
          for (const PGate* h : rots) {
            const uint32_t bit = 1u << bitref(h->q, rb).idx;
            distinct = distinct && !(used & bit);
            used |= bit;
          }
          if (!(allow_factored && r <= 4 && jj == its.size() && distinct && emit_factored(rots)))
            for (const PGate* h : rots) {
              record_order(h, (int)plan.ops.size() - st.op_begin);
              plan.ops.push_back(to_devop(*h, rb));
            }
          ii = jj - 1;
          continue;
        }
        // a run of uncontrolled rotations on distinct register bits that ends the
        // stage's ops (they commute): one factored op, U_j = X^f P_j T_j E_j with
        // diagonal P_j, E_j, a real T_j of two multiply-adds per amplitude and a
        // swap X^f left to the stage's exit addressing; the P's (and E's) form one
        // table over the register index.  Taken when cheaper than the rotations one
        // by one (instructions per amplitude pair: 16 per general rotation, 8 per
        // RY; factored 4 per register bit, 8 per table).
        if (allow_factored && r <= 4 && (g->kind == PG_U || g->kind == PG_RY) && g->q2 < 0) {
          size_t jj = ii;
          std::vector<const PGate*> run;
          uint32_t used = 0;
          for (; jj < its.size(); ++jj) {
            const PGate* h = its[jj];
            if ((h->kind != PG_U && h->kind != PG_RY) || h->q2 >= 0) break;
            const BitRef b = bitref(h->q, rb);
            if (b.kind != BK_REG || ((used >> b.idx) & 1u)) break;
            used |= 1u << b.idx;
            run.push_back(h);
          }
          if (jj == its.size() && emit_factored(run)) {
            ii = jj - 1;
            continue;
          }
        }
        // r uncontrolled rotations of one kind on all r register bits (distinct qubits,
        // so they commute): one op applying them bit by bit
        if (allow_fused_bits && r <= 4 && (g->kind == PG_U || g->kind == PG_RY) && g->q2 < 0 &&
            ii + r <= its.size()) {
          std::vector<int> slot_of(r, -1);
          bool full = true;
          for (int k = 0; k < r && full; ++k) {
            const PGate* h = its[ii + k];
            if (h->kind != g->kind || h->q2 >= 0) {  // (terms have no qubit: check the kind first)
              full = false;
              break;
            }
            const BitRef b = bitref(h->q, rb);
            if (b.kind != BK_REG || slot_of[b.idx] >= 0) full = false;
            else slot_of[b.idx] = (int)(ii + k);
          }
          if (full) {
            DevOp head;
            std::memset(&head, 0, sizeof(head));
            head.type = g->kind == PG_U ? OP_UALL : OP_RYALL;
            head.slot = r;
            const int at = (int)plan.ops.size() - st.op_begin;
            plan.ops.push_back(head);
            for (int j = 0; j < r; ++j) {
              const PGate* h = its[slot_of[j]];
              plan.ops.push_back(to_devop(*h, rb));
              for (int src : h->srcs) {
                plan.order.push_back(pass_no);
                plan.order.push_back(si);
                plan.order.push_back(at);
                plan.order.push_back(src);
              }
            }
            ii += r - 1;
            continue;
          }
        }
        if (g->kind == PG_CZ && ii + 1 < its.size() && its[ii + 1]->kind == PG_CZ) {
          // a run of CZs (diagonal, they commute): one sign pattern over the
          // register index, the pairs on two register bits folded in on the host
          size_t jj = ii;
          while (jj < its.size() && its[jj]->kind == PG_CZ) ++jj;
          DevOp head;
          std::memset(&head, 0, sizeof(head));
          head.type = OP_CZS;
          std::vector<DevOp> recs;
          for (size_t k = ii; k < jj; ++k) {
            const BitRef a = bitref(its[k]->q, rb), b = bitref(its[k]->q2, rb);
            if (a.kind == BK_REG && b.kind == BK_REG) {
              for (int i = 0; i < (1 << r); ++i)
                if (((i >> a.idx) & 1) && ((i >> b.idx) & 1)) head.rz ^= 1u << i;
            } else {
              recs.push_back(to_devop(*its[k], rb));
            }
          }
          head.j = (uint8_t)recs.size();
          const int at = (int)plan.ops.size() - st.op_begin;
          for (size_t k = ii; k < jj; ++k) record_order(its[k], at);
          plan.ops.push_back(head);
          for (const DevOp& d : recs) plan.ops.push_back(d);
          ii = jj - 1;
          continue;
        }
        if (g->kind == PG_MEAS_Z) {  // a run of diagonal terms becomes one grouped op
          size_t jj = ii;
          while (jj < its.size() && its[jj]->kind == PG_MEAS_Z) ++jj;
          emit_zgroup(its, ii, jj, rb);
          any_meas = true;
          ii = jj - 1;
          continue;
        }
        DevOp op = to_devop(*g, rb);
        if (g->kind == PG_GRAD) {
          op.slot = plan.n_gslots++;
          gmin = std::min(gmin, op.slot);
          ++gcount;
          plan.gslot_param.push_back(g->slot);  // a gradient probe's slot field holds its parameter index
        }
        if (g->kind == PG_MEAS_Z || g->kind == PG_MEAS_F) any_meas = true;
        for (int src : g->srcs) {
          plan.order.push_back(pass_no);
          plan.order.push_back(si);
          plan.order.push_back((int)plan.ops.size() - st.op_begin);
          plan.order.push_back(src);
        }
        plan.ops.push_back(op);
      }
      st.op_end = (int)plan.ops.size();
      fill_perm(sb[si], st);
      for (const PGate* g : sb[si].perm)
        for (int src : g->srcs) {
          plan.order.push_back(pass_no);
          plan.order.push_back(si);
          plan.order.push_back(st.op_end - st.op_begin);  // after the stage's ops
          plan.order.push_back(src);
        }
      plan.stages.push_back(st);
    }
    pd.stage_end = (int)plan.stages.size();
    if (!sb.back().perm.empty() && store_rel == (int)sb.size() - 1) {
      // the last stage's CNOT run goes into the store addresses: destination
      // offsets of its thread and register bits under l -> M l ^ b
      std::vector<uint32_t> col;
      std::vector<std::pair<int, uint32_t>> aff;
      perm_images(sb.back(), col, aff);
      const StageBuild& sl = sb.back();
      pd.exit_perm = 1;
      int t = 0;
      for (int k : sl.tord) pd.xcol[t++] = phys(col[k]);
      for (int j = 0; j < r; ++j) pd.xreg[j] = phys(col[sl.rb[j]]);
      pd.n_xaff = 0;
      for (auto& a : aff)
        if (a.second && pd.n_xaff < kMaxAffine) {
          pd.xaff_pos[pd.n_xaff] = (uint8_t)a.first;
          pd.xaff[pd.n_xaff] = phys(a.second);
          ++pd.n_xaff;
        }
    }
    if (any_meas) {
      pd.flags |= PF_MEASURE;
      pd.meas_index = plan.n_meas++;
    }
    if (gcount) {
      pd.flags |= PF_GRAD;
      pd.grad_begin = gmin;
      pd.grad_count = gcount;
    }
    (void)src_pass_index;
    plan.passes.push_back(pd);
  }
};

// LDS slot maps.  The exchange after stage s of a pass (written by stage s
// through its exit permutation, read by stage s + 1) stores local index l at
// slot sigma(l), a linear bijection over GF(2) (rows: sigma(l) bit i = parity
// of row[i] & l).  An 8-byte slot's bank pair is its low five bits: reads serve
// 32 lanes per cycle and writes 16, so the low five rows are the reader's lane
// bits 0..4 plus terms outside them chosen so that the writer's lane bits 0..3
// also land in distinct banks.  In an exchange that keeps every amplitude in
// its wave the wave bits are the top rows: each wave owns one block of slots.
struct SlotMap {
  int m = 0;
  uint32_t row[kMaxLocal] = {0};
  uint32_t operator()(uint32_t l) const {
    uint32_t v = 0;
    for (int i = 0; i < m; ++i) v |= (uint32_t)(__builtin_popcount(row[i] & l) & 1) << i;
    return v;
  }
};

static int rank_low5(const SlotMap& sg, const uint32_t* v, int k) {
  uint32_t b[5] = {0, 0, 0, 0, 0};
  int r = 0;
  for (int i = 0; i < k; ++i) {
    uint32_t x = sg(v[i]) & 31u;
    for (int j = 4; j >= 0 && x; --j)
      if ((x >> j) & 1u) {
        if (!b[j]) {
          b[j] = x;
          ++r;
          break;
        }
        x ^= b[j];
      }
  }
  return r;
}

// reader lanes 0..4 (local indices), writer lane images 0..3, wave bits (mask, 0: none)
static SlotMap make_slot_map(int m, const uint8_t* rd_lanes, int n_rd, const uint32_t* wr_imgs, int n_wr,
                             uint32_t waves) {
  SlotMap sg;
  sg.m = m;
  if (n_rd < 5 || m < 5 + __builtin_popcount(waves)) {
    for (int i = 0; i < m; ++i) sg.row[i] = 1u << i;
    return sg;
  }
  uint32_t P = 0;
  for (int i = 0; i < 5; ++i) P |= 1u << rd_lanes[i];
  std::vector<int> Q;  // the rest, outside the wave bits
  for (int k = 0; k < m; ++k)
    if (!((P | waves) >> k & 1u)) Q.push_back(k);
  int i = 5;
  for (int k : Q) sg.row[i++] = 1u << k;
  for (int k = 0; k < m; ++k)
    if ((waves >> k) & 1u) sg.row[i++] = 1u << k;
  // low rows: the reader's lane bits, plus terms over Q (zero on the reader's
  // lanes) until the writer's lanes 0..3 reach four distinct bank bits
  for (int b = 0; b < 5; ++b) sg.row[b] = 1u << rd_lanes[b];
  const int want = std::min(n_wr, 4);
  int best = rank_low5(sg, wr_imgs, want);
  uint32_t rs = 0x9e3779b9u;
  SlotMap trial = sg;
  for (int t = 0; t < 256 && best < want && !Q.empty(); ++t) {
    for (int b = 0; b < 5; ++b) {
      uint32_t g = 0;
      for (int k : Q) {
        rs = rs * 1664525u + 1013904223u;
        if (rs >> 31) g |= 1u << k;
      }
      trial.row[b] = (1u << rd_lanes[b]) | g;
    }
    const int rk = rank_low5(trial, wr_imgs, want);
    if (rk > best) {
      best = rk;
      sg = trial;
    }
  }
  return sg;
}

// Fills the precomputed LDS addressing of every stage of a plan (StageDesc
// rd_* / wr_* fields and flags) from its register bits, thread bits and exit
// permutation, with one slot map per exchange.
void stage_addressing(Plan& plan) {
  for (const PassDesc& pd : plan.passes) {
    const int m = pd.m, r = pd.r, nt = m - r, nw = std::max(0, nt - 6);
    for (int s = pd.stage_begin; s < pd.stage_end; ++s) {
      StageDesc& st = plan.stages[s];
      std::memset(st.rd_lane, 0, sizeof(st.rd_lane));
      std::memset(st.rd_reg, 0, sizeof(st.rd_reg));
      std::memset(st.rd_wave, 0, sizeof(st.rd_wave));
      std::memset(st.wr_lane, 0, sizeof(st.wr_lane));
      std::memset(st.wr_reg, 0, sizeof(st.wr_reg));
      std::memset(st.wr_wave, 0, sizeof(st.wr_wave));
      std::memset(st.wr_aff, 0, sizeof(st.wr_aff));
      const bool utab = st.op_end > st.op_begin && plan.ops[st.op_end - 1].type == OP_UTAB;
      st.flags = (utab ? SF_LAST_UTAB : 0u) | ((st.op_end - st.op_begin > (utab ? 1 : 0)) ? SF_INDEX_OPS : 0u);
      if (utab) {
        const int slot = plan.ops[st.op_end - 1].slot;
        st.flags |= (uint32_t)slot << 8;
        bool real = !(plan.ops[st.op_end - 1].j & 1);  // no pre-diagonal
        for (int m : plan.slots[slot].srcs) real = real && (m < 0 || plan.slots[m].kind == PG_RY);
        if (real) st.flags |= SF_REAL_TAB;
      }
    }
    for (int s = pd.stage_begin; s + 1 < pd.stage_end; ++s) {
      StageDesc& w = plan.stages[s];
      StageDesc& rd = plan.stages[s + 1];
      // images of the writer's thread and register bits (and affine terms) in the local index
      uint32_t img_t[kMaxLocal] = {0}, img_r[8] = {0};
      for (int k = 0; k < nt; ++k) img_t[k] = w.has_perm ? w.tcol[k] : 1u << w.tb[k];
      for (int j = 0; j < r; ++j) img_r[j] = w.has_perm ? w.preg[1u << j] : 1u << w.rb[j];
      // every amplitude stays in its wave: the same wave bits on both sides,
      // and the writer's images keep the wave coordinates
      uint32_t wmask = 0;
      bool local = nw > 0;
      for (int k = 6; k < nt && local; ++k) {
        wmask |= 1u << w.tb[k];
        local = w.tb[k] == rd.tb[k];
      }
      for (int k = 0; k < nt && local; ++k) local = (img_t[k] & wmask) == ((1u << w.tb[k]) & wmask);
      for (int j = 0; j < r && local; ++j) local = (img_r[j] & wmask) == ((1u << w.rb[j]) & wmask);
      for (int j = 0; j < (int)w.n_aff && local && w.has_perm; ++j) local = (w.aff_mask[j] & wmask) == 0;
      const SlotMap sg = make_slot_map(m, rd.tb, std::min(nt, 6), img_t, std::min(nt, 6), local ? wmask : 0u);
      if (local) w.flags |= SF_WAVE_LOCAL;
      for (int k = 0; k < 6; ++k) {
        rd.rd_lane[k] = k < nt ? (uint16_t)sg(1u << rd.tb[k]) : 0;
        w.wr_lane[k] = k < nt ? (uint16_t)sg(img_t[k]) : 0;
      }
      for (int v = 0; v < 16; ++v) {
        uint32_t a = 0, b = 0;
        for (int bit = 0; bit < 4; ++bit)
          if (((v >> bit) & 1) && 6 + bit < nt) {
            a ^= sg(1u << rd.tb[6 + bit]);
            b ^= sg(img_t[6 + bit]);
          }
        rd.rd_wave[v] = (uint16_t)a;
        w.wr_wave[v] = (uint16_t)b;
      }
      for (int j = 0; j < r; ++j) {
        rd.rd_reg[j] = (uint16_t)sg(1u << rd.rb[j]);
        w.wr_reg[j] = (uint16_t)sg(img_r[j]);
      }
      for (int j = 0; j < kMaxAffine; ++j)
        w.wr_aff[j] = (w.has_perm && j < w.n_aff) ? (uint16_t)sg(w.aff_mask[j]) : 0;
    }
  }
}

// Candidate local sets of a pass that may hold any qubits in the always-local
// low positions, provided it shares at least c_low qubits with the previous
// pass (those are moved into the low positions when the previous pass stores):
// windows of w = m - c_low .. m consecutive qubits topped up with the previous
// pass's qubits nearest to the window, and the set grown from the earliest ready gates.
void relabel_candidates(const std::vector<PGate>& G, const std::vector<int>& pending, uint64_t prev, int n, int m,
                        int c_low, std::vector<uint64_t>& cands) {
  for (int w = m - c_low; w <= m; ++w)
    for (int s = 0; s + w <= n; ++s) {
      const uint64_t win = ((1ull << w) - 1) << s;
      std::vector<std::pair<int, int>> extra;  // (distance to the window, qubit)
      for (int q = 0; q < n; ++q)
        if (((prev >> q) & 1) && !((win >> q) & 1)) extra.push_back({std::min(std::abs(q - s), std::abs(q - (s + w - 1))), q});
      std::sort(extra.begin(), extra.end());
      uint64_t L = win;
      for (auto& e : extra) {
        if (popcount64(L) >= m) break;
        L |= 1ull << e.second;
      }
      if (popcount64(L & prev) >= c_low && popcount64(L) == m) cands.push_back(L);
    }
  const uint64_t g = grow_candidate(G, pending, 0, n, m);
  if (popcount64(g & prev) >= c_low) cands.push_back(g);
}

// Split gates into passes; returns the local masks and applied gate lists.
// Without 'relabel' the c_low lowest qubits are local in every pass.
// With 'left' the terms in G are measured in the passes where they are ready
// and local; 'left' receives those that no gate pass reaches.
void split_passes(int n, int m, int c_low, const std::vector<PGate>& G, int max_grad, std::vector<uint64_t>& Ls,
                  std::vector<std::vector<int>>& applied_lists, bool relabel = false,
                  std::vector<int>* left = nullptr) {
  std::vector<int> pending;
  int n_gates = 0;
  for (int i = 0; i < (int)G.size(); ++i) {
    const bool t = is_term(G[i]);
    if (!t || left) pending.push_back(i);
    n_gates += !t;
  }
  const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
  const uint64_t base = (1ull << c_low) - 1;
  while (n_gates > 0) {
    std::vector<uint64_t> cands;
    if (n <= m) {
      cands.push_back(all);
    } else if (relabel) {
      relabel_candidates(G, pending, Ls.empty() ? base : Ls.back(), n, m, c_low, cands);
    } else {
      cands.push_back(grow_candidate(G, pending, base, n, m));
      const int w = m - c_low;
      for (int s = c_low; s + w <= n; ++s) cands.push_back(base | (((1ull << w) - 1) << s));
    }
    double best = -1;
    uint64_t bestL = cands[0];
    for (uint64_t L : cands) {
      const double sc = scan_pass(G, pending, L, n, max_grad, nullptr);
      if (sc > best + 1e-9) {
        best = sc;
        bestL = L;
      }
    }
    std::vector<int> applied;
    scan_pass(G, pending, bestL, n, max_grad, &applied);
    if (applied.empty()) break;  // cannot happen: the first pending gate is always applicable
    std::vector<int> rest;
    size_t a = 0;
    for (int idx : pending) {
      if (a < applied.size() && applied[a] == idx) {
        ++a;
        n_gates -= !is_term(G[idx]);
      } else {
        rest.push_back(idx);
      }
    }
    Ls.push_back(bestL);
    applied_lists.push_back(std::move(applied));
    pending.swap(rest);
  }
  if (left) *left = pending;
}

// Measurement-only (or H-apply) passes for flip terms not covered yet.
void cover_terms(int n, int m, int c_low, const std::vector<const PGate*>& terms, std::vector<uint64_t>& Ls,
                 std::vector<std::vector<const PGate*>>& groups) {
  std::vector<const PGate*> left = terms;
  const uint64_t base = (1ull << c_low) - 1;
  while (!left.empty()) {
    uint64_t L = n <= m ? (n >= 64 ? ~0ull : ((1ull << n) - 1)) : base;
    std::vector<const PGate*> grp, rest;
    for (const PGate* g : left) {
      if (popcount64(L | g->fmask) <= m) {
        L |= g->fmask;
        grp.push_back(g);
      } else {
        rest.push_back(g);
      }
    }
    for (int q = 0; q < n && popcount64(L) < m; ++q) L |= 1ull << q;
    Ls.push_back(L);
    groups.push_back(grp);
    left.swap(rest);
  }
}

// Gates (and terms) of every pass in index-bit coordinates; with 'relabel' a
// storing pass ends with the swaps that move the next pass's c_low chosen
// qubits into the low index bits (the shared ones already there stay).  Sp:
// local index bits per pass; pos: qubit -> index bit after the last pass.
// With 'restore' the last pass ends with the swaps that put every qubit back at
// its own index bit; returns 1 (nothing else changed) when those bits are not all
// local in the last pass.
int relabel_passes(int n, int c_low, bool relabel, const std::vector<PGate>& G, const std::vector<uint64_t>& Ls,
                   const std::vector<std::vector<int>>& lists, std::vector<std::vector<PGate>>& pass_gates,
                   std::vector<uint64_t>& Sp, std::vector<int>& pos, std::string& err, bool restore = false) {
  const int np = (int)Ls.size();
  pos.assign(n, 0);
  std::vector<int> occ(n);  // index bit -> qubit
  std::iota(pos.begin(), pos.end(), 0);
  std::iota(occ.begin(), occ.end(), 0);
  pass_gates.assign(np, {});
  Sp.assign(np, 0);
  auto to_bits = [&](uint64_t mask) {
    uint64_t v = 0;
    for (int q = 0; q < n; ++q)
      if ((mask >> q) & 1) v |= 1ull << pos[q];
    return v;
  };
  for (int p = 0; p < np; ++p) {
    Sp[p] = to_bits(Ls[p]);
    std::vector<PGate>& pgl = pass_gates[p];
    for (int idx : lists[p]) {
      PGate g = G[idx];
      if (g.q >= 0) g.q = pos[g.q];
      if (g.q2 >= 0) g.q2 = pos[g.q2];
      g.fmask = to_bits(g.fmask);
      g.zmask = to_bits(g.zmask);
      pgl.push_back(std::move(g));
    }
    auto swap_bits = [&](int b, int hb) {  // index bits b and hb, both local in this pass
      for (int k = 0; k < 3; ++k) {
        PGate x;
        x.kind = PG_X;
        x.q = (k == 1) ? b : hb;   // target
        x.q2 = (k == 1) ? hb : b;  // control
        pgl.push_back(x);
      }
      const int qa = occ[b], qb = occ[hb];
      pos[qa] = hb;
      pos[qb] = b;
      occ[b] = qb;
      occ[hb] = qa;
    };
    if (relabel && restore && p + 1 == np) {
      bool inside = true;
      for (int b = 0; b < n; ++b) inside &= occ[b] == b || ((Sp[p] >> b) & 1);
      if (inside) {
        for (int b = 0; b < n; ++b)
          while (occ[b] != b) swap_bits(b, pos[b]);
        continue;
      }
      // else a pass of its own holding the displaced index bits and the low ones
      uint64_t S = (1ull << c_low) - 1;
      for (int b = 0; b < n; ++b)
        if (occ[b] != b) S |= 1ull << b;
      const int m = __builtin_popcountll(Sp[p]);
      if (__builtin_popcountll(S) > m) return 1;
      for (int b = 0; b < n && __builtin_popcountll(S) < m; ++b) S |= 1ull << b;
      Sp.push_back(S);
      pass_gates.emplace_back();
      std::vector<PGate>& rg = pass_gates.back();
      for (int b = 0; b < n; ++b)
        while (occ[b] != b) {
          const int hb = pos[b];
          for (int k = 0; k < 3; ++k) {
            PGate x;
            x.kind = PG_X;
            x.q = (k == 1) ? b : hb;
            x.q2 = (k == 1) ? hb : b;
            rg.push_back(x);
          }
          const int qa = occ[b], qb = occ[hb];
          pos[qa] = hb;
          pos[qb] = b;
          occ[b] = qb;
          occ[hb] = qa;
        }
      return 2;
    }
    if (!relabel || p + 1 == np) continue;
    if ((Sp[p] & ((1ull << c_low) - 1)) != ((1ull << c_low) - 1)) {
      err = "internal: a pass does not hold the low index bits";
      return -1;
    }
    // qubits for the next pass's low positions: the shared ones already there first
    const uint64_t shared = Ls[p] & Ls[p + 1];
    std::vector<int> want;
    for (int b = 0; b < c_low; ++b)
      if ((shared >> occ[b]) & 1) want.push_back(occ[b]);
    for (int q = 0; q < n && (int)want.size() < c_low; ++q)
      if (((shared >> q) & 1) && pos[q] >= c_low) want.push_back(q);
    for (int b = 0; b < c_low; ++b) {
      if (std::find(want.begin(), want.end(), occ[b]) != want.end()) continue;
      int a = -1;
      for (int q : want)
        if (pos[q] >= c_low) {
          a = q;
          break;
        }
      if (a < 0) {
        err = "internal: consecutive passes share too few qubits";
        return -1;
      }
      swap_bits(b, pos[a]);
    }
  }
  return 0;
}

int check_terms(const std::vector<PGate>& terms, int r, std::string& err) {
  for (const PGate& t : terms)
    if (popcount64(t.fmask) > r) {
      err = "a Pauli term with more than " + std::to_string(r) + " X/Y factors is not supported";
      return -1;
    }
  return 0;
}

}  // namespace

int plan_forward(int n, const std::vector<PGate>& gates_in, const std::vector<PGate>& meas, const PlanOptions& o,
                 Plan& plan, std::string& err) {
  if (n > kMaxQubits) {
    err = "dense mode supports at most 40 qubits";
    return -1;
  }
  // Product-state start: on every qubit, the fused single-qubit gate that comes
  // before any two-qubit gate on it acts on |0>, so the first pass can generate
  // prod_q U_q|0> instead of |0...0> and the gate leaves the plan.
  const std::vector<PGate>* gp = &gates_in;
  std::vector<PGate> rest;
  std::vector<int> lead_slot(n, -1);
  std::vector<const PGate*> lead;
  if (o.init && o.factored && o.init_factors && !plan.slots.empty()) {
    std::vector<char> touched(n, 0);
    for (const PGate& g : gates_in) {
      const bool one = (g.kind == PG_U || g.kind == PG_RY || g.kind == PG_PHASE) && g.q2 < 0;
      if (one && !touched[g.q] && g.slot >= 0) {
        lead_slot[g.q] = g.slot;
        lead.push_back(&g);
        touched[g.q] = 1;
        continue;
      }
      if (g.q >= 0) touched[g.q] = 1;
      if (g.q2 >= 0) touched[g.q2] = 1;
      rest.push_back(g);
    }
    if (!lead.empty()) gp = &rest;
  }
  const std::vector<PGate>& gates = *gp;
  plan.n = n;
  plan.m = std::min(n, o.m_max);
  plan.r = std::min(o.r, plan.m);
  const int m = plan.m, r = plan.r;
  // a kept final state is put back in qubit order by its last pass (or the plan
  // is made again without relabelling when that pass cannot)
  bool relabel = o.relabel && (!o.store_final || o.relabel_kept) && n > m;
  const bool restore = o.store_final;
again:
  const int c_low = n <= m ? 0 : std::min(relabel ? o.c_low_relabel : o.c_low, m - r);
  if (check_terms(meas, r, err)) return -1;

  // Relabelling: when the final state is not kept, the qubit held at each
  // index bit may change from pass to pass.  A pass that stores moves the
  // c_low qubits the next pass will hold in its low positions there (swaps of
  // index bits local to both, applied as CNOT triples in the pass's last
  // permutation), so any qubits can be local together as long as consecutive
  // passes share c_low of them.  Gates and terms are rewritten in index-bit
  // coordinates; plan.qmap keeps the final map for terms added later.
  // Early terms: a term with X/Y factors is measured in the first pass that
  // holds its flipped qubits after the last gate it does not commute with
  // (every later gate commutes with it, so the value is the final state's);
  // such terms ride along in the op list after that gate.  Diagonal terms and
  // those no gate pass reaches are measured at the end as before.
  std::vector<PGate> G2;
  G2.reserve(gates.size() + meas.size());
  std::vector<const PGate*> diag_terms;
  {
    std::vector<std::vector<const PGate*>> after(gates.size() + 1);
    for (const PGate& t : meas) {
      if (!o.early_terms || t.fmask == 0 || t.kind != PG_MEAS_F) {
        diag_terms.push_back(&t);
        continue;
      }
      int last = -1;
      for (int i = (int)gates.size() - 1; i >= 0; --i)
        if (!commutes_with_term(gates[i], t)) {
          last = i;
          break;
        }
      after[last + 1].push_back(&t);
    }
    for (size_t i = 0; i <= gates.size(); ++i) {
      if (i > 0) G2.push_back(gates[i - 1]);
      for (const PGate* t : after[i]) G2.push_back(*t);
    }
  }
  std::vector<uint64_t> Ls;
  std::vector<std::vector<int>> lists;
  std::vector<int> late;  // early terms no gate pass reached
  split_passes(n, m, c_low, G2, 1 << 30, Ls, lists, relabel && c_low > 0, &late);
  if (Ls.empty()) {
    Ls.push_back(n <= m ? ((1ull << n) - 1) : ((1ull << m) - 1));
    lists.emplace_back();
  }
  std::vector<std::vector<PGate>> pass_gates;
  std::vector<uint64_t> Sp;
  std::vector<int> pos;
  const int rr = relabel_passes(n, c_low, relabel && c_low > 0, G2, Ls, lists, pass_gates, Sp, pos, err,
                                restore);
  if (rr < 0) return -1;
  if (rr == 1) {
    relabel = false;
    goto again;
  }
  const int np = (int)Sp.size();  // with a pass that only puts the qubits back in order (rr == 2)
  auto to_bits = [&](uint64_t mask) {
    uint64_t v = 0;
    for (int q = 0; q < n; ++q)
      if ((mask >> q) & 1) v |= 1ull << pos[q];
    return v;
  };
  bool moved = false;
  for (int q = 0; q < n; ++q) moved |= pos[q] != q;
  if (moved) plan.qmap = pos;
  std::vector<PGate> meas_b;  // terms left to the end, in index-bit coordinates
  for (const PGate* t : diag_terms) meas_b.push_back(*t);
  for (int idx : late) meas_b.push_back(G2[idx]);
  for (PGate& t : meas_b) {
    t.fmask = to_bits(t.fmask);
    t.zmask = to_bits(t.zmask);
  }
  // terms measured in the final gate pass vs. extra read-only passes
  std::vector<const PGate*> fin, extra;
  for (const PGate& t : meas_b) {
    if ((t.fmask & ~Sp.back()) == 0) fin.push_back(&t);
    else extra.push_back(&t);
  }
  std::vector<uint64_t> mLs;
  std::vector<std::vector<const PGate*>> mgroups;
  cover_terms(n, m, c_low, extra, mLs, mgroups);

  for (int p = 0; p < np; ++p) {
    int flags = (p == 0 && o.init) ? PF_INIT : PF_LOAD_A;
    const bool last = p == np - 1;
    if (!last || o.store_final || !mLs.empty()) flags |= PF_STORE_A;
    PassEmitter em(plan, n, m, r, Sp[p]);
    em.allow_absorb = o.absorb;
    em.allow_fused_bits = true;
    em.allow_factored = o.factored && !plan.slots.empty();
    em.io_lo = o.io_lo;
    // (a pass that only puts the qubits back in order swaps through an exchange:
    // folded into its loads, the swaps would scatter the lanes' reads)
    em.allow_entry = o.factored && o.entry_perm && !(rr == 2 && last);
    em.allow_exit = o.factored && o.exit_perm;
    em.lanes_by_image = relabel && (!last || restore);
    std::vector<const PGate*> mod;
    for (const PGate& g : pass_gates[p]) mod.push_back(&g);
    em.emit(mod, last ? fin : std::vector<const PGate*>{}, flags, c_low, p);
  }
  for (size_t k = 0; k < mLs.size(); ++k) {
    PassEmitter em(plan, n, m, r, mLs[k]);
    em.emit({}, mgroups[k], PF_LOAD_A, c_low, -1);
    ++plan.meas_passes;
  }
  if (!lead.empty() && !plan.passes.empty() && (plan.passes[0].flags & PF_INIT)) {
    PGate blk;
    blk.kind = PG_INITF;
    blk.q = n;
    blk.srcs = lead_slot;
    plan.passes[0].init_fac = 1;
    plan.passes[0].init_slot = (int)plan.slots.size();
    for (int chunk = 0; chunk < init_slots(n); ++chunk) {
      blk.gen = chunk;
      blk.slot = (int)plan.slots.size();
      plan.slots.push_back(blk);
    }
    for (const PGate* g : lead)  // applied by the start state: ahead of everything
      for (int src : g->srcs) {
        plan.order.push_back(0);
        plan.order.push_back(0);
        plan.order.push_back(-2);
        plan.order.push_back(src);
      }
  }
  stage_addressing(plan);
  return 0;
}

int plan_happly(int n, const std::vector<PGate>& hterms, const PlanOptions& o, Plan& plan, std::string& err) {
  if (n > kMaxQubits) {
    err = "dense mode supports at most 40 qubits";
    return -1;
  }
  plan.n = n;
  plan.m = std::min(n, o.m_max);
  plan.r = std::min(o.r, plan.m);
  const int m = plan.m, r = plan.r;
  const int c_low = n <= m ? 0 : std::min(o.c_low, m - r);
  if (check_terms(hterms, r, err)) return -1;
  std::vector<const PGate*> diag, flips;
  for (const PGate& t : hterms) (t.fmask ? flips : diag).push_back(&t);
  std::vector<uint64_t> Ls;
  std::vector<std::vector<const PGate*>> groups;
  cover_terms(n, m, c_low, flips, Ls, groups);
  if (Ls.empty()) {
    Ls.push_back(n <= m ? ((1ull << n) - 1) : ((1ull << m) - 1));
    groups.emplace_back();
  }
  for (size_t p = 0; p < Ls.size(); ++p) {
    std::vector<const PGate*> mod = groups[p];
    if (p == 0) mod.insert(mod.begin(), diag.begin(), diag.end());
    const int flags = (p == 0 ? (PF_ZERO_B | PF_LOAD_A) : (PF_LOAD_A | PF_LOAD_B)) | PF_STORE_B;
    PassEmitter em(plan, n, m, r, Ls[p]);
    em.emit(mod, {}, flags, c_low, (int)p);
  }
  stage_addressing(plan);
  return 0;
}

int plan_adjoint(int n, const std::vector<PGate>& gates, const PlanOptions& o, Plan& plan, std::string& err) {
  if (n > kMaxQubits) {
    err = "dense mode supports at most 40 qubits";
    return -1;
  }
  plan.n = n;
  plan.m = std::min(n, o.m_max);
  plan.r = std::min(o.r, plan.m);
  const int m = plan.m, r = plan.r;
  // the sweep's final states are not used: its passes may relabel (see plan_forward)
  const bool relabel = o.relabel && n > m;
  const int c_low = n <= m ? 0 : std::min(relabel ? o.c_low_relabel : o.c_low, m - r);
  std::vector<uint64_t> Ls;
  std::vector<std::vector<int>> lists;
  split_passes(n, m, c_low, gates, o.max_grad, Ls, lists, relabel && c_low > 0);
  if (Ls.empty()) {  // no gates: one pass that changes nothing
    Ls.push_back(n <= m ? ((1ull << n) - 1) : ((1ull << m) - 1));
    lists.emplace_back();
  }
  const int np = (int)Ls.size();
  std::vector<std::vector<PGate>> pass_gates;
  std::vector<uint64_t> Sp;
  std::vector<int> pos;
  if (relabel_passes(n, c_low, relabel && c_low > 0, gates, Ls, lists, pass_gates, Sp, pos, err) < 0) return -1;
  for (int p = 0; p < np; ++p) {
    int flags = PF_LOAD_A | PF_LOAD_B;
    if (p != np - 1) flags |= PF_STORE_A | PF_STORE_B;
    PassEmitter em(plan, n, m, r, Sp[p]);
    em.allow_absorb = o.absorb;
    em.batch_probes = o.batch_probes;
    em.allow_factored = o.factored && !plan.slots.empty();
    em.allow_entry = o.factored && o.entry_perm;
    em.allow_exit = o.factored && o.exit_perm;
    em.lanes_by_image = relabel && p != np - 1;
    std::vector<const PGate*> mod;
    for (const PGate& g : pass_gates[p]) mod.push_back(&g);
    em.emit(mod, {}, flags, c_low, p);
  }
  stage_addressing(plan);
  return 0;
}

void append_diag_measure(Plan& plan, const std::vector<PGate>& meas) {
  if (meas.empty() || plan.passes.empty()) return;
  PassDesc& pd = plan.passes.back();
  const bool utab_last = plan.stages.back().op_end > plan.stages.back().op_begin &&
                         plan.ops[plan.stages.back().op_end - 1].type == OP_UTAB;
  if (utab_last || pd.exit_perm) {
    // a factored op ends the stage, or its CNOT run is left to the store
    // addresses: measure in a stage of its own with the same register bits (the
    // exchange between them applies the op's register swaps and the CNOT run)
    StageDesc nx = plan.stages.back();
    nx.has_perm = 0;
    nx.n_aff = 0;
    nx.op_begin = nx.op_end = (int)plan.ops.size();
    plan.stages.push_back(nx);
    pd.stage_end = (int)plan.stages.size();
  }
  StageDesc& st = plan.stages.back();
  uint64_t L = 0;
  for (int k = 0; k < pd.m; ++k) L |= 1ull << pd.lpos[k];
  PassEmitter em(plan, pd.n, pd.m, pd.r, L);
  std::vector<int> rb(st.rb, st.rb + pd.r);
  std::vector<PGate> meas_b = meas;  // in the index bits the plan ends with
  if (!plan.qmap.empty())
    for (PGate& t : meas_b) {
      uint64_t z = 0;
      for (int q = 0; q < pd.n; ++q)
        if ((t.zmask >> q) & 1) z |= 1ull << plan.qmap[q];
      t.zmask = z;
    }
  std::vector<const PGate*> items;
  for (const PGate& g : meas_b) items.push_back(&g);
  em.emit_zgroup(items, 0, items.size(), rb);
  if (plan.want_trace) {
    for (const PGate& g : meas_b) plan.trace.push_back(g);
    plan.trace.push_back(PGate{-1});
  }
  st.op_end = (int)plan.ops.size();
  if (!(pd.flags & PF_MEASURE)) {
    pd.flags |= PF_MEASURE;
    pd.meas_index = plan.n_meas++;
  }
  stage_addressing(plan);
}

// ---------------------------------------------------------------------------
// light cones
// ---------------------------------------------------------------------------

void light_cone(const CircuitDesc& c, const std::vector<int>& support, std::vector<int>& set,
                std::vector<int>& gates, const std::vector<char>* skip) {
  std::vector<char> in(c.n, 0);
  for (int q : support) in[q] = 1;
  gates.clear();
  for (int g = (int)c.gates.size() - 1; g >= 0; --g) {
    if (skip && (*skip)[g]) continue;
    const Gate& x = c.gates[g];
    if (x.kind == G_CZ || x.kind == G_CNOT) {
      if (in[x.q0] || in[x.q1]) {
        in[x.q0] = in[x.q1] = 1;
        gates.push_back(g);
      }
    } else if (in[x.q0]) {
      gates.push_back(g);
    }
  }
  std::reverse(gates.begin(), gates.end());
  set.clear();
  for (int q = 0; q < c.n; ++q)
    if (in[q]) set.push_back(q);
}

std::vector<char> trailing_diagonal(const CircuitDesc& c) {
  std::vector<char> drop(c.gates.size(), 0), open(c.n, 1);
  for (int g = (int)c.gates.size() - 1; g >= 0; --g) {
    const Gate& x = c.gates[g];
    const bool two = x.kind == G_CZ || x.kind == G_CNOT;
    const bool diag = x.kind == G_RZ || x.kind == G_CZ;
    const bool all_open = open[x.q0] && (!two || open[x.q1]);
    if (diag && all_open) {
      drop[g] = 1;
    } else {
      open[x.q0] = 0;
      if (two) open[x.q1] = 0;
    }
  }
  return drop;
}

// ---------------------------------------------------------------------------
// coefficients
// ---------------------------------------------------------------------------
// The matrices and blocks themselves are defined once (coefmath.h) for the
// host rows built here and the rows a device kernel builds from parameters
// resident in device memory.

namespace {

cm::M2 gate_matrix(const Gate& g, const double* th) {
  const double t = g.param >= 0 ? th[g.param] : g.angle;
  return cm::gate_m2(g.kind, t, g.mat);
}

// Matrix of a coefficient slot: product of its source gates, adjoint if flagged.
cm::M2 slot_m2(const CircuitDesc& c, const PGate& p, const double* th) {
  cm::M2 M = cm::eye();
  for (int g : p.srcs) M = cm::mul(gate_matrix(c.gates[g], th), M);
  return p.inverse ? cm::adjoint(M) : M;
}

}  // namespace

template <class T>
static void build_rows(const CircuitDesc& c, const std::vector<PGate>& slots, const double* params, int b0, int b1,
                       int64_t row_stride, T* out) {
  std::vector<cm::M2> ms(slots.size());
  for (int b = b0; b < b1; ++b) {
    const double* th = params ? params + (size_t)b * c.n_params : nullptr;
    T* row = out + (size_t)b * row_stride;
    for (size_t s = 0; s < slots.size(); ++s) {
      const PGate& p = slots[s];
      if (p.kind == PG_TAB || p.kind == PG_INITF) continue;
      T* o = row + s * 8;
      for (int k = 0; k < 8; ++k) o[k] = 0;
      const cm::M2 M = ms[s] = slot_m2(c, p, th);
      if (p.kind == PG_RY) {
        o[0] = (T)M.a[0][0].re;
        o[1] = (T)M.a[1][0].re;
      } else if (p.kind == PG_PHASE) {
        o[0] = (T)M.a[0][0].re; o[1] = (T)M.a[0][0].im;
        o[2] = (T)M.a[1][1].re; o[3] = (T)M.a[1][1].im;
      } else {
        o[0] = (T)M.a[0][0].re; o[1] = (T)M.a[0][0].im;
        o[2] = (T)M.a[0][1].re; o[3] = (T)M.a[0][1].im;
        o[4] = (T)M.a[1][0].re; o[5] = (T)M.a[1][0].im;
        o[6] = (T)M.a[1][1].re; o[7] = (T)M.a[1][1].im;
      }
    }
    // product-state start: (U_q|0>)_0, (U_q|0>)_1 per qubit over init_slots(n) slots
    for (size_t s = 0; s < slots.size(); ++s) {
      const PGate& p = slots[s];
      if (p.kind != PG_INITF || p.gen != 0) continue;
      T* o = row + s * 8;
      for (int e = 0; e < 8 * init_slots(p.q); ++e) o[e] = 0;
      for (int q = 0; q < p.q; ++q) {
        cm::C f0 = cm::mk(1), f1 = cm::mk(0);
        if (p.srcs[q] >= 0) {
          f0 = ms[p.srcs[q]].a[0][0];
          f1 = ms[p.srcs[q]].a[1][0];
        }
        o[4 * q] = (T)f0.re;
        o[4 * q + 1] = (T)f0.im;
        o[4 * q + 2] = (T)f1.re;
        o[4 * q + 3] = (T)f1.im;
      }
    }
    // factored groups: one block over kTabSlots consecutive slots, from the member matrices
    for (size_t s = 0; s < slots.size(); ++s) {
      const PGate& p = slots[s];
      if (p.kind != PG_TAB || p.gen != 0) continue;
      double blk[cm::kTabScalars];
      cm::M2 mm[4];
      int has[4] = {0, 0, 0, 0};
      const int r = std::min<int>(4, (int)p.srcs.size());
      for (int j = 0; j < r; ++j)
        if (p.srcs[j] >= 0) {
          mm[j] = ms[p.srcs[j]];
          has[j] = 1;
        }
      cm::tab_block(mm, has, r, blk);
      T* o = row + s * 8;
      for (int e = 0; e < 8 * kTabSlots; ++e) {
        if (e == 68 || e == 69) cm::put_raw(&o[e], (uint32_t)blk[e]);
        else o[e] = (T)blk[e];
      }
    }
  }
}

template <class T>
void build_coefficients(const CircuitDesc& c, const std::vector<PGate>& slots, const double* params, int batch,
                        int64_t row_stride, T* out) {
  // rows are independent: large batches are split over a few host threads
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::min({hw, 16, batch / 16});
  if (nt <= 1) {
    build_rows<T>(c, slots, params, 0, batch, row_stride, out);
    return;
  }
  std::vector<std::thread> th;
  const int per = (batch + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int b0 = t * per, b1 = std::min(batch, b0 + per);
    if (b0 < b1) th.emplace_back(build_rows<T>, std::cref(c), std::cref(slots), params, b0, b1, row_stride, out);
  }
  for (auto& x : th) x.join();
}

template void build_coefficients<float>(const CircuitDesc&, const std::vector<PGate>&, const double*, int, int64_t,
                                        float*);
template void build_coefficients<double>(const CircuitDesc&, const std::vector<PGate>&, const double*, int, int64_t,
                                         double*);

void coef_slot_table(const std::vector<PGate>& slots, std::vector<CoefSlot>& out, std::vector<int32_t>& srcs) {
  out.clear();
  srcs.clear();
  for (const PGate& p : slots) {
    CoefSlot s;
    s.kind = p.kind == PG_RY ? CK_RY : p.kind == PG_PHASE ? CK_PHASE : p.kind == PG_TAB ? CK_TAB
             : p.kind == PG_INITF ? CK_INITF : CK_U;
    s.inverse = p.inverse ? 1 : 0;
    s.gen = p.gen;
    s.q = p.q;
    s.src_off = (int32_t)srcs.size();
    s.src_cnt = (int32_t)p.srcs.size();
    for (int g : p.srcs) srcs.push_back(g);
    out.push_back(s);
  }
}

void coef_gate_table(const CircuitDesc& c, std::vector<CoefGate>& out) {
  out.resize(c.gates.size());
  for (size_t g = 0; g < c.gates.size(); ++g) {
    const Gate& x = c.gates[g];
    CoefGate& y = out[g];
    y.kind = x.kind;
    y.param = x.param;
    y.angle = x.angle;
    for (int k = 0; k < 8; ++k) y.mat[k] = x.mat[k];
  }
}

std::string structure_key(const CircuitDesc& c, const std::vector<Term>& terms, int extra) {
  // every field a plan depends on, in a fixed byte layout: equal keys mean equal structure
  size_t words = 5 + 2 * c.gates.size();
  for (const Term& t : terms) words += 2 + t.ops.size();
  std::string k(words * sizeof(uint64_t), '\0');
  char* wp = &k[0];
  auto put = [&](uint64_t v) {
    std::memcpy(wp, &v, sizeof v);
    wp += sizeof v;
  };
  put((uint64_t)c.n);
  put((uint64_t)c.n_params);
  put((uint64_t)(uint32_t)extra);
  put((uint64_t)c.gates.size());
  for (const Gate& g : c.gates) {
    put((uint64_t)(uint32_t)g.kind | ((uint64_t)(uint32_t)g.q0 << 32));
    put((uint64_t)(uint32_t)g.q1 | ((uint64_t)(uint32_t)g.param << 32));
  }
  put((uint64_t)terms.size());
  for (const Term& t : terms) {
    uint64_t cb;
    std::memcpy(&cb, &t.c, 8);
    put(cb);
    put((uint64_t)t.ops.size());
    for (auto [q, L] : t.ops) put(((uint64_t)(uint32_t)q << 8) | (uint8_t)L);
  }
  return k;
}

}  // namespace qsim
