// Evaluation paths: dense passes, light-cone batches and the adjoint sweep.
#include "engine.h"

#include <algorithm>
#include <functional>
#include <iterator>
#include <map>
#include <cstdlib>
#include <cstring>

namespace qsim {

void set_error(qsim_ctx* ctx, const std::string& msg) {
  if (!ctx) return;
  std::lock_guard<std::mutex> g(ctx->err_mu);
  ctx->err = msg;
}

int hip_fail(qsim_ctx* ctx, hipError_t e, const char* where) {
  set_error(ctx, std::string(where) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? QSIM_ENOMEM : QSIM_EDEVICE;
}

#define HIP_TRY(expr, where)                       \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

int timing_begin(qsim_ctx* ctx, hipStream_t st, double bytes, int flags, int kind, double flops) {
  if (!ctx->timing) return -1;
  TimingRec r;
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
  r.bytes = bytes;
  r.flops = flops;
  r.flags = flags;
  r.kind = kind;
  (void)hipEventRecord(r.a, st);
  ctx->tpending.push_back(r);
  return (int)ctx->tpending.size() - 1;
}

void timing_end(qsim_ctx* ctx, int idx, hipStream_t st) {
  if (idx >= 0) (void)hipEventRecord(ctx->tpending[idx].b, st);
}

void timing_collect(qsim_ctx* ctx) {
  for (TimingRec& r : ctx->tpending) {
    float ms = 0.f;
    (void)hipEventSynchronize(r.b);
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    r.ms = ms;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
    r.a = r.b = nullptr;
    ctx->tdone.push_back(r);
  }
  ctx->tpending.clear();
}

static double pass_bytes(const PassDesc& p, int rows, int c128) {
  const double amps = (double)rows * (double)(1ull << p.n);
  int k = 0;
  k += (p.flags & PF_LOAD_A) ? 1 : 0;
  k += (p.flags & PF_STORE_A) ? 1 : 0;
  k += (p.flags & PF_LOAD_B) ? 1 : 0;
  k += (p.flags & PF_STORE_B) ? 1 : 0;
  return amps * k * (c128 ? 16.0 : 8.0);
}

// Tuning knobs read once from the environment (for A/B measurements):
// QSIM_FWD_R = register bits of complex64 forward passes (3..5, default 4),
// QSIM_FWD_M = tile qubits of complex64 forward passes (12..14, default 13),
// QSIM_FWD_CLOW = index bits always local for coalescing (3..6, default 4),
// QSIM_DUAL_CLOW = the same for dual-state (adjoint) passes (default 6),
// QSIM_ABSORB = 0 disables CNOT exit permutations.
static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// Algorithmic floating-point operations per amplitude of one pass: 16 for a
// general 2x2 complex matrix (two complex products and a sum per output), 8
// for a real rotation, 6 for a diagonal phase, 0 for CNOT and CZ (sign or
// permutation); measurements 3 for |a|^2 once per group, then 2 per diagonal
// term and 4 per flip term; gradient probes 4; H-apply terms 4.
static double pass_flops_per_amp(const Plan& P, const PassDesc& pd, bool dual = false) {
  const double g = dual ? 2.0 : 1.0;  // gate ops of dual-state passes act on both states
  double f = 0;
  for (int s = pd.stage_begin; s < pd.stage_end; ++s) {
    const StageDesc& st = P.stages[s];
    for (int o = st.op_begin; o < st.op_end; ++o) {
      const DevOp& op = P.ops[o];
      switch (op.type) {
        case OP_U: f += 16 * g; break;
        case OP_UTAB: f += 4 * P.r + 6; break;  // a real 2x2 per register bit + the post table
        case OP_DTAB: f += 6; break;
        case OP_RY: f += 8 * g; break;
        case OP_PHASE: f += 6 * g; break;
        case OP_MEAS_ZS: f += 3 + 2.0 * op.slot; o += op.slot; break;
        case OP_MEAS_F: f += 4; break;
        case OP_GRAD_X: case OP_GRAD_Y: case OP_GRAD_Z: f += 4; break;
        case OP_PTAB: f += 6 * g; o += op.j; break;
        case OP_GZS: case OP_GXYS: f += 4.0 * op.slot; o += op.slot; break;
        case OP_CZS: o += op.j; break;  // sign flips
        case OP_H_Z: case OP_H_F: f += 4; break;
        default: break;
      }
    }
  }
  return f;
}

// Option value: the context's field when set (non-zero), else the environment
// variable of the same meaning (measurement sweeps), else the default.
static int opt_int(int field, const char* env, int dflt) { return field != 0 ? field : env_int(env, dflt); }

static bool opt_off(const qsim_options& co, int bit, const char* env, bool env_default_on) {
  if (co.disable & bit) return true;
  return env_int(env, env_default_on ? 1 : 0) == 0;
}

PlanOptions fwd_options(const qsim_options& co, int c128) {
  // 2^13-amplitude tiles with 16 per thread: two 512-thread workgroups per CU
  // (64 KiB of LDS each), so one workgroup's exchanges and barriers overlap the
  // other's arithmetic (measured faster than one 2^14 tile with 32 per thread).
  const int r64 = std::min(5, std::max(3, opt_int(co.register_bits, "QSIM_FWD_R", 4)));
  const int m64 = std::min(14, std::max(12, opt_int(co.tile_qubits, "QSIM_FWD_M", 13)));
  // four always-local low bits: 128-byte contiguous segments per access (a full
  // cache line) while leaving more local positions for gates (23 passes instead
  // of 33 at six for the n=30 workload; measured faster)
  const int clow = std::min(6, std::max(3, opt_int(co.coalesce_bits, "QSIM_FWD_CLOW", 4)));
  // with relabelling, five (256-byte segments): the passes it adds are fewer
  // than without (17 instead of 15 at n=30; measured faster)
  const int clow_rl = std::min(6, std::max(3, opt_int(co.coalesce_bits, "QSIM_FWD_CLOW", 5)));
  const bool absorb = !opt_off(co, QSIM_OFF_ABSORB, "QSIM_ABSORB", true);
  // uncontrolled rotations on a stage's register bits as one factored op (two
  // multiply-adds per amplitude and bit plus one diagonal table) in float plans
  const bool factored = !opt_off(co, QSIM_OFF_FACTORED, "QSIM_FACTORED", true);
  // lowest local bit that load/store stages may hold in registers (-1: the
  // always-local low bits stay lane bits, so every access covers whole segments;
  // default 0: a load/store stage may hold them too, which saves the extra stage
  // a pass would otherwise need to store, at the price of accesses that cover
  // each segment over several instructions; measured slightly faster)
  const int io_lo = (co.disable & QSIM_OFF_IO_REGS) ? -1 : std::min(6, std::max(-1, env_int("QSIM_IO_LO", 0)));
  PlanOptions o;
  o.m_max = c128 ? 13 : m64;
  o.r = c128 ? 4 : std::max(r64, o.m_max - 10);  // at most 1024 threads per workgroup
  o.c_low = clow;
  o.absorb = absorb;
  o.factored = factored && !c128 && o.r <= 4;
  o.io_lo = io_lo;
  // permutation folds and the product-state start (with factored; default on)
  const int folds = env_int("QSIM_FOLDS", 7);
  o.entry_perm = (folds & 1) != 0 && !(co.disable & QSIM_OFF_ENTRY);
  o.exit_perm = (folds & 2) != 0 && !(co.disable & QSIM_OFF_EXIT);
  o.init_factors = (folds & 4) != 0 && !(co.disable & QSIM_OFF_PRODUCT);
  // expectation-only plans: any c_low qubits shared by consecutive passes may
  // sit in the low index bits (fewer passes; measured faster)
  o.relabel = !opt_off(co, QSIM_OFF_RELABEL, "QSIM_RELABEL", true);
  o.c_low_relabel = clow_rl;
  o.relabel_kept = o.relabel && env_int("QSIM_RELABEL_KEPT", 1) != 0;
  o.early_terms = !opt_off(co, QSIM_OFF_EARLY_TERMS, "QSIM_EARLY_TERMS", true);
  return o;
}

PlanOptions cone_options(const qsim_options& co, int c128) {
  PlanOptions o = fwd_options(co, c128);
  o.relabel = false;  // a cone's sub-state keeps its qubit order
  o.early_terms = false;  // its terms are measured at its end
  o.r = 4;  // the cone kernel keeps 16 amplitudes per thread
  // factored rotation groups (float cones); every cone starts from |0...0>
  // (its coefficient slots are shared between cones, the start state's are not)
  o.init_factors = false;
  o.io_lo = -1;
  return o;
}

PlanOptions dual_options(const qsim_options& co, int c128) {
  PlanOptions o;
  o.absorb = !opt_off(co, QSIM_OFF_ABSORB, "QSIM_ABSORB", true);
  o.m_max = c128 ? 12 : std::min(13, std::max(12, env_int("QSIM_DUAL_M", 13)));
  o.r = c128 ? 3 : std::min(4, std::max(3, env_int("QSIM_DUAL_R", 4)));
  o.c_low = std::min(6, std::max(3, opt_int(co.dual_coalesce_bits, "QSIM_DUAL_CLOW", 6)));
  o.fuse = false;
  o.batch_probes = !opt_off(co, QSIM_OFF_BATCH_PROBES, "QSIM_BATCH_PROBES", true);
  // the rotations that end a stage as one factored group on both states (float, r <= 4)
  o.factored = !c128 && o.r <= 4 && !opt_off(co, QSIM_OFF_FACTORED, "QSIM_FACTORED", true);
  // the sweep's final states are not used: its passes relabel (with the rotations
  // sunk to their stage ends they still form factored groups; measured faster)
  o.relabel = !opt_off(co, QSIM_OFF_RELABEL, "QSIM_RELABEL", true);
  o.c_low_relabel = std::min(6, std::max(3, env_int("QSIM_DUAL_CLOW_RL", 5)));
  // permute-only first stages folded into the loads, last CNOT runs into the store
  // addresses of both states
  o.entry_perm = !(co.disable & QSIM_OFF_ENTRY);
  o.exit_perm = !(co.disable & QSIM_OFF_EXIT);
  return o;
}

bool prefetch_on(const qsim_options& co) { return !opt_off(co, QSIM_OFF_PREFETCH, "QSIM_FWD_PF", true); }

DevPlan::DevPlan() {
  static std::atomic<uint64_t> next{1};
  uid = next++;
}

DevPlan::~DevPlan() {
  (void)hipFree(d_passes);
  (void)hipFree(d_stages);
  (void)hipFree(d_ops);
  (void)hipFree(d_cones);
  (void)hipFree(d_order);
  (void)hipFree(d_poff);
  (void)hipFree(d_pslots);
  (void)hipFree(d_cslots);
  (void)hipFree(d_csrcs);
  (void)hipFree(d_toff);
  (void)hipFree(d_tfac);
  (void)hipFree(d_tcoef);
  (void)hipFree(d_gcone);
  (void)hipFree(d_foff);
  (void)hipFree(d_fterms);
}

template <class V>
static hipError_t upload_vec(const std::vector<V>& v, V** d) {
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(V);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(d), bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*d, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice);
  return e;
}

hipError_t DevPlan::upload(bool mock) {
  if (mock) return hipSuccess;
  hipError_t e;
  if ((e = upload_vec(plan.passes, &d_passes)) != hipSuccess) return e;
  if ((e = upload_vec(plan.stages, &d_stages)) != hipSuccess) return e;
  if ((e = upload_vec(plan.ops, &d_ops)) != hipSuccess) return e;
  {
    std::vector<CoefSlot> cs;
    std::vector<int32_t> srcs;
    coef_slot_table(plan.slots, cs, srcs);
    if ((e = upload_vec(cs, &d_cslots)) != hipSuccess) return e;
    if ((e = upload_vec(srcs, &d_csrcs)) != hipSuccess) return e;
  }
  if (!cones.empty()) {
    if ((e = upload_vec(cones, &d_cones)) != hipSuccess) return e;
    if ((e = upload_vec(order, &d_order)) != hipSuccess) return e;
  }
  if (factored) {
    if ((e = upload_vec(t_off, &d_toff)) != hipSuccess) return e;
    if ((e = upload_vec(t_fac, &d_tfac)) != hipSuccess) return e;
    if ((e = upload_vec(t_coef, &d_tcoef)) != hipSuccess) return e;
  }
  if (cone_grad) {
    if ((e = upload_vec(g_cone, &d_gcone)) != hipSuccess) return e;
    if ((e = upload_vec(f_off, &d_foff)) != hipSuccess) return e;
    if ((e = upload_vec(f_terms, &d_fterms)) != hipSuccess) return e;
  }
  if (plan.n_gslots > 0) {
    int np = 0;
    for (int p : plan.gslot_param) np = std::max(np, p + 1);
    std::vector<int32_t> off(np + 1, 0), slots;
    for (int p : plan.gslot_param) off[p + 1]++;
    for (int p = 0; p < np; ++p) off[p + 1] += off[p];
    slots.resize(plan.gslot_param.size());
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int s = 0; s < (int)plan.gslot_param.size(); ++s) slots[fill[plan.gslot_param[s]]++] = s;
    if ((e = upload_vec(off, &d_poff)) != hipSuccess) return e;
    if ((e = upload_vec(slots, &d_pslots)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------

int to_circuit(qsim_ctx* ctx, const qsim_circuit* c, CircuitDesc& out) {
  if (!c || c->n_gates < 0 || (c->n_gates > 0 && !c->gates)) {
    set_error(ctx, "circuit: null or negative gate count");
    return QSIM_EINVAL;
  }
  out.n = c->n_qubits;
  out.n_params = c->n_params;
  out.gates.resize(c->n_gates);
  for (int g = 0; g < c->n_gates; ++g) {
    const qsim_gate& x = c->gates[g];
    Gate& y = out.gates[g];
    y.kind = x.kind;
    y.q0 = x.q0;
    y.q1 = x.q1;
    y.param = (x.kind == QSIM_RX || x.kind == QSIM_RY || x.kind == QSIM_RZ) ? x.param : -1;
    if (y.param < -1) y.param = -1;
    y.angle = x.angle;
    std::memset(y.mat, 0, sizeof(y.mat));
    if (x.kind == QSIM_U1) {
      if (!x.mat) {
        set_error(ctx, "gate " + std::to_string(g) + ": U1 without a matrix");
        return QSIM_EINVAL;
      }
      std::memcpy(y.mat, x.mat, sizeof(y.mat));
    }
  }
  const std::string err = validate_circuit(out);
  if (!err.empty()) {
    set_error(ctx, "circuit: " + err);
    return QSIM_EINVAL;
  }
  return QSIM_OK;
}

int to_terms(qsim_ctx* ctx, const qsim_hamiltonian* H, int n, std::vector<Term>& out) {
  out.clear();
  if (!H) {
    set_error(ctx, "hamiltonian: null");
    return QSIM_EINVAL;
  }
  if (H->n_terms < 0 || (H->n_terms > 0 && (!H->coeff || !H->term_off))) {
    set_error(ctx, "hamiltonian: bad arrays");
    return QSIM_EINVAL;
  }
  out.resize(H->n_terms);
  for (int t = 0; t < H->n_terms; ++t) {
    const int a = H->term_off[t], b = H->term_off[t + 1];
    if (b < a || (b > a && (!H->qubits || !H->paulis))) {
      set_error(ctx, "hamiltonian: bad term offsets");
      return QSIM_EINVAL;
    }
    out[t].c = H->coeff[t];
    out[t].ops.resize(b - a);
    for (int k = a; k < b; ++k) out[t].ops[k - a] = {H->qubits[k], (char)H->paulis[k]};
  }
  const std::string err = validate_terms(out, n);
  if (!err.empty()) {
    set_error(ctx, "hamiltonian: " + err);
    return QSIM_EINVAL;
  }
  return QSIM_OK;
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------

static std::shared_ptr<DevPlan> cache_get(qsim_ctx* ctx, const std::string& key) {
  std::lock_guard<std::mutex> g(ctx->plan_mu);
  auto it = ctx->plans.find(key);
  return it == ctx->plans.end() ? nullptr : it->second;
}

static void cache_put(qsim_ctx* ctx, const std::string& key, std::shared_ptr<DevPlan> p) {
  std::lock_guard<std::mutex> g(ctx->plan_mu);
  if (ctx->plans.size() >= 256) ctx->plans.clear();
  ctx->plans[key] = std::move(p);
}

// Plan of the gates alone (no measurement), on the host.
static int plan_gates_host(qsim_ctx* ctx, const CircuitDesc& c, int c128, bool init, bool store_final, Plan& out,
                           bool trace = false) {
  out = Plan();
  out.want_trace = trace;
  std::vector<PGate> pg;
  forward_pgates(c, true, pg, out.slots);
  PlanOptions o = fwd_options(ctx->opt, c128);
  o.init = init;
  o.store_final = store_final;
  std::string err;
  if (plan_forward(c.n, pg, {}, o, out, err)) {
    set_error(ctx, err);
    return QSIM_EINVAL;
  }
  return QSIM_OK;
}

// Plan of the gates alone, cached by circuit structure.
static std::shared_ptr<DevPlan> gate_plan(qsim_ctx* ctx, const CircuitDesc& c, int c128, bool init, bool store_final,
                                          int& rc) {
  const int extra = 0x500 | c128 | (init << 1) | (store_final << 2);
  const std::string key = structure_key(c, {}, extra);
  if (auto p = cache_get(ctx, key)) return p;
  auto dp = std::make_shared<DevPlan>();
  if ((rc = plan_gates_host(ctx, c, c128, init, store_final, dp->plan))) return nullptr;
  hipError_t e = dp->upload(ctx->mock);
  if (e != hipSuccess) {
    rc = hip_fail(ctx, e, "plan upload");
    return nullptr;
  }
  cache_put(ctx, key, dp);
  return dp;
}

int host_dense_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms, int c128, bool init,
                    bool store_final, Plan& out, bool trace) {
  // the same plan get_dense_plan(..., measure = true) builds, without its device copy
  std::vector<PGate> meas;
  double cst = 0;
  term_pgates(terms, false, meas, cst);
  bool diag = true;
  for (const PGate& t : meas) diag &= t.fmask == 0;
  if (meas.empty() || diag) {
    int rc = plan_gates_host(ctx, c, c128, init, store_final, out, trace);
    if (rc) return rc;
    if (meas.empty() && cst == 0.0) return QSIM_OK;
    append_diag_measure(out, meas);
    out.const_term = cst;
    return QSIM_OK;
  }
  out = Plan();
  out.want_trace = trace;
  std::vector<PGate> pg;
  forward_pgates(c, true, pg, out.slots);
  PlanOptions o = fwd_options(ctx->opt, c128);
  o.init = init;
  o.store_final = store_final;
  std::string err;
  if (plan_forward(c.n, pg, meas, o, out, err)) {
    set_error(ctx, err);
    return QSIM_EINVAL;
  }
  out.const_term = cst;
  return QSIM_OK;
}

int host_forward_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms, bool store_final,
                      Plan& out) {
  int rc = QSIM_OK;
  std::vector<PGate> meas;
  double cst = 0;
  term_pgates(terms, false, meas, cst);
  bool diag = true;
  for (const PGate& t : meas) diag &= t.fmask == 0;
  if (diag) {
    auto gp = gate_plan(ctx, c, 0, true, store_final, rc);
    if (!gp) return rc;
    out = gp->plan;
    append_diag_measure(out, meas);
    out.const_term = cst;
    return QSIM_OK;
  }
  out = Plan();
  std::vector<PGate> pg;
  forward_pgates(c, true, pg, out.slots);
  PlanOptions o = fwd_options(ctx->opt, 0);
  o.store_final = store_final;
  std::string err;
  if (plan_forward(c.n, pg, meas, o, out, err)) {
    set_error(ctx, err);
    return QSIM_EINVAL;
  }
  out.const_term = cst;
  return QSIM_OK;
}

int host_happly_plan(qsim_ctx* ctx, int n, const std::vector<Term>& terms, Plan& out) {
  std::vector<PGate> ht;
  double cst = 0;
  term_pgates(terms, true, ht, cst);
  if (cst != 0.0) {
    PGate p;
    p.kind = PG_H_Z;
    p.c = cst;
    ht.push_back(p);
  }
  out = Plan();
  std::string err;
  if (plan_happly(n, ht, dual_options(ctx->opt, 0), out, err)) {
    set_error(ctx, err);
    return QSIM_EINVAL;
  }
  return QSIM_OK;
}

std::shared_ptr<DevPlan> get_dense_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms,
                                        int c128, bool init, bool store_final, bool measure, int& rc) {
  rc = QSIM_OK;
  std::vector<PGate> meas;
  double cst = 0;
  if (measure) term_pgates(terms, false, meas, cst);
  bool diag = true;
  for (const PGate& t : meas) diag &= t.fmask == 0;
  if (!measure || meas.empty() || diag) {
    // gates from the structure cache, diagonal terms appended to its last stage
    // (the combined plan cached under the circuit and the terms)
    auto gp = gate_plan(ctx, c, c128, init, store_final, rc);
    if (!gp) return nullptr;
    if (meas.empty() && cst == 0.0) return gp;
    const int dextra = 0x700 | c128 | (init << 1) | (store_final << 2) | (measure << 3);
    const std::string dkey = structure_key(c, terms, dextra);
    if (auto p = cache_get(ctx, dkey)) return p;
    auto dp = std::make_shared<DevPlan>();
    dp->plan = gp->plan;
    append_diag_measure(dp->plan, meas);
    dp->plan.const_term = cst;
    hipError_t e = dp->upload(ctx->mock);
    if (e != hipSuccess) {
      rc = hip_fail(ctx, e, "plan upload");
      return nullptr;
    }
    cache_put(ctx, dkey, dp);
    return dp;
  }
  const int extra = 0x100 | c128 | (init << 1) | (store_final << 2) | (measure << 3);
  const std::string key = structure_key(c, terms, extra);
  if (auto p = cache_get(ctx, key)) return p;
  auto dp = std::make_shared<DevPlan>();
  std::vector<PGate> pg;
  forward_pgates(c, true, pg, dp->plan.slots);
  PlanOptions o = fwd_options(ctx->opt, c128);
  o.init = init;
  o.store_final = store_final;
  std::string err;
  if (plan_forward(c.n, pg, meas, o, dp->plan, err)) {
    set_error(ctx, err);
    rc = QSIM_EINVAL;
    return nullptr;
  }
  dp->plan.const_term = cst;
  hipError_t e = dp->upload(ctx->mock);
  if (e != hipSuccess) {
    rc = hip_fail(ctx, e, "plan upload");
    return nullptr;
  }
  cache_put(ctx, key, dp);
  return dp;
}

std::shared_ptr<DevPlan> get_grad_plans(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms,
                                        int c128, std::shared_ptr<DevPlan>& happly, int& rc) {
  rc = QSIM_OK;
  const PlanOptions o = dual_options(ctx->opt, c128);
  // lambda = H psi
  {
    CircuitDesc shape;
    shape.n = c.n;
    const std::string key = structure_key(shape, terms, 0x300 | c128);
    happly = cache_get(ctx, key);
    if (!happly) {
      auto dp = std::make_shared<DevPlan>();
      std::vector<PGate> ht;
      double cst = 0;
      term_pgates(terms, true, ht, cst);
      // identity terms: lambda gets c * psi as a diagonal term with an empty mask
      if (cst != 0.0) {
        PGate p;
        p.kind = PG_H_Z;
        p.c = cst;
        ht.push_back(p);
      }
      std::string err;
      if (plan_happly(c.n, ht, o, dp->plan, err)) {
        set_error(ctx, err);
        rc = QSIM_EINVAL;
        return nullptr;
      }
      hipError_t e = dp->upload(ctx->mock);
      if (e != hipSuccess) {
        rc = hip_fail(ctx, e, "plan upload");
        return nullptr;
      }
      cache_put(ctx, key, dp);
      happly = dp;
    }
  }
  return get_adjoint_plan(ctx, c, c128, rc);
}

std::shared_ptr<DevPlan> get_adjoint_plan(qsim_ctx* ctx, const CircuitDesc& c, int c128, int& rc) {
  rc = QSIM_OK;
  const PlanOptions o = dual_options(ctx->opt, c128);
  const std::string key = structure_key(c, {}, 0x200 | c128);
  if (auto p = cache_get(ctx, key)) return p;
  auto dp = std::make_shared<DevPlan>();
  std::vector<PGate> pg;
  std::vector<int> gsp;
  adjoint_pgates(c, pg, dp->plan.slots, gsp);
  std::string err;
  if (plan_adjoint(c.n, pg, o, dp->plan, err)) {
    set_error(ctx, err);
    rc = QSIM_EINVAL;
    return nullptr;
  }
  hipError_t e = dp->upload(ctx->mock);
  if (e != hipSuccess) {
    rc = hip_fail(ctx, e, "plan upload");
    return nullptr;
  }
  cache_put(ctx, key, dp);
  return dp;
}

PlanOptions cone_grad_options(const qsim_options& co, int c128) {
  PlanOptions o = dual_options(co, c128);
  o.r = 4;  // the cone kernel keeps 16 amplitudes per thread and state
  o.init_factors = false;  // every cone starts from |0...0> (its slots are shared between cones)
  o.relabel = false;       // cone sub-states keep their qubit order
  o.early_terms = false;
  return o;
}

// Shared state while packing cones into one plan.  In gradient mode every cone
// runs forward (measuring its observable with coefficient 1), lambda = P psi,
// then the adjoint sweep; cone values are weighted on the device afterwards.
struct ConePacker {
  DevPlan& dp;
  const CircuitDesc& c;
  PlanOptions base;
  int cap;
  bool grad;
  std::vector<int> relabel;
  // shared coefficient table: (kind, inverse, source gates) -> slot
  std::map<std::tuple<int, bool, std::vector<int>>, int> slot_id;
  ConePacker(DevPlan& d, const CircuitDesc& cc, const qsim_options& co, int c128, int cap_, bool grad_ = false)
      : dp(d), c(cc), base(grad_ ? cone_grad_options(co, c128) : cone_options(co, c128)), cap(cap_), grad(grad_),
        relabel(cc.n, -1) {}

  // Appends a sub-plan's passes, stages and ops to the packed plan; its
  // coefficient slots go through the shared table, its gradient slots are
  // renumbered after the ones already packed and tagged with 'cone'.
  void append(const Plan& cp, const std::vector<PGate>& slots, int cone) {
    Plan& all = dp.plan;
    const int sb = (int)all.stages.size(), ob = (int)all.ops.size(), gb = all.n_gslots;
    for (PassDesc pd : cp.passes) {
      pd.stage_begin += sb;
      pd.stage_end += sb;
      if (pd.store_stage >= 0) pd.store_stage += sb;
      pd.grad_begin += gb;
      all.passes.push_back(pd);
    }
    for (StageDesc st : cp.stages) {
      st.op_begin += ob;
      st.op_end += ob;
      all.stages.push_back(st);
    }
    const size_t first_new_stage = all.stages.size() - cp.stages.size();
    std::vector<int> remap(slots.size(), -1);
    for (size_t k = 0; k < slots.size(); ++k) {
      if (remap[k] >= 0) continue;
      if (slots[k].kind == PG_TAB) {
        // a table block: kTabSlots consecutive chunks whose sources are member
        // slots (listed earlier); kept consecutive, shared by member slots
        std::vector<int> mem;
        for (int m : slots[k].srcs) mem.push_back(m >= 0 ? remap[m] : -1);
        auto key = std::make_tuple((int)PG_TAB, false, mem);
        auto it = slot_id.find(key);
        if (it == slot_id.end()) {
          it = slot_id.emplace(key, (int)all.slots.size()).first;
          for (int chunk = 0; chunk < kTabSlots; ++chunk) {
            PGate t = slots[k + chunk];
            t.srcs = mem;
            t.slot = (int)all.slots.size();
            all.slots.push_back(t);
          }
        }
        for (int chunk = 0; chunk < kTabSlots; ++chunk) remap[k + chunk] = it->second + chunk;
        continue;
      }
      auto key = std::make_tuple(slots[k].kind, slots[k].inverse, slots[k].srcs);
      auto it = slot_id.find(key);
      if (it == slot_id.end()) {
        it = slot_id.emplace(key, (int)all.slots.size()).first;
        all.slots.push_back(slots[k]);
      }
      remap[k] = it->second;
    }
    for (size_t k = 0; k < cp.ops.size(); ++k) {
      DevOp op = cp.ops[k];
      if (op.type == OP_U || op.type == OP_RY || op.type == OP_PHASE || op.type == OP_UTAB || op.type == OP_DTAB ||
          (op.type == OP_PTAB && op.slot >= 0))
        op.slot = remap[op.slot];
      if (op.type == OP_GRAD_X || op.type == OP_GRAD_Y || op.type == OP_GRAD_Z) op.slot += gb;
      all.ops.push_back(op);
      if (op.type == OP_GZS || op.type == OP_GXYS)  // probe records: gradient slots
        for (int t = 0; t < op.slot; ++t) {
          DevOp rec = cp.ops[++k];
          rec.slot += gb;
          all.ops.push_back(rec);
        }
      if (op.type == OP_PTAB)  // phase records: coefficient slots
        for (int t = 0; t < (int)op.j; ++t) {
          DevOp rec = cp.ops[++k];
          rec.slot = remap[rec.slot];
          all.ops.push_back(rec);
        }
    }
    // a stage header names its trailing factored group's slot: follow the remap
    for (size_t k = first_new_stage; k < all.stages.size(); ++k) {
      StageDesc& st = all.stages[k];
      if (st.flags & SF_LAST_UTAB) st.flags = (st.flags & 0xffu) | ((uint32_t)remap[st.flags >> 8] << 8);
    }
    for (int g = 0; g < cp.n_gslots; ++g) {
      all.gslot_param.push_back(cp.gslot_param[g]);
      dp.g_cone.push_back(cone);
    }
    all.n_gslots += cp.n_gslots;
    dp.cone_m_max = std::max(dp.cone_m_max, cp.m);
  }

  // Adds one cone evaluating coefficient * <obs> on the gates not in 'skip'
  // (gradient mode: <obs> alone); returns QSIM_OK or an error code (message in err).
  int add(const Term& obs, const std::vector<char>* skip, std::string& err) {
    Plan& all = dp.plan;
    std::vector<int> support, set, gates;
    for (auto [q, L] : obs.ops) support.push_back(q);
    light_cone(c, support, set, gates, skip);
    const int s = (int)set.size();
    if (s > cap) {
      err = "light cone of " + std::to_string(s) + " qubits exceeds the cap of " + std::to_string(cap);
      return QSIM_ETOOBIG;
    }
    const int s_eff = std::max(s, 4);  // the cone kernel holds 16 amplitudes per thread
    for (int k = 0; k < s; ++k) relabel[set[k]] = k;
    CircuitDesc sub;
    sub.n = s_eff;
    sub.n_params = c.n_params;
    for (int g : gates) {
      Gate x = c.gates[g];
      x.q0 = relabel[x.q0];
      if (x.kind == G_CZ || x.kind == G_CNOT) x.q1 = relabel[x.q1];
      sub.gates.push_back(x);
    }
    auto to_circuit_gates = [&](std::vector<PGate>& v) {
      for (PGate& p : v)
        for (int& src : p.srcs) src = gates[src];
    };
    std::vector<PGate> pg, slots, meas, hterms;
    forward_pgates(sub, true, pg, slots);
    to_circuit_gates(pg);
    to_circuit_gates(slots);
    Term unit = obs;
    if (grad) unit.c = 1.0;
    double cst = 0;
    term_pgates({unit}, false, meas, cst, &relabel);
    if (grad) term_pgates({unit}, true, hterms, cst, &relabel);
    for (int k = 0; k < s; ++k) relabel[set[k]] = -1;
    PlanOptions o = base;
    o.init = true;
    o.store_final = grad;
    Plan cp;
    cp.slots = slots;  // factored groups append their table blocks after these
    if (plan_forward(s_eff, pg, meas, o, cp, err)) return QSIM_EINVAL;
    const int cone = (int)dp.cones.size();
    ConeDesc cd;
    std::memset(&cd, 0, sizeof(cd));
    cd.pass_begin = (int)all.passes.size();
    cd.coef_begin = 0;
    cd.out_index = cone;
    cd.n = s_eff;
    if (grad || s_eff > cp.m) {  // gradient cones keep psi and lambda between passes
      cd.scratch_off = dp.scratch_amps;
      dp.scratch_amps += (int64_t)(grad ? 2 : 1) << s_eff;
    }
    append(cp, cp.slots, cone);
    if (grad) {
      Plan hp, ap;
      if (plan_happly(s_eff, hterms, base, hp, err)) return QSIM_EINVAL;
      append(hp, {}, cone);
      std::vector<PGate> apg, aslots;
      std::vector<int> gsp;
      adjoint_pgates(sub, apg, aslots, gsp);
      to_circuit_gates(apg);
      to_circuit_gates(aslots);
      ap.slots = aslots;  // table blocks of the adjoint plan are appended after these
      if (plan_adjoint(s_eff, apg, base, ap, err)) return QSIM_EINVAL;
      append(ap, ap.slots, cone);
    }
    cd.pass_end = (int)all.passes.size();
    dp.cones.push_back(cd);
    return QSIM_OK;
  }

  // largest cones first, so the tail of the launch holds the short ones
  void finish() {
    Plan& all = dp.plan;
    dp.order.resize(dp.cones.size());
    for (int i = 0; i < (int)dp.order.size(); ++i) dp.order[i] = i;
    auto nops = [&](const ConeDesc& x) {
      return all.stages[all.passes[x.pass_end - 1].stage_end - 1].op_end -
             all.stages[all.passes[x.pass_begin].stage_begin].op_begin;
    };
    std::stable_sort(dp.order.begin(), dp.order.end(), [&](int a, int b) {
      const ConeDesc &x = dp.cones[a], &y = dp.cones[b];
      if (x.n != y.n) return x.n > y.n;
      return nops(x) > nops(y);
    });
    all.n = c.n;
    all.r = 4;
  }
};

// HBM scratch bytes (only cones above the tile size touch it) and algorithmic
// flops of a cone launch, for its timing record.
static void cone_costs(DevPlan& dp, int c128) {
  dp.cone_bytes = dp.cone_flops = 0;
  for (const PassDesc& pd : dp.plan.passes) {
    if (pd.n > pd.m) dp.cone_bytes += pass_bytes(pd, 1, c128);
    dp.cone_flops += pass_flops_per_amp(dp.plan, pd) * (double)(1ull << pd.n);
  }
}

// Levels of batched passes for canonical cones (complex64): every cone's k-th
// pass in level k, the measuring passes' tile partials laid out cone after
// cone.  Left empty (cones run one workgroup each) when a measuring pass has a
// measurement index above 0.
static void cone_levels(DevPlan& dp) {
  const Plan& P = dp.plan;
  int depth = 0;
  for (const ConeDesc& x : dp.cones) depth = std::max(depth, x.pass_end - x.pass_begin);
  dp.lvl_cone.assign(depth, {});
  dp.lvl_pass.assign(depth, {});
  dp.lvl_part.assign(depth, {});
  int64_t parts = 0;
  for (int ci = 0; ci < (int)dp.cones.size(); ++ci) {
    const ConeDesc& x = dp.cones[ci];
    for (int p = x.pass_begin; p < x.pass_end; ++p) {
      const PassDesc& pd = P.passes[p];
      const int k = p - x.pass_begin;
      int64_t off = -1;
      if (pd.flags & PF_MEASURE) {
        if (pd.meas_index != 0) {
          dp.lvl_cone.clear();
          dp.lvl_pass.clear();
          dp.lvl_part.clear();
          dp.n_parts = 0;
          return;
        }
        off = parts;
        parts += 1ll << (pd.n - pd.m);
      }
      dp.lvl_cone[k].push_back(ci);
      dp.lvl_pass[k].push_back(p);
      dp.lvl_part[k].push_back(off);
    }
  }
  dp.n_parts = parts;
}

std::shared_ptr<DevPlan> get_cone_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms, int c128,
                                       int& rc) {
  rc = QSIM_OK;
  const std::string key = structure_key(c, terms, 0x400 | c128);
  if (auto p = cache_get(ctx, key)) return p;
  auto dp = std::make_shared<DevPlan>();
  ConePacker pk(*dp, c, ctx->opt, c128, ctx->opt.cone_cap > 0 ? ctx->opt.cone_cap : 20);
  for (const Term& t : terms) {
    if (t.ops.empty()) {
      dp->plan.const_term += t.c;
      continue;
    }
    std::string err;
    if ((rc = pk.add(t, nullptr, err)) != QSIM_OK) {
      set_error(ctx, err);
      return nullptr;
    }
  }
  pk.finish();
  cone_costs(*dp, c128);
  if (!c128) cone_levels(*dp);
  hipError_t e = dp->upload(ctx->mock);
  if (e != hipSuccess) {
    rc = hip_fail(ctx, e, "plan upload");
    return nullptr;
  }
  cache_put(ctx, key, dp);
  return dp;
}

std::shared_ptr<DevPlan> get_factor_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms,
                                         int c128, int& rc, bool grad, bool split) {
  rc = QSIM_OK;
  const std::string key = structure_key(c, terms, 0x600 | c128 | (grad ? 2 : 0) | (split ? 0 : 4));
  if (auto p = cache_get(ctx, key)) return p;
  auto dp = std::make_shared<DevPlan>();
  dp->factored = true;
  dp->cone_grad = grad;
  ConePacker pk(*dp, c, ctx->opt, c128, ctx->opt.cone_cap > 0 ? ctx->opt.cone_cap : 20, grad);
  const std::vector<char> drop = trailing_diagonal(c);
  std::map<std::vector<int>, int> factor_id;  // (pruned flag, qubit*4 + letter ...) -> cone
  auto factor = [&](const Term& obs, bool pruned, std::string& err, int& id) {
    std::vector<int> k{pruned ? 1 : 0};
    for (auto [q, L] : obs.ops) k.push_back(q * 4 + (L == 'X' ? 1 : L == 'Y' ? 2 : 3));
    auto it = factor_id.find(k);
    if (it != factor_id.end()) {
      id = it->second;
      return QSIM_OK;
    }
    id = (int)dp->cones.size();
    const int r = pk.add(obs, pruned ? &drop : nullptr, err);
    if (r == QSIM_OK) factor_id.emplace(k, id);
    return r;
  };
  dp->t_off.push_back(0);
  for (const Term& t : terms) {
    if (t.ops.empty()) {
      dp->plan.const_term += t.c;
      continue;
    }
    bool zstring = split;
    for (auto [q, L] : t.ops) zstring &= L == 'Z';
    std::string err;
    std::vector<std::vector<std::pair<int, char>>> parts;
    if (!zstring) {
      parts.push_back(t.ops);  // the whole term on its canonical cone
    } else {
      // pruned cone of each qubit; qubits whose cones meet share a factor
      const int k = (int)t.ops.size();
      std::vector<std::vector<int>> sets(k);
      for (int i = 0; i < k; ++i) {
        std::vector<int> gs;
        light_cone(c, {t.ops[i].first}, sets[i], gs, &drop);
      }
      std::vector<int> root(k);
      for (int i = 0; i < k; ++i) root[i] = i;
      std::function<int(int)> find = [&](int x) { return root[x] == x ? x : root[x] = find(root[x]); };
      for (int i = 0; i < k; ++i)
        for (int j = i + 1; j < k; ++j) {
          std::vector<int> inter;
          std::set_intersection(sets[i].begin(), sets[i].end(), sets[j].begin(), sets[j].end(),
                                std::back_inserter(inter));
          if (!inter.empty()) root[find(i)] = find(j);
        }
      std::map<int, std::vector<std::pair<int, char>>> groups;
      for (int i = 0; i < k; ++i) groups[find(i)].push_back(t.ops[i]);
      for (auto& g : groups) {
        std::sort(g.second.begin(), g.second.end());
        parts.push_back(g.second);
      }
    }
    for (auto& ops : parts) {
      Term f;
      f.c = 1.0;
      f.ops = ops;
      int id = 0;
      if ((rc = factor(f, zstring, err, id)) != QSIM_OK) {
        set_error(ctx, err);
        return nullptr;
      }
      dp->t_fac.push_back(id);
    }
    dp->t_off.push_back((int32_t)dp->t_fac.size());
    dp->t_coef.push_back(t.c);
  }
  if (grad) {  // factor -> terms that use it, in term order
    const int F = (int)dp->cones.size(), T = (int)dp->t_coef.size();
    dp->f_off.assign(F + 1, 0);
    for (int32_t f : dp->t_fac) dp->f_off[f + 1]++;
    for (int f = 0; f < F; ++f) dp->f_off[f + 1] += dp->f_off[f];
    std::vector<int32_t> fill(dp->f_off.begin(), dp->f_off.end() - 1);
    dp->f_terms.resize(dp->t_fac.size());
    for (int t = 0; t < T; ++t)
      for (int k = dp->t_off[t]; k < dp->t_off[t + 1]; ++k) dp->f_terms[fill[dp->t_fac[k]]++] = t;
  }
  pk.finish();
  cone_costs(*dp, c128);
  hipError_t e = dp->upload(ctx->mock);
  if (e != hipSuccess) {
    rc = hip_fail(ctx, e, "plan upload");
    return nullptr;
  }
  cache_put(ctx, key, dp);
  return dp;
}

// ---------------------------------------------------------------------------
// runs
// ---------------------------------------------------------------------------

// Coefficient rows of a plan's slots: built on the host from host parameters and
// uploaded, or built on the device from device parameters (the circuit's gate
// table is uploaded when it differs from the last one).
// Slots x rows from which coefficient rows of host parameters are built on the device.
constexpr size_t kDeviceCoefSlots = 512;

static int stage_coefficients(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c,
                              const ParamSrc& params, int rows, int c128, hipStream_t st, int64_t& crs) {
  const std::vector<PGate>& slots = dp.plan.slots;
  const size_t scal = c128 ? 8 : 4;
  crs = (int64_t)std::max<size_t>(1, slots.size()) * 8;
  const size_t bytes = (size_t)rows * crs * scal;
  HIP_TRY(ws.coef.ensure(bytes), "coefficient buffer");
  // many slots: the parameters go to the device and the rows are built there
  // (the same definition as on the host, bit for bit)
  const double* dev_params = params.dev ? params.p : nullptr;
  if (!params.dev && params.p && c.n_params > 0 && slots.size() * (size_t)rows >= kDeviceCoefSlots) {
    const size_t pb = (size_t)rows * c.n_params * sizeof(double);
    HIP_TRY(ws.params.ensure(pb), "parameter buffer");
    HIP_TRY(ws.h_params.ensure(pb), "pinned parameter buffer");
    std::memcpy(ws.h_params.p, params.p, pb);
    HIP_TRY(hipMemcpyAsync(ws.params.p, ws.h_params.p, pb, hipMemcpyHostToDevice, st), "parameter upload");
    dev_params = (const double*)ws.params.p;
  }
  if (dev_params) {
    if (slots.empty()) return QSIM_OK;
    std::vector<CoefGate> gt;
    coef_gate_table(c, gt);
    const size_t gbytes = std::max<size_t>(1, gt.size()) * sizeof(CoefGate);
    const bool same = ws.gates.p && ws.last_gates.size() == gt.size() &&
                      (gt.empty() || std::memcmp(ws.last_gates.data(), gt.data(), gt.size() * sizeof(CoefGate)) == 0);
    if (!same) {
      HIP_TRY(ws.gates.ensure(gbytes), "gate table");
      HIP_TRY(ws.h_gates.ensure(gbytes), "pinned gate table");
      if (!gt.empty()) {
        std::memcpy(ws.h_gates.p, gt.data(), gt.size() * sizeof(CoefGate));
        HIP_TRY(hipMemcpyAsync(ws.gates.p, ws.h_gates.p, gt.size() * sizeof(CoefGate), hipMemcpyHostToDevice, st),
                "gate table upload");
      }
      ws.last_gates.swap(gt);
    }
    HIP_TRY(launch_build_coef(dp.d_cslots, (int)slots.size(), dp.d_csrcs, (const CoefGate*)ws.gates.p, dev_params,
                              c.n_params, rows, ws.coef.p, crs, c128, st),
            "coefficient build");
    return QSIM_OK;
  }
  HIP_TRY(ws.h_coef.ensure(bytes), "pinned coefficient buffer");
  if (c128) build_coefficients<double>(c, slots, params.p, rows, crs, (double*)ws.h_coef.p);
  else build_coefficients<float>(c, slots, params.p, rows, crs, (float*)ws.h_coef.p);
  HIP_TRY(hipMemcpyAsync(ws.coef.p, ws.h_coef.p, bytes, hipMemcpyHostToDevice, st), "coefficient upload");
  return QSIM_OK;
}

static int fetch_out(qsim_ctx* ctx, Workspace& ws, size_t count, hipStream_t st, double* out_host) {
  HIP_TRY(ws.h_out.ensure(count * sizeof(double)), "pinned result buffer");
  HIP_TRY(hipMemcpyAsync(ws.h_out.p, ws.out.p, count * sizeof(double), hipMemcpyDeviceToHost, st), "result copy");
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  timing_collect(ctx);
  std::memcpy(out_host, ws.h_out.p, count * sizeof(double));
  return QSIM_OK;
}

int coef_rows(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c, const ParamSrc& params, int rows,
              int c128, hipStream_t st, void* out_host, uint64_t cap, uint64_t* bytes) {
  int64_t crs = 8;
  const uint64_t need = (uint64_t)rows * (uint64_t)std::max<size_t>(1, dp.plan.slots.size()) * 8 * (c128 ? 8 : 4);
  *bytes = need;
  if (need > cap) return QSIM_ETOOBIG;
  int rc = stage_coefficients(ctx, ws, dp, c, params, rows, c128, st, crs);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(out_host, ws.coef.p, need, hipMemcpyDeviceToHost, st), "coefficient copy");
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  return QSIM_OK;
}

int enqueue_dense_passes(qsim_ctx* ctx, const Plan& P, const DenseBufs& b, int rows, int c128, void* A, void* B,
                         hipStream_t st, bool timed) {
  for (size_t p = 0; p < P.passes.size(); ++p) {
    PassLaunch L;
    L.d_pass = b.passes + p;
    L.h_pass = &P.passes[p];
    L.d_stages = b.stages;
    L.d_ops = b.ops;
    L.A = A;
    L.B = B;
    L.row_stride = 1ll << P.n;
    L.coef = b.coef;
    L.coef_row_stride = b.coef_row_stride;
    L.meas = b.meas;
    L.n_meas = P.n_meas;
    L.grad = nullptr;
    L.n_gslots = 0;
    L.rows = rows;
    L.c128 = c128;
    L.dual = 0;
    L.prefetch = prefetch_on(ctx->opt);
    const int ti = timed ? timing_begin(ctx, st, pass_bytes(P.passes[p], rows, c128), P.passes[p].flags, 0,
                                        pass_flops_per_amp(P, P.passes[p]) * (double)rows * (double)(1ull << P.n))
                         : -1;
    HIP_TRY(launch_pass(L, st), "pass launch");
    if (timed) timing_end(ctx, ti, st);
  }
  return QSIM_OK;
}

// Sums of rows x per_row partials (plus add) written by the reduction kernel
// straight into the pinned result buffer (device-visible host memory), so the
// call ends with one stream synchronisation and no device-to-host copy.
static int reduce_to_host(qsim_ctx* ctx, Workspace& ws, const double* part, int rows, int64_t per_row, double add,
                          hipStream_t st, double* out_host) {
  HIP_TRY(ws.h_out.ensure((size_t)rows * sizeof(double)), "pinned result buffer");
  double* dres = nullptr;
  HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&dres), ws.h_out.p, 0), "pinned result address");
  HIP_TRY(launch_reduce_rows(part, rows, per_row, add, dres, st), "reduce launch");
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  timing_collect(ctx);
  std::memcpy(out_host, ws.h_out.p, (size_t)rows * sizeof(double));
  return QSIM_OK;
}

int run_dense(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c, const ParamSrc& params, int rows,
              int c128, void* A, void* B, hipStream_t st, double* out_host) {
  const Plan& P = dp.plan;
  int64_t crs = 8;
  int rc = stage_coefficients(ctx, ws, dp, c, params, rows, c128, st, crs);
  if (rc) return rc;
  const int64_t tiles = 1ll << (P.n - P.m);
  if (P.n_meas > 0) HIP_TRY(ws.meas.ensure((size_t)rows * P.n_meas * tiles * sizeof(double)), "partials buffer");
  const DenseBufs bufs{dp.d_passes, dp.d_stages, dp.d_ops, ws.coef.p, crs, (double*)ws.meas.p};
  if ((rc = enqueue_dense_passes(ctx, P, bufs, rows, c128, A, B, st, true))) return rc;
  if (out_host) {
    if (P.n_meas == 0) {
      HIP_TRY(hipStreamSynchronize(st), "stream sync");
      timing_collect(ctx);
      for (int r = 0; r < rows; ++r) out_host[r] = P.const_term;
      return QSIM_OK;
    }
    return reduce_to_host(ctx, ws, (const double*)ws.meas.p, rows, (int64_t)P.n_meas * tiles, P.const_term, st,
                          out_host);
  }
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  timing_collect(ctx);
  return QSIM_OK;
}

int run_grad(qsim_ctx* ctx, Workspace& ws, const DevPlan& hp, const DevPlan& ap, const CircuitDesc& c,
             const ParamSrc& params, int rows, int c128, void* A, void* B, hipStream_t st, double* grad_host) {
  const Plan& H = hp.plan;
  const Plan& P = ap.plan;
  int64_t crs = 8;
  int rc = stage_coefficients(ctx, ws, ap, c, params, rows, c128, st, crs);
  if (rc) return rc;
  auto mk = [&](const DevPlan& d, size_t p) {
    PassLaunch L;
    L.d_pass = d.d_passes + p;
    L.h_pass = &d.plan.passes[p];
    L.d_stages = d.d_stages;
    L.d_ops = d.d_ops;
    L.A = A;
    L.B = B;
    L.row_stride = 1ll << d.plan.n;
    L.coef = ws.coef.p;
    L.coef_row_stride = crs;
    L.meas = nullptr;
    L.n_meas = 0;
    L.grad = (double*)ws.grad.p;
    L.n_gslots = d.plan.n_gslots;
    L.rows = rows;
    L.c128 = c128;
    L.dual = 1;
    L.prefetch = env_int("QSIM_DUAL_PF", 1);
    return L;
  };
  const int64_t tiles = 1ll << (P.n - P.m);
  const int ns = P.n_gslots;
  if (ns > 0) HIP_TRY(ws.grad.ensure((size_t)rows * ns * tiles * sizeof(double)), "gradient partials");
  const double amps = (double)rows * (double)(1ull << P.n);
  for (size_t p = 0; p < H.passes.size(); ++p) {
    const int ti = timing_begin(ctx, st, pass_bytes(H.passes[p], rows, c128), H.passes[p].flags, 0,
                                pass_flops_per_amp(H, H.passes[p], true) * amps);
    HIP_TRY(launch_pass(mk(hp, p), st), "H-apply launch");
    timing_end(ctx, ti, st);
  }
  for (size_t p = 0; p < P.passes.size(); ++p) {
    const int ti = timing_begin(ctx, st, pass_bytes(P.passes[p], rows, c128), P.passes[p].flags, 0,
                                pass_flops_per_amp(P, P.passes[p], true) * amps);
    HIP_TRY(launch_pass(mk(ap, p), st), "adjoint launch");
    timing_end(ctx, ti, st);
  }
  const int np = c.n_params;
  if (np == 0) {
    HIP_TRY(hipStreamSynchronize(st), "stream sync");
    timing_collect(ctx);
    return QSIM_OK;
  }
  if (ns == 0) {
    HIP_TRY(hipStreamSynchronize(st), "stream sync");
    timing_collect(ctx);
    std::memset(grad_host, 0, sizeof(double) * (size_t)rows * np);
    return QSIM_OK;
  }
  HIP_TRY(ws.slot_total.ensure((size_t)rows * ns * sizeof(double)), "slot totals");
  HIP_TRY(launch_reduce_rows((const double*)ws.grad.p, rows * ns, tiles, 0.0, (double*)ws.slot_total.p, st),
          "gradient reduce");
  // parameters that no gate uses keep a zero gradient: CSR covers [0, max used param]
  int np_used = 0;
  for (int p : P.gslot_param) np_used = std::max(np_used, p + 1);
  HIP_TRY(ws.out.ensure((size_t)rows * np * sizeof(double)), "gradient buffer");
  if (np_used == np) {
    HIP_TRY(launch_grad_scatter((const double*)ws.slot_total.p, rows, ns, ap.d_poff, ap.d_pslots, np,
                                (double*)ws.out.p, st),
            "gradient scatter");
    return fetch_out(ctx, ws, (size_t)rows * np, st, grad_host);
  }
  // fewer used parameters than declared: scatter into a [rows][np_used] block, then widen on the host
  HIP_TRY(launch_grad_scatter((const double*)ws.slot_total.p, rows, ns, ap.d_poff, ap.d_pslots, np_used,
                              (double*)ws.out.p, st),
          "gradient scatter");
  std::vector<double> tmp((size_t)rows * np_used);
  rc = fetch_out(ctx, ws, tmp.size(), st, tmp.data());
  if (rc) return rc;
  for (int r = 0; r < rows; ++r) {
    std::memcpy(grad_host + (size_t)r * np, tmp.data() + (size_t)r * np_used, sizeof(double) * np_used);
    std::memset(grad_host + (size_t)r * np + np_used, 0, sizeof(double) * (np - np_used));
  }
  return QSIM_OK;
}

int run_cones(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c, const ParamSrc& params, int c128,
              hipStream_t st, double* out_host, double* terms_host) {
  const Plan& P = dp.plan;
  if (dp.cones.empty()) {
    if (out_host) *out_host = P.const_term;
    return QSIM_OK;
  }
  int64_t crs = 8;
  int rc = stage_coefficients(ctx, ws, dp, c, params, 1, c128, st, crs);
  if (rc) return rc;
  const size_t amp = c128 ? 16 : 8;
  if (dp.scratch_amps > 0) HIP_TRY(ws.scratch.ensure((size_t)dp.scratch_amps * amp), "cone scratch");
  const size_t nc = dp.cones.size();
  HIP_TRY(ws.meas.ensure(nc * sizeof(double)), "cone partials");
  ConeLaunch L;
  L.d_cones = dp.d_cones;
  L.d_order = dp.d_order;
  L.n_cones = (int)nc;
  L.d_passes = dp.d_passes;
  L.d_stages = dp.d_stages;
  L.d_ops = dp.d_ops;
  L.scratch = ws.scratch.p;
  L.coef = ws.coef.p;
  L.out = (double*)ws.meas.p;
  L.grad = nullptr;
  L.m_max = dp.cone_m_max;
  L.r = 4;
  L.c128 = c128;
  L.dual = 0;
  if (!dp.factored && !terms_host && !c128 && !dp.lvl_pass.empty()) {
    // every cone's k-th pass in one launch, its tiles spread over workgroups;
    // E = the sum of all measuring tiles' partials
    HIP_TRY(ws.slot_total.ensure(std::max<int64_t>(1, dp.n_parts) * sizeof(double)), "cone tile partials");
    const float* cf = (const float*)ws.coef.p;
    if (ws.items_uid != dp.uid || ws.items_coef != ws.coef.p || ws.items_scratch != ws.scratch.p ||
        ws.items_parts != ws.slot_total.p) {
      std::vector<PassItem> items;
      ws.items_lvl_begin.clear();
      ws.items_lvl_tiles.clear();
      ws.items_lvl_m.clear();
      for (size_t k = 0; k < dp.lvl_pass.size(); ++k) {
        ws.items_lvl_begin.push_back((int64_t)items.size());
        int64_t tiles = 0;
        int mm = 0;
        for (size_t i = 0; i < dp.lvl_pass[k].size(); ++i) {
          const ConeDesc& x = dp.cones[dp.lvl_cone[k][i]];
          const int p = dp.lvl_pass[k][i];
          const PassDesc& pd = P.passes[p];
          PassItem it;
          it.pass = dp.d_passes + p;
          it.stages = dp.d_stages;
          it.ops = dp.d_ops;
          it.A = (char*)ws.scratch.p + (size_t)x.scratch_off * amp;
          it.B = nullptr;
          it.coef = cf + (int64_t)x.coef_begin * 8;
          it.meas = dp.lvl_part[k][i] >= 0 ? (double*)ws.slot_total.p + dp.lvl_part[k][i] : nullptr;
          it.grad = nullptr;
          it.tile_begin = tiles;
          tiles += 1ll << (pd.n - pd.m);
          mm = std::max(mm, (int)pd.m);
          items.push_back(it);
        }
        ws.items_lvl_tiles.push_back(tiles);
        ws.items_lvl_m.push_back(mm);
      }
      ws.items_lvl_begin.push_back((int64_t)items.size());
      HIP_TRY(ws.items.ensure(items.size() * sizeof(PassItem)), "cone items");
      HIP_TRY(hipMemcpy(ws.items.p, items.data(), items.size() * sizeof(PassItem), hipMemcpyHostToDevice),
              "cone items upload");
      ws.items_uid = dp.uid;
      ws.items_coef = ws.coef.p;
      ws.items_scratch = ws.scratch.p;
      ws.items_parts = ws.slot_total.p;
    }
    const int ti = timing_begin(ctx, st, dp.cone_bytes, 0, 1, dp.cone_flops);
    for (size_t k = 0; k + 1 < ws.items_lvl_begin.size(); ++k) {
      const int64_t b = ws.items_lvl_begin[k], e = ws.items_lvl_begin[k + 1];
      HIP_TRY(launch_pass_multi((const PassItem*)ws.items.p + b, (int)(e - b), ws.items_lvl_tiles[k],
                                ws.items_lvl_m[k], 4, 0, 0, st),
              "cone pass launch");
    }
    timing_end(ctx, ti, st);
    return reduce_to_host(ctx, ws, (const double*)ws.slot_total.p, 1, dp.n_parts, P.const_term, st, out_host);
  }
  const int ti = timing_begin(ctx, st, dp.cone_bytes, 0, 1, dp.cone_flops);
  HIP_TRY(launch_cones(L, st), "cone launch");
  timing_end(ctx, ti, st);
  HIP_TRY(ws.out.ensure(sizeof(double)), "result buffer");
  if (dp.factored) {  // term values = coefficient x product of its factors, then the sum over terms
    const int T = (int)dp.t_coef.size();
    HIP_TRY(ws.slot_total.ensure(std::max(1, T) * sizeof(double)), "term values");
    HIP_TRY(launch_term_products((const double*)ws.meas.p, dp.d_toff, dp.d_tfac, dp.d_tcoef, T,
                                 (double*)ws.slot_total.p, st),
            "term products");
    if (terms_host) {
      HIP_TRY(ws.out.ensure(std::max(1, T) * sizeof(double)), "result buffer");
      HIP_TRY(hipMemcpyAsync(ws.out.p, ws.slot_total.p, T * sizeof(double), hipMemcpyDeviceToDevice, st),
              "term values copy");
      return fetch_out(ctx, ws, T, st, terms_host);
    }
    return reduce_to_host(ctx, ws, (const double*)ws.slot_total.p, 1, T, P.const_term, st, out_host);
  }
  return reduce_to_host(ctx, ws, (const double*)ws.meas.p, 1, (int64_t)nc, P.const_term, st, out_host);
}

int run_cone_grad(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c, const ParamSrc& params,
                  int c128, hipStream_t st, double* E_host, double* grad_host) {
  const Plan& P = dp.plan;
  const int np = c.n_params, ns = P.n_gslots;
  const size_t nc = dp.cones.size();
  if (nc == 0) {
    *E_host = P.const_term;
    std::memset(grad_host, 0, sizeof(double) * (size_t)np);
    return QSIM_OK;
  }
  int64_t crs = 8;
  int rc = stage_coefficients(ctx, ws, dp, c, params, 1, c128, st, crs);
  if (rc) return rc;
  const size_t amp = c128 ? 16 : 8;
  HIP_TRY(ws.scratch.ensure((size_t)dp.scratch_amps * amp), "cone scratch");
  HIP_TRY(ws.meas.ensure(nc * sizeof(double)), "cone values");
  HIP_TRY(ws.grad.ensure((size_t)std::max(1, ns) * sizeof(double)), "cone gradient slots");
  ConeLaunch L;
  L.d_cones = dp.d_cones;
  L.d_order = dp.d_order;
  L.n_cones = (int)nc;
  L.d_passes = dp.d_passes;
  L.d_stages = dp.d_stages;
  L.d_ops = dp.d_ops;
  L.scratch = ws.scratch.p;
  L.coef = ws.coef.p;
  L.out = (double*)ws.meas.p;
  L.grad = (double*)ws.grad.p;
  L.m_max = dp.cone_m_max;
  L.r = 4;
  L.c128 = c128;
  L.dual = 1;
  double bytes = 0, flops = 0;  // psi and lambda through scratch between a cone's passes
  for (const PassDesc& pd : P.passes) {
    bytes += pass_bytes(pd, 1, c128);
    const bool two = (pd.flags & (PF_LOAD_B | PF_STORE_B | PF_ZERO_B)) != 0;
    flops += pass_flops_per_amp(P, pd, two) * (double)(1ull << pd.n);
  }
  const int ti = timing_begin(ctx, st, bytes, PF_GRAD, 1, flops);
  HIP_TRY(launch_cones(L, st), "gradient cone launch");
  timing_end(ctx, ti, st);
  // E = const + sum_t coef_t prod_f v_f; weights w_f = d<H>/d v_f; grad = sum_slots w g
  int np_used = 0;
  for (int p : P.gslot_param) np_used = std::max(np_used, p + 1);
  const int T = (int)dp.t_coef.size();
  HIP_TRY(ws.slot_total.ensure((size_t)std::max(1, T) * sizeof(double)), "term values");
  HIP_TRY(ws.weights.ensure(nc * sizeof(double)), "factor weights");
  HIP_TRY(ws.out.ensure((size_t)(1 + np_used) * sizeof(double)), "result buffer");
  double* out = (double*)ws.out.p;
  const double* fval = (const double*)ws.meas.p;
  HIP_TRY(launch_term_products(fval, dp.d_toff, dp.d_tfac, dp.d_tcoef, T, (double*)ws.slot_total.p, st),
          "term products");
  HIP_TRY(launch_reduce_rows((const double*)ws.slot_total.p, 1, T, P.const_term, out, st), "term reduce");
  HIP_TRY(launch_factor_weights(fval, dp.d_foff, dp.d_fterms, dp.d_toff, dp.d_tfac, dp.d_tcoef, (int)nc,
                                (double*)ws.weights.p, st),
          "factor weights");
  if (np_used > 0)
    HIP_TRY(launch_weighted_scatter((const double*)ws.grad.p, dp.d_gcone, (const double*)ws.weights.p, dp.d_poff,
                                    dp.d_pslots, np_used, out + 1, st),
            "gradient scatter");
  std::vector<double> tmp((size_t)(1 + np_used));
  if ((rc = fetch_out(ctx, ws, tmp.size(), st, tmp.data()))) return rc;
  *E_host = tmp[0];
  std::memcpy(grad_host, tmp.data() + 1, sizeof(double) * (size_t)np_used);
  std::memset(grad_host + np_used, 0, sizeof(double) * (size_t)(np - np_used));
  return QSIM_OK;
}

}  // namespace qsim
