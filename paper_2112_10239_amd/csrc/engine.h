// Internal engine: device workspaces, cached plans and the evaluation paths
// behind the C-ABI.  Host C++ on the HIP runtime.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.h"
#include "planner.h"
#include "../../include/qsim.h"

namespace qsim {

// A grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) bytes = want;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// A pinned host staging buffer.
struct HostBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e == hipSuccess) bytes = want;
    return e;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// A plan with its device copy.
struct DevPlan {
  Plan plan;
  PassDesc* d_passes = nullptr;
  StageDesc* d_stages = nullptr;
  DevOp* d_ops = nullptr;
  // light-cone / small-circuit batches
  std::vector<ConeDesc> cones;
  std::vector<int32_t> order;
  ConeDesc* d_cones = nullptr;
  int32_t* d_order = nullptr;
  int64_t scratch_amps = 0;
  int cone_m_max = 0;
  // gradient scatter (CSR parameter -> gradient slots)
  int32_t* d_poff = nullptr;
  int32_t* d_pslots = nullptr;
  // coefficient slots for rows built on the device (parameters in device memory)
  CoefSlot* d_cslots = nullptr;
  int32_t* d_csrcs = nullptr;
  // factored light cones: term t = t_coef[t] * prod of cone values t_fac[t_off[t] .. t_off[t+1])
  bool factored = false;
  std::vector<int32_t> t_off, t_fac;
  std::vector<double> t_coef;
  int32_t* d_toff = nullptr;
  int32_t* d_tfac = nullptr;
  double* d_tcoef = nullptr;
  // light-cone gradients: gradient slot -> factor, factor -> terms (CSR)
  bool cone_grad = false;
  std::vector<int32_t> g_cone, f_off, f_terms;
  int32_t* d_gcone = nullptr;
  int32_t* d_foff = nullptr;
  int32_t* d_fterms = nullptr;
  // cone launches: HBM scratch bytes and algorithmic flops (timing records), once per plan
  double cone_bytes = -1, cone_flops = 0;
  // canonical cones as batched passes: level k holds the k-th pass of every
  // cone that has one (each pass split into its tiles across workgroups); the
  // measuring passes write their tile partials at part_off (empty: not batched)
  std::vector<std::vector<int32_t>> lvl_cone, lvl_pass;
  std::vector<std::vector<int64_t>> lvl_part;  // partial offset of the item, -1: none
  int64_t n_parts = 0;
  uint64_t uid = 0;  // distinct per plan object (workspace caches of device pointers)
  DevPlan();
  ~DevPlan();
  hipError_t upload(bool mock);
};

struct Workspace {
  DevBuf coef, meas, grad, slot_total, out, scratch, lambda, weights, table, dens, gates, block, params, items;
  HostBuf h_coef, h_out, h_gates, h_params;
  // batched cone items on the device: plan uid and the buffers they point into
  uint64_t items_uid = 0;
  const void *items_coef = nullptr, *items_scratch = nullptr, *items_parts = nullptr;
  std::vector<int64_t> items_lvl_begin, items_lvl_tiles;
  std::vector<int> items_lvl_m;
  std::vector<CoefGate> last_gates;  // content of 'gates' (device gate table)
  void release() {
    gates.release();
    h_gates.release();
    last_gates.clear();
    coef.release();
    meas.release();
    grad.release();
    slot_total.release();
    out.release();
    scratch.release();
    lambda.release();
    weights.release();
    table.release();
    dens.release();
    block.release();
    h_coef.release();
    h_out.release();
    params.release();
    h_params.release();
    items.release();
    items_uid = 0;
  }
};

class Server;  // serving loop (serve.cpp)

}  // namespace qsim

namespace qsim {
struct TimingRec {
  hipEvent_t a = nullptr, b = nullptr;
  double bytes = 0, ms = 0, flops = 0;
  int flags = 0, kind = 0;
};
}  // namespace qsim

struct qsim_ctx {
  int device = 0;
  bool timing = false;
  std::vector<qsim::TimingRec> tpending, tdone;
  bool mock = false;     // no device: plans only, serving simulates execution (host tests)
  hipStream_t stream = nullptr;
  qsim_options opt{};
  std::mutex api_mu;     // synchronous calls
  std::mutex plan_mu;    // plan cache
  std::unordered_map<std::string, std::shared_ptr<qsim::DevPlan>> plans;  // by structure key
  std::unordered_map<std::string, std::shared_ptr<qsim::Plan>> host_plans;  // host-only plans (no device copy)
  qsim::Workspace ws;
  qsim::DevBuf psi;      // state workspace of qsim_expect_circuit
  std::mutex err_mu;
  std::string err;
  std::unique_ptr<qsim::Server> server;
};

struct qsim_state {
  qsim_ctx* ctx = nullptr;
  int n = 0, batch = 0, dtype = 0;
  void* buf = nullptr;
  bool owned = true;
  bool fresh = true;      // content is |0...0> but not yet written
  hipStream_t stream = nullptr;
  qsim::CircuitDesc queue;          // gates not yet applied
  std::vector<double> qparams;      // [batch][queue.n_params] (host parameters)
  bool qdev = false;                // parameters of the queue are in dparams (device) instead
  qsim::DevBuf dparams;             // [batch][queue.n_params] float64 in device memory
};

namespace qsim {

void set_error(qsim_ctx* ctx, const std::string& msg);
int hip_fail(qsim_ctx* ctx, hipError_t e, const char* where);

// Conversions from the ABI structs.
int to_circuit(qsim_ctx* ctx, const qsim_circuit* c, CircuitDesc& out);
int to_terms(qsim_ctx* ctx, const qsim_hamiltonian* H, int n, std::vector<Term>& out);

// Plan construction (cached).
std::shared_ptr<DevPlan> get_dense_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms,
                                        int c128, bool init, bool store_final, bool measure, int& rc);
std::shared_ptr<DevPlan> get_grad_plans(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms,
                                        int c128, std::shared_ptr<DevPlan>& happly, int& rc);
std::shared_ptr<DevPlan> get_adjoint_plan(qsim_ctx* ctx, const CircuitDesc& c, int c128, int& rc);
// The plan get_dense_plan(..., measure = true) returns, built on the host only
// (no device copy, not cached).
// With 'trace' the plan records its stage trace (Plan::trace).
int host_dense_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms, int c128, bool init,
                    bool store_final, Plan& out, bool trace = false);
// Host-only plans for the serving loop (complex64): the forward plan reuses
// the structure-cached gate plan and appends this H's measurement.
int host_forward_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms, bool store_final,
                      Plan& out);
int host_happly_plan(qsim_ctx* ctx, int n, const std::vector<Term>& terms, Plan& out);
std::shared_ptr<DevPlan> get_cone_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms,
                                       int c128, int& rc);
// Light cones after dropping trailing diagonal gates (Z-string terms) and
// splitting terms into factors with disjoint cones, shared across terms.
// Factored light cones (split = true: Z-string terms split into disjoint pruned
// factors; false: one canonical cone per term).  grad = true packs gradient cones.
std::shared_ptr<DevPlan> get_factor_plan(qsim_ctx* ctx, const CircuitDesc& c, const std::vector<Term>& terms,
                                         int c128, int& rc, bool grad = false, bool split = true);

// Where a call's parameters are: float64 rows [rows][n_params] in host memory,
// or in device memory (coefficient rows are then built on the device).
struct ParamSrc {
  const double* p = nullptr;
  bool dev = false;
  ParamSrc() = default;
  ParamSrc(const double* p_, bool dev_) : p(p_), dev(dev_) {}
  ParamSrc row(int b, int n_params) const { return ParamSrc(p ? p + (size_t)b * n_params : nullptr, dev); }
};

// Device copies of a dense plan's descriptors and the buffers its passes use.
struct DenseBufs {
  const PassDesc* passes;
  const StageDesc* stages;
  const DevOp* ops;
  const void* coef;         // [rows][coef_row_stride] scalars
  int64_t coef_row_stride;
  double* meas;             // [rows][n_meas][tiles] partial sums
};
// Launch every pass of P on states A (and B) on stream st, without synchronising
// (timed: each launch is recorded for qsim_timing_get when timing is on).
int enqueue_dense_passes(qsim_ctx* ctx, const Plan& P, const DenseBufs& b, int rows, int c128, void* A, void* B,
                         hipStream_t st, bool timed);
// Run a dense plan on states A (and B) with 'rows' rows; coefficients from params.
int run_dense(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c, const ParamSrc& params, int rows,
              int c128, void* A, void* B, hipStream_t st, double* out_host);
// The coefficient rows a dense plan's passes read (host- or device-built), copied to host memory.
int coef_rows(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c, const ParamSrc& params, int rows,
              int c128, hipStream_t st, void* out_host, uint64_t cap, uint64_t* bytes);
int run_grad(qsim_ctx* ctx, Workspace& ws, const DevPlan& hp, const DevPlan& ap, const CircuitDesc& c,
             const ParamSrc& params, int rows, int c128, void* A, void* B, hipStream_t st, double* grad_host);
// One cone launch; out_host receives <H> (terms_host == nullptr) or, for a
// factored plan, the value of every non-identity term (terms_host[T']).
int run_cones(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c, const ParamSrc& params, int c128,
              hipStream_t st, double* out_host, double* terms_host = nullptr);
// <H> and its gradient from a gradient cone plan (one parameter row).
int run_cone_grad(qsim_ctx* ctx, Workspace& ws, const DevPlan& dp, const CircuitDesc& c, const ParamSrc& params,
                  int c128, hipStream_t st, double* E_host, double* grad_host);

// Device address of the fixed working memory of qsim_expect_circuit_noalloc on
// 'device' (current), taken once per device; the stored status on later calls.
hipError_t noalloc_setup(int device);

// Launch bracketing for qsim_timing_*: returns the record index or -1.
int timing_begin(qsim_ctx* ctx, hipStream_t st, double bytes, int flags, int kind, double flops = 0);
void timing_end(qsim_ctx* ctx, int idx, hipStream_t st);
void timing_collect(qsim_ctx* ctx);  // after a stream sync

// Tile options per state precision and kernel kind, from a context's options.
PlanOptions fwd_options(const qsim_options& co, int c128);
PlanOptions dual_options(const qsim_options& co, int c128);
PlanOptions cone_options(const qsim_options& co, int c128);
bool prefetch_on(const qsim_options& co);

}  // namespace qsim
