// Dense <H> evaluation that allocates no memory on the device, for callers
// that cannot call hipMalloc (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).  The same passes as
// qsim_expect_circuit (dense mode, the variant that stores the final state)
// run on a caller-provided state buffer; everything else they need (plan
// descriptors, coefficient rows, partial sums, the results) lives in one
// file-scope device array of fixed size.
#include <cstring>
#include <mutex>
#include <vector>

#include "engine.h"

namespace qsim {
namespace {

constexpr uint64_t kScratchBytes = 64ull << 20;
constexpr uint64_t kAlign = 256;

// Working memory of qsim_expect_circuit_noalloc.  Each GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never uses this name as an address: the device address is taken once per
// device with hipGetSymbolAddress and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_done[kMaxDevices];
void* g_scratch[kMaxDevices];
hipError_t g_err[kMaxDevices];

uint64_t up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Offsets of the regions of one call inside the scratch array.
struct Layout {
  uint64_t passes = 0, stages = 0, ops = 0, cslots = 0, csrcs = 0, gates = 0, coef = 0, meas = 0, out = 0, end = 0;
};

// Waits for the stream on every exit once host buffers have been handed to
// asynchronous copies (they must stay valid until the copies are done).
struct SyncOnExit {
  hipStream_t st;
  bool armed = false;
  ~SyncOnExit() {
    if (armed) (void)hipStreamSynchronize(st);
  }
};

}  // namespace

// Device address of the scratch array on ctx's device (current), taken once
// per device; called by qsim_init for every device context.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_done[device]) {
    void* ptr = nullptr;
    g_err[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch[device] = g_err[device] == hipSuccess ? ptr : nullptr;
    g_done[device] = true;
  }
  return g_err[device];
}

static void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  return g_done[device] ? g_scratch[device] : nullptr;
}

}  // namespace qsim

using namespace qsim;

#define HIP_TRY(expr, where)                               \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

extern "C" int qsim_expect_circuit_noalloc(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch,
                                           int params_on_device, const qsim_hamiltonian* H, int dtype, void* state,
                                           uint64_t state_bytes, void* stream, double* out) {
  if (!ctx || !out || !state || batch < 1 || (dtype != QSIM_C64 && dtype != QSIM_C128)) return QSIM_EINVAL;
  if (ctx->mock) {
    set_error(ctx, "host-only context: no device");
    return QSIM_EDEVICE;
  }
  CircuitDesc cd;
  int rc = to_circuit(ctx, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if ((rc = to_terms(ctx, H, cd.n, terms))) return rc;
  if (cd.n_params > 0 && !params) {
    set_error(ctx, "expect_circuit_noalloc: params missing");
    return QSIM_EINVAL;
  }
  if (cd.n > kMaxQubits) {
    set_error(ctx, "dense mode supports at most 40 qubits");
    return QSIM_ETOOBIG;
  }
  const int c128 = dtype == QSIM_C128;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  unsigned char* base = static_cast<unsigned char*>(scratch_of(ctx->device));
  if (!base) {
    set_error(ctx, std::string("expect_circuit_noalloc: no scratch address for this device: ") +
                       hipGetErrorString(noalloc_setup(ctx->device)));
    return QSIM_EDEVICE;
  }
  hipStream_t st = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;

  // the plan on the host (host memory only; kept per structure in the context)
  const std::string key = structure_key(cd, terms, 0x900 | c128);
  std::shared_ptr<Plan> hold;
  {
    std::lock_guard<std::mutex> pg(ctx->plan_mu);
    auto it = ctx->host_plans.find(key);
    if (it != ctx->host_plans.end()) hold = it->second;
  }
  if (!hold) {
    hold = std::make_shared<Plan>();
    if ((rc = host_dense_plan(ctx, cd, terms, c128, true, true, *hold))) return rc;
    std::lock_guard<std::mutex> pg(ctx->plan_mu);
    if (ctx->host_plans.size() >= 64) ctx->host_plans.clear();
    ctx->host_plans[key] = hold;
  }
  const Plan* P = hold.get();

  // regions of the scratch array
  const size_t scal = c128 ? 8 : 4;
  const int64_t crs = (int64_t)std::max<size_t>(1, P->slots.size()) * 8;
  const uint64_t tiles = 1ull << (P->n - P->m);
  std::vector<CoefSlot> cslots;
  std::vector<int32_t> csrcs;
  std::vector<CoefGate> gates;
  const bool dev_params = params_on_device != 0 && !P->slots.empty();
  if (dev_params) {
    coef_slot_table(P->slots, cslots, csrcs);
    coef_gate_table(cd, gates);
  }
  Layout L;
  L.passes = 0;
  L.stages = up(L.passes + P->passes.size() * sizeof(PassDesc));
  L.ops = up(L.stages + P->stages.size() * sizeof(StageDesc));
  L.cslots = up(L.ops + P->ops.size() * sizeof(DevOp));
  L.csrcs = up(L.cslots + cslots.size() * sizeof(CoefSlot));
  L.gates = up(L.csrcs + csrcs.size() * sizeof(int32_t));
  L.coef = up(L.gates + gates.size() * sizeof(CoefGate));
  L.meas = up(L.coef + (uint64_t)batch * (uint64_t)crs * scal);
  L.out = up(L.meas + (uint64_t)batch * (uint64_t)P->n_meas * tiles * sizeof(double));
  L.end = up(L.out + (uint64_t)batch * sizeof(double));
  if (L.end > kScratchBytes) {
    set_error(ctx, "expect_circuit_noalloc: this call needs " + std::to_string(L.end) +
                       " bytes of working memory; the fixed maximum is " + std::to_string(kScratchBytes) +
                       " (partial sums take batch * measurement passes * 2^(n - m) * 8 bytes)");
    return QSIM_ETOOBIG;
  }
  const uint64_t need_state = (uint64_t)batch * (1ull << cd.n) * (c128 ? 16u : 8u);
  if (state_bytes < need_state) {
    set_error(ctx, "expect_circuit_noalloc: state buffer of " + std::to_string(state_bytes) + " bytes, " +
                       std::to_string(need_state) + " needed");
    return QSIM_EINVAL;
  }

  std::vector<float> hc32;
  std::vector<double> hc64;
  SyncOnExit guard{st};  // declared after every host buffer a copy reads
  auto put = [&](uint64_t off, const void* src, size_t bytes) {
    guard.armed = true;
    return bytes ? hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  HIP_TRY(put(L.passes, P->passes.data(), P->passes.size() * sizeof(PassDesc)), "pass descriptors");
  HIP_TRY(put(L.stages, P->stages.data(), P->stages.size() * sizeof(StageDesc)), "stage descriptors");
  HIP_TRY(put(L.ops, P->ops.data(), P->ops.size() * sizeof(DevOp)), "op descriptors");
  if (dev_params) {
    HIP_TRY(put(L.cslots, cslots.data(), cslots.size() * sizeof(CoefSlot)), "slot table");
    HIP_TRY(put(L.csrcs, csrcs.data(), csrcs.size() * sizeof(int32_t)), "slot sources");
    HIP_TRY(put(L.gates, gates.data(), gates.size() * sizeof(CoefGate)), "gate table");
    HIP_TRY(launch_build_coef(reinterpret_cast<const CoefSlot*>(base + L.cslots), (int)P->slots.size(),
                              reinterpret_cast<const int32_t*>(base + L.csrcs),
                              reinterpret_cast<const CoefGate*>(base + L.gates), params, cd.n_params, batch,
                              base + L.coef, crs, c128, st),
            "coefficient build");
  } else if (c128) {
    hc64.assign((size_t)batch * crs, 0.0);
    build_coefficients<double>(cd, P->slots, params, batch, crs, hc64.data());
    HIP_TRY(put(L.coef, hc64.data(), hc64.size() * sizeof(double)), "coefficient rows");
  } else {
    hc32.assign((size_t)batch * crs, 0.0f);
    build_coefficients<float>(cd, P->slots, params, batch, crs, hc32.data());
    HIP_TRY(put(L.coef, hc32.data(), hc32.size() * sizeof(float)), "coefficient rows");
  }
  // every partial-sum entry is written by its tile before it is read, and the
  // rows and descriptors are copied in full: nothing needs clearing
  const DenseBufs bufs{reinterpret_cast<const PassDesc*>(base + L.passes),
                       reinterpret_cast<const StageDesc*>(base + L.stages),
                       reinterpret_cast<const DevOp*>(base + L.ops), base + L.coef, crs,
                       reinterpret_cast<double*>(base + L.meas)};
  guard.armed = true;
  if ((rc = enqueue_dense_passes(ctx, *P, bufs, batch, c128, state, nullptr, st, false))) return rc;
  if (P->n_meas == 0) {
    HIP_TRY(hipStreamSynchronize(st), "stream sync");
    for (int r = 0; r < batch; ++r) out[r] = P->const_term;
    return QSIM_OK;
  }
  double* dout = reinterpret_cast<double*>(base + L.out);
  HIP_TRY(launch_reduce_rows(reinterpret_cast<const double*>(base + L.meas), batch, (int64_t)P->n_meas * (int64_t)tiles,
                             P->const_term, dout, st),
          "reduce launch");
  HIP_TRY(hipMemcpyAsync(out, dout, (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, st), "result copy");
  HIP_TRY(hipStreamSynchronize(st), "stream sync");
  return QSIM_OK;
}
