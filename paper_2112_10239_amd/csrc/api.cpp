// The C-ABI of libqsim (declared in include/qsim.h).
#include <algorithm>
#include <array>
#include <cstring>
#include <new>

#include "engine.h"
#include "serve.h"

using namespace qsim;

#define HIP_TRY(expr, where)                                 \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where);   \
  } while (0)

namespace {

size_t amp_bytes(int dtype) { return dtype == QSIM_C128 ? 16 : 8; }

bool valid_dtype(int dtype) { return dtype == QSIM_C64 || dtype == QSIM_C128; }

hipStream_t pick_stream(qsim_ctx* ctx, void* stream) {
  return stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
}

// Apply the state's queued gates; measure terms if given.
int flush(qsim_state* st, const std::vector<Term>* terms, double* out) {
  qsim_ctx* ctx = st->ctx;
  const bool has_gates = !st->queue.gates.empty();
  const bool need_store = has_gates || (st->fresh && !terms);
  if (!has_gates && !terms && !st->fresh) return QSIM_OK;
  st->queue.n = st->n;
  int rc = QSIM_OK;
  auto dp = get_dense_plan(ctx, st->queue, terms ? *terms : std::vector<Term>{}, st->dtype == QSIM_C128, st->fresh,
                           need_store, terms != nullptr, rc);
  if (!dp) return rc;
  const ParamSrc ps = st->qdev ? ParamSrc((const double*)st->dparams.p, true)
                              : ParamSrc(st->qparams.empty() ? nullptr : st->qparams.data(), false);
  rc = run_dense(ctx, ctx->ws, *dp, st->queue, ps, st->batch, st->dtype == QSIM_C128, st->buf, nullptr, st->stream,
                 out);
  if (rc) return rc;
  if (need_store) st->fresh = false;
  st->queue.gates.clear();
  st->queue.n_params = 0;
  st->qparams.clear();
  st->qdev = false;
  return QSIM_OK;
}

int check_state(qsim_state* st) { return (st && st->ctx) ? QSIM_OK : QSIM_EINVAL; }

int no_device(qsim_ctx* ctx) {
  set_error(ctx, "host-only context: no device");
  return QSIM_EDEVICE;
}

}  // namespace

extern "C" {

const char* qsim_strerror(int code) {
  switch (code) {
    case QSIM_OK: return "ok";
    case QSIM_PENDING: return "pending";
    case QSIM_EINVAL: return "invalid argument";
    case QSIM_ENOMEM: return "out of memory";
    case QSIM_ETOOBIG: return "too big for the budget or the light-cone cap";
    case QSIM_EAGAIN: return "queue full, retry";
    case QSIM_ENOTFOUND: return "unknown or consumed ticket";
    case QSIM_EDEVICE: return "device error";
    case QSIM_ECANCELED: return "cancelled";
    case QSIM_ESHUTDOWN: return "shut down";
    default: return "unknown status";
  }
}

const char* qsim_last_error(qsim_ctx* ctx) {
  if (!ctx) return "";
  std::lock_guard<std::mutex> g(ctx->err_mu);
  return ctx->err.c_str();
}

int qsim_init(qsim_ctx** out, const qsim_options* opt) {
  if (!out) return QSIM_EINVAL;
  *out = nullptr;
  qsim_ctx* ctx = new (std::nothrow) qsim_ctx();
  if (!ctx) return QSIM_ENOMEM;
  if (opt) ctx->opt = *opt;
  if (ctx->opt.max_queue <= 0) ctx->opt.max_queue = 4096;
  if (ctx->opt.cone_cap <= 0) ctx->opt.cone_cap = 20;
  if (ctx->opt.hbm_budget_bytes == 0) ctx->opt.hbm_budget_bytes = 64ull << 30;
  if (ctx->opt.max_inflight <= 0) ctx->opt.max_inflight = 3;
  if (ctx->opt.max_inflight > 8) ctx->opt.max_inflight = 8;
  ctx->device = ctx->opt.device;
  if (ctx->device < 0) {  // host-only context: planning and a simulated serving loop
    ctx->mock = true;
    *out = ctx;
    return QSIM_OK;
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= ctx->device || ctx->device < 0) {
    delete ctx;
    return QSIM_EDEVICE;
  }
  if (hipSetDevice(ctx->device) != hipSuccess || hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return QSIM_EDEVICE;
  }
  // address of the allocation-free entry point's working memory on this device;
  // a failure is reported by that entry point, the rest of the library works
  (void)noalloc_setup(ctx->device);
  *out = ctx;
  return QSIM_OK;
}

void qsim_finalize(qsim_ctx* ctx) {
  if (!ctx) return;
  ctx->server.reset();  // stops the scheduler; pending tickets end with QSIM_ESHUTDOWN
  if (ctx->mock) {
    delete ctx;
    return;
  }
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->plans.clear();
  ctx->ws.release();
  ctx->psi.release();
  (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

int qsim_create_state(qsim_ctx* ctx, int n_qubits, int batch, int dtype, void* dev_buf, void* stream,
                      qsim_state** out) {
  if (!ctx || !out) return QSIM_EINVAL;
  *out = nullptr;
  if (ctx->mock) return no_device(ctx);
  if (n_qubits < 1 || n_qubits > kMaxQubits || batch < 1 || !valid_dtype(dtype)) {
    set_error(ctx, "create_state: n_qubits in [1, 40], batch >= 1 and dtype C64/C128 required");
    return QSIM_EINVAL;
  }
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  qsim_state* st = new (std::nothrow) qsim_state();
  if (!st) return QSIM_ENOMEM;
  st->ctx = ctx;
  st->n = n_qubits;
  st->batch = batch;
  st->dtype = dtype;
  st->stream = pick_stream(ctx, stream);
  st->queue.n = n_qubits;
  if (dev_buf) {
    st->buf = dev_buf;
    st->owned = false;
  } else {
    const size_t bytes = (size_t)batch * ((size_t)1 << n_qubits) * amp_bytes(dtype);
    hipError_t e = hipMalloc(&st->buf, bytes);
    if (e != hipSuccess) {
      delete st;
      return hip_fail(ctx, e, "state allocation");
    }
  }
  *out = st;
  return QSIM_OK;
}

int qsim_destroy_state(qsim_state* st) {
  if (!st) return QSIM_EINVAL;
  if (st->ctx) {
    (void)hipSetDevice(st->ctx->device);
    (void)hipStreamSynchronize(st->stream);
  }
  if (st->owned && st->buf) (void)hipFree(st->buf);
  st->dparams.release();
  delete st;
  return QSIM_OK;
}

int qsim_apply_layer(qsim_state* st, const qsim_gate* gates, int n_gates, const double* params, int n_params,
                     int params_on_device) {
  if (check_state(st)) return QSIM_EINVAL;
  qsim_ctx* ctx = st->ctx;
  if (n_gates < 0 || n_params < 0) return QSIM_EINVAL;
  qsim_circuit view{st->n, n_gates, n_params, 0, gates};
  CircuitDesc layer;
  int rc = to_circuit(ctx, &view, layer);
  if (rc) return rc;
  bool uses = false;
  for (const Gate& g : layer.gates) uses |= g.param >= 0;
  if (uses && !params) {
    set_error(ctx, "apply_layer: parameterised gates need params");
    return QSIM_EINVAL;
  }
  std::lock_guard<std::mutex> g(ctx->api_mu);
  const int old = st->queue.n_params;
  const int total = old + n_params;
  const size_t B = (size_t)st->batch;
  if (params_on_device || st->qdev) {
    // the queue's parameters move to (or stay in) device memory: [batch][total]
    HIP_TRY(hipSetDevice(ctx->device), "set device");
    HIP_TRY(hipStreamSynchronize(st->stream), "stream sync");
    DevBuf nb;
    HIP_TRY(nb.ensure(std::max<size_t>(1, B * total) * sizeof(double)), "parameter buffer");
    const size_t w = sizeof(double);
    hipError_t e = hipSuccess;
    if (old > 0)
      e = st->qdev ? hipMemcpy2D(nb.p, total * w, st->dparams.p, old * w, old * w, B, hipMemcpyDeviceToDevice)
                   : hipMemcpy2D(nb.p, total * w, st->qparams.data(), old * w, old * w, B, hipMemcpyHostToDevice);
    if (e == hipSuccess && n_params > 0 && params)
      e = hipMemcpy2D((char*)nb.p + old * w, total * w, params, n_params * w, n_params * w, B,
                      params_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      nb.release();
      return hip_fail(ctx, e, "parameter copy");
    }
    st->dparams.release();
    st->dparams = nb;
    st->qparams.clear();
    st->qdev = true;
  } else {
    std::vector<double> np(B * total);
    for (size_t b = 0; b < B; ++b) {
      for (int k = 0; k < old; ++k) np[b * total + k] = st->qparams[b * old + k];
      for (int k = 0; k < n_params; ++k) np[b * total + old + k] = params[b * n_params + k];
    }
    st->qparams.swap(np);
  }
  for (Gate x : layer.gates) {
    if (x.param >= 0) x.param += old;
    st->queue.gates.push_back(x);
  }
  st->queue.n_params = total;
  return QSIM_OK;
}

int qsim_expect(qsim_state* st, const qsim_hamiltonian* H, double* out) {
  if (check_state(st) || !out) return QSIM_EINVAL;
  qsim_ctx* ctx = st->ctx;
  std::vector<Term> terms;
  int rc = to_terms(ctx, H, st->n, terms);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  return flush(st, &terms, out);
}

int qsim_state_to_host(qsim_state* st, void* host) {
  if (check_state(st) || !host) return QSIM_EINVAL;
  qsim_ctx* ctx = st->ctx;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  int rc = flush(st, nullptr, nullptr);
  if (rc) return rc;
  const size_t bytes = (size_t)st->batch * ((size_t)1 << st->n) * amp_bytes(st->dtype);
  HIP_TRY(hipMemcpyAsync(host, st->buf, bytes, hipMemcpyDeviceToHost, st->stream), "state copy");
  HIP_TRY(hipStreamSynchronize(st->stream), "stream sync");
  return QSIM_OK;
}

int qsim_apply_block5(qsim_state* st, const double* u, int method, double* ms) {
  if (check_state(st) || !u || (method != 0 && method != 1)) return QSIM_EINVAL;
  qsim_ctx* ctx = st->ctx;
  if (st->dtype != QSIM_C64 || st->n < 5) {
    set_error(ctx, "apply_block5: complex64 states of at least 5 qubits");
    return QSIM_EINVAL;
  }
  const int64_t rows = (int64_t)st->batch << (st->n - 5);
  if (method == 0 && rows % 32) {
    set_error(ctx, "apply_block5: the matrix-core kernel needs a multiple of 32 rows (batch * 2^(n-5))");
    return QSIM_EINVAL;
  }
  if (ctx->mock) return no_device(ctx);
  // the block in the form each kernel reads (fp32, rounded once from fp64)
  std::vector<float> w;
  if (method == 0) {
    // W[c][j]: c < 32 real part of input amplitude c, else imaginary part of c - 32;
    // j < 32 real part of output j, else imaginary part of output j - 32
    auto W = [&](int c, int j) -> double {
      const int i = c & 31, o = j & 31;
      const double ur = u[(o * 32 + i) * 2], ui = u[(o * 32 + i) * 2 + 1];
      if (c < 32) return j < 32 ? ur : ui;
      return j < 32 ? -ui : ur;
    };
    w.resize(2 * 32 * 64);
    for (int t = 0; t < 2; ++t)
      for (int s = 0; s < 32; ++s)
        for (int l = 0; l < 64; ++l) {
          const int g = l >> 5;
          const int krow = s < 16 ? g * 16 + s : 32 + g * 16 + (s - 16);
          w[(t * 32 + s) * 64 + l] = (float)W(krow, t * 32 + (l & 31));
        }
  } else {
    w.resize(2048);
    for (int k = 0; k < 2048; ++k) w[k] = (float)u[k];
  }
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  int rc = flush(st, nullptr, nullptr);
  if (rc) return rc;
  Workspace& ws = ctx->ws;
  hipStream_t s = st->stream;
  HIP_TRY(hipStreamSynchronize(s), "stream sync");  // the pinned staging buffer may still feed an upload
  HIP_TRY(ws.block.ensure(w.size() * sizeof(float)), "block buffer");
  HIP_TRY(ws.h_coef.ensure(w.size() * sizeof(float)), "pinned block staging");
  std::memcpy(ws.h_coef.p, w.data(), w.size() * sizeof(float));
  HIP_TRY(hipMemcpyAsync(ws.block.p, ws.h_coef.p, w.size() * sizeof(float), hipMemcpyHostToDevice, s), "block upload");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    HIP_TRY(hipEventRecord(e0, s), "event record");
  }
  const double amps = (double)st->batch * (double)(1ull << st->n);
  const int ti = timing_begin(ctx, s, 16.0 * amps, PF_LOAD_A | PF_STORE_A, 3, 256.0 * amps);
  hipError_t le = launch_block5(st->buf, rows, (const float*)ws.block.p, method, s);
  timing_end(ctx, ti, s);
  if (ms) (void)hipEventRecord(e1, s);
  hipError_t se = hipStreamSynchronize(s);
  timing_collect(ctx);
  if (ms) {
    float t = 0;
    if (le == hipSuccess && se == hipSuccess) (void)hipEventElapsedTime(&t, e0, e1);
    *ms = t;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  HIP_TRY(le, "block launch");
  HIP_TRY(se, "stream sync");
  return QSIM_OK;
}

int qsim_reduced_density(qsim_state* st, const int32_t* qubits, int m, void* rho, int rho_on_device) {
  if (check_state(st) || !qubits || !rho) return QSIM_EINVAL;
  qsim_ctx* ctx = st->ctx;
  const int n = st->n;
  if (m < 1 || m > n || m > 15) {
    set_error(ctx, "reduced_density: need 1 <= m <= min(n, 15) kept qubits");
    return QSIM_EINVAL;
  }
  uint64_t keep_mask = 0;
  for (int a = 0; a < m; ++a) {
    if (qubits[a] < 0 || qubits[a] >= n || ((keep_mask >> qubits[a]) & 1)) {
      set_error(ctx, "reduced_density: kept qubits must be distinct and in [0, n)");
      return QSIM_EINVAL;
    }
    keep_mask |= 1ull << qubits[a];
  }
  if (ctx->mock) return no_device(ctx);
  // offsets (in amplitudes) of the kept index i and of the traced index k = (hi, lo)
  const int64_t N = 1ll << m, K = 1ll << (n - m);
  const int lo_bits = std::min(n - m, 10);
  std::vector<int> traced;
  for (int q = 0; q < n; ++q)
    if (!((keep_mask >> q) & 1)) traced.push_back(q);
  std::vector<int64_t> tab((size_t)(N + (1ll << lo_bits) + (K >> lo_bits)));
  int64_t* off_i = tab.data();
  int64_t* klo = off_i + N;
  int64_t* khi = klo + (1ll << lo_bits);
  for (int64_t i = 0; i < N; ++i) {
    int64_t o = 0;
    for (int a = 0; a < m; ++a) o |= ((i >> a) & 1) << qubits[a];
    off_i[i] = o;
  }
  for (int64_t k = 0; k < (1ll << lo_bits); ++k) {
    int64_t o = 0;
    for (int b = 0; b < lo_bits; ++b) o |= ((k >> b) & 1) << traced[b];
    klo[k] = o;
  }
  for (int64_t k = 0; k < (K >> lo_bits); ++k) {
    int64_t o = 0;
    for (int b = lo_bits; b < n - m; ++b) o |= ((k >> (b - lo_bits)) & 1) << traced[b];
    khi[k] = o;
  }
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  int rc = flush(st, nullptr, nullptr);
  if (rc) return rc;
  Workspace& ws = ctx->ws;
  hipStream_t s = st->stream;
  HIP_TRY(hipStreamSynchronize(s), "stream sync");  // the pinned staging buffer may still feed an upload
  HIP_TRY(ws.table.ensure(tab.size() * sizeof(int64_t)), "density tables");
  HIP_TRY(ws.h_coef.ensure(tab.size() * sizeof(int64_t)), "pinned table staging");
  std::memcpy(ws.h_coef.p, tab.data(), tab.size() * sizeof(int64_t));
  HIP_TRY(hipMemcpyAsync(ws.table.p, ws.h_coef.p, tab.size() * sizeof(int64_t), hipMemcpyHostToDevice, s),
          "density table upload");
  const size_t amp = amp_bytes(st->dtype);
  const size_t out_bytes = (size_t)st->batch * (size_t)N * (size_t)N * amp;
  void* dst = rho;
  if (!rho_on_device) {
    HIP_TRY(ws.dens.ensure(out_bytes), "density output buffer");
    dst = ws.dens.p;
  }
  DensityLaunch L;
  L.psi = st->buf;
  L.row_stride = 1ll << n;
  L.batch = st->batch;
  L.off_i = static_cast<const int64_t*>(ws.table.p);
  L.klo = L.off_i + N;
  L.khi = L.klo + (1ll << lo_bits);
  L.lo_bits = lo_bits;
  L.N = (int)N;
  L.K = K;
  L.rho = dst;
  L.c128 = st->dtype == QSIM_C128;
  const double bytes = (double)st->batch * ((double)(1ll << n) * amp + (double)N * (double)N * amp);
  const double flops = 4.0 * (double)N * (double)(N + 1) * (double)K * st->batch;
  const int ti = timing_begin(ctx, s, bytes, 0, 2, flops);
  HIP_TRY(launch_density(L, s), "density launch");
  timing_end(ctx, ti, s);
  if (!rho_on_device) HIP_TRY(hipMemcpyAsync(rho, dst, out_bytes, hipMemcpyDeviceToHost, s), "density copy");
  HIP_TRY(hipStreamSynchronize(s), "stream sync");
  timing_collect(ctx);
  return QSIM_OK;
}

int qsim_state_device_ptr(qsim_state* st, void** ptr) {
  if (check_state(st) || !ptr) return QSIM_EINVAL;
  qsim_ctx* ctx = st->ctx;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  int rc = flush(st, nullptr, nullptr);
  if (rc) return rc;
  *ptr = st->buf;
  return QSIM_OK;
}

int qsim_expect_circuit(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch, int params_on_device,
                        const qsim_hamiltonian* H, int mode, int dtype, void* stream, double* out, qsim_state** keep) {
  if (!ctx || !out || batch < 1 || !valid_dtype(dtype)) return QSIM_EINVAL;
  if (keep) *keep = nullptr;
  if (ctx->mock) return no_device(ctx);
  CircuitDesc cd;
  int rc = to_circuit(ctx, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if ((rc = to_terms(ctx, H, cd.n, terms))) return rc;
  if (cd.n_params > 0 && !params) {
    set_error(ctx, "expect_circuit: params missing");
    return QSIM_EINVAL;
  }
  if (mode == QSIM_MODE_AUTO) mode = (cd.n > 30 && !keep) ? QSIM_MODE_LIGHTCONE_FACTORED : QSIM_MODE_DENSE;
  const int c128 = dtype == QSIM_C128;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  hipStream_t st = pick_stream(ctx, stream);
  if (mode == QSIM_MODE_LIGHTCONE || mode == QSIM_MODE_LIGHTCONE_FACTORED) {
    if (keep) {
      set_error(ctx, "expect_circuit: keep is only available in dense mode");
      return QSIM_EINVAL;
    }
    auto dp = mode == QSIM_MODE_LIGHTCONE ? get_cone_plan(ctx, cd, terms, c128, rc)
                                          : get_factor_plan(ctx, cd, terms, c128, rc);
    if (!dp) return rc;
    const ParamSrc ps(params, params_on_device != 0);
    for (int b = 0; b < batch; ++b) {
      rc = run_cones(ctx, ctx->ws, *dp, cd, ps.row(b, cd.n_params), c128, st, out + b);
      if (rc) return rc;
    }
    return QSIM_OK;
  }
  if (mode != QSIM_MODE_DENSE) return QSIM_EINVAL;
  if (cd.n > kMaxQubits) {
    set_error(ctx, "dense mode supports at most 40 qubits");
    return QSIM_ETOOBIG;
  }
  auto dp = get_dense_plan(ctx, cd, terms, c128, true, keep != nullptr, true, rc);
  if (!dp) return rc;
  const size_t bytes = (size_t)batch * ((size_t)1 << cd.n) * amp_bytes(dtype);
  void* A = nullptr;
  if (keep) {
    HIP_TRY(hipMalloc(&A, bytes), "state allocation");
  } else {
    HIP_TRY(ctx->psi.ensure(bytes), "state workspace");
    A = ctx->psi.p;
  }
  rc = run_dense(ctx, ctx->ws, *dp, cd, ParamSrc(params, params_on_device != 0), batch, c128, A, nullptr, st, out);
  if (rc) {
    if (keep) (void)hipFree(A);
    return rc;
  }
  if (keep) {
    qsim_state* s = new (std::nothrow) qsim_state();
    if (!s) {
      (void)hipFree(A);
      return QSIM_ENOMEM;
    }
    s->ctx = ctx;
    s->n = cd.n;
    s->batch = batch;
    s->dtype = dtype;
    s->buf = A;
    s->owned = true;
    s->fresh = false;
    s->stream = st;
    s->queue.n = cd.n;
    *keep = s;
  }
  return QSIM_OK;
}

int qsim_expect_terms(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch, int params_on_device,
                      const qsim_hamiltonian* H, int mode, int dtype, void* stream, double* out) {
  if (!ctx || !out || batch < 1 || !valid_dtype(dtype)) return QSIM_EINVAL;
  if (ctx->mock) return no_device(ctx);
  CircuitDesc cd;
  int rc = to_circuit(ctx, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if ((rc = to_terms(ctx, H, cd.n, terms))) return rc;
  if (cd.n_params > 0 && !params) {
    set_error(ctx, "expect_terms: params missing");
    return QSIM_EINVAL;
  }
  if (mode == QSIM_MODE_AUTO) mode = cd.n > 30 ? QSIM_MODE_LIGHTCONE_FACTORED : QSIM_MODE_DENSE;
  if (mode < QSIM_MODE_DENSE || mode > QSIM_MODE_LIGHTCONE_FACTORED) return QSIM_EINVAL;
  const int T = (int)terms.size();
  if (T == 0) return QSIM_OK;
  // every term with coefficient 1: the values are <P_t> themselves
  std::vector<Term> unit = terms;
  std::vector<int> live;  // non-identity terms, in order
  for (int t = 0; t < T; ++t) {
    unit[t].c = 1.0;
    if (!terms[t].ops.empty()) live.push_back(t);
  }
  for (int b = 0; b < batch; ++b)
    for (int t = 0; t < T; ++t) out[(size_t)b * T + t] = 1.0;  // identity terms
  if (live.empty()) return QSIM_OK;
  const int c128 = dtype == QSIM_C128;
  const ParamSrc ps(params, params_on_device != 0);
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  hipStream_t st = pick_stream(ctx, stream);
  if (mode == QSIM_MODE_LIGHTCONE || mode == QSIM_MODE_LIGHTCONE_FACTORED) {
    // one factor product per term: the canonical cone (LIGHTCONE) or disjoint pruned factors
    auto dp = get_factor_plan(ctx, cd, unit, c128, rc, false, mode == QSIM_MODE_LIGHTCONE_FACTORED);
    if (!dp) return rc;
    std::vector<double> vals(live.size());
    for (int b = 0; b < batch; ++b) {
      if ((rc = run_cones(ctx, ctx->ws, *dp, cd, ps.row(b, cd.n_params), c128, st, nullptr, vals.data()))) return rc;
      for (size_t k = 0; k < live.size(); ++k) out[(size_t)b * T + live[k]] = vals[k];
    }
    return QSIM_OK;
  }
  if (cd.n > kMaxQubits) {
    set_error(ctx, "dense mode supports at most 40 qubits");
    return QSIM_ETOOBIG;
  }
  // the final states once, then one read-only measurement per term
  auto fp = get_dense_plan(ctx, cd, {}, c128, true, true, false, rc);
  if (!fp) return rc;
  const size_t bytes = (size_t)batch * ((size_t)1 << cd.n) * amp_bytes(dtype);
  HIP_TRY(ctx->psi.ensure(bytes), "state workspace");
  void* A = ctx->psi.p;
  if ((rc = run_dense(ctx, ctx->ws, *fp, cd, ps, batch, c128, A, nullptr, st, nullptr))) return rc;
  CircuitDesc empty;
  empty.n = cd.n;
  std::vector<double> vals(batch);
  for (int t : live) {
    auto mp = get_dense_plan(ctx, empty, {unit[t]}, c128, false, false, true, rc);
    if (!mp) return rc;
    if ((rc = run_dense(ctx, ctx->ws, *mp, empty, ParamSrc(), batch, c128, A, nullptr, st, vals.data()))) return rc;
    for (int b = 0; b < batch; ++b) out[(size_t)b * T + t] = vals[b];
  }
  return QSIM_OK;
}

int qsim_expect_grad_cones(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch,
                           int params_on_device, const qsim_hamiltonian* H, int mode, int dtype, void* stream,
                           double* E, double* grad) {
  if (!ctx || !grad || batch < 1 || !valid_dtype(dtype)) return QSIM_EINVAL;
  if (mode == QSIM_MODE_AUTO) mode = QSIM_MODE_LIGHTCONE_FACTORED;
  if (mode != QSIM_MODE_LIGHTCONE && mode != QSIM_MODE_LIGHTCONE_FACTORED) {
    set_error(ctx, "expect_grad_cones: mode must be LIGHTCONE, LIGHTCONE_FACTORED or AUTO");
    return QSIM_EINVAL;
  }
  if (ctx->mock) return no_device(ctx);
  CircuitDesc cd;
  int rc = to_circuit(ctx, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if ((rc = to_terms(ctx, H, cd.n, terms))) return rc;
  if (cd.n_params > 0 && !params) {
    set_error(ctx, "expect_grad_cones: params missing");
    return QSIM_EINVAL;
  }
  const int c128 = dtype == QSIM_C128;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  hipStream_t st = pick_stream(ctx, stream);
  auto dp = get_factor_plan(ctx, cd, terms, c128, rc, true, mode == QSIM_MODE_LIGHTCONE_FACTORED);
  if (!dp) return rc;
  const ParamSrc ps(params, params_on_device != 0);
  for (int b = 0; b < batch; ++b) {
    double e = 0;
    rc = run_cone_grad(ctx, ctx->ws, *dp, cd, ps.row(b, cd.n_params), c128, st, &e, grad + (size_t)b * cd.n_params);
    if (rc) return rc;
    if (E) E[b] = e;
  }
  return QSIM_OK;
}

int qsim_expect_grad(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch, int params_on_device,
                     const qsim_hamiltonian* H, int dtype, void* stream, qsim_state* saved, double* E, double* grad) {
  if (!ctx || batch < 1 || !valid_dtype(dtype) || !grad) return QSIM_EINVAL;
  if (ctx->mock) return no_device(ctx);
  CircuitDesc cd;
  int rc = to_circuit(ctx, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if ((rc = to_terms(ctx, H, cd.n, terms))) return rc;
  if (cd.n_params > 0 && !params) {
    set_error(ctx, "expect_grad: params missing");
    return QSIM_EINVAL;
  }
  if (cd.n > kMaxQubits) {
    set_error(ctx, "gradients use the dense mode: at most 40 qubits");
    return QSIM_ETOOBIG;
  }
  if (saved && (saved->n != cd.n || saved->batch != batch || saved->dtype != dtype || !saved->queue.gates.empty())) {
    set_error(ctx, "expect_grad: saved state does not match the circuit, batch or dtype");
    return QSIM_EINVAL;
  }
  const int c128 = dtype == QSIM_C128;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  hipStream_t st = pick_stream(ctx, stream);
  const size_t bytes = (size_t)batch * ((size_t)1 << cd.n) * amp_bytes(dtype);
  void* A = nullptr;
  if (saved) {
    A = saved->buf;
    if (E) {  // <H> of the saved state: a measurement-only plan
      CircuitDesc empty;
      empty.n = cd.n;
      auto mp = get_dense_plan(ctx, empty, terms, c128, false, false, true, rc);
      if (!mp) return rc;
      if ((rc = run_dense(ctx, ctx->ws, *mp, empty, ParamSrc(), batch, c128, A, nullptr, st, E))) return rc;
    }
  } else {
    auto fp = get_dense_plan(ctx, cd, terms, c128, true, true, true, rc);
    if (!fp) return rc;
    HIP_TRY(ctx->psi.ensure(bytes), "state workspace");
    A = ctx->psi.p;
    std::vector<double> e_tmp(batch);
    if ((rc = run_dense(ctx, ctx->ws, *fp, cd, ParamSrc(params, params_on_device != 0), batch, c128, A, nullptr, st,
                        E ? E : e_tmp.data())))
      return rc;
  }
  std::shared_ptr<DevPlan> hp;
  auto ap = get_grad_plans(ctx, cd, terms, c128, hp, rc);
  if (!ap) return rc;
  HIP_TRY(ctx->ws.lambda.ensure(bytes), "lambda workspace");
  return run_grad(ctx, ctx->ws, *hp, *ap, cd, ParamSrc(params, params_on_device != 0), batch, c128, A,
                  ctx->ws.lambda.p, st, grad);
}

int qsim_timing_enable(qsim_ctx* ctx, int on) {
  if (!ctx) return QSIM_EINVAL;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  if (on) ctx->tdone.clear();
  ctx->timing = on != 0;
  return QSIM_OK;
}

int qsim_timing_get(qsim_ctx* ctx, double* ms, double* bytes, double* flops, int32_t* flags, int32_t* kind, int cap,
                    int* count) {
  if (!ctx || !count) return QSIM_EINVAL;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  const int n = std::min<int>(cap, (int)ctx->tdone.size());
  for (int i = 0; i < n; ++i) {
    if (ms) ms[i] = ctx->tdone[i].ms;
    if (bytes) bytes[i] = ctx->tdone[i].bytes;
    if (flops) flops[i] = ctx->tdone[i].flops;
    if (flags) flags[i] = ctx->tdone[i].flags;
    if (kind) kind[i] = ctx->tdone[i].kind;
  }
  *count = n;
  return QSIM_OK;
}

int qsim_copy_probe(qsim_ctx* ctx, uint64_t bytes, int reps, double* ms) {
  if (!ctx || !ms || bytes == 0 || bytes % 16 || reps < 1) return QSIM_EINVAL;
  if (ctx->mock) return no_device(ctx);
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  void *src = nullptr, *dst = nullptr;
  HIP_TRY(hipMalloc(&src, bytes), "copy source");
  hipError_t e = hipMalloc(&dst, bytes);
  if (e != hipSuccess) {
    (void)hipFree(src);
    return hip_fail(ctx, e, "copy destination");
  }
  hipEvent_t a = nullptr, b = nullptr;
  e = hipMemsetAsync(src, 0, bytes, ctx->stream);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = launch_copy(src, dst, bytes / 16, ctx->stream);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(src, dst, bytes / 16, ctx->stream);
  if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(src);
  (void)hipFree(dst);
  if (e != hipSuccess) return hip_fail(ctx, e, "copy probe");
  *ms = t / reps;
  return QSIM_OK;
}

int qsim_lightcone_sets(const qsim_circuit* c, const qsim_hamiltonian* H, int32_t* off, int32_t* qubits, int cap) {
  if (!off || (cap > 0 && !qubits)) return QSIM_EINVAL;
  CircuitDesc cd;
  int rc = to_circuit(nullptr, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if ((rc = to_terms(nullptr, H, cd.n, terms))) return rc;
  int pos = 0;
  off[0] = 0;
  for (size_t t = 0; t < terms.size(); ++t) {
    std::vector<int> support, set, gates;
    for (auto [q, L] : terms[t].ops) support.push_back(q);
    light_cone(cd, support, set, gates);
    if (pos + (int)set.size() > cap) return QSIM_ETOOBIG;
    for (int q : set) qubits[pos++] = q;
    off[t + 1] = pos;
  }
  return QSIM_OK;
}

int qsim_plan_dense(const qsim_circuit* c, const qsim_hamiltonian* H, int dtype, int64_t* info, int32_t* order,
                    int cap_entries) {
  if (!info || !valid_dtype(dtype)) return QSIM_EINVAL;
  CircuitDesc cd;
  int rc = to_circuit(nullptr, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if (H && (rc = to_terms(nullptr, H, cd.n, terms))) return rc;
  if (cd.n > kMaxQubits) return QSIM_ETOOBIG;
  Plan plan;
  std::vector<PGate> pg, meas;
  forward_pgates(cd, true, pg, plan.slots);
  double cst = 0;
  term_pgates(terms, false, meas, cst);
  const qsim_options defaults{};
  PlanOptions o = fwd_options(defaults, dtype == QSIM_C128);
  o.store_final = false;
  std::string err;
  if (plan_forward(cd.n, pg, meas, o, plan, err)) return QSIM_EINVAL;
  info[0] = (int64_t)plan.passes.size();
  info[1] = (int64_t)plan.stages.size();
  info[2] = (int64_t)plan.ops.size();
  info[3] = plan.meas_passes;
  if (order) {
    if ((int)plan.order.size() / 4 > cap_entries) return QSIM_ETOOBIG;
    std::memcpy(order, plan.order.data(), plan.order.size() * sizeof(int32_t));
  }
  return QSIM_OK;
}

int qsim_plan_passes(qsim_ctx* ctx, const qsim_circuit* c, const qsim_hamiltonian* H, int dtype, int keep,
                     int32_t* rec, int cap, int* count) {
  if (!ctx || !H || !count || !valid_dtype(dtype) || (cap > 0 && !rec)) return QSIM_EINVAL;
  *count = 0;
  CircuitDesc cd;
  int rc = to_circuit(ctx, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if ((rc = to_terms(ctx, H, cd.n, terms))) return rc;
  if (cd.n > kMaxQubits) return QSIM_ETOOBIG;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  if (!ctx->mock) HIP_TRY(hipSetDevice(ctx->device), "set device");
  auto dp = get_dense_plan(ctx, cd, terms, dtype == QSIM_C128, true, keep != 0, true, rc);
  if (!dp) return rc;
  const Plan& P = dp->plan;
  const int np = (int)P.passes.size();
  if (np > cap) {
    *count = np;
    return QSIM_ETOOBIG;
  }
  for (int p = 0; p < np; ++p) {
    const PassDesc& pd = P.passes[p];
    int32_t* o = rec + 8 * p;
    o[0] = pd.flags;
    o[1] = pd.stage_end - pd.stage_begin;
    o[2] = pd.store_stage >= 0 ? pd.store_stage - pd.stage_begin : -1;
    o[3] = pd.entry_perm;
    o[4] = pd.exit_perm;
    o[5] = pd.meas_index;
    o[6] = pd.grad_count;
    o[7] = pd.m;
  }
  *count = np;
  return QSIM_OK;
}

int qsim_plan_trace(qsim_ctx* ctx, const qsim_circuit* c, const qsim_hamiltonian* H, int dtype, int keep,
                    int64_t* rec, double* coef, int cap, int32_t* srcs, int cap_srcs, int* count, int* n_srcs) {
  if (!ctx || !H || !count || !n_srcs || !valid_dtype(dtype) || (cap > 0 && (!rec || !coef)) ||
      (cap_srcs > 0 && !srcs))
    return QSIM_EINVAL;
  *count = 0;
  *n_srcs = 0;
  CircuitDesc cd;
  int rc = to_circuit(ctx, c, cd);
  if (rc) return rc;
  std::vector<Term> terms;
  if ((rc = to_terms(ctx, H, cd.n, terms))) return rc;
  if (cd.n > kMaxQubits) return QSIM_ETOOBIG;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  Plan P;
  if ((rc = host_dense_plan(ctx, cd, terms, dtype == QSIM_C128, true, keep != 0, P, true))) return rc;
  std::vector<std::array<int64_t, 8>> out;
  std::vector<double> w;
  std::vector<int32_t> sv;
  for (size_t k = 0; k + 3 < P.order.size(); k += 4)
    if (P.order[k + 2] == -2) {
      out.push_back({5, -1, -1, (int64_t)sv.size(), 1, 0, 0, 0});
      w.push_back(0);
      sv.push_back(P.order[k + 3]);
    }
  for (const PGate& g : P.trace) {
    std::array<int64_t, 8> r{0, g.q, g.q2, 0, 0, 0, 0, 0};
    if (g.kind == -1) {
      r = {4, -1, -1, 0, 0, 0, 0, 0};
    } else if (g.kind == PG_X) {
      r[0] = 1;
    } else if (g.kind == PG_CZ) {
      r[0] = 2;
    } else if (g.kind == PG_MEAS_Z || g.kind == PG_MEAS_F) {
      r = {3, -1, -1, 0, 0, g.ph, (int64_t)g.fmask, (int64_t)g.zmask};
    } else if (g.kind == PG_U || g.kind == PG_RY || g.kind == PG_PHASE) {
      r[2] = -1;
      r[3] = (int64_t)sv.size();
      r[4] = (int64_t)g.srcs.size();
      for (int src : g.srcs) sv.push_back(src);
    } else {
      set_error(ctx, "plan_trace: unexpected item");
      return QSIM_EINVAL;
    }
    out.push_back(r);
    w.push_back(r[0] == 3 ? g.c : 0.0);
  }
  *count = (int)out.size();
  *n_srcs = (int)sv.size();
  if ((int)out.size() > cap || (int)sv.size() > cap_srcs) return QSIM_ETOOBIG;
  for (size_t i = 0; i < out.size(); ++i) {
    std::memcpy(rec + 8 * i, out[i].data(), 8 * sizeof(int64_t));
    coef[i] = w[i];
  }
  if (!sv.empty()) std::memcpy(srcs, sv.data(), sv.size() * sizeof(int32_t));
  return QSIM_OK;
}

int qsim_coef_rows(qsim_ctx* ctx, const qsim_circuit* c, const double* params, int batch, int params_on_device,
                   int dtype, void* out, uint64_t cap, uint64_t* bytes) {
  if (!ctx || !bytes || batch < 1 || !valid_dtype(dtype) || (cap > 0 && !out)) return QSIM_EINVAL;
  *bytes = 0;
  if (ctx->mock) return no_device(ctx);
  CircuitDesc cd;
  int rc = to_circuit(ctx, c, cd);
  if (rc) return rc;
  if (cd.n_params > 0 && !params) return QSIM_EINVAL;
  if (cd.n > kMaxQubits) return QSIM_ETOOBIG;
  std::lock_guard<std::mutex> g(ctx->api_mu);
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  auto dp = get_dense_plan(ctx, cd, {}, dtype == QSIM_C128, true, true, false, rc);
  if (!dp) return rc;
  return coef_rows(ctx, ctx->ws, *dp, cd, ParamSrc(params, params_on_device != 0), batch, dtype == QSIM_C128,
                   ctx->stream, out, cap, bytes);
}

}  // extern "C"
