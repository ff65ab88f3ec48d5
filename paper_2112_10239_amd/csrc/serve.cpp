// Serving loop with continuous batching (see serve.h).
#include "serve.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

namespace qsim {

namespace {

constexpr size_t kMaxRunning = 512;

enum Phase { PH_FWD = 0, PH_HAPPLY = 1, PH_ADJ = 2, PH_DONE = 3 };

}  // namespace

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SReq {
  uint64_t ticket = 0;
  CircuitDesc c;
  std::vector<Term> terms;
  std::vector<double> params;
  bool want_grad = false;
  size_t footprint = 0;
  // lifecycle
  bool cancelled = false, done = false, failed = false, prepared = false;
  int status = QSIM_PENDING;
  double E = 0;
  std::vector<double> grad;
  // execution
  std::shared_ptr<DevPlan> fp, hp, ap;
  int phase = PH_FWD;
  int next = 0;
  int ended = -1;  // phase that ended in the current step
  size_t state_bytes = 0, coef_f_bytes = 0, coef_a_bytes = 0, meas_bytes = 0, gpart_bytes = 0, res_bytes = 0;
  void *A = nullptr, *B = nullptr, *coef_f = nullptr, *coef_a = nullptr;
  double *meas = nullptr, *gpart = nullptr, *res = nullptr;
  std::vector<float> h_coef_f, h_coef_a;
  std::vector<double> h_res;
  int passes_done = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

// ---------------------------------------------------------------------------
// block pool
// ---------------------------------------------------------------------------

static int g_fail_alloc_countdown = [] {
  const char* s = std::getenv("QSIM_TEST_FAIL_ALLOC");
  return s ? std::atoi(s) : 0;
}();

BlockPool::~BlockPool() { trim(0); }

void* BlockPool::get(size_t bytes) {
  if (g_fail_alloc_countdown > 0 && --g_fail_alloc_countdown == 0) return nullptr;  // test hook
  auto it = free_.find(bytes);
  if (it != free_.end()) {
    void* p = it->second;
    free_.erase(it);
    cached_ -= bytes;
    return p;
  }
  if (mock_) {
    const uintptr_t p = fake_;
    fake_ += (bytes + 255) & ~(size_t)255;
    return reinterpret_cast<void*>(p);
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    trim(0);  // give cached blocks back and retry once
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  return p;
}

void BlockPool::put(void* p, size_t bytes) {
  if (!p) return;
  free_.emplace(bytes, p);
  cached_ += bytes;
}

void BlockPool::trim(size_t keep_bytes) {
  while (cached_ > keep_bytes && !free_.empty()) {
    auto it = std::prev(free_.end());  // largest first
    if (!mock_) (void)hipFree(it->second);
    cached_ -= it->first;
    free_.erase(it);
  }
}

// ---------------------------------------------------------------------------
// server
// ---------------------------------------------------------------------------

Server::Server(qsim_ctx* ctx, bool mock) : ctx_(ctx), mock_(mock), pool_(mock) {
  if (!mock_) {
    (void)hipSetDevice(ctx_->device);
    (void)hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
  }
  thread_ = std::thread([this] { loop(); });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (thread_.joinable()) thread_.join();
  if (!mock_) {
    (void)hipStreamSynchronize(stream_);
    pool_.trim(0);
    ws_.release();
    d_items_.release();
    (void)hipStreamDestroy(stream_);
  }
}

static size_t footprint_of(const CircuitDesc& c, const std::vector<Term>& terms, bool grad) {
  const size_t amps = (size_t)1 << c.n;
  size_t rot = 0, flips = 0;
  for (const Gate& g : c.gates) rot += (g.param >= 0);
  for (const Term& t : terms)
    for (auto [q, L] : t.ops)
      if (L != 'Z') {
        ++flips;
        break;
      }
  const size_t tiles_f = (size_t)1 << std::max(0, c.n - 14);
  const size_t tiles_d = (size_t)1 << std::max(0, c.n - 13);
  size_t bytes = (grad ? 2 : 1) * amps * 8;                // psi (+ lambda)
  bytes += (1 + flips) * tiles_f * 8;                      // measurement partials
  bytes += c.gates.size() * 32 * (grad ? 2 : 1);           // coefficients
  if (grad) bytes += rot * tiles_d * 8 + (2 * rot + c.n_params + 1) * 8;  // gradient partials and results
  else bytes += 8;
  return bytes;
}

int Server::submit(const qsim_request* rq, uint64_t* ticket) {
  if (!rq || !ticket) return QSIM_EINVAL;
  auto r = std::make_unique<SReq>();
  int rc = to_circuit(ctx_, rq->circuit, r->c);
  if (rc) return rc;
  if ((rc = to_terms(ctx_, rq->H, r->c.n, r->terms))) return rc;
  if (r->c.n > 30 || r->c.n < 6) {
    set_error(ctx_, "serving takes dense requests of 6 to 30 qubits");
    return QSIM_EINVAL;
  }
  if (r->c.n_params > 0 && !rq->params) {
    set_error(ctx_, "submit: params missing");
    return QSIM_EINVAL;
  }
  r->params.assign(rq->params, rq->params + r->c.n_params);
  r->want_grad = rq->want_grad != 0;
  r->footprint = footprint_of(r->c, r->terms, r->want_grad);
  std::lock_guard<std::mutex> g(mu_);
  if (stop_) return QSIM_ESHUTDOWN;
  if (r->footprint > ctx_->opt.hbm_budget_bytes) {
    st_.rejected++;
    set_error(ctx_, "request footprint exceeds the memory budget");
    return QSIM_ETOOBIG;
  }
  if (queue_.size() + running_.size() >= (size_t)ctx_->opt.max_queue) {
    st_.rejected++;
    return QSIM_EAGAIN;
  }
  r->ticket = next_ticket_++;
  *ticket = r->ticket;
  r->t_submit = now_s();
  queue_.push_back(r.get());
  all_.emplace(r->ticket, std::move(r));
  st_.submitted++;
  cv_.notify_all();
  return QSIM_OK;
}

int Server::poll(uint64_t ticket, double* E, double* grad, double* times) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) return QSIM_ENOTFOUND;
  SReq* r = it->second.get();
  if (!r->done) return QSIM_PENDING;
  const int status = r->status;
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_admit;
    times[2] = r->t_done;
  }
  if (status == QSIM_OK) {
    if (E) *E = r->E;
    if (grad && r->want_grad) std::memcpy(grad, r->grad.data(), sizeof(double) * r->grad.size());
  }
  all_.erase(it);
  return status;
}

int Server::cancel(uint64_t ticket) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end() || it->second->done) return QSIM_ENOTFOUND;
  SReq* r = it->second.get();
  r->cancelled = true;
  auto q = std::find(queue_.begin(), queue_.end(), r);
  if (q != queue_.end()) {
    queue_.erase(q);
    r->done = true;
    r->t_done = now_s();
    r->status = QSIM_ECANCELED;
    st_.cancelled++;
  }
  return QSIM_OK;
}

void Server::stats(qsim_server_stats* out) {
  std::lock_guard<std::mutex> g(mu_);
  *out = st_;
  out->inflight_bytes = inflight_;
  out->peak_inflight_bytes = peak_;
  out->queued = queue_.size();
  out->running = running_.size();
}

int Server::prepare(SReq* r) {
  int rc = QSIM_OK;
  r->fp = get_dense_plan(ctx_, r->c, r->terms, 0, true, r->want_grad, true, rc);
  if (!r->fp) return rc;
  if (r->want_grad) {
    r->ap = get_grad_plans(ctx_, r->c, r->terms, 0, r->hp, rc);
    if (!r->ap) return rc;
  }
  const Plan& F = r->fp->plan;
  r->state_bytes = ((size_t)1 << r->c.n) * 8;
  const int64_t crs_f = (int64_t)std::max<size_t>(1, F.slots.size()) * 8;
  r->coef_f_bytes = (size_t)crs_f * sizeof(float);
  r->meas_bytes = std::max<size_t>(1, (size_t)F.n_meas << (F.n - F.m)) * sizeof(double);
  size_t ns = 0, np = r->c.n_params;
  if (r->want_grad) {
    const Plan& P = r->ap->plan;
    ns = P.n_gslots;
    r->coef_a_bytes = std::max<size_t>(1, P.slots.size()) * 8 * sizeof(float);
    r->gpart_bytes = std::max<size_t>(1, ns << (P.n - P.m)) * sizeof(double);
  }
  r->res_bytes = (1 + ns + np) * sizeof(double);
  r->A = pool_.get(r->state_bytes);
  if (r->want_grad) r->B = pool_.get(r->state_bytes);
  r->coef_f = pool_.get(r->coef_f_bytes);
  if (r->want_grad) r->coef_a = pool_.get(r->coef_a_bytes);
  r->meas = (double*)pool_.get(r->meas_bytes);
  if (r->want_grad) r->gpart = (double*)pool_.get(r->gpart_bytes);
  r->res = (double*)pool_.get(r->res_bytes);
  r->prepared = true;
  if (!r->A || (r->want_grad && (!r->B || !r->coef_a || !r->gpart)) || !r->coef_f || !r->meas || !r->res) {
    set_error(ctx_, "serving: device allocation failed");
    return QSIM_ENOMEM;
  }
  r->h_coef_f.resize((size_t)crs_f);
  build_coefficients<float>(r->c, F.slots, r->params.data(), 1, crs_f, r->h_coef_f.data());
  if (r->want_grad) {
    const int64_t crs_a = (int64_t)std::max<size_t>(1, r->ap->plan.slots.size()) * 8;
    r->h_coef_a.resize((size_t)crs_a);
    build_coefficients<float>(r->c, r->ap->plan.slots, r->params.data(), 1, crs_a, r->h_coef_a.data());
  }
  if (!mock_) {
    if (hipMemcpyAsync(r->coef_f, r->h_coef_f.data(), r->coef_f_bytes, hipMemcpyHostToDevice, stream_) != hipSuccess)
      return hip_fail(ctx_, hipGetLastError(), "serving coefficient upload");
    if (r->want_grad &&
        hipMemcpyAsync(r->coef_a, r->h_coef_a.data(), r->coef_a_bytes, hipMemcpyHostToDevice, stream_) != hipSuccess)
      return hip_fail(ctx_, hipGetLastError(), "serving coefficient upload");
  }
  r->h_res.assign(1 + np, 0.0);
  return QSIM_OK;
}

void Server::release(SReq* r) {
  if (!r->prepared) return;
  pool_.put(r->A, r->state_bytes);
  pool_.put(r->B, r->state_bytes);
  pool_.put(r->coef_f, r->coef_f_bytes);
  pool_.put(r->coef_a, r->coef_a_bytes);
  pool_.put(r->meas, r->meas_bytes);
  pool_.put(r->gpart, r->gpart_bytes);
  pool_.put(r->res, r->res_bytes);
  r->A = r->B = r->coef_f = r->coef_a = nullptr;
  r->meas = r->gpart = r->res = nullptr;
  r->prepared = false;
  r->fp.reset();
  r->hp.reset();
  r->ap.reset();
  // keep the pool within the memory budget
  const size_t budget = ctx_->opt.hbm_budget_bytes;
  const size_t limit = budget > inflight_ ? budget - inflight_ : 0;
  if (pool_.cached() > limit) pool_.trim(limit);
}

// Launch one pass for every running request; returns false on a device error.
bool Server::step(std::vector<SReq*>& run) {
  std::vector<PassItem> single, dual;
  int64_t tiles_s = 0, tiles_d = 0;
  int m_s = 4, m_d = 4, r_s = 0, r_d = 0;
  for (SReq* r : run) {
    r->ended = -1;
    if (r->failed || r->cancelled || r->phase == PH_DONE) continue;
    const DevPlan* dp = r->phase == PH_FWD ? r->fp.get() : r->phase == PH_HAPPLY ? r->hp.get() : r->ap.get();
    const Plan& P = dp->plan;
    const int p = r->next;
    PassItem it;
    it.pass = dp->d_passes + p;
    it.stages = dp->d_stages;
    it.ops = dp->d_ops;
    it.A = r->A;
    it.B = r->B;
    it.coef = r->phase == PH_FWD ? r->coef_f : r->coef_a;
    it.meas = r->meas;
    it.grad = r->gpart;
    const int64_t tiles = 1ll << (P.n - P.m);
    if (r->phase == PH_FWD) {
      it.tile_begin = tiles_s;
      tiles_s += tiles;
      m_s = std::max(m_s, P.m);
      r_s = P.r;
      single.push_back(it);
    } else {
      it.tile_begin = tiles_d;
      tiles_d += tiles;
      m_d = std::max(m_d, P.m);
      r_d = P.r;
      dual.push_back(it);
    }
    r->passes_done++;
    if (++r->next == (int)P.passes.size()) r->ended = r->phase;
  }
  if (mock_) return true;
  items_.clear();
  items_.insert(items_.end(), single.begin(), single.end());
  items_.insert(items_.end(), dual.begin(), dual.end());
  if (items_.empty()) return true;
  const size_t bytes = items_.size() * sizeof(PassItem);
  if (ws_.h_out.ensure(bytes) != hipSuccess || d_items_.ensure(bytes) != hipSuccess) return false;
  // the previous step synchronised the stream, so the pinned staging buffer is free
  std::memcpy(ws_.h_out.p, items_.data(), bytes);
  if (hipMemcpyAsync(d_items_.p, ws_.h_out.p, bytes, hipMemcpyHostToDevice, stream_) != hipSuccess) return false;
  const PassItem* d = reinterpret_cast<const PassItem*>(d_items_.p);
  if (launch_pass_multi(d, (int)single.size(), tiles_s, m_s, r_s, 0, 0, stream_) != hipSuccess) return false;
  if (launch_pass_multi(d + single.size(), (int)dual.size(), tiles_d, m_d, r_d, 0, 1, stream_) != hipSuccess)
    return false;
  st_.launches += (single.empty() ? 0 : 1) + (dual.empty() ? 0 : 1);
  // reductions of requests whose phase ended in this step
  for (SReq* r : run) {
    if (r->ended == PH_FWD) {
      const Plan& F = r->fp->plan;
      if (launch_reduce_rows(r->meas, 1, (int64_t)F.n_meas << (F.n - F.m), F.const_term, r->res, stream_) !=
          hipSuccess)
        return false;
      if (!r->want_grad &&
          hipMemcpyAsync(r->h_res.data(), r->res, sizeof(double), hipMemcpyDeviceToHost, stream_) != hipSuccess)
        return false;
    } else if (r->ended == PH_ADJ) {
      const Plan& P = r->ap->plan;
      const int ns = P.n_gslots, np = r->c.n_params;
      double* slot_total = r->res + 1;
      double* g = r->res + 1 + ns;
      if (ns > 0) {
        if (launch_reduce_rows(r->gpart, ns, 1ll << (P.n - P.m), 0.0, slot_total, stream_) != hipSuccess) return false;
        int np_used = 0;
        for (int p : P.gslot_param) np_used = std::max(np_used, p + 1);
        if (launch_grad_scatter(slot_total, 1, ns, r->ap->d_poff, r->ap->d_pslots, np_used, g, stream_) !=
            hipSuccess)
          return false;
        if (hipMemcpyAsync(r->h_res.data() + 1, g, sizeof(double) * np_used, hipMemcpyDeviceToHost, stream_) !=
            hipSuccess)
          return false;
      }
      (void)np;
      if (hipMemcpyAsync(r->h_res.data(), r->res, sizeof(double), hipMemcpyDeviceToHost, stream_) != hipSuccess)
        return false;
    }
  }
  return hipStreamSynchronize(stream_) == hipSuccess;
}

void Server::loop() {
  if (!mock_) (void)hipSetDevice(ctx_->device);
  const size_t budget = ctx_->opt.hbm_budget_bytes;
  while (true) {
    std::vector<SReq*> fresh, run;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || !queue_.empty() || !running_.empty(); });
      if (stop_) break;
      while (!queue_.empty() && running_.size() < kMaxRunning) {
        SReq* r = queue_.front();
        if (inflight_ + r->footprint > budget) break;  // FIFO: the head waits for memory
        queue_.pop_front();
        running_.push_back(r);
        inflight_ += r->footprint;
        peak_ = std::max(peak_, inflight_);
        r->t_admit = now_s();
        fresh.push_back(r);
      }
      run = running_;
    }
    for (SReq* r : fresh) {
      const int rc = prepare(r);
      if (rc) {
        r->failed = true;
        r->status = rc;
      }
    }
    const bool ok = step(run);
    std::lock_guard<std::mutex> g(mu_);
    st_.steps++;
    for (SReq* r : run) {
      if (!ok && !r->failed) {
        r->failed = true;
        r->status = QSIM_EDEVICE;
      }
      if (!r->failed && !r->cancelled) {
        if (r->ended == PH_FWD) {
          if (r->want_grad) {
            r->phase = PH_HAPPLY;
            r->next = 0;
          } else {
            r->phase = PH_DONE;
          }
        } else if (r->ended == PH_HAPPLY) {
          r->phase = PH_ADJ;
          r->next = 0;
        } else if (r->ended == PH_ADJ) {
          r->phase = PH_DONE;
        }
      }
      const bool finished = r->failed || r->cancelled || r->phase == PH_DONE;
      if (!finished) continue;
      if (r->failed) {
        st_.failed++;
      } else if (r->cancelled) {
        r->status = QSIM_ECANCELED;
        st_.cancelled++;
      } else {
        r->status = QSIM_OK;
        r->E = mock_ ? (double)r->passes_done : r->h_res[0];
        if (r->want_grad) {
          r->grad.assign(r->c.n_params, 0.0);
          if (!mock_) {
            int np_used = 0;
            for (int p : r->ap->plan.gslot_param) np_used = std::max(np_used, p + 1);
            for (int k = 0; k < np_used; ++k) r->grad[k] = r->h_res[1 + k];
          }
        }
        st_.completed++;
      }
      inflight_ -= r->footprint;
      release(r);
      r->t_done = now_s();
      r->done = true;
      running_.erase(std::find(running_.begin(), running_.end(), r));
    }
  }
  // shutdown: everything still pending ends with ESHUTDOWN
  std::lock_guard<std::mutex> g(mu_);
  if (!mock_) (void)hipStreamSynchronize(stream_);
  for (SReq* r : running_) {
    release(r);
    r->done = true;
    r->status = QSIM_ESHUTDOWN;
  }
  running_.clear();
  for (SReq* r : queue_) {
    r->done = true;
    r->status = QSIM_ESHUTDOWN;
  }
  queue_.clear();
}

}  // namespace qsim

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

using qsim::Server;

static Server* server_of(qsim_ctx* ctx) {
  std::lock_guard<std::mutex> g(ctx->api_mu);
  if (!ctx->server) ctx->server.reset(new Server(ctx, ctx->mock));
  return ctx->server.get();
}

extern "C" {

int qsim_submit(qsim_ctx* ctx, const qsim_request* req, uint64_t* ticket) {
  if (!ctx) return QSIM_EINVAL;
  return server_of(ctx)->submit(req, ticket);
}

int qsim_poll(qsim_ctx* ctx, uint64_t ticket, double* E, double* grad) {
  if (!ctx) return QSIM_EINVAL;
  return server_of(ctx)->poll(ticket, E, grad, nullptr);
}

int qsim_poll_timed(qsim_ctx* ctx, uint64_t ticket, double* E, double* grad, double* times) {
  if (!ctx) return QSIM_EINVAL;
  return server_of(ctx)->poll(ticket, E, grad, times);
}

double qsim_clock(void) { return qsim::now_s(); }

int qsim_cancel(qsim_ctx* ctx, uint64_t ticket) {
  if (!ctx) return QSIM_EINVAL;
  return server_of(ctx)->cancel(ticket);
}

int qsim_server_stats_get(qsim_ctx* ctx, qsim_server_stats* out) {
  if (!ctx || !out) return QSIM_EINVAL;
  server_of(ctx)->stats(out);
  return QSIM_OK;
}

}  // extern "C"
