// Serving loop with continuous batching (see serve.h).
#include "serve.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

namespace qsim {

namespace {

constexpr size_t kMaxRunning = 512;          // requests launching passes at once
constexpr size_t kDefaultSteps = 3;          // steps in flight on the device (default)
constexpr size_t kRingBytes = 64ull << 20;   // pinned staging for plan/coefficient uploads

enum Phase { PH_FWD = 0, PH_HAPPLY = 1, PH_ADJ = 2, PH_DONE = 3 };

}  // namespace

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device copy of a per-request plan, in pooled blocks.
struct ReqPlan {
  PassDesc* P = nullptr;
  StageDesc* S = nullptr;
  DevOp* O = nullptr;
  size_t bp = 0, bs = 0, bo = 0;
};

struct SReq {
  uint64_t ticket = 0;
  CircuitDesc c;
  std::vector<Term> terms;
  std::vector<double> params;
  bool want_grad = false;
  size_t footprint = 0;
  // lifecycle (under the server mutex once queued)
  bool cancelled = false, done = false, failed = false, admitted = false;
  int status = QSIM_PENDING;
  double E = 0;
  std::vector<double> grad;
  double t_submit = 0, t_admit = 0, t_done = 0;
  // host preparation, done by the submitting thread
  Plan fplan, hplan;            // forward (+ measurement) and H-apply plans
  std::shared_ptr<DevPlan> ap;  // adjoint plan, shared by requests of one circuit structure
  std::vector<float> coef_f, coef_a;
  int np_used = 0;
  // device state (scheduler thread)
  ReqPlan df, dh;
  void *A = nullptr, *B = nullptr, *cf = nullptr, *ca = nullptr;
  double *meas = nullptr, *gpart = nullptr, *res = nullptr;
  size_t state_bytes = 0, cf_bytes = 0, ca_bytes = 0, meas_bytes = 0, gpart_bytes = 0, res_bytes = 0;
  double* h_res = nullptr;  // pinned ring space of the final step: E, then the gradient
  int phase = PH_FWD, next = 0, passes_done = 0;
};

// ---------------------------------------------------------------------------
// block pool and pinned ring
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
    out_ += bytes;
    return p;
  }
  if (mock_) {
    const uintptr_t p = fake_;
    fake_ += (bytes + 255) & ~(size_t)255;
    out_ += bytes;
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
  out_ += bytes;
  return p;
}

void BlockPool::put(void* p, size_t bytes) {
  if (!p) return;
  free_.emplace(bytes, p);
  cached_ += bytes;
  out_ -= bytes;
}

void BlockPool::trim(size_t keep_bytes) {
  while (cached_ > keep_bytes && !free_.empty()) {
    auto it = std::prev(free_.end());  // largest first
    if (!mock_) (void)hipFree(it->second);
    cached_ -= it->first;
    free_.erase(it);
  }
}

PinnedRing::~PinnedRing() {
  if (!base_) return;
  if (mock_) std::free(base_);
  else (void)hipHostFree(base_);
}

bool PinnedRing::init(size_t bytes, bool mock) {
  mock_ = mock;
  if (mock) base_ = static_cast<char*>(std::malloc(bytes));
  else if (hipHostMalloc(reinterpret_cast<void**>(&base_), bytes, hipHostMallocDefault) != hipSuccess)
    base_ = nullptr;
  cap_ = base_ ? bytes : 0;
  return base_ != nullptr;
}

void* PinnedRing::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (!base_ || bytes > cap_) return nullptr;
  uint64_t start = head_;
  const uint64_t pos = head_ % cap_;
  if (pos + bytes > cap_) start += cap_ - pos;  // no room before the end: wrap to the front
  if (start + bytes - tail_ > cap_) return nullptr;
  head_ = start + bytes;
  return base_ + (start % cap_);
}

// ---------------------------------------------------------------------------
// server
// ---------------------------------------------------------------------------

Server::Server(qsim_ctx* ctx, bool mock) : ctx_(ctx), mock_(mock), pool_(mock) {
  max_steps_ = ctx_->opt.max_inflight > 0 ? (size_t)ctx_->opt.max_inflight : kDefaultSteps;
  if (mock_) {  // test hook: simulated steps take this long, so tests can act on queued requests
    const char* s = std::getenv("QSIM_TEST_MOCK_STEP_MS");
    mock_step_ms_ = s ? std::max(0, std::atoi(s)) : 0;
  }
  if (!mock_) {
    (void)hipSetDevice(ctx_->device);
    (void)hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
  }
  ok_ = ring_.init(kRingBytes, mock_);
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
    for (hipEvent_t e : free_events_) (void)hipEventDestroy(e);
    pool_.trim(0);
    d_items_.release();
    (void)hipStreamDestroy(stream_);
  }
}

// Device bytes of a request while admitted: exactly the blocks admit() takes
// from the pool (plan descriptors, states, coefficients, partial sums,
// results), computed from its plans once they are built.
static void plan_block_sizes(const Plan& p, ReqPlan& d) {
  d.bp = std::max<size_t>(1, p.passes.size()) * sizeof(PassDesc);
  d.bs = std::max<size_t>(1, p.stages.size()) * sizeof(StageDesc);
  d.bo = std::max<size_t>(1, p.ops.size()) * sizeof(DevOp);
}

static void request_sizes(SReq* r) {
  const Plan& F = r->fplan;
  plan_block_sizes(F, r->df);
  r->state_bytes = ((size_t)1 << r->c.n) * 8;
  r->cf_bytes = r->coef_f.size() * sizeof(float);
  r->meas_bytes = std::max<size_t>(1, (size_t)F.n_meas << (F.n - F.m)) * sizeof(double);
  size_t ns = 0;
  size_t bytes = r->df.bp + r->df.bs + r->df.bo + r->state_bytes + r->cf_bytes + r->meas_bytes;
  if (r->want_grad) {
    const Plan& P = r->ap->plan;
    ns = P.n_gslots;
    plan_block_sizes(r->hplan, r->dh);
    r->ca_bytes = r->coef_a.size() * sizeof(float);
    r->gpart_bytes = std::max<size_t>(1, ns << (P.n - P.m)) * sizeof(double);
    bytes += r->dh.bp + r->dh.bs + r->dh.bo + r->state_bytes + r->ca_bytes + r->gpart_bytes;
  }
  r->res_bytes = (1 + ns + (size_t)r->c.n_params) * sizeof(double);
  r->footprint = bytes + r->res_bytes;
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
  // the states alone bound the footprint from below: reject before planning
  r->footprint = (r->want_grad ? 2 : 1) * ((size_t)1 << r->c.n) * 8;
  auto admissible = [&]() -> int {
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
    return QSIM_OK;
  };
  {
    std::lock_guard<std::mutex> g(mu_);
    if ((rc = admissible())) return rc;
  }
  // Host preparation runs here, in the caller's thread, so the scheduler never
  // waits for it: plans (gate passes from the structure cache) and coefficients.
  if (!mock_) (void)hipSetDevice(ctx_->device);
  if ((rc = host_forward_plan(ctx_, r->c, r->terms, r->want_grad, r->fplan))) return rc;
  const int64_t crs_f = (int64_t)std::max<size_t>(1, r->fplan.slots.size()) * 8;
  r->coef_f.resize((size_t)crs_f);
  build_coefficients<float>(r->c, r->fplan.slots, r->params.data(), 1, crs_f, r->coef_f.data());
  if (r->want_grad) {
    if ((rc = host_happly_plan(ctx_, r->c.n, r->terms, r->hplan))) return rc;
    r->ap = get_adjoint_plan(ctx_, r->c, 0, rc);
    if (!r->ap) return rc;
    const int64_t crs_a = (int64_t)std::max<size_t>(1, r->ap->plan.slots.size()) * 8;
    r->coef_a.resize((size_t)crs_a);
    build_coefficients<float>(r->c, r->ap->plan.slots, r->params.data(), 1, crs_a, r->coef_a.data());
    for (int p : r->ap->plan.gslot_param) r->np_used = std::max(r->np_used, p + 1);
  }
  request_sizes(r.get());
  std::lock_guard<std::mutex> g(mu_);
  if ((rc = admissible())) return rc;
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
  out->pool_outstanding_bytes = pool_.outstanding();
  out->queued = queue_.size();
  out->running = running_.size();
}

// Pinned ring space; when the ring is full, the oldest steps in flight are
// retired until it fits (nullptr only if it cannot fit at all).
void* Server::ring_alloc(size_t bytes) {
  while (true) {
    void* p = ring_.alloc(bytes);
    if (p || steps_.empty()) return p;
    retire(steps_.front());
    steps_.pop_front();
  }
}

// Copies host bytes through the pinned ring into device memory, asynchronously
// on the server stream; the ring space is reclaimed when the current step retires.
void* Server::stage_upload(const void* src, size_t bytes, void* dst) {
  if (bytes == 0) return dst;
  void* h = ring_alloc(bytes);
  if (!h) return nullptr;
  std::memcpy(h, src, bytes);
  if (!mock_ && hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, stream_) != hipSuccess) return nullptr;
  return dst;
}

int Server::admit(SReq* r) {
  r->admitted = true;  // from here on release() gives back whatever was taken
  auto plan_blocks = [&](const Plan& p, ReqPlan& d) {  // sizes from request_sizes()
    (void)p;
    d.P = static_cast<PassDesc*>(pool_.get(d.bp));
    d.S = static_cast<StageDesc*>(pool_.get(d.bs));
    d.O = static_cast<DevOp*>(pool_.get(d.bo));
    return d.P && d.S && d.O;
  };
  auto upload_plan = [&](const Plan& p, const ReqPlan& d) {
    return stage_upload(p.passes.data(), p.passes.size() * sizeof(PassDesc), d.P) &&
           stage_upload(p.stages.data(), p.stages.size() * sizeof(StageDesc), d.S) &&
           stage_upload(p.ops.data(), p.ops.size() * sizeof(DevOp), d.O);
  };
  const Plan& F = r->fplan;
  bool ok = plan_blocks(F, r->df);
  r->A = pool_.get(r->state_bytes);
  r->cf = pool_.get(r->cf_bytes);
  r->meas = static_cast<double*>(pool_.get(r->meas_bytes));
  ok = ok && r->A && r->cf && r->meas;
  if (r->want_grad) {
    ok = plan_blocks(r->hplan, r->dh) && ok;
    r->B = pool_.get(r->state_bytes);
    r->ca = pool_.get(r->ca_bytes);
    r->gpart = static_cast<double*>(pool_.get(r->gpart_bytes));
    ok = ok && r->B && r->ca && r->gpart;
  }
  r->res = static_cast<double*>(pool_.get(r->res_bytes));
  if (!ok || !r->res) {
    set_error(ctx_, "serving: device allocation failed");
    return QSIM_ENOMEM;
  }
  bool up = upload_plan(F, r->df) && stage_upload(r->coef_f.data(), r->cf_bytes, r->cf);
  if (up && r->want_grad) up = upload_plan(r->hplan, r->dh) && stage_upload(r->coef_a.data(), r->ca_bytes, r->ca);
  if (!up) {
    set_error(ctx_, "serving: staging upload failed");
    return QSIM_ENOMEM;
  }
  r->phase = PH_FWD;
  r->next = 0;
  return QSIM_OK;
}

void Server::release(SReq* r) {
  if (!r->admitted) return;
  for (ReqPlan* d : {&r->df, &r->dh}) {
    pool_.put(d->P, d->bp);
    pool_.put(d->S, d->bs);
    pool_.put(d->O, d->bo);
    *d = ReqPlan();
  }
  pool_.put(r->A, r->state_bytes);
  pool_.put(r->B, r->state_bytes);
  pool_.put(r->cf, r->cf_bytes);
  pool_.put(r->ca, r->ca_bytes);
  pool_.put(r->meas, r->meas_bytes);
  pool_.put(r->gpart, r->gpart_bytes);
  pool_.put(r->res, r->res_bytes);
  r->A = r->B = r->cf = r->ca = nullptr;
  r->meas = r->gpart = r->res = nullptr;
  r->h_res = nullptr;
  r->admitted = false;
  // keep the pool within the memory budget
  const size_t budget = ctx_->opt.hbm_budget_bytes;
  const size_t limit = budget > inflight_ ? budget - inflight_ : 0;
  if (pool_.cached() > limit) pool_.trim(limit);
}

// Launches the next pass of every request in 'run' (one multi-request launch
// per kernel kind).  Requests whose last pass this was get their reductions and
// result copies queued behind it and move to st.finishing; 'run' keeps the rest.
int Server::launch_step(std::vector<SReq*>& run, Step& st) {
  std::vector<PassItem> single, dual;  // single-state (forward) and dual-state passes
  int64_t tiles_s = 0, tiles_d = 0;
  int m_s = 4, m_d = 4, r_s = 0, r_d = 0;
  std::vector<SReq*> still;
  for (SReq* r : run) {
    if (r->failed || r->cancelled) {
      st.finishing.push_back(r);
      continue;
    }
    const bool fwd = r->phase == PH_FWD;
    const Plan& P = fwd ? r->fplan : r->phase == PH_HAPPLY ? r->hplan : r->ap->plan;
    PassItem it;
    if (r->phase == PH_ADJ) {
      it.pass = r->ap->d_passes + r->next;
      it.stages = r->ap->d_stages;
      it.ops = r->ap->d_ops;
    } else {
      const ReqPlan& d = fwd ? r->df : r->dh;
      it.pass = d.P + r->next;
      it.stages = d.S;
      it.ops = d.O;
    }
    it.A = r->A;
    it.B = r->B;
    it.coef = fwd ? r->cf : r->ca;
    it.meas = r->meas;
    it.grad = r->gpart;
    const int64_t tiles = 1ll << (P.n - P.m);
    if (fwd) {
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
    if (++r->next < (int)P.passes.size()) {
      still.push_back(r);
    } else if (r->phase == PH_FWD && r->want_grad) {
      r->phase = PH_HAPPLY;
      r->next = 0;
      still.push_back(r);
    } else if (r->phase == PH_HAPPLY) {
      r->phase = PH_ADJ;
      r->next = 0;
      still.push_back(r);
    } else {
      r->phase = PH_DONE;
      st.finishing.push_back(r);
    }
  }
  const size_t n_single = single.size();
  std::vector<PassItem>& items = single;
  items.insert(items.end(), dual.begin(), dual.end());
  run.swap(still);
  if (!mock_ && !items.empty()) {
    const size_t bytes = items.size() * sizeof(PassItem);
    if (d_items_.bytes < bytes) {
      // earlier steps may still read the buffer
      if (hipStreamSynchronize(stream_) != hipSuccess || d_items_.ensure(2 * bytes) != hipSuccess)
        return QSIM_EDEVICE;
    }
    // steps run in stream order, so this copy lands after the previous step's kernels
    if (!stage_upload(items.data(), bytes, d_items_.p)) return QSIM_ENOMEM;
    const PassItem* d = static_cast<const PassItem*>(d_items_.p);
    const int n_dual = (int)(items.size() - n_single);
    if (n_single && launch_pass_multi(d, (int)n_single, tiles_s, m_s, r_s, 0, 0, stream_) != hipSuccess)
      return QSIM_EDEVICE;
    if (n_dual && launch_pass_multi(d + n_single, n_dual, tiles_d, m_d, r_d, 0, 1, stream_) != hipSuccess)
      return QSIM_EDEVICE;
    st_.launches += (n_single ? 1 : 0) + (n_dual ? 1 : 0);
  }
  if (!mock_) {
    for (SReq* r : st.finishing) {
      if (r->failed || r->cancelled || r->phase != PH_DONE) continue;
      r->h_res = static_cast<double*>(ring_alloc((1 + (size_t)r->np_used) * sizeof(double)));
      if (!r->h_res) return QSIM_ENOMEM;
      const Plan& F = r->fplan;
      if (launch_reduce_rows(r->meas, 1, (int64_t)F.n_meas << (F.n - F.m), F.const_term, r->res, stream_) !=
          hipSuccess)
        return QSIM_EDEVICE;
      if (r->want_grad && r->np_used > 0) {
        const Plan& P = r->ap->plan;
        const int ns = P.n_gslots;
        double* slot_total = r->res + 1;
        double* g = r->res + 1 + ns;
        if (launch_reduce_rows(r->gpart, ns, 1ll << (P.n - P.m), 0.0, slot_total, stream_) != hipSuccess ||
            launch_grad_scatter(slot_total, 1, ns, r->ap->d_poff, r->ap->d_pslots, r->np_used, g, stream_) !=
                hipSuccess ||
            hipMemcpyAsync(r->h_res + 1, g, sizeof(double) * r->np_used, hipMemcpyDeviceToHost, stream_) !=
                hipSuccess)
          return QSIM_EDEVICE;
      }
      if (hipMemcpyAsync(r->h_res, r->res, sizeof(double), hipMemcpyDeviceToHost, stream_) != hipSuccess)
        return QSIM_EDEVICE;
    }
    if (free_events_.empty()) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return QSIM_EDEVICE;
      free_events_.push_back(e);
    }
    st.ev = free_events_.back();
    free_events_.pop_back();
    if (hipEventRecord(st.ev, stream_) != hipSuccess) return QSIM_EDEVICE;
  }
  return QSIM_OK;
}

// Waits for a step's work and publishes the requests that finished in it.
void Server::retire(Step& st) {
  bool ok = ok_;
  if (!mock_ && st.ev) {
    ok = ok && hipEventSynchronize(st.ev) == hipSuccess;
    free_events_.push_back(st.ev);
    st.ev = nullptr;
  }
  if (!ok) ok_ = false;
  std::lock_guard<std::mutex> g(mu_);
  st_.steps++;
  for (SReq* r : st.finishing) {
    if (!ok && !r->failed) {
      r->failed = true;
      r->status = QSIM_EDEVICE;
    }
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
        if (!mock_)
          for (int k = 0; k < r->np_used; ++k) r->grad[k] = r->h_res[1 + k];
      }
      st_.completed++;
    }
    inflight_ -= r->footprint;
    release(r);
    r->t_done = now_s();
    r->done = true;
  }
  // everything staged up to this step's launch has been consumed
  ring_.release_to(st.ring_mark);
}

void Server::loop() {
  if (!mock_) (void)hipSetDevice(ctx_->device);
  const size_t budget = ctx_->opt.hbm_budget_bytes;
  auto retire_front = [&] {
    retire(steps_.front());
    steps_.pop_front();
  };
  std::vector<SReq*> run;  // admitted requests still launching passes (scheduler-owned copy of running_)
  while (true) {
    while (!steps_.empty() && (mock_ || hipEventQuery(steps_.front().ev) != hipErrorNotReady)) retire_front();
    std::vector<SReq*> fresh;
    {
      std::unique_lock<std::mutex> lk(mu_);
      if (run.empty() && steps_.empty()) cv_.wait(lk, [&] { return stop_ || !queue_.empty(); });
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
    }
    for (SReq* r : fresh) {
      const int rc = admit(r);
      if (rc) {
        r->failed = true;
        r->status = rc;
      }
      run.push_back(r);
      if (pool_.outstanding() > inflight_) {  // accounting check: the budget covers every block handed out
        std::lock_guard<std::mutex> g(mu_);
        st_.accounting_violations++;
      }
    }
    if (!run.empty()) {
      Step st;
      if (launch_step(run, st) != QSIM_OK) ok_ = false;
      st.ring_mark = ring_.mark();
      {
        std::lock_guard<std::mutex> g(mu_);
        for (SReq* r : st.finishing) running_.erase(std::find(running_.begin(), running_.end(), r));
      }
      steps_.push_back(std::move(st));
      if (mock_ && mock_step_ms_ > 0) std::this_thread::sleep_for(std::chrono::milliseconds(mock_step_ms_));
    }
    // bound the steps in flight; with nothing left to launch, wait for the oldest
    if (!steps_.empty() && (mock_ || steps_.size() >= max_steps_ || run.empty())) retire_front();
  }
  // shutdown: launched work finishes normally, everything else ends with ESHUTDOWN
  while (!steps_.empty()) retire_front();
  std::lock_guard<std::mutex> g(mu_);
  for (SReq* r : running_) {
    inflight_ -= r->footprint;
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
