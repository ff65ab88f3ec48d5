// Serving loop: requests of mixed sizes share the GPU by continuous batching
// at pass granularity.  Every scheduler step launches, for each running
// request, its next pass, all in one multi-request kernel launch per kernel
// kind.  Requests are admitted FIFO while their device footprint fits the
// budget and leave (freeing their memory) as soon as their last pass and
// reduction are done, so new arrivals join at the next step.
//
// Host work is kept off the device's critical path: plans and coefficients
// are prepared by the submitting thread; the scheduler only takes pooled
// device blocks, uploads through a pinned ring buffer, and keeps up to a few
// steps in flight, noticing finished steps through events.
#pragma once
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

namespace qsim {

struct SReq;

double now_s();

// Size-keyed cache of device blocks, so steady-state serving does not call
// hipMalloc/hipFree per request.
class BlockPool {
 public:
  explicit BlockPool(bool mock) : mock_(mock) {}
  ~BlockPool();
  void* get(size_t bytes);
  void put(void* p, size_t bytes);
  void trim(size_t keep_bytes);
  size_t cached() const { return cached_; }
  // bytes handed out and not yet returned (read by other threads for statistics)
  size_t outstanding() const { return out_.load(std::memory_order_relaxed); }

 private:
  bool mock_;
  std::multimap<size_t, void*> free_;
  size_t cached_ = 0;
  std::atomic<size_t> out_{0};
  uintptr_t fake_ = 0x1000;
};

// Pinned host staging used as a ring: allocations are released in order
// once the step that consumed them has finished on the device.
class PinnedRing {
 public:
  ~PinnedRing();
  bool init(size_t bytes, bool mock);
  void* alloc(size_t bytes);  // nullptr when full
  uint64_t mark() const { return head_; }
  void release_to(uint64_t mark) { tail_ = mark; }
  bool empty() const { return head_ == tail_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0;
  uint64_t head_ = 0, tail_ = 0;  // monotonic byte counters
  bool mock_ = false;
};

class Server {
 public:
  Server(qsim_ctx* ctx, bool mock);
  ~Server();
  int submit(const qsim_request* r, uint64_t* ticket);
  int poll(uint64_t ticket, double* E, double* grad, double* times);
  int cancel(uint64_t ticket);
  void stats(qsim_server_stats* out);

 private:
  struct Step {
    hipEvent_t ev = nullptr;
    uint64_t ring_mark = 0;
    std::vector<SReq*> finishing;
  };
  void loop();
  int admit(SReq* r);               // device blocks and uploads
  void release(SReq* r);
  int launch_step(std::vector<SReq*>& run, Step& st);
  void retire(Step& st);            // wait for a step, publish its finished requests
  void* ring_alloc(size_t bytes);
  void* stage_upload(const void* src, size_t bytes, void* dst);

  qsim_ctx* ctx_;
  int mock_step_ms_ = 0;  // simulated step time (test hook)
  bool mock_;
  hipStream_t stream_ = nullptr;
  std::thread thread_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
  uint64_t next_ticket_ = 1;
  std::deque<SReq*> queue_;
  std::vector<SReq*> running_;      // admitted, still launching passes
  std::unordered_map<uint64_t, std::unique_ptr<SReq>> all_;
  size_t inflight_ = 0, peak_ = 0;
  qsim_server_stats st_{};
  BlockPool pool_;
  PinnedRing ring_;
  std::deque<Step> steps_;          // launched, not yet retired
  std::vector<hipEvent_t> free_events_;
  DevBuf d_items_;                  // pass items of the step being launched
  bool ok_ = true;
  size_t max_steps_ = 3;            // steps in flight (context option max_inflight)
};

}  // namespace qsim
