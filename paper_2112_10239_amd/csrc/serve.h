// Serving loop: requests of mixed sizes share the GPU by continuous batching
// at pass granularity.  Every scheduler step launches, for each running
// request, its next pass, all in one multi-request kernel launch per kernel
// kind; requests are admitted FIFO while their device footprint fits the
// budget, and leave (freeing their memory) as soon as their last pass and
// reduction are done, so new arrivals join at the next step.
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

 private:
  bool mock_;
  std::multimap<size_t, void*> free_;
  size_t cached_ = 0;
  uintptr_t fake_ = 0x1000;
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
  void loop();
  int prepare(SReq* r);
  void release(SReq* r);
  bool step(std::vector<SReq*>& run);

  qsim_ctx* ctx_;
  bool mock_;
  hipStream_t stream_ = nullptr;
  std::thread thread_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
  uint64_t next_ticket_ = 1;
  std::deque<SReq*> queue_;
  std::vector<SReq*> running_;
  std::unordered_map<uint64_t, std::unique_ptr<SReq>> all_;
  size_t inflight_ = 0, peak_ = 0;
  qsim_server_stats st_{};
  BlockPool pool_;
  Workspace ws_;        // pinned staging for coefficients
  DevBuf d_items_;
  std::vector<PassItem> items_;
};

}  // namespace qsim
