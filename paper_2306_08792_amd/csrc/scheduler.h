// Continuous batching of serving requests (host-only C++, no HIP).
//
// A server keeps `lanes` batches on the device at once.  Requests wait in
// FIFO order; whenever a lane is free, the scheduler forms a batch from the
// head of the queue: requests are taken while their query rows fit the
// lane's query region (max_batch rows), the batch holds at most
// max_requests requests, and each request gets one of `slots` request
// scratch slots (the per-request device memory a server sizes from its
// memory budget).  A request never waits behind a later one (no skipping
// ahead), so none starves; a 1-query request takes one row, not a partition.
// Finishing a batch frees its lane and its slots.  The class is not
// thread-safe: the server calls it under its own lock.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <vector>

namespace gcr {

struct SchedConfig {
  int lanes = 2;          // batches in flight
  int max_batch = 512;    // query rows of one batch
  int max_requests = 16;  // requests of one batch
  int slots = 32;         // request scratch slots in all
};

struct SchedItem {
  uint64_t ticket = 0;
  int b = 0;     // query rows
  int row0 = 0;  // first row in the batch
  int slot = 0;  // request scratch slot
};

struct SchedBatch {
  int lane = -1;
  int rows = 0;
  std::vector<SchedItem> items;
};

class Scheduler {
 public:
  explicit Scheduler(const SchedConfig& c);
  // Queue a request of b query rows (1 <= b <= max_batch); false otherwise.
  bool push(uint64_t ticket, int b);
  // Form the next batch if a lane is free and the head request fits; the
  // lane and the slots are taken until finish(lane).
  bool next(SchedBatch* out);
  // The batch of `lane` completed.
  void finish(int lane);
  // Remove and return every queued request (not the ones in batches).
  std::vector<uint64_t> drain();
  size_t pending() const { return queue_.size(); }
  int free_lanes() const;
  int free_slots() const { return (int)free_slots_.size(); }
  int busy_lanes() const { return cfg_.lanes - free_lanes(); }
  const SchedConfig& config() const { return cfg_; }

 private:
  struct Pending {
    uint64_t ticket;
    int b;
  };
  SchedConfig cfg_;
  std::deque<Pending> queue_;
  std::vector<int> free_slots_;
  std::vector<std::vector<int>> lane_slots_;  // slots held by each lane's batch
  std::vector<char> lane_busy_;
};

}  // namespace gcr
