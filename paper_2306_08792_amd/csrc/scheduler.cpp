// Continuous batching of serving requests; see scheduler.h.
#include "scheduler.h"

#include <algorithm>

namespace gcr {

Scheduler::Scheduler(const SchedConfig& c) : cfg_(c) {
  cfg_.lanes = std::max(1, cfg_.lanes);
  cfg_.max_batch = std::max(1, cfg_.max_batch);
  cfg_.max_requests = std::max(1, cfg_.max_requests);
  cfg_.slots = std::max(1, cfg_.slots);
  // lowest slot numbers first
  for (int s = cfg_.slots - 1; s >= 0; --s) free_slots_.push_back(s);
  lane_slots_.assign(cfg_.lanes, {});
  lane_busy_.assign(cfg_.lanes, 0);
}

bool Scheduler::push(uint64_t ticket, int b) {
  if (b < 1 || b > cfg_.max_batch) return false;
  queue_.push_back({ticket, b});
  return true;
}

int Scheduler::free_lanes() const {
  int n = 0;
  for (char x : lane_busy_) n += x ? 0 : 1;
  return n;
}

bool Scheduler::next(SchedBatch* out) {
  if (queue_.empty() || free_slots_.empty()) return false;
  int lane = -1;
  for (int l = 0; l < cfg_.lanes; ++l)
    if (!lane_busy_[l]) {
      lane = l;
      break;
    }
  if (lane < 0) return false;
  out->lane = lane;
  out->rows = 0;
  out->items.clear();
  while (!queue_.empty() && !free_slots_.empty() && (int)out->items.size() < cfg_.max_requests &&
         out->rows + queue_.front().b <= cfg_.max_batch) {
    SchedItem it;
    it.ticket = queue_.front().ticket;
    it.b = queue_.front().b;
    it.row0 = out->rows;
    it.slot = free_slots_.back();
    free_slots_.pop_back();
    lane_slots_[lane].push_back(it.slot);
    out->rows += it.b;
    out->items.push_back(it);
    queue_.pop_front();
  }
  lane_busy_[lane] = 1;
  return true;
}

void Scheduler::finish(int lane) {
  if (lane < 0 || lane >= cfg_.lanes || !lane_busy_[lane]) return;
  for (int s : lane_slots_[lane]) free_slots_.push_back(s);
  std::sort(free_slots_.begin(), free_slots_.end(), [](int a, int b) { return a > b; });
  lane_slots_[lane].clear();
  lane_busy_[lane] = 0;
}

std::vector<uint64_t> Scheduler::drain() {
  std::vector<uint64_t> t;
  for (const Pending& p : queue_) t.push_back(p.ticket);
  queue_.clear();
  return t;
}

}  // namespace gcr
