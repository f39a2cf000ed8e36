// Mock-executor, fake-clock test of the serving scheduler (host-only).
// Requests arrive on a simulated clock (Poisson arrivals, log-uniform sizes
// 1..max_batch from a fixed-seed generator); a mock executor completes each
// batch after a service time that grows with its rows.  After every event
// the invariants are checked: a lane holds at most one batch; a batch's rows
// fit max_batch and its requests max_requests; slots are unique and never
// lost; requests leave the queue in submission order; every request
// completes exactly once.  Exit status 0 when everything holds.
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <vector>

#include "../paper_2306_08792_amd/csrc/scheduler.h"

using gcr::SchedBatch;
using gcr::SchedConfig;
using gcr::Scheduler;

static int failures = 0;
#define CHECK(c, ...)                         \
  do {                                        \
    if (!(c)) {                               \
      ++failures;                             \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);           \
      fprintf(stderr, "\n");                  \
      return;                                 \
    }                                         \
  } while (0)

struct Rng {  // 64-bit LCG + xorshift output, fixed seed
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed * 6364136223846793005ull + 1442695040888963407ull) {}
  double uniform() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    uint64_t x = s ^ (s >> 29);
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
  }
};

static void run(const SchedConfig& c, int nreq, double rate, uint64_t seed) {
  Scheduler s(c);
  Rng rng(seed);
  // rejected sizes
  CHECK(!s.push(999999, 0), "b = 0 accepted");
  CHECK(!s.push(999998, c.max_batch + 1), "b > max_batch accepted");
  std::vector<double> arrival(nreq);
  std::vector<int> size(nreq);
  double t = 0.0;
  for (int i = 0; i < nreq; ++i) {
    t += -std::log(1.0 - rng.uniform()) / rate;
    arrival[i] = t;
    size[i] = std::min(c.max_batch, std::max(1, (int)std::floor(std::exp(rng.uniform() * std::log(c.max_batch + 1.0)))));
  }
  std::map<int, std::pair<double, SchedBatch>> running;  // lane -> (finish time, batch)
  std::vector<int> done(nreq, 0);
  std::vector<double> finish_at(nreq, 0.0);
  uint64_t next_out = 0;  // submission order check
  int next_in = 0, completed = 0;
  double now = 0.0;
  std::set<int> held;
  auto check_slots = [&](void) -> bool {
    return (int)held.size() + s.free_slots() == c.slots;
  };
  while (completed < nreq) {
    // next event: an arrival or a completion, whichever is first
    double t_arr = next_in < nreq ? arrival[next_in] : INFINITY;
    double t_fin = INFINITY;
    int lane_fin = -1;
    for (auto& kv : running)
      if (kv.second.first < t_fin) {
        t_fin = kv.second.first;
        lane_fin = kv.first;
      }
    if (t_arr <= t_fin) {
      now = t_arr;
      CHECK(s.push((uint64_t)next_in, size[next_in]), "push refused");
      ++next_in;
    } else {
      now = t_fin;
      SchedBatch& b = running[lane_fin].second;
      for (const auto& it : b.items) {
        CHECK(!done[it.ticket], "ticket %llu completed twice", (unsigned long long)it.ticket);
        done[it.ticket] = 1;
        finish_at[it.ticket] = now;
        held.erase(it.slot);
        ++completed;
      }
      s.finish(lane_fin);
      running.erase(lane_fin);
      CHECK(check_slots(), "slots lost after finish");
    }
    SchedBatch b;
    while (s.next(&b)) {
      CHECK(b.lane >= 0 && b.lane < c.lanes, "bad lane %d", b.lane);
      CHECK(!running.count(b.lane), "lane %d given two batches", b.lane);
      CHECK(!b.items.empty(), "empty batch");
      CHECK(b.rows <= c.max_batch, "batch of %d rows", b.rows);
      CHECK((int)b.items.size() <= c.max_requests, "batch of %zu requests", b.items.size());
      int rows = 0;
      for (const auto& it : b.items) {
        CHECK(it.ticket == next_out, "ticket %llu out of order (expected %llu)", (unsigned long long)it.ticket,
              (unsigned long long)next_out);
        ++next_out;
        CHECK(it.row0 == rows, "row offsets not packed");
        rows += it.b;
        CHECK(it.slot >= 0 && it.slot < c.slots, "slot %d out of range", it.slot);
        CHECK(!held.count(it.slot), "slot %d given twice", it.slot);
        held.insert(it.slot);
      }
      CHECK(rows == b.rows, "rows do not add up");
      CHECK(check_slots(), "slots lost after next");
      // mock executor: a fixed launch cost plus a cost per row
      running[b.lane] = {now + 1e-3 + 2e-6 * b.rows, b};
    }
  }
  CHECK(next_in == nreq && s.pending() == 0 && running.empty(), "not drained");
  CHECK(s.free_lanes() == c.lanes && s.free_slots() == c.slots, "resources not returned");
  std::vector<double> lat(nreq);
  for (int i = 0; i < nreq; ++i) lat[i] = finish_at[i] - arrival[i];
  std::sort(lat.begin(), lat.end());
  printf("lanes %d max_batch %d max_requests %d slots %d: %d requests, p50 %.3f ms p99 %.3f ms\n", c.lanes,
         c.max_batch, c.max_requests, c.slots, nreq, 1e3 * lat[nreq / 2], 1e3 * lat[(nreq * 99) / 100]);
}

static void drain_case() {
  SchedConfig c;
  c.lanes = 1;
  c.max_batch = 8;
  c.max_requests = 2;
  c.slots = 2;
  Scheduler s(c);
  for (int i = 0; i < 5; ++i) s.push(i, 3);
  SchedBatch b;
  CHECK(s.next(&b) && b.items.size() == 2 && b.rows == 6, "first batch");
  CHECK(!s.next(&b), "second lane does not exist");
  std::vector<uint64_t> d = s.drain();
  CHECK(d.size() == 3 && d[0] == 2 && d[2] == 4, "drain order");
  s.finish(0);
  CHECK(s.free_slots() == 2 && s.free_lanes() == 1 && !s.next(&b), "after finish");
  s.finish(0);  // finishing an idle lane changes nothing
  CHECK(s.free_slots() == 2, "double finish");
  // the head request never waits behind a later one
  s.push(10, 7);
  s.push(11, 2);
  s.push(12, 1);  // would fit beside 10, but must not pass 11
  CHECK(s.next(&b) && b.items.size() == 1 && b.items[0].ticket == 10, "head first");
  s.finish(0);
  CHECK(s.next(&b) && b.items.size() == 2 && b.items[0].ticket == 11 && b.items[1].ticket == 12, "then in order");
}

int main() {
  SchedConfig a;  // defaults
  run(a, 20000, 400.0, 1);
  SchedConfig one;
  one.lanes = 1;
  one.max_batch = 1;
  one.max_requests = 1;
  one.slots = 1;
  run(one, 2000, 100.0, 2);
  SchedConfig scarce;  // memory for fewer request slots than lanes x requests
  scarce.lanes = 4;
  scarce.max_batch = 512;
  scarce.max_requests = 16;
  scarce.slots = 6;
  run(scarce, 20000, 2000.0, 3);
  SchedConfig wide;
  wide.lanes = 3;
  wide.max_batch = 64;
  wide.max_requests = 64;
  wide.slots = 256;
  run(wide, 20000, 5000.0, 4);
  drain_case();
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("scheduler ok\n");
  return 0;
}
