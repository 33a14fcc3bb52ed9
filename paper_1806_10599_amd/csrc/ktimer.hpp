// Live kernel timing: HIP events taken by the launches of selected kernel
// classes inside the solver's own iteration (the kernel's own start and end
// through the extended launch; event-record nodes around the kernels of
// captured CG graphs), summed after each stream synchronisation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <vector>

#include "common.hpp"

namespace rve {

class KernelTimer {
 public:
  static constexpr int kClasses = 8;
  using Pair = std::pair<int, std::pair<hipEvent_t, hipEvent_t>>;

  ~KernelTimer() { release(); }

  uint32_t mask() const { return mask_; }
  void set_mask(uint32_t m) { mask_ = m & ((1u << kClasses) - 1); }
  bool on(int k) const { return (mask_ >> k) & 1u; }
  // direct launches of the classes in `sampled` are timed one in every
  // `stride` (per class, from the first), the others every launch
  void set_stride(int stride, uint32_t sampled) {
    stride_ = stride < 1 ? 1 : stride;
    sampled_ = sampled;
    for (int k = 0; k < kClasses; ++k) seq_[k] = 0;
  }
  int stride() const { return stride_; }

  // times the next kernel launched through rve::launch as class k (no-op
  // when k is off or not sampled this time): the launch records the events
  // itself
  void begin(int k, hipStream_t) {
    active_ = false;
    if (!on(k)) return;
    ++seen_[k];
    if (((sampled_ >> k) & 1u) && (seq_[k]++ % stride_) != 0) return;
    active_ = true;
    open_ = take();
    close_ = take();
    g_next_launch_events = NextLaunchEvents{open_, close_};
  }
  void end(int k, hipStream_t) {
    if (!on(k) || !active_) return;
    active_ = false;
    if (g_next_launch_events.start) {
      g_next_launch_events = NextLaunchEvents{};
      throw Error(-1, "timed kernel class was not launched through rve::launch");
    }
    pending_.push_back(Pair{k, {open_, close_}});
  }
  // times everything between the two calls on stream s as class k (for
  // classes made of several kernels)
  void begin_span(int k, hipStream_t s) {
    if (!on(k)) return;
    open_ = take();
    RVE_HIP(hipEventRecord(open_, s));
  }
  void end_span(int k, hipStream_t s) {
    if (!on(k)) return;
    hipEvent_t e = take();
    RVE_HIP(hipEventRecord(e, s));
    pending_.push_back(Pair{k, {open_, e}});
  }

  // a pair of events for the event-record nodes of a graph; the graph's
  // pairs are queued again after each replay
  Pair graph_pair(int k) {
    hipEvent_t a = take();
    hipEvent_t b = take();
    return Pair{k, {a, b}};
  }
  void replayed(const std::vector<Pair>& pairs) {
    for (const Pair& p : pairs) replay_.push_back(p);
  }

  // after the stream has been synchronised: accumulate, recycle
  void flush() {
    for (auto* q : {&pending_, &replay_}) {
      for (const Pair& p : *q) {
        float t = 0.f;
        RVE_HIP(hipEventElapsedTime(&t, p.second.first, p.second.second));
        ms_[p.first] += (double)t;
        count_[p.first] += 1;
      }
    }
    for (const Pair& p : pending_) {
      free_.push_back(p.second.first);
      free_.push_back(p.second.second);
    }
    pending_.clear();
    replay_.clear();
  }

  // summed ms and counts of the timed launches; `seen`: every direct
  // launch of a timed class, sampled or not (graph replays not included)
  void read(double* ms, int64_t* count, int n, bool reset,
            int64_t* seen = nullptr) {
    for (int k = 0; k < n && k < kClasses; ++k) {
      if (ms) ms[k] = ms_[k];
      if (count) count[k] = count_[k];
      if (seen) seen[k] = seen_[k];
    }
    if (reset)
      for (int k = 0; k < kClasses; ++k) {
        ms_[k] = 0.0;
        count_[k] = 0;
        seen_[k] = 0;
      }
  }

  // events of a destroyed graph go back to the pool
  void recycle(std::vector<Pair>& pairs) {
    for (const Pair& p : pairs) {
      free_.push_back(p.second.first);
      free_.push_back(p.second.second);
    }
    pairs.clear();
  }

  void release() {
    for (hipEvent_t e : all_) hipEventDestroy(e);
    all_.clear();
    free_.clear();
    pending_.clear();
    replay_.clear();
  }

 private:
  hipEvent_t take() {
    if (free_.empty()) {
      hipEvent_t e;
      RVE_HIP(hipEventCreate(&e));
      all_.push_back(e);
      return e;
    }
    hipEvent_t e = free_.back();
    free_.pop_back();
    return e;
  }

  uint32_t mask_ = 0;
  int stride_ = 1;
  uint32_t sampled_ = 0;
  int64_t seq_[kClasses] = {};
  int64_t seen_[kClasses] = {};
  bool active_ = false;
  hipEvent_t open_ = nullptr, close_ = nullptr;
  std::vector<hipEvent_t> all_, free_;
  std::vector<Pair> pending_, replay_;
  double ms_[kClasses] = {};
  int64_t count_[kClasses] = {};
};

}  // namespace rve
