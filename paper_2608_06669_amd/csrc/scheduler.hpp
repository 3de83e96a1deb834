// Admission, slot accounting and request lifetime of the serving loop
// (include/pnkcc.h, "Serving"), free of any HIP call so that it can be built
// and checked on the host alone (a ThreadSanitizer test drives it with
// fake solves).
//
// Requests queue in arrival order. A worker asks for work with take(); it
// is given the first queued request whose device footprint fits in the
// unused part of the budget. A request may be passed over by later, smaller
// ones at most `max_overtake` times; after that nothing behind it is
// admitted before it (no starvation of large requests). complete() returns
// the footprint and wakes the waiting workers. hold()/unhold() count device
// memory kept between requests (cached engines) against the same budget;
// take() lets the caller free such memory when a queued request does not
// fit. release() hands a finished
// request's payload to the caller and drops it, keeping only its times and
// status, so a long stream holds host memory only for requests in flight or
// finished and not yet collected.
#pragma once

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>

namespace pnk {

template <class Payload>
class Scheduler {
 public:
  enum class State { Queued, Running, Done };
  struct Entry {
    uint64_t id = 0;
    size_t footprint = 0;
    State state = State::Queued;
    int status = 0;
    int overtaken = 0;
    uint64_t admit_seq = 0;  // order of admission (1, 2, ...)
    double t_submit = 0, t_admit = 0, t_finish = 0;
    std::unique_ptr<Payload> payload;
  };
  struct Times {
    double t_submit = 0, t_admit = 0, t_finish = 0;
    int status = 0;
  };
  struct Stats {
    uint64_t queued = 0, running = 0, finished = 0, rejected = 0;
    size_t bytes_in_use = 0, peak_bytes = 0, budget = 0;
    int peak_running = 0;
    size_t held_payload_bytes = 0;  // host bytes of payloads not yet released
    uint64_t entries = 0;           // requests not yet released
  };

  // `clock` returns seconds since the server's start; `held` the host bytes
  // a payload keeps alive.
  Scheduler(size_t budget, int max_overtake, std::function<double()> clock,
            std::function<size_t(const Payload&)> held)
      : budget_(budget), max_overtake_(max_overtake), clock_(std::move(clock)), held_(std::move(held)) {}

  // Queue a request. Returns false (and counts a rejection) when its
  // footprint exceeds the whole budget, since it could never be admitted.
  bool submit(std::unique_ptr<Payload> p, size_t footprint, uint64_t* id) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (footprint > budget_) {
        ++rejected_;
        return false;
      }
      auto e = std::make_unique<Entry>();
      e->id = next_id_++;
      e->footprint = footprint;
      e->payload = std::move(p);
      e->t_submit = clock_();
      *id = e->id;
      queue_.push_back(e->id);
      entries_[e->id] = std::move(e);
      ++gen_;
    }
    cv_.notify_all();
    return true;
  }

  // Block until a queued request is admitted (returned in state Running,
  // its footprint counted) or stop() was called (nullptr). When requests
  // are queued but none fits, `reclaim` (called without the lock) may free
  // held bytes (unhold) and return true, and admission is tried again.
  Entry* take(const std::function<bool()>& reclaim = nullptr) {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      if (stop_) return nullptr;
      Entry* got = pick_locked();
      if (got) {
        got->state = State::Running;
        got->admit_seq = ++admitted_;
        got->t_admit = clock_();
        in_use_ += got->footprint;
        peak_ = in_use_ > peak_ ? in_use_ : peak_;
        ++running_;
        peak_running_ = running_ > peak_running_ ? running_ : peak_running_;
        return got;
      }
      const uint64_t seen = gen_;
      if (!queue_.empty() && reclaim) {
        lk.unlock();
        const bool freed = reclaim();
        lk.lock();
        if (freed) continue;
      }
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
    }
  }

  // Bytes held outside any request (cached device memory), counted against
  // the budget like admitted footprints.
  void hold(size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    in_use_ += bytes;
    peak_ = in_use_ > peak_ ? in_use_ : peak_;
    ++gen_;
  }
  void unhold(size_t bytes) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      in_use_ -= bytes;
      ++gen_;
    }
    cv_.notify_all();
  }

  // The worker is done with a request: record its status, return its
  // footprint except `keep` bytes, which stay held (memory the worker keeps
  // for later requests, at most the footprint), drop what `trim` frees of
  // its payload, wake the others.
  void complete(Entry* e, int status, const std::function<void(Payload&)>& trim = nullptr, size_t keep = 0) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (trim && e->payload) trim(*e->payload);
      e->status = status;
      e->state = State::Done;
      e->t_finish = clock_();
      if (keep > e->footprint) keep = e->footprint;
      in_use_ -= e->footprint - keep;
      --running_;
      ++finished_;
      ++gen_;
    }
    cv_.notify_all();
  }

  // -1: unknown (or already released) id; 0: not finished; 1: finished, in
  // which case `collect` sees the entry (under the lock) and the request is
  // released: its payload is destroyed and only its times and status kept.
  int release(uint64_t id, const std::function<void(Entry&)>& collect) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = entries_.find(id);
    if (it == entries_.end()) return -1;
    Entry& e = *it->second;
    if (e.state != State::Done) return 0;
    if (collect) collect(e);
    Times t;
    t.t_submit = e.t_submit;
    t.t_admit = e.t_admit;
    t.t_finish = e.t_finish;
    t.status = e.status;
    released_[id] = t;
    entries_.erase(it);
    return 1;
  }

  bool times(uint64_t id, Times* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = entries_.find(id);
    if (it != entries_.end()) {
      out->t_submit = it->second->t_submit;
      out->t_admit = it->second->t_admit;
      out->t_finish = it->second->t_finish;
      out->status = it->second->status;
      return true;
    }
    auto jt = released_.find(id);
    if (jt == released_.end()) return false;
    *out = jt->second;
    return true;
  }

  // Wait until nothing is queued or running.
  void drain() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return queue_.empty() && running_ == 0; });
  }

  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
  }

  Stats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    Stats s;
    s.queued = queue_.size();
    s.running = (uint64_t)running_;
    s.finished = finished_;
    s.rejected = rejected_;
    s.bytes_in_use = in_use_;
    s.peak_bytes = peak_;
    s.budget = budget_;
    s.peak_running = peak_running_;
    s.entries = entries_.size();
    for (const auto& kv : entries_)
      if (kv.second->payload) s.held_payload_bytes += held_(*kv.second->payload);
    return s;
  }

 private:
  // First queued request that fits; requests before it that do not fit are
  // passed over (counted), unless one of them has been passed over
  // max_overtake_ times already, which stops the search at it.
  Entry* pick_locked() {
    for (auto it = queue_.begin(); it != queue_.end(); ++it) {
      Entry* e = entries_[*it].get();
      if (in_use_ + e->footprint <= budget_) {
        for (auto jt = queue_.begin(); jt != it; ++jt) entries_[*jt]->overtaken++;
        queue_.erase(it);
        return e;
      }
      if (e->overtaken >= max_overtake_) return nullptr;
    }
    return nullptr;
  }

  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<uint64_t> queue_;
  std::map<uint64_t, std::unique_ptr<Entry>> entries_;
  std::map<uint64_t, Times> released_;
  size_t budget_;
  int max_overtake_;
  std::function<double()> clock_;
  std::function<size_t(const Payload&)> held_;
  uint64_t next_id_ = 1;
  size_t in_use_ = 0, peak_ = 0;
  int running_ = 0, peak_running_ = 0;
  uint64_t finished_ = 0, rejected_ = 0;
  uint64_t admitted_ = 0;
  uint64_t gen_ = 0;  // bumped by every change that can make a request admissible
  bool stop_ = false;
};

}  // namespace pnk
