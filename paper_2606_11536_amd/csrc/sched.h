// The continuous-batching schedule of the server, with no device in it: which
// queued query goes to which column slot, which slot range each step scans,
// and when a query has met every slot once.  The server (server.cpp) drives
// it and issues the kernel launches; pir_server_simulate runs it against a
// stand-in executor on the host.
//
// The flat slot index s = k N + t of the database is cut into n_chunks ranges
// [n_slots c / n_chunks, n_slots (c+1) / n_chunks), none empty (n_chunks <=
// n_slots), which the steps scan round-robin.  At a step boundary queued
// queries are admitted, oldest first, into the lowest free column slots; the
// step then scans its range for every active query, and a query that has now
// been active for n_chunks consecutive steps -- so has met every range
// exactly once -- completes and frees its slot.
#pragma once

#include <stdint.h>

#include <deque>
#include <vector>

namespace pir {

class CircularScan {
 public:
  struct Slot {
    bool active = false;
    uint64_t ticket = 0;
    uint32_t done = 0;  // ranges scanned since admission
  };

  CircularScan(uint32_t max_batch, uint32_t n_slots, uint32_t n_chunks)
      : slots_(max_batch), n_slots_(n_slots), n_chunks_(n_chunks) {}

  uint32_t max_batch() const { return (uint32_t)slots_.size(); }
  uint32_t n_chunks() const { return n_chunks_; }
  uint32_t chunk() const { return chunk_; }
  const Slot &slot(uint32_t k) const { return slots_[k]; }

  // Slot range of chunk c: [begin, end), never empty.
  uint32_t range_begin(uint32_t c) const { return (uint32_t)((uint64_t)n_slots_ * c / n_chunks_); }
  uint32_t range_end(uint32_t c) const { return range_begin(c + 1); }

  void submit(uint64_t ticket) { queue_.push_back(ticket); }
  uint32_t queued() const { return (uint32_t)queue_.size(); }

  // The next admission, if a query is queued and a column slot is free: the
  // oldest queued ticket and the lowest free slot.  Changes nothing.
  bool next_admission(uint32_t *slot, uint64_t *ticket) const {
    if (queue_.empty()) return false;
    for (uint32_t k = 0; k < slots_.size(); ++k)
      if (!slots_[k].active) {
        *slot = k;
        *ticket = queue_.front();
        return true;
      }
    return false;
  }

  // Commit the admission next_admission() reported.
  void admit(uint32_t slot) {
    Slot &s = slots_[slot];
    s.active = true;
    s.ticket = queue_.front();
    s.done = 0;
    queue_.pop_front();
  }

  // Batch width of this step's scan: highest active slot + 1 (0: nothing to scan).
  uint32_t b_eff() const {
    uint32_t b = 0;
    for (uint32_t k = 0; k < slots_.size(); ++k)
      if (slots_[k].active) b = k + 1;
    return b;
  }

  uint32_t active() const {
    uint32_t a = 0;
    for (const Slot &s : slots_) a += s.active;
    return a;
  }

  // After this step's range was scanned: every active slot has met one more
  // range; the step moves to the next range.  Returns the slots whose query
  // has now met all of them (still marked active until release()).
  std::vector<uint32_t> advance() {
    std::vector<uint32_t> fin;
    for (uint32_t k = 0; k < slots_.size(); ++k) {
      Slot &s = slots_[k];
      if (s.active && ++s.done == n_chunks_) fin.push_back(k);
    }
    chunk_ = chunk_ + 1 == n_chunks_ ? 0 : chunk_ + 1;
    return fin;
  }

  void release(uint32_t slot) { slots_[slot] = Slot{}; }

 private:
  std::vector<Slot> slots_;
  std::deque<uint64_t> queue_;
  uint32_t n_slots_, n_chunks_, chunk_ = 0;
};

}  // namespace pir
