// Scheduling core of the continuous-batching server, free of any GPU call so
// that its policy can be exercised on a host: a FIFO request queue, a
// first-fit allocator over a fixed device arena (admission by memory
// footprint), and slot bookkeeping per quantum of sweeps.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

namespace ising {

// First-fit allocator of byte ranges inside [0, capacity); every range is a
// multiple of `align` and starts on an `align` boundary.
class ArenaAllocator {
  public:
    explicit ArenaAllocator(size_t capacity = 0, size_t align = 256) : align_(align) { reset(capacity); }

    void reset(size_t capacity) {
        capacity_ = capacity - capacity % align_;
        free_.clear();
        if (capacity_) free_[0] = capacity_;
        used_ = 0;
    }

    size_t round(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

    // Returns true and the offset on success.
    bool alloc(size_t bytes, size_t* off) {
        const size_t need = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const size_t rest = it->second - need;
            const size_t rest_off = it->first + need;
            free_.erase(it);
            if (rest) free_[rest_off] = rest;
            used_ += need;
            return true;
        }
        return false;
    }

    void release(size_t off, size_t bytes) {
        const size_t len = round(bytes);
        used_ -= len;
        auto it = free_.emplace(off, len).first;
        // merge with the next range
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        // merge with the previous range
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    size_t capacity() const { return capacity_; }
    size_t used() const { return used_; }
    size_t largest_free() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    size_t capacity_ = 0, align_ = 256, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Request {
    uint64_t id = 0;
    int32_t L = 0;
    double T = 0;
    int64_t sweeps = 0;
    uint64_t seed = 0;
    int32_t init = 0;
    size_t bytes = 0;       // packed words
    double t_submit = 0;
};

struct Slot {
    bool active = false;
    Request req;
    size_t off = 0;         // arena offset of the words
    int64_t done = 0;       // sweeps completed
    int64_t planned = 0;    // sweeps scheduled in the current quantum
    double t_admit = 0;
};

class Scheduler {
  public:
    Scheduler(size_t budget, int32_t max_slots, int32_t quantum)
        : arena_(budget), slots_(max_slots), quantum_(quantum) {}

    size_t budget() const { return arena_.capacity(); }
    int32_t quantum() const { return quantum_; }
    const std::vector<Slot>& slots() const { return slots_; }
    std::vector<Slot>& slots() { return slots_; }
    size_t queued() const { return queue_.size(); }
    size_t bytes_in_use() const { return arena_.used(); }
    int32_t active() const {
        int32_t n = 0;
        for (auto& s : slots_) n += s.active;
        return n;
    }

    // false if the request can never fit (larger than the whole arena)
    bool submit(const Request& r) {
        if (arena_.round(r.bytes) > arena_.capacity()) return false;
        queue_.push_back(r);
        return true;
    }

    // Admit queued requests in arrival order while a slot and arena space
    // are free; stops at the first request that does not fit (no overtaking,
    // so a large request cannot starve).  Returns the admitted slot indices.
    std::vector<int32_t> admit(double now) {
        std::vector<int32_t> out;
        while (!queue_.empty()) {
            int32_t free_slot = -1;
            for (int32_t i = 0; i < (int32_t)slots_.size(); ++i)
                if (!slots_[i].active) {
                    free_slot = i;
                    break;
                }
            if (free_slot < 0) break;
            size_t off = 0;
            if (!arena_.alloc(queue_.front().bytes, &off)) break;
            Slot& s = slots_[free_slot];
            s.active = true;
            s.req = queue_.front();
            s.off = off;
            s.done = 0;
            s.planned = 0;
            s.t_admit = now;
            queue_.pop_front();
            out.push_back(free_slot);
        }
        return out;
    }

    // Sweeps of every active slot in the next quantum: min(quantum, left).
    void plan_quantum() {
        for (auto& s : slots_) s.planned = s.active ? std::min<int64_t>(quantum_, s.req.sweeps - s.done) : 0;
    }

    void complete_quantum() {
        for (auto& s : slots_)
            if (s.active) s.done += s.planned;
    }

    std::vector<int32_t> finished() const {
        std::vector<int32_t> out;
        for (int32_t i = 0; i < (int32_t)slots_.size(); ++i)
            if (slots_[i].active && slots_[i].done >= slots_[i].req.sweeps) out.push_back(i);
        return out;
    }

    void retire(int32_t i) {
        Slot& s = slots_[i];
        arena_.release(s.off, s.req.bytes);
        s.active = false;
    }

  private:
    ArenaAllocator arena_;
    std::vector<Slot> slots_;
    std::deque<Request> queue_;
    int32_t quantum_;
};

}  // namespace ising
