// Host-side bookkeeping of the request server (no HIP): the output-pool
// ring allocator and the ticket table. Kept in a header of their own so they
// can be tested on the CPU.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>

namespace rngx {

// Ring allocator over [0, size) in 256-byte granules. Requests are admitted
// in FIFO order and (with automatic release) freed in that order, so the
// pool is used as a circular buffer: allocate at the head, free from the
// tail. A block released out of order is only marked; the tail advances
// over it once every older block is free as well. Allocation and release
// are O(1); a request that does not fit at the head waits (FIFO admission).
class PoolRing {
  public:
    void reset(uint64_t size)
    {
        blocks_.clear();
        cap_ = size;
        head_ = base_seq_ = used_ = peak_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t *off, uint64_t *seq)
    {
        bytes = (bytes + 255) & ~(uint64_t)255;
        if (bytes > cap_)
            return false;
        uint64_t at;
        if (blocks_.empty()) {
            head_ = 0;
            at = 0;
        } else {
            const uint64_t tail = blocks_.front().off;
            if (head_ > tail) { // used: [tail, head)
                if (bytes <= cap_ - head_) {
                    at = head_;
                } else if (bytes <= tail) {
                    push(head_, cap_ - head_, true); // skip the end of the pool
                    at = 0;
                } else {
                    return false;
                }
            } else if (head_ < tail) { // used: [tail, cap) and [0, head)
                if (bytes > tail - head_)
                    return false;
                at = head_;
            } else {
                return false; // head == tail with blocks live: full
            }
        }
        *seq = push(at, bytes, false);
        *off = at;
        head_ = at + bytes == cap_ ? 0 : at + bytes;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
    }
    void release(uint64_t seq)
    {
        if (seq < base_seq_ || seq - base_seq_ >= blocks_.size())
            return;
        Block &b = blocks_[seq - base_seq_];
        if (b.freed)
            return;
        b.freed = true;
        used_ -= b.size;
        while (!blocks_.empty() && blocks_.front().freed) {
            blocks_.pop_front();
            ++base_seq_;
        }
    }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    void reset_peak() { peak_ = used_; }

  private:
    struct Block {
        uint64_t off, size;
        bool freed;
    };
    uint64_t push(uint64_t off, uint64_t size, bool freed)
    {
        blocks_.push_back({off, size, freed});
        return base_seq_ + blocks_.size() - 1;
    }
    std::deque<Block> blocks_;
    uint64_t cap_ = 0, head_ = 0, base_seq_ = 0, used_ = 0, peak_ = 0;
};

// Entries by ticket: tickets are consecutive, so a deque indexed by
// (ticket - first ticket) whose released front entries are dropped. R needs
// a `bool live` member.
template <typename R> class TicketTable {
  public:
    void clear(uint64_t first)
    {
        q_.clear();
        first_ = first;
    }
    R &add(const R &r)
    {
        q_.push_back(r);
        return q_.back();
    }
    uint64_t next_ticket() const { return first_ + q_.size(); }
    R *find(uint64_t t)
    {
        if (t < first_ || t - first_ >= q_.size())
            return nullptr;
        R &r = q_[t - first_];
        return r.live ? &r : nullptr;
    }
    void erase(uint64_t t)
    {
        R *r = find(t);
        if (!r)
            return;
        r->live = false;
        while (!q_.empty() && !q_.front().live) {
            q_.pop_front();
            ++first_;
        }
    }

  private:
    std::deque<R> q_;
    uint64_t first_ = 1;
};


} // namespace rngx
