// Host-side admission control of the sort server (no HIP: unit-tested on the CPU).
//
// Arena: first-fit allocator over a fixed byte range (the server's resident
// HBM budget), with coalescing of adjacent free blocks.
// Admission: FIFO of waiting jobs; the scheduler admits the longest prefix of
// the queue whose jobs all fit into the arena (a job that does not fit blocks
// the ones behind it, so large jobs are not starved); a job larger than the
// whole budget is refused at submission.
#pragma once
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace ssd {

class Arena {
  public:
    Arena(size_t size, size_t align) : size_(size), align_(align) {
        if (size) free_[0] = size;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    // Offset of a block of at least n bytes, or false when none is free.
    bool alloc(size_t n, size_t *off) {
        n = round(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                busy_[*off] = n;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    bool fits(size_t n) const {
        n = round(n ? n : 1);
        for (auto &f : free_)
            if (f.second >= n) return true;
        return false;
    }
    void release(size_t off) {
        auto b = busy_.find(off);
        if (b == busy_.end()) return;
        size_t start = off, len = b->second;
        used_ -= len;
        busy_.erase(b);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    size_t free_blocks() const { return free_.size(); }

  private:
    size_t round(size_t n) const { return (n + align_ - 1) / align_ * align_; }
    size_t size_, align_, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> busy_;   // offset -> length
};

struct Waiting {
    uint64_t ticket;
    size_t bytes;
};

class Admission {
  public:
    explicit Admission(size_t budget, size_t align = 256) : arena_(budget, align) {}
    // false: the job can never fit (larger than the whole budget)
    bool submit(uint64_t ticket, size_t bytes) {
        if (bytes > arena_.size()) return false;
        q_.push_back({ticket, bytes});
        return true;
    }
    // Admit waiting jobs in FIFO order while they fit, at most max_jobs and
    // max_strings-like weight (caller's accounting through `weight`).
    // Returns (ticket, arena offset) pairs.
    template <typename Weight>
    std::vector<std::pair<uint64_t, size_t>> admit(size_t max_jobs, uint64_t max_weight, Weight weight) {
        std::vector<std::pair<uint64_t, size_t>> out;
        uint64_t w = 0;
        while (!q_.empty() && out.size() < max_jobs) {
            const Waiting &j = q_.front();
            const uint64_t jw = weight(j.ticket);
            if (!out.empty() && w + jw > max_weight) break;
            size_t off;
            if (!arena_.alloc(j.bytes, &off)) break;   // head of line waits for memory
            out.push_back({j.ticket, off});
            w += jw;
            q_.pop_front();
        }
        return out;
    }
    std::vector<std::pair<uint64_t, size_t>> admit(size_t max_jobs) {
        return admit(max_jobs, ~0ull, [](uint64_t) { return (uint64_t)0; });
    }
    // Admit the longest FIFO prefix (at most max_jobs) whose jobs, packed
    // together, fit into one free arena block: add(ticket) accumulates a job,
    // bytes() gives the packed size of the jobs added so far or SIZE_MAX when
    // the batch exceeds another limit.  Allocates that block; false when even
    // the first waiting job does not fit now.
    template <typename Add, typename Bytes>
    bool admit_batch(size_t max_jobs, Add add, Bytes bytes, std::vector<uint64_t> *out, size_t *off) {
        out->clear();
        size_t best = 0;
        for (size_t i = 0; i < q_.size() && out->size() < max_jobs; ++i) {
            add(q_[i].ticket);
            const size_t b = bytes();
            if (b == (size_t)-1 || !arena_.fits(b)) break;
            out->push_back(q_[i].ticket);
            best = b;
        }
        if (out->empty()) return false;
        if (!arena_.alloc(best, off)) {
            out->clear();
            return false;
        }
        q_.erase(q_.begin(), q_.begin() + (long)out->size());
        return true;
    }
    void release(size_t off) { arena_.release(off); }
    bool cancel(uint64_t ticket) {
        for (auto it = q_.begin(); it != q_.end(); ++it)
            if (it->ticket == ticket) {
                q_.erase(it);
                return true;
            }
        return false;
    }
    size_t waiting() const { return q_.size(); }
    size_t used() const { return arena_.used(); }
    const Arena &arena() const { return arena_; }

  private:
    Arena arena_;
    std::deque<Waiting> q_;
};

}  // namespace ssd
