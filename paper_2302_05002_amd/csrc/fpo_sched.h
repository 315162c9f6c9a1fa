// Admission control of the request server, free of HIP so that it can be
// driven by a simulated executor on the CPU: an arena of `budget` bytes with
// first-fit allocation and coalescing frees, and a FIFO of waiting requests
// admitted, in arrival order, while a slot and enough memory are free (the
// head of the queue waits for memory rather than being overtaken, so no
// request starves).  Not thread-safe: the server holds its own lock.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <utility>

namespace fpo {

class Arena {
public:
    explicit Arena(uint64_t bytes) : total_(bytes)
    {
        if (bytes) free_[0] = bytes;
    }

    // First fit: the lowest-addressed free block that holds `bytes`.
    bool alloc(uint64_t bytes, uint64_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes;
            const uint64_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }

    // Returns [off, off + bytes) and merges it with free neighbours.
    void release(uint64_t off, uint64_t bytes)
    {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

    uint64_t total() const { return total_; }
    uint64_t used() const { return used_; }
    const std::map<uint64_t, uint64_t> &free_blocks() const { return free_; }

private:
    uint64_t total_;
    uint64_t used_ = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> bytes, disjoint, never adjacent
};

// Requests of type T (a handle) wait in arrival order; `admit` hands every
// request that can start now, with its arena offset, to a callback.
template <typename T>
class Admission {
public:
    Admission(uint64_t budget, uint32_t slots) : arena_(budget), slots_(slots) {}

    void submit(T item, uint64_t bytes) { waiting_.push_back({item, bytes}); }

    // Takes a request that has not been admitted out of the queue.
    bool remove_waiting(T item)
    {
        auto it = std::find_if(waiting_.begin(), waiting_.end(), [&](const Entry &e) { return e.item == item; });
        if (it == waiting_.end()) return false;
        waiting_.erase(it);
        return true;
    }

    template <typename F>
    void admit(F &&start)
    {
        while (!waiting_.empty() && running_ < slots_) {
            const Entry e = waiting_.front();
            uint64_t off = 0;
            if (!arena_.alloc(e.bytes, &off)) break;
            waiting_.pop_front();
            ++running_;
            start(e.item, off);
        }
    }

    void finished() { --running_; }                                   // a slot is free again
    void release(uint64_t off, uint64_t bytes) { arena_.release(off, bytes); }

    uint32_t running() const { return running_; }
    uint32_t slots() const { return slots_; }
    size_t waiting() const { return waiting_.size(); }
    const Arena &arena() const { return arena_; }

private:
    struct Entry {
        T item;
        uint64_t bytes;
    };
    Arena arena_;
    uint32_t slots_;
    uint32_t running_ = 0;
    std::deque<Entry> waiting_;
};

}  // namespace fpo
