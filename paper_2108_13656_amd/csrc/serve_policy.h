// Host-only policy pieces of the continuous-batching server: the device-memory
// arena (first fit over a sorted free list, blocks rounded to 256-byte
// granules, neighbours coalesced on release), FIFO admission against it, and
// cancellation of requests that are still queued.
// No HIP here, so the policy can be exercised on the CPU with simulated
// launches; runtime.cpp drives it with real streams and events.
#ifndef DC_SERVE_POLICY_H
#define DC_SERVE_POLICY_H

#include <cstddef>
#include <deque>
#include <iterator>
#include <map>
#include <utility>

namespace dc {

constexpr size_t kGranule = 256;

inline size_t granules(size_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }

// Offsets into a fixed block of `total` bytes (a multiple of kGranule).
class Arena {
  public:
    void reset(size_t total)
    {
        total_ = total;
        free_.clear();
        if (total)
            free_[0] = total;
    }
    size_t total() const { return total_; }
    // First fit: the lowest free block that holds `bytes` (a granule
    // multiple) gives its front. False when no block is large enough now.
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest)
                    free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    // Returns [off, off + bytes) and merges it with free neighbours.
    void release(size_t off, size_t bytes)
    {
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
    const std::map<size_t, size_t> &free_blocks() const { return free_; }

  private:
    size_t total_ = 0;
    std::map<size_t, size_t> free_; // offset -> size
};

// FIFO admission: moves requests from the front of `waiting` to the back of
// `admitted` while the arena can hold what each needs (need(q): granule
// bytes, 0 for a request that takes no budget). A request needing more than
// the whole arena can never run and goes to reject(q); admission stops at the
// first request that does not fit now, so no later request overtakes it.
// place(q, off, bytes) sees every admitted request (off and bytes 0 when it
// takes no budget) before it joins `admitted`.
template <class Req, class Need, class Place, class Reject>
void admit_fifo(std::deque<Req> &waiting, std::deque<Req> &admitted, Arena &arena, Need need,
                Place place, Reject reject)
{
    while (!waiting.empty()) {
        Req &q = waiting.front();
        const size_t bytes = need(q);
        if (bytes > arena.total()) {
            reject(q);
            waiting.pop_front();
            continue;
        }
        size_t off = 0;
        if (bytes > 0 && !arena.alloc(bytes, &off))
            break;
        place(q, off, bytes);
        admitted.push_back(q);
        waiting.pop_front();
    }
}

// Cancels the first queued request that match(q) accepts, looking in
// `waiting` and then in `admitted` (requests not yet in a launch); an
// admitted request's block (block(q) -> {offset, bytes}, bytes 0 for none)
// returns to the arena. drop(q) sees the request before it leaves its queue.
// True when a request was cancelled; a request that is already launched
// cannot be.
template <class Req, class Match, class Block, class Drop>
bool cancel_queued(std::deque<Req> &waiting, std::deque<Req> &admitted, Arena &arena, Match match,
                   Block block, Drop drop)
{
    for (auto it = waiting.begin(); it != waiting.end(); ++it)
        if (match(*it)) {
            drop(*it);
            waiting.erase(it);
            return true;
        }
    for (auto it = admitted.begin(); it != admitted.end(); ++it)
        if (match(*it)) {
            const auto b = block(*it);
            if (b.second)
                arena.release(b.first, b.second);
            drop(*it);
            admitted.erase(it);
            return true;
        }
    return false;
}

} // namespace dc

#endif
