// CPU simulation of the serving loop around the library's own admission
// policy (serve_policy.h): requests arrive over simulated time, are admitted
// in FIFO order against the arena, launched in batches of up to max_batch on
// idle lanes, and retire after a duration proportional to their bytes. The
// checks are the policy's promises: admission order is submission order (less
// the rejected and those cancelled while waiting), no two live blocks overlap
// and none leaves the arena, every request completes exactly once (run,
// rejected or cancelled), requests larger than the arena are rejected, a
// cancel succeeds exactly when the request is still queued and returns its
// block, the free list never holds two adjacent blocks, and the arena is one
// free block again at the end.
//
// usage: serve_sim SEED
// prints "ok <admitted> <rejected> <max bytes in use> <steps that left requests waiting>
// <cancelled>"
#include "../paper_2108_13656_amd/csrc/serve_policy.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <iterator>
#include <map>
#include <random>
#include <utility>
#include <vector>

namespace {

struct Req {
    int id = 0;
    double arrival = 0;
    size_t need = 0; // granule bytes, 0 = takes no budget
    size_t off = 0, bytes = 0;
};

struct Lane {
    std::vector<Req> batch;
    double done_at = 0;
    bool busy = false;
};

int fails = 0;
void check(bool ok, const char *what, int id)
{
    if (!ok && fails++ < 10)
        std::printf("FAIL %s (request %d)\n", what, id);
}

} // namespace

int main(int argc, char **argv)
{
    const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    const size_t arena_bytes = dc::granules((size_t)(64 + rng() % 192) << 20); // 64..255 MiB
    const int nreq = 3000, nlanes = 1 + (int)(rng() % 8), max_batch = 1 + (int)(rng() % 64);

    std::vector<Req> trace(nreq);
    double t = 0;
    for (int i = 0; i < nreq; ++i) {
        t += -std::log(1.0 - u01(rng)) * 1e-4;
        trace[i].id = i;
        trace[i].arrival = t;
        const double r = u01(rng);
        size_t raw;
        if (r < 0.05)
            raw = 0; // caller-owned output
        else if (r < 0.07)
            raw = arena_bytes + 1 + rng() % arena_bytes; // never fits
        else
            raw = 1 + (size_t)(std::exp(u01(rng) * std::log((double)arena_bytes / 2)));
        trace[i].need = raw ? dc::granules(raw) : 0;
    }

    dc::Arena arena;
    arena.reset(arena_bytes);
    std::deque<Req> waiting, admitted;
    std::vector<Lane> lanes(nlanes);
    std::map<size_t, std::pair<size_t, int>> live; // off -> (bytes, id)
    std::vector<int> admit_order, done(nreq, 0), rejected(nreq, 0), cancelled(nreq, 0),
        was_admitted(nreq, 0);
    int ncancel = 0;
    size_t in_use = 0, max_in_use = 0;
    int next = 0, finished = 0, blocked = 0;
    double now = 0;

    while (finished < nreq) {
        // retire lanes whose launch has ended
        for (auto &ln : lanes) {
            if (!ln.busy || ln.done_at > now)
                continue;
            for (auto &q : ln.batch) {
                if (q.bytes) {
                    auto it = live.find(q.off);
                    check(it != live.end() && it->second.second == q.id, "retire a live block",
                          q.id);
                    live.erase(q.off);
                    arena.release(q.off, q.bytes);
                    in_use -= q.bytes;
                }
                done[q.id] += 1;
                ++finished;
            }
            ln.batch.clear();
            ln.busy = false;
        }
        // arrivals up to now
        while (next < nreq && trace[next].arrival <= now)
            waiting.push_back(trace[next++]);
        // admission through the library's policy
        dc::admit_fifo(
            waiting, admitted, arena, [](const Req &q) { return q.need; },
            [&](Req &q, size_t off, size_t bytes) {
                q.off = off;
                q.bytes = bytes;
                admit_order.push_back(q.id);
                was_admitted[q.id] = 1;
                if (!bytes)
                    return;
                check(bytes == q.need, "block size", q.id);
                check(off % dc::kGranule == 0 && off + bytes <= arena_bytes, "block in arena",
                      q.id);
                auto hi = live.lower_bound(off);
                if (hi != live.end())
                    check(off + bytes <= hi->first, "overlap with the next block", q.id);
                if (hi != live.begin()) {
                    auto lo = std::prev(hi);
                    check(lo->first + lo->second.first <= off, "overlap with the previous block",
                          q.id);
                }
                live[off] = {bytes, q.id};
                in_use += bytes;
                max_in_use = std::max(max_in_use, in_use);
            },
            [&](const Req &q) {
                check(q.need > arena_bytes, "rejected only when larger than the arena", q.id);
                rejected[q.id] += 1;
                ++finished;
            });
        // now and then a client cancels one of the requests it has sent
        if (next > 0 && u01(rng) < 0.1) {
            const int span = next < 40 ? next : 40; // mostly recent requests
            const int id = next - 1 - (int)(rng() % (uint64_t)span);
            bool queued = false;
            for (const auto &q : waiting)
                queued |= q.id == id;
            for (const auto &q : admitted)
                queued |= q.id == id;
            const bool hit = dc::cancel_queued(
                waiting, admitted, arena, [id](const Req &q) { return q.id == id; },
                [](const Req &q) { return std::pair<size_t, size_t>(q.off, q.bytes); },
                [&](const Req &q) {
                    if (q.bytes) {
                        check(live.count(q.off) && live[q.off].second == q.id, "cancel a live block",
                              q.id);
                        live.erase(q.off);
                        in_use -= q.bytes;
                    }
                    cancelled[q.id] += 1;
                    ++finished;
                });
            check(hit == queued, "cancel succeeds exactly for queued requests", id);
            ncancel += hit;
        }
        check(in_use <= arena_bytes, "budget", -1);
        if (!waiting.empty())
            ++blocked; // the front request waits for memory: FIFO holds the rest back
        // free list: sorted, disjoint, never two adjacent blocks
        size_t end = 0;
        bool first = true;
        for (const auto &b : arena.free_blocks()) {
            check(first || b.first > end, "free blocks coalesced and disjoint", -1);
            end = b.first + b.second;
            first = false;
        }
        // launches on idle lanes
        for (auto &ln : lanes) {
            if (admitted.empty())
                break;
            if (ln.busy)
                continue;
            size_t bytes = 0;
            for (int k = 0; k < max_batch && !admitted.empty(); ++k) {
                bytes += admitted.front().need;
                ln.batch.push_back(admitted.front());
                admitted.pop_front();
            }
            ln.busy = true;
            ln.done_at = now + 1e-4 + (double)bytes * 2e-11;
        }
        // next event: an arrival or a lane finishing
        double nxt = next < nreq ? trace[next].arrival : 1e300;
        for (const auto &ln : lanes)
            if (ln.busy && ln.done_at < nxt)
                nxt = ln.done_at;
        if (nxt == 1e300) {
            check(finished == nreq, "no request left behind", -1);
            break;
        }
        now = nxt > now ? nxt : now;
    }

    // FIFO: admission order is submission order without the rejected and
    // those cancelled while still waiting
    std::vector<int> want;
    for (int i = 0; i < nreq; ++i)
        if (!rejected[i] && !(cancelled[i] && !was_admitted[i]))
            want.push_back(i);
    check(admit_order == want, "FIFO admission order", -1);
    for (int i = 0; i < nreq; ++i) {
        check(done[i] + rejected[i] + cancelled[i] == 1, "each request completes exactly once", i);
        check(!rejected[i] || trace[i].need > arena_bytes, "only oversized requests rejected", i);
    }
    check(ncancel > 0, "some cancels hit queued requests", -1);
    check(live.empty() && in_use == 0, "all blocks returned", -1);
    check(arena.free_blocks().size() == 1 && arena.free_blocks().begin()->first == 0 &&
              arena.free_blocks().begin()->second == arena_bytes,
          "arena whole again", -1);
    int nrej = 0;
    for (int r : rejected)
        nrej += r;
    if (fails)
        return 1;
    std::printf("ok %zu %d %zu %d %d\n", admit_order.size(), nrej, max_in_use, blocked, ncancel);
    return 0;
}
