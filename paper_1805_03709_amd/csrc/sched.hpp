// Admission of client requests into batches for the serving loop (host code, plain C++).
//
// Each client has a FIFO of requests and at most one request in flight, so every answer
// starts at the cursor that the client's previous answer returned (Sec. 4.2: a client
// receives the blocks updated since its last request, at most its request size).  A
// request is admitted when its client is idle, a result slot is free and its result bytes
// fit the arena (first fit).  A request that can never fit (more bytes than the whole
// arena, or more log chunks than the log has) is rejected.  Both forms of the serving loop
// (rounds of kernels on streams, and the persistent launch) build their batches here.
#pragma once
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <utility>
#include <vector>

#include "arena.hpp"

namespace vbh {

inline int64_t align256(int64_t n) { return (n + 255) & ~int64_t(255); }

// Arena bytes of a request with `limit` answers over `n_chunks` log chunks: selected pool
// indices (4 B each), chunk counts (8 B), keys (12 B), MC voxels (2048 B) and the count /
// next-cursor pair, each 256-byte aligned.
inline int64_t req_bytes(int64_t limit, int64_t n_chunks) {
    return align256(limit * 4) + align256(n_chunks * 8) + align256(limit * 12) + align256(limit * 2048) + 256;
}

struct Admitted {
    int64_t req;       // request index
    int client;
    int slot;          // result slot
    int64_t off;       // arena range
    int64_t bytes;
    uint64_t cursor;   // first log position the answer considers
    uint64_t end;      // log end of the scene version it answers
    int64_t limit;
    int64_t n_chunks;  // log chunks from cursor to end
};

class Admission {
public:
    void init(int n_clients, int max_inflight, int max_batch, int64_t arena_bytes, int64_t chunk,
              int64_t cap_chunks) {
        queue_.assign(size_t(n_clients), {});
        busy_.assign(size_t(n_clients), 0);
        cursor_.assign(size_t(n_clients), 0);
        slots_.clear();
        for (int i = max_inflight - 1; i >= 0; --i) slots_.push_back(i);
        max_batch_ = max_batch;
        arena_bytes_ = arena_bytes;
        chunk_ = chunk;
        cap_chunks_ = cap_chunks;
        arena_.init(arena_bytes);
    }
    // Start of a run: queues empty, every client idle, every slot and arena byte free
    // (nothing is in flight between runs); cursors are kept.
    void begin_run() {
        for (auto &q : queue_) q.clear();
        for (auto &b : busy_) b = 0;
        const int n = int(slots_.size()) + in_flight_;
        slots_.clear();
        for (int i = n - 1; i >= 0; --i) slots_.push_back(i);
        in_flight_ = 0;
        arena_.init(arena_bytes_);
    }
    int n_clients() const { return int(queue_.size()); }
    uint64_t cursor(int c) const { return cursor_[size_t(c)]; }
    void set_cursor(int c, uint64_t v) { cursor_[size_t(c)] = v; }
    bool busy(int c) const { return busy_[size_t(c)] != 0; }
    int free_slots() const { return int(slots_.size()); }
    void arrive(int client, int64_t req, int64_t limit) { queue_[size_t(client)].push_back({req, limit}); }
    // some idle client has a queued request
    bool work_pending() const {
        for (size_t c = 0; c < queue_.size(); ++c)
            if (!busy_[c] && !queue_[c].empty()) return true;
        return false;
    }
    bool any_queued() const {
        for (const auto &q : queue_)
            if (!q.empty()) return true;
        return false;
    }
    // One batch for log end `end`: in client order, the head request of each idle client,
    // while result slots last, up to max_batch requests; a head whose bytes do not fit the
    // free arena waits (its client stays idle); a head that can never fit is rejected.
    void build(uint64_t end, std::vector<Admitted> &batch, std::vector<int64_t> &rejected) {
        batch.clear();
        rejected.clear();
        for (size_t c = 0; c < queue_.size() && int(batch.size()) < max_batch_; ++c) {
            if (busy_[c] || queue_[c].empty() || slots_.empty()) continue;
            const int64_t ri = queue_[c].front().first, lim = queue_[c].front().second;
            const uint64_t cur = cursor_[c];
            const int64_t nch = cur < end ? int64_t((end - cur + uint64_t(chunk_) - 1) / uint64_t(chunk_)) : 0;
            const int64_t bytes = req_bytes(lim, nch);
            if (nch > cap_chunks_ || bytes > arena_bytes_) {
                rejected.push_back(ri);
                queue_[c].pop_front();
                continue;
            }
            const int64_t off = arena_.alloc(bytes);
            if (off < 0) continue;
            queue_[c].pop_front();
            busy_[c] = 1;
            const int slot = slots_.back();
            slots_.pop_back();
            ++in_flight_;
            batch.push_back({ri, int(c), slot, off, bytes, cur, end, lim, nch});
        }
    }
    // The answer of `a` is complete: its client continues from `cursor_out`.
    void complete(const Admitted &a, uint64_t cursor_out) {
        cursor_[size_t(a.client)] = cursor_out;
        busy_[size_t(a.client)] = 0;
        arena_.release(a.off, a.bytes);
        slots_.push_back(a.slot);
        --in_flight_;
    }
    const Arena &arena() const { return arena_; }

private:
    std::vector<std::deque<std::pair<int64_t, int64_t>>> queue_;  // (request, limit)
    std::vector<char> busy_;
    std::vector<uint64_t> cursor_;
    std::vector<int> slots_;
    int in_flight_ = 0;
    int max_batch_ = 1;
    int64_t arena_bytes_ = 0, chunk_ = 1, cap_chunks_ = 0;
    Arena arena_;
};

// The rounds form fuses frames on a thread of its own while batches are served: a frame's
// MC update rewrites MC voxels and the log that batches in flight read, so the two exclude
// each other.  The updater asks and waits; the serving side stops admitting while a request
// stands and grants it once nothing is in flight; the updater publishes the new log end and
// version under the same lock and lets serving resume.
class McGate {
public:
    // updater: returns once serving has granted (nothing in flight)
    void acquire() {
        std::unique_lock<std::mutex> lk(mu_);
        request_ = true;
        cv_.wait(lk, [&] { return granted_; });
    }
    // updater: `publish` runs under the lock, then serving may resume
    template <class F>
    void release(F &&publish) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            publish();
            request_ = false;
            granted_ = false;
        }
        cv_.notify_all();
    }
    // updater: no more updates (a request still standing is withdrawn)
    void finish() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            request_ = false;
        }
        cv_.notify_all();
    }
    // serving: `read` runs under the lock (the published log end and version); a standing
    // request is granted when `idle` (nothing in flight).  Returns true while admission is
    // closed (a request stands, granted or not).
    template <class F>
    bool poll(bool idle, F &&read) {
        bool grant = false, closed;
        {
            std::lock_guard<std::mutex> lk(mu_);
            read();
            closed = request_;
            if (request_ && !granted_ && idle) grant = granted_ = true;
        }
        if (grant) cv_.notify_all();
        return closed;
    }

private:
    std::mutex mu_;
    std::condition_variable cv_;
    bool request_ = false, granted_ = false;
};

}  // namespace vbh
