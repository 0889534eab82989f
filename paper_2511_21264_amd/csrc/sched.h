// Host-only core of the serving loop: a first-fit arena over a fixed byte
// range, and the admission / iteration bookkeeping of continuous batching.
// Nothing here touches the device; serve.hip maps arena offsets onto its
// device and pinned regions and launches the work.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

namespace mppi {

constexpr size_t NO_SPACE = ~(size_t)0;

// First-fit allocator over [0, capacity): free ranges kept by offset and
// merged with their neighbours on release.
class Arena {
public:
    explicit Arena(size_t bytes = 0, size_t align = 256) : align_(align) { reset(bytes); }

    void reset(size_t bytes)
    {
        capacity_ = bytes;
        used_ = high_ = 0;
        free_.clear();
        live_.clear();
        if (bytes) free_[0] = bytes;
    }

    size_t round(size_t bytes) const { return bytes == 0 ? align_ : (bytes + align_ - 1) / align_ * align_; }

    size_t alloc(size_t bytes)
    {
        const size_t n = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            live_[off] = n;
            used_ += n;
            if (used_ > high_) high_ = used_;
            return off;
        }
        return NO_SPACE;
    }

    // false for an offset that is not a live block
    bool release(size_t off)
    {
        auto it = live_.find(off);
        if (it == live_.end()) return false;
        size_t start = off, n = it->second;
        live_.erase(it);
        used_ -= n;
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && start + n == nx->first) {
            n += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(start);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == start) {
                start = pv->first;
                n += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = n;
        return true;
    }

    size_t capacity() const { return capacity_; }
    size_t used() const { return used_; }
    size_t high_water() const { return high_; }
    size_t largest_free() const
    {
        size_t b = 0;
        for (auto &f : free_) b = f.second > b ? f.second : b;
        return b;
    }
    size_t n_free_ranges() const { return free_.size(); }

private:
    size_t align_, capacity_ = 0, used_ = 0, high_ = 0;
    std::map<size_t, size_t> free_, live_;
};

enum ReqState { RS_PENDING = 0, RS_ACTIVE = 1, RS_FINISHING = 2, RS_DONE = 3 };

struct SchedReq {
    uint64_t id = 0;
    int cell = -1;
    int M = 1;
    int m = 0;                 // next iteration to run
    size_t dev_bytes = 0, host_bytes = 0;
    size_t dev_off = NO_SPACE, host_off = NO_SPACE;
    bool cancel = false;
    int state = RS_PENDING;
    double deadline = INFINITY;  // absolute, in the caller's clock (ms); INFINITY: none
    double work = 0.0;           // env-steps of one of its iterations (K * H)
    double pred_end = 0.0;       // predicted end when admitted (without the margin)
};

// Predicted device time of one packed iteration over active requests whose
// iterations hold W env-steps in total: max(floor_ms, base_ms + ms_per_work W)
// (a small launch is bound by one sample's chain of steps, a large one by
// throughput).  A zero model predicts no time (admission then only orders by
// deadline and sheds requests already past theirs).
struct IterModel {
    double base_ms = 0.0, ms_per_work = 0.0, floor_ms = 0.0;
    double margin_ms = 0.0;  // added to every predicted end (how late past predictions were)
    double time(double W) const { return std::max(floor_ms, base_ms + ms_per_work * W); }
};

// Admission and iteration order of the requests of a server.
//   * Queue: earliest deadline first, ties (and requests without deadline)
//     in submission order, so with no deadlines the queue is FIFO.  A
//     request waits while an earlier request of its cell is queued or
//     active (a cell's requests run in submission order); the scan stops at
//     the first request that does not fit in memory (no overtaking on
//     memory, so a large request cannot starve).
//   * Deadlines: a request is admitted only when, with the iteration model
//     at the load it would join, its M iterations (behind the one already in
//     flight, if any) end by its deadline, and no active request predicted on time
//     would become late; otherwise the scan stops there (it waits for load
//     to drain, nothing overtakes it).  A queued request that cannot end by
//     its deadline even alone is shed: it leaves the queue unrun.
//   * Active set: at most max_active requests; each iteration runs one
//     MPPI iteration of every active request, each at its own index m.
//   * A request leaves the active set when its last iteration has been
//     launched (state FINISHING; its cell may admit its next request, whose
//     work is ordered after it on the stream); its memory is returned by
//     release() once that work has completed.
class Scheduler {
public:
    Scheduler(size_t dev_bytes = 0, size_t host_bytes = 0, int max_active = 1, int max_pending = 1)
        : dev_(dev_bytes), host_(host_bytes), max_active_(max_active), max_pending_(max_pending)
    {
    }

    // 0 = queued, 1 = queue full, 2 = can never fit the arenas
    int enqueue(const SchedReq &r0, bool supersede, std::vector<uint64_t> *superseded)
    {
        if (dev_.round(r0.dev_bytes) > dev_.capacity() || host_.round(r0.host_bytes) > host_.capacity()) return 2;
        if (supersede && r0.cell >= 0) {
            for (auto it = pending_.begin(); it != pending_.end();) {
                SchedReq &q = reqs_.at(*it);
                if (q.cell == r0.cell) {
                    if (superseded) superseded->push_back(q.id);
                    q.state = RS_DONE;
                    q.cancel = true;
                    it = pending_.erase(it);
                } else {
                    ++it;
                }
            }
        }
        if ((int)pending_.size() >= max_pending_) return 1;
        SchedReq r = r0;
        r.state = RS_PENDING;
        r.m = 0;
        r.cancel = false;
        reqs_[r.id] = r;
        pending_.push_back(r.id);
        return 0;
    }

    // predicted end of request r admitted at `now` into a load of W: its M - m
    // remaining iterations after `extra` iterations already in flight
    static double predicted_end(const SchedReq &r, double now, const IterModel &im, double W, int extra)
    {
        return now + (double)(r.M - r.m + extra) * im.time(W) + im.margin_ms;
    }

    // admitted ids, in admission order; requests shed (see above) go to *shed
    // (their state becomes RS_DONE; they hold no memory).  `extra`: packed
    // iterations already launched that every admitted request waits behind.
    std::vector<uint64_t> admit(double now = 0.0, const IterModel &im = IterModel{},
                                std::vector<uint64_t> *shed = nullptr, int extra = 1)
    {
        std::vector<uint64_t> out;
        if (shed) {
            for (auto it = pending_.begin(); it != pending_.end();) {
                SchedReq &r = reqs_.at(*it);
                if (predicted_end(r, now, im, r.work, extra) > r.deadline) {
                    shed->push_back(r.id);
                    r.state = RS_DONE;
                    r.cancel = true;
                    it = pending_.erase(it);
                } else {
                    ++it;
                }
            }
        }
        std::vector<uint64_t> order(pending_.begin(), pending_.end());
        std::stable_sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
            const double da = reqs_.at(a).deadline, db = reqs_.at(b).deadline;
            return da < db || (da == db && a < b);
        });
        // a cell's requests run in submission order: only its oldest queued
        // request may be admitted, and only while none of it is active
        std::unordered_map<int, uint64_t> oldest;
        for (uint64_t id : pending_) {
            const int c = reqs_.at(id).cell;
            if (c >= 0 && !oldest.count(c)) oldest[c] = id;
        }
        std::unordered_map<int, bool> blocked;
        double W = 0.0;
        for (uint64_t a : active_) {
            const SchedReq &r = reqs_.at(a);
            if (r.cell >= 0) blocked[r.cell] = true;
            W += r.work;
        }
        for (uint64_t id : order) {
            if ((int)active_.size() >= max_active_) break;
            SchedReq &r = reqs_.at(id);
            if (r.cell >= 0 && (blocked.count(r.cell) || oldest.at(r.cell) != id)) continue;
            const double W1 = W + r.work;
            bool fits = predicted_end(r, now, im, W1, extra) <= r.deadline;
            for (uint64_t a : active_) {
                const SchedReq &q = reqs_.at(a);
                if (fits && std::isfinite(q.deadline) && predicted_end(q, now, im, W, extra) <= q.deadline)
                    fits = predicted_end(q, now, im, W1, extra) <= q.deadline;
            }
            if (!fits) break;  // wait for the load to drain; nothing overtakes it
            const size_t d = dev_.alloc(r.dev_bytes);
            if (d == NO_SPACE) break;
            const size_t h = host_.alloc(r.host_bytes);
            if (h == NO_SPACE) {
                dev_.release(d);
                break;
            }
            r.dev_off = d;
            r.host_off = h;
            r.state = RS_ACTIVE;
            r.pred_end = predicted_end(r, now, im, W1, extra) - im.margin_ms;
            if (r.cell >= 0) blocked[r.cell] = true;
            W = W1;
            active_.push_back(r.id);
            out.push_back(r.id);
            pending_.erase(std::find(pending_.begin(), pending_.end(), id));
        }
        return out;
    }

    // 0 = unknown or already finishing/done, 1 = dropped from the queue,
    // 2 = active: flagged, dropped at the next iteration boundary
    int cancel(uint64_t id)
    {
        auto f = reqs_.find(id);
        if (f == reqs_.end()) return 0;
        SchedReq &r = f->second;
        if (r.state == RS_PENDING) {
            for (auto it = pending_.begin(); it != pending_.end(); ++it)
                if (*it == id) {
                    pending_.erase(it);
                    break;
                }
            r.state = RS_DONE;
            r.cancel = true;
            return 1;
        }
        if (r.state == RS_ACTIVE) {
            r.cancel = true;
            return 2;
        }
        return 0;
    }

    // Active requests of the next iteration, after removing the cancelled
    // ones (their ids go to *dropped; their memory stays held until
    // release(), since earlier launches may still use it).
    std::vector<const SchedReq *> next_iteration(std::vector<uint64_t> *dropped)
    {
        std::vector<const SchedReq *> out;
        for (auto it = active_.begin(); it != active_.end();) {
            SchedReq &r = reqs_.at(*it);
            if (r.cancel) {
                r.state = RS_FINISHING;
                if (dropped) dropped->push_back(r.id);
                it = active_.erase(it);
                continue;
            }
            out.push_back(&r);
            ++it;
        }
        return out;
    }

    // After an iteration was launched over the active set: every active
    // request moves to its next index; those that ran their last iteration
    // leave the active set (returned).
    std::vector<uint64_t> advance()
    {
        std::vector<uint64_t> fin;
        for (auto it = active_.begin(); it != active_.end();) {
            SchedReq &r = reqs_.at(*it);
            ++r.m;
            if (r.m >= r.M) {
                r.state = RS_FINISHING;
                fin.push_back(r.id);
                it = active_.erase(it);
            } else {
                ++it;
            }
        }
        return fin;
    }

    // return the memory of a finishing request and forget it
    bool release(uint64_t id)
    {
        auto f = reqs_.find(id);
        if (f == reqs_.end()) return false;
        SchedReq &r = f->second;
        if (r.state == RS_PENDING || r.state == RS_ACTIVE) return false;
        if (r.dev_off != NO_SPACE) dev_.release(r.dev_off);
        if (r.host_off != NO_SPACE) host_.release(r.host_off);
        reqs_.erase(f);
        return true;
    }

    // forget a request that was dropped from the queue (no memory held)
    void forget(uint64_t id)
    {
        auto f = reqs_.find(id);
        if (f != reqs_.end() && f->second.state == RS_DONE) reqs_.erase(f);
    }

    const SchedReq *find(uint64_t id) const
    {
        auto f = reqs_.find(id);
        return f == reqs_.end() ? nullptr : &f->second;
    }
    bool cell_idle(int cell) const
    {
        for (auto &kv : reqs_)
            if (kv.second.cell == cell && kv.second.state != RS_DONE) return false;
        return true;
    }
    int n_active() const { return (int)active_.size(); }
    int n_pending() const { return (int)pending_.size(); }
    const Arena &dev() const { return dev_; }
    const Arena &host() const { return host_; }

private:
    Arena dev_, host_;
    int max_active_, max_pending_;
    std::deque<uint64_t> pending_;
    std::vector<uint64_t> active_;
    std::unordered_map<uint64_t, SchedReq> reqs_;
};

}  // namespace mppi
