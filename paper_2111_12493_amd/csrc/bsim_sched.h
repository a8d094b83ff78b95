// bsim_sched.h -- request scheduling of the serving loop (a11): continuous
// batching of summarize and update requests by device footprint.
//
// Host code only (no HIP): the server runs the requests; this decides when.
//   - A request is admitted when its footprint fits the budget left by the
//     running requests and the server-owned states; among those that fit,
//     submission order.
//   - Updates of one state run one at a time, in submission order.
//   - A request that cannot fit beside the owned states even with nothing
//     else running is refused at submit (BSIM_E_BUSY), or failed with
//     BSIM_E_BUSY once that becomes true while it waits.
//   - Every ticket is answered once; stopping cancels the queued requests
//     (BSIM_E_BUSY) and lets the running ones finish.
//   - The device bytes of a state are read (by the caller's bytes_of) only
//     when no request of that state is queued or running; otherwise the
//     size recorded when its last request finished is used.
// All members are guarded by one mutex; waiting uses two condition
// variables (work for the workers, done for pollers).  The CPU tests drive
// it with many threads under the thread and address sanitizers.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "bsim.h"

namespace bsim {

// The outcome of one request.
struct SchedDone {
    int status = BSIM_OK;
    void* result = nullptr;
    void* state = nullptr;
};

struct SchedStats {
    uint64_t submitted = 0, completed = 0, failed = 0, bytes_in_use = 0, bytes_budget = 0;
    double p50_ms[3] = {0, 0, 0}, p99_ms[3] = {0, 0, 0};  // all, summarize, update
    double busy_ms = 0;
};

// Payload: what the executor needs to run a request.  Owned: what the
// server keeps for a state it owns (it must have a `bytes` member).
template <class Payload, class Owned>
class Scheduler {
public:
    using Clock = std::chrono::steady_clock;

    struct Entry {
        uint64_t ticket = 0;
        uint32_t kind = 0;            // BSIM_REQ_SUMMARIZE or BSIM_REQ_UPDATE; 0 = none
        const void* state = nullptr;  // an update's state
        uint64_t footprint = 0;
        Clock::time_point t_submit;
        Payload payload;
    };

    explicit Scheduler(uint64_t budget) : budget_(budget) {}

    // Queue e (kind, state, payload and, for a summarize, footprint set by
    // the caller).  An update's footprint is footprint_of(state bytes).
    template <class BytesOf, class FootprintOf>
    int submit(Entry e, BytesOf bytes_of, FootprintOf footprint_of, uint64_t* ticket) {
        std::unique_lock<std::mutex> lk(mu_);
        if (stopping_) return BSIM_E_INVALID;
        if (e.kind == BSIM_REQ_UPDATE) {
            bool in_flight = busy_.count(e.state) != 0;
            for (const Entry& q : queue_) in_flight = in_flight || q.state == e.state;
            auto it = sbytes_.find(e.state);
            uint64_t sb = 0;
            if (in_flight && it != sbytes_.end()) {
                sb = it->second;
            } else {
                sb = bytes_of(e.state);
                sbytes_[e.state] = sb;
            }
            e.footprint = footprint_of(sb);
        }
        if (e.footprint + owned_bytes_ > budget_) return BSIM_E_BUSY;
        e.ticket = next_ticket_++;
        collected_.push_back(false);
        *ticket = e.ticket;
        if (!any_submit_) {
            first_submit_ = e.t_submit;
            any_submit_ = true;
        }
        submitted_++;
        queue_.push_back(std::move(e));
        lk.unlock();
        cv_work_.notify_all();
        return BSIM_OK;
    }

    // A worker's next request: blocks until one may start; false once the
    // scheduler stops with nothing queued.
    bool next(Entry& out) {
        std::unique_lock<std::mutex> lk(mu_);
        bool got = false;
        cv_work_.wait(lk, [&] { return (got = pick_locked(out)) || (stopping_ && queue_.empty()); });
        if (!got) return false;
        in_use_ += out.footprint;
        running_++;
        if (out.kind == BSIM_REQ_UPDATE) busy_.insert(out.state);
        return true;
    }

    // The request ran.  `owned` (nullable): the state it created, kept by the
    // server; new_state_bytes: an update's state size afterwards.
    void complete(const Entry& e, const SchedDone& d, const Owned* owned, uint64_t new_state_bytes) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            in_use_ -= e.footprint;
            running_--;
            if (owned && d.state) {
                owned_[d.state] = *owned;
                in_use_ += owned->bytes;
                owned_bytes_ += owned->bytes;
                sbytes_[d.state] = owned->bytes;
            }
            if (e.kind == BSIM_REQ_UPDATE) {
                busy_.erase(e.state);
                sbytes_[e.state] = new_state_bytes;
                auto it = owned_.find(e.state);
                if (it != owned_.end()) {  // an update may grow an owned state
                    in_use_ = in_use_ - it->second.bytes + new_state_bytes;
                    owned_bytes_ = owned_bytes_ - it->second.bytes + new_state_bytes;
                    it->second.bytes = new_state_bytes;
                }
            }
            finish_locked(e, d);
        }
        cv_done_.notify_all();
        cv_work_.notify_all();
    }

    // The outcome of a ticket: BSIM_E_INVALID for an unknown or collected
    // ticket, BSIM_E_BUSY when not ready and !wait, else its status.
    int poll(uint64_t ticket, bool wait, SchedDone* out) {
        std::unique_lock<std::mutex> lk(mu_);
        if (ticket == 0 || ticket >= next_ticket_) return BSIM_E_INVALID;
        if (collected_[ticket - 1]) return BSIM_E_INVALID;
        auto ready = [&] { return done_.count(ticket) != 0; };
        if (!ready()) {
            if (!wait) return BSIM_E_BUSY;
            cv_done_.wait(lk, ready);
        }
        *out = done_[ticket];
        done_.erase(ticket);
        collected_[ticket - 1] = true;
        return out->status;
    }

    // f() under the lock when nothing is queued or running, else BSIM_E_BUSY.
    template <class F>
    int with_idle(F f) {
        std::lock_guard<std::mutex> lk(mu_);
        if (running_ || !queue_.empty()) return BSIM_E_BUSY;
        return f(owned_);
    }

    // Stop owning `state`: waits until none of its requests is queued or
    // running.  False if the server does not own it.
    bool release(const void* state, Owned* out) {
        bool ok = false;
        {
            std::unique_lock<std::mutex> lk(mu_);
            auto it = owned_.find(state);
            if (it == owned_.end()) return false;
            cv_done_.wait(lk, [&] {
                if (busy_.count(state)) return false;
                for (const Entry& q : queue_)
                    if (q.state == state) return false;
                return true;
            });
            it = owned_.find(state);
            if (it != owned_.end()) {
                *out = it->second;
                in_use_ -= it->second.bytes;
                owned_bytes_ -= it->second.bytes;
                owned_.erase(it);
                sbytes_.erase(state);
                ok = true;
            }
        }
        cv_work_.notify_all();
        return ok;
    }

    // Cancel the queued requests (BSIM_E_BUSY) and let the workers end once
    // the running ones finish.
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
            for (const Entry& e : queue_) finish_locked(e, SchedDone{BSIM_E_BUSY, nullptr, nullptr});
            queue_.clear();
        }
        cv_work_.notify_all();
        cv_done_.notify_all();
    }

    // After stop() and the workers' end: outcomes nobody collected, and the
    // owned states.
    void drain(std::vector<SchedDone>* uncollected, std::map<const void*, Owned>* owned) {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& kv : done_) uncollected->push_back(kv.second);
        done_.clear();
        owned->swap(owned_);
    }

    SchedStats stats() {
        SchedStats s;
        std::lock_guard<std::mutex> lk(mu_);
        s.submitted = submitted_;
        s.completed = completed_;
        s.failed = failed_;
        s.bytes_in_use = in_use_;
        s.bytes_budget = budget_;
        for (int i = 0; i < 3; i++) {
            std::vector<double> v = lat_[i];
            if (v.empty()) continue;
            std::sort(v.begin(), v.end());
            auto pct = [&](double q) { return v[std::min(v.size() - 1, static_cast<size_t>(q * (v.size() - 1) + 0.5))]; };
            s.p50_ms[i] = pct(0.50);
            s.p99_ms[i] = pct(0.99);
        }
        if (any_submit_ && completed_)
            s.busy_ms = std::chrono::duration<double, std::milli>(last_done_ - first_submit_).count();
        return s;
    }

    uint64_t budget() const { return budget_; }

private:
    // Record an outcome.  Holds mu_.
    void finish_locked(const Entry& e, const SchedDone& d) {
        const auto now = Clock::now();
        const double ms = std::chrono::duration<double, std::milli>(now - e.t_submit).count();
        lat_[0].push_back(ms);
        lat_[e.kind == BSIM_REQ_SUMMARIZE ? 1 : 2].push_back(ms);
        last_done_ = now;
        completed_++;
        if (d.status != BSIM_OK) failed_++;
        done_[e.ticket] = d;
    }

    // With nothing running, a queued request larger than what the owned
    // states leave of the budget can never start: fail it.  Holds mu_.
    void fail_unfit_locked() {
        if (running_) return;
        bool any = false;
        for (auto it = queue_.begin(); it != queue_.end();) {
            if (owned_bytes_ + it->footprint > budget_) {
                finish_locked(*it, SchedDone{BSIM_E_BUSY, nullptr, nullptr});
                it = queue_.erase(it);
                any = true;
            } else {
                ++it;
            }
        }
        if (any) cv_done_.notify_all();
    }

    // The first queued request in submission order that fits and keeps the
    // per-state order of updates.  Holds mu_.
    bool pick_locked(Entry& out) {
        fail_unfit_locked();
        std::set<const void*> earlier;
        for (auto it = queue_.begin(); it != queue_.end(); ++it) {
            if (it->kind == BSIM_REQ_UPDATE) {
                const bool blocked = busy_.count(it->state) || earlier.count(it->state);
                earlier.insert(it->state);
                if (blocked) continue;
            }
            if (in_use_ + it->footprint > budget_) continue;
            out = std::move(*it);
            queue_.erase(it);
            return true;
        }
        return false;
    }

    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    uint64_t budget_ = 0, in_use_ = 0, owned_bytes_ = 0;
    std::deque<Entry> queue_;
    std::set<const void*> busy_;
    std::map<uint64_t, SchedDone> done_;
    std::vector<bool> collected_;  // by ticket: outcome already handed out
    std::map<const void*, Owned> owned_;
    std::map<const void*, uint64_t> sbytes_;  // device bytes of each state seen
    uint32_t running_ = 0;
    uint64_t next_ticket_ = 1, submitted_ = 0, completed_ = 0, failed_ = 0;
    bool stopping_ = false;
    std::vector<double> lat_[3];
    Clock::time_point first_submit_, last_done_;
    bool any_submit_ = false;
};

}  // namespace bsim
