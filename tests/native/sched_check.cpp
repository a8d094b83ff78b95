// Sanitizer driver for the serving loop's scheduler (csrc/bsim_sched.h),
// built by tests/test_sanitizers.py twice -- with -fsanitize=thread and with
// -fsanitize=address,undefined -- and run on the CPU.
//
// Submitter, worker and poller threads drive one Scheduler; the workers run
// a fake executor (a short sleep; a summarize may create a "state" of some
// size, an update changes its size).  Checked while it runs and at the end:
//   - the bytes in use (running footprints plus owned states) never exceed
//     the budget;
//   - two updates of one state never run at the same time, and they run in
//     submission order;
//   - every ticket is answered exactly once: OK, or BSIM_E_BUSY for a
//     request that could never fit; an unknown or collected ticket is
//     BSIM_E_INVALID;
//   - releasing a state waits for its queued updates; stopping cancels the
//     queued requests with BSIM_E_BUSY and the workers end.
// Prints "ok <requests>" and exits 0, or the failed check and exits 1.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "bsim_sched.h"

namespace {

#define CHECK(cond, what)                                                   \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::printf("FAIL: %s (line %d)\n", what, __LINE__);            \
            std::fflush(stdout);                                            \
            std::abort();                                                   \
        }                                                                   \
    } while (0)

struct FakeState {
    int id;
    std::atomic<int> running{0};
    std::atomic<uint64_t> bytes{0};
    std::mutex mu;
    std::vector<uint64_t> order;  // sequence numbers of the updates, as run
};

struct Payload {
    uint64_t seq = 0;  // an update's position among its state's submissions
    bool keep = false;
    uint64_t keep_bytes = 0;
    FakeState* state = nullptr;
    int64_t grow = 0;
    int sleep_us = 0;
};

struct Owned {
    uint64_t bytes = 0;
    FakeState* st = nullptr;
};

using Sched = bsim::Scheduler<Payload, Owned>;

uint64_t rnd(uint64_t& s, uint64_t bound) {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return bound ? s % bound : 0;
}

}  // namespace

int main(int argc, char** argv) {
    const uint64_t seed = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 1;
    const uint64_t budget = 1000;
    Sched sched(budget);
    std::atomic<uint64_t> running_bytes{0};
    std::atomic<int> requests{0};
    // ---- workers
    auto worker = [&]() {
        Sched::Entry e;
        while (sched.next(e)) {
            const uint64_t now = running_bytes.fetch_add(e.footprint) + e.footprint;
            CHECK(now <= budget, "running footprints within the budget");
            CHECK(sched.stats().bytes_in_use <= budget, "bytes in use within the budget");
            bsim::SchedDone d;
            Owned own;
            uint64_t new_bytes = 0;
            Payload& p = e.payload;
            if (e.kind == BSIM_REQ_UPDATE) {
                FakeState* st = p.state;
                CHECK(st->running.fetch_add(1) == 0, "one update of a state at a time");
                {
                    std::lock_guard<std::mutex> lk(st->mu);
                    st->order.push_back(p.seq);
                }
                std::this_thread::sleep_for(std::chrono::microseconds(p.sleep_us));
                const int64_t b = static_cast<int64_t>(st->bytes.load()) + p.grow;
                st->bytes.store(b < 1 ? 1 : static_cast<uint64_t>(b));
                new_bytes = st->bytes.load();
                st->running.fetch_sub(1);
            } else {
                std::this_thread::sleep_for(std::chrono::microseconds(p.sleep_us));
                if (p.keep) {
                    own.bytes = p.keep_bytes;
                    own.st = p.state;  // created by the submitter, owned from now on
                    p.state->bytes.store(p.keep_bytes);
                    d.state = p.state;
                }
            }
            running_bytes.fetch_sub(e.footprint);
            sched.complete(e, d, p.keep ? &own : nullptr, new_bytes);
            e = Sched::Entry{};
        }
    };
    std::vector<std::thread> workers;
    for (int i = 0; i < 6; i++) workers.emplace_back(worker);

    // ---- phase 1: summaries that create states, each polled
    std::vector<FakeState*> states;
    for (int i = 0; i < 8; i++) {
        FakeState* st = new FakeState();
        st->id = i;
        states.push_back(st);
        Sched::Entry e;
        e.kind = BSIM_REQ_SUMMARIZE;
        e.footprint = 40;
        e.t_submit = Sched::Clock::now();
        e.payload.keep = true;
        e.payload.keep_bytes = 20 + 5 * i;
        e.payload.state = st;
        uint64_t t = 0;
        CHECK(sched.submit(std::move(e), [](const void*) { return uint64_t(0); },
                           [](uint64_t) { return uint64_t(0); }, &t) == BSIM_OK, "submit a state's summary");
        bsim::SchedDone d;
        CHECK(sched.poll(t, true, &d) == BSIM_OK && d.state == st, "the state comes back");
        CHECK(sched.poll(t, true, &d) == BSIM_E_INVALID, "a ticket is collected once");
        requests++;
    }
    bsim::SchedDone dd;
    CHECK(sched.poll(0, false, &dd) == BSIM_E_INVALID, "ticket 0 is unknown");
    CHECK(sched.poll(1u << 30, false, &dd) == BSIM_E_INVALID, "a future ticket is unknown");

    // ---- phase 2: submitters and pollers in parallel
    std::mutex seq_mu;
    std::map<FakeState*, uint64_t> next_seq;
    std::mutex tk_mu;
    std::vector<std::pair<uint64_t, bool>> tickets;  // (ticket, may be refused later)
    std::atomic<bool> submit_done{false};
    auto submitter = [&](uint64_t s) {
        for (int i = 0; i < 400; i++) {
            Sched::Entry e;
            e.t_submit = Sched::Clock::now();
            e.payload.sleep_us = static_cast<int>(rnd(s, 200));
            bool maybe_unfit = false;
            if (rnd(s, 3) == 0) {
                e.kind = BSIM_REQ_SUMMARIZE;
                // now and then larger than what the owned states leave
                e.footprint = rnd(s, 10) == 0 ? 700 + rnd(s, 400) : 10 + rnd(s, 200);
                maybe_unfit = e.footprint > 600;
            } else {
                e.kind = BSIM_REQ_UPDATE;
                FakeState* st = states[rnd(s, states.size())];
                e.state = st;
                e.payload.state = st;
                e.payload.grow = static_cast<int64_t>(rnd(s, 21)) - 10;
                maybe_unfit = true;  // an owned state may grow past the budget's share
            }
            uint64_t t = 0;
            int rc;
            {
                // the sequence number and the submission must be taken together
                std::lock_guard<std::mutex> lk(seq_mu);
                if (e.kind == BSIM_REQ_UPDATE) e.payload.seq = next_seq[e.payload.state]++;
                rc = sched.submit(std::move(e), [](const void* p) { return static_cast<const FakeState*>(p)->bytes.load(); },
                                  [](uint64_t sb) { return 5 + sb / 4; }, &t);
            }
            requests++;
            if (rc == BSIM_E_BUSY) continue;  // refused at submit
            CHECK(rc == BSIM_OK, "submit");
            std::lock_guard<std::mutex> lk(tk_mu);
            tickets.push_back({t, maybe_unfit});
        }
    };
    std::atomic<uint64_t> answered{0};
    auto poller = [&]() {
        for (;;) {
            std::pair<uint64_t, bool> t{0, false};
            {
                std::lock_guard<std::mutex> lk(tk_mu);
                if (!tickets.empty()) {
                    t = tickets.back();
                    tickets.pop_back();
                }
            }
            if (!t.first) {
                if (submit_done.load()) {
                    std::lock_guard<std::mutex> lk(tk_mu);
                    if (tickets.empty()) return;
                }
                std::this_thread::yield();
                continue;
            }
            bsim::SchedDone d;
            const int rc = sched.poll(t.first, true, &d);
            CHECK(rc == BSIM_OK || (rc == BSIM_E_BUSY && t.second), "a ticket's outcome");
            answered++;
        }
    };
    std::vector<std::thread> subs, polls;
    for (int i = 0; i < 3; i++) subs.emplace_back(submitter, seed * 7919 + 13 * i + 1);
    for (int i = 0; i < 3; i++) polls.emplace_back(poller);
    for (auto& t : subs) t.join();
    submit_done = true;
    for (auto& t : polls) t.join();

    // per-state order of the updates
    for (FakeState* st : states) {
        std::lock_guard<std::mutex> lk(st->mu);
        for (size_t i = 1; i < st->order.size(); i++)
            CHECK(st->order[i] > st->order[i - 1], "updates of a state run in submission order");
    }
    // ---- release: waits for the state's queued updates
    for (int i = 0; i < 4; i++) {
        Owned o;
        CHECK(sched.release(states[i], &o), "release an owned state");
        CHECK(o.st == states[i], "the released state's record");
        CHECK(!sched.release(states[i], &o), "a released state is no longer owned");
    }
    // ---- stop with requests queued behind a long one
    {
        Sched::Entry e;
        e.kind = BSIM_REQ_SUMMARIZE;
        e.footprint = 10;
        e.t_submit = Sched::Clock::now();
        e.payload.sleep_us = 20000;
        std::vector<uint64_t> ts;
        for (int i = 0; i < 40; i++) {
            uint64_t t = 0;
            Sched::Entry c = e;
            CHECK(sched.submit(std::move(c), [](const void*) { return uint64_t(0); },
                               [](uint64_t) { return uint64_t(0); }, &t) == BSIM_OK, "submit before stop");
            ts.push_back(t);
            requests++;
        }
        sched.stop();
        uint64_t t = 0;
        Sched::Entry c = e;
        CHECK(sched.submit(std::move(c), [](const void*) { return uint64_t(0); }, [](uint64_t) { return uint64_t(0); },
                           &t) == BSIM_E_INVALID, "no submit after stop");
        for (auto& w : workers) w.join();
        int cancelled = 0;
        for (uint64_t tk : ts) {
            bsim::SchedDone d;
            const int rc = sched.poll(tk, true, &d);
            CHECK(rc == BSIM_OK || rc == BSIM_E_BUSY, "outcome after stop");
            cancelled += rc == BSIM_E_BUSY;
        }
        CHECK(cancelled > 0, "stopping cancels queued requests");
    }
    std::vector<bsim::SchedDone> left;
    std::map<const void*, Owned> owned;
    sched.drain(&left, &owned);
    CHECK(left.empty(), "every outcome was collected");
    CHECK(owned.size() == 4, "the states not released stay owned");
    const bsim::SchedStats st = sched.stats();
    CHECK(st.completed == st.submitted, "every admitted request completed");
    for (FakeState* s : states) delete s;
    std::printf("ok %d\n", requests.load());
    return 0;
}
