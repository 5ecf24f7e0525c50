// The serving scheduler (paper_1207_5558_amd/csrc/sched.h) against a fake executor on the
// CPU: admission order and budget, the bound on passing a blocked head, ETOOBIG, failures
// in preparation, launch and on the device, cancellation, grouping, shutdown with work
// queued, and (mode "threads") a multi-threaded run with the real worker thread.
#include <atomic>
#include <cassert>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_1207_5558_amd/csrc/sched.h"

namespace {

using slsht::SchedRequest;
using slsht::Scheduler;

struct FakeExec : slsht::Executor {
    bool real_clock = false;
    double clock = 0.0;                   // manual clock (deterministic tests)
    double duration = 1.0;                // device time of a launched group
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::vector<std::vector<uint64_t>> launches;
    std::map<uint64_t, double> finish_at;
    std::set<uint64_t> fail_prepare, fail_launch, fail_device;
    std::map<uint64_t, double> expect;    // submitted input marker by ticket (single-thread tests)
    std::map<uint64_t, double> dur;       // device time by ticket (default: duration)
    std::atomic<int> live{0}, staged{0};
    std::mt19937 rng{7};

    double now() override {
        if (!real_clock) return clock;
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void* stage_alloc(size_t n) override {
        ++staged;
        return ::operator new(n ? n : 1);
    }
    void stage_free(void* p) override {
        --staged;
        ::operator delete(p);
    }
    int prepare(SchedRequest& r) override {
        if (fail_prepare.count(r.ticket)) return SLSHT_EINVAL;
        r.exec = new int(r.d.L_h);
        ++live;
        return SLSHT_OK;
    }
    const void* group_key(const SchedRequest& r) override {
        if (r.d.output_mode == SLSHT_OUT_ENERGY) return nullptr;
        return reinterpret_cast<const void*>((uintptr_t)(r.d.L_h + 1));
    }
    int launch(const std::vector<SchedRequest*>& g) override {
        std::vector<uint64_t> t;
        for (auto* r : g) {
            t.push_back(r->ticket);
            // the staged inputs must still hold what was submitted
            const double* f = static_cast<const double*>(r->host_in);
            auto e = expect.find(r->ticket);
            assert(e == expect.end() || f[0] == e->second);
        }
        launches.push_back(t);
        for (auto* r : g)
            if (fail_launch.count(r->ticket)) return SLSHT_EDEVICE;
        for (auto* r : g) {
            const auto it = dur.find(r->ticket);
            const double d = real_clock ? 1e-4 * (1 + rng() % 20)
                                        : (it != dur.end() ? it->second : duration);
            finish_at[r->ticket] = now() + d;
        }
        return SLSHT_OK;
    }
    int query(SchedRequest& r) override {
        if (now() < finish_at.at(r.ticket)) return 0;
        return fail_device.count(r.ticket) ? SLSHT_EDEVICE : 1;
    }
    void forget(SchedRequest& r) override {
        delete static_cast<int*>(r.exec);
        r.exec = nullptr;
        --live;
    }
    void drain() override {}
};

slsht_desc desc(int L_h, int mode = SLSHT_OUT_FULL) {
    slsht_desc d{};
    d.L_f = 8;
    d.L_h = L_h;
    d.output_mode = mode;
    return d;
}

uint64_t submit(FakeExec& ex, Scheduler& s, size_t out, size_t in, int L_h = 4,
                int mode = SLSHT_OUT_FULL) {
    static double marker = 1.0;
    double f[4] = {marker, 0, 0, 0};
    double h[2] = {0, 0};
    uint64_t t = 0;
    const int rc = s.submit(desc(L_h, mode), out, in, f, sizeof f, h, sizeof h, &t);
    assert(rc == SLSHT_OK);
    ex.expect[t] = marker;
    marker += 1.0;
    return t;
}

int state_of(Scheduler& s, uint64_t t, int* err = nullptr) {
    int st = -1, e = 0;
    const int rc = s.poll(t, &st, nullptr, nullptr, &e);
    if (rc != SLSHT_OK) return rc;
    if (err) *err = e;
    return st;
}

const size_t K = 1024;

void test_order_budget_and_release() {
    FakeExec ex;
    Scheduler s(&ex, 10 * K, 16);
    const uint64_t a = submit(ex, s, 4 * K, K), b = submit(ex, s, 4 * K, K), c = submit(ex, s, 4 * K, K),
                   d = submit(ex, s, 768, 256);
    assert(s.step() == 2);
    assert(state_of(s, a) == SLSHT_REQ_RUNNING && state_of(s, b) == SLSHT_REQ_RUNNING);
    assert(state_of(s, c) == SLSHT_REQ_QUEUED && state_of(s, d) == SLSHT_REQ_QUEUED);
    size_t used = 0;
    s.stats(&used, nullptr, nullptr, nullptr);
    assert(used == 10 * K);
    ex.clock = 1.5;                       // a and b finish: inputs free (two 1K holes),
    assert(s.step() == 1);                // outputs held; d passes c, which does not fit
    assert(state_of(s, a) == SLSHT_REQ_DONE && state_of(s, b) == SLSHT_REQ_DONE);
    assert(state_of(s, d) == SLSHT_REQ_RUNNING && state_of(s, c) == SLSHT_REQ_QUEUED);
    size_t off = 0, ob = 0;
    int st = 0;
    assert(s.poll(a, &st, &off, &ob, nullptr) == SLSHT_OK && ob == 4 * K && off != slsht::Arena::kFail);
    assert(s.release(a) == SLSHT_OK && s.release(b) == SLSHT_OK);
    assert(state_of(s, a) == SLSHT_ENOTFOUND);
    assert(s.step() == 1);
    assert(state_of(s, c) == SLSHT_REQ_RUNNING);
    assert(s.release(c) == SLSHT_EBUSY);  // running
    ex.clock = 3.0;
    s.step();
    assert(state_of(s, c) == SLSHT_REQ_DONE && state_of(s, d) == SLSHT_REQ_DONE);
    assert(ex.launches.size() == 3);      // {a, b}, {d}, {c}: one group per pass and key
    assert(ex.launches[0].size() == 2);
    double ts, t0, td;
    assert(s.times(c, &ts, &t0, &td) == SLSHT_OK && ts <= t0 && t0 <= td);
    assert(s.release(c) == SLSHT_OK && s.release(d) == SLSHT_OK);
    s.stats(&used, nullptr, nullptr, nullptr);
    assert(used == 0);
    s.shutdown();
    assert(ex.live == 0 && ex.staged == 0);
    printf("order/budget/release ok\n");
}

void test_bypass_bound() {
    FakeExec ex;
    Scheduler s(&ex, 16 * K, 1);
    const uint64_t r0 = submit(ex, s, 8 * K, K);        // long-running, holds 9K
    ex.dur[r0] = 1e9;
    assert(s.step() == 1);
    const uint64_t head = submit(ex, s, 12 * K, K);     // cannot fit while r0 runs
    std::vector<uint64_t> small;
    for (int i = 0; i < 20; ++i) small.push_back(submit(ex, s, 256, 256));
    // small requests pass the blocked head, kMaxBypass times in all
    for (int pass = 0; pass < 10; ++pass) {
        s.step();
        ex.clock += 2.0;
        s.step();
        for (uint64_t t : small)
            if (state_of(s, t) == SLSHT_REQ_DONE) assert(s.release(t) == SLSHT_OK);
    }
    int ran = 0;
    for (uint64_t t : small) ran += state_of(s, t) != SLSHT_REQ_QUEUED;
    assert(ran == Scheduler::kMaxBypass);
    assert(state_of(s, head) == SLSHT_REQ_QUEUED && state_of(s, r0) == SLSHT_REQ_RUNNING);
    ex.clock = 2e9;                                     // r0 finishes; its output is released
    s.step();
    assert(state_of(s, r0) == SLSHT_REQ_DONE && state_of(s, head) == SLSHT_REQ_QUEUED);
    assert(s.release(r0) == SLSHT_OK);
    s.step();                                           // the head goes before the rest
    assert(state_of(s, head) == SLSHT_REQ_RUNNING);
    s.shutdown();
    assert(ex.live == 0 && ex.staged == 0);
    printf("bypass bound ok\n");
}

void test_too_big_and_failures() {
    FakeExec ex;
    Scheduler s(&ex, 8 * K, 16);
    double f[4] = {0}, h[2] = {0};
    uint64_t t = 0;
    assert(s.submit(desc(4), 8 * K, 1, f, sizeof f, h, sizeof h, &t) == SLSHT_ETOOBIG);
    const uint64_t p = submit(ex, s, K, K), l = submit(ex, s, K, K, 5), dv = submit(ex, s, K, K, 6),
                   ok = submit(ex, s, K, K, 7);
    ex.fail_prepare.insert(p);
    ex.fail_launch.insert(l);
    ex.fail_device.insert(dv);
    assert(s.step() == 4);
    int err = 0;
    assert(state_of(s, p, &err) == SLSHT_REQ_FAILED && err == SLSHT_EINVAL);
    assert(state_of(s, l, &err) == SLSHT_REQ_FAILED && err == SLSHT_EDEVICE);
    assert(state_of(s, dv) == SLSHT_REQ_RUNNING);
    ex.clock = 2.0;
    s.step();
    assert(state_of(s, dv, &err) == SLSHT_REQ_FAILED && err == SLSHT_EDEVICE);
    assert(state_of(s, ok) == SLSHT_REQ_DONE);
    size_t used = 0;
    s.stats(&used, nullptr, nullptr, nullptr);
    assert(used == Scheduler::aligned(K));        // only the finished output is held
    for (uint64_t x : {p, l, dv, ok}) assert(s.release(x) == SLSHT_OK);
    s.shutdown();
    assert(ex.live == 0 && ex.staged == 0);
    printf("too big / failures ok\n");
}

void test_cancel_grouping_shutdown() {
    FakeExec ex;
    Scheduler s(&ex, 64 * K, 2);
    const uint64_t c1 = submit(ex, s, K, K);
    assert(s.release(c1) == SLSHT_OK);             // cancelled while queued
    assert(state_of(s, c1) == SLSHT_ENOTFOUND);
    const uint64_t g1 = submit(ex, s, K, K, 9), g2 = submit(ex, s, K, K, 9), g3 = submit(ex, s, K, K, 9),
                   e1 = submit(ex, s, K, K, 9, SLSHT_OUT_ENERGY), o1 = submit(ex, s, K, K, 3);
    assert(s.step() == 5);
    // key 9 in groups of at most 2, the ENERGY request alone, key 3 alone
    assert(ex.launches.size() == 4);
    assert((ex.launches[0] == std::vector<uint64_t>{g1, g2}));
    assert((ex.launches[1] == std::vector<uint64_t>{g3}));
    assert((ex.launches[2] == std::vector<uint64_t>{e1}));
    assert((ex.launches[3] == std::vector<uint64_t>{o1}));
    // more work queued behind a full arena, then shutdown
    FakeExec ex2;
    Scheduler s2(&ex2, 4 * K, 16);
    const uint64_t r = submit(ex2, s2, 2 * K, K), q1 = submit(ex2, s2, 2 * K, K), q2 = submit(ex2, s2, K, K);
    s2.step();
    assert(state_of(s2, r) == SLSHT_REQ_RUNNING && state_of(s2, q1) == SLSHT_REQ_QUEUED);
    s2.shutdown();
    int err = 0;
    assert(state_of(s2, q1, &err) == SLSHT_REQ_FAILED && err == SLSHT_EBUSY);
    assert(state_of(s2, q2, &err) == SLSHT_REQ_FAILED && err == SLSHT_EBUSY);
    double f[4] = {0}, h[2] = {0};
    uint64_t t = 0;
    assert(s2.submit(desc(4), K, K, f, sizeof f, h, sizeof h, &t) == SLSHT_EBUSY);
    assert(ex2.live == 0 && ex2.staged == 0);
    s.shutdown();
    assert(ex.live == 0 && ex.staged == 0);
    printf("cancel/grouping/shutdown ok\n");
}

// Worker thread + submitting and polling threads (run under ThreadSanitizer too).
void test_threads() {
    FakeExec ex;
    ex.real_clock = true;
    Scheduler s(&ex, 256 * K, 16);
    s.start();
    std::atomic<int> done{0}, failed{0};
    const int per = 150, nthreads = 4;
    std::vector<std::thread> th;
    for (int i = 0; i < nthreads; ++i)
        th.emplace_back([&, i] {
            std::mt19937 rng(100 + i);
            std::vector<uint64_t> mine;
            for (int k = 0; k < per; ++k) {
                double f[4] = {0}, h[2] = {0};
                uint64_t t = 0;
                const size_t out = 256 * (1 + rng() % 64), in = 256 * (1 + rng() % 8);
                int rc;
                do {
                    rc = s.submit(desc(4 + (int)(rng() % 3)), out, in, f, sizeof f, h, sizeof h, &t);
                } while (rc != SLSHT_OK);
                mine.push_back(t);
            }
            // release in completion order (a client that held finished outputs while it
            // waited for an earlier request could hold the budget the earlier one needs)
            while (!mine.empty()) {
                for (size_t k = 0; k < mine.size();) {
                    int st = 0;
                    assert(s.poll(mine[k], &st, nullptr, nullptr, nullptr) == SLSHT_OK);
                    if (st == SLSHT_REQ_DONE || st == SLSHT_REQ_FAILED) {
                        (st == SLSHT_REQ_DONE ? done : failed)++;
                        assert(s.release(mine[k]) == SLSHT_OK);
                        mine[k] = mine.back();
                        mine.pop_back();
                    } else {
                        ++k;
                    }
                }
                if (!mine.empty()) {
                    const int wr = s.wait(mine[0], 5);   // short: keep releasing the rest
                    assert(wr == SLSHT_OK || wr == SLSHT_EBUSY);
                }
            }
        });
    for (auto& t : th) t.join();
    s.shutdown();
    assert(done == per * nthreads && failed == 0);
    size_t used = 1;
    s.stats(&used, nullptr, nullptr, nullptr);
    assert(used == 0 && ex.live == 0 && ex.staged == 0);
    printf("threads ok: %d requests\n", done.load());
}

}  // namespace

int main(int argc, char** argv) {
    const std::string mode = argc > 1 ? argv[1] : "all";
    if (mode == "all" || mode == "steps") {
        test_order_budget_and_release();
        test_bypass_bound();
        test_too_big_and_failures();
        test_cancel_grouping_shutdown();
    }
    if (mode == "all" || mode == "threads") test_threads();
    printf("sched ok\n");
    return 0;
}
