// Continuous-batching scheduler of the serving loop (host code only, header-only).
//
// Requests are submitted with their sizes (arena bytes for the output, and for inputs plus
// scratch) and host inputs, which are copied at once into staging memory the executor hands
// out (pinned on the GPU).  One worker thread admits queued requests in arrival order as
// their blocks fit the arena: a later, smaller request may pass a head that does not fit,
// but only kMaxBypass times; then the head is reserved and admission waits for it.  The
// requests admitted in one pass are prepared and launched with the scheduler lock released
// (table builds, copies and launches never block submit, poll or wait), in groups of up to
// `max_group` that share an executor group key; requests retire as the executor reports
// them finished.  All device work goes through the Executor interface, so the scheduler
// runs unchanged against a fake executor on the CPU.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/slsht.h"
#include "arena.h"

namespace slsht {

struct SchedRequest {
    uint64_t ticket = 0;
    slsht_desc d{};
    int state = SLSHT_REQ_QUEUED;   // RUNNING from admission on
    int err = SLSHT_OK;
    double t_submit = 0, t_start = 0, t_done = 0;
    size_t out_bytes = 0, in_bytes = 0;
    size_t out_off = Arena::kFail, in_off = Arena::kFail;
    void* host_in = nullptr;        // staged inputs: f (fb bytes) then h (hb bytes)
    size_t fb = 0, hb = 0;
    bool staged_by_executor = false;
    int bypassed = 0;               // later requests admitted past this one while it waited
    void* exec = nullptr;           // executor state of an admitted request
};

class Executor {
public:
    virtual ~Executor() = default;
    // Monotonic clock (seconds).
    virtual double now() = 0;
    // Host staging memory for a request's inputs (any thread; the scheduler serialises the
    // calls); nullptr when none is free, in which case the scheduler uses the heap.
    virtual void* stage_alloc(size_t bytes) = 0;
    virtual void stage_free(void* p) = 0;
    // Worker thread, scheduler lock released.  Host-side preparation of an admitted
    // request (device tables, plan view); returns an slsht_status.
    virtual int prepare(SchedRequest& r) = 0;
    // Requests whose equal non-null keys allow one launch (after prepare).
    virtual const void* group_key(const SchedRequest& r) = 0;
    // Worker thread, lock released: copies the group's inputs and enqueues its work;
    // returns an slsht_status (on failure nothing of the group is left in flight).
    virtual int launch(const std::vector<SchedRequest*>& group) = 0;
    // Worker thread: 1 finished, 0 still running, < 0 failed with that status.
    virtual int query(SchedRequest& r) = 0;
    // Drops the executor state of a request that finished, failed or never launched.
    virtual void forget(SchedRequest& r) = 0;
    // Waits for all device work (shutdown).
    virtual void drain() = 0;
    // Called once on the worker thread before its first pass (device binding).
    virtual void bind_thread() {}
};

class Scheduler {
public:
    static constexpr int kMaxBypass = 8;

    Scheduler(Executor* ex, size_t budget, int max_group)
        : ex_(ex), max_group_(max_group < 1 ? 1 : max_group) {
        arena_.reset(budget, 256);
    }
    ~Scheduler() { shutdown(); }

    void start() {
        worker_ = std::thread([this] { loop(); });
    }

    size_t budget() const { return arena_.capacity(); }
    static size_t aligned(size_t n) { return (n + 255) / 256 * 256; }

    int submit(const slsht_desc& d, size_t out_bytes, size_t in_bytes, const void* f, size_t fb,
               const void* h, size_t hb, uint64_t* ticket) {
        if (aligned(out_bytes) + aligned(in_bytes) > arena_.capacity()) return SLSHT_ETOOBIG;
        auto r = std::make_unique<SchedRequest>();
        r->d = d;
        r->out_bytes = out_bytes;
        r->in_bytes = in_bytes;
        r->fb = fb;
        r->hb = hb;
        {
            std::lock_guard<std::mutex> lk(stage_mu_);
            r->host_in = ex_->stage_alloc(fb + hb);
        }
        r->staged_by_executor = r->host_in != nullptr;
        if (!r->host_in) r->host_in = std::malloc(fb + hb ? fb + hb : 1);
        if (!r->host_in) return SLSHT_ENOMEM;
        std::memcpy(r->host_in, f, fb);
        std::memcpy(static_cast<char*>(r->host_in) + fb, h, hb);
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stop_) {
                free_staging(*r);
                return SLSHT_EBUSY;
            }
            r->ticket = next_ticket_++;
            r->t_submit = ex_->now();
            *ticket = r->ticket;
            queue_.push_back(r->ticket);
            reqs_.emplace(r->ticket, std::move(r));
        }
        work_cv_.notify_all();
        return SLSHT_OK;
    }

    // state, output offset (DONE only), output bytes and error of a request
    int poll(uint64_t t, int* state, size_t* out_off, size_t* out_bytes, int* err) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return SLSHT_ENOTFOUND;
        const SchedRequest& r = *it->second;
        *state = r.state;
        if (out_off) *out_off = r.state == SLSHT_REQ_DONE ? r.out_off : Arena::kFail;
        if (out_bytes) *out_bytes = r.state == SLSHT_REQ_DONE ? r.out_bytes : 0;
        if (err) *err = r.err;
        return SLSHT_OK;
    }

    int wait(uint64_t t, int timeout_ms) {
        std::unique_lock<std::mutex> lk(mu_);
        auto finished = [&] {
            auto it = reqs_.find(t);
            return it == reqs_.end() || it->second->state == SLSHT_REQ_DONE ||
                   it->second->state == SLSHT_REQ_FAILED;
        };
        if (reqs_.find(t) == reqs_.end()) return SLSHT_ENOTFOUND;
        // timed waits on the system clock (pthread_cond_timedwait): the predicate is
        // re-checked, so a clock step only moves the wake-up
        if (!done_cv_.wait_until(lk, until(std::chrono::milliseconds(timeout_ms)), finished))
            return SLSHT_EBUSY;
        return SLSHT_OK;
    }

    // Cancels a queued request or returns a finished request's blocks; EBUSY while running.
    int release(uint64_t t) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = reqs_.find(t);
            if (it == reqs_.end()) return SLSHT_ENOTFOUND;
            SchedRequest& r = *it->second;
            if (r.state == SLSHT_REQ_RUNNING) return SLSHT_EBUSY;
            if (r.state == SLSHT_REQ_QUEUED) {
                for (auto q = queue_.begin(); q != queue_.end(); ++q)
                    if (*q == t) {
                        queue_.erase(q);
                        break;
                    }
            }
            free_blocks(r, true);
            free_staging(r);
            reqs_.erase(it);
        }
        work_cv_.notify_all();
        return SLSHT_OK;
    }

    int times(uint64_t t, double* ts, double* t0, double* td) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return SLSHT_ENOTFOUND;
        if (ts) *ts = it->second->t_submit;
        if (t0) *t0 = it->second->t_start;
        if (td) *td = it->second->t_done;
        return SLSHT_OK;
    }

    void stats(size_t* used, size_t* budget, int* nq, int* nr) {
        std::lock_guard<std::mutex> lk(mu_);
        if (used) *used = arena_.used();
        if (budget) *budget = arena_.capacity();
        if (nq) *nq = (int)queue_.size();
        if (nr) *nr = (int)running_.size();
    }

    // Fails the queued requests (EBUSY), waits for the running ones, stops the worker.
    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stop_ && !worker_.joinable()) return;
            stop_ = true;
            for (uint64_t t : queue_) {
                SchedRequest& r = *reqs_[t];
                r.state = SLSHT_REQ_FAILED;
                r.err = SLSHT_EBUSY;
                r.t_done = ex_->now();
            }
            queue_.clear();
        }
        work_cv_.notify_all();
        done_cv_.notify_all();
        if (worker_.joinable()) worker_.join();
        ex_->drain();
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& kv : reqs_) {
            SchedRequest& r = *kv.second;
            if (r.state == SLSHT_REQ_RUNNING) {            // only without a worker (tests)
                r.state = SLSHT_REQ_FAILED;
                r.err = SLSHT_EBUSY;
            }
            if (r.exec) ex_->forget(r);
            free_staging(r);
        }
        running_.clear();
    }

    // One scheduling pass (the worker runs these in a loop; tests call it directly):
    // retire finished requests, admit what fits, prepare and launch it.  Returns the
    // number of requests admitted.
    int step() {
        std::unique_lock<std::mutex> lk(mu_);
        return step_locked(lk);
    }

private:
    template <class D>
    static std::chrono::system_clock::time_point until(D d) {
        return std::chrono::system_clock::now() +
               std::chrono::duration_cast<std::chrono::system_clock::duration>(d);
    }

    Executor* ex_;
    int max_group_;
    Arena arena_;
    std::mutex mu_, stage_mu_;
    std::condition_variable work_cv_, done_cv_;
    std::deque<uint64_t> queue_;
    std::vector<uint64_t> running_;
    std::unordered_map<uint64_t, std::unique_ptr<SchedRequest>> reqs_;
    std::thread worker_;
    bool stop_ = false;
    uint64_t next_ticket_ = 1;

    void free_blocks(SchedRequest& r, bool output) {
        if (r.in_off != Arena::kFail) arena_.release(r.in_off);
        r.in_off = Arena::kFail;
        if (output && r.out_off != Arena::kFail) {
            arena_.release(r.out_off);
            r.out_off = Arena::kFail;
        }
    }

    void free_staging(SchedRequest& r) {
        if (!r.host_in) return;
        if (r.staged_by_executor) {
            std::lock_guard<std::mutex> lk(stage_mu_);
            ex_->stage_free(r.host_in);
        } else {
            std::free(r.host_in);
        }
        r.host_in = nullptr;
    }

    void finish(SchedRequest& r, int state, int err) {
        r.state = state;
        r.err = err;
        r.t_done = ex_->now();
        free_blocks(r, state != SLSHT_REQ_DONE);
        free_staging(r);
        if (r.exec) ex_->forget(r);
    }

    void retire_finished() {
        for (size_t i = 0; i < running_.size();) {
            SchedRequest& r = *reqs_[running_[i]];
            const int q = ex_->query(r);
            if (q == 0) {
                ++i;
                continue;
            }
            finish(r, q > 0 ? SLSHT_REQ_DONE : SLSHT_REQ_FAILED, q > 0 ? SLSHT_OK : q);
            running_[i] = running_.back();
            running_.pop_back();
            done_cv_.notify_all();
        }
    }

    // Arrival order; a later request may pass a head that does not fit, at most kMaxBypass
    // times, after which nothing passes it (its blocks are as good as reserved).
    std::vector<SchedRequest*> admit() {
        std::vector<SchedRequest*> fresh;
        bool head_blocked = false;
        SchedRequest* head = nullptr;
        for (auto qi = queue_.begin(); qi != queue_.end();) {
            SchedRequest& r = *reqs_[*qi];
            if (head_blocked && head->bypassed >= kMaxBypass) break;
            size_t out = arena_.alloc(r.out_bytes), in = Arena::kFail;
            if (out != Arena::kFail) {
                in = arena_.alloc(r.in_bytes);
                if (in == Arena::kFail) arena_.release(out);
            }
            if (in == Arena::kFail) {
                if (!head_blocked) {
                    head_blocked = true;
                    head = &r;
                }
                ++qi;
                continue;
            }
            if (head_blocked) ++head->bypassed;
            r.out_off = out;
            r.in_off = in;
            r.t_start = ex_->now();
            r.state = SLSHT_REQ_RUNNING;
            fresh.push_back(&r);
            qi = queue_.erase(qi);
        }
        return fresh;
    }

    int step_locked(std::unique_lock<std::mutex>& lk) {
        retire_finished();
        if (stop_) return 0;
        std::vector<SchedRequest*> fresh = admit();
        if (fresh.empty()) return 0;
        lk.unlock();
        // preparation and launches with the lock released (tables, copies, kernels)
        std::vector<int> prep(fresh.size());
        for (size_t i = 0; i < fresh.size(); ++i) prep[i] = ex_->prepare(*fresh[i]);
        std::vector<std::pair<std::vector<SchedRequest*>, int>> groups;
        std::vector<char> used(fresh.size(), 0);
        for (size_t i = 0; i < fresh.size(); ++i) {
            if (used[i] || prep[i] != SLSHT_OK) continue;
            std::vector<SchedRequest*> grp{fresh[i]};
            used[i] = 1;
            const void* key = ex_->group_key(*fresh[i]);
            for (size_t j = i + 1; key && j < fresh.size() && (int)grp.size() < max_group_; ++j)
                if (!used[j] && prep[j] == SLSHT_OK && ex_->group_key(*fresh[j]) == key) {
                    grp.push_back(fresh[j]);
                    used[j] = 1;
                }
            const int rc = ex_->launch(grp);
            groups.emplace_back(std::move(grp), rc);
        }
        lk.lock();
        for (size_t i = 0; i < fresh.size(); ++i)
            if (prep[i] != SLSHT_OK) finish(*fresh[i], SLSHT_REQ_FAILED, prep[i]);
        for (auto& g : groups)
            for (SchedRequest* r : g.first) {
                if (g.second == SLSHT_OK) running_.push_back(r->ticket);
                else finish(*r, SLSHT_REQ_FAILED, g.second);
            }
        done_cv_.notify_all();
        return (int)fresh.size();
    }

    void loop() {
        ex_->bind_thread();
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            step_locked(lk);
            if (stop_ && running_.empty()) break;
            if (running_.empty() && queue_.empty() && !stop_)
                work_cv_.wait(lk, [&] { return stop_ || !queue_.empty(); });
            else
                work_cv_.wait_until(lk, until(std::chrono::microseconds(100)));
        }
    }
};

}  // namespace slsht
