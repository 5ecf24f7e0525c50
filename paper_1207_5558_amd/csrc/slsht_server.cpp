// Serving loop: continuous batching of forward transforms of uneven size on one GPU.
//
// Callers submit descriptors with host coefficient arrays and get a ticket back at
// once.  A worker thread admits queued requests in arrival order whenever their
// footprint (output + inputs + coupling scratch) fits the server's HBM arena,
// letting smaller later requests pass a head that does not fit yet.  The requests
// admitted in one round are launched together: FULL transforms that share a synthesis
// kernel go into one grid (a tile list over up to kSynthBatchMax requests), each group
// on the next of the server's streams, so groups of different rounds also overlap on
// the device; requests retire as their completion events fire.  Device tables (Wigner-d, twiddles) are cached by the fields they
// depend on and stay resident across requests.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "slsht_internal.h"

namespace {

struct Request {
    uint64_t ticket = 0;
    slsht_desc d{};
    std::vector<double2> f, h;          // host copies taken at submit
    int state = SLSHT_REQ_QUEUED;
    int err = SLSHT_OK;
    double t_submit = 0, t_start = 0, t_done = 0;
    size_t out_bytes = 0, in_bytes = 0;
    size_t out_off = slsht::Arena::kFail, in_off = slsht::Arena::kFail;
    hipEvent_t done = nullptr;
    slsht::DevPlan P;
};

size_t al(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

struct slsht_server_s {
    int device = 0;
    size_t budget = 0;
    size_t lds_limit = 0;
    char* base = nullptr;
    slsht::Arena arena;
    std::vector<hipStream_t> streams;
    size_t next_stream = 0;
    std::mutex mu;
    std::condition_variable work_cv, done_cv;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> running;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::unordered_map<std::string, std::shared_ptr<slsht::Tables>> tables;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // Frees a request's input block (and output if requested); caller holds mu.
    void free_blocks(Request& r, bool output) {
        if (r.in_off != slsht::Arena::kFail) arena.release(r.in_off);
        r.in_off = slsht::Arena::kFail;
        if (output && r.out_off != slsht::Arena::kFail) arena.release(r.out_off);
        if (output) r.out_off = slsht::Arena::kFail;
        if (r.done) (void)hipEventDestroy(r.done);
        r.done = nullptr;
    }

    void retire_finished() {
        for (size_t i = 0; i < running.size();) {
            Request& r = *reqs[running[i]];
            const hipError_t q = hipEventQuery(r.done);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            r.t_done = now();
            if (q == hipSuccess) {
                r.state = SLSHT_REQ_DONE;
                free_blocks(r, false);
            } else {
                r.state = SLSHT_REQ_FAILED;
                r.err = SLSHT_EDEVICE;
                free_blocks(r, true);
            }
            running[i] = running.back();
            running.pop_back();
            done_cv.notify_all();
        }
    }

    // Keeps the table cache bounded: beyond kMaxTables entries, drops the sets that no
    // request holds (a request's plan keeps its own reference until it is released).
    static constexpr size_t kMaxTables = 64;
    void trim_tables() {
        if (tables.size() <= kMaxTables) return;
        for (auto it = tables.begin(); it != tables.end() && tables.size() > kMaxTables;)
            it = it->second.use_count() == 1 ? tables.erase(it) : std::next(it);
    }

    // Host side of a launch: device tables (cached) and the request's plan view.
    int prepare(Request& r) {
        const std::string key = slsht::tables_key(r.d);
        auto it = tables.find(key);
        if (it == tables.end()) {
            trim_tables();
            std::shared_ptr<slsht::Tables> T;
            int rc = slsht::build_tables(r.d, device, T);
            if (rc) return rc;
            it = tables.emplace(key, T).first;
        }
        return slsht::make_view(r.d, it->second, lds_limit, r.P);
    }

    struct DevPtrs {
        double2 *f, *h, *A;
        void* g;
        void* work;
    };
    // Input block layout: [f][h][A][ENERGY or staged-synthesis workspace], each 256-B aligned.
    DevPtrs ptrs(Request& r) {
        char* in = base + r.in_off;
        DevPtrs p;
        const size_t fb = al(r.f.size() * sizeof(double2)), hb = al(r.h.size() * sizeof(double2));
        p.f = reinterpret_cast<double2*>(in);
        p.h = reinterpret_cast<double2*>(in + fb);
        p.A = reinterpret_cast<double2*>(in + fb + hb);
        p.work = in + fb + hb + al(slsht::coupling_bytes(r.d));
        p.g = base + r.out_off;
        return p;
    }

    // Enqueues one group on one stream: inputs, couplings, then one synthesis grid for all
    // of its transforms (FULL requests sharing a kernel) or the energy kernel (a group of
    // one); each request gets its own completion event.
    hipError_t launch_group(const std::vector<Request*>& grp) {
        hipStream_t s = streams[next_stream++ % streams.size()];
        hipError_t e = hipSuccess;
        std::vector<const slsht::DevPlan*> P;
        std::vector<const double2*> A, H;
        std::vector<void*> G;
        for (Request* r : grp) {
            const DevPtrs d = ptrs(*r);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d.f, r->f.data(), r->f.size() * sizeof(double2),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d.h, r->h.data(), r->h.size() * sizeof(double2),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = slsht::launch_coupling(r->P, d.f, d.A, s);
            r->P.ework = d.work;
            P.push_back(&r->P);
            A.push_back(d.A);
            H.push_back(d.h);
            G.push_back(d.g);
        }
        if (e == hipSuccess) {
            if (grp[0]->d.output_mode != SLSHT_OUT_FULL)
                e = slsht::launch_energy(*P[0], A[0], H[0], (float*)G[0], s);
            else if (grp.size() == 1)
                e = slsht::launch_synthesis(*P[0], A[0], H[0], G[0], s);
            else
                e = slsht::launch_synthesis_batch(P.data(), A.data(), H.data(), G.data(),
                                                  (int)grp.size(), s);
        }
        for (Request* r : grp) {
            if (e == hipSuccess) e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(r->done, s);
        }
        // on failure the group's arena blocks are released: let what was enqueued drain first
        if (e != hipSuccess) (void)hipStreamSynchronize(s);
        return e;
    }

    // Launches the requests admitted in one scheduling round: FULL requests that share a
    // synthesis kernel go into common grids of up to kSynthBatchMax transforms.
    void launch_round(std::vector<Request*>& fresh) {
        std::vector<char> used(fresh.size(), 0);
        for (size_t i = 0; i < fresh.size(); ++i) {
            if (used[i]) continue;
            std::vector<Request*> grp{fresh[i]};
            used[i] = 1;
            if (fresh[i]->d.output_mode == SLSHT_OUT_FULL) {
                const void* key = slsht::synthesis_kernel_key(fresh[i]->P);
                for (size_t j = i + 1; j < fresh.size() && (int)grp.size() < slsht::kSynthBatchMax; ++j) {
                    Request& rj = *fresh[j];
                    if (used[j] || rj.d.output_mode != SLSHT_OUT_FULL ||
                        slsht::synthesis_kernel_key(rj.P) != key || rj.P.block != fresh[i]->P.block)
                        continue;
                    grp.push_back(&rj);
                    used[j] = 1;
                }
            }
            const hipError_t e = launch_group(grp);
            for (Request* r : grp) {
                if (e != hipSuccess) {
                    r->state = SLSHT_REQ_FAILED;
                    r->err = slsht::set_error(SLSHT_EDEVICE, "enqueue: %s", hipGetErrorString(e));
                    r->t_done = now();
                    free_blocks(*r, true);
                } else {
                    r->state = SLSHT_REQ_RUNNING;
                    running.push_back(r->ticket);
                }
            }
            done_cv.notify_all();
        }
    }

    void admit() {
        std::vector<Request*> fresh;
        for (auto qi = queue.begin(); qi != queue.end();) {
            Request& r = *reqs[*qi];
            const size_t out = arena.alloc(r.out_bytes);
            if (out == slsht::Arena::kFail) {
                ++qi;
                continue;
            }
            const size_t in = arena.alloc(r.in_bytes);
            if (in == slsht::Arena::kFail) {
                arena.release(out);
                ++qi;
                continue;
            }
            r.out_off = out;
            r.in_off = in;
            r.t_start = now();
            const int rc = prepare(r);
            if (rc) {
                r.state = SLSHT_REQ_FAILED;
                r.err = rc;
                r.t_done = now();
                free_blocks(r, true);
                done_cv.notify_all();
            } else {
                fresh.push_back(&r);
            }
            qi = queue.erase(qi);
        }
        if (!fresh.empty()) launch_round(fresh);
    }

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            retire_finished();
            if (!stop) admit();
            if (stop && running.empty()) break;
            if (running.empty() && queue.empty())
                work_cv.wait(lk, [&] { return stop || !queue.empty(); });
            else
                work_cv.wait_for(lk, std::chrono::microseconds(100));
        }
    }
};

extern "C" {

int slsht_server_create(int device, size_t hbm_budget, int n_streams, slsht_server_t* out) {
    if (!out) return slsht::set_error(SLSHT_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_streams < 1 || n_streams > 8)
        return slsht::set_error(SLSHT_EINVAL, "n_streams=%d outside [1, 8]", n_streams);
    if (hbm_budget < (1u << 20)) return slsht::set_error(SLSHT_EINVAL, "hbm_budget below 1 MiB");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return slsht::set_error(SLSHT_EINVAL, "device %d not available", device);
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    auto* S = new slsht_server_s();
    S->device = device;
    S->budget = hbm_budget / 256 * 256;
    S->lds_limit = slsht::device_lds_limit(device);
    hipError_t e = hipMalloc((void**)&S->base, S->budget);
    if (e == hipSuccess) {
        S->arena.reset(S->budget, 256);
        for (int i = 0; i < n_streams && e == hipSuccess; ++i) {
            hipStream_t s = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e == hipSuccess) S->streams.push_back(s);
        }
    }
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
        if (S->base) (void)hipFree(S->base);
        delete S;
        return slsht::set_error(SLSHT_ENOMEM, "server setup: %s", hipGetErrorString(e));
    }
    S->worker = std::thread([S] { S->loop(); });
    *out = S;
    return SLSHT_OK;
}

int slsht_server_destroy(slsht_server_t S) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (uint64_t t : S->queue) {
            Request& r = *S->reqs[t];
            r.state = SLSHT_REQ_FAILED;
            r.err = SLSHT_EBUSY;
        }
        S->queue.clear();
    }
    S->work_cv.notify_all();
    S->worker.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    for (hipStream_t s : S->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (auto& kv : S->reqs)
        if (kv.second->done) (void)hipEventDestroy(kv.second->done);
    S->reqs.clear();
    S->tables.clear();
    (void)hipFree(S->base);
    if (prev >= 0 && prev != S->device) (void)hipSetDevice(prev);
    delete S;
    return SLSHT_OK;
}

int slsht_submit(slsht_server_t S, const slsht_desc* desc, const void* f_host, const void* h_host,
                 uint64_t* ticket) {
    if (!S || !f_host || !h_host || !ticket) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    int rc = slsht::check_desc(desc);
    if (rc) return rc;
    auto r = std::make_unique<Request>();
    r->d = *desc;
    r->f.resize((size_t)desc->L_f * desc->L_f);
    r->h.resize((size_t)desc->L_h * desc->L_h);
    std::memcpy(r->f.data(), f_host, r->f.size() * sizeof(double2));
    std::memcpy(r->h.data(), h_host, r->h.size() * sizeof(double2));
    r->out_bytes = slsht::output_bytes(*desc);
    r->in_bytes = al(r->f.size() * sizeof(double2)) + al(r->h.size() * sizeof(double2)) +
                  al(slsht::coupling_bytes(*desc)) + al(slsht::workspace_bytes(*desc));
    if (al(r->out_bytes) + r->in_bytes > S->budget)
        return slsht::set_error(SLSHT_ETOOBIG, "request needs %zu bytes, budget is %zu",
                                al(r->out_bytes) + r->in_bytes, S->budget);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return slsht::set_error(SLSHT_EBUSY, "server is shutting down");
        r->ticket = S->next_ticket++;
        r->t_submit = S->now();
        *ticket = r->ticket;
        S->queue.push_back(r->ticket);
        S->reqs.emplace(r->ticket, std::move(r));
    }
    S->work_cv.notify_all();
    return SLSHT_OK;
}

int slsht_poll(slsht_server_t S, uint64_t ticket, int* state, const void** g_dev, size_t* out_bytes,
               int* err) {
    if (!S || !state) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return slsht::set_error(SLSHT_ENOTFOUND, "unknown ticket %llu",
                                                     (unsigned long long)ticket);
    const Request& r = *it->second;
    *state = r.state;
    if (g_dev) *g_dev = r.state == SLSHT_REQ_DONE ? S->base + r.out_off : nullptr;
    if (out_bytes) *out_bytes = r.state == SLSHT_REQ_DONE ? r.out_bytes : 0;
    if (err) *err = r.err;
    return SLSHT_OK;
}

int slsht_wait(slsht_server_t S, uint64_t ticket, int timeout_ms) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto finished = [&] {
        auto it = S->reqs.find(ticket);
        return it == S->reqs.end() || it->second->state == SLSHT_REQ_DONE ||
               it->second->state == SLSHT_REQ_FAILED;
    };
    if (S->reqs.find(ticket) == S->reqs.end())
        return slsht::set_error(SLSHT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (!S->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished))
        return slsht::set_error(SLSHT_EBUSY, "ticket %llu not finished after %d ms",
                                (unsigned long long)ticket, timeout_ms);
    return SLSHT_OK;
}

int slsht_release(slsht_server_t S, uint64_t ticket) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end())
            return slsht::set_error(SLSHT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
        Request& r = *it->second;
        if (r.state == SLSHT_REQ_RUNNING)
            return slsht::set_error(SLSHT_EBUSY, "ticket %llu is still running",
                                    (unsigned long long)ticket);
        if (r.state == SLSHT_REQ_QUEUED) {
            for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
                if (*q == ticket) {
                    S->queue.erase(q);
                    break;
                }
        }
        S->free_blocks(r, true);
        S->reqs.erase(it);
    }
    S->work_cv.notify_all();
    return SLSHT_OK;
}

int slsht_request_times(slsht_server_t S, uint64_t ticket, double* t_submit, double* t_start,
                        double* t_done) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end())
        return slsht::set_error(SLSHT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (t_submit) *t_submit = it->second->t_submit;
    if (t_start) *t_start = it->second->t_start;
    if (t_done) *t_done = it->second->t_done;
    return SLSHT_OK;
}

double slsht_server_clock(slsht_server_t S) { return S ? S->now() : 0.0; }

int slsht_server_stats(slsht_server_t S, size_t* used_bytes, size_t* budget_bytes, int* n_queued,
                       int* n_running) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    if (used_bytes) *used_bytes = S->arena.used();
    if (budget_bytes) *budget_bytes = S->arena.capacity();
    if (n_queued) *n_queued = (int)S->queue.size();
    if (n_running) *n_running = (int)S->running.size();
    return SLSHT_OK;
}

}  // extern "C"
