// Serving loop: continuous batching of forward transforms of uneven size on one GPU.
//
// The scheduling (arrival order, admission by HBM footprint into one arena, grouping,
// retirement) is the host-only Scheduler of sched.h; this file supplies its device side:
// a HIP executor that stages inputs in a pinned host ring, keeps device tables (Wigner-d,
// twiddles) cached by the fields they depend on, builds plan views, and enqueues each group
// on the next of the server's streams: input copies, couplings, then one synthesis grid for
// FULL requests that share a synthesis kernel (a tile list over up to kSynthBatchMax
// requests), or a request's own launches (ENERGY, the W/U synthesis of L_h > 16).  Table
// builds, copies and launches run on the scheduler's worker thread with the scheduler lock
// released.
#include <hip/hip_runtime.h>

#include <chrono>
#include <iterator>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "sched.h"
#include "slsht_internal.h"

namespace {

struct ExecState {
    slsht::DevPlan P;
    hipEvent_t done = nullptr;
};

size_t al(size_t n) { return (n + 255) / 256 * 256; }

class HipExecutor final : public slsht::Executor {
public:
    static constexpr size_t kStagingBytes = (size_t)64 << 20;   // pinned input ring
    static constexpr size_t kMaxTables = 64;

    int device = 0;
    size_t lds_limit = 0;
    char* base = nullptr;                  // device arena
    std::vector<hipStream_t> streams;
    size_t next_stream = 0;
    char* pinned = nullptr;                // pinned staging ring (host)
    slsht::Arena ring;
    std::unordered_map<std::string, std::shared_ptr<slsht::Tables>> tables;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() override {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void* stage_alloc(size_t n) override {
        if (!pinned) return nullptr;
        const size_t off = ring.alloc(n);
        return off == slsht::Arena::kFail ? nullptr : pinned + off;
    }
    void stage_free(void* p) override { ring.release(static_cast<char*>(p) - pinned); }

    void bind_thread() override { (void)hipSetDevice(device); }

    // Keeps the table cache bounded: beyond kMaxTables entries, drops the sets that no
    // request holds (a request's plan view keeps its own reference until it is forgotten).
    void trim_tables() {
        if (tables.size() <= kMaxTables) return;
        for (auto it = tables.begin(); it != tables.end() && tables.size() > kMaxTables;)
            it = it->second.use_count() == 1 ? tables.erase(it) : std::next(it);
    }

    int prepare(slsht::SchedRequest& r) override {
        const std::string key = slsht::tables_key(r.d);
        auto it = tables.find(key);
        if (it == tables.end()) {
            trim_tables();
            std::shared_ptr<slsht::Tables> T;
            const int rc = slsht::build_tables(r.d, device, T);
            if (rc) return rc;
            it = tables.emplace(key, T).first;
        }
        auto st = std::make_unique<ExecState>();
        const int rc = slsht::make_view(r.d, it->second, lds_limit, st->P);
        if (rc) return rc;
        r.exec = st.release();
        return SLSHT_OK;
    }

    const void* group_key(const slsht::SchedRequest& r) override {
        const slsht::DevPlan& P = static_cast<ExecState*>(r.exec)->P;
        if (P.d.output_mode != SLSHT_OUT_FULL) return nullptr;    // ENERGY runs alone
        return slsht::synthesis_kernel_key(P);                     // unique for W/U plans
    }

    struct DevPtrs {
        double2 *f, *h, *A;
        void* g;
        void* work;
    };
    // Input block layout: [f][h][A][ENERGY or W/U-synthesis workspace], 256-B aligned.
    DevPtrs ptrs(const slsht::SchedRequest& r) const {
        char* in = base + r.in_off;
        DevPtrs p;
        p.f = reinterpret_cast<double2*>(in);
        p.h = reinterpret_cast<double2*>(in + al(r.fb));
        p.A = reinterpret_cast<double2*>(in + al(r.fb) + al(r.hb));
        p.work = in + al(r.fb) + al(r.hb) + al(slsht::coupling_bytes(r.d));
        p.g = base + r.out_off;
        return p;
    }

    int launch(const std::vector<slsht::SchedRequest*>& grp) override {
        hipStream_t s = streams[next_stream++ % streams.size()];
        hipError_t e = hipSuccess;
        std::vector<const slsht::DevPlan*> P;
        std::vector<const double2*> A, H;
        std::vector<void*> G;
        for (slsht::SchedRequest* r : grp) {
            ExecState* st = static_cast<ExecState*>(r->exec);
            const DevPtrs d = ptrs(*r);
            const char* src = static_cast<const char*>(r->host_in);
            if (e == hipSuccess) e = hipMemcpyAsync(d.f, src, r->fb, hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d.h, src + r->fb, r->hb, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = slsht::launch_coupling(st->P, d.f, d.A, s);
            st->P.ework = d.work;
            P.push_back(&st->P);
            A.push_back(d.A);
            H.push_back(d.h);
            G.push_back(d.g);
        }
        if (e == hipSuccess) {
            if (P[0]->d.output_mode != SLSHT_OUT_FULL)
                e = slsht::launch_energy(*P[0], A[0], H[0], (float*)G[0], s);
            else if (grp.size() == 1)
                e = slsht::launch_synthesis(*P[0], A[0], H[0], G[0], s);
            else
                e = slsht::launch_synthesis_batch(P.data(), A.data(), H.data(), G.data(),
                                                  (int)grp.size(), s);
        }
        for (slsht::SchedRequest* r : grp) {
            ExecState* st = static_cast<ExecState*>(r->exec);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&st->done, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(st->done, s);
        }
        if (e != hipSuccess) {
            // let what was enqueued drain: the group's blocks and staging are released next
            (void)hipStreamSynchronize(s);
            return slsht::set_error(SLSHT_EDEVICE, "enqueue: %s", hipGetErrorString(e));
        }
        return SLSHT_OK;
    }

    int query(slsht::SchedRequest& r) override {
        const hipError_t q = hipEventQuery(static_cast<ExecState*>(r.exec)->done);
        if (q == hipErrorNotReady) return 0;
        return q == hipSuccess ? 1 : SLSHT_EDEVICE;
    }

    void forget(slsht::SchedRequest& r) override {
        ExecState* st = static_cast<ExecState*>(r.exec);
        if (st->done) (void)hipEventDestroy(st->done);
        delete st;
        r.exec = nullptr;
    }

    void drain() override {
        for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
    }

    ~HipExecutor() override {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device);
        for (hipStream_t s : streams) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        tables.clear();
        if (base) (void)hipFree(base);
        if (pinned) (void)hipHostFree(pinned);
        if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct slsht_server_s {
    HipExecutor ex;
    std::unique_ptr<slsht::Scheduler> sched;
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
    slsht::DeviceGuard guard(device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice(%d) failed", device);
    auto S = std::make_unique<slsht_server_s>();
    S->ex.device = device;
    S->ex.lds_limit = slsht::device_lds_limit(device);
    const size_t budget = hbm_budget / 256 * 256;
    hipError_t e = hipMalloc((void**)&S->ex.base, budget);
    for (int i = 0; i < n_streams && e == hipSuccess; ++i) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) S->ex.streams.push_back(s);
    }
    if (e != hipSuccess)
        return slsht::set_error(SLSHT_ENOMEM, "server setup: %s", hipGetErrorString(e));
    // pinned staging ring for request inputs (without it inputs are staged in pageable memory)
    if (hipHostMalloc((void**)&S->ex.pinned, HipExecutor::kStagingBytes, hipHostMallocDefault) ==
        hipSuccess)
        S->ex.ring.reset(HipExecutor::kStagingBytes, 256);
    else
        S->ex.pinned = nullptr;
    S->sched = std::make_unique<slsht::Scheduler>(&S->ex, budget, slsht::kSynthBatchMax);
    S->sched->start();
    *out = S.release();
    return SLSHT_OK;
}

int slsht_server_destroy(slsht_server_t S) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    S->sched->shutdown();
    S->sched.reset();
    delete S;
    return SLSHT_OK;
}

int slsht_submit(slsht_server_t S, const slsht_desc* desc, const void* f_host, const void* h_host,
                 uint64_t* ticket) {
    if (!S || !f_host || !h_host || !ticket) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    int rc = slsht::check_desc(desc);
    if (rc) return rc;
    const size_t fb = (size_t)desc->L_f * desc->L_f * sizeof(double2);
    const size_t hb = (size_t)desc->L_h * desc->L_h * sizeof(double2);
    const size_t out_bytes = slsht::output_bytes(*desc);
    const size_t in_bytes = al(fb) + al(hb) + al(slsht::coupling_bytes(*desc)) +
                            al(slsht::workspace_bytes(*desc));
    rc = S->sched->submit(*desc, out_bytes, in_bytes, f_host, fb, h_host, hb, ticket);
    if (rc == SLSHT_ETOOBIG)
        return slsht::set_error(SLSHT_ETOOBIG, "request needs %zu bytes, budget is %zu",
                                al(out_bytes) + al(in_bytes), S->sched->budget());
    if (rc == SLSHT_EBUSY) return slsht::set_error(SLSHT_EBUSY, "server is shutting down");
    if (rc) return slsht::set_error(rc, "submit failed");
    return SLSHT_OK;
}

int slsht_poll(slsht_server_t S, uint64_t ticket, int* state, const void** g_dev, size_t* out_bytes,
               int* err) {
    if (!S || !state) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    size_t off = slsht::Arena::kFail;
    const int rc = S->sched->poll(ticket, state, &off, out_bytes, err);
    if (rc) return slsht::set_error(rc, "unknown ticket %llu", (unsigned long long)ticket);
    if (g_dev) *g_dev = off == slsht::Arena::kFail ? nullptr : S->ex.base + off;
    return SLSHT_OK;
}

int slsht_wait(slsht_server_t S, uint64_t ticket, int timeout_ms) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    const int rc = S->sched->wait(ticket, timeout_ms);
    if (rc == SLSHT_ENOTFOUND)
        return slsht::set_error(rc, "unknown ticket %llu", (unsigned long long)ticket);
    if (rc == SLSHT_EBUSY)
        return slsht::set_error(rc, "ticket %llu not finished after %d ms",
                                (unsigned long long)ticket, timeout_ms);
    return SLSHT_OK;
}

int slsht_release(slsht_server_t S, uint64_t ticket) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    const int rc = S->sched->release(ticket);
    if (rc == SLSHT_ENOTFOUND)
        return slsht::set_error(rc, "unknown ticket %llu", (unsigned long long)ticket);
    if (rc == SLSHT_EBUSY)
        return slsht::set_error(rc, "ticket %llu is still running", (unsigned long long)ticket);
    return SLSHT_OK;
}

int slsht_request_times(slsht_server_t S, uint64_t ticket, double* t_submit, double* t_start,
                        double* t_done) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    const int rc = S->sched->times(ticket, t_submit, t_start, t_done);
    if (rc) return slsht::set_error(rc, "unknown ticket %llu", (unsigned long long)ticket);
    return SLSHT_OK;
}

double slsht_server_clock(slsht_server_t S) { return S ? S->ex.now() : 0.0; }

int slsht_server_stats(slsht_server_t S, size_t* used_bytes, size_t* budget_bytes, int* n_queued,
                       int* n_running) {
    if (!S) return slsht::set_error(SLSHT_EINVAL, "server is NULL");
    S->sched->stats(used_bytes, budget_bytes, n_queued, n_running);
    return SLSHT_OK;
}

}  // extern "C"
