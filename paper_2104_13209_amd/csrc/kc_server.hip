// Serving: continuous batching of (graph, k, pivot) count queries over oriented
// graphs kept resident on the device.
//
// Queries are admitted in arrival order.  A query needs the workspace bytes
// kc_count_workspace reports for its graph, k and mode, and an estimate of the
// LDS its traversal keeps resident (one wavefront's rows and stacks times the
// wavefronts it launches, at most one per root, capped at the device's LDS).  It
// is admitted when a worker slot is free, a block of its workspace can be carved
// from the server's device arena (first fit) and, unless nothing else runs, the
// LDS of the admitted queries stays within the device's: many small queries run
// side by side, a query that fills the device runs with few others.  Every
// worker owns one HIP stream (default priority); the kernels of concurrent
// queries overlap on the device.  A query whose workspace exceeds the whole
// arena is refused (KC_ENOMEM) at once.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "kc_count_impl.h"

namespace kc {
namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Query {
    uint64_t ticket;
    int graph, k, pivot;
    size_t need;
    size_t lds = 0;     // estimated resident LDS while running
    double t_submit, t_start = 0, t_done = 0;
    int status = KC_OK;
    kc_u128 count{0, 0};
    size_t off = 0;     // arena offset while running
    bool done = false;
};

// First-fit allocator over [0, size) with coalescing of free blocks.
class Arena {
   public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t need, size_t* off) {
        need = (need + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need;
                const size_t start = it->first + need;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t need) {
        need = (need + 255) & ~size_t(255);
        auto it = free_.emplace(off, need).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

   private:
    std::map<size_t, size_t> free_;
};

}  // namespace
}  // namespace kc

struct kc_server {
    int device = 0;
    std::vector<kc_dag> dags;
    char* arena_mem = nullptr;
    size_t arena_size = 0;
    kc::Arena* arena = nullptr;
    int slots = 1;
    size_t lds_total = 0;                  // the device's LDS
    size_t lds_used = 0;                   // estimated LDS of the admitted queries
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<kc::Query*> pending;        // not yet admitted, arrival order
    std::deque<kc::Query*> ready;          // admitted, waiting for a worker
    std::map<uint64_t, kc::Query*> all;
    uint64_t next_ticket = 1;
    int running = 0;
    int waiters = 0;                       // threads inside kc_server_wait
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;

    // admit from the head of the pending queue while slots and memory allow
    void admit_locked() {
        while (!pending.empty() && running + static_cast<int>(ready.size()) < slots) {
            kc::Query* q = pending.front();
            const bool alone = running + static_cast<int>(ready.size()) == 0;
            if (!alone && lds_used + q->lds > lds_total) break;   // wait for on-chip memory
            size_t off = 0;
            if (!arena->alloc(q->need, &off)) break;   // wait for memory (keep arrival order)
            lds_used += q->lds;
            q->off = off;
            pending.pop_front();
            ready.push_back(q);
            cv_work.notify_one();
        }
    }

    void worker(int idx) {
        (void)hipSetDevice(device);
        hipStream_t s = streams[idx];
        for (;;) {
            kc::Query* q = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || !ready.empty(); });
                if (stop && ready.empty()) return;
                q = ready.front();
                ready.pop_front();
                running++;
            }
            q->t_start = kc::now_s();
            const kc_dag* d = &dags[q->graph];
            // concurrency comes from the other queries: keep each count on its worker's
            // stream, and let idle wavefronts leave instead of waiting for handoffs
            kc_opts o{};
            o.flags = KC_OPT_SINGLE_STREAM | KC_OPT_NO_HANDOFF;
            q->status = kc_count(d, q->k, q->pivot, &q->count, arena_mem + q->off, q->need, &o, s);
            q->t_done = kc::now_s();
            {
                std::lock_guard<std::mutex> lk(mu);
                arena->release(q->off, q->need);
                lds_used -= q->lds;
                running--;
                q->done = true;
                admit_locked();
            }
            cv_done.notify_all();
        }
    }
};

extern "C" KC_API int32_t kc_server_create(const kc_dag* dags, int32_t ndags, int32_t slots, uint64_t mem_budget,
                                           kc_server** out) {
    if (!out || !dags || ndags < 1 || slots < 1 || slots > 64 || mem_budget < 4096) return KC_EINVAL;
    *out = nullptr;
    kc_server* sv = new (std::nothrow) kc_server();
    if (!sv) return KC_ENOMEM;
    if (hipGetDevice(&sv->device) != hipSuccess) { delete sv; return KC_EDEVICE; }
    sv->dags.assign(dags, dags + ndags);
    sv->slots = slots;
    sv->arena_size = mem_budget;
    sv->lds_total = kc::device_lds_bytes();
    if (hipMalloc(reinterpret_cast<void**>(&sv->arena_mem), mem_budget) != hipSuccess) {
        delete sv;
        return KC_ENOMEM;
    }
    sv->arena = new kc::Arena(mem_budget);
    sv->streams.resize(slots);
    for (int i = 0; i < slots; i++) {
        if (hipStreamCreateWithFlags(&sv->streams[i], hipStreamNonBlocking) != hipSuccess) {
            for (int j = 0; j < i; j++) (void)hipStreamDestroy(sv->streams[j]);
            (void)hipFree(sv->arena_mem);
            delete sv->arena;
            delete sv;
            return KC_EDEVICE;
        }
    }
    for (int i = 0; i < slots; i++) sv->workers.emplace_back(&kc_server::worker, sv, i);
    *out = sv;
    return KC_OK;
}

extern "C" KC_API int32_t kc_server_submit(kc_server* sv, int32_t graph, int32_t k, int32_t pivot, uint64_t* ticket) {
    if (!sv || !ticket || graph < 0 || graph >= static_cast<int>(sv->dags.size()) || k < 1) return KC_EINVAL;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return KC_ECANCELED;   // the server is shutting down
    }
    kc::Query* q = new (std::nothrow) kc::Query();
    if (!q) return KC_ENOMEM;
    q->graph = graph;
    q->k = k;
    q->pivot = pivot ? 1 : 0;
    q->need = kc_count_workspace(&sv->dags[graph], k, q->pivot, nullptr);
    q->lds = kc::count_lds_demand(&sv->dags[graph], k, q->pivot);
    q->t_submit = kc::now_s();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
        delete q;
        return KC_ECANCELED;
    }
    q->ticket = sv->next_ticket++;
    *ticket = q->ticket;
    sv->all[q->ticket] = q;
    if (((q->need + 255) & ~size_t(255)) > sv->arena_size) {
        // can never fit: refuse now
        q->status = KC_ENOMEM;
        q->t_start = q->t_done = q->t_submit;
        q->done = true;
        sv->cv_done.notify_all();
        return KC_OK;
    }
    sv->pending.push_back(q);
    sv->admit_locked();
    return KC_OK;
}

extern "C" KC_API int32_t kc_server_wait(kc_server* sv, uint64_t ticket, kc_query_result* res) {
    if (!sv || !res) return KC_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return KC_EINVAL;
    kc::Query* q = it->second;
    sv->waiters++;
    sv->cv_done.wait(lk, [&] { return q->done; });
    sv->waiters--;
    res->ticket = q->ticket;
    res->graph = q->graph;
    res->k = q->k;
    res->pivot = q->pivot;
    res->status = q->status;
    res->count = q->count;
    res->t_submit = q->t_submit;
    res->t_start = q->t_start;
    res->t_done = q->t_done;
    res->workspace = q->need;
    res->lds = q->lds;
    sv->all.erase(it);
    delete q;
    if (sv->stop && sv->waiters == 0) sv->cv_done.notify_all();   // kc_server_destroy may proceed
    return KC_OK;
}

extern "C" KC_API int32_t kc_server_destroy(kc_server* sv) {
    if (!sv) return KC_EINVAL;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        // queries never admitted end now with KC_ECANCELED; threads blocked on
        // them in kc_server_wait wake up and take that result
        for (kc::Query* q : sv->pending) {
            q->status = KC_ECANCELED;
            q->t_start = q->t_done = kc::now_s();
            q->done = true;
        }
        sv->pending.clear();
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
    // admitted queries finish on their workers
    for (auto& t : sv->workers) t.join();
    {
        // nothing is freed while a waiter still reads its query
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [&] { return sv->waiters == 0; });
        for (auto& kv : sv->all) delete kv.second;
        sv->all.clear();
    }
    for (auto s : sv->streams) (void)hipStreamDestroy(s);
    (void)hipFree(sv->arena_mem);
    delete sv->arena;
    delete sv;
    return KC_OK;
}
